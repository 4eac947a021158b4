"""An independent float64 restatement of the PVFinder forward pass in PyTorch CPU.

Used only to pin the C oracle: it is written from the paper's description
(Section 2: per-track FC network, histogram, UNet, peak finding) with
PyTorch's own library routines (``linear``, ``conv1d``, ``conv_transpose1d``,
``max_pool1d``), so it shares no code with the oracle.
"""

import numpy as np
import torch
import torch.nn.functional as F


def _t(a):
    return torch.as_tensor(np.asarray(a, dtype=np.float64))


def histogram(tracks, w, z_min=-100.0, interval_mm=10.0, n_intervals=40):
    s = w.shape
    f = _t(tracks)
    H = torch.zeros(n_intervals * s.n_out, dtype=torch.float64)
    if f.shape[1] == 0:
        return H
    ok = torch.isfinite(f).all(0)
    f = f[:, ok]
    i = torch.floor((f[0] - z_min) / interval_mm).long()
    inw = (i >= 0) & (i < n_intervals)
    f, i = f[:, inw], i[inw]
    g = (f - _t(w.shift)[:, None]) * _t(w.scale)[:, None]
    g[0] = (f[0] - (z_min + interval_mm * i.double())) / (interval_mm / 2) - 1
    h = g.T
    for l in range(s.n_hidden):
        h = F.leaky_relu(F.linear(h, _t(w[f"mlp{l}.w"]), _t(w[f"mlp{l}.b"])), w.leaky)
    o = F.softplus(F.linear(h, _t(w[f"mlp{s.n_hidden}.w"]), _t(w[f"mlp{s.n_hidden}.b"])))
    idx = (i[:, None] * s.n_out + torch.arange(s.n_out)[None, :]).reshape(-1)
    H.index_add_(0, idx, o.reshape(-1))
    return H


def unet(x0, w):
    """x0: [L] or [B][L] float64 (already scaled) -> logits of the same shape."""
    s = w.shape
    x = _t(x0)
    squeeze = x.dim() == 1
    x = x.reshape(-1, 1, x.shape[-1])
    r = (s.ksize - 1) // 2
    skips = []
    for lv in range(s.n_levels):
        for j in (1, 2):
            x = F.leaky_relu(F.conv1d(x, _t(w[f"enc{lv}.c{j}.w"]), _t(w[f"enc{lv}.c{j}.b"]),
                                      padding=r), w.leaky)
        skips.append(x)
        if lv < s.n_levels - 1:
            x = F.max_pool1d(x, 2)
    for lv in range(s.n_levels - 2, -1, -1):
        u = F.conv_transpose1d(x, _t(w[f"up{lv}.w"]), _t(w[f"up{lv}.b"]), stride=2)
        x = torch.cat([skips[lv], u], 1)
        for j in (1, 2):
            x = F.leaky_relu(F.conv1d(x, _t(w[f"dec{lv}.c{j}.w"]), _t(w[f"dec{lv}.c{j}.b"]),
                                      padding=r), w.leaky)
    logit = F.conv1d(x, _t(w["head.w"])[:, :, None], _t(w["head.b"]))[:, 0]
    return logit[0] if squeeze else logit
