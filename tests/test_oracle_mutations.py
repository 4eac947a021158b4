"""Planted mistakes in the oracle must be caught by its pins.

Each case rebuilds the C oracle with one plausible mistake (a flipped kernel,
a transposed operand, a wrong sign, an off-by-one window, a dropped term ...)
into a temporary library and runs the pin tests that should catch it against
that library.  The product library is not involved.
"""

import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "pvf_oracle.c")

# (name, original text, planted text, pin files that must catch it)
MUTATIONS = [
    ("convolution instead of correlation", "int u = t + j - r;", "int u = t - j + r;",
     ["test_oracle_ops.py"]),
    ("transposed-conv weight transposed", "W[((int64_t)c * Cout + o) * 2 + j]",
     "W[((int64_t)o * Cin + c) * 2 + j]", ["test_oracle_ops.py"]),
    ("transposed-conv taps swapped", "y[(int64_t)o * 2 * L + 2 * t + j] = s;",
     "y[(int64_t)o * 2 * L + 2 * t + (1 - j)] = s;", ["test_oracle_ops.py"]),
    ("min-pool", "y[(int64_t)c * Lo + t] = a > b ? a : b;", "y[(int64_t)c * Lo + t] = a < b ? a : b;",
     ["test_oracle_ops.py"]),
    ("LeakyReLU sign", "return x >= 0.0 ? x : slope * x;", "return x >= 0.0 ? x : -slope * x;",
     ["test_oracle_ops.py"]),
    ("softplus tail", "log1p(exp(-fabs(x)))", "log1p(exp(-x))", ["test_oracle_ops.py"]),
    ("concat order", "memcpy(cat, skip[l], sizeof(double) * act(C, Lo));\n        orc_convT2(x, Cup, Ll, WT, bT, C, cat + act(C, Lo));",
     "memcpy(cat + act(C, Lo), skip[l], sizeof(double) * act(C, Lo));\n        orc_convT2(x, Cup, Ll, WT, bT, C, cat);",
     ["test_oracle_unet.py"]),
    ("non-strict local maximum", "if (!(p[t - 1] < p[t] && p[t] > p[t + 1])) continue;",
     "if (!(p[t - 1] <= p[t] && p[t] > p[t + 1])) continue;", ["test_oracle_peaks.py"]),
    ("window one bin short", "int hi = t + hw > L - 1 ? L - 1 : t + hw;",
     "int hi = t + hw - 1 > L - 1 ? L - 1 : t + hw - 1;", ["test_oracle_peaks.py"]),
    ("closed interval", "if (zd >= lo && zd < hi) return i;", "if (zd >= lo && zd <= hi) return i;",
     ["test_oracle_ops.py"]),
    ("z feature scale", "g[0] = ((double)f[0] - lo) / (interval_mm / 2.0) - 1.0;",
     "g[0] = ((double)f[0] - lo) / interval_mm - 1.0;", ["test_oracle_ops.py"]),
    ("histogram overwrites", "H[(int64_t)n_out * i + j] += o[j];", "H[(int64_t)n_out * i + j] = o[j];",
     ["test_oracle_hist.py"]),
    ("head bias dropped", "double s = (double)bh[0];", "double s = 0.0;", ["test_oracle_unet.py"]),
    ("bin centre without the half", "M += p[j] * (z_min + bw * (j + 0.5));",
     "M += p[j] * (z_min + bw * j);", ["test_oracle_peaks.py"]),
    ("input scale dropped", "x0[t] = s_in * H[t];", "x0[t] = H[t];", ["test_oracle_forward.py"]),
    ("sigmoid sign", "return 1.0 / (1.0 + exp(-x));", "return 1.0 / (1.0 + exp(x));",
     ["test_oracle_ops.py"]),
    ("feature shift sign", "((double)f[k * stride] - (double)shift[k])",
     "((double)f[k * stride] + (double)shift[k])", ["test_oracle_hist.py"]),
    ("height threshold not strict", "if (!(p[t] > p_min)) continue;", "if (!(p[t] >= p_min)) continue;",
     ["test_oracle_peaks.py"]),
    ("boundary neighbour on the wrong side", "if (zd - lo < boundary_mm && i > 0) return i - 1;",
     "if (zd - lo < boundary_mm && i > 0 && i < n_intervals - 1) return i + 1;", ["test_oracle_variants.py"]),
    ("boundary distance not strict", "if (zd - lo < boundary_mm && i > 0)", "if (zd - lo <= boundary_mm && i > 0)",
     ["test_oracle_variants.py"]),
    ("upper distance sign", "if (hi - zd < boundary_mm", "if (zd - hi < boundary_mm", ["test_oracle_variants.py"]),
    ("neighbour in the track's own frame", "orc_features(ft, stride, n_feat, nb,", "orc_features(ft, stride, n_feat, i,",
     ["test_oracle_variants.py"]),
    ("interval layout reads interval 0", "rc = orc_unet(x0 + (int64_t)i * n_out, n_out,",
     "rc = orc_unet(x0, n_out,", ["test_oracle_variants.py"]),
]


@pytest.mark.slow
@pytest.mark.parametrize("name,orig,planted,pins", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_is_caught(name, orig, planted, pins, tmp_path):
    src = open(SRC).read()
    assert src.count(orig) >= 1, "mutation anchor not found in the oracle source"
    mutated = tmp_path / "mutant.c"
    mutated.write_text(src.replace(orig, planted, 1))
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-ffp-contract=off",
                    "-o", str(lib), str(mutated), "-lm"], check=True)
    env = dict(os.environ, PVF_ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider"]
                       + [os.path.join(ROOT, "tests", p) for p in pins],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert r.returncode != 0, f"planted mistake '{name}' passed every pin:\n{r.stdout[-2000:]}"
