"""Continuous-batching request loop over the C ABI.

The trigger framework of the paper (Section 3) runs inference on a fixed
memory pool with work enqueued on framework streams.  This loop serves
*requests* -- slices of events arriving over time -- on one GPU:

* a fixed HBM pool budget holds the engines' arenas plus every admitted
  request's device-resident state (its tracks, and its output buffers until
  the results are read back); a request is admitted as soon as its state fits
  in the pool, otherwise it waits;
* several lanes (one engine = arena + stream each) run steps concurrently, so
  work of different requests overlaps on the device;
* continuous batching: whenever a lane is free it packs events of the
  admitted requests, shortest remaining request first -- possibly the tail of
  one request and the head of the next -- into one step of at most its
  capacity; a request can span several steps and lanes;
* a request completes when its last event's results are back on the host
  (results="host"), or as soon as they are complete in HBM for consumers on
  the device (results="device": the Extract phase of Section 3 leaves the
  outputs in place and nothing is copied back); its latency is completion
  time minus arrival time;
* a request that can never fit (its state larger than the pool minus the
  lanes' arenas) is rejected on arrival with an error instead of blocking
  the queue; requests behind it are served as usual.

Every kernel is batch-invariant (fixed k order), so an event's results are
the same bits whether it ran alone or packed with others.  PyTorch only
provides device memory, streams, events and the copies that gather a step's
inputs and scatter its outputs.
"""

from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np

from ._binding import Engine, arena_bytes, default_spec

OUT_KEYS = ("n_vertices", "z", "peak_prob", "integral", "status", "bin")


@dataclass
class Request:
    rid: int
    batch: object                 # synth.EventBatch (host)
    arrival: float                # seconds, loop clock
    feat: object = None           # device float32 [9][T]
    offsets: object = None        # device int32 [E+1]
    out: dict = None              # device outputs per key, [E] or [E][max_peaks]
    state_bytes: int = 0
    next_event: int = 0           # first event not yet packed into a step
    done_events: int = 0
    t_admit: float = 0.0
    t_done: float = 0.0
    result: dict = None           # host copy of the outputs (results="host")
    feat_host: object = None      # optional page-locked torch copy of batch.feat
    error: str = None             # set when the request was rejected

    @property
    def n_events(self):
        return self.batch.n_events


@dataclass
class _Step:
    lane: int
    pieces: list                  # (request, first event, count, first row in the step)
    n_events: int
    done_event: object = None     # torch.cuda.Event recorded after the step


@dataclass
class ServeStats:
    latencies_s: list = field(default_factory=list)
    sizes: list = field(default_factory=list)
    t_first_arrival: float = 0.0
    t_last_done: float = 0.0
    steps: int = 0
    max_pool_used: int = 0
    rejected: list = field(default_factory=list)

    def summary(self):
        lat = np.array(self.latencies_s)
        per_ev = lat / np.array(self.sizes)
        total = int(np.sum(self.sizes))
        span = self.t_last_done - self.t_first_arrival
        return {
            "requests": len(lat), "rejected": len(self.rejected), "events": total, "steps": self.steps,
            "events_per_s": total / span if span > 0 else float("nan"),
            "slice_latency_ms_p50": float(np.percentile(lat, 50) * 1e3),
            "slice_latency_ms_p99": float(np.percentile(lat, 99) * 1e3),
            "us_per_event_p50": float(np.percentile(per_ev, 50) * 1e6),
            "us_per_event_p99": float(np.percentile(per_ev, 99) * 1e6),
            "max_pool_used_gb": self.max_pool_used / 1e9,
        }


def admit(waiting, pool_used: int, pool_bytes: int, state_room: int, size_of):
    """Admission by HBM budget, in arrival order.  Takes requests from the
    head of `waiting` (a deque) while their state fits beside what is in use;
    a request larger than `state_room` (the pool minus the lanes' fixed
    buffers) can never fit and is rejected instead of blocking the queue.
    Returns (admitted, rejected, pool_used after admission)."""
    admitted, rejected = [], []
    while waiting:
        need = size_of(waiting[0])
        if need > state_room:
            rejected.append(waiting.popleft())
            continue
        if pool_used + need > pool_bytes:
            break
        admitted.append(waiting.popleft())
        pool_used += need
    return admitted, rejected, pool_used


class PinnedSlab:
    """First-fit allocator over one page-locked host buffer allocated once, so
    the loop never pins memory per request.  Offsets are 256-byte aligned."""

    def __init__(self, torch, nbytes: int):
        nbytes = max(256, (int(nbytes) + 255) // 256 * 256)
        self.buf = torch.empty(nbytes, dtype=torch.uint8, pin_memory=True)
        self.free = [(0, nbytes)]             # (offset, size), ascending, coalesced

    @staticmethod
    def _round(n):
        return (int(n) + 255) // 256 * 256

    def alloc(self, n: int):
        """Offset of a free block of n bytes, or None."""
        n = self._round(n)
        for i, (o, sz) in enumerate(self.free):
            if sz >= n:
                if sz == n:
                    del self.free[i]
                else:
                    self.free[i] = (o + n, sz - n)
                return o
        return None

    def release(self, o: int, n: int):
        n = self._round(n)
        self.free.append((o, n))
        self.free.sort()
        merged = [self.free[0]]
        for fo, fs in self.free[1:]:
            lo, ls = merged[-1]
            if lo + ls == fo:
                merged[-1] = (lo, ls + fs)
            else:
                merged.append((fo, fs))
        self.free = merged

    def view(self, o: int, dtype, shape):
        import math
        n = math.prod(shape) * dtype.itemsize
        return self.buf[o:o + n].view(dtype).view(shape)


class Server:
    def __init__(self, weights_blob: bytes, pool_bytes: int = 8 << 30, lanes: int = 2,
                 lane_events: int | None = None, compute_dtype: str = "bf16",
                 max_tracks_per_event: int = 1500, max_peaks: int = 2000, device: str = "cuda:0",
                 fp8_amax=None, results: str = "host"):
        """fp8_amax: calibration table (Engine.calibrate) for an FP8 compute_dtype.
        results: "host" copies each request's outputs back into page-locked
        host memory (Request.result); "device" leaves them in HBM
        (Request.out) for consumers on the GPU."""
        import torch
        if results not in ("host", "device"):
            raise ValueError("results must be 'host' or 'device'")
        self.results = results
        self.torch = torch
        self.device = torch.device(device)
        self.pool_bytes = int(pool_bytes)
        self.max_peaks = max_peaks
        per_event_state = self._state_bytes_per_event(max_tracks_per_event=200)
        if lane_events is None:
            # the lanes' arenas take the pool minus room for a few of the
            # largest slices in flight (their tracks and output buffers)
            probe = default_spec(max_events=1, compute_dtype=compute_dtype, max_peaks_per_event=max_peaks)
            a1 = arena_bytes(probe)
            probe.max_events = 101
            per_ev_arena = (arena_bytes(probe) - a1) / 100
            reserve = min(self.pool_bytes // 4, 4 * 2000 * per_event_state)
            lane_events = max(1, int((self.pool_bytes - reserve) // lanes // (per_ev_arena + per_event_state)))
        self.lane_events = lane_events
        self.lanes = []
        for _ in range(lanes):
            spec = default_spec(max_events=lane_events, compute_dtype=compute_dtype,
                                max_tracks_per_event=max_tracks_per_event, max_peaks_per_event=max_peaks,
                                max_tracks_total=lane_events * max_tracks_per_event)
            self.lanes.append(Engine(weights_blob, spec, device=device, fp8_amax=fp8_amax))
        # per-lane step buffers, allocated once: gathered inputs and step outputs
        self.step_out = [e.alloc_outputs(lane_events, with_prob=False) for e in self.lanes]
        step_bytes = sum(v.numel() * v.element_size() for v in self.step_out[0].__dict__.values() if v is not None)
        step_bytes += 36 * lane_events * max_tracks_per_event + 4 * (lane_events + 1)
        self.arena_total = sum(e.arena_bytes for e in self.lanes) + lanes * step_bytes
        if self.arena_total >= self.pool_bytes:
            raise ValueError("pool budget too small for the lanes' arenas and step buffers")
        self.copy_stream = torch.cuda.Stream(device=self.device)
        self.pool_used = self.arena_total
        # results="host": one page-locked buffer for the readbacks, as large as
        # the pool's room for request state (every request being read back
        # still counts against the pool, so its outputs always fit)
        self.slab = PinnedSlab(torch, self.pool_bytes - self.arena_total) if results == "host" else None
        self.busy = [None] * lanes            # _Step or None per lane

    # -- accounting ----------------------------------------------------------
    def _state_bytes_per_event(self, max_tracks_per_event):
        return 36 * max_tracks_per_event + 4 + self.max_peaks * (8 + 4 + 8 + 4) + 8

    def request_bytes(self, batch) -> int:
        return int(batch.feat.nbytes + batch.offsets.nbytes + batch.n_events * (self.max_peaks * 24 + 8))

    # -- request life cycle --------------------------------------------------
    def _admit(self, r: Request, now: float):
        t = self.torch
        with t.cuda.stream(self.copy_stream):
            src = r.feat_host if r.feat_host is not None else t.from_numpy(r.batch.feat).pin_memory()
            r.feat = src.to(self.device, non_blocking=True)
            r.offsets = t.from_numpy(r.batch.offsets).to(self.device)
            E, mp = r.n_events, self.max_peaks
            r.out = {
                "n_vertices": t.zeros(E, dtype=t.int32, device=self.device),
                "z": t.empty(E, mp, dtype=t.float64, device=self.device),
                "peak_prob": t.empty(E, mp, dtype=t.float32, device=self.device),
                "integral": t.empty(E, mp, dtype=t.float64, device=self.device),
                "status": t.zeros(E, dtype=t.int32, device=self.device),
                "bin": t.empty(E, mp, dtype=t.int32, device=self.device),
            }
        r.uploaded = t.cuda.Event()
        r.uploaded.record(self.copy_stream)
        r.state_bytes = self.request_bytes(r.batch)
        r.t_admit = now
        self.pool_used += r.state_bytes

    def _launch_step(self, lane: int, queue):
        """Pack up to lane_events events into one step, shortest remaining
        request first (small slices do not wait behind large ones; the order
        never changes a result, the kernels being batch-invariant)."""
        t = self.torch
        eng = self.lanes[lane]
        pieces, rows = [], 0
        for r in sorted(queue, key=lambda q: (q.n_events - q.next_event, q.arrival)):
            if rows >= self.lane_events:
                break
            take = min(r.n_events - r.next_event, self.lane_events - rows)
            if take <= 0:
                continue
            pieces.append((r, r.next_event, take, rows))
            r.next_event += take
            rows += take
        if not pieces:
            return None
        s = eng.stream
        for r, _, _, _ in pieces:
            s.wait_event(r.uploaded)
        with t.cuda.stream(s):
            full = self.step_out[lane]
            if len(pieces) == 1:
                # one request: the step reads its tracks in place (SoA planes
                # of the request's buffer) and writes straight into its outputs
                r, e0, n, _ = pieces[0]
                a, b = int(r.batch.offsets[e0]), int(r.batch.offsets[e0 + n])
                feat = r.feat[:, a:b]
                off = r.offsets[e0:e0 + n + 1] - a
                out = type(full)(**{k: (r.out[k][e0:e0 + n] if k in r.out else None) for k in full.__dict__})
                eng.execute(feat, off, out, stream=s)
            else:
                feats, offs, base = [], [t.zeros(1, dtype=t.int32, device=self.device)], 0
                for r, e0, n, _ in pieces:
                    a, b = int(r.batch.offsets[e0]), int(r.batch.offsets[e0 + n])
                    feats.append(r.feat[:, a:b])
                    offs.append(r.offsets[e0 + 1:e0 + n + 1] - a + base)
                    base += b - a
                feat = (t.cat(feats, dim=1).contiguous() if base > 0
                        else t.zeros(9, 0, dtype=t.float32, device=self.device))
                off = t.cat(offs).contiguous()
                out = type(full)(**{k: (None if v is None else v[:rows]) for k, v in full.__dict__.items()})
                eng.execute(feat, off, out, stream=s)
                for r, e0, n, row in pieces:
                    for k in OUT_KEYS:
                        r.out[k][e0:e0 + n].copy_(getattr(out, k)[row:row + n])
            ev = t.cuda.Event()
            ev.record(s)
        step = _Step(lane, pieces, rows, ev)
        step._keep = (feat, off, out)
        self.busy[lane] = step
        return step

    def _finish_step(self, step: _Step, now: float, done: list):
        for r, e0, n, _ in step.pieces:
            r.done_events += n
            if r.done_events == r.n_events:
                r.out_ready = step.done_event
                done.append(r)

    def _start_readback(self, r: Request) -> bool:
        """Queue the device-to-host copy of a finished request's outputs on the
        copy stream, into blocks of the page-locked slab (asynchronous).
        False if the slab has no room yet (retried on a later pass)."""
        t = self.torch
        sizes = {k: v.numel() * v.element_size() for k, v in r.out.items()}
        offs = {}
        for k, n in sizes.items():
            o = self.slab.alloc(n)
            if o is None:
                for k2, o2 in offs.items():
                    self.slab.release(o2, sizes[k2])
                return False
            offs[k] = o
        r.host_blocks = [(offs[k], sizes[k]) for k in offs]
        self.copy_stream.wait_event(r.out_ready)
        r.host = {k: self.slab.view(offs[k], v.dtype, tuple(v.shape)) for k, v in r.out.items()}
        with t.cuda.stream(self.copy_stream):
            for k, v in r.out.items():
                r.host[k].copy_(v, non_blocking=True)
                v.record_stream(self.copy_stream)
        r.readback = t.cuda.Event()
        r.readback.record(self.copy_stream)
        return True

    def _complete(self, r: Request, on_complete=None):
        r.t_done = time.perf_counter() - self.t0
        if self.results == "host":
            if on_complete is not None:
                # the consumer reads the slab's blocks in place, during the call
                r.result = {k: v.numpy() for k, v in r.host.items()}
                on_complete(r)
                r.result = None
            else:
                r.result = {k: v.numpy().copy() for k, v in r.host.items()}
            for o, n in r.host_blocks:
                self.slab.release(o, n)
            r.host_blocks = None
        elif on_complete is not None:
            on_complete(r)          # device outputs in r.out, still inside the pool
        r.feat = r.offsets = r.host = r.out = None
        self.pool_used -= r.state_bytes

    # -- the loop --------------------------------------------------------------
    def run(self, requests: list, realtime: bool = True, on_complete=None) -> ServeStats:
        """Serve `requests` (arrival times in seconds from the start).  With
        realtime=False every request counts as arrived at time 0.
        on_complete(request), if given, is called as each request completes,
        while its outputs are still held: with results="device" in
        request.out (device tensors, still counted against the pool); with
        results="host" in request.result (numpy views of the page-locked
        slab, valid only during the call).  Without it, results="host"
        copies each request's outputs into request.result for the caller."""
        t = self.torch
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        waiting = collections.deque()          # arrived, not admitted (pool full)
        queue = []                             # admitted, with events left to pack
        reading = []                           # outputs on their way to the host
        unread = []                            # finished, waiting for slab room
        stats = ServeStats()
        if not realtime:
            for r in pending:
                r.arrival = 0.0
        self.t0 = time.perf_counter()
        n_left = len(requests)
        room = self.pool_bytes - self.arena_total
        while n_left:
            now = time.perf_counter() - self.t0
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            admitted, rejected, _ = admit(waiting, self.pool_used, self.pool_bytes, room,
                                          lambda q: self.request_bytes(q.batch))
            for r in rejected:
                r.error = (f"request {r.rid}: {self.request_bytes(r.batch)} bytes of device state exceed the "
                           f"pool's {room} bytes beside the lanes")
                stats.rejected.append(r)
                n_left -= 1
            for r in admitted:
                self._admit(r, now)
                queue.append(r)
            stats.max_pool_used = max(stats.max_pool_used, self.pool_used)
            # retire finished steps; a request whose last event is done starts its readback
            for lane, step in enumerate(self.busy):
                if step is not None and step.done_event.query():
                    self.busy[lane] = None
                    finished = []
                    self._finish_step(step, now, finished)
                    for r in finished:
                        if self.results == "host":
                            unread.append(r)
                        else:
                            r.readback = r.out_ready
                            reading.append(r)
            if unread:
                waiting_room = []
                for r in unread:
                    (reading if self._start_readback(r) else waiting_room).append(r)
                unread = waiting_room
            still = []
            for r in reading:
                if r.readback.query():
                    self._complete(r, on_complete)
                    stats.latencies_s.append(r.t_done - r.arrival)
                    stats.sizes.append(r.n_events)
                    stats.t_last_done = r.t_done
                    n_left -= 1
                else:
                    still.append(r)
            reading = still
            queue = [r for r in queue if r.next_event < r.n_events]
            # fill free lanes
            for lane in range(len(self.lanes)):
                if self.busy[lane] is None and queue:
                    if self._launch_step(lane, queue) is not None:
                        stats.steps += 1
                    queue = [r for r in queue if r.next_event < r.n_events]
            if not queue and not waiting and n_left:
                nxt = pending[0].arrival - (time.perf_counter() - self.t0) if pending else 0.0
                time.sleep(min(1e-4, max(2e-5, nxt)))
        t.cuda.synchronize()
        stats.t_first_arrival = min(r.arrival for r in requests)
        if not stats.latencies_s:
            stats.t_last_done = stats.t_first_arrival
        return stats

    def close(self):
        for e in self.lanes:
            e.close()


def poisson_requests(rate_hz: float, n: int, seed: int, pool, min_events: int = 100, max_events: int = 2000,
                     pinned: bool = False):
    """n requests with Poisson arrivals at `rate_hz` (first at t = 0) and sizes
    uniform in [min_events, max_events]; each slice is a run of consecutive
    events cut from the pre-drawn batch `pool` (a synth.EventBatch), wrapping
    around its end.  pinned: each request's features also arrive in
    page-locked host memory (as a producer writing into a pinned input ring
    would deliver them), so admission uploads them with one DMA and no host
    copy."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, n)
    sizes = rng.integers(min_events, max_events + 1, n)
    starts = rng.integers(0, pool.n_events, n)
    t = np.cumsum(gaps) - gaps[0]
    reqs = []
    for i in range(n):
        idx = [(int(starts[i]) + k) % pool.n_events for k in range(int(sizes[i]))]
        r = Request(i, pool.subset(idx), float(t[i]))
        if pinned:
            import torch
            r.feat_host = torch.from_numpy(r.batch.feat).pin_memory()
        reqs.append(r)
    return reqs
