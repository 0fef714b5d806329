"""Continuous-batching detection server.

Frames of mixed resolutions arrive as requests (here replayed from
Poisson arrival times).  The server keeps the filters, the pyramid
workspaces and the frame buffers resident on the device.  A slot is a
stream with a device slab of `slab_bytes` for the frames and pyramid
buffers (workspace) of one batch.  Requests are admitted by bytes: as soon
as a slot frees up, the waiting frames of one resolution (oldest first)
join its batch for as long as the batch's frames and pyramid buffers,
hog_workspace_bytes of that resolution and batch size, fit the slab; so a
slab holds more small frames than large ones.  The batch is copied host to
device asynchronously, detected with hog_detect_batch and its detections
copied back, all on the slot's stream; batches on different slots overlap
on the GPU while new requests keep arriving.  The detection of each
(resolution, batch size) that fits is captured once per slot as a hipGraph
over the slab (at start-up), so a batch costs one graph launch instead of
a launch per kernel.  Latency is completion time minus arrival time.

    python -m paper_2006_00816_amd.serve --rates 500,2000,8000 --seconds 60
"""
from __future__ import annotations

import argparse
import collections
import dataclasses
import gc
import json
import time

import numpy as np
import torch

from . import hog355, synth


@dataclasses.dataclass
class Request:
    rid: int
    shape: tuple
    frame: torch.Tensor          # pinned host uint8 [h][w]
    arrival: float               # seconds on the server clock
    done: float = -1.0
    batch_index: int = -1        # position in the batch it ran in (its detections' frame field)
    n_dets: int = 0
    dets: np.ndarray = None


def _align(v, a=256):
    return (v + a - 1) // a * a


def batch_bytes(h: int, w: int, n: int, nf: int) -> int:
    """Device bytes of a batch of n frames of h x w in a slab: the frames,
    then the pyramid buffers (hog_workspace_bytes)."""
    return _align(n * h * w) + hog355.workspace_bytes(h, w, 1, n, nf)


def batch_limit(h: int, w: int, nf: int, slab_bytes: int, max_batch: int) -> int:
    """The largest batch of h x w frames whose bytes fit a slab (0: none)."""
    n = 0
    while n < max_batch and batch_bytes(h, w, n + 1, nf) <= slab_bytes:
        n += 1
    return n


class _Slot:
    def __init__(self, max_batch, slab_bytes, cap, device):
        self.stream = torch.cuda.Stream(device=device)
        self.slab = torch.empty(slab_bytes, dtype=torch.uint8, device=device)
        self.graphs = {}
        self.dets = torch.empty((max_batch, cap, 10), dtype=torch.int32, device=device)
        self.n_dets = torch.empty(max_batch, dtype=torch.int32, device=device)
        self.h_dets = torch.empty((max_batch, cap, 10), dtype=torch.int32).pin_memory()
        self.h_n = torch.empty(max_batch, dtype=torch.int32).pin_memory()
        self.event = torch.cuda.Event()
        self.batch = None


class HogServer:
    def __init__(self, W: torch.Tensor, b: torch.Tensor, shapes, max_batch: int = 16, slots: int = 4,
                 cap: int = 256, thresh: float = 0.0, iou: float = 0.5, device="cuda", slab_bytes: int = 64 << 20):
        self.W, self.b = W, b
        self.max_batch, self.cap, self.thresh, self.iou = max_batch, cap, thresh, iou
        nf = int(W.shape[0])
        # admission by bytes: the batch sizes of each resolution that fit a slab
        self.limit = {tuple(s): batch_limit(s[0], s[1], nf, slab_bytes, max_batch) for s in shapes}
        too_big = [s for s, n in self.limit.items() if n == 0]
        if too_big:
            raise ValueError(f"slab of {slab_bytes} bytes holds no frame of {too_big}")
        self.slab_bytes = slab_bytes
        self.slots = [_Slot(max_batch, slab_bytes, cap, device) for _ in range(slots)]
        for slot in self.slots:
            slot.slab.zero_()
        torch.cuda.synchronize()
        for slot in self.slots:
            for (h, w), nmax in self.limit.items():
                for n in range(1, nmax + 1):
                    fr = slot.slab[:n * h * w].view(n, h, w)
                    ws = slot.slab[_align(n * h * w):]
                    slot.graphs[(h, w, n)] = hog355.BoundGraph(fr, W, b, slot.dets[:n], slot.n_dets[:n], ws,
                                                               thresh, iou, 1, slot.stream)
        # one replay of every graph (on blank frames) and one pass of every
        # copy and event on each slot's stream before serving, so that no
        # request pays for a first use
        max_bytes = max(h * w for h, w in shapes)
        blank = torch.zeros(max_bytes, dtype=torch.uint8).pin_memory()
        for slot in self.slots:
            with torch.cuda.stream(slot.stream):
                slot.slab[:max_bytes].copy_(blank, non_blocking=True)
                for g in slot.graphs.values():
                    g.launch(slot.stream)
                slot.h_dets.copy_(slot.dets, non_blocking=True)
                slot.h_n.copy_(slot.n_dets, non_blocking=True)
                slot.event.record(slot.stream)
            slot.event.query()
        torch.cuda.synchronize()
        self.pending = collections.OrderedDict((tuple(s), collections.deque()) for s in shapes)
        self.completed = []
        self.batches = 0

    def submit(self, req: Request):
        self.pending[req.shape].append(req)

    def _launch(self, slot: _Slot, reqs):
        h, w = reqs[0].shape
        n = len(reqs)
        with torch.cuda.stream(slot.stream):
            fr = slot.slab[:n * h * w].view(n, h, w)
            for i, r in enumerate(reqs):
                fr[i].copy_(r.frame, non_blocking=True)
            slot.graphs[(h, w, n)].launch(slot.stream)
            slot.h_dets[:n].copy_(slot.dets[:n], non_blocking=True)
            slot.h_n[:n].copy_(slot.n_dets[:n], non_blocking=True)
            slot.event.record(slot.stream)
        slot.batch = reqs
        self.batches += 1

    def pump(self, now_fn) -> int:
        """Retire finished batches, then fill free slots; returns the number
        of requests in flight."""
        for slot in self.slots:
            if slot.batch is not None and slot.event.query():
                t = now_fn()
                for i, r in enumerate(slot.batch):
                    r.done = t
                    r.batch_index = i
                    r.n_dets = int(slot.h_n[i])
                    m = min(r.n_dets, self.cap)
                    r.dets = slot.h_dets[i, :m].numpy().copy().view(hog355.DET_DTYPE).reshape(m)
                    self.completed.append(r)
                slot.batch = None
        for slot in self.slots:
            if slot.batch is not None:
                continue
            # the resolution whose oldest waiting request arrived first
            best = None
            for shape, q in self.pending.items():
                if q and (best is None or q[0].arrival < self.pending[best][0].arrival):
                    best = shape
            if best is None:
                break
            q = self.pending[best]
            # as many of them as the slab's bytes hold
            reqs = [q.popleft() for _ in range(min(len(q), self.limit.get(best, self.max_batch)))]
            self._launch(slot, reqs)
        return sum(len(s.batch) for s in self.slots if s.batch is not None)


def run_stream(server: HogServer, frames, shapes, arrivals):
    """Replay requests at their arrival times (seconds from start) and wait
    for all of them; returns the completed requests.  The garbage
    collector is paused while serving (a full collection over the request
    objects stalls the loop for tens of milliseconds)."""
    gc.collect()
    paused = gc.isenabled()
    gc.disable()
    try:
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0
        i = 0
        n = len(arrivals)
        while i < n or server.pump(now) or any(server.pending.values()):
            t = now()
            while i < n and arrivals[i] <= t:
                server.submit(Request(i, shapes[i], frames[i], float(arrivals[i])))
                i += 1
            server.pump(now)
    finally:
        if paused:
            gc.enable()
    return sorted(server.completed, key=lambda r: r.rid)


def served_stream(rate: float, seconds: float, W, b, pools_pinned, seed: int = 2, max_batch: int = 16, slots: int = 4,
                  slab_bytes: int = 64 << 20):
    t, res = synth.poisson_arrivals(seed, rate, seconds)
    shapes = [tuple(r) for r in res]
    idx = collections.Counter()
    frames = []
    for s in shapes:
        pool = pools_pinned[s]
        frames.append(pool[idx[s] % len(pool)])
        idx[s] += 1
    server = HogServer(W, b, list(pools_pinned.keys()), max_batch=max_batch, slots=slots, slab_bytes=slab_bytes)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    done = run_stream(server, frames, shapes, t)
    wall = time.perf_counter() - t_start
    lat = np.array([r.done - r.arrival for r in done]) * 1e3
    return {"rate": rate, "seconds": seconds, "frames": len(done),
            "fps": len(done) / wall, "p50_ms": float(np.percentile(lat, 50)) if len(lat) else None,
            "p99_ms": float(np.percentile(lat, 99)) if len(lat) else None,
            "batches": server.batches, "mean_batch": len(done) / max(server.batches, 1),
            "slab_bytes": server.slab_bytes, "slots": slots,
            "batch_limit": {f"{h}x{w}": n for (h, w), n in server.limit.items()}}, done, frames


def pinned_pools(per_res: int = 64, seed: int = 2):
    pools, W, b = synth.config2_pools(seed, per_res)
    out = {s: [torch.from_numpy(f).pin_memory() for f in fr] for s, fr in pools.items()}
    return out, torch.from_numpy(W).cuda(), torch.from_numpy(b).cuda()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--rates", default="500,2000,8000")
    ap.add_argument("--seconds", type=float, default=60.0)
    ap.add_argument("--pool", type=int, default=256)
    args = ap.parse_args()
    pools, W, b = pinned_pools(args.pool)
    for rate in (float(r) for r in args.rates.split(",")):
        stats, _, _ = served_stream(rate, args.seconds, W, b, pools)
        print(json.dumps(stats), flush=True)


if __name__ == "__main__":
    main()
