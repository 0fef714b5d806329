"""Schedule autotuner cache for hog_detect_batch.

The library's autotuner (hog_autotune) times the per-stage schedule and
the fused persistent kernel under several work-list settings on real
frames and keeps the fastest for the shape in the process.  This module
persists those choices as JSON keyed by (h, w, upsample, n, nf, arch), and
re-applies them in a later process before any detection call:

    python -m paper_2006_00816_amd.autotune --h 480 --w 640 --n 64 --nf 5
"""
from __future__ import annotations

import argparse
import json
import os

import torch

from . import hog355

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "hog355_tuning.json")


def _arch(device=0) -> str:
    return str(torch.cuda.get_device_properties(device).gcnArchName).split(":")[0]


def _key(h, w, upsample, n, nf, arch) -> str:
    return f"{h}x{w}/u{upsample}/n{n}/nf{nf}/{arch}"


def load(path: str = DEFAULT_CACHE) -> dict:
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def save(entries: dict, path: str = DEFAULT_CACHE):
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(entries, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def apply(path: str = DEFAULT_CACHE, device=0) -> int:
    """Install every cached schedule for this device's architecture; returns
    how many were applied."""
    arch = _arch(device)
    count = 0
    for e in load(path).values():
        if e.get("arch") != arch:
            continue
        hog355.tuning_set(e["h"], e["w"], e["upsample"], e["n"], e["nf"], e["tuning"])
        count += 1
    return count


def tune(frames: torch.Tensor, W: torch.Tensor, b: torch.Tensor, upsample: int = 1, reps: int = 5,
         path: str | None = DEFAULT_CACHE, **kw):
    """Autotune hog_detect_batch for these frames' shape; the choice is in
    effect at once and, with a path, stored in the cache."""
    n, h, w = (int(v) for v in frames.shape)
    nf = int(W.shape[0])
    best, ms = hog355.autotune(frames, W, b, upsample=upsample, reps=reps, **kw)
    if path:
        entries = load(path)
        arch = _arch(frames.device.index or 0)
        entries[_key(h, w, upsample, n, nf, arch)] = {"h": h, "w": w, "upsample": upsample, "n": n, "nf": nf,
                                                      "arch": arch, "tuning": best, "ms": ms}
        save(entries, path)
    return best, ms


def main():
    from . import synth
    ap = argparse.ArgumentParser()
    ap.add_argument("--h", type=int, default=480)
    ap.add_argument("--w", type=int, default=640)
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--nf", type=int, default=5)
    ap.add_argument("--upsample", type=int, default=1)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--cache", default=DEFAULT_CACHE)
    a = ap.parse_args()
    gen = synth.ClipGenerator(1, a.h, a.w)
    frames = torch.from_numpy(gen.frames(a.n)).cuda()
    W, b = synth.filters(list(range(101, 101 + a.nf)))
    best, ms = tune(frames, torch.from_numpy(W).cuda(), torch.from_numpy(b).cuda(), a.upsample, a.reps, a.cache)
    print(json.dumps({"tuning": best, "ms_per_call": ms}))


if __name__ == "__main__":
    main()
