"""Filter training on crops with the hand-written gradient kernels.

The linear window filter of the detector (Sec. IV-A, linear classification
filter) is trained by full-batch gradient descent on 80x80 crops (one
window each): forward window scores, hinge loss + l2 * ||W||^2 and its
score gradient, then the filter gradient with features recomputed from
the crops.  Every step runs in libhog355 kernels; torch only holds the
tensors and applies the update.

    python -m paper_2006_00816_amd.train [--steps 50] [--lr 0.5]
"""
from __future__ import annotations

import argparse
import json
import time

import torch

from . import hog355, synth


def train(crops: torch.Tensor, labels: torch.Tensor, W: torch.Tensor, b: torch.Tensor, steps: int = 50,
          lr: float = 0.5, l2: float = 1e-4, log=None):
    """Full-batch gradient descent; returns the loss history."""
    n = int(crops.shape[0])
    win = hog355.windows_tensor(torch.arange(n, dtype=torch.int32), 0, 0, 0, 0, crops.device)
    ws = hog355.Workspace()
    hist = []
    for step in range(steps):
        s = hog355.window_scores(crops, W, b, win, ws=ws)
        loss, dscore, dW = hog355.hinge_loss(s, labels, W, l2)
        dW, db, _ = hog355.filter_backward(crops, W, win, dscore, dW=dW, ws=ws)
        W.sub_(lr * dW)
        b.sub_(lr * db)
        hist.append(float(loss.item()))
        if log:
            log(step, hist[-1])
    return hist


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--lr", type=float, default=0.5)
    ap.add_argument("--pos", type=int, default=4096)
    ap.add_argument("--neg", type=int, default=16384)
    args = ap.parse_args()
    crops, labels = synth.config3(seed=3, n_pos=args.pos, n_neg=args.neg)
    W0, b0 = synth.filters([3])
    crops_t = torch.from_numpy(crops).cuda()
    labels_t = torch.from_numpy(labels).cuda()
    W = torch.from_numpy(W0).cuda()
    b = torch.from_numpy(b0).cuda()
    t0 = time.perf_counter()
    hist = train(crops_t, labels_t, W, b, args.steps, args.lr)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    s = hog355.window_scores(crops_t, W, b,
                             hog355.windows_tensor(torch.arange(len(crops), dtype=torch.int32), 0, 0, 0, 0))
    acc = float(((s > 0).float() * 2 - 1 == labels_t).float().mean())
    print(json.dumps({"steps": args.steps, "crops": len(crops), "loss_first": hist[0], "loss_last": hist[-1],
                      "train_accuracy": acc, "ms_per_step": 1e3 * dt / args.steps}))


if __name__ == "__main__":
    main()
