"""Training loop of the learned window-kernel generator.

Every arithmetic step runs in the library (fdirw_nn_backward generates the
FP32 FD targets, runs the MFMA forward / backward and reduces the gradient;
fdirw_nn_adam updates the FP32 parameters).  This module only draws the
source indices of each batch and calls the ABI.

    python -m paper_2408_11376_amd.surrogate_train --n 64 --steps 400
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import Domain, NN_RADIUS, Surrogate


def train(nn: Surrogate, domains, steps: int, batch: int = 32, lr: float = 2e-3, seed: int = 0,
          lr_final: float | None = None, log_every: int = 0):
    """``steps`` Adam steps on batches of ``batch`` windows drawn uniformly
    over the cells of ``domains`` (a list of Domain with r = NN_RADIUS and the
    surrogate's n_sub).  The learning rate decays geometrically to
    ``lr_final`` (default: lr / 10).  Returns the per-step mean loss (KL, L1)."""
    import torch
    for d in domains:
        if d.r != NN_RADIUS or d.n_sub != nn.n_sub:
            raise ValueError("training domains must have r = NN_RADIUS and the surrogate's n_sub")
    rng = np.random.default_rng(seed)
    sizes = np.array([d.n for d in domains])
    lr_final = lr / 10 if lr_final is None else lr_final
    decay = (lr_final / lr) ** (1.0 / max(1, steps - 1))
    hist = []
    for k in range(steps):
        i = int(rng.integers(0, len(domains))) if len(domains) > 1 else 0
        src = torch.from_numpy(rng.integers(0, sizes[i], batch).astype(np.int64)).cuda()
        (kl, l1), _ = nn.backward(domains[i], src)
        nn.adam(lr * decay ** k)
        hist.append((kl, l1))
        if log_every and (k % log_every == 0 or k == steps - 1):
            print(json.dumps({"step": k, "kl": kl, "l1": l1}), flush=True)
    return hist


def main(argv=None):
    import synth                                  # seeded synthetic geometries
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--n", type=int, default=64, help="edge of the training geometries")
    ap.add_argument("--geometries", type=int, default=2)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--out", type=str, default="")
    a = ap.parse_args(argv)
    doms = [Domain.from_synth(synth.config2(seed=100 + i, n=a.n)) for i in range(a.geometries)]
    nn = Surrogate(doms[0].n_sub, seed=0)
    t = time.time()
    train(nn, doms, a.steps, a.batch, a.lr, log_every=max(1, a.steps // 10))
    print(json.dumps({"seconds": time.time() - t}))
    if a.out:
        nn.save(a.out)


if __name__ == "__main__":
    main()
