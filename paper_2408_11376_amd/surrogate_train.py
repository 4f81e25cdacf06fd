"""Training loop of the learned window-kernel generator.

Every arithmetic step runs in the library (fdirw_nn_backward generates the
FP32 FD targets, runs the MFMA forward / backward and reduces the gradient;
fdirw_nn_adam updates the FP32 parameters).  This module only draws the
source indices of each batch and calls the ABI.

    python -m paper_2408_11376_amd.surrogate_train --n 64 --steps 400

The recipe of the surrogate workload (``--recipe grf192``): a fixed set of
``--windows`` FD windows (200,000) drawn uniformly from ``--geometries`` (8)
seeded 192^3 GRF geometries of the benchmark's kind (seeds 100, 101, ...),
``--epochs`` passes over it in a seeded random order at batch 256 with a
geometrically decaying learning rate, and the mean per-kernel L1 error on
``--eval-windows`` sources of each unseen 192^3 geometry (seeds 200, 201)
after every epoch, next to the prior's (the network's input log U alone).
One JSON line per epoch; ``--out`` saves the parameters with the lowest
evaluation error.
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


def fixed_windows(domains, count: int, seed: int):
    """(domain index, source) pairs of a fixed training set: count // len
    sources per domain, uniform over its cells (seeded)."""
    rng = np.random.default_rng(seed)
    per = count // len(domains)
    return [(i, rng.integers(0, d.n, per).astype(np.int64)) for i, d in enumerate(domains)]


def evaluate(nn: Surrogate, domains, srcs, batch: int = 256):
    """Mean per-kernel L1 term of the loss (sum |q - G| over the support,
    q the normalised FP32 FD kernel) over the sources srcs[i] of domains[i]."""
    import torch
    tot, cnt = 0.0, 0
    for d, s in zip(domains, srcs):
        for a in range(0, len(s), batch):
            b = torch.from_numpy(s[a:a + batch]).cuda()
            (_, l1), _ = nn.backward(d, b)
            tot += l1 * b.numel()
            cnt += b.numel()
    return tot / cnt


def prior_l1(domains, srcs, n_sub: int, batch: int = 256):
    """The same statistic for the prior alone (a network whose output is 0)."""
    from . import fdirw_nn_num_params
    z = Surrogate(n_sub, seed=0)
    z.set_params(np.zeros(fdirw_nn_num_params(), dtype=np.float32))
    try:
        return evaluate(z, domains, srcs, batch)
    finally:
        z.close()


def train_recipe(nn: Surrogate, domains, eval_domains, windows: int = 200_000, epochs: int = 10,
                 batch: int = 256, lr: float = 2e-3, lr_final: float = 1e-4, eval_windows: int = 1024,
                 seed: int = 0, out: str = "", log=print):
    """Epochs over a fixed set of FD windows; returns the per-epoch records."""
    import torch
    rng = np.random.default_rng(seed + 1)
    sets = fixed_windows(domains, windows, seed)
    ev_src = [np.random.default_rng(seed + 2 + i).integers(0, d.n, eval_windows).astype(np.int64)
              for i, d in enumerate(eval_domains)]
    steps_per_epoch = sum(len(s) // batch for _, s in sets)
    total = steps_per_epoch * epochs
    decay = (lr_final / lr) ** (1.0 / max(1, total - 1))
    rec = []
    best = float("inf")
    p_l1 = prior_l1(eval_domains, ev_src, nn.n_sub)
    e0 = evaluate(nn, eval_domains, ev_src)
    log(json.dumps({"epoch": 0, "eval_l1": e0, "prior_eval_l1": p_l1, "steps_per_epoch": steps_per_epoch}))
    k = 0
    t0 = time.time()
    for ep in range(1, epochs + 1):
        # every batch holds windows of one geometry (one call per batch);
        # windows shuffled within each geometry, batches in a random order
        batches = []
        for i, s in sets:
            p = rng.permutation(s)
            batches += [(i, p[j * batch:(j + 1) * batch]) for j in range(len(s) // batch)]
        kl_sum = l1_sum = 0.0
        for j in rng.permutation(len(batches)):
            di, src = batches[j]
            (kl, l1), _ = nn.backward(domains[di], torch.from_numpy(src).cuda())
            nn.adam(lr * decay ** k)
            kl_sum += kl
            l1_sum += l1
            k += 1
        ev = evaluate(nn, eval_domains, ev_src)
        r = {"epoch": ep, "steps": k, "train_kl": kl_sum / steps_per_epoch, "train_l1": l1_sum / steps_per_epoch,
             "eval_l1": ev, "prior_eval_l1": p_l1, "lr": lr * decay ** (k - 1), "seconds": time.time() - t0}
        rec.append(r)
        log(json.dumps(r))
        if out and ev < best:
            best = ev
            nn.save(out)
    return rec


def analyze(nn: Surrogate, domains, count: int = 512, seed: int = 7):
    """Where the error of a network sits, on ``count`` sources per domain:
    the mean per-kernel L1 (the loss's L1 term) over pore sources and over
    solid sources separately (fdirw_nn_backward), and for pore sources the
    share of sum |G_nn - q| that lies in the cells farther than 5 cells (the
    network's receptive-field radius: five 3^3 layers) from the source in the
    max norm, next to the share of the FD kernel's mass there (host arithmetic
    on the kernels of fdirw_nn_forward and fdirw_kernels; a report, not part of
    the path)."""
    import torch
    from . import fdirw_kernels, FP32
    rng = np.random.default_rng(seed)
    out = {"pore_l1": [], "solid_l1": [], "far_err_share": [], "far_mass_share": []}
    W = 2 * NN_RADIUS + 1
    z, y, x = np.meshgrid(*[np.arange(W) - NN_RADIUS] * 3, indexing="ij")
    far = np.maximum(np.maximum(np.abs(z), np.abs(y)), np.abs(x)) > 5
    for d in domains:
        lab = d.label.cpu().numpy().reshape(-1) if hasattr(d.label, "cpu") else np.asarray(d.label).reshape(-1)
        dph = np.asarray(d.d_phase)
        src = rng.integers(0, d.n, 8 * count).astype(np.int64)
        solid = dph[lab[src]] < 1e-3 * dph.max()
        for key, sel in (("pore_l1", ~solid), ("solid_l1", solid)):
            ss = src[sel][:count]
            if len(ss):
                (_, l1), _ = nn.backward(d, torch.from_numpy(ss).cuda())
                out[key].append(l1)
        ss = torch.from_numpy(src[~solid][:count]).cuda()
        Gn = nn.forward(d, ss)["G"].double().cpu().numpy()
        Gf, m = fdirw_kernels(d, ss, prec=FP32)
        q = Gf.double().cpu().numpy() / m.cpu().numpy()[:, None, None, None]
        e = np.abs(Gn - q)
        out["far_err_share"].append(float((e[:, far].sum(axis=1) / e.reshape(len(ss), -1).sum(axis=1)).mean()))
        out["far_mass_share"].append(float(q[:, far].sum(axis=1).mean()))
    return {k: float(np.mean(v)) for k, v in out.items() if v}


def main(argv=None):
    import synth                                  # seeded synthetic geometries
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--n", type=int, default=64, help="edge of the training geometries")
    ap.add_argument("--geometries", type=int, default=2)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--out", type=str, default="")
    ap.add_argument("--recipe", type=str, default="", help="grf192: the surrogate workload's recipe")
    ap.add_argument("--windows", type=int, default=200_000)
    ap.add_argument("--epochs", type=int, default=10)
    ap.add_argument("--eval-windows", type=int, default=1024)
    ap.add_argument("--lr-final", type=float, default=1e-4)
    ap.add_argument("--analyze", type=str, default="", help="parameter file: report where its error sits")
    a = ap.parse_args(argv)
    if a.analyze:
        evs = [Domain.from_synth(synth.config2(seed=200 + i, n=192)) for i in range(2)]
        nn = Surrogate(evs[0].n_sub, seed=0)
        nn.load(a.analyze)
        print(json.dumps({"trained": analyze(nn, evs)}), flush=True)
        from . import fdirw_nn_num_params
        nn.set_params(np.zeros(fdirw_nn_num_params(), dtype=np.float32))
        print(json.dumps({"prior": analyze(nn, evs)}), flush=True)
        return
    if a.recipe == "grf192":
        t = time.time()
        doms = [Domain.from_synth(synth.config2(seed=100 + i, n=192)) for i in range(a.geometries)]
        evs = [Domain.from_synth(synth.config2(seed=200 + i, n=192)) for i in range(2)]
        print(json.dumps({"geometries_seconds": time.time() - t}), flush=True)
        nn = Surrogate(doms[0].n_sub, seed=0)
        train_recipe(nn, doms, evs, windows=a.windows, epochs=a.epochs, batch=a.batch, lr=a.lr,
                     lr_final=a.lr_final, eval_windows=a.eval_windows, out=a.out,
                     log=lambda m: print(m, flush=True))
        return
    doms = [Domain.from_synth(synth.config2(seed=100 + i, n=a.n)) for i in range(a.geometries)]
    nn = Surrogate(doms[0].n_sub, seed=0)
    t = time.time()
    train(nn, doms, a.steps, a.batch, a.lr, log_every=max(1, a.steps // 10))
    print(json.dumps({"seconds": time.time() - t}))
    if a.out:
        nn.save(a.out)


if __name__ == "__main__":
    main()
