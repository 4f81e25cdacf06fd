"""One fused FDiRW step on a seeded porous grid, for profiler runs.

    python -m paper_2408_11376_amd.profile_step --n 96 --prec fp32 [--copy-mib 1024] [--gen nn] [--bank 1]
        [--coarse B] [--flow U]

Runs one untimed warm-up step, then ``--reps`` steps of the config-2 style
workload (GRF porous grid, r = 8, 200 sub-steps) at edge ``--n``.  With
``--copy-mib`` it also runs one plain device-to-device copy of that many MiB,
the reference for scaling HBM byte counters (FETCH_SIZE / WRITE_SIZE).
With ``--gen nn`` the steps use a surrogate (default initialisation, audit
disabled, so every kernel is the network's) instead of the FD kernels.  With
``--bank 1`` each repetition is instead one fdirw_run call that stores every
kernel once in a bank of the precision ``--prec`` (fp32, fp16_bank, ...) and
applies it for one big step.  With ``--coarse B`` the coarse-mesh operator
over B^3 blocks is built once (P stored in ``--prec``) and each repetition is
one coarse step, or with ``--ensemble E1,E2,..`` three ensemble products (P
in FP16) of each listed member count on seeded node fields.  With ``--mp K`` the integrated near-field solver of the
particle case (porous particle of radius 50 n / 192, Table 1 values, coarse
blocks of 5, P in ``--prec``) is built once and each repetition runs K big
steps (``--mp-r`` / ``--mp-nsub``: window radius and fast sub-steps of the
liquid's operator, 8 / 200 by default; 40 / 1000 is Table 1's big step).  With
``--flow U`` each repetition generates the window
kernels of a 64^3-cell sample of sources with a seeded steady flow of
magnitude up to U (fdirw_kernels_flow, precision ``--prec``).
"""
import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=96)
    ap.add_argument("--prec", default="fp32")
    ap.add_argument("--reps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--copy-mib", type=int, default=0)
    ap.add_argument("--tune", type=int, default=-1)
    ap.add_argument("--gen", default="fd", choices=["fd", "nn"])
    ap.add_argument("--bank", type=int, default=0)
    ap.add_argument("--coarse", type=int, default=0)
    ap.add_argument("--ensemble", default="")
    ap.add_argument("--flow", type=float, default=0.0)
    ap.add_argument("--mp", type=int, default=0)
    ap.add_argument("--mp-r", type=int, default=8)
    ap.add_argument("--mp-nsub", type=int, default=200)
    args = ap.parse_args()
    import torch
    import synth
    import paper_2408_11376_amd as fd
    d = synth.config2(n=args.n)
    dom = fd.Domain(d.label, d.d_phase, d.r, d.n_sub, d.h, d.dt)
    c = torch.from_numpy(d.c0).cuda()
    out = torch.empty_like(c)
    kw = {}
    if args.gen == "nn":
        kw = {"nn": fd.Surrogate(d.n_sub, seed=0), "audit_tol": 1e30, "audit_samples": 1}
    if args.flow > 0.0:
        u = torch.from_numpy((synth.uniform(99, 3 * d.n).reshape((3,) + d.shape) * 2.0 - 1.0) * args.flow).cuda()
        src = torch.arange(0, d.n, max(1, d.n // 262144), dtype=torch.int64, device="cuda")
        for i in range(args.reps):
            ev0 = torch.cuda.Event(enable_timing=True)
            ev1 = torch.cuda.Event(enable_timing=True)
            ev0.record()
            fd.fdirw_kernels_flow(dom, u, src, prec=args.prec)
            ev1.record()
            torch.cuda.synchronize()
            ms = ev0.elapsed_time(ev1)
            print(f"[profile_step] n={args.n} flow {args.flow} prec={args.prec} rep {i}: {src.numel()} kernels in "
                  f"{ms:.1f} ms", flush=True)
        args.reps = 0
        args.warmup = 0
    if args.mp:
        import numpy as np
        dp, t = synth.particle_case(args.n, 50.0 * args.n / 192.0, r=args.mp_r, n_sub=args.mp_nsub)
        far = dp.label == synth.PHASE_FAR_LIQUID
        m_total = float(dp.c0[~far].sum()) + t["V_ff_cells"] * t["c0_L"]
        s = fd.Multiphysics(fd.Domain.from_synth(dp), [fd.ROLE_LIQUID, fd.ROLE_SOLID, fd.ROLE_FAR_FIELD], t["k"],
                            t["c_eq_L"], t["c_eq_S"], t["V_ff_cells"],
                            a_over_rt=np.array([t["A_L_RT"], t["A_S_RT"], t["A_L_RT"]]), block=5, prec=args.prec)
        print(f"[profile_step] n={args.n} integrated prec={args.prec}: {s.n_nodes} nodes, {s.n_faces} faces, "
              f"build {s.build_seconds:.2f} s", flush=True)
        cp = torch.from_numpy(dp.c0).cuda()
        for i in range(args.reps):
            cff, hist, st = s.step(cp, t["c0_L"], m_total, args.mp, stats=True)
            print(f"[profile_step] integrated rep {i}: {args.mp} big steps, "
                  f"{st['kernel_seconds'] * 1e3 / args.mp:.4f} ms / step, Q_S {hist[-1, 1]:.4g}", flush=True)
        s.close()
        args.reps = 0
        args.warmup = 0
    if args.coarse:
        cg = fd.Coarse(dom, args.coarse, args.prec)
        print(f"[profile_step] n={args.n} coarse block {args.coarse} prec={args.prec}: {cg.n_nodes} nodes, "
              f"build {cg.build_seconds:.2f} s", flush=True)
        for i in range(args.reps if not args.ensemble else 0):
            _, st = cg.step(c, out, stats=True)
            print(f"[profile_step] coarse step {i}: kernels {st['kernel_seconds'] * 1e3:.3f} ms", flush=True)
        for E in [int(v) for v in args.ensemble.split(",") if v]:
            C = torch.from_numpy(synth.uniform(900 + E, E * cg.n_nodes).reshape(E, cg.n_nodes)).cuda()
            Co = torch.empty_like(C)
            for _ in range(3):
                _, ks = cg.apply_ensemble(C, Co, timed=True)
            print(f"[profile_step] ensemble E={E}: {ks * 1e3:.4f} ms", flush=True)
        cg.close()
        args.reps = 0
        args.warmup = 0
    if args.bank:
        for i in range(args.reps):
            cb = c.clone()
            _, st = fd.fdirw_run(dom, cb, 1, prec=args.prec, stats=True, bank_budget_bytes=1 << 40)
            print(f"[profile_step] n={args.n} bank prec={args.prec} rep {i}: bank used {st['bank_used']}, "
                  f"apply {st['kernel_seconds'] * 1e3:.2f} ms", flush=True)
            fd.fdirw_release()
        args.reps = 0
        args.warmup = 0
    for _ in range(args.warmup):
        fd.fdirw_step(dom, c, out, prec=args.prec, tune=args.tune, **kw)
    torch.cuda.synchronize()
    for i in range(args.reps):
        _, st = fd.fdirw_step(dom, c, out, prec=args.prec, stats=True, tune=args.tune, **kw)
        print(f"[profile_step] n={args.n} prec={args.prec} gen={args.gen} rep {i}: "
              f"kernel {st['kernel_seconds'] * 1e3:.2f} ms, wall {st['seconds'] * 1e3:.2f} ms", flush=True)
    if args.copy_mib > 0:
        nbytes = args.copy_mib << 20
        a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(f"[profile_step] copied {args.copy_mib} MiB", flush=True)


if __name__ == "__main__":
    main()
