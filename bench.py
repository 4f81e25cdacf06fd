#!/usr/bin/env python3
"""Benchmark of the fused FDiRW big step on one MI355X.

Workload (the configuration the headline metric is quoted on): a 192^3 porous
grid from a thresholded Gaussian random field (correlation length 6 voxels,
solid fraction 0.35), D_pore = 1, D_solid = 1e-6, window radius r = 8
(17^3 window), 200 explicit sub-steps per big step, c0 ~ U[0, 1]; every one of
the 7,077,888 cells is a source.  Synthetic and seeded (the paper's
phase-field particle geometry is not available).

A "step" is one fdirw_step call: coefficients, kernel generation for every
source, FP64 scatter-add superposition and the FP64 mass balance.  Steps are
chained (output -> next input).  ``value`` = 192^3 cells / seconds per step in
the headline precision (default FP32, the fastest fused mode on gfx950); the
mixed precision steps (FP32 state with FP16 or BF16 neighbour copies) are timed
the same way and reported under ``modes`` with their speedup over FP32 and
their relative L1 difference from the FP32 field; the ``deterministic`` leg
times the FP32 step without floating-point atomics (bitwise repeatable).
The ``bank`` leg stores
every kernel once (in FP32 and in FP16, the paper's stored-P use) and times
the HBM-streaming apply of one big step; the ``coarse`` leg runs the paper's
coarse-mesh method (5^3 blocks, mapping / P C / remapping) in the four
precisions of its Table 2 (FP64, FP32, mixed FP32/FP16, FP16).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--prec fp32] [--nn-epochs E]

The learned generator (surrogate) is trained for E epochs of its recipe
(200,000 FD windows of eight other seeded 192^3 geometries of the same kind,
evaluated on two unseen ones) and its step is timed under ``modes`` as "nn":
the audited step as the library runs it (audit L1 and fallback flag) and the
surrogate-only step with its speedup and field error.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

# MI355X published peaks
PEAK_FP32_VECTOR_TFLOPS = 157.3
# The FP32 FMA rate without packed FP32 instructions (the library is compiled
# without them): 256 CUs x 4 SIMDs x 16 lanes x 2 flop x 2.4 GHz.
PEAK_FP32_UNPACKED_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0
# Algorithmic work of one cell-sub-step of the 7-point update: 7 products and
# 6 additions (13 flop); exchange: one write and four in-plane reads of the
# neighbour copy (the two z neighbours stay in registers).
FLOP_PER_CELL_SUBSTEP = 13
LDS_ACCESSES_PER_CELL_SUBSTEP = 5
FMA_PER_CELL_SUBSTEP = 7
# Chip rates for the secondary ceilings of the fused kernel: 256 CUs at
# 2.4 GHz; one FP32 FMA per lane per clock on 4 x 16 lanes per CU (packed FP32
# is not used); LDS rates measured on the MI355X with a microbenchmark:
# 128-bit reads ~198 B/clk/CU, writes ~75 B/clk/CU.
CU_HZ = 256 * 2.4e9
LDS_READ_B_PER_CLK = 198.0
LDS_WRITE_B_PER_CLK = 75.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def window_cells(shape, r):
    """Sum over sources of the number of in-domain cells of its window
    (separable: product over axes of sum over positions of clipped lengths)."""
    total = 1
    for n in shape:
        s = sum(min(n - 1, p + r) - max(0, p - r) + 1 for p in range(n))
        total *= s
    return total


def kernel_source_hash():
    """Hash of the sources that define the fused line kernel."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2408_11376_amd", "csrc")
    for f in ("fdirw_device.h", "fdirw_kernels.hip", "fdirw_flat.hip"):
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def read_profile_values(kernel_tag, suffix, keys):
    """Values from a committed rocprofv3 counter summary
    (profiles/<kernel_tag>_<suffix>.md, lines "key: value"), if it was taken
    on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", f"{kernel_tag}_{suffix}.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_hash = re.search(r"source_sha:\s*([0-9a-f]+)", text)
    if not m_hash or m_hash.group(1) != kernel_source_hash():
        return None
    out = {}
    for k in keys:
        m = re.search(rf"{k}:\s*([0-9.eE+-]+)", text)
        if not m:
            return None
        out[k] = float(m.group(1))
    return out


def read_traffic(kernel_tag):
    """HBM bytes per launch from the committed rocprofv3 counter summary."""
    v = read_profile_values(kernel_tag, "traffic", ["hbm_bytes_per_launch"])
    return None if v is None else v["hbm_bytes_per_launch"]


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(dom, block: int):
    """The CPU oracle on a bounded sample: c0 kept only on a block^3 cube of
    sources (the oracle skips zero sources), so the sample is block^3 kernels
    of the same workload.  cells/s = sources per second (a full step is one
    source per cell)."""
    import oracle
    p = oracle.Problem.from_domain(dom)
    import synth
    m = synth.sub_block_sources(dom.shape, block)
    c0 = np.where(m, dom.c0, 0.0)
    t = time.perf_counter()
    _, used, _ = p.step(c0)
    dt = time.perf_counter() - t
    out = {"value": used / dt, "unit": "cells/s", "cores": oracle.num_threads(), "kind": "oracle",
           "cpu_model": cpu_model(),
           "sample": f"{block}^3 = {used} sources of the {dom.shape[0]}^3 step (c0 zeroed elsewhere), {dt:.2f} s"}
    # one core (the paper's CPU reference is one core): a smaller cube of sources
    b1 = max(2, block // 3)
    m1 = synth.sub_block_sources(dom.shape, b1)
    threads = oracle.num_threads()
    oracle.set_num_threads(1)
    try:
        t = time.perf_counter()
        _, used1, _ = p.step(np.where(m1, dom.c0, 0.0))
        dt1 = time.perf_counter() - t
    finally:
        oracle.set_num_threads(threads)
    out["value_1core"] = used1 / dt1
    out["sample_1core"] = f"{b1}^3 = {used1} sources on 1 thread, {dt1:.2f} s"
    return out


def surrogate_mode(fd, d, dom, c0, bufs, stream, args):
    """Train the learned generator on the surrogate workload's recipe (a fixed
    set of 200,000 FD windows from eight seeded 192^3 GRF geometries of the
    benchmark's kind, batch 256, decaying learning rate; ``--nn-epochs``
    passes), with its per-kernel L1 on two unseen 192^3 geometries next to the
    prior's; then time its step on the workload: the audited step as the
    library runs it (falls back to FD when the mean per-kernel L1 of 1024
    audited sources exceeds 1e-3) and the surrogate-only step (audit off)
    with its field error against the FP32 FD step."""
    import torch
    import synth
    from paper_2408_11376_amd.surrogate_train import train_recipe
    log(f"nn: {args.nn_epochs} epochs of the 200k-window recipe on eight 192^3 GRF geometries")
    nn = fd.Surrogate(d.n_sub, seed=0)
    tdoms = [fd.Domain.from_synth(synth.config2(seed=100 + i, n=192)) for i in range(8)]
    edoms = [fd.Domain.from_synth(synth.config2(seed=200 + i, n=192)) for i in range(2)]
    t = time.perf_counter()
    rec = train_recipe(nn, tdoms, edoms, windows=200_000, epochs=args.nn_epochs, batch=256, lr=2e-3,
                       lr_final=1e-4, eval_windows=1024, log=lambda m: log(f"nn: {m}"))
    train_s = time.perf_counter() - t
    del tdoms, edoms
    out = {"train_epochs": args.nn_epochs, "train_windows": 200_000, "train_seconds": train_s,
           "eval_l1_unseen": rec[-1]["eval_l1"], "prior_eval_l1_unseen": rec[-1]["prior_eval_l1"],
           "eval_l1_per_epoch": [r["eval_l1"] for r in rec]}
    # the audited step (what fdirw_step with GEN_NN does)
    _, st = fd.fdirw_step(dom, c0, bufs[0], nn=nn, stats=True)
    out["audit_l1"] = st["audit_l1"]
    out["fallback_used"] = st["fallback_used"]
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.steps):
        fd.fdirw_step(dom, c0, bufs[0], nn=nn)
    torch.cuda.synchronize()
    out["audited_ms_per_step"] = 1e3 * (time.perf_counter() - t) / args.steps
    # surrogate-only step
    kw = {"nn": nn, "audit_tol": 1e30, "audit_samples": 1}
    for _ in range(args.warmup):
        fd.fdirw_step(dom, c0, bufs[0], **kw)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    kern = []
    cur = c0
    ev0.record(stream)
    for k in range(args.steps):
        o = bufs[k % 2]
        _, st = fd.fdirw_step(dom, cur, o, stats=True, **kw)
        kern.append(st["kernel_seconds"])
        cur = o
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    first, st = fd.fdirw_step(dom, c0, torch.empty_like(c0), stats=True, **kw)
    out.update({"cells_per_s": d.n / (ms * 1e-3), "ms_per_step": ms, "kernel_ms": 1e3 * float(np.mean(kern)),
                "mass_rel_drift": abs(st["mass_out"] - st["mass_in"]) / st["mass_in"],
                "kernel_mass_range": [st["kmass_min"], st["kmass_max"]], "sources": st["n_sources"]})
    log(f"nn: audit L1 {out['audit_l1']:.4f} (fallback {out['fallback_used']}), surrogate-only {ms:.1f} ms/step")
    return out, first


def batched_leg(fd, args):
    """The batched workload: 64 GRF domains (edges 32..128, r in {4, 6, 8},
    contrast 1e2..1e6) in one persistent launch per step, FP32, autotuned
    (the first call tunes; the timed calls reuse the cached choice)."""
    import torch
    import synth
    log("batched: generating 64 domains")
    ds = synth.config3()
    doms = [fd.Domain.from_synth(x) for x in ds]
    cin = [torch.from_numpy(x.c0).cuda() for x in ds]
    cout = [torch.empty_like(c) for c in cin]
    cells = sum(x.n for x in ds)
    cs = sum(window_cells(x.shape, x.r) * x.n_sub for x in ds)
    _, st = fd.fdirw_step(doms, cin, cout, prec="fp32", stats=True, tune=-1)     # tunes
    torch.cuda.synchronize()
    t = time.perf_counter()
    kern = []
    for _ in range(args.steps):
        _, st = fd.fdirw_step(doms, cin, cout, prec="fp32", stats=True, tune=-1)
        kern.append(st[0]["kernel_seconds"])
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t) / args.steps
    drift = max(abs(x["mass_out"] - x["mass_in"]) / x["mass_in"] for x in st)
    out = {"domains": len(ds), "cells": cells, "cell_substeps": cs, "ms_per_step": ms,
           "kernel_ms": 1e3 * float(np.mean(kern)), "cells_per_s": cells / (ms * 1e-3),
           "cell_substeps_per_s": cs / (ms * 1e-3), "tuned_config_id": st[0]["tuned_config_id"],
           "mass_rel_drift_max": drift}
    log(f"batched: {ms:.1f} ms/step, {out['cells_per_s'] / 1e6:.3f} Mcells/s, "
        f"{out['cell_substeps_per_s'] / 1e12:.3f} T cell-substeps/s, shape {out['tuned_config_id']}")
    return out


def deterministic_leg(fd, d, dom, c0, bufs, stream, ref, args):
    """The headline step with deterministic = 1 (no floating-point atomics:
    completed planes to partial slots, then a fixed-order reduction), timed
    like the modes; its field from c0 twice (bitwise equal) and its relative
    L1 difference from the atomic FP32 field."""
    import torch
    log(f"deterministic fp32: {args.warmup} warm-up + {args.steps} timed steps")
    for _ in range(args.warmup):
        fd.fdirw_step(dom, c0, bufs[0], prec="fp32", deterministic=True)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    kern = []
    cur = c0
    ev0.record(stream)
    for k in range(args.steps):
        out = bufs[k % 2]
        _, st = fd.fdirw_step(dom, cur, out, prec="fp32", stats=True, deterministic=True)
        kern.append(st["kernel_seconds"])
        cur = out
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    a = fd.fdirw_step(dom, c0, torch.empty_like(c0), prec="fp32", deterministic=True)
    b = fd.fdirw_step(dom, c0, torch.empty_like(c0), prec="fp32", deterministic=True)
    res = {"ms_per_step": ms, "kernel_ms": 1e3 * float(np.mean(kern)), "cells_per_s": d.n / (ms * 1e-3),
           "repeat_bitwise": bool(torch.equal(a, b))}
    if ref is not None:
        res["rel_l1_vs_fp32"] = float((a - ref).abs().sum()) / float(ref.abs().sum())
    log(f"deterministic fp32: {ms:.1f} ms/step, repeat bitwise {res['repeat_bitwise']}")
    return res


def bank_leg(fd, d, dom, c0, ref, args):
    """fdirw_run with every kernel stored once (the paper's stored-P use: P is
    fixed for a fixed geometry) and each big step applied by streaming the bank
    from HBM in the row form of the superposition.  Per storage precision
    (FP32, then FP16 as the paper stores P): one generation pass plus one big
    step, the apply time and HBM rate of that step, and the field error
    against the fused FP32 step."""
    import torch
    W3 = (2 * d.r + 1) ** 3
    out = {}
    for prec, esz in (("fp32", 4), ("fp16_bank", 2)):
        bank_bytes = d.n * W3 * esz
        budget = bank_bytes + d.n * 8 + (d.shape[0] + 2 * d.r) * (d.shape[1] + 2 * d.r) * (d.shape[2] + 2 * d.r) * 8 + (1 << 30)
        free, _ = torch.cuda.mem_get_info()
        if budget > free:
            log(f"bank {prec}: needs {budget / 1e9:.1f} GB, {free / 1e9:.1f} GB free: skipped")
            out[prec] = {"skipped": f"needs {budget / 1e9:.1f} GB"}
            continue
        log(f"bank {prec}: fdirw_run, generation + 1 step, bank of {bank_bytes / 1e9:.1f} GB")
        c = c0.clone()
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, st = fd.fdirw_run(dom, c, 1, prec=prec, stats=True, bank_budget_bytes=budget)
        torch.cuda.synchronize()
        total = time.perf_counter() - t
        ks = st["kernel_seconds"]
        rec = {"seconds_generation_and_step": total, "bank_used": st["bank_used"],
               "apply_ms": 1e3 * ks, "bank_bytes": bank_bytes,
               "apply_GBps": bank_bytes / ks / 1e9 if ks > 0 else None,
               "mass_rel_drift": abs(st["mass_out"] - st["mass_in"]) / st["mass_in"]}
        if rec["apply_GBps"]:
            rec["hbm_frac"] = rec["apply_GBps"] / PEAK_HBM_GBS
        # P computed once and reused (the paper's use): cost per step over 10 steps
        rec["amortised_ms_per_step_10"] = (1e3 * total + 9 * rec["apply_ms"]) / 10
        if ref is not None:
            rec["rel_l1_vs_fp32"] = float((c - ref).abs().sum()) / float(ref.abs().sum())
        out[prec] = rec
        fd.fdirw_release()
        log(f"bank {prec}: {total:.2f} s, apply {rec['apply_ms']:.2f} ms ({rec['apply_GBps']:.0f} GB/s)")
    if out.get("fp32", {}).get("apply_ms") and out.get("fp16_bank", {}).get("apply_ms"):
        out["apply_speedup_fp16_vs_fp32"] = out["fp32"]["apply_ms"] / out["fp16_bank"]["apply_ms"]
    return out


def coarse_leg(fd, d, dom, c0, c1, args):
    """Coarse-mesh FDiRW, the paper's GPU method (Sec. 3.1-3.3, Eqs. 13-15):
    blocks of B^3 cells, P built once from the fine window kernels, then per
    step mapping, P C and remapping.  Per storage precision of P (FP32, FP16):
    the build time, the step time (20 chained steps between events), the mass
    drift, and the field error against the fused FP32 step, from c0 (noise) and
    from c1 = one fused FP32 step of c0 (a diffused field).  Only the fast
    phase is grouped (D_pore = 1); solid cells keep their values."""
    import torch
    B = args.coarse_block
    # the liquid (pore, D = 1) is the grouped phase; the solid (D = 1e-6)
    # keeps its value, as the paper maps the liquid nodes only
    grouped = [1 if D >= 1e-3 * max(d.d_phase) else 0 for D in d.d_phase]
    fine2 = fd.fdirw_step(dom, c1, prec="fp32") if c1 is not None else None
    torch.cuda.synchronize()
    out = {"block": B, "grouped_phases": grouped}
    stream = torch.cuda.current_stream()
    # Table 2's precisions: (P storage, product arithmetic); "fp16_bank" with
    # FP64 arithmetic is the library's default coarse step
    legs = (("fp64", "fp64"), ("fp32", "fp32"), ("fp16_bank", "mixed"), ("fp16_bank", "fp16"),
            ("fp32", "fp64"), ("fp16_bank", "fp64"))
    handles = {}
    base = None
    for prec, arith in legs:
        if prec not in handles:
            log(f"coarse {prec}: building P over {B}^3 blocks")
            handles[prec] = fd.Coarse(dom, B, prec, grouped=grouped)
        cg = handles[prec]
        cg.set_arith(arith)
        bufs = [torch.empty_like(c0), torch.empty_like(c0)]
        cg.step(c0, bufs[0])
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        n = 20
        cur = c0
        ev0.record(stream)
        for k in range(n):
            cg.step(cur, bufs[k % 2])
            cur = bufs[k % 2]
        ev1.record(stream)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / n
        o0, st = cg.step(c0, stats=True)
        rec = {"P": prec, "arith": arith, "nodes": cg.n_nodes, "K": cg.K, "build_seconds": cg.build_seconds,
               "ms_per_step": ms, "cells_per_s": d.n / (ms * 1e-3), "kernel_ms": 1e3 * st["kernel_seconds"],
               "mass_rel_drift": abs(st["mass_out"] - st["mass_in"]) / st["mass_in"]}
        if base is None:
            base = (o0.clone(), ms)
        rec["rel_l1_vs_coarse_fp64"] = float((o0 - base[0]).abs().sum()) / float(base[0].abs().sum())
        rec["speedup_vs_coarse_fp64"] = base[1] / ms
        if c1 is not None:
            rec["rel_l1_vs_fp32_from_c0"] = float((o0 - c1).abs().sum()) / float(c1.abs().sum())
            o1 = cg.step(c1)
            rec["rel_l1_vs_fp32_from_c1"] = float((o1 - fine2).abs().sum()) / float(fine2.abs().sum())
        out[f"{prec}/{arith}"] = rec
        log(f"coarse P {prec}, arithmetic {arith}: {ms:.4f} ms / step, rel L1 vs coarse FP64 "
            f"{rec['rel_l1_vs_coarse_fp64']:.2e}, mass drift {rec['mass_rel_drift']:.1e}")
    if "fp16_bank" in handles:
        out["ensemble"] = ensemble_leg(fd, handles["fp16_bank"], args)
    for cg in handles.values():
        cg.close()
    return out


def ensemble_leg(fd, cg, args):
    """The coarse product for an ensemble of E coarse fields at once (Eq. 14
    with E right-hand sides, mixed FP32/FP16 on the matrix cores): device
    time per call (20 chained calls between events) for E = 1, 16, 64, 256,
    the time per member against E = 1, the achieved HBM rate of the
    algorithmic bytes (P's fragments once, each member's FP64 C read twice
    (its largest magnitude, then the scaled FP16 copy) and C' written, its
    FP16 grid written and read) and, for E = 16, the relative L1
    difference from the FP64 product of the same members (host)."""
    import torch
    import synth
    kw = 2 * cg.K + 1
    ncz, ncy, ncx = cg.coarse_shape
    n = cg.n_nodes
    tx, ty = (ncx + 3) // 4, (ncy + 3) // 4
    row = (4 + 2 * cg.K + 7) // 8 * 8
    kst = (row * (4 + 2 * cg.K) + 31) // 32
    frag_bytes = tx * ty * ncz * kw * kst * 64 * 16
    msize = (4 * tx - 4 + row) * (4 * ty + 2 * cg.K) * (ncz + 2 * cg.K)
    stream = torch.cuda.current_stream()
    Pm = cg.matrix()                                  # [o, I]: the stored FP16 values, widened
    nnz = float(np.count_nonzero(Pm))
    out = {"K": cg.K, "nodes": n, "fragment_bytes": frag_bytes, "nonzeros": nnz}
    t1 = None
    for E in (1, 16, 64, 256):
        C = torch.from_numpy(synth.uniform(900 + E, E * n).reshape(E, n)).cuda()
        Co = torch.empty_like(C)
        cg.apply_ensemble(C, Co)
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        reps = 20
        ev0.record(stream)
        for _ in range(reps):
            cg.apply_ensemble(C, Co)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / reps
        if t1 is None:
            t1 = ms
        bytes_ = frag_bytes + E * n * 24 + 2 * ((E + 15) // 16 * 16) * msize * 2
        rec = {"ms": ms, "us_per_member": 1e3 * ms / E, "speedup_per_member_vs_E1": t1 * E / ms,
               "hbm_GBps": bytes_ / (ms * 1e-3) / 1e9, "hbm_frac": bytes_ / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS}
        rec["useful_tflops"] = 2.0 * E * nnz / (ms * 1e-3) / 1e12
        if E == 16:
            Ch = C.cpu().numpy()
            ref = np.zeros((E, n))
            Cg = Ch.reshape(E, ncz, ncy, ncx)
            for o in range(kw ** 3):
                oz, rem = divmod(o, kw * kw)
                oy, ox = divmod(rem, kw)
                dz, dy, dx = oz - cg.K, oy - cg.K, ox - cg.K
                # C'[I] += P[o, I] C[I - d]
                src = np.zeros_like(Cg)
                zs, ys, xs = slice(max(dz, 0), ncz + min(dz, 0)), slice(max(dy, 0), ncy + min(dy, 0)), \
                    slice(max(dx, 0), ncx + min(dx, 0))
                zt, yt, xt = slice(max(-dz, 0), ncz - max(dz, 0)), slice(max(-dy, 0), ncy - max(dy, 0)), \
                    slice(max(-dx, 0), ncx - max(dx, 0))
                src[:, zs, ys, xs] = Cg[:, zt, yt, xt]
                ref += Pm[o][None, :] * src.reshape(E, n)
            got = Co.cpu().numpy()
            rec["rel_l1_vs_fp64_product"] = float(np.abs(got - ref).sum() / np.abs(ref).sum())
        out[f"E{E}"] = rec
        log(f"coarse ensemble E={E}: {ms:.4f} ms ({1e3 * ms / E:.2f} us / member), "
            f"{rec['hbm_GBps']:.0f} GB/s")
    return out


def mp_bytes_per_step(n_liq, n_sol, n_used_nodes, K, p_bytes):
    """Algorithmic HBM bytes of one integrated big step, which touches the
    active cells only: the mapping reads value and node index of every
    near-field liquid cell; the product reads P and C of the nodes that hold
    cells and writes C'; the fused local kernel reads node index and value (and
    the label of a solid cell) of every active cell and writes its value.  The
    far-field cells are written once per call, not per step."""
    kw3 = (2 * K + 1) ** 3
    b = 12 * n_liq
    b += n_used_nodes * (kw3 * p_bytes + 16)
    b += 20 * (n_liq + n_sol) + n_sol
    return b


def mp_leg(fd, args):
    """The integrated near-field solver (Sec. 2, Eqs. 1-7, flowchart of Sec.
    3.4) on the paper's particle case: a porous particle of radius 50 cells in
    the 192^3 grid (near-field shell of 5 cells, the rest far field), Table 1
    values, 5^3 coarse blocks.  Two big steps: 200 fast sub-steps (100 us) with
    the per-source kernels of r = 8 (the workload's r and n), P in FP32 and in
    FP16; and Table 1's own 1000 sub-steps (500 us) with node windows of r = 40
    (K = 8), P in FP16.  Per case: build time, device time per big step over
    ``--mp-steps`` chained steps, interface faces, the Eq. 7 balance residual,
    the solid uptake and the device time for 0.5 s of physical time."""
    import torch
    import synth
    n = args.n
    r_p = 50.0 * n / 192.0
    out = {"workload": f"particle{n}_R{int(r_p)}", "block": 5, "steps": args.mp_steps}
    stream = torch.cuda.current_stream()
    cases = [("dt100us_r8", 8, 200, ("fp32", "fp16_bank")), ("dt500us_r40", 40, 1000, ("fp16_bank",))]
    for name, r, n_sub, precs in cases:
        d, t = synth.particle_case(n, r_p, r=r, n_sub=n_sub)
        role = [fd.ROLE_LIQUID, fd.ROLE_SOLID, fd.ROLE_FAR_FIELD]
        a_rt = np.array([t["A_L_RT"], t["A_S_RT"], t["A_L_RT"]])
        far = d.label == synth.PHASE_FAR_LIQUID
        liq = d.label == synth.PHASE_NEAR_LIQUID
        v_ff, c_ff0 = t["V_ff_cells"], t["c0_L"]
        m_total = float(d.c0[~far].sum()) + v_ff * c_ff0
        dom = fd.Domain.from_synth(d)
        blk = (np.arange(n) // 5)
        used = np.unique(((blk[:, None, None] * 1000 + blk[None, :, None]) * 1000 + blk[None, None, :])[liq]).size
        case = {"r": r, "n_sub": n_sub, "big_step_s": n_sub * d.dt, "near_liquid_cells": int(liq.sum()),
                "solid_cells": int((d.label == synth.PHASE_SOLID).sum()), "nodes_with_cells": used}
        for prec in precs:
            log(f"integrated {name} {prec}: building the liquid operator")
            s = fd.Multiphysics(dom, role, t["k"], t["c_eq_L"], t["c_eq_S"], v_ff, a_over_rt=a_rt, block=5,
                                prec=prec)
            c = torch.from_numpy(d.c0).cuda()
            s.step(c, c_ff0, m_total, 1)                   # warm-up
            c.copy_(torch.from_numpy(d.c0))
            torch.cuda.synchronize()
            ev0 = torch.cuda.Event(enable_timing=True)
            ev1 = torch.cuda.Event(enable_timing=True)
            ev0.record(stream)
            cff, hist, st = s.step(c, c_ff0, m_total, args.mp_steps, stats=True)
            ev1.record(stream)
            torch.cuda.synchronize()
            ms = ev0.elapsed_time(ev1) / args.mp_steps
            resid = float(np.max(np.abs(hist[:, 0] + hist[:, 1] + v_ff * hist[:, 2] - m_total))) / m_total
            pb = 4 if prec == "fp32" else 2
            byts = mp_bytes_per_step(int(liq.sum()), case["solid_cells"], used, s.K, pb)
            case[prec] = {
                "build_seconds": s.build_seconds, "ms_per_step": ms,
                "kernel_ms_per_step": 1e3 * st["kernel_seconds"] / args.mp_steps, "K": s.K,
                "interface_faces": s.n_faces, "balance_rel_residual": resid,
                "solid_uptake_Q_S": [float(hist[0, 1]), float(hist[-1, 1])], "c_ff_end": cff,
                "hbm_bytes_per_step": byts, "hbm_GBps": byts / (ms * 1e-3) / 1e9,
                "hbm_frac": byts / (ms * 1e-3) / (PEAK_HBM_GBS * 1e9),
                "seconds_per_physical_0p5s": ms * 1e-3 * 0.5 / (n_sub * d.dt)}
            s.close()
            log(f"integrated {name} {prec}: build {case[prec]['build_seconds']:.2f} s, {ms:.4f} ms / big step, "
                f"{case[prec]['seconds_per_physical_0p5s']:.3f} s per 0.5 s physical, balance {resid:.1e}")
        out[name] = case
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--prec", default="fp32", help="headline precision mode")
    ap.add_argument("--modes", default="fp32,fp16x32,bf16x32", help="modes timed for the comparison")
    ap.add_argument("--n", type=int, default=192, help="grid edge (192 = the benchmark workload)")
    ap.add_argument("--cpu-block", type=int, default=40, help="edge of the oracle's source sample (0: skip)")
    ap.add_argument("--tune", type=int, default=-1)
    ap.add_argument("--nn-epochs", type=int, default=4,
                    help="epochs of the surrogate recipe before its step is timed (0: skip the surrogate)")
    ap.add_argument("--det", type=int, default=1, help="also time the FP32 step with deterministic = 1 (0: skip)")
    ap.add_argument("--batched", type=int, default=1, help="also time the 64-domain batched step (0: skip)")
    ap.add_argument("--bank", type=int, default=1, help="also time fdirw_run with FP32 and FP16 kernel banks (0: skip)")
    ap.add_argument("--mp-steps", type=int, default=50,
                    help="big steps of the integrated-solver leg (particle case); 0: skip the leg")
    ap.add_argument("--coarse-block", type=int, default=5,
                    help="block edge of the coarse-mesh leg (the paper's 1/125 nodes); 0: skip the leg")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the FDiRW step here is a single-GPU build "
              "(multi-GPU sharding is a design note, not implemented).", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    import paper_2408_11376_amd as fd

    torch.cuda.set_device(0)
    log(f"generating the {args.n}^3 workload")
    d = synth.config2(n=args.n)
    dom = fd.Domain(d.label, d.d_phase, d.r, d.n_sub, d.h, d.dt)
    N = d.n
    c0 = torch.from_numpy(d.c0).cuda()
    bufs = [torch.empty_like(c0), torch.empty_like(c0)]
    stream = torch.cuda.current_stream()

    modes = [m.strip() for m in args.modes.split(",") if m.strip()]
    if args.prec not in modes:
        modes.append(args.prec)
    results = {}
    fields = {}
    for mode in modes:
        log(f"{mode}: {args.warmup} warm-up + {args.steps} timed steps")
        cur = c0
        for _ in range(args.warmup):
            fd.fdirw_step(dom, cur, bufs[0], prec=mode, tune=args.tune)
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        kern = []
        cur = c0
        t_host = time.perf_counter()
        ev0.record(stream)
        for k in range(args.steps):
            out = bufs[k % 2]
            _, st = fd.fdirw_step(dom, cur, out, prec=mode, stats=True, tune=args.tune)
            kern.append(st["kernel_seconds"])
            cur = out
        ev1.record(stream)
        torch.cuda.synchronize()
        t_host = time.perf_counter() - t_host
        ms = ev0.elapsed_time(ev1) / args.steps
        # one more (untimed) step from c0 for the accuracy comparison
        first_out, first_st = fd.fdirw_step(dom, c0, torch.empty_like(c0), prec=mode, stats=True,
                                            tune=args.tune)
        fields[mode] = first_out
        results[mode] = {
            "cells_per_s": N / (ms * 1e-3),
            "ms_per_step": ms,
            "kernel_ms": 1e3 * float(np.mean(kern)),
            "host_ms_per_step": 1e3 * t_host / args.steps,
            "mass_rel_drift": abs(first_st["mass_out"] - first_st["mass_in"]) / first_st["mass_in"],
            "kernel_mass_range": [first_st["kmass_min"], first_st["kmass_max"]],
            "sources": first_st["n_sources"],
            "cell_substeps_per_s": window_cells(d.shape, d.r) * d.n_sub / (ms * 1e-3),
        }
        log(f"{mode}: {ms:.1f} ms/step, kernel {results[mode]['kernel_ms']:.1f} ms, "
            f"{results[mode]['cells_per_s'] / 1e6:.3f} Mcells/s")

    if args.nn_epochs > 0:
        results["nn"], fields["nn"] = surrogate_mode(fd, d, dom, c0, bufs, stream, args)

    extra = {}
    if args.det:
        extra["deterministic"] = deterministic_leg(fd, d, dom, c0, bufs, stream, fields.get("fp32"), args)
    if args.batched:
        extra["batched"] = batched_leg(fd, args)
    if args.bank:
        extra["bank"] = bank_leg(fd, d, dom, c0, fields.get("fp32"), args)
    if args.coarse_block > 0:
        extra["coarse"] = coarse_leg(fd, d, dom, c0, fields.get("fp32"), args)
    if args.mp_steps > 0:
        extra["integrated"] = mp_leg(fd, args)

    if "fp32" in fields:
        ref = fields["fp32"]
        den = float(ref.abs().sum())
        for mode in results:
            results[mode]["rel_l1_vs_fp32"] = float((fields[mode] - ref).abs().sum()) / den
            results[mode]["speedup_vs_fp32"] = results["fp32"]["ms_per_step"] / results[mode]["ms_per_step"]

    head = results[args.prec]
    cs = window_cells(d.shape, d.r) * d.n_sub          # in-domain cell-sub-steps per step
    flops = FLOP_PER_CELL_SUBSTEP * cs
    achieved = flops / (head["kernel_ms"] * 1e-3) / 1e12
    esize = {"fp32": 4, "fp64": 8}.get(args.prec, 2)
    t_kern = head["kernel_ms"] * 1e-3
    lds_tbs = LDS_ACCESSES_PER_CELL_SUBSTEP * esize * cs / t_kern / 1e12
    # exchange time at the LDS rates (four neighbour reads, one write per
    # cell-sub-step) and FMA issue time at one FMA per lane per clock
    t_lds = cs * (4 * esize / LDS_READ_B_PER_CLK + esize / LDS_WRITE_B_PER_CLK) / CU_HZ
    t_valu = cs * FMA_PER_CELL_SUBSTEP / (64 * CU_HZ)
    flat = args.prec == "fp32" and 4 <= d.r <= 8 and os.environ.get("FDIRW_FUSED_LAYOUT") != "segments"
    kname = "flat_line_kernel" if flat else "line_kernel"
    kernel_tag = f"{kname}_{args.prec}_grf{args.n}"
    traffic = read_traffic(kernel_tag)
    roofline = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP32_VECTOR_TFLOPS, "traffic": traffic,
                "peak_unpacked_fp32": PEAK_FP32_UNPACKED_TFLOPS,
                "frac_unpacked_fp32": achieved / PEAK_FP32_UNPACKED_TFLOPS,
                "kernel": f"{kname}<{args.prec}, r={d.r}>",
                "cell_substeps_per_launch": cs, "flop_per_cell_substep": FLOP_PER_CELL_SUBSTEP,
                "lds_exchange_TBps_model": lds_tbs,
                "lds_bound_s_model": t_lds, "lds_frac_model": t_lds / t_kern,
                "fma_issue_bound_s": t_valu, "fma_issue_frac": t_valu / t_kern}
    # LDS from the committed counter summary of this kernel (instructions and
    # bytes per launch, busy fraction of the LDS pipe), when it matches the
    # sources; the launch's bytes are scaled to the time measured here
    lds = read_profile_values(kernel_tag, "lds", ["lds_bytes_per_launch", "lds_busy_frac", "valu_busy_frac"])
    if lds is not None:
        roofline["lds_bytes_per_launch"] = lds["lds_bytes_per_launch"]
        roofline["lds_TBps_counters"] = lds["lds_bytes_per_launch"] / t_kern / 1e12
        roofline["lds_busy_frac_counters"] = lds["lds_busy_frac"]
        roofline["valu_busy_frac_counters"] = lds["valu_busy_frac"]

    cpu = None
    if args.cpu_block > 0:
        log(f"timing the CPU oracle on a {args.cpu_block}^3 source sample")
        cpu = cpu_baseline(d, args.cpu_block)
        log(f"oracle: {cpu['value']:.1f} cells/s on {cpu['cores']} threads")

    line = {
        "metric": "FDiRW big-step cells/s @192^3 (fused kernel generation + FP64 superposition)",
        "value": head["cells_per_s"],
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp16x32": "f32 (f16 neighbour copies, f64 superposition)",
                  "bf16x32": "f32 (bf16 neighbour copies, f64 superposition)",
                  "fp32": "f32 (f64 superposition)", "fp64": "f64"}.get(args.prec, args.prec),
        "data": "synthetic (seeded GRF porous medium standing in for the paper's particle geometry)",
        "config": {"workload": f"grf{args.n}_r{d.r}_n{d.n_sub}", "grid": list(d.shape), "r": d.r,
                   "n_sub": d.n_sub, "solid_fraction": 0.35, "D": [1.0, 1e-6], "prec": args.prec,
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "modes": results,
    }
    line.update(extra)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
