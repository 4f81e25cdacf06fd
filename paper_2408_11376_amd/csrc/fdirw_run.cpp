// fdirw_run.cpp -- time marching of the superposition (Eq. 8 of arXiv
// 2408.11376 applied once per big step) with an optional kernel bank.
//
// The paper computes the proportions P once for a fixed geometry and reuses
// them every step (Sec. 3.1, "preconditioned"; Sec. 5 on the fixed domain).
// When the caller's budget allows, fdirw_run does the same: one pass of the
// window kernel stores every G_s (with its mass) offset-major, P[o][s + o] =
// G_s(o), and each big step streams the bank from HBM once in the row form of
// the superposition, c'(x) = sum_o P[o][x] c(x - o) / m_(x - o) (coalesced,
// no atomics, fixed order).  Otherwise every step regenerates the kernels
// (fused path).
#include <hip/hip_runtime.h>

#include <cmath>

#include "fdirw_host.h"
#include "fdirw_launch.h"

namespace fdirw {

int run_one(const fdirw_domain *d, const fdirw_opts *o, int n_steps, double *c, double *scratch,
            fdirw_stats *st, DevCache &dc, hipStream_t stream)
{
    int rc;
    Geometry geo;
    const void *lam = nullptr;
    if ((rc = coef_buffers(d, o->prec, stream, dc, &geo, &lam))) return rc;
    const int64_t n = geo.n;
    const int W = 2 * d->r + 1;
    const int64_t W3 = (int64_t)W * W * W;
    const size_t esz = bank_elem_bytes(o->prec);
    const size_t bank_alloc = (size_t)bank_elems(d->nx, d->ny, d->nz, d->r, (int)esz) * esz;
    const int64_t n_chat = bank_chat_elems(d->nx, d->ny, d->nz, d->r);
    const double bank_bytes = (double)bank_alloc + (double)n * 8.0 + (double)n_chat * 8.0;
    bool use_bank = n_steps >= 1 && o->bank_budget_bytes > 0 && bank_bytes <= (double)o->bank_budget_bytes;
    if (use_bank) {
        // a bank that does not fit in device memory silently falls back to the
        // fused path (identical results up to FP64 summation order)
        if (ensure(dc.bank, bank_alloc) != FDIRW_OK ||
            ensure(dc.bank_mass, (size_t)n * sizeof(double)) != FDIRW_OK ||
            ensure(dc.bank_chat, (size_t)n_chat * sizeof(double)) != FDIRW_OK)
            use_bank = false;
    }
    double kmin = INFINITY, kmax = -INFINITY;
    if (use_bank) {
        // entries P[o][x] whose source x - o lies outside the domain are never
        // written: clear the bank once (they meet a zero c^ in the apply, and
        // 0 * stale bits could be NaN)
        hipError_t e0 = launch_fill_u32((unsigned *)dc.bank.p, (int64_t)(bank_alloc / 4), 0u, stream);
        if (e0 != hipSuccess) return hip_fail(e0, "bank clear");
        WindowArgs a;
        a.nx = d->nx; a.ny = d->ny; a.nz = d->nz; a.n = n;
        a.n_sub = d->n_sub;
        a.lx = lam;
        a.src = nullptr; a.n_src = n;
        a.G = dc.bank.p; a.mass = (double *)dc.bank_mass.p;
        a.normalize = 0;
        a.out_lp = 1;
        a.offset_major = 1;
        hipError_t e = launch_window(o->prec, d->r, a, stream);
        if (e != hipSuccess) return hip_fail(e, "bank generation launch");
        if (st) {
            if ((rc = ensure(dc.small, 64))) return rc;
            if ((rc = ensure(dc.wgk, 512 * sizeof(double)))) return rc;
            double *mm = (double *)dc.small.p + 4;
            double h_mm[2] = {INFINITY, -INFINITY};
            e = launch_minmax_scalar((const double *)dc.bank_mass.p, n, (double *)dc.wgk.p, mm, stream);
            if (e == hipSuccess) e = hipMemcpyAsync(h_mm, mm, sizeof h_mm, hipMemcpyDeviceToHost, stream);
            if (e == hipSuccess) e = hipStreamSynchronize(stream);
            if (e != hipSuccess) return hip_fail(e, "bank statistics");
            kmin = h_mm[0];
            kmax = h_mm[1];
        }
    }
    double *cur = c, *nxt = scratch;
    for (int step = 0; step < n_steps; ++step) {
        const bool last = step == n_steps - 1;
        fdirw_stats *sst = (st && last) ? st : nullptr;
        if (use_bank) {
            if (sst) {
                if ((rc = field_sum_dev(cur, n, stream, dc, &sst->mass_in))) return rc;
                if (!std::isfinite(sst->mass_in)) return fail(FDIRW_E_NONFINITE, "input mass is not finite");
            }
            hipError_t e = hipSuccess;
            BankArgs b;
            b.nx = d->nx; b.ny = d->ny; b.nz = d->nz;
            b.n = n;
            b.bank = dc.bank.p;
            b.mass = (const double *)dc.bank_mass.p;
            b.c_in = cur; b.c_out = nxt;
            b.chat = (double *)dc.bank_chat.p;
            EventPair ev;
            if (sst && e == hipSuccess) e = ev.create();
            if (sst && e == hipSuccess) e = hipEventRecord(ev.a, stream);
            if (e == hipSuccess) e = launch_bank_apply(o->prec, d->r, b, stream);
            if (sst && e == hipSuccess) e = hipEventRecord(ev.b, stream);
            if (e != hipSuccess) return hip_fail(e, "bank apply launch");
            if (sst) {
                if ((rc = field_sum_dev(nxt, n, stream, dc, &sst->mass_out))) return rc;
                sst->kmass_min = kmin;
                sst->kmass_max = kmax;
                sst->n_sources = -1;
                sst->audit_l1 = 0.0;
                sst->fallback_used = 0;
                sst->bank_used = 1;
                sst->tuned_config_id = 0;
                sst->kernel_seconds = ev.seconds();
            }
        } else {
            if ((rc = step_one(d, o, cur, nxt, sst, dc, stream, true, lam, &geo))) return rc;
        }
        double *t = cur; cur = nxt; nxt = t;
    }
    if (cur != c) {
        hipError_t e = hipMemcpyAsync(c, cur, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, stream);
        if (e != hipSuccess) return hip_fail(e, "result copy");
    }
    if (st) {
        hipError_t e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return hip_fail(e, "run");
        if (n_steps == 0) {
            double m = 0.0;
            if ((rc = field_sum_dev(c, n, stream, dc, &m))) return rc;
            st->mass_in = st->mass_out = m;
            st->kmass_min = INFINITY;
            st->kmass_max = -INFINITY;
            st->n_sources = 0;
            st->bank_used = 0;
        }
    }
    return FDIRW_OK;
}

}  // namespace fdirw
