// fdirw_mp_api.cpp -- host side of the integrated near-field solver
// (include/fdirw.h; Sec. 2, Eqs. 1-7, and the flowchart of Sec. 3.4 of arXiv
// 2408.11376).
//
// A handle owns the coarse operator of the liquid (built by
// fdirw_coarse_create on the domain with the solid walled off), the list of
// tiles that hold an active cell (near-field liquid or solid), a copy of the
// labels, the sorted lists of the active and of the solid cells with the
// solid step's face coefficients (used when a big step has several solid
// sub-steps), a second field buffer and the far-field value on the device.
// A step is four launches: mapping, product, the fused local kernel
// (remapping, the six reaction passes, one solid sub-step and the Eq. 7 sums,
// tile by tile) and the Eq. 7 finish; with several solid sub-steps the fused
// kernel stops after the reaction and the solid list and the balance kernels
// follow.  The
// steps alternate between the caller's field and the second buffer, and the
// far-field cells are written once, after the last step.  Nothing returns to
// the host between steps.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/fdirw.h"
#include "fdirw_host.h"
#include "fdirw_launch.h"

namespace fdirw {

namespace {

struct Mp {
    int dev = -1;
    int n_solid = 0;                    // solid phases (compact indices 0 .. n_solid - 1)
    int nx = 0, ny = 0, nz = 0;
    int64_t n = 0;
    double h = 1.0, dt = 0.0;           // grid spacing, big step
    double kappa_dt = 0.0;              // k dt / (c_L^eq c_S^eq)
    double c_eq_l = 1.0, c_eq_s = 1.0, v_ff = 1.0;
    int n_sub_solid = 1;
    double solid[256];                  // D A / RT of every solid phase, 0 for the others
    void *dsol = nullptr;               // device copy of solid (by label)
    void *dsolc = nullptr;              // D A / RT of the solid phases by compact index
    void *coarse = nullptr;
    int64_t n_faces = 0;                // interface faces (liquid / solid)
    int64_t n_tiles = 0;
    void *tiles = nullptr;              // int [n_tiles] tiles of the fused local kernel
    void *pair_off = nullptr;           // int [6 n_tiles + 1] start of each tile's reaction pass
    void *pairs = nullptr;              // uint16 interface pairs of every tile's box
    void *scode = nullptr;              // uint8 [N] compact solid-phase index of every cell
    int64_t n_act = 0, n_sol = 0;
    void *act = nullptr;                // int [n_act] active cells, ascending
    void *sol = nullptr;                // int [n_sol] solid cells, ascending
    void *slam = nullptr;               // double [6][n_sol] face coefficients of the solid step
    void *snb = nullptr;                // int [6][n_sol] solid neighbours (list positions)
    void *sa = nullptr, *sb = nullptr;  // double [n_sol] sub-step values
    void *tmp = nullptr;                // double [N]
    void *part = nullptr;               // double [2 * max(MP_SUM_BLOCKS, n_tiles)]
    void *cff = nullptr;                // double [1]
    void *hist = nullptr;               // double [3 * hist_cap]
    int64_t hist_cap = 0;

    ~Mp()
    {
        for (void *p : {tiles, pair_off, pairs, scode, dsol, dsolc, act, sol, slam, snb, sa, sb, tmp, part, cff, hist})
            if (p) (void)hipFree(p);
        if (coarse) (void)fdirw_coarse_destroy(coarse);
    }
};

int mp_alloc(void **p, size_t bytes)
{
    if (bytes == 0) bytes = 16;
    if (hipMalloc(p, bytes) != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(FDIRW_E_NOMEM, "integrated solver: could not allocate %zu bytes", bytes);
    }
    return FDIRW_OK;
}

int check_mp(const Mp *h)
{
    if (!h) return fail(FDIRW_E_ARG, "solver handle is null");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != h->dev)
        return fail(FDIRW_E_ARG, "solver handle belongs to device %d, current device is %d", h->dev, dev);
    return FDIRW_OK;
}

int check_params(const fdirw_domain *d, const fdirw_mp_params *p)
{
    if (!p) return fail(FDIRW_E_ARG, "params is null");
    if (!p->role) return fail(FDIRW_E_ARG, "params->role is null");
    for (int i = 0; i < d->n_phase; ++i) {
        if (p->role[i] > FDIRW_ROLE_FAR_FIELD) return fail(FDIRW_E_ARG, "role[%d] = %d is not a role", i, p->role[i]);
        if (p->a_over_rt && !(std::isfinite(p->a_over_rt[i]) && p->a_over_rt[i] >= 0.0))
            return fail(FDIRW_E_ARG, "a_over_rt[%d] must be finite and >= 0", i);
    }
    if (!(std::isfinite(p->k) && p->k >= 0.0)) return fail(FDIRW_E_ARG, "k must be finite and >= 0");
    if (!(std::isfinite(p->c_eq_liquid) && p->c_eq_liquid > 0.0)) return fail(FDIRW_E_ARG, "c_eq_liquid must be > 0");
    if (!(std::isfinite(p->c_eq_solid) && p->c_eq_solid > 0.0)) return fail(FDIRW_E_ARG, "c_eq_solid must be > 0");
    if (p->n_sub_solid < 1) return fail(FDIRW_E_ARG, "n_sub_solid = %d < 1", p->n_sub_solid);
    if (!(std::isfinite(p->v_far_field) && p->v_far_field > 0.0)) return fail(FDIRW_E_ARG, "v_far_field must be > 0");
    if (!(d->dt > 0.0)) return fail(FDIRW_E_ARG, "the integrated solver needs the fast sub-step d->dt > 0");
    return FDIRW_OK;
}

// Sorted list of the cells of one kind (launch_mp_list_* mode) into *list
// (allocated here; *count entries).
int build_list(const int *node, int64_t n, int mode, hipStream_t st, void **list, int64_t *count)
{
    const int64_t chunks = (n + MP_CHUNK - 1) / MP_CHUNK;
    int *cc = nullptr;
    int64_t *off = nullptr;
    int rc = mp_alloc((void **)&cc, (size_t)chunks * sizeof(int));
    if (!rc) rc = mp_alloc((void **)&off, (size_t)chunks * sizeof(int64_t));
    std::vector<int> hc((size_t)chunks);
    std::vector<int64_t> ho((size_t)chunks);
    hipError_t e = hipSuccess;
    if (!rc) {
        e = launch_mp_list_count(node, n, mode, cc, st);
        if (e == hipSuccess) e = hipMemcpyAsync(hc.data(), cc, hc.size() * sizeof(int), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
    }
    int64_t total = 0;
    if (!rc && e == hipSuccess) {
        for (int64_t k = 0; k < chunks; ++k) {
            ho[(size_t)k] = total;
            total += hc[(size_t)k];
        }
        rc = mp_alloc(list, (size_t)total * sizeof(int));
    }
    if (!rc && e == hipSuccess) {
        e = hipMemcpyAsync(off, ho.data(), ho.size() * sizeof(int64_t), hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = launch_mp_list_write(node, n, mode, off, (int *)*list, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
    }
    (void)hipFree(cc);
    (void)hipFree(off);
    if (rc) return rc;
    if (e != hipSuccess) return hip_fail(e, "cell list");
    *count = total;
    return FDIRW_OK;
}

}  // namespace

}  // namespace fdirw

using namespace fdirw;

extern "C" {

int fdirw_mp_create(const fdirw_domain *d, const fdirw_mp_params *p, int32_t block, int32_t prec, void *stream,
                    void **handle, double *seconds)
{
    if (!handle) return fail(FDIRW_E_ARG, "handle is null");
    *handle = nullptr;
    int rc = check_domain(d, FDIRW_MAX_COARSE_RADIUS);
    if (rc) return rc;
    if ((rc = check_params(d, p))) return rc;
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t st = (hipStream_t)stream;
    // Eq. 1 with Eqs. 2-3: coefficient D A / RT per phase; the liquid's
    // kernels see the solid as a wall, the solid step sees the liquid as one
    std::vector<double> d_liq(d->n_phase), coef(d->n_phase);
    std::vector<uint8_t> grouped(d->n_phase), reservoir(d->n_phase);
    double dsol_max = 0.0;
    if ((int64_t)d->nx * d->ny * d->nz > 0x7fffffffLL)
        return fail(FDIRW_E_ARG, "the integrated solver indexes cells with 32-bit integers (N < 2^31)");
    for (int i = 0; i < d->n_phase; ++i) {
        coef[i] = d->d_phase[i] * (p->a_over_rt ? p->a_over_rt[i] : 1.0);
        if (!std::isfinite(coef[i])) return fail(FDIRW_E_ARG, "D A / RT of phase %d is not finite", i);
        d_liq[i] = p->role[i] == FDIRW_ROLE_SOLID ? 0.0 : coef[i];
        grouped[i] = p->role[i] == FDIRW_ROLE_LIQUID;
        reservoir[i] = p->role[i] == FDIRW_ROLE_FAR_FIELD;
        if (p->role[i] == FDIRW_ROLE_SOLID) dsol_max = std::fmax(dsol_max, coef[i]);
    }
    const double dt = (double)d->n_sub * d->dt;
    const double dts = dt / p->n_sub_solid;
    const double cfl = 6.0 * dsol_max * dts / (d->h * d->h);
    if (cfl > 1.0 + 1e-12)
        return fail(FDIRW_E_UNSTABLE, "solid: 6 max(D A / RT) dt_s / h^2 = %.17g > 1 (raise n_sub_solid)", cfl);
    const double kappa_dt = p->k / (p->c_eq_liquid * p->c_eq_solid) * dt;
    if (!std::isfinite(kappa_dt)) return fail(FDIRW_E_ARG, "k dt / (c_eq_liquid c_eq_solid) is not finite");
    auto *h = new (std::nothrow) Mp;
    if (!h) return fail(FDIRW_E_NOMEM, "solver handle");
    if (hipGetDevice(&h->dev) != hipSuccess) {
        delete h;
        return fail(FDIRW_E_DEVICE, "hipGetDevice failed");
    }
    h->nx = d->nx; h->ny = d->ny; h->nz = d->nz;
    h->n = (int64_t)d->nx * d->ny * d->nz;
    h->h = d->h;
    h->dt = dt;
    h->c_eq_l = p->c_eq_liquid;
    h->c_eq_s = p->c_eq_solid;
    h->kappa_dt = kappa_dt;
    h->v_ff = p->v_far_field;
    h->n_sub_solid = p->n_sub_solid;
    std::memset(h->solid, 0, sizeof h->solid);
    for (int i = 0; i < d->n_phase; ++i) h->solid[i] = p->role[i] == FDIRW_ROLE_SOLID ? coef[i] : 0.0;
    fdirw_domain dl = *d;
    dl.d_phase = d_liq.data();
    if ((rc = fdirw_coarse_create(&dl, block, prec, grouped.data(), reservoir.data(), nullptr, stream, &h->coarse,
                                  nullptr))) {
        h->coarse = nullptr;
        delete h;
        return rc;
    }
    // interface faces (counted for the caller), the tiles that hold an active
    // cell, a copy of the labels
    const int *node = coarse_node(h->coarse);
    const int64_t nt = mp_tile_count(d->nx, d->ny, d->nz);
    unsigned long long *cnt = nullptr;
    int *flag = nullptr;
    rc = mp_alloc((void **)&cnt, 6 * sizeof(unsigned long long));
    if (!rc) rc = mp_alloc((void **)&flag, (size_t)nt * sizeof(int));
    if (!rc) rc = mp_alloc(&h->tmp, (size_t)h->n * sizeof(double));
    if (!rc) rc = mp_alloc(&h->scode, (size_t)h->n);
    if (!rc) rc = mp_alloc(&h->dsol, sizeof h->solid);
    if (!rc) rc = mp_alloc(&h->dsolc, sizeof h->solid);
    if (!rc) rc = mp_alloc(&h->cff, sizeof(double));
    if (rc) {
        (void)hipFree(cnt);
        (void)hipFree(flag);
        delete h;
        return rc;
    }
    unsigned long long hc[6];
    std::vector<int> hflag((size_t)nt);
    hipError_t e = launch_fill_u32((unsigned *)cnt, 12, 0u, st);
    // compact indices of the solid phases (the fused kernel's role byte)
    unsigned char sidx[256];
    double dc[256];
    std::memset(sidx, 0, sizeof sidx);
    int n_solid_phases = 0;
    for (int i = 0; i < d->n_phase; ++i)
        if (p->role[i] == FDIRW_ROLE_SOLID) {
            sidx[i] = (unsigned char)n_solid_phases;
            dc[n_solid_phases++] = h->solid[i];
        }
    h->n_solid = n_solid_phases;
    if (n_solid_phases > MP_MAX_SOLID_PHASES) {
        (void)hipFree(cnt);
        (void)hipFree(flag);
        delete h;
        return fail(FDIRW_E_UNSUPPORTED, "%d solid phases: at most %d", n_solid_phases, MP_MAX_SOLID_PHASES);
    }
    if (e == hipSuccess) e = launch_mp_code(d->label, h->n, sidx, (uint8_t *)h->scode, st);
    if (e == hipSuccess) e = hipMemcpyAsync(h->dsol, h->solid, sizeof h->solid, hipMemcpyHostToDevice, st);
    if (e == hipSuccess && n_solid_phases)
        e = hipMemcpyAsync(h->dsolc, dc, n_solid_phases * sizeof(double), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = launch_mp_faces(node, d->nx, d->ny, d->nz, cnt, st);
    if (e == hipSuccess) e = launch_mp_tile_flags(node, d->nx, d->ny, d->nz, flag, st);
    if (e == hipSuccess) e = hipMemcpyAsync(hc, cnt, sizeof hc, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(hflag.data(), flag, hflag.size() * sizeof(int), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(cnt);
    (void)hipFree(flag);
    if (e != hipSuccess) {
        delete h;
        return hip_fail(e, "interface faces and tiles");
    }
    h->n_faces = 0;
    for (int k = 0; k < 6; ++k) h->n_faces += (int64_t)hc[k];
    std::vector<int> tl;
    for (int64_t t = 0; t < nt; ++t)
        if (hflag[(size_t)t]) tl.push_back((int)t);
    h->n_tiles = (int64_t)tl.size();
    const int64_t n_part = h->n_tiles > MP_SUM_BLOCKS ? h->n_tiles : MP_SUM_BLOCKS;
    rc = mp_alloc(&h->tiles, tl.size() * sizeof(int));
    if (!rc) rc = mp_alloc(&h->part, (size_t)2 * n_part * sizeof(double));
    if (rc) {
        delete h;
        return rc;
    }
    if (!tl.empty()) {
        e = hipMemcpyAsync(h->tiles, tl.data(), tl.size() * sizeof(int), hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) {
            delete h;
            return hip_fail(e, "tile list");
        }
    }
    // every tile's interface pairs per reaction pass: count, scan, list
    {
        const size_t n6 = (size_t)6 * h->n_tiles;
        int *pc = nullptr;
        rc = mp_alloc((void **)&pc, n6 * sizeof(int));
        if (!rc) rc = mp_alloc(&h->pair_off, (n6 + 1) * sizeof(int));
        std::vector<int> hcnt(n6), hoff(n6 + 1, 0);
        if (!rc) {
            e = launch_mp_tile_pairs(node, d->nx, d->ny, d->nz, (const int *)h->tiles, h->n_tiles, nullptr, nullptr,
                                     pc, st);
            if (e == hipSuccess && n6) e = hipMemcpyAsync(hcnt.data(), pc, n6 * sizeof(int), hipMemcpyDeviceToHost, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            int64_t tot = 0;
            for (size_t k = 0; k < n6; ++k) {
                hoff[k] = (int)tot;
                tot += hcnt[k];
            }
            hoff[n6] = (int)tot;
            if (tot > 0x7fffffffLL) rc = fail(FDIRW_E_ARG, "too many interface pairs");
            if (!rc && e == hipSuccess) rc = mp_alloc(&h->pairs, (size_t)tot * sizeof(uint16_t));
            if (!rc && e == hipSuccess)
                e = hipMemcpyAsync(h->pair_off, hoff.data(), hoff.size() * sizeof(int), hipMemcpyHostToDevice, st);
            if (!rc && e == hipSuccess)
                e = launch_mp_tile_pairs(node, d->nx, d->ny, d->nz, (const int *)h->tiles, h->n_tiles,
                                         (const int *)h->pair_off, (uint16_t *)h->pairs, pc, st);
            std::vector<int> hcnt2(n6);
            if (!rc && e == hipSuccess && n6)
                e = hipMemcpyAsync(hcnt2.data(), pc, n6 * sizeof(int), hipMemcpyDeviceToHost, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            if (!rc && e == hipSuccess && hcnt2 != hcnt) rc = fail(FDIRW_E_DEVICE, "interface pair count changed");
        }
        (void)hipFree(pc);
        if (!rc && e != hipSuccess) rc = hip_fail(e, "interface pairs");
        if (rc) {
            delete h;
            return rc;
        }
    }
    // the active and solid lists, and the solid step's coefficients
    if ((rc = build_list(node, h->n, 0, st, &h->act, &h->n_act)) ||
        (rc = build_list(node, h->n, 1, st, &h->sol, &h->n_sol))) {
        delete h;
        return rc;
    }
    int *inv = nullptr;
    rc = mp_alloc((void **)&inv, (size_t)h->n * sizeof(int));
    if (!rc) rc = mp_alloc(&h->slam, (size_t)6 * h->n_sol * sizeof(double));
    if (!rc) rc = mp_alloc(&h->snb, (size_t)6 * h->n_sol * sizeof(int));
    if (!rc) rc = mp_alloc(&h->sa, (size_t)h->n_sol * sizeof(double));
    if (!rc) rc = mp_alloc(&h->sb, (size_t)h->n_sol * sizeof(double));
    if (rc) {
        (void)hipFree(inv);
        delete h;
        return rc;
    }
    e = launch_fill_u32((unsigned *)inv, h->n, 0xffffffffu, st);
    if (e == hipSuccess)
        e = launch_mp_solid_prep((const int *)h->sol, h->n_sol, d->label, (const double *)h->dsol, inv, d->nx, d->ny,
                                 d->nz, dts,
                                 d->h, (double *)h->slam, (int *)h->snb, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(inv);
    if (e != hipSuccess) {
        delete h;
        return hip_fail(e, "solid coefficients");
    }
    if (seconds) *seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    *handle = h;
    return FDIRW_OK;
}

int fdirw_mp_step(void *handle, double *c, double *c_ff, double m_total, int32_t n_steps, double *history,
                  void *stream, fdirw_stats *stats)
{
    Mp *h = (Mp *)handle;
    int rc = check_mp(h);
    if (rc) return rc;
    if (!c || !c_ff) return fail(FDIRW_E_ARG, "c and c_ff must not be null");
    if (n_steps < 0) return fail(FDIRW_E_ARG, "n_steps = %d < 0", n_steps);
    if (!std::isfinite(*c_ff) || !std::isfinite(m_total)) return fail(FDIRW_E_NONFINITE, "c_ff and m_total must be finite");
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t st = (hipStream_t)stream;
    if (n_steps > h->hist_cap) {
        if (h->hist) (void)hipFree(h->hist);
        h->hist = nullptr;
        h->hist_cap = 0;
        if ((rc = mp_alloc(&h->hist, (size_t)3 * n_steps * sizeof(double)))) return rc;
        h->hist_cap = n_steps;
    }
    EventPair ev;
    hipError_t e = stats ? ev.create() : hipSuccess;
    if (e == hipSuccess) e = launch_fill((double *)h->cff, 1, *c_ff, st);
    if (stats && e == hipSuccess) e = hipEventRecord(ev.a, st);
    if (e != hipSuccess) return hip_fail(e, "integrated step set-up");
    const int *node = coarse_node(h->coarse);
    double *tmp = (double *)h->tmp;
    MpLocalArgs a;
    std::memset(&a, 0, sizeof a);
    a.nx = h->nx; a.ny = h->ny; a.nz = h->nz;
    a.tiles = (const int *)h->tiles;
    a.n_tiles = h->n_tiles;
    a.pair_off = (const int *)h->pair_off;
    a.pairs = (const uint16_t *)h->pairs;
    a.node = node;
    a.scode = (const uint8_t *)h->scode;
    a.dsolc = (const double *)h->dsolc;
    a.n_solid = h->n_solid;
    a.c_eq_l = h->c_eq_l; a.c_eq_s = h->c_eq_s; a.kappa_dt = h->kappa_dt;
    a.solid = h->n_sub_solid == 1 && h->n_tiles > 0;
    a.dt_s = h->dt / h->n_sub_solid;
    a.h = h->h;
    a.part = (double *)h->part;
    a.m_total = m_total;
    a.v_ff = h->v_ff;
    a.cff = (double *)h->cff;
    for (int s = 0; s < n_steps; ++s) {
        double *in = (s % 2 == 0) ? c : tmp, *out = (s % 2 == 0) ? tmp : c;
        double *row = (double *)h->hist + 3 * (int64_t)s;
        // 1. fast diffusion of the near-field liquid: mapping and product
        if ((rc = coarse_map_apply(h->coarse, in, (const double *)h->cff, st, &a.cnew))) return rc;
        // remapping, the reaction passes and (one sub-step) the solid step
        // and Eq. 7, tile by tile
        a.c_in = in;
        a.out = out;
        a.hist_row = row;
        e = launch_mp_local(a, st);
        if (e == hipSuccess && !a.solid) {
            // several solid sub-steps on the solid list (or no active tile),
            // then Eq. 7
            e = launch_mp_solid((const int *)h->sol, h->n_sol, (const double *)h->slam, (const int *)h->snb, h->nx,
                                h->ny, h->n_sub_solid, out, (double *)h->sa, (double *)h->sb, st);
            if (e == hipSuccess)
                e = launch_mp_balance((const int *)h->act, h->n_act, node, out, (double *)h->part, m_total,
                                      h->v_ff, (double *)h->cff, row, st);
        }
        if (e != hipSuccess) return hip_fail(e, "integrated step launch");
    }
    // the far-field cells take c_ff; after an odd count the field is in tmp
    if (n_steps > 0 && (e = launch_mp_far_fill(node, h->n, (const double *)h->cff, n_steps % 2 ? tmp : c, c, st)) !=
                           hipSuccess)
        return hip_fail(e, "far-field fill");
    if (stats && (e = hipEventRecord(ev.b, st)) != hipSuccess) return hip_fail(e, "event record");
    double cff = *c_ff;
    e = hipMemcpyAsync(&cff, h->cff, sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && history && n_steps > 0)
        e = hipMemcpyAsync(history, h->hist, (size_t)3 * n_steps * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "integrated step");
    *c_ff = cff;
    if (stats) {
        fdirw_stats loc;
        std::memset(&loc, 0, sizeof loc);
        loc.mass_in = m_total;
        loc.mass_out = m_total;
        if (n_steps > 0) {
            double last[3];
            e = hipMemcpy(last, (double *)h->hist + 3 * (int64_t)(n_steps - 1), sizeof last, hipMemcpyDeviceToHost);
            if (e != hipSuccess) return hip_fail(e, "history copy");
            loc.mass_out = last[0] + last[1] + last[2] * h->v_ff;
        }
        loc.kmass_min = INFINITY;
        loc.kmass_max = -INFINITY;
        loc.n_sources = h->n_faces;
        loc.kernel_seconds = ev.seconds();
        loc.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        *stats = loc;
    }
    return FDIRW_OK;
}

int fdirw_mp_info(const void *handle, int64_t *n_faces, void **coarse)
{
    const Mp *h = (const Mp *)handle;
    if (!h) return fail(FDIRW_E_ARG, "solver handle is null");
    if (n_faces) *n_faces = h->n_faces;
    if (coarse) *coarse = h->coarse;
    return FDIRW_OK;
}

int fdirw_mp_destroy(void *handle)
{
    Mp *h = (Mp *)handle;
    if (!h) return FDIRW_OK;
    int dev = -1;
    (void)hipGetDevice(&dev);
    const int own = h->dev;
    if (dev != own) (void)hipSetDevice(own);
    delete h;
    if (dev != own && dev >= 0) (void)hipSetDevice(dev);
    return FDIRW_OK;
}

}  // extern "C"
