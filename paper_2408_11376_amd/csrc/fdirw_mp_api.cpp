// fdirw_mp_api.cpp -- host side of the integrated near-field solver
// (include/fdirw.h; Sec. 2, Eqs. 1-7, and the flowchart of Sec. 3.4 of arXiv
// 2408.11376).
//
// A handle owns the coarse operator of the liquid (built by
// fdirw_coarse_create on the domain with the solid walled off), the six lists
// of interface faces, a second field buffer and the far-field value on the
// device.  A step launches, in order: mapping / product / remapping, the six
// reaction passes, the solid sub-steps, the two-level balance of Eq. 7 and
// the far-field fill; nothing returns to the host between steps.
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
    int nx = 0, ny = 0, nz = 0;
    int64_t n = 0;
    double h = 1.0, dt = 0.0;           // grid spacing, big step
    double kappa_dt = 0.0;              // k dt / (c_L^eq c_S^eq)
    double c_eq_l = 1.0, c_eq_s = 1.0, v_ff = 1.0;
    int n_sub_solid = 1;
    bool has_solid = false;
    const uint8_t *label = nullptr;     // caller's labels (device)
    SolidTable solid;
    void *coarse = nullptr;
    MpFaceLists lists;
    int64_t n_pass[6] = {0, 0, 0, 0, 0, 0};
    int64_t n_faces = 0;
    void *faces = nullptr;              // int64 entries of the six passes
    void *tmp = nullptr;                // double [N]
    void *part = nullptr;               // double [2 * MP_SUM_BLOCKS]
    void *cff = nullptr;                // double [1]
    void *hist = nullptr;               // double [3 * hist_cap]
    int64_t hist_cap = 0;

    ~Mp()
    {
        for (void *p : {faces, tmp, part, cff, hist})
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

}  // namespace

}  // namespace fdirw

using namespace fdirw;

extern "C" {

int fdirw_mp_create(const fdirw_domain *d, const fdirw_mp_params *p, int32_t block, int32_t prec, void *stream,
                    void **handle, double *seconds)
{
    if (!handle) return fail(FDIRW_E_ARG, "handle is null");
    *handle = nullptr;
    int rc = check_domain(d);
    if (rc) return rc;
    if ((rc = check_params(d, p))) return rc;
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t st = (hipStream_t)stream;
    // Eq. 1 with Eqs. 2-3: coefficient D A / RT per phase; the liquid's
    // kernels see the solid as a wall, the solid step sees the liquid as one
    std::vector<double> d_liq(d->n_phase), coef(d->n_phase);
    std::vector<uint8_t> grouped(d->n_phase), reservoir(d->n_phase);
    double dsol_max = 0.0;
    bool has_solid = false;
    for (int i = 0; i < d->n_phase; ++i) {
        coef[i] = d->d_phase[i] * (p->a_over_rt ? p->a_over_rt[i] : 1.0);
        if (!std::isfinite(coef[i])) return fail(FDIRW_E_ARG, "D A / RT of phase %d is not finite", i);
        d_liq[i] = p->role[i] == FDIRW_ROLE_SOLID ? 0.0 : coef[i];
        grouped[i] = p->role[i] == FDIRW_ROLE_LIQUID;
        reservoir[i] = p->role[i] == FDIRW_ROLE_FAR_FIELD;
        if (p->role[i] == FDIRW_ROLE_SOLID) {
            has_solid = true;
            dsol_max = std::fmax(dsol_max, coef[i]);
        }
    }
    const double dt = (double)d->n_sub * d->dt;
    const double dts = dt / p->n_sub_solid;
    const double cfl = 6.0 * dsol_max * dts / (d->h * d->h);
    if (cfl > 1.0 + 1e-12)
        return fail(FDIRW_E_UNSTABLE, "solid: 6 max(D A / RT) dt_s / h^2 = %.17g > 1 (raise n_sub_solid)", cfl);
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
    h->kappa_dt = p->k / (p->c_eq_liquid * p->c_eq_solid) * dt;
    h->v_ff = p->v_far_field;
    h->n_sub_solid = p->n_sub_solid;
    h->has_solid = has_solid;
    h->label = d->label;
    std::memset(&h->solid, 0, sizeof h->solid);
    for (int i = 0; i < d->n_phase; ++i) h->solid.d[i] = p->role[i] == FDIRW_ROLE_SOLID ? coef[i] : 0.0;
    fdirw_domain dl = *d;
    dl.d_phase = d_liq.data();
    if ((rc = fdirw_coarse_create(&dl, block, prec, grouped.data(), reservoir.data(), nullptr, stream, &h->coarse,
                                  nullptr))) {
        h->coarse = nullptr;
        delete h;
        return rc;
    }
    // interface faces: count, reserve, list
    unsigned long long *cnt = nullptr;
    rc = mp_alloc((void **)&cnt, 6 * sizeof(unsigned long long));
    if (!rc) rc = mp_alloc(&h->tmp, (size_t)h->n * sizeof(double));
    if (!rc) rc = mp_alloc(&h->part, (size_t)2 * MP_SUM_BLOCKS * sizeof(double));
    if (!rc) rc = mp_alloc(&h->cff, sizeof(double));
    if (rc) {
        (void)hipFree(cnt);
        delete h;
        return rc;
    }
    const int *node = coarse_node(h->coarse);
    std::memset(&h->lists, 0, sizeof h->lists);
    unsigned long long hc[6];
    hipError_t e = launch_fill_u32((unsigned *)cnt, 12, 0u, st);
    if (e == hipSuccess) e = launch_mp_faces(node, d->nx, d->ny, d->nz, h->lists, nullptr, cnt, st);
    if (e == hipSuccess) e = hipMemcpyAsync(hc, cnt, sizeof hc, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e == hipSuccess) {
        int64_t off = 0;
        for (int k = 0; k < 6; ++k) {
            h->lists.off[k] = off;
            h->lists.cap[k] = (int64_t)hc[k];
            h->n_pass[k] = (int64_t)hc[k];
            off += (int64_t)hc[k];
        }
        h->n_faces = off;
        if ((rc = mp_alloc(&h->faces, (size_t)off * sizeof(int64_t)))) {
            (void)hipFree(cnt);
            delete h;
            return rc;
        }
        e = launch_fill_u32((unsigned *)cnt, 12, 0u, st);
        if (e == hipSuccess)
            e = launch_mp_faces(node, d->nx, d->ny, d->nz, h->lists, (int64_t *)h->faces, cnt, st);
        if (e == hipSuccess) e = hipMemcpyAsync(hc, cnt, sizeof hc, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e == hipSuccess)
            for (int k = 0; k < 6; ++k)
                if ((int64_t)hc[k] != h->n_pass[k]) {
                    (void)hipFree(cnt);
                    delete h;
                    return fail(FDIRW_E_DEVICE, "interface face count changed between passes");
                }
    }
    (void)hipFree(cnt);
    if (e != hipSuccess) {
        delete h;
        return hip_fail(e, "interface faces");
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
    const int64_t stride[3] = {1, h->nx, (int64_t)h->nx * h->ny};
    for (int s = 0; s < n_steps; ++s) {
        // 1. fast diffusion of the near-field liquid: c -> tmp
        if ((rc = coarse_fast_step(h->coarse, c, tmp, (const double *)h->cff, st))) return rc;
        // 2. absorption at the interface, in place on tmp
        for (int k = 0; k < 6 && e == hipSuccess; ++k)
            e = launch_mp_react((const int64_t *)h->faces + h->lists.off[k], h->n_pass[k], stride[k / 2], tmp,
                                h->c_eq_l, h->c_eq_s, h->kappa_dt, st);
        // 3. slow diffusion in the solid, ping-pong between tmp and c
        double *cur = tmp, *nxt = c;
        if (h->has_solid)
            for (int k = 0; k < h->n_sub_solid && e == hipSuccess; ++k) {
                e = launch_mp_solid(h->label, h->solid, h->nx, h->ny, h->nz, h->dt / h->n_sub_solid, h->h, cur, nxt,
                                    st);
                double *t = cur; cur = nxt; nxt = t;
            }
        // 4. Eq. 7 and the far-field cells; the result ends in c
        if (e == hipSuccess)
            e = launch_mp_balance(node, cur, h->n, (double *)h->part, m_total, h->v_ff, (double *)h->cff,
                                  (double *)h->hist + 3 * (int64_t)s, st);
        if (e == hipSuccess) e = launch_mp_far_fill(node, h->n, (const double *)h->cff, cur, c, st);
        if (e != hipSuccess) return hip_fail(e, "integrated step launch");
    }
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
