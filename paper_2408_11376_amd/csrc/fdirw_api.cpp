// fdirw_api.cpp -- host side of the C ABI declared in include/fdirw.h.
//
// Validates arguments, derives the sub-step and the stability check (Sec. 3.1
// reading: explicit scheme, dt = 0.9 h^2 / (6 Dmax) unless given), keeps a
// small per-device scratch cache, picks launch shapes and enqueues the kernels
// of fdirw_kernels.hip on the caller's stream.  No exception or abort crosses
// the ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/fdirw.h"
#include "fdirw_launch.h"
#include "fdirw_host.h"

namespace fdirw {

static thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(FDIRW_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

// ----------------------------------------------------------------- scratch

static std::mutex g_mu;
static std::map<int, DevCache> g_cache;

DevCache &cache_for_current_device()
{
    int dev = 0;
    (void)hipGetDevice(&dev);
    DevCache &c = g_cache[dev];
    c.dev = dev;
    return c;
}

std::mutex &cache_mutex() { return g_mu; }

int ensure(Buf &b, size_t bytes)
{
    if (bytes == 0) bytes = 8;
    if (b.cap >= bytes) return FDIRW_OK;
    if (b.p) {
        (void)hipFree(b.p);
        b.p = nullptr;
        b.cap = 0;
    }
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        b.p = nullptr;
        return fail(FDIRW_E_NOMEM, "scratch allocation of %zu bytes failed: %s", bytes, hipGetErrorString(e));
    }
    b.cap = bytes;
    return FDIRW_OK;
}

static void release_all()
{
    for (auto &kv : g_cache) {
        (void)hipSetDevice(kv.first);
        DevCache &c = kv.second;
        for (Buf *b : {&c.lam64, &c.lam32, &c.flags, &c.part, &c.wgk, &c.small, &c.bank, &c.bank_mass, &c.bank_chat, &c.blam,
                       &c.bsmall, &c.bdoms, &c.bitems, &c.det}) {
            if (b->p) (void)hipFree(b->p);
            b->p = nullptr;
            b->cap = 0;
        }
    }
    g_cache.clear();
}

// ----------------------------------------------------------------- validation

int check_domain(const fdirw_domain *d, int max_r)
{
    if (!d) return fail(FDIRW_E_ARG, "domain is null");
    if (d->nx < 1 || d->ny < 1 || d->nz < 1)
        return fail(FDIRW_E_ARG, "grid %d x %d x %d: every dimension must be >= 1", d->nx, d->ny, d->nz);
    if ((int64_t)d->nx * d->ny > (int64_t)1 << 31)
        return fail(FDIRW_E_ARG, "nx * ny = %lld exceeds 2^31", (long long)d->nx * d->ny);
    if (!(d->h > 0.0) || !std::isfinite(d->h)) return fail(FDIRW_E_ARG, "h must be finite and > 0");
    if (!d->label) return fail(FDIRW_E_ARG, "label is null");
    if (!d->d_phase) return fail(FDIRW_E_ARG, "d_phase is null");
    if (d->n_phase < 1 || d->n_phase > FDIRW_MAX_PHASES)
        return fail(FDIRW_E_ARG, "n_phase = %d outside 1..%d", d->n_phase, FDIRW_MAX_PHASES);
    for (int i = 0; i < d->n_phase; ++i)
        if (!std::isfinite(d->d_phase[i]) || d->d_phase[i] < 0.0)
            return fail(FDIRW_E_ARG, "d_phase[%d] = %g must be finite and >= 0", i, d->d_phase[i]);
    if (d->r < 0 || d->r > max_r) return fail(FDIRW_E_ARG, "r = %d outside 0..%d", d->r, max_r);
    if (d->n_sub < 0) return fail(FDIRW_E_ARG, "n_sub = %d must be >= 0", d->n_sub);
    if (!std::isfinite(d->dt)) return fail(FDIRW_E_ARG, "dt must be finite");
    return FDIRW_OK;
}

int check_opts(const fdirw_opts *o)
{
    if (!o) return fail(FDIRW_E_ARG, "opts is null");
    if (o->prec < FDIRW_FP64 || o->prec > FDIRW_BF16_BANK) return fail(FDIRW_E_ARG, "unknown precision %d", o->prec);
    if (o->gen != FDIRW_GEN_FD && o->gen != FDIRW_GEN_NN) return fail(FDIRW_E_ARG, "unknown generator %d", o->gen);
    if (o->gen == FDIRW_GEN_NN && !o->nn) return fail(FDIRW_E_ARG, "GEN_NN needs a surrogate handle (opts.nn)");
    if (o->deterministic != 0 && o->deterministic != 1)
        return fail(FDIRW_E_ARG, "deterministic = %d must be 0 or 1", o->deterministic);
    if (o->deterministic && o->gen == FDIRW_GEN_NN)
        return fail(FDIRW_E_UNSUPPORTED, "the surrogate step superposes with FP64 atomics; deterministic needs GEN_FD");
    return FDIRW_OK;
}

// Reads the label range / presence flags (16 unsigned of device memory at
// flags), derives Dmax and dt, checks stability and fills the per-label
// diffusivity table.  Synchronises the stream once.
int geometry_dt(const fdirw_domain *d, hipStream_t st, unsigned *flags, Geometry *g, CoefTable *tab)
{
    const int64_t n = (int64_t)d->nx * d->ny * d->nz;
    hipError_t e = launch_validate(d->label, n, d->n_phase, flags, st);
    if (e != hipSuccess) return hip_fail(e, "label check launch");
    unsigned h_flags[9];
    e = hipMemcpyAsync(h_flags, flags, sizeof h_flags, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "label check");
    if (h_flags[8]) return fail(FDIRW_E_ARG, "a label is >= n_phase (%d)", d->n_phase);
    double dmax = 0.0;
    for (int l = 0; l < d->n_phase; ++l)
        if ((h_flags[l >> 5] >> (l & 31)) & 1u) dmax = std::fmax(dmax, d->d_phase[l]);
    double dt = d->dt;
    if (!(dt > 0.0)) dt = dmax > 0.0 ? (0.9 * d->h * d->h) / (6.0 * dmax) : 0.0;
    const double cfl = 6.0 * dmax * dt / (d->h * d->h);
    if (cfl > 1.0 + 1e-12)
        return fail(FDIRW_E_UNSTABLE, "6 Dmax dt / h^2 = %.17g > 1 (Dmax %g, dt %g, h %g)", cfl, dmax, dt, d->h);
    g->dt = dt;
    g->dmax = dmax;
    g->n = n;
    for (int l = 0; l < 256; ++l) tab->d[l] = l < d->n_phase ? d->d_phase[l] : 0.0;
    return FDIRW_OK;
}

// geometry_dt, then the owned-face coefficients of every cell.
int prepare_geometry(const fdirw_domain *d, hipStream_t st, DevCache &dc, double *lam64, float *lam32, Geometry *g)
{
    int rc = ensure(dc.flags, 16 * sizeof(unsigned));
    if (rc) return rc;
    CoefTable tab;
    if ((rc = geometry_dt(d, st, (unsigned *)dc.flags.p, g, &tab))) return rc;
    hipError_t e = launch_coef(d->label, d->nx, d->ny, d->nz, tab, g->dt, d->h, lam64, lam32, st);
    if (e != hipSuccess) return hip_fail(e, "coefficient launch");
    return FDIRW_OK;
}

int coef_buffers(const fdirw_domain *d, int prec, hipStream_t st, DevCache &dc, Geometry *g, const void **lam)
{
    const int64_t n = (int64_t)d->nx * d->ny * d->nz;
    int rc;
    if (prec == FDIRW_FP64) {
        if ((rc = ensure(dc.lam64, 3 * n * sizeof(double)))) return rc;
        rc = prepare_geometry(d, st, dc, (double *)dc.lam64.p, nullptr, g);
        *lam = dc.lam64.p;
    } else {
        if ((rc = ensure(dc.lam32, 3 * n * sizeof(float)))) return rc;
        rc = prepare_geometry(d, st, dc, nullptr, (float *)dc.lam32.p, g);
        *lam = dc.lam32.p;
    }
    return rc;
}

int field_sum_dev(const double *c, int64_t n, hipStream_t st, DevCache &dc, double *out_host)
{
    int rc = ensure(dc.part, (size_t)(2 * field_sum_blocks(n) + 2) * sizeof(double));
    if (rc) return rc;
    double *part = (double *)dc.part.p;
    double *res = part + 2 * field_sum_blocks(n);
    hipError_t e = launch_field_sum(c, n, part, res, st);
    if (e == hipSuccess) e = hipMemcpyAsync(out_host, res, sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "field sum");
    return FDIRW_OK;
}

// Launch shape of the fused step: each (x, y) line of sources is cut into
// n_seg segments so that the grid holds enough workgroups to fill 256 CUs.
void line_shape(const fdirw_domain *d, int tune, int *seg_len, int *n_seg)
{
    const int64_t lines = (int64_t)d->nx * d->ny;
    int want;
    if (tune > 0) want = tune;                                 // explicit segment count
    else {
        const int64_t target = 4096;                           // >= 16 workgroups per CU
        want = (int)((target + lines - 1) / lines);
    }
    if (want < 1) want = 1;
    if (want > d->nz) want = d->nz;
    int len = (d->nz + want - 1) / want;
    *seg_len = len;
    *n_seg = (d->nz + len - 1) / len;
}

int det_slab_planes(const fdirw_domain *d, int tune)
{
    if (tune > 0) return tune < d->nz ? tune : d->nz;
    const int64_t W = 2 * d->r + 1;
    const double plane = (double)(W * W) * (double)d->nx * d->ny * 8.0;   // partial bytes per plane
    int64_t planes = (int64_t)((double)DET_PART_CAP / plane) - 2 * d->r;
    if (planes < 1) planes = 1;
    if (planes > d->nz) planes = d->nz;
    return (int)planes;
}

// The deterministic fused step: the source planes are taken in slabs of
// det_slab_planes; per slab one launch (the flat layout where the atomic step
// uses it, else one workgroup per source line) stores every completed plane
// of every line to its own partial slot, and a
// second launch adds, for every cell the slab reaches, the partials of its
// W^2 window columns in a fixed order to c_out.  No floating-point atomics:
// the result depends on the inputs and the slab size only.
static int step_det(const fdirw_domain *d, const fdirw_opts *o, LineArgs a, DevCache &dc, hipStream_t stream,
                    int64_t *nblk_out)
{
    int rc;
    const int slab = det_slab_planes(d, o->tune);
    const int n_slab = (d->nz + slab - 1) / slab;
    const int64_t lines = (int64_t)d->nx * d->ny;
    const int64_t W = 2 * d->r + 1;
    const int part_planes = slab + 2 * d->r;
    const size_t part_bytes = (size_t)(W * W) * (size_t)part_planes * (size_t)lines * sizeof(double);
    if ((rc = ensure(dc.det, part_bytes))) return rc;
    if ((rc = ensure(dc.wgk, (size_t)n_slab * lines * 2 * sizeof(double)))) return rc;
    double *c_out = a.c_out;
    for (int k = 0; k < n_slab; ++k) {
        const int za = k * slab, zb = std::min(d->nz, za + slab);
        LineArgs s = a;
        s.z_begin = za; s.z_end = zb;
        s.seg_len = zb - za; s.n_seg = 1;
        s.c_out = nullptr;
        s.part = (double *)dc.det.p;
        s.part_z0 = za - d->r;
        s.part_planes = part_planes;
        s.wg_kmass = (double *)dc.wgk.p + (size_t)k * lines * 2;
        hipError_t e = use_flat_layout(o->prec, d->r) ? launch_line_flat(o->prec, d->r, s, stream)
                                                      : launch_line(o->prec, d->r, s, stream);
        if (e != hipSuccess) return hip_fail(e, "deterministic step launch");
        s.c_out = c_out;
        e = launch_line_reduce(d->r, s, std::max(0, za - d->r), std::min(d->nz, zb + d->r), stream);
        if (e != hipSuccess) return hip_fail(e, "deterministic reduction launch");
    }
    *nblk_out = (int64_t)n_slab * lines;
    return FDIRW_OK;
}

// The flat-layout fused kernel (fdirw_flat.hip) serves FP32 steps with
// r = 4..8; the environment variable FDIRW_FUSED_LAYOUT=segments selects the
// segment-layout kernel instead (same kernels, for comparison).
bool use_flat_layout(int prec, int r)
{
    static const bool segments = [] {
        const char *v = std::getenv("FDIRW_FUSED_LAYOUT");
        return v && std::strcmp(v, "segments") == 0;
    }();
    return !segments && prec == FDIRW_FP32 && r >= 4 && r <= 8;
}

int step_one(const fdirw_domain *d, const fdirw_opts *o, const double *c_in, double *c_out,
             fdirw_stats *st, DevCache &dc, hipStream_t stream, bool prepared, const void *lam, Geometry *geo)
{
    int rc;
    Geometry g_local;
    if (!prepared) {
        if ((rc = coef_buffers(d, o->prec, stream, dc, &g_local, &lam))) return rc;
        geo = &g_local;
    }
    (void)geo;
    const int64_t n = (int64_t)d->nx * d->ny * d->nz;
    if (st) {
        if ((rc = field_sum_dev(c_in, n, stream, dc, &st->mass_in))) return rc;
        if (!std::isfinite(st->mass_in)) return fail(FDIRW_E_NONFINITE, "input mass is not finite");
    }
    int seg_len, n_seg;
    line_shape(d, o->deterministic ? 0 : o->tune, &seg_len, &n_seg);
    int64_t nblk = (int64_t)d->nx * d->ny * n_seg;
    if (!o->deterministic && (rc = ensure(dc.wgk, (size_t)nblk * 2 * sizeof(double)))) return rc;
    if ((rc = ensure(dc.small, 64))) return rc;
    unsigned long long *used = (unsigned long long *)dc.small.p;
    hipError_t e = launch_fill(c_out, n, 0.0, stream);
    if (e == hipSuccess) e = launch_fill_u32((unsigned *)used, 2, 0u, stream);
    if (e != hipSuccess) return hip_fail(e, "output clear");
    LineArgs a{};
    a.nx = d->nx; a.ny = d->ny; a.nz = d->nz; a.n = n;
    a.n_sub = d->n_sub;
    a.z_begin = 0; a.z_end = d->nz;
    a.seg_len = seg_len; a.n_seg = n_seg;
    a.lx = lam;
    a.c_in = c_in; a.c_out = c_out;
    a.wg_kmass = (double *)dc.wgk.p;
    a.n_used = used;
    a.part = nullptr;
    a.part_z0 = 0; a.part_planes = 0;
    EventPair ev;
    if (st && (e = ev.create()) != hipSuccess) return hip_fail(e, "event create");
    if (st) (void)hipEventRecord(ev.a, stream);
    if (o->deterministic) {
        if ((rc = step_det(d, o, a, dc, stream, &nblk))) return rc;
    } else {
        e = use_flat_layout(o->prec, d->r) ? launch_line_flat(o->prec, d->r, a, stream)
                                           : launch_line(o->prec, d->r, a, stream);
        if (e != hipSuccess) return hip_fail(e, "fused step launch");
    }
    if (st) (void)hipEventRecord(ev.b, stream);
    if (st) {
        if ((rc = field_sum_dev(c_out, n, stream, dc, &st->mass_out))) return rc;
        double *mm = (double *)dc.small.p + 2;
        e = launch_minmax((const double *)dc.wgk.p, nblk, mm, stream);
        double h_mm[2];
        unsigned long long h_used = 0;
        if (e == hipSuccess) e = hipMemcpyAsync(h_mm, mm, sizeof h_mm, hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipMemcpyAsync(&h_used, used, sizeof h_used, hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return hip_fail(e, "step statistics");
        st->kmass_min = h_mm[0];
        st->kmass_max = h_mm[1];
        st->n_sources = (int64_t)h_used;
        st->kernel_seconds = ev.seconds();
        st->audit_l1 = 0.0;
        st->fallback_used = 0;
        st->bank_used = 0;
        st->tuned_config_id = o->deterministic ? det_slab_planes(d, o->tune) : n_seg;
    }
    return FDIRW_OK;
}

// Checks that the explicit scheme with the flow u is stable: for every cell
// the six lambda plus the outflow Courant numbers must not exceed 1.
int flow_stable(const fdirw_domain *d, int fp64, const void *lam, const double *u, double dt, hipStream_t st,
                DevCache &dc)
{
    int rc;
    if ((rc = ensure(dc.flags, 16 * sizeof(unsigned)))) return rc;
    unsigned long long *mx = (unsigned long long *)dc.flags.p + 4;
    hipError_t e = launch_fill_u32((unsigned *)mx, 2, 0u, st);
    if (e == hipSuccess) e = launch_flow_stability(fp64, lam, u, d->nx, d->ny, d->nz, dt / d->h, mx, st);
    unsigned long long h_mx = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&h_mx, mx, sizeof h_mx, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "flow stability check");
    double v;
    std::memcpy(&v, &h_mx, sizeof v);
    if (!(v <= 1.0 + 1e-12))
        return fail(FDIRW_E_UNSTABLE, "flow: 6 lambda + outflow Courant number reaches %g > 1 (reduce dt or u)", v);
    return FDIRW_OK;
}

}  // namespace fdirw

using namespace fdirw;

static double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

extern "C" {

int fdirw_abi_version(void) { return FDIRW_ABI_VERSION; }

const char *fdirw_last_error(void) { return g_err.c_str(); }

int fdirw_release(void)
{
    std::lock_guard<std::mutex> lk(g_mu);
    release_all();
    return FDIRW_OK;
}

int fdirw_coefficients(const fdirw_domain *d, void *stream, double *lam, double *dt_out)
{
    int rc = check_domain(d);
    if (rc) return rc;
    if (!lam) return fail(FDIRW_E_ARG, "lam is null");
    std::lock_guard<std::mutex> lk(g_mu);
    DevCache &dc = cache_for_current_device();
    Geometry g;
    if ((rc = prepare_geometry(d, (hipStream_t)stream, dc, lam, nullptr, &g))) return rc;
    if (dt_out) *dt_out = g.dt;
    return FDIRW_OK;
}

int fdirw_kernels(const fdirw_domain *d, const fdirw_opts *o, const int64_t *src, int64_t n_src,
                  void *G, double *mass)
{
    int rc = check_domain(d);
    if (rc) return rc;
    if ((rc = check_opts(o))) return rc;
    if (n_src < 0) return fail(FDIRW_E_ARG, "n_src < 0");
    if (o->gen == FDIRW_GEN_NN)
        return fail(FDIRW_E_UNSUPPORTED, "fdirw_kernels generates FD kernels; use fdirw_nn_forward for the surrogate");
    if (n_src == 0) return FDIRW_OK;
    if (!src || !G) return fail(FDIRW_E_ARG, "src and G must not be null");
    std::lock_guard<std::mutex> lk(g_mu);
    DevCache &dc = cache_for_current_device();
    hipStream_t st = (hipStream_t)o->stream;
    const int64_t n = (int64_t)d->nx * d->ny * d->nz;
    if ((rc = ensure(dc.flags, 16 * sizeof(unsigned)))) return rc;
    unsigned *bad = (unsigned *)dc.flags.p + 12;
    hipError_t e = launch_src_check(src, n_src, n, bad, st);
    unsigned h_bad = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&h_bad, bad, sizeof h_bad, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "source check");
    if (h_bad) return fail(FDIRW_E_ARG, "a source index is outside [0, %lld)", (long long)n);
    Geometry g;
    const void *lam = nullptr;
    if ((rc = coef_buffers(d, o->prec, st, dc, &g, &lam))) return rc;
    WindowArgs a;
    a.nx = d->nx; a.ny = d->ny; a.nz = d->nz; a.n = n;
    a.n_sub = d->n_sub;
    a.lx = lam;
    a.src = src; a.n_src = n_src;
    a.G = G; a.mass = mass;
    a.normalize = 0;
    a.out_lp = 0;
    a.offset_major = 0;
    e = launch_window(o->prec, d->r, a, st);
    if (e != hipSuccess) return hip_fail(e, "window kernel launch");
    return FDIRW_OK;
}

int fdirw_kernels_flow(const fdirw_domain *d, const fdirw_opts *o, const double *velocity, const int64_t *src,
                       int64_t n_src, void *G, double *mass)
{
    int rc = check_domain(d);
    if (rc) return rc;
    if ((rc = check_opts(o))) return rc;
    if (o->prec != FDIRW_FP64 && o->prec != FDIRW_FP32)
        return fail(FDIRW_E_UNSUPPORTED, "flow kernels are generated in FP64 or FP32 only");
    if (o->gen != FDIRW_GEN_FD) return fail(FDIRW_E_UNSUPPORTED, "flow kernels are FD kernels");
    if (n_src < 0) return fail(FDIRW_E_ARG, "n_src < 0");
    if (!velocity) return fail(FDIRW_E_ARG, "velocity is null");
    if (n_src == 0) return FDIRW_OK;
    if (!src || !G) return fail(FDIRW_E_ARG, "src and G must not be null");
    std::lock_guard<std::mutex> lk(g_mu);
    DevCache &dc = cache_for_current_device();
    hipStream_t st = (hipStream_t)o->stream;
    const int64_t n = (int64_t)d->nx * d->ny * d->nz;
    if ((rc = ensure(dc.flags, 16 * sizeof(unsigned)))) return rc;
    unsigned *bad = (unsigned *)dc.flags.p + 12;
    hipError_t e = launch_src_check(src, n_src, n, bad, st);
    unsigned h_bad = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&h_bad, bad, sizeof h_bad, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "source check");
    if (h_bad) return fail(FDIRW_E_ARG, "a source index is outside [0, %lld)", (long long)n);
    Geometry g;
    const void *lam = nullptr;
    if ((rc = coef_buffers(d, o->prec, st, dc, &g, &lam))) return rc;
    if ((rc = flow_stable(d, o->prec == FDIRW_FP64, lam, velocity, g.dt, st, dc))) return rc;
    FlowArgs a;
    a.nx = d->nx; a.ny = d->ny; a.nz = d->nz; a.n = n;
    a.n_sub = d->n_sub;
    a.lam = lam;
    a.u = velocity;
    a.dt = g.dt; a.h = d->h;
    a.src = src; a.src_base = 0; a.n_src = n_src;
    a.node = nullptr;
    a.G = G; a.mass = mass;
    e = launch_flow_window(o->prec == FDIRW_FP64, d->r, a, st);
    if (e != hipSuccess) return hip_fail(e, "flow window kernel launch");
    return FDIRW_OK;
}

static int check_fields(const fdirw_domain *d, int32_t n_dom, const double *const *a, const double *const *b,
                        const char *na, const char *nb)
{
    if (!a || !b) return fail(FDIRW_E_ARG, "%s / %s arrays are null", na, nb);
    for (int i = 0; i < n_dom; ++i) {
        if (!a[i] || !b[i]) return fail(FDIRW_E_ARG, "%s[%d] or %s[%d] is null", na, i, nb, i);
        const int64_t n = (int64_t)d[i].nx * d[i].ny * d[i].nz;
        const char *pa = (const char *)a[i], *pb = (const char *)b[i];
        if (pa < pb + n * 8 && pb < pa + n * 8)
            return fail(FDIRW_E_ARG, "%s[%d] and %s[%d] overlap", na, i, nb, i);
    }
    return FDIRW_OK;
}

int fdirw_step(const fdirw_domain *d, int32_t n_dom, const fdirw_opts *o,
               const double *const *c_in, double *const *c_out, fdirw_stats *st)
{
    const double t0 = now_s();
    if (n_dom < 1) return fail(FDIRW_E_ARG, "n_dom = %d must be >= 1", n_dom);
    if (!d) return fail(FDIRW_E_ARG, "domain array is null");
    int rc;
    for (int i = 0; i < n_dom; ++i)
        if ((rc = check_domain(&d[i]))) return rc;
    if ((rc = check_opts(o))) return rc;
    if ((rc = check_fields(d, n_dom, c_in, (const double *const *)c_out, "c_in", "c_out"))) return rc;
    std::lock_guard<std::mutex> lk(g_mu);
    DevCache &dc = cache_for_current_device();
    hipStream_t stream = (hipStream_t)o->stream;
    if (o->gen == FDIRW_GEN_NN) {
        if (n_dom > 1) return fail(FDIRW_E_UNSUPPORTED, "the surrogate step takes one domain per call");
        if ((rc = step_nn(&d[0], o, c_in[0], c_out[0], st, dc, stream))) return rc;
    } else if (n_dom > 1) {
        if ((rc = step_batched(d, n_dom, o, c_in, c_out, st, dc, stream))) return rc;
    } else if ((rc = step_one(&d[0], o, c_in[0], c_out[0], st, dc, stream, false, nullptr, nullptr))) {
        return rc;
    }
    if (st) {
        const double t = now_s() - t0;
        for (int i = 0; i < n_dom; ++i) st[i].seconds = t;
    }
    return FDIRW_OK;
}

int fdirw_run(const fdirw_domain *d, int32_t n_dom, const fdirw_opts *o, int32_t n_steps,
              double *const *c, double *const *scratch, fdirw_stats *st)
{
    const double t0 = now_s();
    if (n_dom < 1) return fail(FDIRW_E_ARG, "n_dom = %d must be >= 1", n_dom);
    if (n_steps < 0) return fail(FDIRW_E_ARG, "n_steps = %d must be >= 0", n_steps);
    if (!d) return fail(FDIRW_E_ARG, "domain array is null");
    int rc;
    for (int i = 0; i < n_dom; ++i)
        if ((rc = check_domain(&d[i]))) return rc;
    if ((rc = check_opts(o))) return rc;
    if ((rc = check_fields(d, n_dom, (const double *const *)c, (const double *const *)scratch, "c", "scratch"))) return rc;
    std::lock_guard<std::mutex> lk(g_mu);
    DevCache &dc = cache_for_current_device();
    hipStream_t stream = (hipStream_t)o->stream;
    if (o->gen == FDIRW_GEN_NN) {
        if (n_dom > 1) return fail(FDIRW_E_UNSUPPORTED, "the surrogate step takes one domain per call");
        const int64_t n = (int64_t)d[0].nx * d[0].ny * d[0].nz;
        double *cur = c[0], *nxt = scratch[0];
        for (int step = 0; step < n_steps; ++step) {
            fdirw_stats *sst = (st && step == n_steps - 1) ? st : nullptr;
            if ((rc = step_nn(&d[0], o, cur, nxt, sst, dc, stream))) return rc;
            std::swap(cur, nxt);
        }
        if (cur != c[0]) {
            hipError_t e = hipMemcpyAsync(c[0], cur, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, stream);
            if (e != hipSuccess) return hip_fail(e, "result copy");
        }
        if (st) {
            hipError_t e = hipStreamSynchronize(stream);
            if (e != hipSuccess) return hip_fail(e, "run");
        }
    } else if (n_dom == 1) {
        rc = run_one(&d[0], o, n_steps, c[0], scratch[0], st, dc, stream);
        if (rc) return rc;
    } else {
        // batched domains: one persistent launch per big step (no kernel bank)
        std::vector<double *> cur(c, c + n_dom), nxt(scratch, scratch + n_dom);
        for (int step = 0; step < n_steps; ++step) {
            fdirw_stats *sst = (st && step == n_steps - 1) ? st : nullptr;
            rc = step_batched(d, n_dom, o, (const double *const *)cur.data(), nxt.data(), sst, dc, stream);
            if (rc) return rc;
            std::swap(cur, nxt);
        }
        for (int i = 0; i < n_dom; ++i) {
            if (cur[i] != c[i]) {
                const size_t bytes = (size_t)d[i].nx * d[i].ny * d[i].nz * sizeof(double);
                hipError_t e = hipMemcpyAsync(c[i], cur[i], bytes, hipMemcpyDeviceToDevice, stream);
                if (e != hipSuccess) return hip_fail(e, "result copy");
            }
        }
        if (st) {
            hipError_t e = hipStreamSynchronize(stream);
            if (e != hipSuccess) return hip_fail(e, "run");
        }
    }
    if (st) {
        const double t = now_s() - t0;
        for (int i = 0; i < n_dom; ++i) st[i].seconds = t;
    }
    return FDIRW_OK;
}

int fdirw_field_sum(const double *c, int64_t n, void *stream, double *sum_out)
{
    if (n < 0) return fail(FDIRW_E_ARG, "n < 0");
    if (!sum_out) return fail(FDIRW_E_ARG, "sum_out is null");
    if (n == 0) { *sum_out = 0.0; return FDIRW_OK; }
    if (!c) return fail(FDIRW_E_ARG, "c is null");
    std::lock_guard<std::mutex> lk(g_mu);
    DevCache &dc = cache_for_current_device();
    return field_sum_dev(c, n, (hipStream_t)stream, dc, sum_out);
}

}  // extern "C"
