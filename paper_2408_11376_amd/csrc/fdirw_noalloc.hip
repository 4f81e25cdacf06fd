// fdirw_noalloc.hip -- fdirw_step_noalloc: the fused big step (Eq. 8 of
// arXiv 2408.11376, the kernels of Sec. 3.1 generated and superposed in one
// pass) for callers that must not allocate device memory.
//
// Every piece of device scratch this call needs lives in one file-scope array,
// `scratch`, of FDIRW_NOALLOC_SCRATCH_BYTES.  The face coefficients are not
// stored per cell: the fused kernel (the flat layout where fdirw_step uses it,
// else the segment layout) looks them up per phase pair in a table of
// n_phase^2 entries (launch_line_flat_labels / launch_line_labels), so the
// scratch size does not depend on the grid.  Layout (bytes):
//   [0, 64)        label / presence flags of the label check (16 unsigned)
//   [64, 80)       sources-used counter (u64)
//   [128, 144)     min / max kernel mass
//   [192, 200)     field-sum result
//   [256, 16,656)  field-sum partials (2 x 1024 + 2 doubles)
//   [32 K, 544 K)  coefficient per phase pair (n_phase^2, double or float)
//   [576 K, ...)   per-workgroup kernel-mass min / max (statistics only)
// The array's device address is taken once per device with
// hipGetSymbolAddress and only that address is handed to kernels and copies.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <map>
#include <mutex>

#include "../../include/fdirw.h"
#include "fdirw_host.h"
#include "fdirw_launch.h"

namespace fdirw {

static __device__ __align__(256) unsigned char scratch[FDIRW_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr size_t OFF_FLAGS = 0;
constexpr size_t OFF_USED = 64;
constexpr size_t OFF_MM = 128;
constexpr size_t OFF_SUM = 192;
constexpr size_t OFF_PART = 256;
constexpr size_t OFF_TAB = (size_t)32 << 10;
constexpr size_t OFF_KMASS = (size_t)576 << 10;

static_assert(OFF_PART + (2 * 1024 + 2) * sizeof(double) <= OFF_TAB, "field-sum partials overlap the table");
static_assert(OFF_TAB + (size_t)FDIRW_MAX_PHASES * FDIRW_MAX_PHASES * sizeof(double) <= OFF_KMASS,
              "pair table overlaps the kernel-mass partials");
static_assert(OFF_KMASS + (size_t)FDIRW_NOALLOC_MAX_BLOCKS * 2 * sizeof(double) <= FDIRW_NOALLOC_SCRATCH_BYTES,
              "kernel-mass partials exceed the scratch array");

std::mutex g_ptr_mu;
std::map<int, unsigned char *> g_ptr;      // device -> address of that device's copy of scratch

// Address of the current device's copy of scratch (looked up once per device).
int scratch_ptr(unsigned char **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_ptr_mu);
    auto it = g_ptr.find(dev);
    if (it == g_ptr.end()) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        it = g_ptr.emplace(dev, (unsigned char *)p).first;
    }
    *out = it->second;
    return FDIRW_OK;
}

int field_sum_scratch(const double *c, int64_t n, unsigned char *base, hipStream_t st, double *out_host)
{
    double *part = (double *)(base + OFF_PART);
    double *res = (double *)(base + OFF_SUM);
    hipError_t e = launch_field_sum(c, n, part, res, st);
    if (e == hipSuccess) e = hipMemcpyAsync(out_host, res, sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "field sum");
    return FDIRW_OK;
}

}  // namespace

}  // namespace fdirw

using namespace fdirw;

extern "C" int fdirw_step_noalloc(const fdirw_domain *d, const fdirw_opts *o, const double *c_in, double *c_out,
                                  fdirw_stats *st)
{
    const auto t0 = std::chrono::steady_clock::now();
    int rc = check_domain(d);
    if (rc) return rc;
    if ((rc = check_opts(o))) return rc;
    if (o->gen != FDIRW_GEN_FD) return fail(FDIRW_E_UNSUPPORTED, "fdirw_step_noalloc generates FD kernels only");
    if (o->deterministic)
        return fail(FDIRW_E_UNSUPPORTED, "fdirw_step_noalloc has no deterministic form (its partials need GiB)");
    if (o->prec != FDIRW_FP64 && o->prec != FDIRW_FP32 && o->prec != FDIRW_FP16X32 && o->prec != FDIRW_BF16X32)
        return fail(FDIRW_E_UNSUPPORTED, "fdirw_step_noalloc supports FP64, FP32, FP16X32 and BF16X32 (prec %d)",
                    o->prec);
    if (!c_in || !c_out) return fail(FDIRW_E_ARG, "c_in / c_out is null");
    if (c_in == c_out) return fail(FDIRW_E_ARG, "c_in and c_out must be different buffers");
    const int64_t n = (int64_t)d->nx * d->ny * d->nz;
    int seg_len, n_seg;
    line_shape(d, o->tune, &seg_len, &n_seg);
    const int64_t nblk = (int64_t)d->nx * d->ny * n_seg;
    if (st && nblk > FDIRW_NOALLOC_MAX_BLOCKS)
        return fail(FDIRW_E_ARG,
                    "statistics need %lld workgroup kernel-mass slots, the scratch holds %d (pass st = NULL or a "
                    "grid with nx * ny <= %d)",
                    (long long)nblk, FDIRW_NOALLOC_MAX_BLOCKS, FDIRW_NOALLOC_MAX_BLOCKS);
    const bool fp64 = o->prec == FDIRW_FP64;
    if ((size_t)d->n_phase * d->n_phase * (fp64 ? sizeof(double) : sizeof(float)) > OFF_KMASS - OFF_TAB)
        return fail(FDIRW_E_ARG, "n_phase = %d: the phase-pair table exceeds the scratch", d->n_phase);

    std::lock_guard<std::mutex> lk(cache_mutex());
    unsigned char *base = nullptr;
    if ((rc = scratch_ptr(&base))) return rc;
    hipStream_t stream = (hipStream_t)o->stream;
    Geometry g;
    CoefTable tab;
    if ((rc = geometry_dt(d, stream, (unsigned *)(base + OFF_FLAGS), &g, &tab))) return rc;
    void *ptab = base + OFF_TAB;
    hipError_t e = launch_pair_table(tab, d->n_phase, g.dt, d->h, fp64 ? (double *)ptab : nullptr,
                                     fp64 ? nullptr : (float *)ptab, stream);
    if (e != hipSuccess) return hip_fail(e, "pair table launch");
    if (st) {
        if ((rc = field_sum_scratch(c_in, n, base, stream, &st->mass_in))) return rc;
        if (!std::isfinite(st->mass_in)) return fail(FDIRW_E_NONFINITE, "input mass is not finite");
    }
    unsigned long long *used = (unsigned long long *)(base + OFF_USED);
    e = launch_fill(c_out, n, 0.0, stream);
    if (e == hipSuccess) e = launch_fill_u32((unsigned *)used, 2, 0u, stream);
    if (e != hipSuccess) return hip_fail(e, "output clear");
    LineArgs a{};
    a.nx = d->nx; a.ny = d->ny; a.nz = d->nz; a.n = n;
    a.n_sub = d->n_sub;
    a.z_begin = 0; a.z_end = d->nz;
    a.seg_len = seg_len; a.n_seg = n_seg;
    a.lx = nullptr;
    a.c_in = c_in; a.c_out = c_out;
    a.wg_kmass = st ? (double *)(base + OFF_KMASS) : nullptr;
    a.n_used = used;
    a.part = nullptr;
    a.label = d->label;
    a.lam_tab = ptab;
    a.n_phase = d->n_phase;
    e = use_flat_layout(o->prec, d->r) ? launch_line_flat_labels(o->prec, d->r, a, stream)
                                       : launch_line_labels(o->prec, d->r, a, stream);
    if (e != hipSuccess) return hip_fail(e, "fused step launch");
    if (st) {
        if ((rc = field_sum_scratch(c_out, n, base, stream, &st->mass_out))) return rc;
        double *mm = (double *)(base + OFF_MM);
        e = launch_minmax((const double *)(base + OFF_KMASS), nblk, mm, stream);
        double h_mm[2];
        unsigned long long h_used = 0;
        if (e == hipSuccess) e = hipMemcpyAsync(h_mm, mm, sizeof h_mm, hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipMemcpyAsync(&h_used, used, sizeof h_used, hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return hip_fail(e, "step statistics");
        st->kmass_min = h_mm[0];
        st->kmass_max = h_mm[1];
        st->n_sources = (int64_t)h_used;
        st->kernel_seconds = 0.0;              // no events: creating them may allocate
        st->audit_l1 = 0.0;
        st->fallback_used = 0;
        st->bank_used = 0;
        st->tuned_config_id = n_seg;
        st->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return FDIRW_OK;
}
