// fdirw_host.h -- internal host helpers shared by the ABI translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stddef.h>
#include <stdint.h>

#include <mutex>

#include "../../include/fdirw.h"

namespace fdirw {

struct CoefTable;

struct Buf {
    void *p = nullptr;
    size_t cap = 0;
};

// Scratch kept per device: coefficients (FP64 / FP32), flag words, reduction
// partials, per-workgroup kernel masses, a few counters, and the kernel bank.
struct DevCache {
    int dev = -1;
    Buf lam64, lam32, flags, part, wgk, small, bank, bank_mass, bank_chat;
    Buf det;                              // deterministic step: per-column plane partials
    Buf blam, bsmall, bdoms, bitems;      // batched launch
};

// Two HIP events around one launch; destroyed with the object.
struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t create()
    {
        hipError_t e = hipEventCreate(&a);
        if (e == hipSuccess) e = hipEventCreate(&b);
        return e;
    }
    double seconds() const
    {
        float ms = 0.0f;
        if (a && b && hipEventElapsedTime(&ms, a, b) == hipSuccess) return 1e-3 * (double)ms;
        return -1.0;
    }
    ~EventPair()
    {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

struct Geometry {
    double dt = 0.0;
    double dmax = 0.0;
    int64_t n = 0;
};

int fail(int code, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);
int ensure(Buf &b, size_t bytes);
DevCache &cache_for_current_device();
std::mutex &cache_mutex();

int check_domain(const fdirw_domain *d, int max_r = FDIRW_MAX_RADIUS);
int check_opts(const fdirw_opts *o);
// Label validation (flags: 16 unsigned of device memory), Dmax, dt, the
// stability check and the per-label diffusivity table; synchronises once.
int geometry_dt(const fdirw_domain *d, hipStream_t st, unsigned *flags, Geometry *g, CoefTable *tab);
int prepare_geometry(const fdirw_domain *d, hipStream_t st, DevCache &dc, double *lam64, float *lam32, Geometry *g);
int coef_buffers(const fdirw_domain *d, int prec, hipStream_t st, DevCache &dc, Geometry *g, const void **lam);
int field_sum_dev(const double *c, int64_t n, hipStream_t st, DevCache &dc, double *out_host);
void line_shape(const fdirw_domain *d, int tune, int *seg_len, int *n_seg);
// True when the fused step of this precision and radius runs the flat-layout kernel.
bool use_flat_layout(int prec, int r);
// Source planes per launch of the deterministic step (a function of the
// domain's shape and radius only, or tune > 0 planes).
int det_slab_planes(const fdirw_domain *d, int tune);
// Bytes of partials kept by the deterministic step (caps det_slab_planes).
constexpr size_t DET_PART_CAP = (size_t)4 << 30;
int step_one(const fdirw_domain *d, const fdirw_opts *o, const double *c_in, double *c_out,
             fdirw_stats *st, DevCache &dc, hipStream_t stream, bool prepared, const void *lam, Geometry *geo);
int run_one(const fdirw_domain *d, const fdirw_opts *o, int n_steps, double *c, double *scratch,
            fdirw_stats *st, DevCache &dc, hipStream_t stream);
int step_batched(const fdirw_domain *d, int n_dom, const fdirw_opts *o, const double *const *c_in,
                 double *const *c_out, fdirw_stats *st, DevCache &dc, hipStream_t stream);
int batch_config_count();
int flow_stable(const fdirw_domain *d, int fp64, const void *lam, const double *u, double dt, hipStream_t st,
                DevCache &dc);
int step_nn(const fdirw_domain *d, const fdirw_opts *o, const double *c_in, double *c_out, fdirw_stats *st,
            DevCache &dc, hipStream_t stream);

// Coarse handle internals used by the integrated solver (fdirw_coarse_api.cpp).
int coarse_map_apply(void *handle, const double *c_in, const double *cff_dev, hipStream_t st, const double **cnew);
const int *coarse_node(const void *handle);

// Bytes per stored kernel value of a precision mode in the bank.
inline size_t bank_elem_bytes(int prec)
{
    if (prec == FDIRW_FP64) return 8;
    if (prec == FDIRW_FP16_BANK || prec == FDIRW_BF16_BANK) return 2;
    return 4;
}

}  // namespace fdirw
