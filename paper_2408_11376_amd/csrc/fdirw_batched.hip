// fdirw_batched.hip -- one persistent launch for many domains of uneven size,
// window radius and sub-step count (fdirw_step with n_dom > 1).
//
// Work items are (domain, group of source lines, z range); the host builds
// them, orders them by cost (longest first) and the resident workgroups pull
// them from an atomic counter until the list is exhausted.  Each item runs the
// same window stencil as the single-domain path (fdirw_device.h) with the
// radius taken from its domain: the workgroup has BATCH_NT threads and, for
// small windows, processes several source lines at once (one window per
// wave-aligned thread group), so threads are not left idle by small r.
#include "fdirw_device.h"
#include "fdirw_launch.h"

namespace fdirw {

constexpr int BATCH_NT = 640;

// Cells per thread segment chosen per radius for the 640-thread workgroup.
constexpr int batch_sc(int r)
{
    return r == 8 ? 9 : r == 7 ? 8 : r == 6 ? 5 : r == 5 ? 6 : r == 4 ? 5 : 2 * r + 1;
}

template <int M, int R> struct BGeo {
    static constexpr int SC = batch_sc(R);
    using G_ = Geo<M, R, SC>;
    static constexpr int NTG = G_::NT;                       // threads per window (wave multiple)
    static constexpr int NG = BATCH_NT / NTG;                // windows per workgroup
    static constexpr size_t XB = ru(2 * G_::XLEN * (int)sizeof(typename G_::E), 16);
    static constexpr size_t RING = (size_t)G_::W * G_::W2 * sizeof(double);
    static constexpr size_t LDS = NG * (XB + RING);
    static_assert(NG >= 1, "window does not fit the batched workgroup");
};

template <int M> constexpr size_t batch_lds()
{
    size_t m = BGeo<M, 0>::LDS;
    m = m > BGeo<M, 1>::LDS ? m : BGeo<M, 1>::LDS;
    m = m > BGeo<M, 2>::LDS ? m : BGeo<M, 2>::LDS;
    m = m > BGeo<M, 3>::LDS ? m : BGeo<M, 3>::LDS;
    m = m > BGeo<M, 4>::LDS ? m : BGeo<M, 4>::LDS;
    m = m > BGeo<M, 5>::LDS ? m : BGeo<M, 5>::LDS;
    m = m > BGeo<M, 6>::LDS ? m : BGeo<M, 6>::LDS;
    m = m > BGeo<M, 7>::LDS ? m : BGeo<M, 7>::LDS;
    m = m > BGeo<M, 8>::LDS ? m : BGeo<M, 8>::LDS;
    return m;
}

int batch_windows_per_group(int r)
{
    switch (r) {
    case 0: return BGeo<M_FP32, 0>::NG;
    case 1: return BGeo<M_FP32, 1>::NG;
    case 2: return BGeo<M_FP32, 2>::NG;
    case 3: return BGeo<M_FP32, 3>::NG;
    case 4: return BGeo<M_FP32, 4>::NG;
    case 5: return BGeo<M_FP32, 5>::NG;
    case 6: return BGeo<M_FP32, 6>::NG;
    case 7: return BGeo<M_FP32, 7>::NG;
    case 8: return BGeo<M_FP32, 8>::NG;
    default: return 1;
    }
}

// Sum of one value per thread over each wave-aligned group of NTG threads
// (fixed order).  red: BATCH_NT / 64 doubles.
template <int NTG, int NG>
__device__ __forceinline__ double group_sum(double v, double *red)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    constexpr int WPG = NTG / 64;
    if (wave / WPG >= NG) return 0.0;                        // threads outside every group
    const int w0 = (wave / WPG) * WPG;
    double s = red[w0];
#pragma unroll
    for (int w = 1; w < WPG; ++w) s += red[w0 + w];
    return s;
}

template <int M, int R>
__device__ __forceinline__ void batch_item(const BatchItem &item, const BatchDom &d, char *smem, double *red,
                                           double *kmm, double *item_kmass, int it)
{
    using B = BGeo<M, R>;
    constexpr int SC = B::SC;
    using G_ = typename B::G_;
    using T = typename G_::T;
    using S = typename G_::S;
    using E = typename G_::E;
    constexpr int L = G_::L0, W = G_::W, W2 = G_::W2;
    const int g = threadIdx.x / B::NTG;
    const int tl = threadIdx.x - g * B::NTG;
    const bool gin = g < B::NG && g < item.nlines;
    const Place p = make_place<M, R, SC>(gin ? tl : B::NTG);
    E *xb = (E *)(smem + (size_t)(g < B::NG ? g : 0) * B::XB);
    double *ring = (double *)(smem + B::NG * B::XB) + (size_t)(g < B::NG ? g : 0) * (W * W2);

    // clear this item's LDS (exchange buffers with their padding, rings)
    {
        unsigned *w32 = (unsigned *)smem;
        const int nw = (int)(B::LDS / 4);
        for (int i = threadIdx.x; i < nw; i += blockDim.x) w32[i] = 0u;
    }
    __syncthreads();

    const int line = item.line0 + g;
    const int sy = gin ? line / d.nx : 0, sx = gin ? line - sy * d.nx : 0;
    const int X = sx - R + p.cx, Y = sy - R + p.cy;
    const bool inxy = p.act && X >= 0 && X < d.nx && Y >= 0 && Y < d.ny;
    const S *lx = (const S *)d.lam, *ly = lx + d.n, *lz = ly + d.n;
    double kmin = INFINITY, kmax = -INFINITY;
    int used = 0;
    for (int sz = item.z0; sz < item.z1; ++sz) {
        // every group runs the sub-steps (barriers); a group with c = 0 or no
        // line adds nothing
        const double cs = gin ? d.c_in[((int64_t)sz * d.ny + sy) * d.nx + sx] : 0.0;
        Seg<M, R, SC> c;
        load_segment<M, R, SC>(c, lx, ly, lz, d.nx, d.ny, d.nz, sx, sy, sz, p);
        compute_diag<T::x32, M, R, SC>(c);
        S G[L];
        init_delta<M, R, SC>(G, p);
        run_substeps<M, R, SC>(G, c, xb, p, d.n_sub);
        const double m = group_sum<B::NTG, B::NG>(kernel_partial_mass<M, R, SC>(G, p), red);
        if (gin && cs != 0.0) {
            ++used;
            kmin = fmin(kmin, m);
            kmax = fmax(kmax, m);
        }
        const double scale = (cs == 0.0) ? 0.0 : (T::renorm ? cs / m : cs);
        if (p.act && scale != 0.0) {
#pragma unroll
            for (int k = 0; k < L; ++k) {
                if (k < p.len) {
                    double &rr = ring[((sz - R + p.j0 + k + W) % W) * W2 + p.col];
                    rr = __builtin_fma(scale, (double)G[k], rr);
                }
            }
        }
        __syncthreads();
        if (p.act && p.seg == 0) {
            const int Z = sz - R;
            double &rr = ring[((Z + W) % W) * W2 + p.col];
            const double v = rr;
            if (v != 0.0 && inxy && Z >= 0) unsafeAtomicAdd(&d.c_out[((int64_t)Z * d.ny + Y) * d.nx + X], v);
            rr = 0.0;
        }
    }
    __syncthreads();
    if (p.act && p.seg == 0) {
        for (int Z = item.z1 - R; Z < item.z1 + R; ++Z) {
            if (Z < 0 || Z >= d.nz) continue;
            double &rr = ring[((Z + W) % W) * W2 + p.col];
            const double v = rr;
            if (v != 0.0 && inxy) unsafeAtomicAdd(&d.c_out[((int64_t)Z * d.ny + Y) * d.nx + X], v);
            rr = 0.0;
        }
    }
    // per-item kernel-mass range and per-domain source count
    if (tl == 0 && g < B::NG) {
        kmm[2 * g] = kmin;
        kmm[2 * g + 1] = kmax;
        if (used && d.n_used) atomicAdd(d.n_used, (unsigned long long)used);
    }
    __syncthreads();
    if (threadIdx.x == 0 && item_kmass) {
        double a = INFINITY, b = -INFINITY;
        for (int q = 0; q < B::NG; ++q) { a = fmin(a, kmm[2 * q]); b = fmax(b, kmm[2 * q + 1]); }
        item_kmass[2 * it] = a;
        item_kmass[2 * it + 1] = b;
    }
}

template <int M>
__global__ void __launch_bounds__(BATCH_NT) __attribute__((amdgpu_waves_per_eu(3)))
batched_kernel(BatchArgs a)
{
    __shared__ __align__(16) char smem[batch_lds<M>()];
    __shared__ double red[BATCH_NT / 64];
    __shared__ double kmm[2 * 16];
    __shared__ int s_item;
    for (;;) {
        if (threadIdx.x == 0) s_item = (int)atomicAdd(a.head, 1u);
        __syncthreads();
        const int it = s_item;
        __syncthreads();
        if (it >= a.n_items) break;                         // uniform: every wave leaves
        const BatchItem item = a.items[it];
        const BatchDom d = a.doms[item.dom];
        switch (d.r) {
        case 0: batch_item<M, 0>(item, d, smem, red, kmm, a.item_kmass, it); break;
        case 1: batch_item<M, 1>(item, d, smem, red, kmm, a.item_kmass, it); break;
        case 2: batch_item<M, 2>(item, d, smem, red, kmm, a.item_kmass, it); break;
        case 3: batch_item<M, 3>(item, d, smem, red, kmm, a.item_kmass, it); break;
        case 4: batch_item<M, 4>(item, d, smem, red, kmm, a.item_kmass, it); break;
        case 5: batch_item<M, 5>(item, d, smem, red, kmm, a.item_kmass, it); break;
        case 6: batch_item<M, 6>(item, d, smem, red, kmm, a.item_kmass, it); break;
        case 7: batch_item<M, 7>(item, d, smem, red, kmm, a.item_kmass, it); break;
        default: batch_item<M, 8>(item, d, smem, red, kmm, a.item_kmass, it); break;
        }
        __syncthreads();                                    // LDS reuse by the next item
    }
}

template <int M>
static hipError_t launch_batched_m(const BatchArgs &a, int grid, hipStream_t st)
{
    hipLaunchKernelGGL(batched_kernel<M>, dim3(grid), dim3(BATCH_NT), 0, st, a);
    return hipGetLastError();
}

template <int M>
static hipError_t occupancy_m(int *blocks)
{
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, batched_kernel<M>, BATCH_NT, 0);
}

hipError_t launch_batched(int mode, const BatchArgs &a, int grid, hipStream_t st)
{
    switch (mode) {
    case M_FP64: return launch_batched_m<M_FP64>(a, grid, st);
    case M_FP32: return launch_batched_m<M_FP32>(a, grid, st);
    case M_F16X32: return launch_batched_m<M_F16X32>(a, grid, st);
    case M_BF16X32: return launch_batched_m<M_BF16X32>(a, grid, st);
    case M_F16ST: return launch_batched_m<M_F16ST>(a, grid, st);
    case M_BF16ST: return launch_batched_m<M_BF16ST>(a, grid, st);
    case M_F16BANK: return launch_batched_m<M_F16BANK>(a, grid, st);
    case M_BF16BANK: return launch_batched_m<M_BF16BANK>(a, grid, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t batched_occupancy(int mode, int *blocks)
{
    switch (mode) {
    case M_FP64: return occupancy_m<M_FP64>(blocks);
    case M_FP32: return occupancy_m<M_FP32>(blocks);
    case M_F16X32: return occupancy_m<M_F16X32>(blocks);
    case M_BF16X32: return occupancy_m<M_BF16X32>(blocks);
    case M_F16ST: return occupancy_m<M_F16ST>(blocks);
    case M_BF16ST: return occupancy_m<M_BF16ST>(blocks);
    case M_F16BANK: return occupancy_m<M_F16BANK>(blocks);
    case M_BF16BANK: return occupancy_m<M_BF16BANK>(blocks);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace fdirw
