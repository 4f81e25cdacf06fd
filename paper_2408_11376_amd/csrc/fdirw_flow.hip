// fdirw_flow.hip -- window kernels with a steady flow on gfx950: the explicit
// diffusion of Sec. 3.1 of arXiv 2408.11376 plus first-order upwind advection
// through every face (the paper's extension of P to diffusion with a steady
// flow, Sec. 5).  Used by fdirw_kernels_flow and by the coarse-mesh build.
//
// One workgroup per source.  The window (W^3 cells, z, y, x order) lives in
// two LDS buffers padded by W^2 cells on each side so that every neighbour
// index is in range; thread t owns the cells t, t + NT, ... and keeps their
// seven update coefficients in registers for the whole source:
//   G'(x) = c0 G(x) + sum over the six faces of c_f G(neighbour)
// c_f = lambda_f + the upwind inflow Courant number through f, c0 = 1 - sum
// of lambda_f - sum of the outflow Courant numbers.  Faces that leave the
// window or the domain carry nothing (no-flux walls).  Far-field cells (the
// coarse build's reservoir) are held at 0 after every sub-step.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fdirw_host.h"
#include "fdirw_launch.h"

namespace fdirw {

constexpr int FLOW_NT = 512;

template <int R> struct FlowGeo {
    static constexpr int W = 2 * R + 1;
    static constexpr int W2 = W * W;
    static constexpr int W3 = W2 * W;
    static constexpr int CPT = (W3 + FLOW_NT - 1) / FLOW_NT;   // cells per thread
    static constexpr int PAD = W2;
    static constexpr int BUF = W3 + 2 * PAD;
};

__device__ __forceinline__ double fma_s(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_s(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

template <int NW>
__device__ __forceinline__ double flow_block_sum(double v, double *red)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = red[0];
#pragma unroll
    for (int w = 1; w < NW; ++w) s += red[w];
    return s;
}

// S: state / coefficient type (double or float); L: face-coefficient type of
// the lambda arrays ([3][N], owned +x / +y / +z faces).
template <typename S, typename L, int R>
__global__ void __launch_bounds__(FLOW_NT) flow_window_kernel(FlowArgs a)
{
    using F = FlowGeo<R>;
    constexpr int W = F::W, W2 = F::W2, W3 = F::W3, CPT = F::CPT, PAD = F::PAD;
    __shared__ S buf[2][F::BUF];
    __shared__ double red[FLOW_NT / 64];
    const L *lx = (const L *)a.lam, *ly = lx + a.n, *lz = ly + a.n;
    const double *ux = a.u, *uy = ux + a.n, *uz = uy + a.n;
    const double cour = a.dt / a.h;
    for (int i = threadIdx.x; i < 2 * F::BUF; i += FLOW_NT) (&buf[0][0])[i] = S(0);
    __syncthreads();

    for (int64_t q = blockIdx.x; q < a.n_src; q += gridDim.x) {
        const int64_t s = a.src ? a.src[q] : a.src_base + q;
        if (a.node && a.node[s] < 0) continue;                 // not a grouped source: uniform per block
        const int sx = (int)(s % a.nx), sy = (int)((s / a.nx) % a.ny), sz = (int)(s / ((int64_t)a.nx * a.ny));
        S c0[CPT], cxm[CPT], cxp[CPT], cym[CPT], cyp[CPT], czm[CPT], czp[CPT], g[CPT];
        bool sink[CPT];
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            const int w = threadIdx.x + k * FLOW_NT;
            const int wx = w % W, wy = (w / W) % W, wz = w / W2;
            const int X = sx - R + wx, Y = sy - R + wy, Z = sz - R + wz;
            const bool in = w < W3 && X >= 0 && X < a.nx && Y >= 0 && Y < a.ny && Z >= 0 && Z < a.nz;
            double fm[3] = {0.0, 0.0, 0.0}, fp[3] = {0.0, 0.0, 0.0};     // lambda of the -/+ faces
            double vm[3] = {0.0, 0.0, 0.0}, vp[3] = {0.0, 0.0, 0.0};     // Courant numbers of the -/+ faces
            sink[k] = false;
            if (in) {
                const int64_t i = ((int64_t)Z * a.ny + Y) * a.nx + X;
                const int64_t sy_ = a.nx, sz_ = (int64_t)a.nx * a.ny;
                if (wx > 0 && X > 0) { fm[0] = (double)lx[i - 1]; vm[0] = ux[i - 1] * cour; }
                if (wx < W - 1 && X < a.nx - 1) { fp[0] = (double)lx[i]; vp[0] = ux[i] * cour; }
                if (wy > 0 && Y > 0) { fm[1] = (double)ly[i - sy_]; vm[1] = uy[i - sy_] * cour; }
                if (wy < W - 1 && Y < a.ny - 1) { fp[1] = (double)ly[i]; vp[1] = uy[i] * cour; }
                if (wz > 0 && Z > 0) { fm[2] = (double)lz[i - sz_]; vm[2] = uz[i - sz_] * cour; }
                if (wz < W - 1 && Z < a.nz - 1) { fp[2] = (double)lz[i]; vp[2] = uz[i] * cour; }
                sink[k] = a.node && a.node[i] == COARSE_RESERVOIR;
            }
            // inflow through the lower face when its flow is positive, through
            // the upper face when negative; outflow the other way round
            double out = 0.0, lam = 0.0;
            for (int ax = 0; ax < 3; ++ax) {
                lam += fm[ax] + fp[ax];
                out += (vm[ax] < 0.0 ? -vm[ax] : 0.0) + (vp[ax] > 0.0 ? vp[ax] : 0.0);
            }
            c0[k] = (S)(1.0 - lam - out);
            cxm[k] = (S)(fm[0] + (vm[0] > 0.0 ? vm[0] : 0.0));
            cxp[k] = (S)(fp[0] + (vp[0] < 0.0 ? -vp[0] : 0.0));
            cym[k] = (S)(fm[1] + (vm[1] > 0.0 ? vm[1] : 0.0));
            cyp[k] = (S)(fp[1] + (vp[1] < 0.0 ? -vp[1] : 0.0));
            czm[k] = (S)(fm[2] + (vm[2] > 0.0 ? vm[2] : 0.0));
            czp[k] = (S)(fp[2] + (vp[2] < 0.0 ? -vp[2] : 0.0));
            g[k] = (w == R * W2 + R * W + R) ? S(1) : S(0);
            if (w < W3) buf[0][PAD + w] = g[k];
        }
        __syncthreads();
        int cur = 0;
        for (int step = 0; step < a.n_sub; ++step) {
            const S *b = buf[cur] + PAD;
            S *o = buf[cur ^ 1] + PAD;
#pragma unroll
            for (int k = 0; k < CPT; ++k) {
                const int w = threadIdx.x + k * FLOW_NT;
                if (w < W3) {
                    S v = c0[k] * g[k];
                    v = fma_s(cxm[k], b[w - 1], v);
                    v = fma_s(cxp[k], b[w + 1], v);
                    v = fma_s(cym[k], b[w - W], v);
                    v = fma_s(cyp[k], b[w + W], v);
                    v = fma_s(czm[k], b[w - W2], v);
                    v = fma_s(czp[k], b[w + W2], v);
                    g[k] = sink[k] ? S(0) : v;
                    o[w] = g[k];
                }
            }
            __syncthreads();
            cur ^= 1;
        }
        double part = 0.0;
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            const int w = threadIdx.x + k * FLOW_NT;
            if (w < W3) {
                part += (double)g[k];
                if (a.G) ((S *)a.G)[q * (int64_t)W3 + w] = g[k];
            }
        }
        const double m = flow_block_sum<FLOW_NT / 64>(part, red);
        if (threadIdx.x == 0 && a.mass) a.mass[q] = m;
        __syncthreads();                                        // LDS buffers are reused
    }
}

// Largest 6 lambda + outflow Courant sum over the cells (stability of the
// explicit scheme with flow must keep it <= 1); positive doubles compare as
// their bit patterns.
template <typename L>
__global__ void flow_stability_kernel(const L *__restrict__ lam, const double *__restrict__ u, int nx, int ny,
                                      int nz, double cour, unsigned long long *__restrict__ out)
{
    const int64_t n = (int64_t)nx * ny * nz;
    const L *lx = lam, *ly = lx + n, *lz = ly + n;
    const double *ux = u, *uy = ux + n, *uz = uy + n;
    double mx = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(i % nx), y = (int)((i / nx) % ny), z = (int)(i / ((int64_t)nx * ny));
        double t = 0.0;
        if (x > 0) { t += (double)lx[i - 1]; t += ux[i - 1] < 0.0 ? -ux[i - 1] * cour : 0.0; }
        if (x < nx - 1) { t += (double)lx[i]; t += ux[i] > 0.0 ? ux[i] * cour : 0.0; }
        if (y > 0) { t += (double)ly[i - nx]; t += uy[i - nx] < 0.0 ? -uy[i - nx] * cour : 0.0; }
        if (y < ny - 1) { t += (double)ly[i]; t += uy[i] > 0.0 ? uy[i] * cour : 0.0; }
        const int64_t sz = (int64_t)nx * ny;
        if (z > 0) { t += (double)lz[i - sz]; t += uz[i - sz] < 0.0 ? -uz[i - sz] * cour : 0.0; }
        if (z < nz - 1) { t += (double)lz[i]; t += uz[i] > 0.0 ? uz[i] * cour : 0.0; }
        if (!(t <= mx)) mx = t;                                 // NaN propagates as "unstable"
    }
    if (!(mx >= 0.0) || mx != mx) mx = 1e300;
    // one atomic per workgroup (256 threads): waves first, then through LDS
    // (the values are >= 0, so their bit patterns order as the values do)
    __shared__ double wm[4];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
    if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0)
        atomicMax(out, (unsigned long long)__double_as_longlong(fmax(fmax(wm[0], wm[1]), fmax(wm[2], wm[3]))));
}

template <typename S, typename L>
static hipError_t launch_flow_sl(int r, const FlowArgs &a, hipStream_t st)
{
    const int64_t nblk = a.n_src < 65536 * 16 ? a.n_src : 65536 * 16;
    if (nblk <= 0) return hipSuccess;
    const dim3 g((unsigned)nblk), b(FLOW_NT);
    switch (r) {
    case 0: hipLaunchKernelGGL((flow_window_kernel<S, L, 0>), g, b, 0, st, a); break;
    case 1: hipLaunchKernelGGL((flow_window_kernel<S, L, 1>), g, b, 0, st, a); break;
    case 2: hipLaunchKernelGGL((flow_window_kernel<S, L, 2>), g, b, 0, st, a); break;
    case 3: hipLaunchKernelGGL((flow_window_kernel<S, L, 3>), g, b, 0, st, a); break;
    case 4: hipLaunchKernelGGL((flow_window_kernel<S, L, 4>), g, b, 0, st, a); break;
    case 5: hipLaunchKernelGGL((flow_window_kernel<S, L, 5>), g, b, 0, st, a); break;
    case 6: hipLaunchKernelGGL((flow_window_kernel<S, L, 6>), g, b, 0, st, a); break;
    case 7: hipLaunchKernelGGL((flow_window_kernel<S, L, 7>), g, b, 0, st, a); break;
    case 8: hipLaunchKernelGGL((flow_window_kernel<S, L, 8>), g, b, 0, st, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_flow_window(int fp64, int r, const FlowArgs &a, hipStream_t st)
{
    if (!fp64 && use_flat_layout(FDIRW_FP32, r)) return launch_flow_flat(r, a, st);
    return fp64 ? launch_flow_sl<double, double>(r, a, st) : launch_flow_sl<float, float>(r, a, st);
}

hipError_t launch_flow_stability(int fp64, const void *lam, const double *u, int nx, int ny, int nz, double cour,
                                 unsigned long long *out, hipStream_t st)
{
    const int64_t n = (int64_t)nx * ny * nz;
    const int64_t b = (n + 255) / 256;
    const unsigned g = (unsigned)(b < 4096 ? (b > 0 ? b : 1) : 4096);
    if (fp64)
        hipLaunchKernelGGL(flow_stability_kernel<double>, dim3(g), dim3(256), 0, st, (const double *)lam, u, nx, ny,
                           nz, cour, out);
    else
        hipLaunchKernelGGL(flow_stability_kernel<float>, dim3(g), dim3(256), 0, st, (const float *)lam, u, nx, ny,
                           nz, cour, out);
    return hipGetLastError();
}

}  // namespace fdirw
