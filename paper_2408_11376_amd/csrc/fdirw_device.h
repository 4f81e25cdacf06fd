// fdirw_device.h -- device-side building blocks of the FDiRW window stencil
// for gfx950 (CDNA4, wave64).  Included by the kernel translation units only.
//
// Execution model of one window kernel (Sec. 3.1 of arXiv 2408.11376: a
// column of P is the explicit-FD response to a unit point source):
//   * the W x W columns of the (2r+1)^3 window are owned by W^2 threads, one
//     z-column of W cells each, kept in registers (state and coefficients);
//   * every sub-step each thread publishes its column to LDS (double-buffered,
//     one barrier per sub-step) and reads its four in-plane neighbours back;
//     the z neighbours come from its own registers;
//   * G' = diag*G + sum_f lam_f * G_nbr, with diag = 1 - sum_f lam_f (the
//     conservative 7-point update written with one product per term).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fdirw {

enum Mode : int {
    M_FP64 = 0,
    M_FP32 = 1,
    M_F16X32 = 2,
    M_BF16X32 = 3,
    M_F16ST = 4,
    M_BF16ST = 5,
    M_F16BANK = 6,
    M_BF16BANK = 7,
    M_COUNT = 8
};

template <int M> struct Traits;
template <> struct Traits<M_FP64> {
    using S = double; using E = double;
    static constexpr bool x32 = false, state = false, bank = false, renorm = false;
};
template <> struct Traits<M_FP32> {
    using S = float; using E = float;
    static constexpr bool x32 = false, state = false, bank = false, renorm = true;
};
template <> struct Traits<M_F16X32> {
    using S = float; using E = _Float16;
    static constexpr bool x32 = true, state = false, bank = false, renorm = true;
};
template <> struct Traits<M_BF16X32> {
    using S = float; using E = __bf16;
    static constexpr bool x32 = true, state = false, bank = false, renorm = true;
};
template <> struct Traits<M_F16ST> {
    using S = float; using E = _Float16;
    static constexpr bool x32 = false, state = true, bank = false, renorm = true;
};
template <> struct Traits<M_BF16ST> {
    using S = float; using E = __bf16;
    static constexpr bool x32 = false, state = true, bank = false, renorm = true;
};
template <> struct Traits<M_F16BANK> {
    using S = float; using E = float;
    using B = _Float16;
    static constexpr bool x32 = false, state = false, bank = true, renorm = true;
};
template <> struct Traits<M_BF16BANK> {
    using S = float; using E = float;
    using B = __bf16;
    static constexpr bool x32 = false, state = false, bank = true, renorm = true;
};

// Round-to-nearest-even into the storage type and back (exact widening).
template <typename E> __device__ __forceinline__ float round_to(float x) { return (float)(E)x; }
template <> __device__ __forceinline__ float round_to<float>(float x) { return x; }

template <int R> struct Win {
    static constexpr int W = 2 * R + 1;
    static constexpr int W2 = W * W;
    static constexpr int W3 = W2 * W;
    static constexpr int NT = ((W2 + 63) / 64) * 64;       // threads per window
    static constexpr int NWAVE = NT / 64;
    static constexpr int PAD = W + 1;                       // LDS halo for t-1, t-W, t+1, t+W
    static constexpr int XLEN = W3 + 2 * PAD;              // one exchange buffer
};

// Per-thread column coefficients: in-plane faces of each cell and the z faces
// between consecutive cells (zf[j] = face between cells j-1 and j; zf[0] and
// zf[W] are the window walls and stay 0).
template <typename S, int W> struct Column {
    S xm[W], xp[W], ym[W], yp[W];
    S zf[W + 1];
    S diag[W];
};

// Coefficients of window cell (X, Y, Z) owned by a thread at window column
// (cx, cy).  Faces leaving the window or the domain are 0.
template <typename S, int W>
__device__ __forceinline__ void load_cell(const S *__restrict__ lx, const S *__restrict__ ly,
                                          int nx, int ny, int nz, int X, int Y, int Z,
                                          int cx, int cy, bool inxy,
                                          S &xm, S &xp, S &ym, S &yp)
{
    const bool in = inxy && Z >= 0 && Z < nz;
    xm = xp = ym = yp = S(0);
    if (in) {
        const int64_t i = ((int64_t)Z * ny + Y) * nx + X;
        if (cx < W - 1) xp = lx[i];
        if (cx > 0 && X > 0) xm = lx[i - 1];
        if (cy < W - 1) yp = ly[i];
        if (cy > 0 && Y > 0) ym = ly[i - nx];
    }
}

// z face between global planes Z-1 and Z of column (X, Y).
template <typename S>
__device__ __forceinline__ S load_zface(const S *__restrict__ lz, int nx, int ny, int nz,
                                        int X, int Y, int Z, bool inxy)
{
    if (inxy && Z >= 1 && Z < nz) return lz[((int64_t)(Z - 1) * ny + Y) * nx + X];
    return S(0);
}

// diag = 1 - sum of the six faces (plain modes), or the sum itself (X32
// modes, where the own-cell term uses the reduced copy).  Fixed order:
// -x, +x, -y, +y, -z, +z.
template <bool X32, typename S, int W>
__device__ __forceinline__ void compute_diag(Column<S, W> &c)
{
#pragma unroll
    for (int j = 0; j < W; ++j) {
        S s = c.xm[j] + c.xp[j];
        s = s + c.ym[j];
        s = s + c.yp[j];
        s = s + c.zf[j];
        s = s + c.zf[j + 1];
        c.diag[j] = X32 ? s : S(1) - s;
    }
}

template <typename S> __device__ __forceinline__ S fmaT(S a, S b, S c);
template <> __device__ __forceinline__ float fmaT<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <> __device__ __forceinline__ double fmaT<double>(double a, double b, double c) { return __builtin_fma(a, b, c); }

// n_sub explicit sub-steps of one window.  All threads of the block call this
// (barriers); threads with act == false only take part in the barriers.
template <int M, int R>
__device__ __forceinline__ void run_substeps(typename Traits<M>::S (&G)[Win<R>::W],
                                             const Column<typename Traits<M>::S, Win<R>::W> &c,
                                             typename Traits<M>::E *xb0,
                                             typename Traits<M>::E *xb1,
                                             int t, bool act, int n_sub)
{
    using T = Traits<M>;
    using S = typename T::S;
    using E = typename T::E;
    constexpr int W = Win<R>::W, W2 = Win<R>::W2, PAD = Win<R>::PAD;
    for (int step = 0; step < n_sub; ++step) {
        E *xb = (step & 1) ? xb1 : xb0;
        S gh[W];                                   // values the neighbours see
#pragma unroll
        for (int j = 0; j < W; ++j) {
            if constexpr (T::x32) gh[j] = round_to<E>(G[j]);
            else gh[j] = G[j];
        }
        if (act) {
#pragma unroll
            for (int j = 0; j < W; ++j) xb[PAD + j * W2 + t] = (E)gh[j];
        }
        __syncthreads();
        if (act) {
#pragma unroll
            for (int j = 0; j < W; ++j) {
                const E *p = xb + PAD + j * W2 + t;
                const S gxm = (S)p[-1], gxp = (S)p[1], gym = (S)p[-W], gyp = (S)p[W];
                S acc;
                if constexpr (T::x32) acc = fmaT<S>(-c.diag[j], gh[j], G[j]);
                else                  acc = c.diag[j] * G[j];
                acc = fmaT<S>(c.xm[j], gxm, acc);
                acc = fmaT<S>(c.xp[j], gxp, acc);
                acc = fmaT<S>(c.ym[j], gym, acc);
                acc = fmaT<S>(c.yp[j], gyp, acc);
                if (j > 0) acc = fmaT<S>(c.zf[j], gh[j - 1], acc);
                if (j < W - 1) acc = fmaT<S>(c.zf[j + 1], gh[j + 1], acc);
                if constexpr (T::state) acc = round_to<E>(acc);
                G[j] = acc;
            }
        }
    }
}

// Block-wide FP64 sum of one value per thread (fixed order: xor butterfly in
// each wave, then waves in index order).  red: NWAVE doubles of LDS.
template <int NWAVE>
__device__ __forceinline__ double block_sum(double v, double *red)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();                 // red may still be read from a previous call
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = red[0];
#pragma unroll
    for (int w = 1; w < NWAVE; ++w) s += red[w];
    return s;
}

}  // namespace fdirw
