// fdirw_device.h -- device-side building blocks of the FDiRW window stencil
// for gfx950 (CDNA4, wave64).  Included by the kernel translation units only.
//
// One window kernel (Sec. 3.1 of arXiv 2408.11376: a column of P is the
// explicit-FD response to a unit point source) is computed by one workgroup:
//   * the W x W z-columns of the (2r+1)^3 window are split into NSEG segments
//     of at most L0 cells; one thread owns one segment in registers (state,
//     face coefficients, and an FP64 accumulator per cell);
//   * every sub-step each thread publishes its segment to LDS and reads the
//     four in-plane neighbour segments back.  The LDS exchange buffer is laid
//     out z-fastest ([column][z]) so that a neighbour segment is a contiguous,
//     16-byte aligned run read with 128-bit LDS loads (on gfx950 these move
//     about twice the bytes per clock of 32/64-bit LDS loads); the column
//     stride is an odd number of 16-byte chunks so the 16 lanes served per
//     clock hit distinct banks;
//   * the two z neighbours come from the thread's own registers, except across
//     a segment boundary where they come from the exchange buffer;
//   * double-buffered exchange: one barrier per sub-step;
//   * update G' = diag*G + sum_f lam_f * G_nbr with diag = 1 - sum_f lam_f
//     (the conservative 7-point update, one product per term; terms added in
//     the order own, -z, +z, -x, +x, -y, +y).
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

// S: state / coefficient type; E: exchange (LDS copy) type; B: bank storage.
template <int M> struct Traits;
template <> struct Traits<M_FP64> {
    using S = double; using E = double; using B = double;
    static constexpr bool x32 = false, state = false, bank = false, renorm = false;
};
template <> struct Traits<M_FP32> {
    using S = float; using E = float; using B = float;
    static constexpr bool x32 = false, state = false, bank = false, renorm = true;
};
template <> struct Traits<M_F16X32> {
    using S = float; using E = _Float16; using B = float;
    static constexpr bool x32 = true, state = false, bank = false, renorm = true;
};
template <> struct Traits<M_BF16X32> {
    using S = float; using E = __bf16; using B = float;
    static constexpr bool x32 = true, state = false, bank = false, renorm = true;
};
template <> struct Traits<M_F16ST> {
    using S = float; using E = _Float16; using B = float;
    static constexpr bool x32 = false, state = true, bank = false, renorm = true;
};
template <> struct Traits<M_BF16ST> {
    using S = float; using E = __bf16; using B = float;
    static constexpr bool x32 = false, state = true, bank = false, renorm = true;
};
template <> struct Traits<M_F16BANK> {
    using S = float; using E = float; using B = _Float16;
    static constexpr bool x32 = false, state = false, bank = true, renorm = true;
};
template <> struct Traits<M_BF16BANK> {
    using S = float; using E = float; using B = __bf16;
    static constexpr bool x32 = false, state = false, bank = true, renorm = true;
};

// Round-to-nearest-even into a storage type and back (exact widening).
template <typename E> __device__ __forceinline__ float round_to(float x) { return (float)(E)x; }
template <> __device__ __forceinline__ float round_to<float>(float x) { return x; }

constexpr int ru(int a, int b) { return (a + b - 1) / b * b; }

// v rounded to FP32 and then to FP16 (two roundings, the route of the mixed
// FP32/FP16 scheme).  The empty asm keeps the compiler from folding the two
// conversions into one direct FP64 -> FP16 rounding, which differs where the
// FP32 value is an FP16 tie.
__device__ __forceinline__ _Float16 f64_to_f16_via_f32(double v)
{
    float f = (float)v;
    asm volatile("" : "+v"(f));
    return (_Float16)f;
}

// Spreads consecutive logical workgroups over one XCD: the hardware hands
// workgroup b to XCD b % 8, so logical index (b % 8) * (g / 8) + b / 8 keeps
// neighbouring source lines (which share coefficients and output planes) in
// the same L2.
__device__ __forceinline__ int xcd_remap(int b, int g)
{
    if (g % 8 != 0) return b;
    return (b % 8) * (g / 8) + b / 8;
}

#ifndef FDIRW_SEG_CELLS
#define FDIRW_SEG_CELLS 9          // most cells of a z-column one thread owns
#endif

// Geometry of the window / thread / LDS layout for mode M and radius R.
//
// A z-column of W cells is cut into NSEG segments of L0 cells (the last one
// has LAST <= L0 real cells; the rest of it is padding that stays 0).  Of each
// segment, the first MAIN = L0 - 1 cells go to the strided array
// main[col][z] (16-byte aligned runs, read with 128-bit loads), the top cell
// to the dense array tail[seg][col], and the first cell is also copied to the
// dense array head[seg][col]; the single-cell accesses of a wave are then
// lane-contiguous and free of bank conflicts.  With one segment the whole
// column is in main[].
template <int M, int R, int SC = FDIRW_SEG_CELLS> struct Geo {
    using T = Traits<M>;
    using S = typename T::S;
    using E = typename T::E;
    static constexpr int W = 2 * R + 1;
    static constexpr int W2 = W * W;
    static constexpr int W3 = W2 * W;
    static constexpr int NSEG = (W + SC - 1) / SC;          // segments per column
    static constexpr int L0 = (W + NSEG - 1) / NSEG;        // cells per thread
    static constexpr int LAST = W - (NSEG - 1) * L0;        // real cells of the last segment
    static constexpr int MAIN = NSEG > 1 ? L0 - 1 : W;      // cells per segment in main[]
    static constexpr int CH = 16 / (int)sizeof(E);          // elements per 16-byte chunk
    static constexpr int SOFF = ru(MAIN, CH);               // offset between segments in a column
    static constexpr int ZS0 = ru((NSEG - 1) * SOFF + MAIN, CH);
    static constexpr int ZS = ((ZS0 / CH) % 2 == 0) ? ZS0 + CH : ZS0;   // column stride
    static constexpr int PADC = W + 1;                      // padding columns on each side
    static constexpr int NCOL = W2 + 2 * PADC;
    static constexpr int TAIL = NCOL * ZS;                  // tail[seg][col]
    static constexpr int HEAD = TAIL + NSEG * NCOL;         // head[seg][col]
    static constexpr int XLEN = ru(HEAD + NSEG * NCOL, CH); // elements of one exchange buffer
    static constexpr int NT = ru(NSEG * W2, 64);            // threads per workgroup
    static constexpr int NWAVE = NT / 64;
    // register budget hint (minimum waves per SIMD): one workgroup per CU
    // (the exchange buffers and the FP64 ring of an r = 8 window take ~100 KB
    // of LDS) needs ceil(NWAVE / 4) waves per SIMD; more registers per thread
    // keep more LDS loads in flight (measured: 128 VGPRs beat 96 VGPRs with
    // two workgroups per CU)
#ifdef FDIRW_MINW
    static constexpr int MINW = FDIRW_MINW;
#else
    static constexpr int MINW = (NWAVE + 3) / 4 < 1 ? 1 : ((NWAVE + 3) / 4 > 8 ? 8 : (NWAVE + 3) / 4);
#endif
    static_assert(LAST >= 1 && LAST <= L0, "segment split");
};

// Per-thread kernel values of one segment.
template <int M, int R, int SC = FDIRW_SEG_CELLS> using SegVals = typename Geo<M, R, SC>::S[Geo<M, R, SC>::L0];

// Per-thread state of one segment.
template <int M, int R, int SC = FDIRW_SEG_CELLS> struct Seg {
    using G_ = Geo<M, R, SC>;
    using S = typename G_::S;
    static constexpr int L = G_::L0;
    S xm[L], xp[L], ym[L], yp[L];
    S zf[L + 1];          // zf[k]: face between segment cells k-1 and k (k = 0..L)
    S diag[L];
};

// Thread placement inside the workgroup.
struct Place {
    int t;        // thread index
    bool act;     // owns a segment
    int seg;      // segment index
    int col;      // window column (cy * W + cx)
    int cx, cy;
    int j0;       // window-relative z of the segment's first cell
    int len;      // real cells in the segment
};

template <int M, int R, int SC = FDIRW_SEG_CELLS>
__device__ __forceinline__ Place make_place(int t)
{
    using G_ = Geo<M, R, SC>;
    Place p;
    p.t = t;
    p.act = t < G_::NSEG * G_::W2;
    p.seg = p.act ? t / G_::W2 : 0;
    p.col = p.act ? t - p.seg * G_::W2 : 0;
    p.cx = p.col % G_::W;
    p.cy = p.col / G_::W;
    p.j0 = p.seg * G_::L0;
    p.len = p.seg == G_::NSEG - 1 ? G_::LAST : G_::L0;
    return p;
}

// Owned-face coefficients from the arrays lx / ly / lz ([nz][ny][nx] each):
// x(i, X) is the face from cell i to its +x neighbour (0 on the last plane of
// the axis, stored as such), likewise y and z.
template <typename S> struct FaceArrays {
    const S *__restrict__ lx;
    const S *__restrict__ ly;
    const S *__restrict__ lz;
    __device__ __forceinline__ S x(int64_t i, int) const { return lx[i]; }
    __device__ __forceinline__ S y(int64_t i, int) const { return ly[i]; }
    __device__ __forceinline__ S z(int64_t i, int) const { return lz[i]; }
};

// Owned-face coefficients from the phase labels and a table of the face
// coefficient of every ordered phase pair, tab[a * n_phase + b] (the face
// value depends on the two phases only); faces leaving the domain are 0.
template <typename S> struct FaceLabels {
    const uint8_t *__restrict__ label;
    const S *__restrict__ tab;
    int n_phase, nx, ny, nz;
    __device__ __forceinline__ S pair(int64_t i, int64_t j) const { return tab[label[i] * n_phase + label[j]]; }
    __device__ __forceinline__ S x(int64_t i, int X) const { return X + 1 < nx ? pair(i, i + 1) : S(0); }
    __device__ __forceinline__ S y(int64_t i, int Y) const { return Y + 1 < ny ? pair(i, i + nx) : S(0); }
    __device__ __forceinline__ S z(int64_t i, int Z) const
    {
        return Z + 1 < nz ? pair(i, i + (int64_t)nx * ny) : S(0);
    }
};

// Loads the coefficients of a thread's segment for the window of source
// (sx, sy, sz) through the owned-face accessor f.  Faces leaving the window
// or the domain, and every face of a cell outside the domain or past the
// segment's real cells, are 0.
template <int M, int R, int SC = FDIRW_SEG_CELLS, typename F>
__device__ __forceinline__ void load_segment_faces(Seg<M, R, SC> &c, const F &f,
                                                   int nx, int ny, int nz, int sx, int sy, int sz, const Place &p)
{
    using G_ = Geo<M, R, SC>;
    using S = typename G_::S;
    constexpr int L = G_::L0, W = G_::W;
    const int X = sx - R + p.cx, Y = sy - R + p.cy;
    const bool inxy = p.act && X >= 0 && X < nx && Y >= 0 && Y < ny;
#pragma unroll
    for (int k = 0; k < L; ++k) {
        const int j = p.j0 + k;                     // window-relative z
        const int Z = sz - R + j;
        const bool in = inxy && k < p.len && Z >= 0 && Z < nz;
        S xm = S(0), xp = S(0), ym = S(0), yp = S(0);
        if (in) {
            const int64_t i = ((int64_t)Z * ny + Y) * nx + X;
            if (p.cx < W - 1) xp = f.x(i, X);
            if (p.cx > 0 && X > 0) xm = f.x(i - 1, X - 1);
            if (p.cy < W - 1) yp = f.y(i, Y);
            if (p.cy > 0 && Y > 0) ym = f.y(i - nx, Y - 1);
        }
        c.xm[k] = xm; c.xp[k] = xp; c.ym[k] = ym; c.yp[k] = yp;
    }
#pragma unroll
    for (int k = 0; k <= L; ++k) {
        const int j = p.j0 + k;                     // face between relative j-1 and j
        const int Z = sz - R + j;
        S v = S(0);
        if (inxy && k <= p.len && j >= 1 && j <= W - 1 && Z >= 1 && Z < nz)
            v = f.z(((int64_t)(Z - 1) * ny + Y) * nx + X, Z - 1);
        c.zf[k] = v;
    }
}

// The same from the owned-face arrays lx / ly / lz.
template <int M, int R, int SC = FDIRW_SEG_CELLS>
__device__ __forceinline__ void load_segment(Seg<M, R, SC> &c, const typename Geo<M, R, SC>::S *__restrict__ lx,
                                             const typename Geo<M, R, SC>::S *__restrict__ ly,
                                             const typename Geo<M, R, SC>::S *__restrict__ lz,
                                             int nx, int ny, int nz, int sx, int sy, int sz, const Place &p)
{
    using S = typename Geo<M, R, SC>::S;
    const FaceArrays<S> f{lx, ly, lz};
    load_segment_faces<M, R, SC>(c, f, nx, ny, nz, sx, sy, sz, p);
}

template <bool X32, int M, int R, int SC = FDIRW_SEG_CELLS>
__device__ __forceinline__ void compute_diag(Seg<M, R, SC> &c)
{
    using S = typename Geo<M, R, SC>::S;
#pragma unroll
    for (int k = 0; k < Geo<M, R, SC>::L0; ++k) {
        S s = c.xm[k] + c.xp[k];
        s = s + c.ym[k];
        s = s + c.yp[k];
        s = s + c.zf[k];
        s = s + c.zf[k + 1];
        c.diag[k] = X32 ? s : S(1) - s;
    }
}

template <typename S> __device__ __forceinline__ S fmaT(S a, S b, S c);
template <> __device__ __forceinline__ float fmaT<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <> __device__ __forceinline__ double fmaT<double>(double a, double b, double c) { return __builtin_fma(a, b, c); }

// One explicit sub-step of one window, exchanging through buffer buf.
template <int M, int R, int SC = FDIRW_SEG_CELLS>
__device__ __forceinline__ void one_substep(SegVals<M, R, SC> &G, const Seg<M, R, SC> &c,
                                            typename Geo<M, R, SC>::E *__restrict__ buf, const Place &p,
                                            int own, int tail_at, int head_at, int zlo_at, int zhi_at)
{
    using G_ = Geo<M, R, SC>;
    using T = typename G_::T;
    using S = typename G_::S;
    using E = typename G_::E;
    constexpr int L = G_::L0, W = G_::W, ZS = G_::ZS, MAIN = G_::MAIN;
    constexpr bool MULTI = G_::NSEG > 1;
    S gh[L];                                        // the values the neighbours see
#pragma unroll
    for (int k = 0; k < L; ++k) {
        if constexpr (T::x32) gh[k] = round_to<E>(G[k]);
        else gh[k] = G[k];
    }
    if (p.act) {
#pragma unroll
        for (int k = 0; k < MAIN; ++k) buf[own + k] = (E)gh[k];
        if constexpr (MULTI) {
            buf[tail_at] = (E)gh[L - 1];
            buf[head_at] = (E)gh[0];
        }
    }
    __syncthreads();
    if (p.act) {
        // own and z terms first (the state is dead afterwards), then the four
        // in-plane directions one at a time so that only one neighbour
        // segment is live; per-cell term order: own, -z, +z, -x, +x, -y, +y
        const E *b = buf + own;
        S zlo = S(0), zhi = S(0);
        if constexpr (MULTI) {
            zlo = (S)buf[zlo_at];
            zhi = (S)buf[zhi_at];
        }
        S acc[L];
#pragma unroll
        for (int k = 0; k < L; ++k) {
            S a2;
            if constexpr (T::x32) a2 = fmaT<S>(-c.diag[k], gh[k], G[k]);
            else                  a2 = c.diag[k] * G[k];
            a2 = fmaT<S>(c.zf[k], k > 0 ? gh[k - 1] : zlo, a2);
            acc[k] = fmaT<S>(c.zf[k + 1], k < L - 1 ? gh[k + 1] : zhi, a2);
        }
        // neighbour cell k of column col + d: main[] for k < MAIN, else the
        // neighbour segment's top cell in tail[]
#define FDIRW_NB(d, k) ((k) < MAIN ? (S)b[(k) + (d) * ZS] : (S)buf[tail_at + (d)])
#pragma unroll
        for (int k = 0; k < L; ++k) acc[k] = fmaT<S>(c.xm[k], FDIRW_NB(-1, k), acc[k]);
#pragma unroll
        for (int k = 0; k < L; ++k) acc[k] = fmaT<S>(c.xp[k], FDIRW_NB(1, k), acc[k]);
#pragma unroll
        for (int k = 0; k < L; ++k) acc[k] = fmaT<S>(c.ym[k], FDIRW_NB(-W, k), acc[k]);
#pragma unroll
        for (int k = 0; k < L; ++k) {
            S a2 = fmaT<S>(c.yp[k], FDIRW_NB(W, k), acc[k]);
            if constexpr (T::state) a2 = round_to<E>(a2);
            G[k] = a2;
        }
#undef FDIRW_NB
    }
}

// n_sub explicit sub-steps of one window.  Every thread of the block calls
// this (barriers); threads with act == false only take part in the barriers.
// xb: two exchange buffers of XLEN elements, 16-byte aligned, padding zeroed;
// sub-steps alternate between them (one barrier per sub-step), unrolled by
// two so that buffer addresses are fixed offsets.
template <int M, int R, int SC = FDIRW_SEG_CELLS>
__device__ __forceinline__ void run_substeps(SegVals<M, R, SC> &G, const Seg<M, R, SC> &c,
                                             typename Geo<M, R, SC>::E *__restrict__ xb, const Place &p, int n_sub)
{
    using G_ = Geo<M, R, SC>;
    constexpr int NCOL = G_::NCOL;
    const int col = G_::PADC + p.col;
    const int own = col * G_::ZS + p.seg * G_::SOFF;
    const int tail_at = G_::TAIL + p.seg * NCOL + col;                 // own top cell
    const int head_at = G_::HEAD + p.seg * NCOL + col;                 // own first cell
    // z neighbours across segment boundaries: the top cell of the segment
    // below and the first cell of the segment above (first / last segments
    // read a finite dummy that their zero wall faces cancel)
    const int zlo_at = G_::TAIL + (p.seg > 0 ? p.seg - 1 : 0) * NCOL + col;
    const int zhi_at = G_::HEAD + (p.seg < G_::NSEG - 1 ? p.seg + 1 : 0) * NCOL + col;
    typename G_::E *xb1 = xb + G_::XLEN;
    int step = 0;
    for (; step + 1 < n_sub; step += 2) {
        one_substep<M, R, SC>(G, c, xb, p, own, tail_at, head_at, zlo_at, zhi_at);
        one_substep<M, R, SC>(G, c, xb1, p, own, tail_at, head_at, zlo_at, zhi_at);
    }
    if (step < n_sub) one_substep<M, R, SC>(G, c, xb, p, own, tail_at, head_at, zlo_at, zhi_at);
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

// After the sub-steps: in BANK modes round the kernel to its storage type;
// return this thread's FP64 share of the kernel mass.
template <int M, int R, int SC = FDIRW_SEG_CELLS>
__device__ __forceinline__ double kernel_partial_mass(SegVals<M, R, SC> &G, const Place &p)
{
    using T = typename Geo<M, R, SC>::T;
    constexpr int L = Geo<M, R, SC>::L0;
    if constexpr (T::bank) {
#pragma unroll
        for (int k = 0; k < L; ++k) G[k] = round_to<typename T::B>(G[k]);
    }
    double s = 0.0;
    if (p.act) {
#pragma unroll
        for (int k = 0; k < L; ++k) s += (double)G[k];
    }
    return s;
}

// Kernel mass over a workgroup that holds one window.
template <int M, int R, int SC = FDIRW_SEG_CELLS>
__device__ __forceinline__ double finish_kernel(SegVals<M, R, SC> &G, double *red, const Place &p)
{
    return block_sum<Geo<M, R, SC>::NWAVE>(kernel_partial_mass<M, R, SC>(G, p), red);
}

// Unit source at the window centre.
template <int M, int R, int SC = FDIRW_SEG_CELLS>
__device__ __forceinline__ void init_delta(SegVals<M, R, SC> &G, const Place &p)
{
    using S = typename Geo<M, R, SC>::S;
#pragma unroll
    for (int k = 0; k < Geo<M, R, SC>::L0; ++k)
        G[k] = (p.act && p.cx == R && p.cy == R && p.j0 + k == R) ? S(1) : S(0);
}

}  // namespace fdirw
