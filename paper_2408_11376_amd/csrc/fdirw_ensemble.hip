// fdirw_ensemble.hip -- the coarse product of Eq. 14 (arXiv 2408.11376) for
// an ensemble of E coarse fields at once, on the matrix cores of gfx950.
//
// With several right-hand sides the E products P C_e are one matrix product
// P [C_1 .. C_E]: P is read once for all members instead of once per member,
// and the work is a dense contraction for v_mfma_f32_16x16x32_f16 in the
// paper's mixed FP32/FP16 precision (Sec. 3.3): P in FP16, C in FP32 rounded
// to FP16, exact FP16 x FP16 products, FP32 accumulation.
//
// P is banded (|I - J| <= K per axis).  A tile is 16 nodes: a 4 x 4 patch of
// (x, y) at one z.  For one z offset oz the sources J of the tile's rows are
// the (4 + 2K) x (4 + 2K) patch around it at z - oz + K, so the tile's part of
// P for that oz is a dense 16 x (4 + 2K)^2 matrix (each row holds the (2K+1)^2
// entries of its (oy, ox) offsets; 39 % nonzero at K = 2), taken in steps of
// 32 columns.  The columns are ordered (jy, jx) with the jx rows padded to a
// multiple of 8, so the 8 columns a lane feeds are 8 consecutive x of the
// padded C grid (two 8-byte loads).  The matrix operand of every tile, z
// offset and step is stored once per handle in the lanes' order (16 bytes per
// lane: one 128-bit load), zeros included.
//
// A wave takes one tile and up to 8 column tiles of 16 members, loads each
// matrix fragment once and feeds it to one MFMA per column tile.
//
// Operands are kept in FP16's normal range: P and every member are scaled by
// powers of two that bring their largest magnitude into [2^14, 2^15) (the
// largest |P| once per handle, the largest |C_e| per call), operands still
// below 2^-14 are taken as 0, and the FP32 sums are scaled back exactly.  The
// scaling changes no normal FP16 value's rounding; it keeps subnormal
// operands, whose products the matrix unit adds less accurately than FP32
// (measured: a 2^-24 x 1 product added to 1e-6 lost 29 ulps), out of it.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "fdirw_device.h"
#include "fdirw_launch.h"

namespace fdirw {

namespace {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int ENS_NT = 256;           // 4 waves, one tile each
constexpr int ENS_MT = 8;             // column tiles of 16 members per wave
constexpr int ENS_SLIDE_MG = 4;       // ... in the plane-walking form

// 2^t that brings m into [2^14, 2^15) (1 for m = 0 or not finite).
__device__ __forceinline__ int pow2_scale(float m)
{
    if (!(m > 0.0f) || !(m <= 3.4e38f)) return 0;
    int e;
    (void)frexpf(m, &e);
    return 15 - e;
}

// v (FP32) as a normal FP16 number, or 0 below 2^-14.
__device__ __forceinline__ _Float16 f16_normal(float v)
{
    const _Float16 h = (_Float16)v;
    return fabsf((float)h) < 0x1p-14f ? (_Float16)0.0f : h;
}

// bits of the largest |value| (non-negative FP32 compare as unsigned) of n
// FP16 numbers, into *out (zeroed by the caller): one atomic per workgroup.
__global__ void __launch_bounds__(256) ensemble_pmax_kernel(const _Float16 *__restrict__ P, int64_t n,
                                                            unsigned *__restrict__ out)
{
    __shared__ float wm[4];
    float m = 0.0f;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        m = fmaxf(m, fabsf((float)P[i]));
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) atomicMax(out, __float_as_uint(fmaxf(fmaxf(wm[0], wm[1]), fmaxf(wm[2], wm[3]))));
}

// Per member m (blockIdx.y) the bits of the largest |FP32(C)| of its nodes,
// into cmax[m] (zeroed by the caller).  The member's row is read as 16-byte
// pairs from its first 16-byte boundary, eight independent loads per thread
// and trip; the one value before that boundary and the one after the last
// pair (rows of odd length or odd start) are taken by the first thread.
// Workgroups of 256 threads (the reduction below assumes four waves).
__device__ __forceinline__ float nan_max(float a, float b) { return b > a || b != b ? b : a; }

constexpr int CMAX_UNR = 8;

__global__ void __launch_bounds__(256) ensemble_cmax_kernel(const double *__restrict__ C, int64_t n_nodes,
                                                            unsigned *__restrict__ cmax)
{
    const int64_t a0 = (int64_t)blockIdx.y * n_nodes, a1 = a0 + n_nodes;
    const int64_t b0 = a0 + (((uintptr_t)(C + a0) & 15) ? 1 : 0);   // first 16-byte boundary of the row
    const int64_t np = (a1 - b0) / 2;                          // whole pairs from there
    const double2 *c2 = (const double2 *)(C + b0);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    float m = 0.0f;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < np; i += CMAX_UNR * stride) {
        double2 v[CMAX_UNR];
#pragma unroll
        for (int u = 0; u < CMAX_UNR; ++u) v[u] = i + u * stride < np ? c2[i + u * stride] : make_double2(0.0, 0.0);
#pragma unroll
        for (int u = 0; u < CMAX_UNR; ++u) {
            m = nan_max(m, fabsf((float)v[u].x));             // a NaN is kept
            m = nan_max(m, fabsf((float)v[u].y));
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (b0 > a0) m = nan_max(m, fabsf((float)C[a0]));
        if (b0 + 2 * np < a1) m = nan_max(m, fabsf((float)C[a1 - 1]));
    }
    // one atomic per workgroup: waves through LDS first
    __shared__ float wm[4];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) m = nan_max(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0)
        atomicMax(cmax + blockIdx.y, __float_as_uint(nan_max(nan_max(wm[0], wm[1]), nan_max(wm[2], wm[3]))));
}

// Matrix fragment of (tile, oz, step) for one lane: row i = lane % 16 (node
// (x0 + i % 4, y0 + i / 4, z)), columns 32 step + 8 (lane / 16) + h, h < 8;
// P scaled by 2^sp.
__global__ void ensemble_frag_kernel(const _Float16 *__restrict__ P, int64_t plane, EnsembleShape s, int sp,
                                     half8 *__restrict__ frag)
{
    const float scale = ldexpf(1.0f, sp);
    const int64_t total = s.n_tiles * s.kw * s.kst * 64;
    const int e = s.row, span = 4 + 2 * s.K;
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total;
         g += (int64_t)gridDim.x * blockDim.x) {
        const int lane = (int)(g & 63);
        const int64_t q = g >> 6;                              // (tile, oz, step)
        const int step = (int)(q % s.kst);
        const int oz = (int)((q / s.kst) % s.kw);
        const int64_t tile = q / ((int64_t)s.kst * s.kw);
        const int txi = (int)(tile % s.tx), tyi = (int)((tile / s.tx) % s.ty);
        const int z = (int)(tile / ((int64_t)s.tx * s.ty));
        const int ix = (lane & 15) & 3, iy = (lane & 15) >> 2;
        const int x = 4 * txi + ix, y = 4 * tyi + iy;
        half8 v;
#pragma unroll
        for (int h = 0; h < 8; ++h) v[h] = (_Float16)0.0f;
        if (x < s.ncx && y < s.ncy) {
            // P's layout (K < 5): per offset, chunks of 8 nodes along z, x fastest
            const int64_t at = (((int64_t)(z / 8) * s.ncy + y) * s.ncx + x) * 8 + z % 8;
#pragma unroll
            for (int h = 0; h < 8; ++h) {
                const int k = 32 * step + 8 * (lane >> 4) + h;
                const int jy = k / e, jx = k - jy * e;
                const int ox = ix - jx + 2 * s.K, oy = iy - jy + 2 * s.K;
                if (jy < span && jx < span && ox >= 0 && ox < s.kw && oy >= 0 && oy < s.kw)
                    v[h] = f16_normal((float)P[(int64_t)((oz * s.kw + oy) * s.kw + ox) * plane + at] * scale);
            }
        }
        frag[g] = v;
    }
}

// Node fields (FP64, member-major, node order) -> the padded FP16 grid of
// the product.  Layout: for every padded (z, y) row, chunks of 4 padded x
// positions; a chunk holds the 4 values of each of the `cap` members
// consecutively (member m at 4 m), so the 16 members of a column tile fill one
// 128-byte run.  Block (row, column tile): thread (j, m) = (t / 16, t % 16)
// writes chunk c0 + j of member 16 mt + m (halo positions and members past
// n_ens as 0); the halo rows keep the zeros written when the grid was
// allocated.
__global__ void __launch_bounds__(256) ensemble_pack_kernel(const double *__restrict__ C, int n_ens, int64_t n_nodes,
                                                            EnsembleShape s, int cap,
                                                            const unsigned *__restrict__ cmax,
                                                            _Float16 *__restrict__ cpad)
{
    const int row = blockIdx.x;                                // z ncy + y
    const int y = row % s.ncy, z = row / s.ncy;
    const int m = 16 * blockIdx.y + (threadIdx.x & 15), j = threadIdx.x >> 4;
    const bool live = m < n_ens;
    const float scale = live ? ldexpf(1.0f, pow2_scale(__uint_as_float(cmax[m]))) : 0.0f;
    const double *src = C + (live ? (int64_t)m * n_nodes : 0) + (int64_t)row * s.ncx;
    const int nchunk = s.px / 4;
    _Float16 *dst = cpad + ((int64_t)(z + s.K) * s.py + (y + s.K)) * nchunk * cap * 4 + (int64_t)m * 4;
    for (int c = j; c < nchunk; c += 16) {
        _Float16 q[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int x = 4 * c + u - s.K;                     // padded x 4c + u
            float f = 0.0f;
            if (live && x >= 0 && x < s.ncx) f = (float)src[x];
            asm volatile("" : "+v"(f));                       // FP32 first, then the scaled FP16
            q[u] = f16_normal(f * scale);
        }
        uint2 w;
        __builtin_memcpy(&w, q, 8);
        *(uint2 *)(dst + (int64_t)c * cap * 4) = w;
    }
}

// C_out[e] = P C_in[e] for the members of column tiles [ENS_MT blockIdx.y,
// + ENS_MT) of one tile per wave (K fixed at compile time: two steps of a z
// offset unrolled, so their loads are issued ahead of the MFMAs).
template <int K>
__global__ void __launch_bounds__(ENS_NT) ensemble_apply_kernel(const half8 *__restrict__ frag,
                                                                const _Float16 *__restrict__ cpad, int n_ens,
                                                                int64_t n_nodes, EnsembleShape s, int cap, int sp,
                                                                const unsigned *__restrict__ cmax,
                                                                double *__restrict__ out)
{
    constexpr int KW = 2 * K + 1, SPAN = 4 + 2 * K, ROW = ru(SPAN, 8), KST = (ROW * SPAN + 31) / 32;
    constexpr int UNR = KST <= 2 ? KST : (KST % 2 ? 1 : 2);   // steps in flight (registers)
    const int lane = threadIdx.x & 63;
    // consecutive tiles (a z-slab) on one XCD: they share their sources' FP16
    // copies in that XCD's L2
    const int64_t tile = xcd_remap(blockIdx.x, gridDim.x) * (int64_t)(ENS_NT / 64) + (threadIdx.x >> 6);
    if (tile >= s.n_tiles) return;                             // uniform per wave (no barrier below)
    const int mt0 = blockIdx.y * ENS_MT;
    const int n_mt = min(ENS_MT, (n_ens + 15) / 16 - mt0);
    const int t32 = (int)tile;                                 // n_tiles < 2^31 (checked by the host)
    const int txi = t32 % s.tx, tyi = (t32 / s.tx) % s.ty, z = t32 / (s.tx * s.ty);
    const int x0 = 4 * txi, y0 = 4 * tyi, kb = lane >> 4, col = lane & 15;
    floatx4 acc[ENS_MT];
#pragma unroll
    for (int t = 0; t < ENS_MT; ++t) acc[t] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    const half8 *fp = frag + tile * (KW * KST * 64) + lane;
    const int nchunk = s.px / 4;
    const _Float16 *cbase = cpad + (int64_t)(16 * mt0 + col) * 4;
#pragma unroll 1
    for (int oz = 0; oz < KW; ++oz) {
        const int zp = z - oz + 2 * K;                        // padded z of the sources
#pragma unroll UNR
        for (int step = 0; step < KST; ++step) {
            const half8 a = fp[(oz * KST + step) * 64];
            const int k = 32 * step + 8 * kb;
            int jy = k / ROW;
            const int jx = k - jy * ROW;
            if (jy >= SPAN) jy = SPAN - 1;                    // padding columns: zero in the fragment
            // padded x of source x0 - K + jx is x0 + jx (pad K): chunks (x0 + jx) / 4
            // and the next one
            const _Float16 *cp = cbase + (((int64_t)zp * s.py + (y0 + jy)) * nchunk + (x0 + jx) / 4) * cap * 4;
            // every column tile's operand is loaded before the first MFMA (tiles
            // past n_mt reload tile 0: in bounds, results dropped), so the loads
            // of a step are in flight together
            half8 b[ENS_MT];
#pragma unroll
            for (int t = 0; t < ENS_MT; ++t) {
                const _Float16 *c = cp + 64 * (t < n_mt ? t : 0);
                const uint2 lo = *(const uint2 *)c, hi = *(const uint2 *)(c + (int64_t)cap * 4);
                __builtin_memcpy(&b[t], &lo, 8);
                __builtin_memcpy((char *)&b[t] + 8, &hi, 8);
            }
#pragma unroll
            for (int t = 0; t < ENS_MT; ++t) acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b[t], acc[t], 0, 0, 0);
        }
    }
    // acc[t][u]: row 4 kb + u of the tile (node (x0 + u, y0 + kb, z)), member
    // 16 (mt0 + t) + col
    const int y = y0 + kb;
    if (y >= s.ncy) return;
#pragma unroll
    for (int t = 0; t < ENS_MT; ++t) {
        const int m = 16 * (mt0 + t) + col;
        if (t < n_mt && m < n_ens) {
            const int back = -(sp + pow2_scale(__uint_as_float(cmax[m])));
            double *o = out + (int64_t)m * n_nodes + ((int64_t)z * s.ncy + y) * s.ncx + x0;
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (x0 + u < s.ncx) o[u] = ldexp((double)acc[t][u], back);
        }
    }
}

// The same product with the source planes walked once (K <= 2, many members):
// a wave takes one tile column (txi, tyi), ZC consecutive output planes and
// MG column tiles of 16 members.  Each source plane's operands (every step,
// every column tile) are loaded once and feed the 2K + 1 output planes whose
// band covers it (accumulators of all ZC planes live in registers), instead
// of being reloaded for every output plane: (ZC + 2K) instead of ZC (2K + 1)
// operand loads.  Same fragments, same sums in the same order per output as
// ensemble_apply_kernel (z offsets in increasing order, then steps).
template <int K, int ZC, int MG>
__global__ void __launch_bounds__(ENS_NT) ensemble_slide_kernel(const half8 *__restrict__ frag,
                                                                const _Float16 *__restrict__ cpad, int n_ens,
                                                                int64_t n_nodes, EnsembleShape s, int cap, int sp,
                                                                const unsigned *__restrict__ cmax,
                                                                double *__restrict__ out)
{
    constexpr int KW = 2 * K + 1, SPAN = 4 + 2 * K, ROW = ru(SPAN, 8), KST = (ROW * SPAN + 31) / 32;
    const int lane = threadIdx.x & 63;
    const int ncol = s.tx * s.ty, nzc = (s.ncz + ZC - 1) / ZC;
    // consecutive waves: consecutive tile columns of one z-chunk (on one XCD)
    const int w = xcd_remap(blockIdx.x, gridDim.x) * (ENS_NT / 64) + (threadIdx.x >> 6);
    if (w >= ncol * nzc) return;                               // uniform per wave (no barrier below)
    const int colt = w % ncol, z0 = (w / ncol) * ZC;
    const int txi = colt % s.tx, tyi = colt / s.tx;
    const int x0 = 4 * txi, y0 = 4 * tyi, kb = lane >> 4, col = lane & 15;
    const int mt0 = blockIdx.y * MG;
    const int n_mt = min(MG, (n_ens + 15) / 16 - mt0);
    const int nchunk = s.px / 4;
    const _Float16 *cbase = cpad + (int64_t)(16 * mt0 + col) * 4;
    floatx4 acc[ZC][MG];
#pragma unroll
    for (int zi = 0; zi < ZC; ++zi)
#pragma unroll
        for (int t = 0; t < MG; ++t) acc[zi][t] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    // the sums of an output plane run over z offsets in increasing order: its
    // source planes in decreasing order, so walk them downwards
#pragma unroll
    for (int j = ZC + 2 * K - 1; j >= 0; --j) {
        const int zp = z0 + j;                                 // padded z of source plane j
        if (zp >= s.pz) continue;                              // uniform: feeds no output plane
        half8 b[KST][MG];
#pragma unroll
        for (int step = 0; step < KST; ++step) {
            const int k = 32 * step + 8 * kb;
            int jy = k / ROW;
            const int jx = k - jy * ROW;
            if (jy >= SPAN) jy = SPAN - 1;                    // padding columns: zero in the fragment
            const _Float16 *cp = cbase + (((int64_t)zp * s.py + (y0 + jy)) * nchunk + (x0 + jx) / 4) * cap * 4;
#pragma unroll
            for (int t = 0; t < MG; ++t) {
                const _Float16 *c = cp + 64 * (t < n_mt ? t : 0);
                const uint2 lo = *(const uint2 *)c, hi = *(const uint2 *)(c + (int64_t)cap * 4);
                __builtin_memcpy(&b[step][t], &lo, 8);
                __builtin_memcpy((char *)&b[step][t] + 8, &hi, 8);
            }
        }
#pragma unroll
        for (int oz = 0; oz < KW; ++oz) {
            const int zi = j + oz - 2 * K;                     // output plane z0 + zi (zp = z - oz + 2K)
            if (zi < 0 || zi >= ZC) continue;                  // compile time
            const int z = z0 + zi;
            if (z >= s.ncz) continue;                          // uniform
            const half8 *fp = frag + (((int64_t)z * s.ty + tyi) * s.tx + txi) * (KW * KST * 64) + lane;
#pragma unroll
            for (int step = 0; step < KST; ++step) {
                const half8 a = fp[(oz * KST + step) * 64];
#pragma unroll
                for (int t = 0; t < MG; ++t)
                    acc[zi][t] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b[step][t], acc[zi][t], 0, 0, 0);
            }
        }
    }
    const int y = y0 + kb;
    if (y >= s.ncy) return;
#pragma unroll
    for (int zi = 0; zi < ZC; ++zi) {
        const int z = z0 + zi;
        if (z >= s.ncz) break;
#pragma unroll
        for (int t = 0; t < MG; ++t) {
            const int m = 16 * (mt0 + t) + col;
            if (t < n_mt && m < n_ens) {
                const int back = -(sp + pow2_scale(__uint_as_float(cmax[m])));
                double *o = out + (int64_t)m * n_nodes + ((int64_t)z * s.ncy + y) * s.ncx + x0;
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (x0 + u < s.ncx) o[u] = ldexp((double)acc[zi][t][u], back);
            }
        }
    }
}

}  // namespace

EnsembleShape ensemble_shape(int ncx, int ncy, int ncz, int K)
{
    EnsembleShape s{};
    s.ncx = ncx; s.ncy = ncy; s.ncz = ncz; s.K = K;
    s.kw = 2 * K + 1;
    s.tx = (ncx + 3) / 4;
    s.ty = (ncy + 3) / 4;
    s.row = ru(4 + 2 * K, 8);
    s.kst = (s.row * (4 + 2 * K) + 31) / 32;
    s.n_tiles = (int64_t)s.tx * s.ty * ncz;
    s.px = 4 * s.tx - 4 + s.row;                              // a multiple of 4: 8-byte aligned loads
    s.py = 4 * s.ty + 2 * K;
    s.pz = ncz + 2 * K;
    s.msize = (int64_t)s.px * s.py * s.pz;
    return s;
}

int64_t ensemble_frag_bytes(const EnsembleShape &s) { return s.n_tiles * s.kw * s.kst * 64 * 16; }

hipError_t launch_ensemble_pmax(const void *P16, int64_t n, unsigned *out, hipStream_t st)
{
    hipError_t e = launch_fill_u32(out, 1, 0u, st);
    if (e != hipSuccess) return e;
    const int grid = (int)std::min<int64_t>((n + 255) / 256, 512);
    ensemble_pmax_kernel<<<grid, 256, 0, st>>>((const _Float16 *)P16, n, out);
    return hipGetLastError();
}

int ensemble_p_scale(unsigned pmax_bits)
{
    float m;
    std::memcpy(&m, &pmax_bits, 4);
    if (!(m > 0.0f) || !std::isfinite(m)) return 0;
    int e;
    (void)std::frexp(m, &e);
    return 15 - e;
}

hipError_t launch_ensemble_frags(const void *P16, int64_t plane, const EnsembleShape &s, int sp, void *frag,
                                 hipStream_t st)
{
    const int64_t total = s.n_tiles * s.kw * s.kst * 64;
    const int grid = (int)std::min<int64_t>((total + 255) / 256, 65536);
    ensemble_frag_kernel<<<grid, 256, 0, st>>>((const _Float16 *)P16, plane, s, sp, (half8 *)frag);
    return hipGetLastError();
}

hipError_t launch_ensemble_pack(const double *C, int n_ens, int64_t n_nodes, const EnsembleShape &s, int cap,
                                unsigned *cmax, void *cpad, hipStream_t st)
{
    hipError_t e = launch_fill_u32(cmax, n_ens, 0u, st);
    if (e != hipSuccess) return e;
    const int64_t per_block = 2 * 256 * CMAX_UNR;              // values per workgroup and trip
    const dim3 gm((unsigned)std::min<int64_t>((n_nodes + per_block - 1) / per_block, 16), (unsigned)n_ens);
    ensemble_cmax_kernel<<<gm, 256, 0, st>>>(C, n_nodes, cmax);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const dim3 grid((unsigned)(s.ncy * s.ncz), (unsigned)((n_ens + 15) / 16));
    ensemble_pack_kernel<<<grid, 256, 0, st>>>(C, n_ens, n_nodes, s, cap, cmax, (_Float16 *)cpad);
    return hipGetLastError();
}

hipError_t launch_ensemble_apply(const void *frag, const void *cpad, int n_ens, int64_t n_nodes,
                                 const EnsembleShape &s, int cap, int sp, const unsigned *cmax, double *out,
                                 hipStream_t st)
{
    const int n_mt = (n_ens + 15) / 16;
    const half8 *f = (const half8 *)frag;
    const _Float16 *c = (const _Float16 *)cpad;
    // the plane-walking form keeps ZC planes of accumulators (two waves per
    // SIMD) and has fewer waves: it pays from 8 column tiles (128 members) on
    if (s.K <= 2 && n_mt >= 2 * ENS_SLIDE_MG) {
        constexpr int ZC = 8, MG = ENS_SLIDE_MG;
        const int64_t waves = (int64_t)s.tx * s.ty * ((s.ncz + ZC - 1) / ZC);
        const int64_t blocks = (waves + ENS_NT / 64 - 1) / (ENS_NT / 64);
        const dim3 grid((unsigned)((blocks + 7) / 8 * 8), (unsigned)((n_mt + MG - 1) / MG));
        switch (s.K) {
        case 0: ensemble_slide_kernel<0, ZC, MG><<<grid, ENS_NT, 0, st>>>(f, c, n_ens, n_nodes, s, cap, sp, cmax, out); break;
        case 1: ensemble_slide_kernel<1, ZC, MG><<<grid, ENS_NT, 0, st>>>(f, c, n_ens, n_nodes, s, cap, sp, cmax, out); break;
        default: ensemble_slide_kernel<2, ZC, MG><<<grid, ENS_NT, 0, st>>>(f, c, n_ens, n_nodes, s, cap, sp, cmax, out); break;
        }
        return hipGetLastError();
    }
    const int64_t blocks = (s.n_tiles + ENS_NT / 64 - 1) / (ENS_NT / 64);
    const dim3 grid((unsigned)((blocks + 7) / 8 * 8), (unsigned)((n_mt + ENS_MT - 1) / ENS_MT));
    switch (s.K) {
    case 0: ensemble_apply_kernel<0><<<grid, ENS_NT, 0, st>>>(f, c, n_ens, n_nodes, s, cap, sp, cmax, out); break;
    case 1: ensemble_apply_kernel<1><<<grid, ENS_NT, 0, st>>>(f, c, n_ens, n_nodes, s, cap, sp, cmax, out); break;
    case 2: ensemble_apply_kernel<2><<<grid, ENS_NT, 0, st>>>(f, c, n_ens, n_nodes, s, cap, sp, cmax, out); break;
    case 3: ensemble_apply_kernel<3><<<grid, ENS_NT, 0, st>>>(f, c, n_ens, n_nodes, s, cap, sp, cmax, out); break;
    case 4: ensemble_apply_kernel<4><<<grid, ENS_NT, 0, st>>>(f, c, n_ens, n_nodes, s, cap, sp, cmax, out); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace fdirw
