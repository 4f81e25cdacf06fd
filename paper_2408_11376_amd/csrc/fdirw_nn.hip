// fdirw_nn.hip -- the learned kernel generator on gfx950: a small 3-D CNN
// that maps the features of a 17^3 window (r = 8) to the window kernel G_s.
// (An extension of the hot path: the paper obtains every column of P by
// explicit FD from a point source, Sec. 3.1.)
//
// Network: five 3x3x3 convolutions with zero "same" padding, channels
// 3 (stored as 8) -> 16 -> 16 -> 16 -> 16 -> 1, SiLU after the first four;
// logits = log U + conv5 output, U the uniform-D window kernel (the prior);
// G = softmax of the logits over the structural support of the window.
//
// Convolutions are implicit GEMMs on v_mfma_f32_16x16x32_bf16 (BF16 operands,
// FP32 accumulation): M = 16 output voxels, N = 16 output channels, K = 27
// taps x input channels in chunks of 32.  Activations are BF16 and
// channel-last ([window][voxel][channel]); a workgroup stages a z-slab of its
// window's input with the zero halo in LDS (channel-last, so the 8 channels a
// lane feeds for one tap are one 128-bit LDS load) and holds the packed
// weights of every K chunk in registers.  The input gradient is the same
// convolution with flipped, channel-transposed weights.  The weight gradient
// is an MFMA GEMM over slab positions (K = 32 positions per instruction) on a
// channel-first copy of the slab, accumulated per workgroup over many slabs
// and reduced in a fixed order by a second kernel.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fdirw_launch.h"

namespace fdirw {
namespace nn {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float floatx4;

constexpr int R = NN_R;
constexpr int W = NN_W;               // 17
constexpr int W2 = W * W;
constexpr int V = NN_V;               // 4913
constexpr int P = W + 2;              // padded edge 19
constexpr int P2 = P * P;             // 361
constexpr int TZ = 3;                 // output planes per slab
constexpr int NSLAB = (W + TZ - 1) / TZ;
constexpr int NTHR = 256;

// SiLU with the hardware exp and reciprocal (about 1 ulp each; the result is
// rounded to BF16, 2^-8 relative, right after)
__device__ __forceinline__ float silu_f(float x) { return x * __builtin_amdgcn_rcpf(1.0f + __expf(-x)); }
__device__ __forceinline__ float silu_grad_f(float x)
{
    const float s = __builtin_amdgcn_rcpf(1.0f + __expf(-x));
    return s * (1.0f + x * (1.0f - s));
}

__device__ __forceinline__ bf16x8 zero8()
{
    bf16x8 z;
#pragma unroll
    for (int i = 0; i < 8; ++i) z[i] = (__bf16)0.0f;
    return z;
}

// ----------------------------------------------------------------- features

// Breadth-first growth of the support from the window centre: sa holds the
// seed (the centre), one face crossing per sweep, at most n_sub sweeps,
// stopping early when a sweep adds nothing.  open[v]: cell v is in the domain
// and permeable.  Returns the array (sa or sb) holding the result.
__device__ const uint8_t *grow_support(const uint8_t *open, uint8_t *sa, uint8_t *sb, int n_sub, int *changed)
{
    uint8_t *cur = sa, *nxt = sb;
    for (int it = 0; it < n_sub; ++it) {
        if (threadIdx.x == 0) *changed = 0;
        __syncthreads();
        int any = 0;
        for (int v = threadIdx.x; v < V; v += blockDim.x) {
            uint8_t r = cur[v];
            if (!r && open[v]) {
                const int wx = v % W, wy = (v / W) % W, wz = v / W2;
                if ((wx > 0 && cur[v - 1] && open[v - 1]) || (wx < W - 1 && cur[v + 1] && open[v + 1]) ||
                    (wy > 0 && cur[v - W] && open[v - W]) || (wy < W - 1 && cur[v + W] && open[v + W]) ||
                    (wz > 0 && cur[v - W2] && open[v - W2]) || (wz < W - 1 && cur[v + W2] && open[v + W2])) {
                    r = 1;
                    any = 1;
                }
            }
            nxt[v] = r;
        }
        if (any) atomicOr(changed, 1);
        __syncthreads();
        const int ch = *changed;
        uint8_t *t = cur;
        cur = nxt;
        nxt = t;
        __syncthreads();                                     // every thread has read changed
        if (!ch) break;
    }
    return cur;
}

// Window q of source src[q]: features X[q][v][0..7] (BF16: channel 0 = the
// cell is in the domain and permeable, 1 = log-D feature or -1 outside the
// domain, 2 = prior / 20, 3..7 = 0) and the structural support S[q][v]:
// cells reached from s in at most n_sub face crossings, a face being passable
// when both of its cells are in the domain and permeable (lambda > 0).
__global__ void __launch_bounds__(NTHR)
features_kernel(NnFeatArgs a)
{
    __shared__ uint8_t open[V], sa[V], sb[V];
    __shared__ int changed, allopen;
    const int q = blockIdx.x;
    const int64_t s = a.src[q];
    const int64_t plane = (int64_t)a.nx * a.ny;
    const int sz = (int)(s / plane);
    const int64_t rem = s - (int64_t)sz * plane;
    const int sy = (int)(rem / a.nx), sx = (int)(rem - (int64_t)sy * a.nx);
    if (threadIdx.x == 0) allopen = 1;
    __syncthreads();
    __bf16 *X = reinterpret_cast<__bf16 *>(a.X) + (int64_t)q * V * 8;
    int notopen = 0;
    for (int v = threadIdx.x; v < V; v += NTHR) {
        const int wx = v % W, wy = (v / W) % W, wz = v / W2;
        const int gx = sx - R + wx, gy = sy - R + wy, gz = sz - R + wz;
        const bool in = gx >= 0 && gx < a.nx && gy >= 0 && gy < a.ny && gz >= 0 && gz < a.nz;
        float f0 = 0.0f, f1 = -1.0f;
        uint8_t op = 0;
        if (in) {
            const int lab = a.label[((int64_t)gz * a.ny + gy) * a.nx + gx];
            op = a.open[lab];
            f0 = op ? 1.0f : 0.0f;
            f1 = a.f1[lab];
            if (!op) notopen = 1;
        }
        bf16x8 f = zero8();
        f[0] = (__bf16)f0;
        f[1] = (__bf16)f1;
        f[2] = (__bf16)(a.prior[v] * (1.0f / 20.0f));
        *reinterpret_cast<bf16x8 *>(X + (int64_t)v * 8) = f;
        open[v] = op;
        sa[v] = (wx == R && wy == R && wz == R) ? 1 : 0;
    }
    if (notopen) atomicAnd(&allopen, 0);
    __syncthreads();
    uint8_t *S = a.support + (int64_t)q * V;
    if (allopen && a.n_sub >= 3 * R) {
        // every in-domain cell is permeable: the in-domain part of the window
        // is a box whose cells all lie within 3R face crossings of s
        for (int v = threadIdx.x; v < V; v += NTHR) {
            const int wx = v % W, wy = (v / W) % W, wz = v / W2;
            const int gx = sx - R + wx, gy = sy - R + wy, gz = sz - R + wz;
            S[v] = (gx >= 0 && gx < a.nx && gy >= 0 && gy < a.ny && gz >= 0 && gz < a.nz) ? 1 : 0;
        }
        return;
    }
    const uint8_t *cur = grow_support(open, sa, sb, a.n_sub, &changed);
    for (int v = threadIdx.x; v < V; v += NTHR) S[v] = cur[v];
}

// ----------------------------------------------------------------- weights

constexpr int nchunks(int CI) { return (27 * CI + 31) / 32; }

// Packs one layer's FP32 weights w[co][ci][27] (tap order z, y, x) into the
// per-lane MFMA B operands Wp[chunk][lane][8] (BF16).  Reduction index k =
// tap * CI + channel; lane l feeds output channel l % 16 and k = 32 chunk +
// 8 (l / 16) + i.  flip: the input-gradient weights w'[ci][co][26 - tap].
__global__ void pack_kernel(const float *__restrict__ w, int co_n, int ci_n, int CI, int flip,
                            uint16_t *__restrict__ out)
{
    const int total = nchunks(CI) * 64 * 8;
    __bf16 *o = reinterpret_cast<__bf16 *>(out);
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
        const int i = e % 8, l = (e / 8) % 64, c = e / 512;
        const int n = l % 16, b = l / 16;
        const int k = c * 32 + b * 8 + i;
        const int tap = k / CI, ch = k % CI;
        float v = 0.0f;
        if (tap < 27) {
            if (!flip) {
                if (n < co_n && ch < ci_n) v = w[((size_t)n * ci_n + ch) * 27 + tap];
            } else {
                // output channel n = the layer's input channel n; input channel
                // ch = the layer's output channel ch
                if (n < ci_n && ch < co_n) v = w[((size_t)ch * ci_n + n) * 27 + (26 - tap)];
            }
        }
        o[e] = (__bf16)v;
    }
}

// ----------------------------------------------------------------- conv

// One workgroup: window blockIdx.x / NSLAB, output planes z0 .. z0 + TZ - 1.
template <int CI>
__global__ void __launch_bounds__(NTHR)
conv_kernel(NnConvArgs a)
{
    constexpr int NCH = nchunks(CI);
    __shared__ __align__(16) __bf16 slab[(TZ + 2) * P2 * CI];
    const int b = blockIdx.x / NSLAB;
    const int z0 = (blockIdx.x % NSLAB) * TZ;
    const int tz = W - z0 < TZ ? W - z0 : TZ;
    const __bf16 *in = reinterpret_cast<const __bf16 *>(a.in) + (int64_t)b * V * CI;

    // planes z0 - 1 .. z0 + TZ with a zero halo, 8 channels per 16-byte vector
    constexpr int VPC = CI / 8;
    constexpr int NCELL = (TZ + 2) * P2;
    for (int e = threadIdx.x; e < NCELL * VPC; e += NTHR) {
        const int cell = e / VPC, vv = e - cell * VPC;
        const int px = cell % P, py = (cell / P) % P, pz = cell / P2;
        const int x = px - 1, y = py - 1, z = z0 + pz - 1;
        bf16x8 val = zero8();
        if (x >= 0 && x < W && y >= 0 && y < W && z >= 0 && z < W)
            val = *reinterpret_cast<const bf16x8 *>(in + (int64_t)((z * W + y) * W + x) * CI + vv * 8);
        *reinterpret_cast<bf16x8 *>(slab + (size_t)cell * CI + vv * 8) = val;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m = lane % 16, kb = lane / 16;
    const bf16x8 *wp = reinterpret_cast<const bf16x8 *>(a.wpack);
    bf16x8 wreg[NCH];
    int offs[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        wreg[c] = wp[c * 64 + lane];
        int tap, ch0;
        if (CI == 16) { tap = 2 * c + (kb >> 1); ch0 = 8 * (kb & 1); }
        else          { tap = 4 * c + kb;        ch0 = 0; }
        if (tap > 26) tap = 26;                              // padding taps carry zero weights
        const int dz = tap / 9, dy = (tap / 3) % 3, dx = tap % 3;
        offs[c] = ((dz * P + dy) * P + dx) * CI + ch0;
    }
    __syncthreads();

    const int nvox = tz * W2;
    const int ntile = (nvox + 15) / 16;
    for (int tile = wave; tile < ntile; tile += NTHR / 64) {
        int t = tile * 16 + m;
        if (t >= nvox) t = nvox - 1;                         // padding rows, results dropped
        const int ox = t % W, oy = (t / W) % W, oz = t / W2;
        const int base = ((oz * P + oy) * P + ox) * CI;
        floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const bf16x8 av = *reinterpret_cast<const bf16x8 *>(slab + base + offs[c]);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, wreg[c], acc, 0, 0, 0);
        }
        // acc[j]: voxel row 4 kb + j of the tile, output channel m
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int tt = tile * 16 + 4 * kb + j;
            if (tt >= nvox) continue;
            const int64_t v = (int64_t)b * V + z0 * W2 + tt;
            const float val = acc[j];
            if (a.mode == 0) {
                const float zz = val + a.bias[m];
                if (a.zpre) a.zpre[v * 16 + m] = zz;
                reinterpret_cast<__bf16 *>(a.hout)[v * 16 + m] = (__bf16)silu_f(zz);
            } else if (a.mode == 1) {
                if (m == 0) a.z5[v] = val + a.bias[0];
            } else {
                a.dh[v * 16 + m] = val;
            }
        }
    }
}

// ----------------------------------------------------------------- softmax / loss

template <typename T, int NW = NTHR / 64>
__device__ __forceinline__ T block_reduce_sum(T x, T *red)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
    __syncthreads();
    if (lane == 0) red[wave] = x;
    __syncthreads();
    T s = 0;
    for (int w = 0; w < NW; ++w) s += red[w];
    return s;
}

// One workgroup per window.  logits = prior + z5; G = softmax over the support
// (0 elsewhere).  With a target q (normalised here by its FP64 sum): loss terms
// KL(q || G) and sum |q - G|, and d loss / d logits = (G - q) + G (sbar -
// sign(q - G)), sbar = sum sign(q - G) G, times grad_scale, written as BF16
// channel 0 of an 8-channel field.  The loss path evaluates G in FP64.
__global__ void __launch_bounds__(NTHR)
softmax_loss_kernel(NnLossArgs a)
{
    __shared__ float redf[NTHR / 64];
    __shared__ double redd[NTHR / 64];
    const int b = blockIdx.x;
    const float *z5 = a.z5 + (int64_t)b * V;
    const uint8_t *S = a.support + (int64_t)b * V;
    float mx = -INFINITY;
    for (int v = threadIdx.x; v < V; v += NTHR)
        if (S[v]) mx = fmaxf(mx, a.prior[v] + z5[v]);
    {
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        for (int off = 32; off >= 1; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 64));
        if (lane == 0) redf[wave] = mx;
        __syncthreads();
        mx = redf[0];
        for (int w = 1; w < NTHR / 64; ++w) mx = fmaxf(mx, redf[w]);
    }
    float *G = a.G ? a.G + (int64_t)b * V : nullptr;
    if (a.logits)
        for (int v = threadIdx.x; v < V; v += NTHR) a.logits[(int64_t)b * V + v] = a.prior[v] + z5[v];
    if (!a.target) {
        double se = 0.0;
        for (int v = threadIdx.x; v < V; v += NTHR)
            if (S[v]) se += (double)expf(a.prior[v] + z5[v] - mx);
        se = block_reduce_sum(se, redd);
        const float inv = (float)(1.0 / se);
        double ms = 0.0;
        for (int v = threadIdx.x; v < V; v += NTHR) {
            const float g = S[v] ? expf(a.prior[v] + z5[v] - mx) * inv : 0.0f;
            if (G) G[v] = g;
            ms += (double)g;
        }
        ms = block_reduce_sum(ms, redd);
        if (threadIdx.x == 0 && a.mass) a.mass[b] = ms;
        return;
    }
    const float *tg = a.target + (int64_t)b * V;
    double se = 0.0, tm = 0.0;
    for (int v = threadIdx.x; v < V; v += NTHR) {
        if (S[v]) se += exp((double)(a.prior[v] + z5[v]) - (double)mx);
        tm += (double)tg[v];
    }
    se = block_reduce_sum(se, redd);
    tm = block_reduce_sum(tm, redd);
    const double lse = log(se), tinv = 1.0 / tm;
    double kl = 0.0, l1 = 0.0, sbar = 0.0;
    for (int v = threadIdx.x; v < V; v += NTHR) {
        if (!S[v]) continue;
        const double lg = (double)(a.prior[v] + z5[v]) - (double)mx - lse;
        const double g = exp(lg), qv = (double)tg[v] * tinv;
        if (qv > 0.0) kl += qv * (log(qv) - lg);
        l1 += fabs(qv - g);
        sbar += (qv > g ? 1.0 : (qv < g ? -1.0 : 0.0)) * g;
    }
    kl = block_reduce_sum(kl, redd);
    l1 = block_reduce_sum(l1, redd);
    sbar = block_reduce_sum(sbar, redd);
    if (threadIdx.x == 0) {
        a.loss[2 * b] = kl;
        a.loss[2 * b + 1] = l1;
    }
    double ms = 0.0;
    __bf16 *d8 = reinterpret_cast<__bf16 *>(a.dlog8) + (int64_t)b * V * 8;
    for (int v = threadIdx.x; v < V; v += NTHR) {
        float dz = 0.0f, gv = 0.0f;
        if (S[v]) {
            const double g = exp((double)(a.prior[v] + z5[v]) - (double)mx - lse);
            const double qv = (double)tg[v] * tinv;
            const double sg = qv > g ? 1.0 : (qv < g ? -1.0 : 0.0);
            dz = (float)(((g - qv) + g * (sbar - sg)) * (double)a.grad_scale);
            gv = (float)g;
        }
        if (G) G[v] = gv;
        ms += (double)gv;
        bf16x8 o = zero8();
        o[0] = (__bf16)dz;
        *reinterpret_cast<bf16x8 *>(d8 + (int64_t)v * 8) = o;
    }
    ms = block_reduce_sum(ms, redd);
    if (threadIdx.x == 0 && a.mass) a.mass[b] = ms;
}

// dz = dh * SiLU'(zpre), rounded to BF16
__global__ void silu_bwd_kernel(const float *__restrict__ dh, const float *__restrict__ zpre,
                                uint16_t *__restrict__ dz, int64_t n)
{
    __bf16 *o = reinterpret_cast<__bf16 *>(dz);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        o[i] = (__bf16)(dh[i] * silu_grad_f(zpre[i]));
}

// ----------------------------------------------------------------- weight gradient

// dW[tap][co][ci] = sum over output positions p of dZ[co][p] H[ci][p + off(tap)],
// as MFMA GEMMs with M = co, N = ci, K = 32 padded slab positions.  Both
// operands are staged channel-first in LDS; H is also stored shifted by one
// element so that every tap's operand starts at an even element and is read
// with 32-bit loads.  Each workgroup accumulates its slabs in registers and
// writes one partial; db[co] = sum of dZ is accumulated alongside.
template <int CI, int COP>
__global__ void __launch_bounds__(NTHR)
wgrad_kernel(NnWgradArgs a)
{
    constexpr int NPOS = TZ * P2;                            // 1083 output positions
    constexpr int KP = (NPOS + 31) / 32 * 32;               // 1088
    constexpr int NIN = (TZ + 2) * P2;                       // staged input planes z0 - 1 .. z0 + TZ
    // Output position p (padded plane coordinates) reads input element
    // p + P2 + (dz - 1) P2 + (dy - 1) P + (dx - 1); the staged copy starts FRONT
    // elements late so that this index is p + dz P2 + dy P + dx >= 0, and ends
    // past the highest element read, KP - 1 + 2 P2 + 2 P + 2.
    constexpr int FRONT = P + 1;
    constexpr int HLEN = (KP + 2 * P2 + 2 * P + 2 + 7) / 8 * 8;
    __shared__ __align__(16) __bf16 hs[2][CI][HLEN];
    __shared__ __align__(16) __bf16 ds[16][KP];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m = lane % 16, kb = lane / 16;
    constexpr int TPW = 7;                                   // taps per wave: wave + 4 i
    floatx4 acc[TPW];
#pragma unroll
    for (int i = 0; i < TPW; ++i) acc[i] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    float bsum = 0.0f;
    const __bf16 *hbase = reinterpret_cast<const __bf16 *>(a.h);
    const __bf16 *dbase = reinterpret_cast<const __bf16 *>(a.dz);

    for (int slab_id = blockIdx.x; slab_id < a.n_slab; slab_id += gridDim.x) {
        const int b = slab_id / NSLAB;
        const int z0 = (slab_id % NSLAB) * TZ;
        const int tz = W - z0 < TZ ? W - z0 : TZ;
        const __bf16 *hin = hbase + (int64_t)b * V * CI;
        const __bf16 *din = dbase + (int64_t)b * V * COP;
        __syncthreads();                                     // previous slab fully consumed
        for (int j = threadIdx.x; j < HLEN; j += NTHR) {
            const int e = j - FRONT;
            const int px = e % P, py = (e / P) % P, pz = e / P2;
            const int x = px - 1, y = py - 1, z = z0 + pz - 1;
            const bool in = e >= 0 && e < NIN && x >= 0 && x < W && y >= 0 && y < W && z >= 0 && z < W;
            __bf16 v[CI];
            if (in) {
                const bf16x8 *src = reinterpret_cast<const bf16x8 *>(hin + (int64_t)((z * W + y) * W + x) * CI);
#pragma unroll
                for (int j = 0; j < CI / 8; ++j) {
                    const bf16x8 t = src[j];
#pragma unroll
                    for (int i = 0; i < 8; ++i) v[8 * j + i] = t[i];
                }
            } else {
#pragma unroll
                for (int c = 0; c < CI; ++c) v[c] = (__bf16)0.0f;
            }
#pragma unroll
            for (int c = 0; c < CI; ++c) {
                hs[0][c][j] = v[c];
                if (j > 0) hs[1][c][j - 1] = v[c];
            }
        }
        if (threadIdx.x < CI) hs[1][threadIdx.x][HLEN - 1] = (__bf16)0.0f;
        for (int e = threadIdx.x; e < KP; e += NTHR) {
            const int px = e % P, py = (e / P) % P, pz = e / P2;
            const int x = px - 1, y = py - 1, z = z0 + pz;
            const bool in = e < NPOS && pz < tz && x >= 0 && x < W && y >= 0 && y < W;
            __bf16 v[16];
#pragma unroll
            for (int c = 0; c < 16; ++c) v[c] = (__bf16)0.0f;
            if (in) {
                const bf16x8 *src = reinterpret_cast<const bf16x8 *>(din + (int64_t)((z * W + y) * W + x) * COP);
#pragma unroll
                for (int j = 0; j < COP / 8; ++j) {
                    const bf16x8 t = src[j];
#pragma unroll
                    for (int i = 0; i < 8; ++i) v[8 * j + i] = t[i];
                }
            }
#pragma unroll
            for (int c = 0; c < 16; ++c) ds[c][e] = c < a.co_n ? v[c] : (__bf16)0.0f;
        }
        __syncthreads();

        for (int p0 = 0; p0 < KP; p0 += 32) {
            const bf16x8 av = *reinterpret_cast<const bf16x8 *>(&ds[m][p0 + 8 * kb]);
            if (wave == 0) {
#pragma unroll
                for (int i = 0; i < 8; ++i) bsum += (float)av[i];
            }
#pragma unroll
            for (int i = 0; i < TPW; ++i) {
                const int tap = wave + 4 * i;
                if (tap > 26) break;
                const int dz = tap / 9, dy = (tap / 3) % 3, dx = tap % 3;
                const int e = p0 + 8 * kb + dz * P2 + dy * P + dx;
                bf16x8 bv;
                if (m < CI) {
                    const int sh = e & 1;
                    const unsigned *src = reinterpret_cast<const unsigned *>(&hs[sh][m][e - sh]);
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const unsigned u = src[j];
                        bv[2 * j] = __builtin_bit_cast(__bf16, (unsigned short)(u & 0xffffu));
                        bv[2 * j + 1] = __builtin_bit_cast(__bf16, (unsigned short)(u >> 16));
                    }
                } else {
                    bv = zero8();
                }
                acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[i], 0, 0, 0);
            }
        }
    }
    // acc[i][j]: co = 4 kb + j, ci = m
    float *part = a.part + (size_t)blockIdx.x * 27 * 256;
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
        const int tap = wave + 4 * i;
        if (tap > 26) break;
#pragma unroll
        for (int j = 0; j < 4; ++j) part[tap * 256 + (4 * kb + j) * 16 + m] = acc[i][j];
    }
    if (wave == 0) {
        bsum += __shfl_xor(bsum, 16, 64);
        bsum += __shfl_xor(bsum, 32, 64);
        if (kb == 0) a.bpart[(size_t)blockIdx.x * 16 + m] = bsum;
    }
}

// gw[(co ci_n + ci) 27 + tap] += sum over g of part[g][tap][co][ci]; gb[co] likewise.
__global__ void wgrad_reduce_kernel(const float *__restrict__ part, const float *__restrict__ bpart, int grid,
                                    int co_n, int ci_n, float *__restrict__ gw, float *__restrict__ gb)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < 27 * 256) {
        const int tap = i / 256, co = (i / 16) % 16, ci = i % 16;
        if (co < co_n && ci < ci_n) {
            float s = 0.0f;
            for (int g = 0; g < grid; ++g) s += part[(size_t)g * 27 * 256 + i];
            gw[((size_t)co * ci_n + ci) * 27 + tap] += s;
        }
    } else if (i < 27 * 256 + 16) {
        const int co = i - 27 * 256;
        if (co < co_n) {
            float s = 0.0f;
            for (int g = 0; g < grid; ++g) s += bpart[(size_t)g * 16 + co];
            gb[co] += s;
        }
    }
}

// ----------------------------------------------------------------- Adam

__global__ void adam_kernel(float *__restrict__ w, float *__restrict__ mo, float *__restrict__ ve,
                            const float *__restrict__ g, int n, float lr, float b1, float b2, float eps,
                            float c1, float c2)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float m1 = b1 * mo[i] + (1.0f - b1) * gi;
        const float v1 = b2 * ve[i] + (1.0f - b2) * gi * gi;
        mo[i] = m1;
        ve[i] = v1;
        w[i] -= lr * (m1 / c1) / (sqrtf(v1 / c2) + eps);
    }
}

// ----------------------------------------------------------------- superposition

// Sources of lines line0 .. line0 + nlines - 1 (line = y nx + x), every plane:
// src[(line - line0) nz + z] = (z ny + y) nx + x.
__global__ void lines_src_kernel(int64_t line0, int nlines, int nx, int ny, int nz, int64_t *__restrict__ src)
{
    const int64_t total = (int64_t)nlines * nz;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < total; q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t line = line0 + q / nz;
        const int z = (int)(q % nz);
        const int64_t y = line / nx, x = line - y * nx;
        src[q] = ((int64_t)z * ny + y) * nx + x;
    }
}

// Scatter c(s) G_s / m_s for the sources of a block of lines: one workgroup
// per (line, z segment); thread (cx, cy) owns one window column and keeps the
// W pending z values of the column in registers, flushing one per source.
constexpr int APPLY_NT = 320;
__global__ void __launch_bounds__(APPLY_NT)
apply_kernel(int nx, int ny, int nz, int64_t line0, int seg_len, int n_seg, const float *__restrict__ G,
             const double *__restrict__ mass, const double *__restrict__ c_in, double *__restrict__ c_out,
             unsigned long long *__restrict__ n_used)
{
    const int t = threadIdx.x;
    const bool act = t < W2;
    const int cx = act ? t % W : 0, cy = act ? t / W : 0;
    const int lloc = blockIdx.x / n_seg, seg = blockIdx.x - lloc * n_seg;
    const int64_t line = line0 + lloc;
    const int sy = (int)(line / nx), sx = (int)(line - (int64_t)sy * nx);
    const int z0 = seg * seg_len;
    const int z1 = min(nz, z0 + seg_len);
    if (z0 >= z1) return;
    if (t == 0 && n_used) {
        unsigned long long cnt = 0;
        for (int sz = z0; sz < z1; ++sz) cnt += c_in[((int64_t)sz * ny + sy) * nx + sx] != 0.0;
        if (cnt) atomicAdd(n_used, cnt);
    }
    if (!act) return;
    const int X = sx - R + cx, Y = sy - R + cy;
    const bool inxy = X >= 0 && X < nx && Y >= 0 && Y < ny;
    double acc[W];
#pragma unroll
    for (int j = 0; j < W; ++j) acc[j] = 0.0;
    for (int sz = z0; sz < z1; ++sz) {
        const int64_t s = ((int64_t)sz * ny + sy) * nx + sx;
        const double cs = c_in[s];
        const int64_t q = (int64_t)lloc * nz + sz;
        if (cs != 0.0) {
            const double scale = cs / mass[q];
            const float *g = G + q * V + t;
#pragma unroll
            for (int j = 0; j < W; ++j) acc[j] = __builtin_fma(scale, (double)g[j * W2], acc[j]);
        }
        const int Z = sz - R;
        if (acc[0] != 0.0 && inxy && Z >= 0) unsafeAtomicAdd(&c_out[((int64_t)Z * ny + Y) * nx + X], acc[0]);
#pragma unroll
        for (int j = 0; j < W - 1; ++j) acc[j] = acc[j + 1];
        acc[W - 1] = 0.0;
    }
#pragma unroll
    for (int j = 0; j < W - 1; ++j) {
        const int Z = z1 - R + j;
        if (acc[j] != 0.0 && inxy && Z >= 0 && Z < nz) unsafeAtomicAdd(&c_out[((int64_t)Z * ny + Y) * nx + X], acc[j]);
    }
}

// out[b] = sum over the window of |x_b - y_b| (FP64)
__global__ void __launch_bounds__(NTHR)
l1_kernel(const float *__restrict__ x, const float *__restrict__ y, double *__restrict__ out)
{
    __shared__ double red[NTHR / 64];
    const int b = blockIdx.x;
    double s = 0.0;
    for (int v = threadIdx.x; v < V; v += NTHR)
        s += fabs((double)x[(int64_t)b * V + v] - (double)y[(int64_t)b * V + v]);
    s = block_reduce_sum(s, red);
    if (threadIdx.x == 0) out[b] = s;
}

__global__ void fill_f32_kernel(float *__restrict__ p, int64_t n, float v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// ----------------------------------------------------------------- fused inference

// One workgroup (8 waves, two per SIMD) per window.  The activations of the
// window live in LDS for all five layers: 17 planes x 289 voxels x 16
// channels of BF16 (157 KB), each plane stored as two halves of 8 channels so
// that the 16 voxels of an MFMA operand are 16 consecutive 16-byte vectors.
// Each layer walks the input planes p = 0 .. 16 once; the operand loaded for
// input plane p feeds the three output planes p + 1, p, p - 1 (taps dz = 0,
// 1, 2) from registers, so LDS is read once per input plane instead of once
// per tap.  A plane's input is dead after its step, so output plane p - 1
// overwrites input plane p - 1 during step p (one barrier per step).  MFMA
// roles: A = weights (rows = output channels), B = activations (columns = 16
// voxels of a plane), so each lane writes 4 consecutive channels of one
// voxel.  Layer 0 reads its 3 (stored as 8) feature channels from the second
// half of each plane's slot, filled from the labels before the first layer;
// the last layer (one output channel) puts the three dz taps in the A rows.
constexpr int FNT = 512;                                    // threads per workgroup
constexpr int FWAVES = FNT / 64;                            // 8
constexpr int FTILES = (W2 + 15) / 16;                      // 19 voxel tiles per plane
constexpr int FPAD = W2 * 8;                                // zero 16-byte vector after each half plane
constexpr int FHALF = W2 * 8 + 8;                           // BF16 elements of one 8-channel half plane + pad
constexpr int FSLOT = 2 * FHALF;                            // BF16 elements of one activation plane
constexpr int FTPW = (FTILES + FWAVES - 1) / FWAVES;        // tiles per wave (3)
constexpr int fchunks(int layer) { return layer == 0 ? 3 : 5; }
constexpr int fpack_count(int layer) { return (layer == 4 ? 1 : 3) * fchunks(layer); }

// Weights in the fused A layout: for each (dz, chunk) a bf16x8 per lane; lane
// l holds row l % 16 (output channel; dz for the last layer) and reduction
// indices 8 (l / 16) + i of the chunk.  Layer 0: chunk c covers plane
// positions 4c .. 4c + 3 (8 channels each); other layers: positions 2c, 2c + 1
// (16 channels each); position = dy * 3 + dx, 9 = padding.
__global__ void fpack_kernel(const float *__restrict__ w, int layer, int co_n, int ci_n, uint16_t *__restrict__ out)
{
    const int nc = fchunks(layer);
    const int total = fpack_count(layer) * 512;
    __bf16 *o = reinterpret_cast<__bf16 *>(out);
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
        const int i = e % 8, l = (e / 8) % 64, idx = e / 512;
        const int row = l % 16, kb = l / 16;
        int dz, c;
        if (layer == 4) { c = idx; dz = row; }
        else            { dz = idx / nc; c = idx % nc; }
        int pos, ch;
        if (layer == 0) { pos = 4 * c + kb;        ch = i; }
        else            { pos = 2 * c + (kb >> 1); ch = 8 * (kb & 1) + i; }
        const int co = layer == 4 ? 0 : row;
        float v = 0.0f;
        if (pos < 9 && dz < 3 && co < co_n && ch < ci_n) v = w[((size_t)co * ci_n + ch) * 27 + dz * 9 + pos];
        o[e] = (__bf16)v;
    }
}

struct FusedCtx {
    int lane, wave, n, kb;
    int sx, sy, sz;
    bool vok[FTPW];
    int vp[FTPW];
    int sto[FTPW];            // element offset of this lane's 4 output channels within a plane
    __bf16 *dummy;            // store target of the lanes past the last voxel
};

__device__ __forceinline__ bool fused_tile(const FusedCtx &f, int i) { return f.wave + FWAVES * i < FTILES; }

// SiLU(acc + bias) of output plane z of one tile into LDS (channels 4 kb .. 4 kb + 3)
__device__ __forceinline__ void fused_store(__bf16 *act, const FusedCtx &f, int i, int z, const floatx4 &acc,
                                            const float *bias4)
{
    typedef __attribute__((ext_vector_type(4))) __bf16 bf16x4;
    bf16x4 h;
#pragma unroll
    for (int j = 0; j < 4; ++j) h[j] = (__bf16)silu_f(acc[j] + bias4[j]);
    // no branch: lanes past the last voxel write a dummy vector
    __bf16 *dst = f.vok[i] ? act + z * FSLOT + f.sto[i] : f.dummy;
    *reinterpret_cast<bf16x4 *>(dst) = h;
}

// Operand of one lane: 8 channels at element offset off of the half plane
// that starts at element pb; off = FPAD reads the half plane's zero pad.
__device__ __forceinline__ bf16x8 fused_load(const __bf16 *act, int pb, int off)
{
    return *reinterpret_cast<const bf16x8 *>(act + pb + off);
}

// One step (input plane p) of a 16-channel layer with NC chunks per dz; xin
// points at the plane.  acc[i][0..2] = outputs p - 1, p, p + 1.
// Step kinds of a layer walk: the first plane (no output p - 1), the second
// (nothing held back yet), the middle planes, and the last (no output p + 1).
enum { FK_FIRST = 0, FK_SECOND = 1, FK_MID = 2, FK_LAST = 3 };
#ifndef FDIRW_NN_PREFETCH
#define FDIRW_NN_PREFETCH 1
#endif
constexpr bool FPREF = FDIRW_NN_PREFETCH != 0;              // carry chunk 0 of the next plane across the barrier
#ifndef FDIRW_NN_SCHED
#define FDIRW_NN_SCHED 1
#endif
constexpr bool FSCHED = FDIRW_NN_SCHED != 0;                // interleave MFMA and VALU in the middle steps

// One step (input plane p, P4 = p mod 4) of a 16-output-channel layer for a
// wave with NT tiles.  acc[i][z mod 4] accumulates output plane z: the
// operand of chunk c feeds output planes p + 1, p, p - 1 (taps dz = 0, 1, 2);
// plane p + 1 starts from a zero accumulator.  Output plane p - 2, complete
// since the previous step, is stored afterwards (its slot was last read in
// step p - 2) so that its SiLU overlaps this step's MFMAs.  b0 holds the
// chunk-0 operands of plane p (loaded before the step's barrier) and receives
// those of plane p + 1: input planes are final until the step that stores
// the same plane's output, two steps later.
template <int NT, int NC, int KIND, int P4>
__device__ __forceinline__ void fused_kstep(__bf16 *act, int pb, int p, const int (&off)[FTPW][5],
                                            const bf16x8 (&wr)[3][5], floatx4 (&acc)[FTPW][4], bf16x8 (&b0)[FTPW],
                                            const FusedCtx &f, const float *b4)
{
    constexpr int SN = (P4 + 1) & 3, SC = P4, SP = (P4 + 3) & 3, SD = (P4 + 2) & 3;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        bf16x8 b[NT];
#pragma unroll
        for (int i = 0; i < NT; ++i) b[i] = (c == 0 && FPREF) ? b0[i] : fused_load(act, pb, off[i][c]);
#pragma unroll
        for (int i = 0; i < NT; ++i) {
            acc[i][SC] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wr[1][c], b[i], acc[i][SC], 0, 0, 0);
            if (KIND != FK_FIRST) acc[i][SP] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wr[2][c], b[i], acc[i][SP], 0, 0, 0);
            if (KIND != FK_LAST) {
                if (c == 0) acc[i][SN] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wr[0][c], b[i], floatx4{0.0f, 0.0f, 0.0f, 0.0f}, 0, 0, 0);
                else        acc[i][SN] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wr[0][c], b[i], acc[i][SN], 0, 0, 0);
            }
        }
    }
    if (FPREF && KIND != FK_LAST) {
#pragma unroll
        for (int i = 0; i < NT; ++i) b0[i] = fused_load(act, pb + FSLOT, off[i][0]);
    }
    if (KIND >= FK_MID) {
#pragma unroll
        for (int i = 0; i < NT; ++i) fused_store(act, f, i, p - 2, acc[i][SD], b4);
    }
    if (KIND == FK_MID && FSCHED) {
        // interleave: each MFMA followed by up to three VALU instructions (the
        // SiLU of the held-back plane), so both pipes stay busy
#pragma unroll
        for (int k = 0; k < NT * NC * 3; ++k) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
            __builtin_amdgcn_sched_group_barrier(0x002, 3, 0);
        }
    }
}

// A whole 16-output-channel layer for a wave with NT tiles.  base: element
// offset of the input half plane of plane 0 (planes are FSLOT apart).  After
// the last step: outputs 15 and 16; plane 16 was read by every wave in the
// last step, hence the barrier before storing it.
template <int NT, int NC>
__device__ __forceinline__ void fused_layer(__bf16 *act, int base, const int (&off)[FTPW][5],
                                            const bf16x8 (&wr)[3][5], const FusedCtx &f, const float *b4)
{
    static_assert(W == 17, "the unrolled walk assumes 17 planes");
    floatx4 acc[FTPW][4];
#pragma unroll
    for (int i = 0; i < FTPW; ++i) acc[i][0] = acc[i][1] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    bf16x8 b0[FTPW];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NT; ++i) b0[i] = FPREF ? fused_load(act, base, off[i][0]) : zero8();
    fused_kstep<NT, NC, FK_FIRST, 0>(act, base, 0, off, wr, acc, b0, f, b4);
    __syncthreads();
    fused_kstep<NT, NC, FK_SECOND, 1>(act, base + FSLOT, 1, off, wr, acc, b0, f, b4);
    for (int p = 2; p < 14; p += 4) {
        __syncthreads();
        fused_kstep<NT, NC, FK_MID, 2>(act, base + p * FSLOT, p, off, wr, acc, b0, f, b4);
        __syncthreads();
        fused_kstep<NT, NC, FK_MID, 3>(act, base + (p + 1) * FSLOT, p + 1, off, wr, acc, b0, f, b4);
        __syncthreads();
        fused_kstep<NT, NC, FK_MID, 0>(act, base + (p + 2) * FSLOT, p + 2, off, wr, acc, b0, f, b4);
        __syncthreads();
        fused_kstep<NT, NC, FK_MID, 1>(act, base + (p + 3) * FSLOT, p + 3, off, wr, acc, b0, f, b4);
    }
    __syncthreads();
    fused_kstep<NT, NC, FK_MID, 2>(act, base + 14 * FSLOT, 14, off, wr, acc, b0, f, b4);
    __syncthreads();
    fused_kstep<NT, NC, FK_MID, 3>(act, base + 15 * FSLOT, 15, off, wr, acc, b0, f, b4);
    __syncthreads();
    fused_kstep<NT, NC, FK_LAST, 0>(act, base + 16 * FSLOT, 16, off, wr, acc, b0, f, b4);
#pragma unroll
    for (int i = 0; i < NT; ++i) fused_store(act, f, i, 15, acc[i][3], b4);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NT; ++i) fused_store(act, f, i, 16, acc[i][0], b4);
}

// The last layer (16 -> 1) for a wave with NT tiles: A rows = dz, so the
// MFMAs of a tile give the contributions of input plane p to output planes
// p + 1, p, p - 1 (rows 0, 1, 2 in the lanes with kb = 0); the lanes keep the
// three running sums and write output plane p - 1 (FP32, + bias) to z5g, the
// window's slice of global scratch.  The layer writes no LDS, so the waves
// walk the planes without barriers.
template <int NT>
__device__ __forceinline__ void fused_last_layer(const __bf16 *act, const int (&off)[FTPW][5], const bf16x8 (&w4)[5],
                                                 const FusedCtx &f, float b5, float *z5g)
{
    float sacc[FTPW][3];
#pragma unroll
    for (int i = 0; i < FTPW; ++i) sacc[i][0] = sacc[i][1] = sacc[i][2] = 0.0f;
#pragma unroll
    for (int p = 0; p < W; ++p) {
        floatx4 ca[NT], cb[NT];                              // even / odd chunks: two independent chains
#pragma unroll
        for (int i = 0; i < NT; ++i) ca[i] = cb[i] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            bf16x8 b[NT];
#pragma unroll
            for (int i = 0; i < NT; ++i) b[i] = fused_load(act, p * FSLOT, off[i][c]);
#pragma unroll
            for (int i = 0; i < NT; ++i) {
                if (c & 1) cb[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w4[c], b[i], cb[i], 0, 0, 0);
                else       ca[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w4[c], b[i], ca[i], 0, 0, 0);
            }
        }
#pragma unroll
        for (int i = 0; i < NT; ++i) {
            if (p + 1 < W) sacc[i][2] += ca[i][0] + cb[i][0];
            sacc[i][1] += ca[i][1] + cb[i][1];
            if (p > 0) {
                sacc[i][0] += ca[i][2] + cb[i][2];
                if (f.kb == 0 && f.vok[i]) z5g[(p - 1) * W2 + f.vp[i]] = sacc[i][0] + b5;
            }
            sacc[i][0] = sacc[i][1];
            sacc[i][1] = sacc[i][2];
            sacc[i][2] = 0.0f;
        }
    }
#pragma unroll
    for (int i = 0; i < NT; ++i)
        if (f.kb == 0 && f.vok[i]) z5g[(W - 1) * W2 + f.vp[i]] = sacc[i][0] + b5;
}

__global__ void __launch_bounds__(FNT)
fused_kernel(NnFusedArgs a)
{
    __shared__ __align__(16) __bf16 act[W * FSLOT];
    __shared__ float f1t[256];
    __shared__ uint8_t opt[256];
    __shared__ unsigned smask[(V + 31) / 32];
    __shared__ float redf[FWAVES];
    __shared__ double redd[FWAVES];
    __shared__ int flag;
    __shared__ __align__(16) __bf16 dummy[8];
    constexpr int PER = (V + FNT - 1) / FNT;                 // window cells per thread (10)

    FusedCtx f;
    const int t = threadIdx.x;
    f.lane = t & 63; f.wave = t >> 6; f.n = f.lane & 15; f.kb = f.lane >> 4;
    const int q = blockIdx.x;
    {
        const int64_t s = a.src[q];
        const int64_t plane = (int64_t)a.nx * a.ny;
        f.sz = (int)(s / plane);
        const int64_t rem = s - (int64_t)f.sz * plane;
        f.sy = (int)(rem / a.nx);
        f.sx = (int)(rem - (int64_t)f.sy * a.nx);
    }
    for (int i = t; i < 256; i += FNT) { f1t[i] = a.f1[i]; opt[i] = a.open[i]; }

    // ---- structural support (scratch in the activation area), kept as a bit mask
    uint8_t *openw = reinterpret_cast<uint8_t *>(act), *sa = openw + V, *sb = sa + V;
    if (t == 0) flag = 1;
    // the labels of this thread's cells (v = t + k FNT), all loads in flight at once
    unsigned labp[(PER + 3) / 4] = {};                       // labels packed 4 per register
    unsigned inmask = 0;
    float pr[PER];                                           // prior of the same cells
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int v = t + k * FNT;
        const int wx = v % W, wy = (v / W) % W, wz = v / W2;
        const int gx = f.sx - R + wx, gy = f.sy - R + wy, gz = f.sz - R + wz;
        const bool in = v < V && gx >= 0 && gx < a.nx && gy >= 0 && gy < a.ny && gz >= 0 && gz < a.nz;
        inmask |= (unsigned)in << k;
        const unsigned lb = in ? a.label[((int64_t)gz * a.ny + gy) * a.nx + gx] : 0u;
        labp[k >> 2] |= lb << (8 * (k & 3));
        pr[k] = v < V ? a.prior[v] : 0.0f;
    }
    __syncthreads();
    int notopen = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int v = t + k * FNT;
        if (v >= V) break;
        const bool in = (inmask >> k) & 1u;
        const uint8_t op = in ? opt[(labp[k >> 2] >> (8 * (k & 3))) & 255u] : 0;
        if (in && !op) notopen = 1;
        openw[v] = op;
        sa[v] = v == (R * W + R) * W + R ? 1 : 0;
    }
    if (notopen) atomicAnd(&flag, 0);
    __syncthreads();
    const bool fast = flag && a.n_sub >= 3 * R;
    __syncthreads();
    const uint8_t *sup = fast ? nullptr : grow_support(openw, sa, sb, a.n_sub, &flag);
    // bit mask: cells v = t + k FNT of a wave are 64 consecutive bits
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int v = t + k * FNT;
        const bool in = fast ? ((inmask >> k) & 1u) != 0 : (v < V && sup[v] != 0);
        const unsigned long long bits = __ballot(in);
        const int wd = (v - f.lane) >> 5;
        if (f.lane == 0 && wd < (V + 31) / 32) smask[wd] = (unsigned)bits;
        if (f.lane == 0 && wd + 1 < (V + 31) / 32) smask[wd + 1] = (unsigned)(bits >> 32);
    }
    __syncthreads();                                         // mask complete; support scratch free
    for (int k = t; k < 2 * W; k += FNT)                     // the zero pad of every half plane
        *reinterpret_cast<bf16x8 *>(act + (size_t)k * FHALF + FPAD) = zero8();
    if (a.support)
        for (int v = t; v < V; v += FNT) a.support[(int64_t)q * V + v] = (smask[v >> 5] >> (v & 31)) & 1u;

    // ---- this lane's voxels and operand offsets (element offsets within a plane)
#pragma unroll
    for (int i = 0; i < FTPW; ++i) {
        const int tile = f.wave + FWAVES * i;
        f.vp[i] = tile * 16 + f.n;
        f.vok[i] = tile < FTILES && f.vp[i] < W2;
        f.sto[i] = (f.kb >> 1) * FHALF + f.vp[i] * 8 + 4 * (f.kb & 1);
    }
    f.dummy = dummy;
    int off8[FTPW][5], off16[FTPW][5];
#pragma unroll
    for (int i = 0; i < FTPW; ++i) {
        const int y = f.vok[i] ? f.vp[i] / W : 0, x = f.vok[i] ? f.vp[i] % W : 0;
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            int pos = 4 * c + f.kb;
            int yy = y + pos / 3 - 1, xx = x + pos % 3 - 1;
            bool ok = c < 3 && f.vok[i] && pos < 9 && yy >= 0 && yy < W && xx >= 0 && xx < W;
            off8[i][c] = ok ? (yy * W + xx) * 8 : FPAD;
            pos = 2 * c + (f.kb >> 1);
            yy = y + pos / 3 - 1;
            xx = x + pos % 3 - 1;
            ok = f.vok[i] && pos < 9 && yy >= 0 && yy < W && xx >= 0 && xx < W;
            off16[i][c] = ok ? (f.kb & 1) * FHALF + (yy * W + xx) * 8 : FPAD;
        }
    }

    // ---- layer-0 input: the features of every plane (8 BF16 channels) in the
    // second half of that plane's activation slot; layer 0's output plane z
    // overwrites slot z only after feature plane z has been consumed
    {
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int v = t + k * FNT;
            if (v >= V) break;
            const int pz = v / W2, vp = v - pz * W2;
            const bool in = (inmask >> k) & 1u;
            bf16x8 x8 = zero8();
            const unsigned lb = (labp[k >> 2] >> (8 * (k & 3))) & 255u;
            x8[0] = (__bf16)(in && opt[lb] ? 1.0f : 0.0f);
            x8[1] = (__bf16)(in ? f1t[lb] : -1.0f);
            x8[2] = (__bf16)(pr[k] * (1.0f / 20.0f));
            *reinterpret_cast<bf16x8 *>(act + (size_t)pz * FSLOT + FHALF + vp * 8) = x8;
        }
    }

    // ---- layer 0 (3 -> 16 channels)
    {
        const bf16x8 *wp = reinterpret_cast<const bf16x8 *>(a.wf[0]);
        bf16x8 wr[3][5];
#pragma unroll
        for (int dz = 0; dz < 3; ++dz)
#pragma unroll
            for (int c = 0; c < 5; ++c) wr[dz][c] = c < 3 ? wp[(dz * 3 + c) * 64 + f.lane] : zero8();
        float b4[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) b4[j] = a.bias[0][4 * f.kb + j];
        if (f.wave < FTILES - (FTPW - 1) * FWAVES) fused_layer<FTPW, 3>(act, FHALF, off8, wr, f, b4);
        else                                      fused_layer<FTPW - 1, 3>(act, FHALF, off8, wr, f, b4);
    }

    // ---- layers 1 .. 3: in place in LDS
    for (int l = 1; l <= 3; ++l) {
        const bf16x8 *wp = reinterpret_cast<const bf16x8 *>(a.wf[l]);
        bf16x8 wr[3][5];
#pragma unroll
        for (int dz = 0; dz < 3; ++dz)
#pragma unroll
            for (int c = 0; c < 5; ++c) wr[dz][c] = wp[(dz * 5 + c) * 64 + f.lane];
        float b4[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) b4[j] = a.bias[l][4 * f.kb + j];
        if (f.wave < FTILES - (FTPW - 1) * FWAVES) fused_layer<FTPW, 5>(act, 0, off16, wr, f, b4);
        else                                      fused_layer<FTPW - 1, 5>(act, 0, off16, wr, f, b4);
    }

    // ---- layer 4 (16 -> 1): z5 (FP32) into the window's global scratch slice
    float *z5g = a.z5g + (int64_t)q * V;
    float prs[PER];                                          // prior again, for the softmax
    {
        const bf16x8 *wp = reinterpret_cast<const bf16x8 *>(a.wf[4]);
        bf16x8 w4[5];
#pragma unroll
        for (int c = 0; c < 5; ++c) w4[c] = wp[c * 64 + f.lane];
        const float b5 = a.bias[4][0];
#pragma unroll
        for (int k = 0; k < PER; ++k) prs[k] = t + k * FNT < V ? a.prior[t + k * FNT] : 0.0f;
        __syncthreads();                                     // layer 3's last plane is stored
        if (f.wave < FTILES - (FTPW - 1) * FWAVES) fused_last_layer<FTPW>(act, off16, w4, f, b5, z5g);
        else                                      fused_last_layer<FTPW - 1>(act, off16, w4, f, b5, z5g);
        __syncthreads();                                     // z5 complete and visible in the workgroup
    }

    // ---- softmax over the support (this thread's cells in registers)
    float lg[PER];
    unsigned smine = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) lg[k] = prs[k];
    float mx = -INFINITY;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int v = t + k * FNT;
        if (v >= V) break;
        lg[k] += z5g[v];
        if (a.logits) a.logits[(int64_t)q * V + v] = lg[k];
        const bool in = (smask[v >> 5] >> (v & 31)) & 1u;
        smine |= (unsigned)in << k;
        if (in) mx = fmaxf(mx, lg[k]);
    }
    for (int off = 32; off >= 1; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 64));
    if (f.lane == 0) redf[f.wave] = mx;
    __syncthreads();
    mx = redf[0];
    for (int w = 1; w < FWAVES; ++w) mx = fmaxf(mx, redf[w]);
    double se = 0.0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        lg[k] = ((smine >> k) & 1u) ? __expf(lg[k] - mx) : 0.0f;
        if ((smine >> k) & 1u) se += (double)lg[k];
    }
    se = block_reduce_sum<double, FWAVES>(se, redd);
    const float inv = (float)(1.0 / se);
    double ms = 0.0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int v = t + k * FNT;
        if (v >= V) break;
        const bool in = (smine >> k) & 1u;
        const float g = in ? lg[k] * inv : 0.0f;
        if (a.G) a.G[(int64_t)q * V + v] = g;
        ms += (double)g;
    }
    ms = block_reduce_sum<double, FWAVES>(ms, redd);
    if (t == 0 && a.mass) a.mass[q] = ms;
}

}  // namespace nn

// ----------------------------------------------------------------- launchers

static unsigned grid_1d(int64_t n, int nt)
{
    int64_t g = (n + nt - 1) / nt;
    if (g < 1) g = 1;
    if (g > 16384) g = 16384;
    return (unsigned)g;
}

int nn_slabs_per_window() { return nn::NSLAB; }
int nn_pack_chunks(int CI) { return nn::nchunks(CI); }

int nn_fpack_elems(int layer) { return nn::fpack_count(layer) * 512; }

hipError_t nn_launch_fpack(const float *w, int layer, int co_n, int ci_n, uint16_t *out, hipStream_t st)
{
    hipLaunchKernelGGL(nn::fpack_kernel, dim3(grid_1d(nn::fpack_count(layer) * 512, 256)), dim3(256), 0, st, w,
                       layer, co_n, ci_n, out);
    return hipGetLastError();
}

hipError_t nn_launch_fused(const NnFusedArgs &a, int batch, hipStream_t st)
{
    if (batch <= 0) return hipSuccess;
    hipLaunchKernelGGL(nn::fused_kernel, dim3(batch), dim3(nn::FNT), 0, st, a);
    return hipGetLastError();
}

hipError_t nn_launch_features(const NnFeatArgs &a, int batch, hipStream_t st)
{
    if (batch <= 0) return hipSuccess;
    hipLaunchKernelGGL(nn::features_kernel, dim3(batch), dim3(nn::NTHR), 0, st, a);
    return hipGetLastError();
}

hipError_t nn_launch_pack(const float *w, int co_n, int ci_n, int CI, int flip, uint16_t *out, hipStream_t st)
{
    hipLaunchKernelGGL(nn::pack_kernel, dim3(grid_1d(nn::nchunks(CI) * 512, 256)), dim3(256), 0, st, w, co_n, ci_n,
                       CI, flip, out);
    return hipGetLastError();
}

hipError_t nn_launch_conv(int CI, const NnConvArgs &a, int batch, hipStream_t st)
{
    if (batch <= 0) return hipSuccess;
    const dim3 g((unsigned)(batch * nn::NSLAB));
    if (CI == 8) hipLaunchKernelGGL(nn::conv_kernel<8>, g, dim3(nn::NTHR), 0, st, a);
    else if (CI == 16) hipLaunchKernelGGL(nn::conv_kernel<16>, g, dim3(nn::NTHR), 0, st, a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t nn_launch_loss(const NnLossArgs &a, int batch, hipStream_t st)
{
    if (batch <= 0) return hipSuccess;
    hipLaunchKernelGGL(nn::softmax_loss_kernel, dim3(batch), dim3(nn::NTHR), 0, st, a);
    return hipGetLastError();
}

hipError_t nn_launch_silu_bwd(const float *dh, const float *zpre, uint16_t *dz, int64_t n, hipStream_t st)
{
    hipLaunchKernelGGL(nn::silu_bwd_kernel, dim3(grid_1d(n, 256)), dim3(256), 0, st, dh, zpre, dz, n);
    return hipGetLastError();
}

hipError_t nn_launch_wgrad(int CI, int COP, const NnWgradArgs &a, int grid, hipStream_t st)
{
    if (grid <= 0) return hipSuccess;
    const dim3 g((unsigned)grid);
    if (CI == 8 && COP == 16) hipLaunchKernelGGL((nn::wgrad_kernel<8, 16>), g, dim3(nn::NTHR), 0, st, a);
    else if (CI == 16 && COP == 16) hipLaunchKernelGGL((nn::wgrad_kernel<16, 16>), g, dim3(nn::NTHR), 0, st, a);
    else if (CI == 16 && COP == 8) hipLaunchKernelGGL((nn::wgrad_kernel<16, 8>), g, dim3(nn::NTHR), 0, st, a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t nn_launch_wgrad_reduce(const float *part, const float *bpart, int grid, int co_n, int ci_n, float *gw,
                                  float *gb, hipStream_t st)
{
    hipLaunchKernelGGL(nn::wgrad_reduce_kernel, dim3((27 * 256 + 16 + 255) / 256), dim3(256), 0, st, part, bpart,
                       grid, co_n, ci_n, gw, gb);
    return hipGetLastError();
}

hipError_t nn_launch_adam(float *w, float *m, float *v, const float *g, int n, float lr, float b1, float b2,
                          float eps, float c1, float c2, hipStream_t st)
{
    hipLaunchKernelGGL(nn::adam_kernel, dim3(grid_1d(n, 256)), dim3(256), 0, st, w, m, v, g, n, lr, b1, b2, eps,
                       c1, c2);
    return hipGetLastError();
}

hipError_t nn_launch_lines_src(int64_t line0, int nlines, int nx, int ny, int nz, int64_t *src, hipStream_t st)
{
    hipLaunchKernelGGL(nn::lines_src_kernel, dim3(grid_1d((int64_t)nlines * nz, 256)), dim3(256), 0, st, line0,
                       nlines, nx, ny, nz, src);
    return hipGetLastError();
}

hipError_t nn_launch_apply(int nx, int ny, int nz, int64_t line0, int nlines, int seg_len, int n_seg,
                           const float *G, const double *mass, const double *c_in, double *c_out,
                           unsigned long long *n_used, hipStream_t st)
{
    if (nlines <= 0) return hipSuccess;
    hipLaunchKernelGGL(nn::apply_kernel, dim3((unsigned)(nlines * n_seg)), dim3(nn::APPLY_NT), 0, st, nx, ny, nz,
                       line0, seg_len, n_seg, G, mass, c_in, c_out, n_used);
    return hipGetLastError();
}

hipError_t nn_launch_l1(const float *a, const float *b, int batch, double *out, hipStream_t st)
{
    if (batch <= 0) return hipSuccess;
    hipLaunchKernelGGL(nn::l1_kernel, dim3(batch), dim3(nn::NTHR), 0, st, a, b, out);
    return hipGetLastError();
}

hipError_t nn_launch_fill_f32(float *p, int64_t n, float v, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(nn::fill_f32_kernel, dim3(grid_1d(n, 256)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

}  // namespace fdirw
