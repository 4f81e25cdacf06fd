// fdirw_coarse.hip -- coarse-mesh FDiRW (Sec. 3.1 of arXiv 2408.11376,
// Eqs. 10-15) on gfx950.
//
// Nodes are the grouped cells (the fast phases) of B x B x B blocks.  The
// coarse matrix is built once per geometry from the fine window kernels: every
// grouped source j of block J adds G_j(i) / m_j (m_j = its mass over grouped
// cells) to S[I - J][I] for the block I of each grouped window cell i (one workgroup per source: LDS bins per block offset, then one
// FP64 atomic per nonzero bin), and P = S / N_I is stored in the offset-major,
// 16-byte-grouped layout of the kernel bank.  A coarse step is then
//   mapping    C = mean of c over each group, on the coarse grid padded by K
//   FDiRW      C' = P C (row form: 2K+1 threads per node, one per z offset)
//   remapping  c'(i) = C'(node of i); cells outside every group keep c(i)
#include "fdirw_device.h"
#include "fdirw_launch.h"

namespace fdirw {

// node[i] = block index of cell i if its phase is grouped, else -1; count[I]
// += 1 for every grouped cell of block I (exact in FP64).
__global__ void coarse_nodes_kernel(const uint8_t *__restrict__ label, CoarseTable tab, int nx, int ny, int nz,
                                    int B, int ncx, int ncy, int *__restrict__ node, double *__restrict__ count)
{
    const int64_t n = (int64_t)nx * ny * nz;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(i % nx), y = (int)((i / nx) % ny), z = (int)(i / ((int64_t)nx * ny));
        const unsigned l = label[i];
        int v = COARSE_OUTSIDE;
        if (tab.reservoir[l]) {
            v = COARSE_RESERVOIR;
        } else if (tab.mobile[l]) {
            v = ((z / B) * ncy + y / B) * ncx + x / B;
            atomicAdd(&count[v], 1.0);
        }
        node[i] = v;
    }
}

// The window sub-steps of fdirw_device.h with the far-field boundary cells of
// the window held at 0 after every sub-step (they absorb what reaches them).
template <int M, int R>
__device__ __forceinline__ void run_substeps_sink(SegVals<M, R> &G, const Seg<M, R> &c,
                                                  typename Geo<M, R>::E *__restrict__ xb, const Place &p, int n_sub,
                                                  const bool (&sink)[Geo<M, R>::L0])
{
    using G_ = Geo<M, R>;
    constexpr int NCOL = G_::NCOL, L = G_::L0;
    const int col = G_::PADC + p.col;
    const int own = col * G_::ZS + p.seg * G_::SOFF;
    const int tail_at = G_::TAIL + p.seg * NCOL + col;
    const int head_at = G_::HEAD + p.seg * NCOL + col;
    const int zlo_at = G_::TAIL + (p.seg > 0 ? p.seg - 1 : 0) * NCOL + col;
    const int zhi_at = G_::HEAD + (p.seg < G_::NSEG - 1 ? p.seg + 1 : 0) * NCOL + col;
    for (int step = 0; step < n_sub; ++step) {
        one_substep<M, R>(G, c, (step & 1) ? xb + G_::XLEN : xb, p, own, tail_at, head_at, zlo_at, zhi_at);
#pragma unroll
        for (int k = 0; k < L; ++k)
            if (sink[k]) G[k] = 0;
    }
}

// One workgroup per grouped source: its fine window kernel over the grouped
// cells, summed per destination block into S[offset][I] (offset = I - J + K
// per axis, J the source's block).  Without a far field the kernel is
// renormalised to unit mass over the grouped cells; with one (SINK) the
// far-field cells absorb and the kernel keeps the mass that is left.
template <int M, int R, bool SINK>
__global__ void __launch_bounds__((Geo<M, R>::NT)) __attribute__((amdgpu_waves_per_eu(Geo<M, R>::MINW)))
coarse_window_kernel(CoarseGenArgs a)
{
    using G_ = Geo<M, R>;
    using T = typename G_::T;
    using S = typename G_::S;
    using E = typename G_::E;
    constexpr int L = G_::L0, W3 = G_::W3;
    __shared__ __align__(16) E xb[2 * G_::XLEN];
    __shared__ double red[G_::NWAVE];
    __shared__ double bins[W3];                    // (2K + 1)^3 <= W^3 block offsets

    const Place p = make_place<M, R>(threadIdx.x);
    for (int i = threadIdx.x; i < 2 * G_::XLEN; i += blockDim.x) xb[i] = (E)0.0f;   // padding stays 0
    for (int i = threadIdx.x; i < W3; i += blockDim.x) bins[i] = 0.0;
    __syncthreads();

    const S *lx = (const S *)a.lx, *ly = lx + a.n, *lz = ly + a.n;
    const int B = a.block, K = a.K, KW = 2 * a.K + 1, nb = KW * KW * KW;
    for (int64_t s = blockIdx.x; s < a.n; s += gridDim.x) {
        if (a.node[s] < 0) continue;                // source outside every group: uniform per block
        const int sx = (int)(s % a.nx), sy = (int)((s / a.nx) % a.ny), sz = (int)(s / ((int64_t)a.nx * a.ny));
        Seg<M, R> c;
        load_segment<M, R>(c, lx, ly, lz, a.nx, a.ny, a.nz, sx, sy, sz, p);
        compute_diag<T::x32, M, R>(c);
        S G[L];
        init_delta<M, R>(G, p);
        const int X = sx - R + p.cx, Y = sy - R + p.cy;
        const bool inxy = p.act && X >= 0 && X < a.nx && Y >= 0 && Y < a.ny;
        bool grp[L];
        if constexpr (SINK) {
            bool sink[L];
#pragma unroll
            for (int k = 0; k < L; ++k) {
                const int Z = sz - R + p.j0 + k;
                sink[k] = inxy && k < p.len && Z >= 0 && Z < a.nz &&
                          a.node[((int64_t)Z * a.ny + Y) * a.nx + X] == COARSE_RESERVOIR;
            }
            run_substeps_sink<M, R>(G, c, xb, p, a.n_sub, sink);
        } else {
            run_substeps<M, R>(G, c, xb, p, a.n_sub);
        }
        // the kernel's mass over the grouped cells (FP64, fixed order)
        double part = 0.0;
#pragma unroll
        for (int k = 0; k < L; ++k) {
            const int Z = sz - R + p.j0 + k;
            grp[k] = inxy && k < p.len && Z >= 0 && Z < a.nz && a.node[((int64_t)Z * a.ny + Y) * a.nx + X] >= 0;
            if (grp[k]) part += (double)G[k];
        }
        const double inv = SINK ? 1.0 : 1.0 / block_sum<G_::NWAVE>(part, red);
        const int jx = sx / B, jy = sy / B, jz = sz / B;
        if (inxy) {
            const int oxy = (Y / B - jy + K) * KW + (X / B - jx + K);
#pragma unroll
            for (int k = 0; k < L; ++k) {
                const int Z = sz - R + p.j0 + k;
                if (grp[k] && G[k] != S(0))
                    atomicAdd(&bins[(Z / B - jz + K) * KW * KW + oxy], (double)G[k] * inv);
            }
        }
        __syncthreads();
        for (int o = threadIdx.x; o < nb; o += blockDim.x) {
            const double v = bins[o];
            if (v != 0.0) {
                const int oz = o / (KW * KW), oy = (o / KW) % KW, ox = o % KW;
                const int64_t I = ((int64_t)(jz + oz - K) * a.ncy + (jy + oy - K)) * a.ncx + (jx + ox - K);
                atomicAdd(&a.S[(int64_t)o * a.n_nodes + I], v);
                bins[o] = 0.0;
            }
        }
        __syncthreads();                            // bins and exchange buffers are reused
    }
}

// The binning of coarse_window_kernel for kernels generated elsewhere (the
// flow kernels): G holds the W^3 window kernels of the sources src_base +
// 0 .. n_src-1 (entries of sources outside every group are not read).
constexpr int BIN_NT = 256;

template <typename T, int R, bool SINK>
__global__ void __launch_bounds__(BIN_NT) coarse_bin_kernel(CoarseGenArgs a, const T *__restrict__ G,
                                                            int64_t src_base, int64_t n_src)
{
    constexpr int W = 2 * R + 1, W2 = W * W, W3 = W2 * W;
    __shared__ double bins[W3];
    __shared__ double red[BIN_NT / 64];
    for (int i = threadIdx.x; i < W3; i += BIN_NT) bins[i] = 0.0;
    const int B = a.block, K = a.K, KW = 2 * a.K + 1, nb = KW * KW * KW;
    for (int64_t q = blockIdx.x; q < n_src; q += gridDim.x) {
        const int64_t s = src_base + q;
        if (a.node[s] < 0) continue;                              // uniform per block
        const int sx = (int)(s % a.nx), sy = (int)((s / a.nx) % a.ny), sz = (int)(s / ((int64_t)a.nx * a.ny));
        const int jx = sx / B, jy = sy / B, jz = sz / B;
        const T *g = G + q * (int64_t)W3;
        double part = 0.0;
        for (int w = threadIdx.x; w < W3; w += BIN_NT) {
            const int X = sx - R + w % W, Y = sy - R + (w / W) % W, Z = sz - R + w / W2;
            if (X >= 0 && X < a.nx && Y >= 0 && Y < a.ny && Z >= 0 && Z < a.nz &&
                a.node[((int64_t)Z * a.ny + Y) * a.nx + X] >= 0)
                part += (double)g[w];
        }
        double inv = 1.0;
        if (!SINK) {
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) part += __shfl_xor(part, off, 64);
            __syncthreads();
            if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = part;
            __syncthreads();
            double m = red[0];
            for (int k = 1; k < BIN_NT / 64; ++k) m += red[k];
            inv = 1.0 / m;
        }
        __syncthreads();
        for (int w = threadIdx.x; w < W3; w += BIN_NT) {
            const int X = sx - R + w % W, Y = sy - R + (w / W) % W, Z = sz - R + w / W2;
            if (X >= 0 && X < a.nx && Y >= 0 && Y < a.ny && Z >= 0 && Z < a.nz &&
                a.node[((int64_t)Z * a.ny + Y) * a.nx + X] >= 0 && g[w] != T(0))
                atomicAdd(&bins[((Z / B - jz + K) * KW + (Y / B - jy + K)) * KW + (X / B - jx + K)],
                          (double)g[w] * inv);
        }
        __syncthreads();
        for (int o = threadIdx.x; o < nb; o += BIN_NT) {
            const double v = bins[o];
            if (v != 0.0) {
                const int oz = o / (KW * KW), oy = (o / KW) % KW, ox = o % KW;
                const int64_t I = ((int64_t)(jz + oz - K) * a.ncy + (jy + oy - K)) * a.ncx + (jx + ox - K);
                atomicAdd(&a.S[(int64_t)o * a.n_nodes + I], v);
                bins[o] = 0.0;
            }
        }
        __syncthreads();
    }
}

// Node windows (window radius beyond the per-source kernels).  The column of
// group J is one FD of unit mass on every grouped cell of J, on the window of
// wb = (2K+1) B cells per axis made of J's block and the K blocks around it
// (clipped at the domain; faces leaving it are walls), for a batch of nodes at
// a time: state [batch][wb^3] in HBM, one launch per sub-step.
// Grid: x over the window's cells (32-bit indices), y over the batch's nodes.
template <typename St>
__global__ void nodewin_init_kernel(NodeWinArgs a, St *__restrict__ g)
{
    const int wb = a.wb, wb2 = wb * wb, wb3 = wb2 * wb;
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= wb3) return;
    const int jb = blockIdx.y;
    const int J = a.batch[jb];
    const int bx = J % a.ncx, by = (J / a.ncx) % a.ncy, bz = J / (a.ncx * a.ncy);
    const int X = (bx - a.K) * a.B + q % wb, Y = (by - a.K) * a.B + (q / wb) % wb, Z = (bz - a.K) * a.B + q / wb2;
    const bool in = X >= 0 && X < a.nx && Y >= 0 && Y < a.ny && Z >= 0 && Z < a.nz;
    g[(int64_t)jb * wb3 + q] = (in && a.node[((int64_t)Z * a.ny + Y) * a.nx + X] == J) ? St(1) : St(0);
}

// One explicit sub-step of every window of the batch: terms in the order -x,
// +x, -y, +y, -z, +z over faces inside both the window and the domain
// (coefficients of the domain's owned faces); cells outside the domain stay
// 0, and far-field cells are held at 0 when a.sink (they absorb).
template <typename St>
__global__ void nodewin_substep_kernel(NodeWinArgs a, const St *__restrict__ in_all, St *__restrict__ out_all)
{
    const int wb = a.wb, wb2 = wb * wb, wb3 = wb2 * wb;
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= wb3) return;
    const int jb = blockIdx.y;
    const St *in = in_all + (int64_t)jb * wb3;
    St *out = out_all + (int64_t)jb * wb3;
    const int J = a.batch[jb];
    const int bx = J % a.ncx, by = (J / a.ncx) % a.ncy, bz = J / (a.ncx * a.ncy);
    const int qx = q % wb, qy = (q / wb) % wb, qz = q / wb2;
    const int X = (bx - a.K) * a.B + qx, Y = (by - a.K) * a.B + qy, Z = (bz - a.K) * a.B + qz;
    if (!(X >= 0 && X < a.nx && Y >= 0 && Y < a.ny && Z >= 0 && Z < a.nz)) {
        out[q] = St(0);
        return;
    }
    const St *lx = (const St *)a.lx, *ly = lx + a.n, *lz = ly + a.n;
    const int64_t sy = a.nx, sz = (int64_t)a.nx * a.ny;
    const int64_t i = Z * sz + Y * sy + X;
    if (a.sink && a.node[i] == COARSE_RESERVOIR) {
        out[q] = St(0);
        return;
    }
    const St gv = in[q];
    St acc = gv;
    if (qx > 0 && X > 0) acc += lx[i - 1] * (in[q - 1] - gv);
    if (qx < wb - 1 && X < a.nx - 1) acc += lx[i] * (in[q + 1] - gv);
    if (qy > 0 && Y > 0) acc += ly[i - sy] * (in[q - wb] - gv);
    if (qy < wb - 1 && Y < a.ny - 1) acc += ly[i] * (in[q + wb] - gv);
    if (qz > 0 && Z > 0) acc += lz[i - sz] * (in[q - wb2] - gv);
    if (qz < wb - 1 && Z < a.nz - 1) acc += lz[i] * (in[q + wb2] - gv);
    out[q] = acc;
}

// Binning of the batch's windows, one workgroup per node J: wave w sums the
// grouped cells of destination block o = w, w + waves, ... (lanes over the
// block's cells in z, y, x order, a fixed butterfly), the bins are added in
// offset order for the scale (N_J over their total without a far field, 1
// with one), and S[o][I] = bin, I = J + o - K: one writer per entry.
constexpr int NODEWIN_BIN_NT = 256;

template <typename St>
__global__ void __launch_bounds__(NODEWIN_BIN_NT) nodewin_bin_kernel(NodeWinArgs a, const St *__restrict__ g,
                                                                    const double *__restrict__ count,
                                                                    double *__restrict__ S)
{
    __shared__ double bins[17 * 17 * 17];
    __shared__ double scale;
    const int jb = blockIdx.x;
    const int J = a.batch[jb];
    const int KW = 2 * a.K + 1, nb = KW * KW * KW, B = a.B, wb = a.wb;
    const int bx = J % a.ncx, by = (J / a.ncx) % a.ncy, bz = J / (a.ncx * a.ncy);
    const St *gw = g + (int64_t)jb * wb * wb * wb;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nwave = NODEWIN_BIN_NT / 64;
    for (int o = w; o < nb; o += nwave) {
        const int ox = o % KW, oy = (o / KW) % KW, oz = o / (KW * KW);
        double sum = 0.0;
        for (int c = lane; c < B * B * B; c += 64) {
            const int cx = c % B, cy = (c / B) % B, cz = c / (B * B);
            const int X = (bx - a.K + ox) * B + cx, Y = (by - a.K + oy) * B + cy, Z = (bz - a.K + oz) * B + cz;
            if (X >= 0 && X < a.nx && Y >= 0 && Y < a.ny && Z >= 0 && Z < a.nz &&
                a.node[((int64_t)Z * a.ny + Y) * a.nx + X] >= 0)
                sum += (double)gw[((int64_t)(oz * B + cz) * wb + (oy * B + cy)) * wb + (ox * B + cx)];
        }
#pragma unroll
        for (int m = 32; m > 0; m >>= 1) sum += __shfl_xor(sum, m, 64);
        if (lane == 0) bins[o] = sum;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot = 0.0;
        for (int o = 0; o < nb; ++o) tot += bins[o];
        scale = a.sink ? 1.0 : (tot > 0.0 ? count[J] / tot : 0.0);
    }
    __syncthreads();
    for (int o = threadIdx.x; o < nb; o += NODEWIN_BIN_NT) {
        const int ox = o % KW, oy = (o / KW) % KW, oz = o / (KW * KW);
        const int Ix = bx + ox - a.K, Iy = by + oy - a.K, Iz = bz + oz - a.K;
        if (Ix < 0 || Ix >= a.ncx || Iy < 0 || Iy >= a.ncy || Iz < 0 || Iz >= a.ncz) continue;
        const int64_t I = ((int64_t)Iz * a.ncy + Iy) * a.ncx + Ix;
        S[(int64_t)o * a.n_nodes + I] = bins[o] * scale;
    }
}

// P[o][I] = S[o][I] / N_I in the bank layout of element type B: per offset
// plane of `plane` elements, chunks of zb nodes along z, chunk (z / zb, y, x)
// (x fastest) at its own index or, with slot, at slot[chunk] (the compact
// layout of the listed chunks; nodes of unlisted chunks hold no cells and are
// not stored).
template <typename B>
__global__ void coarse_finalize_kernel(const double *__restrict__ S, const double *__restrict__ count,
                                       int64_t n_nodes, int nb, int ncx, int ncy, int ncz, const int *__restrict__ slot,
                                       int64_t plane, B *__restrict__ P)
{
    constexpr int zb = 16 / (int)sizeof(B);
    const int64_t total = (int64_t)nb * n_nodes;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t o = i / n_nodes, I = i - o * n_nodes;
        const int x = (int)(I % ncx), y = (int)((I / ncx) % ncy), z = (int)(I / ((int64_t)ncx * ncy));
        const double nI = count[I];
        const double v = nI > 0.0 ? S[i] / nI : 0.0;
        const int64_t ch = ((int64_t)(z / zb) * ncy + y) * ncx + x;
        const int64_t at = slot ? slot[ch] : ch;
        if (at >= 0) P[o * plane + at * zb + z % zb] = (B)v;
    }
}

// Arithmetic of the coarse product (Sec. 3.3, Fig. 3, Table 2): the type of
// the padded C, of the products and of the accumulation.
//   COARSE_FP64   C FP64; products and sums FP64 (P of any storage, widened)
//   COARSE_FP32   C FP32; fused FP32 multiply-adds (P stored in FP32)
//   COARSE_MIXED  C rounded to FP32 then FP16; each product taken in FP16
//                 (P stored in FP16), the products accumulated in FP32
//   COARSE_FP16   as MIXED with FP16 accumulation
template <int A> struct CoarseArith;
template <> struct CoarseArith<COARSE_FP64> { using C = double; using Acc = double; };
template <> struct CoarseArith<COARSE_FP32> { using C = float; using Acc = float; };
template <> struct CoarseArith<COARSE_MIXED> { using C = _Float16; using Acc = float; };
template <> struct CoarseArith<COARSE_FP16> { using C = _Float16; using Acc = _Float16; };

// A mapped value (FP64 mean) in the C type of the arithmetic (FP16 via FP32).
template <typename TC> __device__ __forceinline__ TC to_c(double v) { return (TC)v; }
template <> __device__ __forceinline__ _Float16 to_c<_Float16>(double v) { return f64_to_f16_via_f32(v); }

template <typename T> __device__ __forceinline__ double widen(T v) { return (double)(float)v; }
template <> __device__ __forceinline__ double widen<double>(double v) { return v; }

// acc + p c in the arithmetic A (p: P in its storage type, c: C).
template <int A, typename T>
__device__ __forceinline__ typename CoarseArith<A>::Acc coarse_term(typename CoarseArith<A>::Acc acc, T p,
                                                                    typename CoarseArith<A>::C c)
{
    if constexpr (A == COARSE_FP64) {
        return __builtin_fma(widen<T>(p), c, acc);
    } else if constexpr (A == COARSE_FP32) {
        return __builtin_fmaf(p, c, acc);
    } else {
        _Float16 pr = p * c;                                      // the FP16 product
        asm volatile("" : "+v"(pr));                             // rounded before it is added
        if constexpr (A == COARSE_MIXED) return acc + (float)pr;
        else return (_Float16)(acc + pr);
    }
}

// The far-field term P_BC c_ff (P_BC held in FP64) added in the arithmetic A.
template <int A>
__device__ __forceinline__ typename CoarseArith<A>::Acc coarse_bc_term(typename CoarseArith<A>::Acc acc, double pbc,
                                                                       double cff)
{
    if constexpr (A == COARSE_FP64) return __builtin_fma(pbc, cff, acc);
    else if constexpr (A == COARSE_FP32) return __builtin_fmaf((float)pbc, (float)cff, acc);
    else return coarse_term<A, _Float16>(acc, (_Float16)pbc, to_c<_Float16>(cff));
}

// Eq. 13 on the coarse grid padded by K, for grids where most blocks hold
// grouped cells.  One workgroup per (by, bz) row of blocks: each thread sums
// one fine x column over the block's B x B (z, y) rows (coalesced across the
// threads, eight loads in flight), then one thread per block adds its B
// columns in x order: a fixed order, so the mapping is deterministic.  Blocks
// without grouped cells read nothing and keep the 0 written when the handle
// was built, as does the halo.
template <typename TC>
__global__ void __launch_bounds__(256) coarse_map_rows_kernel(const double *__restrict__ c,
                                                             const int *__restrict__ node,
                                                             const double *__restrict__ count, int nx, int ny, int nz,
                                                             int B, int ncx, int ncy, CoarsePad pad,
                                                             TC *__restrict__ cpad)
{
    __shared__ double col[256];
    const int by = blockIdx.x, bz = blockIdx.y;
    const int y0 = by * B, z0 = bz * B;
    const int y1 = min(ny, y0 + B), z1 = min(nz, z0 + B);
    const double *cnt = count + ((int64_t)bz * ncy + by) * ncx;
    for (int xb0 = 0; xb0 < ncx; xb0 += 256 / B) {               // blocks of this pass
        const int nbk = min(256 / B, ncx - xb0);
        const int x = xb0 * B + threadIdx.x;
        double s = 0.0;
        const bool used = threadIdx.x < nbk * B && cnt[xb0 + threadIdx.x / B] > 0.0;
        if (used && x < nx) {
            const int ny_b = y1 - y0, n_q = (z1 - z0) * ny_b;
            for (int q0 = 0; q0 < n_q; q0 += 8) {
                int64_t at[8];
                int nd[8];
                double v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int q = q0 + u < n_q ? q0 + u : n_q - 1;
                    at[u] = ((int64_t)(z0 + q / ny_b) * ny + (y0 + q % ny_b)) * nx + x;
                    nd[u] = node[at[u]];
                }
                // values loaded with their node indices (every at[] is a cell
                // of the domain), only the grouped ones added
#pragma unroll
                for (int u = 0; u < 8; ++u) v[u] = c[at[u]];
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (q0 + u < n_q && nd[u] >= 0) s += v[u];
            }
        }
        __syncthreads();                                          // col of the previous pass is read
        col[threadIdx.x] = s;
        __syncthreads();
        if (threadIdx.x < nbk) {
            const int bx = xb0 + threadIdx.x;
            const double nI = cnt[bx];
            if (nI > 0.0) {
                double t = 0.0;
                for (int k = 0; k < B; ++k) t += col[threadIdx.x * B + k];
                cpad[coarse_pad_at(pad, bx, by, bz)] = to_c<TC>(t / nI);
            }
        }
    }
}

// Eq. 13 on the coarse grid padded by K, for sparse grids.  One wave per node: lane l sums the
// grouped cells l, l + 64, ... of the node's block (cells in z, y, x order),
// the lanes are combined by a fixed butterfly, and lane 0 writes the mean.
// Empty nodes return at once: their padded entries and the halo hold the 0
// written when the handle was built.
constexpr int MAP_NT = 256;

template <typename TC>
__global__ void __launch_bounds__(MAP_NT) coarse_map_kernel(const double *__restrict__ c, const int *__restrict__ node,
                                                            const double *__restrict__ count, int nx, int ny, int nz,
                                                            int B, int ncx, int ncy, int ncz, CoarsePad pad,
                                                            TC *__restrict__ cpad, const int *__restrict__ used,
                                                            int64_t n_used)
{
    const int64_t wv = blockIdx.x * (int64_t)(MAP_NT / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int64_t n_nodes = (int64_t)ncx * ncy * ncz;
    if (wv >= (used ? n_used : n_nodes)) return;                  // uniform per wave
    const int64_t I = used ? used[wv] : wv;
    const double nI = count[I];
    if (!(nI > 0.0)) return;
    const int bx = (int)(I % ncx), by = (int)((I / ncx) % ncy), bz = (int)(I / ((int64_t)ncx * ncy));
    const int x0 = bx * B, y0 = by * B, z0 = bz * B;
    const int wx = min(nx, x0 + B) - x0, wy = min(ny, y0 + B) - y0, wz = min(nz, z0 + B) - z0;
    const int n_cells = wx * wy * wz;
    double s = 0.0;
    for (int q0 = lane; q0 < n_cells; q0 += 4 * 64) {
        int64_t at[4];
        int nd[4];
        double v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int q = q0 + 64 * u < n_cells ? q0 + 64 * u : q0;
            const int dz = q / (wx * wy), rem = q - dz * wx * wy, dy = rem / wx, dx = rem - dy * wx;
            at[u] = ((int64_t)(z0 + dz) * ny + (y0 + dy)) * nx + (x0 + dx);
            nd[u] = node[at[u]];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = c[at[u]];                  // with the indices; grouped ones added
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (q0 + 64 * u < n_cells && nd[u] >= 0) s += v[u];
    }
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) s += __shfl_xor(s, m, 64);
    if (lane == 0) cpad[coarse_pad_at(pad, bx, by, bz)] = to_c<TC>(s / nI);
}

// Eq. 14 on the coarse grid: C'_I = sum over the (2K+1)^3 offsets o of
// P[o][I] C[I - o] (FP64), with P in the bank layout of element type T (for
// each offset, chunks of zb = 16 / sizeof(T) nodes consecutive along z; the
// chunks ordered x fastest).  Two shapes, fixed by K together with the padded
// grid's layout (coarse_pad).
//
// coarse_apply_rows_kernel (K < COARSE_CHUNK_MIN_K, C padded x fastest): a wave
// takes 64 nodes that are consecutive in the layout (64 / zb chunks), so every
// P load of the wave is one contiguous 128..512-byte run; wave w of the
// workgroup takes the offsets with oz = w, summing its terms in (oy, ox)
// order; the wave partials of a node are then added in wave order.
//
// coarse_apply_chunks_kernel (K >= COARSE_CHUNK_MIN_K, C padded z fastest): one
// lane takes one chunk of the list of chunks holding a node with cells (64
// chunks per wave; the zb entries of P of a chunk are one 16-byte load) and
// one range of offset pairs (oy, ox): for each pair it loads the chunk's C
// column (zb + 2K values, shared by the 2K + 1 z offsets) and, for oz = 0 ..
// 2K, the zb entries of P, so each P element is read once and each load
// serves zb nodes.  Terms are summed in (oy, ox, oz) order within a range;
// coarse_apply_sum_kernel adds the ranges of a node in a fixed order (ranges
// in order within contiguous blocks, then the block sums in order).  P is
// stored compactly: the listed chunks only, in list order.
//
// Either way the sum of every node has one fixed order.
constexpr int APPLY_MAX_WAVES = 16;

// groups: the 64-position groups of P's layout to run (those that hold a node
// with cells).
template <typename T, int KW, int A>
__global__ void __launch_bounds__(64 * APPLY_MAX_WAVES) coarse_apply_rows_kernel(
    const T *__restrict__ P, const typename CoarseArith<A>::C *__restrict__ cpad, int ncx, int ncy, int ncz,
    const double *__restrict__ pbc_pad, double c_ff, const double *__restrict__ cff_dev,
    const double *__restrict__ count, double *__restrict__ cnew, const int *__restrict__ groups)
{
    using TC = typename CoarseArith<A>::C;
    using TA = typename CoarseArith<A>::Acc;
    constexpr int zb = 16 / (int)sizeof(T);
    constexpr int K = (KW - 1) / 2, kw = KW;                      // the x offsets unrolled: kw loads in flight
    __shared__ double part[APPLY_MAX_WAVES * 64];
    const int px = ncx + 2 * K, py = ncy + 2 * K;
    const int nw = blockDim.x >> 6;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t n_chunks = (int64_t)((ncz + zb - 1) / zb) * ncy * ncx;
    const int64_t plane = n_chunks * zb;
    const int64_t ch = (int64_t)groups[blockIdx.x] * (64 / zb) + lane / zb;   // (zg, y, x) chunk
    const int j = lane % zb;
    TA acc = TA(0);
    int x = 0, y = 0, z = ncz;
    if (ch < n_chunks) {
        x = (int)(ch % ncx);
        y = (int)((ch / ncx) % ncy);
        z = (int)(ch / ((int64_t)ncx * ncy)) * zb + j;
    }
    // nodes without grouped cells are never read back: skipped
    if (z < ncz && !(count[((int64_t)z * ncy + y) * ncx + x] > 0.0)) z = ncz;
    if (z < ncz) {
        for (int oz = w; oz < kw; oz += nw) {
            const T *p = P + ch * zb + j + (int64_t)oz * kw * kw * plane;
            int o = 0;
            for (int oy = 0; oy < kw; ++oy) {
                // source (z - oz + K, y - oy + K, x - ox + K) = padded (z - oz + 2K, ...), x fastest
                const TC *crow = cpad + ((int64_t)(z - oz + 2 * K) * py + (y - oy + 2 * K)) * px + (x + 2 * K);
                T pv[kw];
                TC cv[kw];
#pragma unroll
                for (int ox = 0; ox < kw; ++ox) {
                    pv[ox] = p[(o + ox) * plane];
                    cv[ox] = crow[-ox];
                }
#pragma unroll
                for (int ox = 0; ox < kw; ++ox) acc = coarse_term<A, T>(acc, pv[ox], cv[ox]);
                o += kw;
            }
        }
    }
    part[threadIdx.x] = (double)acc;                              // exact: acc is a TA value
    __syncthreads();
    if (w == 0 && z < ncz) {
        TA s = TA(0);
        for (int k = 0; k < nw; ++k) s = (TA)(s + (TA)part[k * 64 + lane]);
        if (pbc_pad)                                              // far-field term of Eq. 14
            s = coarse_bc_term<A>(s, pbc_pad[coarse_pad_at(coarse_pad(ncx, ncy, ncz, K), x, y, z)],
                                  cff_dev ? *cff_dev : c_ff);
        cnew[((int64_t)z * ncy + y) * ncx + x] = (double)s;
    }
}

constexpr int APPLY_NT = 256;

template <typename T, int KW, int A>
__global__ void __launch_bounds__(APPLY_NT) coarse_apply_chunks_kernel(
    const T *__restrict__ P, const typename CoarseArith<A>::C *__restrict__ cpad, int ncx, int ncy, int ncz,
    const int *__restrict__ chunks, int64_t n_chunks, int64_t n_chunk_pad, int pairs_per_range, int n_split,
    double *__restrict__ part)
{
    using TC = typename CoarseArith<A>::C;
    using TA = typename CoarseArith<A>::Acc;
    constexpr int zb = 16 / (int)sizeof(T);
    constexpr int K = (KW - 1) / 2, NC = zb + 2 * K;               // C column: zb nodes and 2K neighbours
    const int64_t n_waves = (n_chunk_pad / 64) * n_split;
    const int64_t wv = blockIdx.x * (int64_t)(APPLY_NT / 64) + (threadIdx.x >> 6);
    if (wv >= n_waves) return;                                    // uniform per wave
    const int lane = threadIdx.x & 63;
    const int split = (int)(wv % n_split);
    const int64_t ci = (wv / n_split) * 64 + lane;                // slot in the chunk list
    TA acc[zb];
#pragma unroll
    for (int j = 0; j < zb; ++j) acc[j] = TA(0);
    if (ci < n_chunks) {
        const int64_t ch = chunks[ci];                            // (zg, y, x) chunk of P's layout
        const int x = (int)(ch % ncx), y = (int)((ch / ncx) % ncy);
        const int z0 = (int)(ch / ((int64_t)ncx * ncy)) * zb;
        const int64_t plane = n_chunks * zb;                      // P stored compactly in list order
        const CoarsePad pad = coarse_pad(ncx, ncy, ncz, K);
        const T *p0 = P + ci * zb;
        const int q0 = split * pairs_per_range;
        const int q1 = q0 + pairs_per_range < KW * KW ? q0 + pairs_per_range : KW * KW;
        for (int q = q0; q < q1; ++q) {
            const int oy = q / KW, ox = q - oy * KW;
            // padded z of node z0 + j and offset oz: z0 + j - oz + 2K, i.e. column entry j + 2K - oz
            const TC *colp = cpad + coarse_pad_at(pad, x - ox + K, y - oy + K, z0 - K);
            TC col[NC];
            if constexpr (A == COARSE_FP64) {
#pragma unroll
                for (int t = 0; t < NC; t += 2) {
                    const double2 v = *(const double2 *)(colp + t);
                    col[t] = v.x;
                    col[t + 1] = v.y;
                }
            } else {
#pragma unroll
                for (int t = 0; t < NC; ++t) col[t] = colp[t];
            }
            uint4 pv[KW];
#pragma unroll
            for (int oz = 0; oz < KW; ++oz) pv[oz] = *(const uint4 *)(p0 + ((int64_t)(oz * KW + oy) * KW + ox) * plane);
#pragma unroll
            for (int oz = 0; oz < KW; ++oz) {
                T e[zb];
                __builtin_memcpy(e, &pv[oz], 16);
#pragma unroll
                for (int j = 0; j < zb; ++j) acc[j] = coarse_term<A, T>(acc[j], e[j], col[j + 2 * K - oz]);
            }
        }
    }
    double *out = part + ((int64_t)split * n_chunk_pad + ci) * zb;
#pragma unroll
    for (int j = 0; j < zb; j += 2) *(double2 *)(out + j) = make_double2((double)acc[j], (double)acc[j + 1]);
}

// C'_I = the ranges' partial sums added in a fixed order, plus P_BC c_ff with
// a far field; nodes without grouped cells are never read back and not
// written.  SUM_TP consecutive lanes share a node: lane u adds the u-th
// contiguous block of ranges in order (sixteen loads in flight), and the
// first lane adds the SUM_TP block sums in lane order.
constexpr int SUM_TP = 8;

template <int A>
__global__ void coarse_apply_sum_kernel(const double *__restrict__ part, const int *__restrict__ chunks,
                                        int64_t n_chunks, int64_t n_chunk_pad, int n_split, int zb, int ncx, int ncy,
                                        int ncz, int K, const double *__restrict__ count,
                                        const double *__restrict__ pbc_pad, double c_ff,
                                        const double *__restrict__ cff_dev, double *__restrict__ cnew)
{
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t slot = t / SUM_TP;                              // (chunk slot, entry) of the node
    const int sub = (int)(t % SUM_TP);
    // every lane reaches the shuffles below: no early return
    bool valid = slot < n_chunks * zb;
    int64_t ci = 0, I = 0;
    int j = 0, x = 0, y = 0, z = 0;
    if (valid) {
        ci = slot / zb;
        j = (int)(slot - ci * zb);
        const int64_t ch = chunks[ci];
        x = (int)(ch % ncx);
        y = (int)((ch / ncx) % ncy);
        z = (int)(ch / ((int64_t)ncx * ncy)) * zb + j;
        valid = z < ncz;
        if (valid) {
            I = ((int64_t)z * ncy + y) * ncx + x;
            valid = count[I] > 0.0;
        }
    }
    using TA = typename CoarseArith<A>::Acc;
    TA s = TA(0);
    if (valid) {
        const int per = (n_split + SUM_TP - 1) / SUM_TP;
        const int k0 = sub * per, k1 = k0 + per < n_split ? k0 + per : n_split;
        const double *pp = part + ci * zb + j;
        const int64_t stride = n_chunk_pad * zb;
        for (int k = k0; k < k1; k += 16) {
            double v[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) v[u] = k + u < k1 ? pp[(int64_t)(k + u) * stride] : 0.0;
#pragma unroll
            for (int u = 0; u < 16; ++u)
                if (k + u < k1) s = (TA)(s + (TA)v[u]);
        }
    }
    const int base = (int)(threadIdx.x & 63) & ~(SUM_TP - 1);
    TA tot = TA(0);
#pragma unroll
    for (int u = 0; u < SUM_TP; ++u) tot = (TA)(tot + (TA)__shfl((double)s, base + u, 64));
    if (!valid || sub != 0) return;
    if (pbc_pad)                                                  // far-field term of Eq. 14
        tot = coarse_bc_term<A>(tot, pbc_pad[coarse_pad_at(coarse_pad(ncx, ncy, ncz, K), x, y, z)],
                                cff_dev ? *cff_dev : c_ff);
    cnew[I] = (double)tot;
}

// Eq. 15: every grouped cell takes its node's value, the others keep theirs;
// far-field cells are written 0 (the Eq. 7 value follows once the rest of the
// field has been summed).
__global__ void coarse_remap_kernel(const double *__restrict__ c_in, const int *__restrict__ node,
                                    const double *__restrict__ cnew, int64_t n, double *__restrict__ c_out)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int I = node[i];
        c_out[i] = I >= 0 ? cnew[I] : (I == COARSE_RESERVOIR ? 0.0 : c_in[i]);
    }
}

// c[i] = v on the far-field cells.
__global__ void coarse_fill_reservoir_kernel(const int *__restrict__ node, int64_t n, double v, double *__restrict__ c)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        if (node[i] == COARSE_RESERVOIR) c[i] = v;
}

// One explicit sub-step on the whole domain (no-flux walls) with the far-field
// cells held at 1: the response p_BC to a unit boundary concentration (Eq. 8).
// Terms in the order -x, +x, -y, +y, -z, +z, then the upwind flow terms in the
// same order (u null: no flow); FP64 state, coefficients of type S.
template <typename S>
__global__ void coarse_pbc_substep_kernel(const S *__restrict__ lx, const int *__restrict__ node, int nx, int ny,
                                          int nz, const double *__restrict__ u, double cour,
                                          const double *__restrict__ in, double *__restrict__ out)
{
    const int64_t n = (int64_t)nx * ny * nz;
    const S *ly = lx + n, *lz = ly + n;
    const int64_t sy = nx, sz = (int64_t)nx * ny;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (node[i] == COARSE_RESERVOIR) {
            out[i] = 1.0;
            continue;
        }
        const int x = (int)(i % nx), y = (int)((i / nx) % ny), z = (int)(i / sz);
        const double g = in[i];
        double acc = g;
        if (x > 0) acc += (double)lx[i - 1] * (in[i - 1] - g);
        if (x < nx - 1) acc += (double)lx[i] * (in[i + 1] - g);
        if (y > 0) acc += (double)ly[i - sy] * (in[i - sy] - g);
        if (y < ny - 1) acc += (double)ly[i] * (in[i + sy] - g);
        if (z > 0) acc += (double)lz[i - sz] * (in[i - sz] - g);
        if (z < nz - 1) acc += (double)lz[i] * (in[i + sz] - g);
        if (u) {
            // upwind flow: inflow through the lower faces, outflow through the upper
            const double *ux = u, *uy = ux + n, *uz = uy + n;
            double v;
            if (x > 0) { v = ux[i - 1] * cour; acc += v > 0.0 ? v * in[i - 1] : v * g; }
            if (x < nx - 1) { v = ux[i] * cour; acc -= v > 0.0 ? v * g : v * in[i + 1]; }
            if (y > 0) { v = uy[i - sy] * cour; acc += v > 0.0 ? v * in[i - sy] : v * g; }
            if (y < ny - 1) { v = uy[i] * cour; acc -= v > 0.0 ? v * g : v * in[i + sy]; }
            if (z > 0) { v = uz[i - sz] * cour; acc += v > 0.0 ? v * in[i - sz] : v * g; }
            if (z < nz - 1) { v = uz[i] * cour; acc -= v > 0.0 ? v * g : v * in[i + sz]; }
        }
        out[i] = acc;
    }
}

static unsigned grid_for(int64_t n)
{
    const int64_t b = (n + 255) / 256;
    return (unsigned)(b < 8192 ? (b > 0 ? b : 1) : 8192);
}

hipError_t launch_coarse_nodes(const uint8_t *label, const CoarseTable &tab, int nx, int ny, int nz, int B,
                               int ncx, int ncy, int *node, double *count, hipStream_t st)
{
    hipLaunchKernelGGL(coarse_nodes_kernel, dim3(grid_for((int64_t)nx * ny * nz)), dim3(256), 0, st, label, tab,
                       nx, ny, nz, B, ncx, ncy, node, count);
    return hipGetLastError();
}

template <int M, int R, bool SINK>
static hipError_t launch_cw_mr(const CoarseGenArgs &a, hipStream_t st)
{
    const int64_t nblk = a.n < 65536 * 16 ? a.n : 65536 * 16;
    if (nblk <= 0) return hipSuccess;
    hipLaunchKernelGGL((coarse_window_kernel<M, R, SINK>), dim3((unsigned)nblk), dim3(Geo<M, R>::NT), 0, st, a);
    return hipGetLastError();
}

template <int M, bool SINK>
static hipError_t launch_cw_m(int r, const CoarseGenArgs &a, hipStream_t st)
{
    switch (r) {
    case 0: return launch_cw_mr<M, 0, SINK>(a, st);
    case 1: return launch_cw_mr<M, 1, SINK>(a, st);
    case 2: return launch_cw_mr<M, 2, SINK>(a, st);
    case 3: return launch_cw_mr<M, 3, SINK>(a, st);
    case 4: return launch_cw_mr<M, 4, SINK>(a, st);
    case 5: return launch_cw_mr<M, 5, SINK>(a, st);
    case 6: return launch_cw_mr<M, 6, SINK>(a, st);
    case 7: return launch_cw_mr<M, 7, SINK>(a, st);
    case 8: return launch_cw_mr<M, 8, SINK>(a, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_coarse_window(int fp64, int sink, int r, const CoarseGenArgs &a, hipStream_t st)
{
    if (sink) return fp64 ? launch_cw_m<M_FP64, true>(r, a, st) : launch_cw_m<M_FP32, true>(r, a, st);
    return fp64 ? launch_cw_m<M_FP64, false>(r, a, st) : launch_cw_m<M_FP32, false>(r, a, st);
}

// n_sub sub-steps of coarse_pbc_substep_kernel from 0 (far-field cells 1),
// ping-ponging between a and b; *result points to the final field.
hipError_t launch_coarse_pbc_fd(int fp64, const void *lam, const int *node, int nx, int ny, int nz, int n_sub,
                                const double *u, double cour, double *a, double *b, double **result, hipStream_t st)
{
    const int64_t n = (int64_t)nx * ny * nz;
    hipError_t e = launch_fill(a, n, 0.0, st);
    if (e == hipSuccess) e = launch_coarse_fill_reservoir(node, n, 1.0, a, st);
    double *in = a, *out = b;
    for (int k = 0; k < n_sub && e == hipSuccess; ++k) {
        if (fp64)
            hipLaunchKernelGGL(coarse_pbc_substep_kernel<double>, dim3(grid_for(n)), dim3(256), 0, st,
                               (const double *)lam, node, nx, ny, nz, u, cour, in, out);
        else
            hipLaunchKernelGGL(coarse_pbc_substep_kernel<float>, dim3(grid_for(n)), dim3(256), 0, st,
                               (const float *)lam, node, nx, ny, nz, u, cour, in, out);
        e = hipGetLastError();
        double *t = in; in = out; out = t;
    }
    *result = in;
    return e;
}

hipError_t launch_nodewin(int fp64, const NodeWinArgs &a, int n_sub, void *ga, void *gb, const double *count,
                          double *S, hipStream_t st)
{
    if (a.n_batch <= 0) return hipSuccess;
    if (2 * a.K + 1 > 17) return hipErrorInvalidValue;
    if ((int64_t)a.wb * a.wb * a.wb > 0x7fffffffLL || a.n_batch > 65535) return hipErrorInvalidValue;
    const dim3 g((unsigned)(((int64_t)a.wb * a.wb * a.wb + 255) / 256), (unsigned)a.n_batch);
    hipError_t e;
    if (fp64) {
        double *in = (double *)ga, *out = (double *)gb;
        hipLaunchKernelGGL(nodewin_init_kernel<double>, g, dim3(256), 0, st, a, in);
        e = hipGetLastError();
        for (int k = 0; k < n_sub && e == hipSuccess; ++k) {
            hipLaunchKernelGGL(nodewin_substep_kernel<double>, g, dim3(256), 0, st, a, (const double *)in, out);
            e = hipGetLastError();
            double *t = in; in = out; out = t;
        }
        if (e == hipSuccess)
            hipLaunchKernelGGL(nodewin_bin_kernel<double>, dim3((unsigned)a.n_batch), dim3(NODEWIN_BIN_NT), 0, st, a,
                               (const double *)in, count, S);
    } else {
        float *in = (float *)ga, *out = (float *)gb;
        hipLaunchKernelGGL(nodewin_init_kernel<float>, g, dim3(256), 0, st, a, in);
        e = hipGetLastError();
        for (int k = 0; k < n_sub && e == hipSuccess; ++k) {
            hipLaunchKernelGGL(nodewin_substep_kernel<float>, g, dim3(256), 0, st, a, (const float *)in, out);
            e = hipGetLastError();
            float *t = in; in = out; out = t;
        }
        if (e == hipSuccess)
            hipLaunchKernelGGL(nodewin_bin_kernel<float>, dim3((unsigned)a.n_batch), dim3(NODEWIN_BIN_NT), 0, st, a,
                               (const float *)in, count, S);
    }
    return e == hipSuccess ? hipGetLastError() : e;
}

hipError_t launch_coarse_fill_reservoir(const int *node, int64_t n, double v, double *c, hipStream_t st)
{
    hipLaunchKernelGGL(coarse_fill_reservoir_kernel, dim3(grid_for(n)), dim3(256), 0, st, node, n, v, c);
    return hipGetLastError();
}

template <typename T, bool SINK>
static hipError_t launch_bin_t(int r, const CoarseGenArgs &a, const T *G, int64_t src_base, int64_t n_src,
                               hipStream_t st)
{
    const int64_t nblk = n_src < 65536 * 16 ? n_src : 65536 * 16;
    if (nblk <= 0) return hipSuccess;
    const dim3 g((unsigned)nblk), b(BIN_NT);
    switch (r) {
    case 0: hipLaunchKernelGGL((coarse_bin_kernel<T, 0, SINK>), g, b, 0, st, a, G, src_base, n_src); break;
    case 1: hipLaunchKernelGGL((coarse_bin_kernel<T, 1, SINK>), g, b, 0, st, a, G, src_base, n_src); break;
    case 2: hipLaunchKernelGGL((coarse_bin_kernel<T, 2, SINK>), g, b, 0, st, a, G, src_base, n_src); break;
    case 3: hipLaunchKernelGGL((coarse_bin_kernel<T, 3, SINK>), g, b, 0, st, a, G, src_base, n_src); break;
    case 4: hipLaunchKernelGGL((coarse_bin_kernel<T, 4, SINK>), g, b, 0, st, a, G, src_base, n_src); break;
    case 5: hipLaunchKernelGGL((coarse_bin_kernel<T, 5, SINK>), g, b, 0, st, a, G, src_base, n_src); break;
    case 6: hipLaunchKernelGGL((coarse_bin_kernel<T, 6, SINK>), g, b, 0, st, a, G, src_base, n_src); break;
    case 7: hipLaunchKernelGGL((coarse_bin_kernel<T, 7, SINK>), g, b, 0, st, a, G, src_base, n_src); break;
    case 8: hipLaunchKernelGGL((coarse_bin_kernel<T, 8, SINK>), g, b, 0, st, a, G, src_base, n_src); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_coarse_bin(int fp64, int sink, int r, const CoarseGenArgs &a, const void *G, int64_t src_base,
                             int64_t n_src, hipStream_t st)
{
    if (fp64)
        return sink ? launch_bin_t<double, true>(r, a, (const double *)G, src_base, n_src, st)
                    : launch_bin_t<double, false>(r, a, (const double *)G, src_base, n_src, st);
    return sink ? launch_bin_t<float, true>(r, a, (const float *)G, src_base, n_src, st)
                : launch_bin_t<float, false>(r, a, (const float *)G, src_base, n_src, st);
}

hipError_t launch_coarse_finalize(int prec, const double *S, const double *count, int64_t n_nodes, int nb, int ncx,
                                  int ncy, int ncz, const int *slot, int64_t plane, void *P, hipStream_t st)
{
    const unsigned g = grid_for((int64_t)nb * n_nodes);
    switch (prec) {
    case M_FP64:
        hipLaunchKernelGGL(coarse_finalize_kernel<double>, dim3(g), dim3(256), 0, st, S, count, n_nodes, nb, ncx,
                           ncy, ncz, slot, plane, (double *)P);
        break;
    case M_FP32:
        hipLaunchKernelGGL(coarse_finalize_kernel<float>, dim3(g), dim3(256), 0, st, S, count, n_nodes, nb, ncx,
                           ncy, ncz, slot, plane, (float *)P);
        break;
    case M_F16BANK:
        hipLaunchKernelGGL(coarse_finalize_kernel<_Float16>, dim3(g), dim3(256), 0, st, S, count, n_nodes, nb, ncx,
                           ncy, ncz, slot, plane, (_Float16 *)P);
        break;
    case M_BF16BANK:
        hipLaunchKernelGGL(coarse_finalize_kernel<__bf16>, dim3(g), dim3(256), 0, st, S, count, n_nodes, nb, ncx,
                           ncy, ncz, slot, plane, (__bf16 *)P);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename TC>
static hipError_t coarse_map_t(const double *c, const int *node, const double *count, int nx, int ny, int nz, int B,
                               int ncx, int ncy, int ncz, int K, TC *cpad, hipStream_t st, int dense,
                               const int *used, int64_t n_used)
{
    if (dense && B <= 256) {
        if (ncx <= 0 || ncy <= 0 || ncz <= 0) return hipSuccess;
        hipLaunchKernelGGL(coarse_map_rows_kernel<TC>, dim3((unsigned)ncy, (unsigned)ncz), dim3(256), 0, st, c, node,
                           count, nx, ny, nz, B, ncx, ncy, coarse_pad(ncx, ncy, ncz, K), cpad);
        return hipGetLastError();
    }
    const int64_t waves = used ? n_used : (int64_t)ncx * ncy * ncz;
    const int64_t g = (waves + MAP_NT / 64 - 1) / (MAP_NT / 64);
    if (g <= 0) return hipSuccess;
    hipLaunchKernelGGL(coarse_map_kernel<TC>, dim3((unsigned)g), dim3(MAP_NT), 0, st, c, node, count, nx, ny, nz, B,
                       ncx, ncy, ncz, coarse_pad(ncx, ncy, ncz, K), cpad, used, n_used);
    return hipGetLastError();
}

hipError_t launch_coarse_map(const double *c, const int *node, const double *count, int nx, int ny, int nz, int B,
                             int ncx, int ncy, int ncz, int K, double *cpad, hipStream_t st, int dense,
                             const int *used, int64_t n_used)
{
    return coarse_map_t<double>(c, node, count, nx, ny, nz, B, ncx, ncy, ncz, K, cpad, st, dense, used, n_used);
}

hipError_t launch_coarse_map_arith(int arith, const double *c, const int *node, const double *count, int nx, int ny,
                                   int nz, int B, int ncx, int ncy, int ncz, int K, void *cpad, hipStream_t st,
                                   int dense, const int *used, int64_t n_used)
{
    switch (arith) {
    case COARSE_FP64:
        return coarse_map_t<double>(c, node, count, nx, ny, nz, B, ncx, ncy, ncz, K, (double *)cpad, st, dense, used,
                                    n_used);
    case COARSE_FP32:
        return coarse_map_t<float>(c, node, count, nx, ny, nz, B, ncx, ncy, ncz, K, (float *)cpad, st, dense, used,
                                   n_used);
    case COARSE_MIXED:
    case COARSE_FP16:
        return coarse_map_t<_Float16>(c, node, count, nx, ny, nz, B, ncx, ncy, ncz, K, (_Float16 *)cpad, st, dense,
                                      used, n_used);
    default: return hipErrorInvalidValue;
    }
}

int coarse_apply_zb(int prec) { return 16 / (prec == M_FP64 ? 8 : (prec == M_FP32 ? 4 : 2)); }

// Offset pairs per range and the number of ranges: enough waves in flight to
// cover the chip (~8 per CU), whole pairs per range.
static void apply_ranges(int K, int64_t n_chunks, int *pairs_per_range, int *n_split)
{
    const int n_pairs = (2 * K + 1) * (2 * K + 1);
    const int64_t groups = (n_chunks + 63) / 64;
    int64_t want = groups > 0 ? (2048 + groups - 1) / groups : 1;
    if (want > n_pairs) want = n_pairs;
    if (want < 1) want = 1;
    *pairs_per_range = (int)((n_pairs + want - 1) / want);
    *n_split = (n_pairs + *pairs_per_range - 1) / *pairs_per_range;
}

int coarse_apply_split(int K, int64_t n_chunks)
{
    if (K < COARSE_CHUNK_MIN_K) return 1;
    int ppr = 0, ns = 0;
    apply_ranges(K, n_chunks, &ppr, &ns);
    return ns;
}

int64_t coarse_apply_part_elems(int prec, int K, int64_t n_chunks)
{
    if (K < COARSE_CHUNK_MIN_K) return 0;
    const int64_t pad = (n_chunks + 63) / 64 * 64;
    return (int64_t)coarse_apply_split(K, n_chunks) * pad * coarse_apply_zb(prec);
}

// Arguments of either product shape.
struct ApplyCall {
    const void *P;
    const void *cpad;
    int ncx, ncy, ncz;
    const double *pbc_pad;
    double c_ff;
    const double *cff_dev, *count;
    double *cnew;
    const int *list;
    int64_t n_list;
    int ppr, ns;
    double *part;
};

template <typename T, int KW, int A>
static hipError_t apply_kw(const ApplyCall &a, hipStream_t st)
{
    using TC = typename CoarseArith<A>::C;
    constexpr int K = (KW - 1) / 2;
    if constexpr (K < COARSE_CHUNK_MIN_K) {
        constexpr int nw = KW < APPLY_MAX_WAVES ? KW : APPLY_MAX_WAVES;
        hipLaunchKernelGGL((coarse_apply_rows_kernel<T, KW, A>), dim3((unsigned)a.n_list), dim3(64 * nw), 0, st,
                           (const T *)a.P, (const TC *)a.cpad, a.ncx, a.ncy, a.ncz, a.pbc_pad, a.c_ff, a.cff_dev,
                           a.count, a.cnew, a.list);
    } else {
        const int64_t pad = (a.n_list + 63) / 64 * 64;
        const int64_t waves = pad / 64 * a.ns;
        const int64_t g = (waves + APPLY_NT / 64 - 1) / (APPLY_NT / 64);
        hipLaunchKernelGGL((coarse_apply_chunks_kernel<T, KW, A>), dim3((unsigned)g), dim3(APPLY_NT), 0, st,
                           (const T *)a.P, (const TC *)a.cpad, a.ncx, a.ncy, a.ncz, a.list, a.n_list, pad, a.ppr,
                           a.ns, a.part);
    }
    return hipGetLastError();
}

template <typename T, int A>
static hipError_t apply_t(int K, const ApplyCall &a, hipStream_t st)
{
#define FDIRW_APPLY_CASE(k)                                                                                        \
    case k: return apply_kw<T, 2 * k + 1, A>(a, st);
    switch (K) {
        FDIRW_APPLY_CASE(0)
        FDIRW_APPLY_CASE(1)
        FDIRW_APPLY_CASE(2)
        FDIRW_APPLY_CASE(3)
        FDIRW_APPLY_CASE(4)
        FDIRW_APPLY_CASE(5)
        FDIRW_APPLY_CASE(6)
        FDIRW_APPLY_CASE(7)
        FDIRW_APPLY_CASE(8)
    default: return hipErrorInvalidValue;
    }
#undef FDIRW_APPLY_CASE
}

template <int A>
static hipError_t launch_sum(const ApplyCall &a, int zb, int K, hipStream_t st)
{
    const int64_t nt = a.n_list * zb * SUM_TP;
    hipLaunchKernelGGL(coarse_apply_sum_kernel<A>, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, st, a.part,
                       a.list, a.n_list, (a.n_list + 63) / 64 * 64, a.ns, zb, a.ncx, a.ncy, a.ncz, K, a.count,
                       a.pbc_pad, a.c_ff, a.cff_dev, a.cnew);
    return hipGetLastError();
}

bool coarse_arith_supported(int arith, int prec)
{
    switch (arith) {
    case COARSE_FP64: return prec == M_FP64 || prec == M_FP32 || prec == M_F16BANK || prec == M_BF16BANK;
    case COARSE_FP32: return prec == M_FP32;
    case COARSE_MIXED:
    case COARSE_FP16: return prec == M_F16BANK;
    default: return false;
    }
}

size_t coarse_c_bytes(int arith)
{
    return arith == COARSE_FP64 ? 8 : (arith == COARSE_FP32 ? 4 : 2);
}

hipError_t launch_coarse_apply_arith(int arith, int prec, const void *P, const void *cpad, int ncx, int ncy, int ncz,
                                     int K, const double *pbc_pad, double c_ff, const double *count, double *cnew,
                                     hipStream_t st, const double *cff_dev, const int *list, int64_t n_list,
                                     int n_split, double *part)
{
    if (n_list <= 0) return hipSuccess;
    if (K < 0 || K > 8 || !coarse_arith_supported(arith, prec)) return hipErrorInvalidValue;
    ApplyCall a{P, cpad, ncx, ncy, ncz, pbc_pad, c_ff, cff_dev, count, cnew, list, n_list, 0, 1, part};
    if (K >= COARSE_CHUNK_MIN_K) {
        apply_ranges(K, n_list, &a.ppr, &a.ns);
        if (a.ns != n_split) return hipErrorInvalidValue;         // part was sized for another split
    }
    hipError_t e;
    switch (arith) {
    case COARSE_FP64:
        switch (prec) {
        case M_FP64: e = apply_t<double, COARSE_FP64>(K, a, st); break;
        case M_FP32: e = apply_t<float, COARSE_FP64>(K, a, st); break;
        case M_F16BANK: e = apply_t<_Float16, COARSE_FP64>(K, a, st); break;
        default: e = apply_t<__bf16, COARSE_FP64>(K, a, st); break;
        }
        break;
    case COARSE_FP32: e = apply_t<float, COARSE_FP32>(K, a, st); break;
    case COARSE_MIXED: e = apply_t<_Float16, COARSE_MIXED>(K, a, st); break;
    default: e = apply_t<_Float16, COARSE_FP16>(K, a, st); break;
    }
    if (e != hipSuccess || K < COARSE_CHUNK_MIN_K) return e;
    const int zb = coarse_apply_zb(prec);
    switch (arith) {
    case COARSE_FP64: return launch_sum<COARSE_FP64>(a, zb, K, st);
    case COARSE_FP32: return launch_sum<COARSE_FP32>(a, zb, K, st);
    case COARSE_MIXED: return launch_sum<COARSE_MIXED>(a, zb, K, st);
    default: return launch_sum<COARSE_FP16>(a, zb, K, st);
    }
}

hipError_t launch_coarse_apply(int prec, const void *P, const double *cpad, int ncx, int ncy, int ncz, int K,
                               const double *pbc_pad, double c_ff, const double *count, double *cnew,
                               hipStream_t st, const double *cff_dev, const int *list, int64_t n_list,
                               int n_split, double *part)
{
    return launch_coarse_apply_arith(COARSE_FP64, prec, P, cpad, ncx, ncy, ncz, K, pbc_pad, c_ff, count, cnew, st,
                                     cff_dev, list, n_list, n_split, part);
}

hipError_t launch_coarse_remap(const double *c_in, const int *node, const double *cnew, int64_t n, double *c_out,
                               hipStream_t st)
{
    hipLaunchKernelGGL(coarse_remap_kernel, dim3(grid_for(n)), dim3(256), 0, st, c_in, node, cnew, n, c_out);
    return hipGetLastError();
}

}  // namespace fdirw
