// fdirw_kernels.hip -- HIP kernels of the FDiRW fast-diffusion step (gfx950).
//
//   coef_validate_kernel   label range check + presence mask (for Dmax)
//   coef_kernel            FP64 face coefficients (+ FP32 copy)
//   window_kernel          window kernels of a source list
//   line_kernel            fused generate + superpose
//   bank_gather_kernel     superposition from a stored kernel bank (row form)
//   fill / field-sum       global mass balance and output clearing
//
// The superposition (Eq. 8 of arXiv 2408.11376 in its column form) is
// organised so that a workgroup walks a line of sources along z and
// accumulates c(s) * G_s into an FP64 ring of W planes; the plane that no later
// source of the line can reach is flushed with one FP64 atomic per window
// column, i.e. W^2 atomics per source instead of W^3.
#include "fdirw_device.h"
#include "fdirw_launch.h"

namespace fdirw {

// Elements of one offset plane of the kernel bank, whose cells are ordered
// [z / zb][y][x][z % zb] (zb z-consecutive values form one 16-byte group).
__host__ __device__ inline int64_t bank_plane_elems(int nx, int ny, int nz, int zb)
{
    return (int64_t)((nz + zb - 1) / zb) * ny * nx * zb;
}

// ----------------------------------------------------------------- coefficients

__global__ void coef_validate_kernel(const uint8_t *__restrict__ label, int64_t n, int n_phase,
                                     unsigned *__restrict__ out /* [8] presence bits, [8] bad flag */)
{
    __shared__ unsigned present[8];
    __shared__ unsigned bad;
    if (threadIdx.x < 8) present[threadIdx.x] = 0u;
    if (threadIdx.x == 0) bad = 0u;
    __syncthreads();
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const unsigned l = label[i];
        if ((int)l >= n_phase) atomicOr(&bad, 1u);
        atomicOr(&present[l >> 5], 1u << (l & 31));
    }
    __syncthreads();
    if (threadIdx.x < 8 && present[threadIdx.x]) atomicOr(&out[threadIdx.x], present[threadIdx.x]);
    if (threadIdx.x == 0 && bad) atomicOr(&out[8], 1u);
}

// Face coefficient, evaluated in exactly this order with no contraction:
// num = (2 Da) Db, den = Da + Db, Df = num / den, lam = (Df dt) / (h h).
__device__ __forceinline__ double face_lambda(double da, double db, double dt, double h)
{
#pragma clang fp contract(off)
    if (!(da > 0.0 && db > 0.0)) return 0.0;
    const double num = (2.0 * da) * db;
    const double den = da + db;
    const double df = num / den;
    return (df * dt) / (h * h);
}

__global__ void coef_kernel(const uint8_t *__restrict__ label, int nx, int ny, int nz,
                            CoefTable tab, double dt, double h,
                            double *__restrict__ lam64, float *__restrict__ lam32)
{
    const int64_t n = (int64_t)nx * ny * nz;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(i % nx);
        const int y = (int)((i / nx) % ny);
        const int z = (int)(i / ((int64_t)nx * ny));
        const double d0 = tab.d[label[i]];
        const double vx = (x + 1 < nx) ? face_lambda(d0, tab.d[label[i + 1]], dt, h) : 0.0;
        const double vy = (y + 1 < ny) ? face_lambda(d0, tab.d[label[i + nx]], dt, h) : 0.0;
        const double vz = (z + 1 < nz) ? face_lambda(d0, tab.d[label[i + (int64_t)nx * ny]], dt, h) : 0.0;
        if (lam64) { lam64[i] = vx; lam64[n + i] = vy; lam64[2 * n + i] = vz; }
        if (lam32) { lam32[i] = (float)vx; lam32[n + i] = (float)vy; lam32[2 * n + i] = (float)vz; }
    }
}

// Face coefficient of every ordered phase pair: tab[a * n_phase + b] =
// face_lambda(D_a, D_b) (the value coef_kernel gives a face whose lower cell
// has phase a and upper cell phase b), in FP64 or rounded to FP32.
__global__ void pair_table_kernel(CoefTable tab, int n_phase, double dt, double h, double *__restrict__ t64,
                                  float *__restrict__ t32)
{
    const int n = n_phase * n_phase;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const double v = face_lambda(tab.d[i / n_phase], tab.d[i % n_phase], dt, h);
        if (t64) t64[i] = v;
        if (t32) t32[i] = (float)v;
    }
}

// ----------------------------------------------------------------- helpers

__global__ void fill_kernel(double *__restrict__ p, int64_t n, double v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void fill_u32_kernel(unsigned *__restrict__ p, int64_t n, unsigned v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Two-sum of (s, c) pairs: exact sum of the leading parts plus the carries.
__device__ __forceinline__ void two_sum_add(double &s, double &c, double s2, double c2)
{
#pragma clang fp contract(off)
    const double t = s + s2;
    const double bp = t - s;
    const double err = (s - (t - bp)) + (s2 - bp);
    s = t;
    c = c + c2 + err;
}

// Field sum, level 1: each thread a Neumaier sum over a fixed strided subset,
// then a fixed-shape tree inside the block; out: (sum, carry) per block.
__global__ void field_sum_partial_kernel(const double *__restrict__ v, int64_t n, double *__restrict__ out)
{
#pragma clang fp contract(off)
    __shared__ double ss[256], cc[256];
    double s = 0.0, c = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double x = v[i];
        const double t = s + x;
        if (fabs(s) >= fabs(x)) c += (s - t) + x;
        else                    c += (x - t) + s;
        s = t;
    }
    ss[threadIdx.x] = s;
    cc[threadIdx.x] = c;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) {
            double a = ss[threadIdx.x], b = cc[threadIdx.x];
            two_sum_add(a, b, ss[threadIdx.x + w], cc[threadIdx.x + w]);
            ss[threadIdx.x] = a;
            cc[threadIdx.x] = b;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) { out[2 * blockIdx.x] = ss[0]; out[2 * blockIdx.x + 1] = cc[0]; }
}

// Level 2: one thread combines the block partials in block order.
__global__ void field_sum_final_kernel(const double *__restrict__ part, int nblk, double *__restrict__ out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0, c = 0.0;
    for (int b = 0; b < nblk; ++b) two_sum_add(s, c, part[2 * b], part[2 * b + 1]);
    out[0] = s + c;
}

// Min / max of kernel masses.  PAIRS: v holds n (min, max) pairs (one per
// workgroup); otherwise v holds n scalars.
template <bool PAIRS>
__global__ void minmax_kernel(const double *__restrict__ v, int64_t n, double *__restrict__ out)
{
    __shared__ double mn[256], mx[256];
    double a = INFINITY, b = -INFINITY;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        a = fmin(a, PAIRS ? v[2 * i] : v[i]);
        b = fmax(b, PAIRS ? v[2 * i + 1] : v[i]);
    }
    mn[threadIdx.x] = a;
    mx[threadIdx.x] = b;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) {
            mn[threadIdx.x] = fmin(mn[threadIdx.x], mn[threadIdx.x + w]);
            mx[threadIdx.x] = fmax(mx[threadIdx.x], mx[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) { out[2 * blockIdx.x] = mn[0]; out[2 * blockIdx.x + 1] = mx[0]; }
}

__global__ void src_check_kernel(const int64_t *__restrict__ src, int64_t n_src, int64_t n,
                                 unsigned *__restrict__ bad)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_src;
         i += (int64_t)gridDim.x * blockDim.x)
        if (src[i] < 0 || src[i] >= n) atomicOr(bad, 1u);
}

// ----------------------------------------------------------------- launch geometry

template <int M, int R>
__device__ __forceinline__ void zero_exchange(typename Geo<M, R>::E *xb)
{
    using E = typename Geo<M, R>::E;
    for (int i = threadIdx.x; i < 2 * Geo<M, R>::XLEN; i += blockDim.x) xb[i] = (E)0.0f;
}

// ----------------------------------------------------------------- window kernels

template <int M, int R>
__global__ void __launch_bounds__((Geo<M, R>::NT)) __attribute__((amdgpu_waves_per_eu(Geo<M, R>::MINW)))
window_kernel(WindowArgs a)
{
    using G_ = Geo<M, R>;
    using T = typename G_::T;
    using S = typename G_::S;
    using E = typename G_::E;
    constexpr int L = G_::L0, W2 = G_::W2, W3 = G_::W3;
    __shared__ __align__(16) E xb[2 * G_::XLEN];
    __shared__ double red[G_::NWAVE];

    const Place p = make_place<M, R>(threadIdx.x);
    zero_exchange<M, R>(xb);
    __syncthreads();

    const S *lx = (const S *)a.lx, *ly = lx + a.n, *lz = ly + a.n;
    for (int64_t q = blockIdx.x; q < a.n_src; q += gridDim.x) {
        const int64_t s = a.src ? a.src[q] : q;
        const int sx = (int)(s % a.nx), sy = (int)((s / a.nx) % a.ny), sz = (int)(s / ((int64_t)a.nx * a.ny));
        Seg<M, R> c;
        load_segment<M, R>(c, lx, ly, lz, a.nx, a.ny, a.nz, sx, sy, sz, p);
        compute_diag<T::x32, M, R>(c);
        S G[L];
        init_delta<M, R>(G, p);
        run_substeps<M, R>(G, c, xb, p, a.n_sub);
        const double m = finish_kernel<M, R>(G, red, p);
        if (threadIdx.x == 0 && a.mass) a.mass[q] = m;
        if (p.act) {
            const bool norm = T::renorm && !T::bank && a.normalize;
            const double inv = norm ? 1.0 / m : 1.0;
            const int X = sx - R + p.cx, Y = sy - R + p.cy;
            const bool inxy = X >= 0 && X < a.nx && Y >= 0 && Y < a.ny;
            // z cells per 16-byte group of the stored element type
            const int zb = M == M_FP64 ? 2 : (T::bank && a.out_lp ? 8 : 4);
#pragma unroll
            for (int k = 0; k < L; ++k) {
                if (k >= p.len) continue;
                int64_t o;
                if (a.offset_major) {
                    // bank layout [offset][z / zb][y][x][z % zb]: the value at
                    // cell x = s + o is P[o][x]; cells outside the domain are
                    // walls (0) and are not stored
                    const int Z = sz - R + p.j0 + k;
                    if (!inxy || Z < 0 || Z >= a.nz) continue;
                    o = (int64_t)((p.j0 + k) * W2 + p.col) * bank_plane_elems(a.nx, a.ny, a.nz, zb) +
                        (((int64_t)(Z / zb) * a.ny + Y) * a.nx + X) * zb + Z % zb;
                } else {
                    o = q * (int64_t)W3 + (int64_t)(p.j0 + k) * W2 + p.col;
                }
                if constexpr (M == M_FP64) {
                    ((double *)a.G)[o] = G[k];
                } else if constexpr (T::bank) {
                    if (a.out_lp) ((typename T::B *)a.G)[o] = (typename T::B)G[k];
                    else ((float *)a.G)[o] = G[k];
                } else {
                    ((float *)a.G)[o] = norm ? (float)((double)G[k] * inv) : G[k];
                }
            }
        }
        __syncthreads();      // exchange buffers are reused by the next source
    }
}

// ----------------------------------------------------------------- fused step

// Adds the completed value v of window column col, plane Z (0 <= Z < nz) of a
// line to the output: an FP64 atomic into c_out, or in the deterministic form
// a plain store of its own partial slot (zeros too, so that every slot the
// reduction reads is written).
__device__ __forceinline__ void flush_column(const LineArgs &a, double v, bool inxy, int X, int Y, int Z, int col)
{
    if (!inxy) return;
    const int64_t nxy = (int64_t)a.nx * a.ny;
    if (a.part) {
        a.part[((int64_t)col * a.part_planes + (Z - a.part_z0)) * nxy + (int64_t)Y * a.nx + X] = v;
    } else if (v != 0.0) {
        unsafeAtomicAdd(&a.c_out[(int64_t)Z * nxy + (int64_t)Y * a.nx + X], v);
    }
}

// Second pass of the deterministic superposition: one thread per output cell
// of planes [z_lo, z_hi) adds the partials of the W^2 window columns (cy, cx)
// whose source line (x + R - cx, y + R - cy) lies in the domain, cy then cx
// ascending, and adds that sum to c_out.
template <int R>
__global__ void line_reduce_kernel(LineArgs a, int z_lo, int z_hi)
{
    constexpr int W = 2 * R + 1;
    const int64_t nxy = (int64_t)a.nx * a.ny;
    const int64_t total = (int64_t)(z_hi - z_lo) * nxy;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int Z = z_lo + (int)(i / nxy);
        const int64_t cell = i - (int64_t)(Z - z_lo) * nxy;
        const int Y = (int)(cell / a.nx), X = (int)(cell - (int64_t)Y * a.nx);
        const double *p = a.part + (int64_t)(Z - a.part_z0) * nxy + cell;
        const int64_t colstride = (int64_t)a.part_planes * nxy;
        double s = 0.0;
        for (int cy = 0; cy < W; ++cy) {
            const int sy = Y + R - cy;
            if (sy < 0 || sy >= a.ny) continue;
            for (int cx = 0; cx < W; ++cx) {
                const int sx = X + R - cx;
                if (sx < 0 || sx >= a.nx) continue;
                s += p[(int64_t)(cy * W + cx) * colstride];
            }
        }
        a.c_out[(int64_t)Z * nxy + cell] += s;
    }
}

// One workgroup walks the sources (sx, sy, z0..z1-1).  c(s) * G_s is
// accumulated in FP64 into an LDS ring of W planes x W^2 columns indexed by
// global plane z mod W (touched once per source, so it costs no sub-step
// bandwidth and keeps the register file for the sub-step loop).  After source
// sz the plane z = sz - R can receive nothing more from this line: it is added
// to c_out with one atomic per window column and cleared.
template <int M, int R, bool LAB = false>
__global__ void __launch_bounds__((Geo<M, R>::NT)) __attribute__((amdgpu_waves_per_eu(Geo<M, R>::MINW)))
line_kernel(LineArgs a)
{
    using G_ = Geo<M, R>;
    using T = typename G_::T;
    using S = typename G_::S;
    using E = typename G_::E;
    constexpr int L = G_::L0, W = G_::W, W2 = G_::W2;
    __shared__ __align__(16) E xb[2 * G_::XLEN];
    __shared__ double red[G_::NWAVE];
    __shared__ double ring[W * W2];

    const Place p = make_place<M, R>(threadIdx.x);
    zero_exchange<M, R>(xb);

    const int b = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    for (int i = threadIdx.x; i < W * W2; i += blockDim.x) ring[i] = 0.0;
    __syncthreads();

    const int line = b / a.n_seg, sgi = b - line * a.n_seg;
    const int sy = line / a.nx, sx = line - sy * a.nx;
    const int z0 = a.z_begin + sgi * a.seg_len;
    const int z1 = min(a.z_end, z0 + a.seg_len);
    if (z0 >= z1) return;                                   // uniform per block
    const int X = sx - R + p.cx, Y = sy - R + p.cy;
    const bool inxy = p.act && X >= 0 && X < a.nx && Y >= 0 && Y < a.ny;
    const S *lx = (const S *)a.lx, *ly = lx + a.n, *lz = ly + a.n;

    double kmin = INFINITY, kmax = -INFINITY;
    int used = 0;
    for (int sz = z0; sz < z1; ++sz) {
        const double cs = a.c_in[((int64_t)sz * a.ny + sy) * a.nx + sx];
        if (cs != 0.0) {                                    // uniform per block
            ++used;
            Seg<M, R> c;
            if constexpr (LAB) {
                const FaceLabels<S> f{a.label, (const S *)a.lam_tab, a.n_phase, a.nx, a.ny, a.nz};
                load_segment_faces<M, R>(c, f, a.nx, a.ny, a.nz, sx, sy, sz, p);
            } else {
                load_segment<M, R>(c, lx, ly, lz, a.nx, a.ny, a.nz, sx, sy, sz, p);
            }
            compute_diag<T::x32, M, R>(c);
            S G[L];
            init_delta<M, R>(G, p);
            run_substeps<M, R>(G, c, xb, p, a.n_sub);
            const double m = finish_kernel<M, R>(G, red, p);
            kmin = fmin(kmin, m);
            kmax = fmax(kmax, m);
            const double scale = T::renorm ? cs / m : cs;
            if (p.act) {
#pragma unroll
                for (int k = 0; k < L; ++k) {
                    if (k < p.len) {
                        double &r = ring[((sz - R + p.j0 + k + W) % W) * W2 + p.col];
                        r = __builtin_fma(scale, (double)G[k], r);
                    }
                }
            }
        }
        __syncthreads();                                    // ring updates visible to the block
        // the lowest plane of this window (z = sz - R) is complete for the line
        if (p.act && p.seg == 0) {
            const int Z = sz - R;
            double &r = ring[((Z + W) % W) * W2 + p.col];
            if (Z >= 0) flush_column(a, r, inxy, X, Y, Z, p.col);
            r = 0.0;
        }
    }
    __syncthreads();
    if (p.act && p.seg == 0) {
        for (int Z = z1 - R; Z < z1 + R; ++Z) {
            if (Z < 0 || Z >= a.nz) continue;
            double &r = ring[((Z + W) % W) * W2 + p.col];
            flush_column(a, r, inxy, X, Y, Z, p.col);
            r = 0.0;
        }
    }
    if (threadIdx.x == 0) {
        if (a.wg_kmass) { a.wg_kmass[2 * b] = kmin; a.wg_kmass[2 * b + 1] = kmax; }
        if (a.n_used && used) atomicAdd(a.n_used, (unsigned long long)used);
    }
}

// ----------------------------------------------------------------- kernel bank

// Bank apply in the row (gather) form of Eq. 8: c'(x) = sum_o P[o][x] c^(x - o)
// with the bank stored offset-major, P[o][x] = G_{x-o}(o) for the W^3 window
// offsets o, and c^(s) = c(s) / m_s (renormalising modes) or c(s) (FP64).
// Within one offset plane the cells are ordered [z / ZB][y][x][z % ZB] with
// ZB = 16 bytes / element size, so that the ZB z-consecutive values a thread
// needs are one 16-byte load and a wave reads 1 KB contiguously.
// A workgroup owns a tile of 64 (x) x 1 (y) x TZ (z) output cells; every bank
// value is read once and every output written once: no atomics, a fixed
// summation order per cell.  c^ is read from a zero-padded copy (halo R on
// each side); per source row y - oy the block stages the (TZ + 2R) x (64 + 2R)
// slab of it in LDS, and each thread keeps the ZB + 2R values its z-run needs
// in registers across the W z-offsets.
template <typename B> struct BankZ {
    static constexpr int ZB = 16 / (int)sizeof(B);   // z cells per 16-byte group
};

#ifndef FDIRW_GATHER_TZW
#define FDIRW_GATHER_TZW 4                    // wave rows (z runs) per bank-apply tile
#endif

template <typename B, int R> struct Gath {
    static constexpr int W = 2 * R + 1;
    static constexpr int W2 = W * W;
    static constexpr int TX = 64;             // x cells per tile (one wave row)
    static constexpr int TZW = FDIRW_GATHER_TZW;
    static constexpr int ZB = BankZ<B>::ZB;   // z cells per thread
    static constexpr int TZ = TZW * ZB;       // z cells per tile
    static constexpr int SX = TX + 2 * R;     // slab extents
    static constexpr int SZ = TZ + 2 * R;
    static constexpr int NT = TX * TZW;
};

// c^ on the padded grid [nz + 2R][ny + 2R][nx + 2R]; the halo is 0.
__global__ void bank_scale_kernel(const double *__restrict__ c, const double *__restrict__ mass, int nx,
                                  int ny, int nz, int r, double *__restrict__ chat)
{
    const int px = nx + 2 * r, py = ny + 2 * r, pz = nz + 2 * r;
    const int64_t np = (int64_t)px * py * pz;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < np;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int X = (int)(i % px) - r;
        const int Y = (int)((i / px) % py) - r;
        const int Z = (int)(i / ((int64_t)px * py)) - r;
        double v = 0.0;
        if (X >= 0 && X < nx && Y >= 0 && Y < ny && Z >= 0 && Z < nz) {
            const int64_t s = ((int64_t)Z * ny + Y) * nx + X;
            v = mass ? c[s] / mass[s] : c[s];
        }
        chat[i] = v;
    }
}

// The ZB stored values of one 16-byte group, widened exactly to FP64.
template <typename B> __device__ __forceinline__ void widen_group(const uint4 &u, double (&v)[BankZ<B>::ZB])
{
    constexpr int ZB = BankZ<B>::ZB;
    B e[ZB];
    __builtin_memcpy(e, &u, 16);
#pragma unroll
    for (int k = 0; k < ZB; ++k) v[k] = (double)(float)e[k];
}
template <> __device__ __forceinline__ void widen_group<double>(const uint4 &u, double (&v)[2])
{
    __builtin_memcpy(v, &u, 16);
}

template <typename B, int R>
__global__ void __launch_bounds__((Gath<B, R>::NT)) bank_gather_kernel(BankArgs a)
{
    using G_ = Gath<B, R>;
    constexpr int W = G_::W, W2 = G_::W2, ZB = G_::ZB, SX = G_::SX, SZ = G_::SZ, NT = G_::NT;
    __shared__ double slab[SZ * SX];
    const int tx = threadIdx.x % G_::TX, tz = threadIdx.x / G_::TX;
    const int x0 = blockIdx.x * G_::TX, y = blockIdx.y, z0 = blockIdx.z * G_::TZ;
    const int x = x0 + tx;
    const int zt = z0 + tz * ZB;                      // first output z of the thread (uniform per wave)
    const int px = a.nx + 2 * R, py = a.ny + 2 * R, pz = a.nz + 2 * R;
    const bool act = x < a.nx && zt < a.nz;
    // the thread's group in every offset plane, and the plane stride
    const int64_t grp = (((int64_t)(zt / ZB) * a.ny + y) * a.nx + x) * ZB;
    const int64_t plane = bank_plane_elems(a.nx, a.ny, a.nz, ZB);
    const B *P = (const B *)a.bank + grp;
    double acc[ZB];
#pragma unroll
    for (int k = 0; k < ZB; ++k) acc[k] = 0.0;

    for (int oy = -R; oy <= R; ++oy) {
        const int64_t row = (int64_t)(y - oy + R) * px;   // padded source row
        __syncthreads();                                  // the previous slab is consumed
        for (int i = threadIdx.x; i < SZ * SX; i += NT) {
            const int iz = i / SX, ix = i - iz * SX;
            const int zz = z0 + iz, xx = x0 + ix;         // padded source coordinates
            slab[i] = (zz < pz && xx < px) ? a.chat[(int64_t)zz * py * px + row + xx] : 0.0;
        }
        __syncthreads();
        if (!act) continue;
        for (int ox = -R; ox <= R; ++ox) {
            // source (z - oz, y - oy, x - ox): slab column tx - ox + R, slab row
            // tz*ZB + k - oz + R = tz*ZB + m with m = k - j + 2R, j = oz + R
            const int ix = tx - ox + R;
            double cc[ZB + 2 * R];
#pragma unroll
            for (int m = 0; m < ZB + 2 * R; ++m) cc[m] = slab[(tz * ZB + m) * SX + ix];
            const int64_t obase = (int64_t)(oy + R) * W + (ox + R);
            // all W groups of this (oy, ox) are requested before the first is
            // used, so that each wave keeps W x 1 KB of bank reads in flight
            uint4 raw[W];
#pragma unroll
            for (int j = 0; j < W; ++j) raw[j] = *(const uint4 *)(P + ((int64_t)j * W2 + obase) * plane);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int j = 0; j < W; ++j) {
                double g[ZB];
                widen_group<B>(raw[j], g);
#pragma unroll
                for (int k = 0; k < ZB; ++k) acc[k] = __builtin_fma(g[k], cc[k - j + 2 * R], acc[k]);
            }
        }
    }
    if (act) {
        const int64_t o0 = ((int64_t)zt * a.ny + y) * a.nx + x;
        const int64_t nxy = (int64_t)a.nx * a.ny;
#pragma unroll
        for (int k = 0; k < ZB; ++k)
            if (zt + k < a.nz) a.c_out[o0 + k * nxy] = acc[k];
    }
}

template <typename B, int R>
static hipError_t launch_gather_r(const BankArgs &a, hipStream_t st)
{
    using G_ = Gath<B, R>;
    const dim3 grid((unsigned)((a.nx + G_::TX - 1) / G_::TX), (unsigned)a.ny, (unsigned)((a.nz + G_::TZ - 1) / G_::TZ));
    hipLaunchKernelGGL((bank_gather_kernel<B, R>), grid, dim3(G_::NT), 0, st, a);
    return hipGetLastError();
}

template <typename B>
static hipError_t launch_gather_b(int r, const BankArgs &a, hipStream_t st)
{
    switch (r) {
    case 0: return launch_gather_r<B, 0>(a, st);
    case 1: return launch_gather_r<B, 1>(a, st);
    case 2: return launch_gather_r<B, 2>(a, st);
    case 3: return launch_gather_r<B, 3>(a, st);
    case 4: return launch_gather_r<B, 4>(a, st);
    case 5: return launch_gather_r<B, 5>(a, st);
    case 6: return launch_gather_r<B, 6>(a, st);
    case 7: return launch_gather_r<B, 7>(a, st);
    case 8: return launch_gather_r<B, 8>(a, st);
    default: return hipErrorInvalidValue;
    }
}

int64_t bank_chat_elems(int nx, int ny, int nz, int r)
{
    return (int64_t)(nx + 2 * r) * (ny + 2 * r) * (nz + 2 * r);
}

int64_t bank_elems(int nx, int ny, int nz, int r, int elem_bytes)
{
    const int64_t w = 2 * r + 1;
    return w * w * w * bank_plane_elems(nx, ny, nz, 16 / elem_bytes);
}

hipError_t launch_bank_apply(int prec, int r, const BankArgs &a, hipStream_t st)
{
    if (r < 0 || r > 8) return hipErrorInvalidValue;
    const int64_t np = bank_chat_elems(a.nx, a.ny, a.nz, r);
    const int64_t blocks = (np + 255) / 256 < 8192 ? (np + 255) / 256 : 8192;
    hipLaunchKernelGGL(bank_scale_kernel, dim3((unsigned)blocks), dim3(256), 0, st, a.c_in,
                       prec == M_FP64 ? nullptr : a.mass, a.nx, a.ny, a.nz, r, a.chat);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_bank_gather(prec, r, a, st);
}

hipError_t launch_bank_gather(int prec, int r, const BankArgs &a, hipStream_t st)
{
    if (r < 0 || r > 8) return hipErrorInvalidValue;
    switch (prec) {
    case M_FP64: return launch_gather_b<double>(r, a, st);
    case M_FP32: case M_F16X32: case M_BF16X32: case M_F16ST: case M_BF16ST:
        return launch_gather_b<float>(r, a, st);
    case M_F16BANK: return launch_gather_b<_Float16>(r, a, st);
    case M_BF16BANK: return launch_gather_b<__bf16>(r, a, st);
    default: return hipErrorInvalidValue;
    }
}


// ----------------------------------------------------------------- dispatch

template <int M, int R, bool LAB = false>
static hipError_t launch_line_mr(const LineArgs &a, hipStream_t st)
{
    const int64_t nblk = (int64_t)a.nx * a.ny * a.n_seg;
    hipLaunchKernelGGL((line_kernel<M, R, LAB>), dim3((unsigned)nblk), dim3(Geo<M, R>::NT), 0, st, a);
    return hipGetLastError();
}

template <int R>
static hipError_t launch_reduce_r(const LineArgs &a, int z_lo, int z_hi, hipStream_t st)
{
    const int64_t total = (int64_t)(z_hi - z_lo) * a.nx * a.ny;
    if (total <= 0) return hipSuccess;
    int64_t g = (total + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL((line_reduce_kernel<R>), dim3((unsigned)g), dim3(256), 0, st, a, z_lo, z_hi);
    return hipGetLastError();
}

hipError_t launch_line_reduce(int r, const LineArgs &a, int z_lo, int z_hi, hipStream_t st)
{
    switch (r) {
    case 0: return launch_reduce_r<0>(a, z_lo, z_hi, st);
    case 1: return launch_reduce_r<1>(a, z_lo, z_hi, st);
    case 2: return launch_reduce_r<2>(a, z_lo, z_hi, st);
    case 3: return launch_reduce_r<3>(a, z_lo, z_hi, st);
    case 4: return launch_reduce_r<4>(a, z_lo, z_hi, st);
    case 5: return launch_reduce_r<5>(a, z_lo, z_hi, st);
    case 6: return launch_reduce_r<6>(a, z_lo, z_hi, st);
    case 7: return launch_reduce_r<7>(a, z_lo, z_hi, st);
    case 8: return launch_reduce_r<8>(a, z_lo, z_hi, st);
    default: return hipErrorInvalidValue;
    }
}

template <int M, int R>
static hipError_t launch_window_mr(const WindowArgs &a, hipStream_t st)
{
    const int64_t nblk = a.n_src < 65536 * 16 ? a.n_src : 65536 * 16;
    if (nblk <= 0) return hipSuccess;
    hipLaunchKernelGGL((window_kernel<M, R>), dim3((unsigned)nblk), dim3(Geo<M, R>::NT), 0, st, a);
    return hipGetLastError();
}

template <int M, bool LAB = false>
static hipError_t launch_line_m(int r, const LineArgs &a, hipStream_t st)
{
    switch (r) {
    case 0: return launch_line_mr<M, 0, LAB>(a, st);
    case 1: return launch_line_mr<M, 1, LAB>(a, st);
    case 2: return launch_line_mr<M, 2, LAB>(a, st);
    case 3: return launch_line_mr<M, 3, LAB>(a, st);
    case 4: return launch_line_mr<M, 4, LAB>(a, st);
    case 5: return launch_line_mr<M, 5, LAB>(a, st);
    case 6: return launch_line_mr<M, 6, LAB>(a, st);
    case 7: return launch_line_mr<M, 7, LAB>(a, st);
    case 8: return launch_line_mr<M, 8, LAB>(a, st);
    default: return hipErrorInvalidValue;
    }
}

template <int M>
static hipError_t launch_window_m(int r, const WindowArgs &a, hipStream_t st)
{
    switch (r) {
    case 0: return launch_window_mr<M, 0>(a, st);
    case 1: return launch_window_mr<M, 1>(a, st);
    case 2: return launch_window_mr<M, 2>(a, st);
    case 3: return launch_window_mr<M, 3>(a, st);
    case 4: return launch_window_mr<M, 4>(a, st);
    case 5: return launch_window_mr<M, 5>(a, st);
    case 6: return launch_window_mr<M, 6>(a, st);
    case 7: return launch_window_mr<M, 7>(a, st);
    case 8: return launch_window_mr<M, 8>(a, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_line(int mode, int r, const LineArgs &a, hipStream_t st)
{
    switch (mode) {
    case M_FP64: return launch_line_m<M_FP64>(r, a, st);
    case M_FP32: return launch_line_m<M_FP32>(r, a, st);
    case M_F16X32: return launch_line_m<M_F16X32>(r, a, st);
    case M_BF16X32: return launch_line_m<M_BF16X32>(r, a, st);
    case M_F16ST: return launch_line_m<M_F16ST>(r, a, st);
    case M_BF16ST: return launch_line_m<M_BF16ST>(r, a, st);
    case M_F16BANK: return launch_line_m<M_F16BANK>(r, a, st);
    case M_BF16BANK: return launch_line_m<M_BF16BANK>(r, a, st);
    default: return hipErrorInvalidValue;
    }
}

// The fused step with the face coefficients looked up per phase pair
// (a.label, a.lam_tab, a.n_phase) instead of read from a.lx.
hipError_t launch_line_labels(int mode, int r, const LineArgs &a, hipStream_t st)
{
    switch (mode) {
    case M_FP64: return launch_line_m<M_FP64, true>(r, a, st);
    case M_FP32: return launch_line_m<M_FP32, true>(r, a, st);
    case M_F16X32: return launch_line_m<M_F16X32, true>(r, a, st);
    case M_BF16X32: return launch_line_m<M_BF16X32, true>(r, a, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_window(int mode, int r, const WindowArgs &a, hipStream_t st)
{
    switch (mode) {
    case M_FP64: return launch_window_m<M_FP64>(r, a, st);
    case M_FP32: return launch_window_m<M_FP32>(r, a, st);
    case M_F16X32: return launch_window_m<M_F16X32>(r, a, st);
    case M_BF16X32: return launch_window_m<M_BF16X32>(r, a, st);
    case M_F16ST: return launch_window_m<M_F16ST>(r, a, st);
    case M_BF16ST: return launch_window_m<M_BF16ST>(r, a, st);
    case M_F16BANK: return launch_window_m<M_F16BANK>(r, a, st);
    case M_BF16BANK: return launch_window_m<M_BF16BANK>(r, a, st);
    default: return hipErrorInvalidValue;
    }
}

static inline unsigned grid_for(int64_t n, int block)
{
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > 8192) g = 8192;
    return (unsigned)g;
}

hipError_t launch_validate(const uint8_t *label, int64_t n, int n_phase, unsigned *out, hipStream_t st)
{
    hipLaunchKernelGGL(fill_u32_kernel, dim3(1), dim3(64), 0, st, out, (int64_t)9, 0u);
    hipLaunchKernelGGL(coef_validate_kernel, dim3(grid_for(n, 256)), dim3(256), 0, st, label, n, n_phase, out);
    return hipGetLastError();
}

hipError_t launch_coef(const uint8_t *label, int nx, int ny, int nz, const CoefTable &tab,
                       double dt, double h, double *lam64, float *lam32, hipStream_t st)
{
    const int64_t n = (int64_t)nx * ny * nz;
    hipLaunchKernelGGL(coef_kernel, dim3(grid_for(n, 256)), dim3(256), 0, st, label, nx, ny, nz, tab, dt, h, lam64, lam32);
    return hipGetLastError();
}

hipError_t launch_pair_table(const CoefTable &tab, int n_phase, double dt, double h, double *t64, float *t32,
                             hipStream_t st)
{
    hipLaunchKernelGGL(pair_table_kernel, dim3(grid_for((int64_t)n_phase * n_phase, 256)), dim3(256), 0, st, tab,
                       n_phase, dt, h, t64, t32);
    return hipGetLastError();
}

hipError_t launch_fill(double *p, int64_t n, double v, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_kernel, dim3(grid_for(n, 256)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_u32(unsigned *p, int64_t n, unsigned v, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u32_kernel, dim3(grid_for(n, 256)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

int field_sum_blocks(int64_t n)
{
    int64_t g = (n + 256 * 8 - 1) / (256 * 8);
    if (g < 1) g = 1;
    if (g > 1024) g = 1024;
    return (int)g;
}

hipError_t launch_field_sum(const double *v, int64_t n, double *part, double *out, hipStream_t st)
{
    const int nblk = field_sum_blocks(n);
    hipLaunchKernelGGL(field_sum_partial_kernel, dim3(nblk), dim3(256), 0, st, v, n, part);
    hipLaunchKernelGGL(field_sum_final_kernel, dim3(1), dim3(64), 0, st, part, nblk, out);
    return hipGetLastError();
}

hipError_t launch_minmax(const double *v, int64_t n, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(minmax_kernel<true>, dim3(1), dim3(256), 0, st, v, n, out);
    return hipGetLastError();
}

// Scalars: with part (room for 2 x 256 doubles) and many values, 256 blocks
// write (min, max) pairs that one block then reduces.
hipError_t launch_minmax_scalar(const double *v, int64_t n, double *part, double *out, hipStream_t st)
{
    if (part && n > 65536) {
        hipLaunchKernelGGL(minmax_kernel<false>, dim3(256), dim3(256), 0, st, v, n, part);
        hipLaunchKernelGGL(minmax_kernel<true>, dim3(1), dim3(256), 0, st, (const double *)part, (int64_t)256, out);
    } else {
        hipLaunchKernelGGL(minmax_kernel<false>, dim3(1), dim3(256), 0, st, v, n, out);
    }
    return hipGetLastError();
}

hipError_t launch_src_check(const int64_t *src, int64_t n_src, int64_t n, unsigned *bad, hipStream_t st)
{
    hipLaunchKernelGGL(fill_u32_kernel, dim3(1), dim3(64), 0, st, bad, (int64_t)1, 0u);
    if (n_src > 0)
        hipLaunchKernelGGL(src_check_kernel, dim3(grid_for(n_src, 256)), dim3(256), 0, st, src, n_src, n, bad);
    return hipGetLastError();
}

}  // namespace fdirw
