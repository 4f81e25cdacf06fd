// fdirw_mp.hip -- device side of the integrated near-field solver of arXiv
// 2408.11376 (Sec. 2, Eqs. 1-7; flowchart of Sec. 3.4): absorption at the
// liquid/solid interface, slow diffusion in the solid and the far-field
// balance.  The fast liquid step is the coarse-mesh step of fdirw_coarse.hip.
//
// Every kernel here is HBM- or latency-bound elementwise work: grid-stride
// loops of 256 threads, coalesced along x, FP64 throughout.
#include <hip/hip_runtime.h>

#include "fdirw_launch.h"

namespace fdirw {

constexpr int MP_NT = 256;

static unsigned mp_grid(int64_t n)
{
    const int64_t b = (n + MP_NT - 1) / MP_NT;
    return (unsigned)(b < 8192 ? (b > 0 ? b : 1) : 8192);
}

// Interface faces per reaction pass: pass p = 2 * axis + parity counts the
// faces along axis (x, y, z) between a cell whose coordinate has that parity
// and its upper neighbour, when one of the two is near-field liquid and the
// other solid.
__global__ void mp_faces_kernel(const int *__restrict__ node, int nx, int ny, int nz,
                                unsigned long long *__restrict__ count)
{
    const int64_t n = (int64_t)nx * ny * nz;
    const int64_t sz = (int64_t)nx * ny;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int ni = node[i];
        const bool li = ni >= 0, si = ni == COARSE_OUTSIDE;
        if (!li && !si) continue;
        const int x = (int)(i % nx), y = (int)((i / nx) % ny), z = (int)(i / sz);
        const int coord[3] = {x, y, z};
        const int dim[3] = {nx, ny, nz};
        const int64_t stride[3] = {1, nx, sz};
        for (int ax = 0; ax < 3; ++ax) {
            if (coord[ax] + 1 >= dim[ax]) continue;
            const int nj = node[i + stride[ax]];
            const bool lj = nj >= 0, sj = nj == COARSE_OUTSIDE;
            if (!((li && sj) || (si && lj))) continue;
            atomicAdd(&count[2 * ax + (coord[ax] & 1)], 1ull);
        }
    }
}

// The interface law (Eqs. 4-6) integrated exactly over one big step for each
// face of one pass: with a = c_L - c_L^eq, b = c_S^eq - c_S and d = (b - a)
// kappa dt the liquid cell gives x = a b (e^d - 1) / (b e^d - a) to the solid
// cell (evaluated with expm1 in the form that cannot overflow); nothing moves
// while the liquid is at or below equilibrium.
__device__ __forceinline__ double pso_transfer(double a, double b, double kappa_dt)    // a > 0
{
    const double d = (b - a) * kappa_dt;
    if (d > 0.0) {
        const double m = -expm1(-d);
        return a * b * m / ((b - a) + a * m);
    }
    if (d < 0.0) {
        const double m = expm1(d);
        return a * b * m / (b * m + (b - a));
    }
    return a * b * kappa_dt / (1.0 + a * kappa_dt);
}

// Sorted cell lists.  mode 0: the active cells (near-field liquid and solid,
// every cell a step reads or writes), mode 1: the solid cells.  Chunks of
// MP_CHUNK cells: one workgroup counts a chunk, the host scans the counts,
// then one workgroup writes a chunk's indices in cell order.
__device__ __forceinline__ bool mp_pick(int I, int mode)
{
    return mode == 0 ? I != COARSE_RESERVOIR : I == COARSE_OUTSIDE;
}

__global__ void __launch_bounds__(MP_NT) mp_list_count_kernel(const int *__restrict__ node, int64_t n, int mode,
                                                             int *__restrict__ chunk_count)
{
    __shared__ int cnt[MP_NT];
    const int64_t base = blockIdx.x * (int64_t)MP_CHUNK + threadIdx.x * (MP_CHUNK / MP_NT);
    int c = 0;
    for (int j = 0; j < MP_CHUNK / MP_NT; ++j)
        if (base + j < n && mp_pick(node[base + j], mode)) ++c;
    cnt[threadIdx.x] = c;
    __syncthreads();
    for (int w = MP_NT / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) cnt[threadIdx.x] += cnt[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) chunk_count[blockIdx.x] = cnt[0];
}

__global__ void __launch_bounds__(MP_NT) mp_list_write_kernel(const int *__restrict__ node, int64_t n, int mode,
                                                             const int64_t *__restrict__ chunk_off,
                                                             int *__restrict__ list)
{
    __shared__ int cnt[MP_NT];
    const int64_t base = blockIdx.x * (int64_t)MP_CHUNK + threadIdx.x * (MP_CHUNK / MP_NT);
    int c = 0;
    for (int j = 0; j < MP_CHUNK / MP_NT; ++j)
        if (base + j < n && mp_pick(node[base + j], mode)) ++c;
    cnt[threadIdx.x] = c;
    __syncthreads();
    if (threadIdx.x == 0) {                                       // exclusive prefix over the threads
        int run = 0;
        for (int t = 0; t < MP_NT; ++t) {
            const int v = cnt[t];
            cnt[t] = run;
            run += v;
        }
    }
    __syncthreads();
    int64_t at = chunk_off[blockIdx.x] + cnt[threadIdx.x];
    for (int j = 0; j < MP_CHUNK / MP_NT; ++j)
        if (base + j < n && mp_pick(node[base + j], mode)) list[at++] = (int)(base + j);
}

// Solid step coefficients, once per handle: for solid cell k (list order) and
// face f in the order -x, +x, -y, +y, -z, +z, lam[f][k] = harmonic mean of
// the two coefficients D A / RT times dt_s / h^2 if the neighbour is a solid
// cell inside the domain with a positive coefficient, else 0, and nb[f][k] =
// the neighbour's position in the solid list (-1 where lam is 0).  inv: the
// list position of every solid cell.
__global__ void mp_solid_prep_kernel(const int *__restrict__ sol, int64_t n_sol, const uint8_t *__restrict__ label,
                                     const double *__restrict__ dsol, const int *__restrict__ inv, int nx, int ny,
                                     int nz, double dt,
                                     double h, double *__restrict__ lam, int *__restrict__ nb)
{
    const int64_t sz = (int64_t)nx * ny;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n_sol;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = sol[k];
        const int x = (int)(i % nx), y = (int)((i / nx) % ny), z = (int)(i / sz);
        const double di = dsol[label[i]];
        const bool in[6] = {x > 0, x < nx - 1, y > 0, y < ny - 1, z > 0, z < nz - 1};
        const int64_t off[6] = {-1, 1, -(int64_t)nx, (int64_t)nx, -sz, sz};
        for (int f = 0; f < 6; ++f) {
            double l = 0.0;
            int m = -1;
            if (in[f] && di > 0.0) {
                const int64_t j = i + off[f];
                const int q = inv[j];
                const double dj = dsol[label[j]];
                if (q >= 0 && dj > 0.0) {
                    const double df = (2.0 * di) * dj / (di + dj);
                    l = (df * dt) / (h * h);
                    m = q;
                }
            }
            lam[f * n_sol + k] = l;
            nb[f * n_sol + k] = m;
        }
    }
}

__global__ void mp_inverse_kernel(const int *__restrict__ list, int64_t n_list, int *__restrict__ inv)
{
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n_list;
         k += (int64_t)gridDim.x * blockDim.x)
        inv[list[k]] = (int)k;
}

// One explicit sub-step of the slow diffusion on the solid list, terms in the
// order -x, +x, -y, +y, -z, +z.  first: reads the field (neighbours by cell
// offset), else the previous sub-step's list values (neighbours by list
// position).
__global__ void mp_solid_first_kernel(const int *__restrict__ sol, int64_t n_sol, const double *__restrict__ lam,
                                      int nx, int64_t sz, const double *__restrict__ field, double *__restrict__ out)
{
    const int64_t off[6] = {-1, 1, -(int64_t)nx, (int64_t)nx, -sz, sz};
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n_sol;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = sol[k];
        const double g = field[i];
        double acc = g;
#pragma unroll
        for (int f = 0; f < 6; ++f) {
            const double l = lam[f * n_sol + k];
            if (l != 0.0) acc += l * (field[i + off[f]] - g);
        }
        out[k] = acc;
    }
}

__global__ void mp_solid_next_kernel(int64_t n_sol, const double *__restrict__ lam, const int *__restrict__ nb,
                                     const double *__restrict__ in, double *__restrict__ out)
{
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n_sol;
         k += (int64_t)gridDim.x * blockDim.x) {
        const double g = in[k];
        double acc = g;
#pragma unroll
        for (int f = 0; f < 6; ++f) {
            const int m = nb[f * n_sol + k];
            if (m >= 0) acc += lam[f * n_sol + k] * (in[m] - g);
        }
        out[k] = acc;
    }
}

__global__ void mp_solid_scatter_kernel(const int *__restrict__ sol, int64_t n_sol, const double *__restrict__ v,
                                        double *__restrict__ field)
{
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n_sol;
         k += (int64_t)gridDim.x * blockDim.x)
        field[sol[k]] = v[k];
}

// Block-wide fixed-order tree sum of two values (every thread gets them), in
// the caller's LDS scratch (2 x MP_NT doubles).
__device__ void mp_block_sum2_in(double &a, double &b, double *sa, double *sb)
{
    __syncthreads();
    sa[threadIdx.x] = a;
    sb[threadIdx.x] = b;
    __syncthreads();
    for (int w = MP_NT / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sa[threadIdx.x] += sa[threadIdx.x + w];
            sb[threadIdx.x] += sb[threadIdx.x + w];
        }
        __syncthreads();
    }
    a = sa[0];
    b = sb[0];
}

__device__ void mp_block_sum2(double &a, double &b)
{
    __shared__ double sa[MP_NT], sb[MP_NT];
    mp_block_sum2_in(a, b, sa, sb);
}

// Eq. 7 from the per-workgroup partials of the previous launch (Q_L in
// part[0..nblk), Q_S in part[nblk..2 nblk)), one workgroup: the partials in
// workgroup order, then c_ff = (M_total - Q_L - Q_S) / V_ff into *cff and the
// history row.
__global__ void __launch_bounds__(MP_NT) mp_finish_kernel(const double *__restrict__ part, int nblk, double m_total,
                                                         double v_ff, double *__restrict__ cff,
                                                         double *__restrict__ hist_row)
{
    double ql = 0.0, qs = 0.0;
    for (int k = threadIdx.x; k < nblk; k += MP_NT) {
        ql += part[k];
        qs += part[nblk + k];
    }
    mp_block_sum2(ql, qs);
    if (threadIdx.x == 0) {
        const double v = (m_total - ql - qs) / v_ff;
        cff[0] = v;
        if (hist_row) {
            hist_row[0] = ql;
            hist_row[1] = qs;
            hist_row[2] = v;
        }
    }
}

// Eq. 7, first level, over the active list: each workgroup sums the
// near-field liquid (Q_L) and the solid (Q_S) over a fixed stride of the list
// and a fixed tree (mp_finish_kernel adds the partials).
__global__ void __launch_bounds__(MP_NT) mp_balance_kernel(const int *__restrict__ act, int64_t n_act,
                                                          const int *__restrict__ node, const double *__restrict__ c,
                                                          double *__restrict__ part)
{
    const int nblk = gridDim.x;
    double ql = 0.0, qs = 0.0;
    const int64_t stride = (int64_t)nblk * MP_NT;
    // the strided sequence of list entries, four per round with every load
    // of a round issued before the adds
    for (int64_t k0 = blockIdx.x * (int64_t)MP_NT + threadIdx.x; k0 < n_act; k0 += 4 * stride) {
        int i[4], nd[4];
        double v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) i[u] = act[k0 + u * stride < n_act ? k0 + u * stride : k0];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            nd[u] = node[i[u]];
            v[u] = c[i[u]];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (k0 + u * stride < n_act) {
                if (nd[u] >= 0) ql += v[u];
                else qs += v[u];
            }
    }
    mp_block_sum2(ql, qs);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = ql;
        part[nblk + blockIdx.x] = qs;
    }
}

// Role of a cell in the LDS box: 0 near-field liquid, 1 solid, -1 neither
// (far field or outside the domain).
__device__ __forceinline__ signed char mp_role(int I) { return I >= 0 ? 0 : (I == COARSE_OUTSIDE ? 1 : -1); }

// The box cell q of a tile (box origin x0, y0, z0 = tile origin - MP_H).
__device__ __forceinline__ void mp_box_cell(int q, int x0, int y0, int z0, int &gx, int &gy, int &gz)
{
    gx = x0 + q % MP_BX;
    gy = y0 + (q / MP_BX) % MP_BY;
    gz = z0 + q / (MP_BX * MP_BY);
}

__device__ __forceinline__ void mp_tile_origin(int t, int nx, int ny, int &x0, int &y0, int &z0)
{
    const int ntx = (nx + MP_TX - 1) / MP_TX, nty = (ny + MP_TY - 1) / MP_TY;
    x0 = (t % ntx) * MP_TX - MP_H;
    y0 = ((t / ntx) % nty) * MP_TY - MP_H;
    z0 = (t / (ntx * nty)) * MP_TZ - MP_H;
}

// The interface pairs of one tile's box for the six reaction passes, found
// once per handle.  Pass p = 2 * axis + parity holds the pairs along the axis
// whose lower cell has global coordinate of that parity, with one cell
// near-field liquid and the other solid; entry (q << 1) | (lower cell is the
// solid one), q the lower cell in the box.  The pairs of a pass are disjoint,
// so their order is free (LDS atomics).  list null: count only (cnt[6 t +
// p]); else the entries go to list[off[6 t + p] ...].
__global__ void __launch_bounds__(MP_NT) mp_tile_pairs_kernel(const int *__restrict__ node, int nx, int ny, int nz,
                                                             const int *__restrict__ tiles,
                                                             const int *__restrict__ off, uint16_t *__restrict__ list,
                                                             int *__restrict__ cnt)
{
    __shared__ signed char role[MP_BOX];
    __shared__ int lcount[6];
    const int t = tiles[blockIdx.x];
    int x0, y0, z0;
    mp_tile_origin(t, nx, ny, x0, y0, z0);
    if (threadIdx.x < 6) lcount[threadIdx.x] = 0;
    for (int q = threadIdx.x; q < MP_BOX; q += MP_NT) {
        int gx, gy, gz;
        mp_box_cell(q, x0, y0, z0, gx, gy, gz);
        const bool in = gx >= 0 && gx < nx && gy >= 0 && gy < ny && gz >= 0 && gz < nz;
        role[q] = in ? mp_role(node[((int64_t)gz * ny + gy) * nx + gx]) : (signed char)-1;
    }
    __syncthreads();
    for (int p = 0; p < 6; ++p) {
        const int ax = p >> 1, par = p & 1;
        const int len = ax == 0 ? MP_BX : (ax == 1 ? MP_BY : MP_BZ);
        const int step = ax == 0 ? 1 : (ax == 1 ? MP_BX : MP_BX * MP_BY);
        const int org = ax == 0 ? x0 : (ax == 1 ? y0 : z0);
        const int first = (par - org) & 1;
        for (int q = threadIdx.x; q < MP_BOX; q += MP_NT) {
            const int l = ax == 0 ? q % MP_BX : (ax == 1 ? (q / MP_BX) % MP_BY : q / (MP_BX * MP_BY));
            if (((l - first) & 1) || l + 1 >= len) continue;
            const signed char rl = role[q], ru = role[q + step];
            if (rl < 0 || ru < 0 || rl == ru) continue;
            const int slot = atomicAdd(&lcount[p], 1);
            if (list) list[off[6 * blockIdx.x + p] + slot] = (uint16_t)((q << 1) | (rl == 1 ? 1 : 0));
        }
    }
    __syncthreads();
    if (threadIdx.x < 6) cnt[6 * blockIdx.x + threadIdx.x] = lcount[threadIdx.x];
}

// One reaction pass of the fused local kernel along axis AX over the tile's
// interface pairs [b, e) of the pass (list positions relative to the tile's
// first entry; the first MP_PAIR_CAP are staged in LDS).  A barrier closes the
// pass.
template <int AX>
__device__ __forceinline__ void mp_pass(double *v, const uint16_t *pl, const uint16_t *gl, int b, int e,
                                        const MpLocalArgs &a)
{
    constexpr int STEP = AX == 0 ? 1 : (AX == 1 ? MP_BX : MP_BX * MP_BY);
    for (int m = b + (int)threadIdx.x; m < e; m += MP_NT) {
        const int ent = m < MP_PAIR_CAP ? pl[m] : gl[m];
        const int q = ent >> 1, qu = q + STEP;
        const int ql = (ent & 1) ? qu : q, qs = (ent & 1) ? q : qu;
        const double cl = v[ql], cs = v[qs];
        const double aa = cl - a.c_eq_l;
        if (!(aa > 0.0)) continue;
        const double x = pso_transfer(aa, a.c_eq_s - cs, a.kappa_dt);
        v[ql] = cl - x;
        v[qs] = cs + x;
    }
    __syncthreads();
}

// The local part of a big step in one launch, one workgroup per tile of
// MP_TX x MP_TY x MP_TZ cells that holds an active cell.  The tile and a halo
// of MP_H cells are loaded into LDS with the remapped values (Eq. 15: node
// value for near-field liquid, own value for solid); the six reaction passes
// run on the box's interface pairs of each pass (listed once per handle by
// mp_tile_pairs_kernel); one solid sub-step follows for the tile's solid cells (if
// a.solid); the tile's cells are written to out, and (if a.solid) its Q_L /
// Q_S partials go to a.part for mp_finish_kernel (Eq. 7).  The passes move information by at most two cells
// per axis and the sub-step by one, so with MP_H = 3 every tile cell gets
// exactly the values of the whole-grid passes.
__global__ void __launch_bounds__(MP_NT) mp_local_kernel(MpLocalArgs a)
{
    // 39.8 KB: four workgroups per CU
    __shared__ double v[MP_BOX];
    __shared__ signed char role[MP_BOX];                          // -1 none, 0 liquid, 1 + s solid of phase s
    __shared__ __align__(8) uint16_t pl[MP_PAIR_CAP];            // then the solid lambda table
    static_assert(MP_PAIR_CAP * sizeof(uint16_t) >= MP_MAX_SOLID_PHASES * sizeof(double), "lambda table");
    const int t = a.tiles[blockIdx.x];
    int x0, y0, z0;
    mp_tile_origin(t, a.nx, a.ny, x0, y0, z0);
    // this tile's interface pairs: the pass bounds and the first MP_PAIR_CAP
    // entries into LDS
    const int *po = a.pair_off + 6 * blockIdx.x;
    const int pbase = po[0];
    const uint16_t *gl = a.pairs + pbase;
    const int n_pairs = po[6] - pbase;
    for (int m = threadIdx.x; m < n_pairs && m < MP_PAIR_CAP; m += MP_NT) pl[m] = gl[m];
    const int64_t sy = a.nx, sz = (int64_t)a.nx * a.ny;
    // load (remapping on the fly), in rounds of ROUND cells per thread: the
    // node indices of a round first, then its values, so that the loads of a
    // stage are in flight together
    constexpr int ROUND = 6;
    constexpr int NONE = -3;                                      // outside the domain
    for (int q0 = threadIdx.x; q0 < MP_BOX; q0 += ROUND * MP_NT) {
        int64_t gi[ROUND];
        int nd[ROUND];
#pragma unroll
        for (int u = 0; u < ROUND; ++u) {
            const int q = q0 + u * MP_NT;
            int gx, gy, gz;
            mp_box_cell(q, x0, y0, z0, gx, gy, gz);
            const bool in = q < MP_BOX && gx >= 0 && gx < a.nx && gy >= 0 && gy < a.ny && gz >= 0 && gz < a.nz;
            gi[u] = in ? gz * sz + gy * sy + gx : 0;
            nd[u] = in ? a.node[gi[u]] : NONE;
        }
        double val[ROUND];
        int sc[ROUND];                                            // ints: no packing, no early waits
#pragma unroll
        for (int u = 0; u < ROUND; ++u) {
            val[u] = 0.0;
            sc[u] = -1;
            if (nd[u] >= 0) {
                val[u] = a.cnew[nd[u]];
                sc[u] = 0;
            } else if (nd[u] == COARSE_OUTSIDE) {
                val[u] = a.c_in[gi[u]];
                sc[u] = 1 + a.scode[gi[u]];
            }
        }
#pragma unroll
        for (int u = 0; u < ROUND; ++u) {
            const int q = q0 + u * MP_NT;
            if (q < MP_BOX) {
                v[q] = val[u];
                role[q] = (signed char)sc[u];
            }
        }
    }
    __syncthreads();
    // the six reaction passes
    mp_pass<0>(v, pl, gl, po[0] - pbase, po[1] - pbase, a);
    mp_pass<0>(v, pl, gl, po[1] - pbase, po[2] - pbase, a);
    mp_pass<1>(v, pl, gl, po[2] - pbase, po[3] - pbase, a);
    mp_pass<1>(v, pl, gl, po[3] - pbase, po[4] - pbase, a);
    mp_pass<2>(v, pl, gl, po[4] - pbase, po[5] - pbase, a);
    mp_pass<2>(v, pl, gl, po[5] - pbase, po[6] - pbase, a);
    // one solid sub-step, the writes and the partial sums.  The pair list is
    // no longer read (the last pass ended with a barrier): its LDS takes
    // lambda = D A / RT dt_s / h^2 of every solid phase by compact index, the
    // face value being the harmonic mean of the two cells' lambdas
    double sl = 0.0, ss = 0.0;
    double *lam = reinterpret_cast<double *>(pl);
    if (a.solid) {
        const double sc = a.dt_s / (a.h * a.h);
        for (int k = threadIdx.x; k < a.n_solid; k += MP_NT) lam[k] = a.dsolc[k] * sc;
        __syncthreads();
    }
    for (int m = threadIdx.x; m < MP_TX * MP_TY * MP_TZ; m += MP_NT) {
        const int lx = MP_H + m % MP_TX, ly = MP_H + (m / MP_TX) % MP_TY, lz = MP_H + m / (MP_TX * MP_TY);
        const int q = (lz * MP_BY + ly) * MP_BX + lx;
        const signed char r = role[q];
        if (r < 0) continue;
        const int64_t i = (int64_t)(z0 + lz) * sz + (int64_t)(y0 + ly) * sy + (x0 + lx);
        double g = v[q];
        if (r == 0) {
            sl += g;
        } else {
            if (a.solid) {
                const double li = lam[r - 1];
                double acc = g;
                if (li > 0.0) {
                    const int nbq[6] = {q - 1, q + 1, q - MP_BX, q + MP_BX, q - MP_BX * MP_BY, q + MP_BX * MP_BY};
#pragma unroll
                    for (int f = 0; f < 6; ++f) {
                        const int qq = nbq[f];
                        const int rq = role[qq];
                        if (rq < 1) continue;
                        const double lj = lam[rq - 1];
                        if (!(lj > 0.0)) continue;
                        acc += (2.0 * li) * lj / (li + lj) * (v[qq] - g);
                    }
                }
                g = acc;
            }
            ss += g;
        }
        a.out[i] = g;
    }
    if (!a.solid) return;
    mp_block_sum2_in(sl, ss, v, v + MP_NT);                       // v is no longer read
    if (threadIdx.x == 0) {
        a.part[blockIdx.x] = sl;
        a.part[gridDim.x + blockIdx.x] = ss;
    }
}

// scode[i] = compact solid-phase index of cell i (the fused kernel's solid
// coefficient table), from the labels.
struct MpCodeTable {
    unsigned char s[256];
};

__global__ void mp_code_kernel(const uint8_t *__restrict__ label, int64_t n, MpCodeTable tab,
                               uint8_t *__restrict__ scode)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        scode[i] = tab.s[label[i]];
}

hipError_t launch_mp_code(const uint8_t *label, int64_t n, const unsigned char *table256, uint8_t *scode,
                          hipStream_t st)
{
    MpCodeTable t;
    for (int k = 0; k < 256; ++k) t.s[k] = table256[k];
    hipLaunchKernelGGL(mp_code_kernel, dim3(mp_grid(n)), dim3(MP_NT), 0, st, label, n, t, scode);
    return hipGetLastError();
}

// Marks the tiles that hold an active cell (flag per tile).
__global__ void __launch_bounds__(MP_NT) mp_tile_flag_kernel(const int *__restrict__ node, int nx, int ny, int nz,
                                                            int *__restrict__ flag)
{
    __shared__ int any;
    if (threadIdx.x == 0) any = 0;
    __syncthreads();
    const int t = blockIdx.x;
    const int ntx = (nx + MP_TX - 1) / MP_TX, nty = (ny + MP_TY - 1) / MP_TY;
    const int x0 = (t % ntx) * MP_TX, y0 = ((t / ntx) % nty) * MP_TY, z0 = (t / (ntx * nty)) * MP_TZ;
    int mine = 0;
    for (int m = threadIdx.x; m < MP_TX * MP_TY * MP_TZ; m += MP_NT) {
        const int gx = x0 + m % MP_TX, gy = y0 + (m / MP_TX) % MP_TY, gz = z0 + m / (MP_TX * MP_TY);
        if (gx < nx && gy < ny && gz < nz && node[((int64_t)gz * ny + gy) * nx + gx] != COARSE_RESERVOIR) mine = 1;
    }
    if (mine) any = 1;                                            // benign: every writer stores 1
    __syncthreads();
    if (threadIdx.x == 0) flag[t] = any;
}

// dst = src with the far-field cells set to *cff (src == dst: only those cells
// are written).
__global__ void mp_far_fill_kernel(const int *__restrict__ node, int64_t n, const double *__restrict__ cff,
                                   const double *src, double *dst)
{
    const double v = cff[0];
    const bool copy = src != dst;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (node[i] == COARSE_RESERVOIR) dst[i] = v;
        else if (copy) dst[i] = src[i];
    }
}

int64_t mp_tile_count(int nx, int ny, int nz)
{
    return (int64_t)((nx + MP_TX - 1) / MP_TX) * ((ny + MP_TY - 1) / MP_TY) * ((nz + MP_TZ - 1) / MP_TZ);
}

hipError_t launch_mp_faces(const int *node, int nx, int ny, int nz, unsigned long long *count, hipStream_t st)
{
    hipLaunchKernelGGL(mp_faces_kernel, dim3(mp_grid((int64_t)nx * ny * nz)), dim3(MP_NT), 0, st, node, nx, ny, nz,
                       count);
    return hipGetLastError();
}

static unsigned mp_chunks(int64_t n) { return (unsigned)((n + MP_CHUNK - 1) / MP_CHUNK); }

hipError_t launch_mp_list_count(const int *node, int64_t n, int mode, int *chunk_count, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(mp_list_count_kernel, dim3(mp_chunks(n)), dim3(MP_NT), 0, st, node, n, mode, chunk_count);
    return hipGetLastError();
}

hipError_t launch_mp_list_write(const int *node, int64_t n, int mode, const int64_t *chunk_off, int *list,
                                hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(mp_list_write_kernel, dim3(mp_chunks(n)), dim3(MP_NT), 0, st, node, n, mode, chunk_off, list);
    return hipGetLastError();
}

hipError_t launch_mp_solid_prep(const int *sol, int64_t n_sol, const uint8_t *label, const double *dsol,
                                int *inv, int nx, int ny, int nz, double dt, double h, double *lam, int *nb,
                                hipStream_t st)
{
    if (n_sol <= 0) return hipSuccess;
    hipLaunchKernelGGL(mp_inverse_kernel, dim3(mp_grid(n_sol)), dim3(MP_NT), 0, st, sol, n_sol, inv);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(mp_solid_prep_kernel, dim3(mp_grid(n_sol)), dim3(MP_NT), 0, st, sol, n_sol, label, dsol,
                       (const int *)inv, nx, ny, nz, dt, h, lam, nb);
    return hipGetLastError();
}

hipError_t launch_mp_solid(const int *sol, int64_t n_sol, const double *lam, const int *nb, int nx, int ny,
                           int n_sub, double *field, double *a, double *b, hipStream_t st)
{
    if (n_sol <= 0 || n_sub <= 0) return hipSuccess;
    const unsigned g = mp_grid(n_sol);
    hipLaunchKernelGGL(mp_solid_first_kernel, dim3(g), dim3(MP_NT), 0, st, sol, n_sol, lam, nx, (int64_t)nx * ny,
                       (const double *)field, a);
    hipError_t e = hipGetLastError();
    for (int k = 1; k < n_sub && e == hipSuccess; ++k) {
        hipLaunchKernelGGL(mp_solid_next_kernel, dim3(g), dim3(MP_NT), 0, st, n_sol, lam, nb, (const double *)a, b);
        e = hipGetLastError();
        double *t = a; a = b; b = t;
    }
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(mp_solid_scatter_kernel, dim3(g), dim3(MP_NT), 0, st, sol, n_sol, (const double *)a, field);
    return hipGetLastError();
}

hipError_t launch_mp_tile_flags(const int *node, int nx, int ny, int nz, int *flag, hipStream_t st)
{
    const int64_t nt = mp_tile_count(nx, ny, nz);
    if (nt <= 0) return hipSuccess;
    hipLaunchKernelGGL(mp_tile_flag_kernel, dim3((unsigned)nt), dim3(MP_NT), 0, st, node, nx, ny, nz, flag);
    return hipGetLastError();
}

hipError_t launch_mp_tile_pairs(const int *node, int nx, int ny, int nz, const int *tiles, int64_t n_tiles,
                                const int *off, uint16_t *list, int *cnt, hipStream_t st)
{
    if (n_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(mp_tile_pairs_kernel, dim3((unsigned)n_tiles), dim3(MP_NT), 0, st, node, nx, ny, nz, tiles,
                       off, list, cnt);
    return hipGetLastError();
}

hipError_t launch_mp_local(const MpLocalArgs &a, hipStream_t st)
{
    if (a.n_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(mp_local_kernel, dim3((unsigned)a.n_tiles), dim3(MP_NT), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !a.solid) return e;
    hipLaunchKernelGGL(mp_finish_kernel, dim3(1), dim3(MP_NT), 0, st, (const double *)a.part, (int)a.n_tiles,
                       a.m_total, a.v_ff, a.cff, a.hist_row);
    return hipGetLastError();
}

unsigned mp_balance_blocks(int64_t n_act)
{
    const int64_t b = (n_act + MP_NT - 1) / MP_NT;
    return (unsigned)(b < 1 ? 1 : (b < MP_SUM_BLOCKS ? b : MP_SUM_BLOCKS));
}

hipError_t launch_mp_balance(const int *act, int64_t n_act, const int *node, const double *c, double *part,
                             double m_total, double v_ff, double *cff, double *hist_row, hipStream_t st)
{
    const unsigned nb = mp_balance_blocks(n_act);
    hipLaunchKernelGGL(mp_balance_kernel, dim3(nb), dim3(MP_NT), 0, st, act, n_act, node, c, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(mp_finish_kernel, dim3(1), dim3(MP_NT), 0, st, (const double *)part, (int)nb, m_total, v_ff,
                       cff, hist_row);
    return hipGetLastError();
}

hipError_t launch_mp_far_fill(const int *node, int64_t n, const double *cff, const double *src, double *dst,
                              hipStream_t st)
{
    hipLaunchKernelGGL(mp_far_fill_kernel, dim3(mp_grid(n)), dim3(MP_NT), 0, st, node, n, cff, src, dst);
    return hipGetLastError();
}

}  // namespace fdirw
