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

// Face lists of the interface reaction.  Pass p = 2 * axis + parity holds the
// faces along axis (x, y, z) between a cell whose coordinate has that parity
// and its upper neighbour, when one of the two is near-field liquid and the
// other solid.  No cell appears twice in a pass, so the order of the entries
// does not matter (they are appended with atomics).  Entry: (lower cell << 1)
// | (lower cell is the solid one).  list null: count only.
__global__ void mp_faces_kernel(const int *__restrict__ node, int nx, int ny, int nz, MpFaceLists lists,
                                int64_t *__restrict__ list, unsigned long long *__restrict__ count)
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
            const int p = 2 * ax + (coord[ax] & 1);
            const unsigned long long slot = atomicAdd(&count[p], 1ull);
            if (list && (int64_t)slot < lists.cap[p]) list[lists.off[p] + (int64_t)slot] = (i << 1) | (si ? 1 : 0);
        }
    }
}

// The interface law (Eqs. 4-6) integrated exactly over one big step for each
// face of one pass: with a = c_L - c_L^eq, b = c_S^eq - c_S and d = (b - a)
// kappa dt the liquid cell gives x = a b (e^d - 1) / (b e^d - a) to the solid
// cell (evaluated with expm1 in the form that cannot overflow); nothing moves
// while the liquid is at or below equilibrium.
__global__ void mp_react_kernel(const int64_t *__restrict__ faces, int64_t n_faces, int64_t stride,
                                double *__restrict__ c, double c_eq_l, double c_eq_s, double kappa_dt)
{
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n_faces;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t f = faces[t];
        const int64_t lo = f >> 1, hi = lo + stride;
        const int64_t il = (f & 1) ? hi : lo, is = (f & 1) ? lo : hi;
        const double cl = c[il], cs = c[is];
        const double a = cl - c_eq_l;
        if (!(a > 0.0)) continue;
        const double b = c_eq_s - cs;
        const double d = (b - a) * kappa_dt;
        double x;
        if (d > 0.0) {
            const double m = -expm1(-d);
            x = a * b * m / ((b - a) + a * m);
        } else if (d < 0.0) {
            const double m = expm1(d);
            x = a * b * m / (b * m + (b - a));
        } else {
            x = a * b * kappa_dt / (1.0 + a * kappa_dt);
        }
        c[il] = cl - x;
        c[is] = cs + x;
    }
}

// One explicit sub-step of the slow diffusion: solid cells exchange with their
// solid neighbours through harmonic-mean faces (coefficient D A / RT per
// phase), every other face is a wall and every other cell is copied.  Terms in
// the order -x, +x, -y, +y, -z, +z.
__global__ void mp_solid_kernel(const uint8_t *__restrict__ label, SolidTable tab, int nx, int ny, int nz, double dt,
                                double h, const double *__restrict__ in, double *__restrict__ out)
{
    const int64_t n = (int64_t)nx * ny * nz;
    const int64_t sy = nx, sz = (int64_t)nx * ny;
    const double hh = h * h;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double g = in[i];
        const double di = tab.d[label[i]];
        if (!(di > 0.0)) {
            out[i] = g;
            continue;
        }
        const int x = (int)(i % nx), y = (int)((i / nx) % ny), z = (int)(i / sz);
        double acc = g;
        auto face = [&](int64_t j) {
            const double dj = tab.d[label[j]];
            if (dj > 0.0) {
                const double df = (2.0 * di) * dj / (di + dj);
                acc += (df * dt) / hh * (in[j] - g);
            }
        };
        if (x > 0) face(i - 1);
        if (x < nx - 1) face(i + 1);
        if (y > 0) face(i - sy);
        if (y < ny - 1) face(i + sy);
        if (z > 0) face(i - sz);
        if (z < nz - 1) face(i + sz);
        out[i] = acc;
    }
}

// Eq. 7, first level: per-workgroup sums of the near-field liquid (Q_L) and of
// the solid (Q_S), each thread over a fixed stride of cells, then a fixed tree.
__global__ void __launch_bounds__(MP_NT) mp_sum_kernel(const int *__restrict__ node, const double *__restrict__ c,
                                                      int64_t n, double *__restrict__ part)
{
    __shared__ double sl[MP_NT], ss[MP_NT];
    double ql = 0.0, qs = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)MP_NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * MP_NT) {
        const int I = node[i];
        const double v = c[i];
        if (I >= 0) ql += v;
        else if (I == COARSE_OUTSIDE) qs += v;
    }
    sl[threadIdx.x] = ql;
    ss[threadIdx.x] = qs;
    __syncthreads();
    for (int w = MP_NT / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sl[threadIdx.x] += sl[threadIdx.x + w];
            ss[threadIdx.x] += ss[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[blockIdx.x] = sl[0];
        part[MP_SUM_BLOCKS + blockIdx.x] = ss[0];
    }
}

// Eq. 7, second level (one workgroup): c_ff = (M_total - Q_L - Q_S) / V_ff,
// written to *cff and, with Q_L and Q_S, to the history row.
__global__ void __launch_bounds__(MP_NT) mp_balance_kernel(const double *__restrict__ part, double m_total,
                                                          double v_ff, double *__restrict__ cff,
                                                          double *__restrict__ hist_row)
{
    __shared__ double sl[MP_NT], ss[MP_NT];
    double ql = 0.0, qs = 0.0;
    for (int k = threadIdx.x; k < MP_SUM_BLOCKS; k += MP_NT) {
        ql += part[k];
        qs += part[MP_SUM_BLOCKS + k];
    }
    sl[threadIdx.x] = ql;
    ss[threadIdx.x] = qs;
    __syncthreads();
    for (int w = MP_NT / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sl[threadIdx.x] += sl[threadIdx.x + w];
            ss[threadIdx.x] += ss[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double v = (m_total - sl[0] - ss[0]) / v_ff;
        cff[0] = v;
        if (hist_row) {
            hist_row[0] = sl[0];
            hist_row[1] = ss[0];
            hist_row[2] = v;
        }
    }
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

hipError_t launch_mp_faces(const int *node, int nx, int ny, int nz, const MpFaceLists &lists, int64_t *list,
                           unsigned long long *count, hipStream_t st)
{
    hipLaunchKernelGGL(mp_faces_kernel, dim3(mp_grid((int64_t)nx * ny * nz)), dim3(MP_NT), 0, st, node, nx, ny, nz,
                       lists, list, count);
    return hipGetLastError();
}

hipError_t launch_mp_react(const int64_t *faces, int64_t n_faces, int64_t stride, double *c, double c_eq_l,
                           double c_eq_s, double kappa_dt, hipStream_t st)
{
    if (n_faces <= 0) return hipSuccess;
    hipLaunchKernelGGL(mp_react_kernel, dim3(mp_grid(n_faces)), dim3(MP_NT), 0, st, faces, n_faces, stride, c, c_eq_l,
                       c_eq_s, kappa_dt);
    return hipGetLastError();
}

hipError_t launch_mp_solid(const uint8_t *label, const SolidTable &tab, int nx, int ny, int nz, double dt, double h,
                           const double *in, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(mp_solid_kernel, dim3(mp_grid((int64_t)nx * ny * nz)), dim3(MP_NT), 0, st, label, tab, nx, ny,
                       nz, dt, h, in, out);
    return hipGetLastError();
}

hipError_t launch_mp_balance(const int *node, const double *c, int64_t n, double *part, double m_total, double v_ff,
                             double *cff, double *hist_row, hipStream_t st)
{
    hipLaunchKernelGGL(mp_sum_kernel, dim3(MP_SUM_BLOCKS), dim3(MP_NT), 0, st, node, c, n, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(mp_balance_kernel, dim3(1), dim3(MP_NT), 0, st, (const double *)part, m_total, v_ff, cff,
                       hist_row);
    return hipGetLastError();
}

hipError_t launch_mp_far_fill(const int *node, int64_t n, const double *cff, const double *src, double *dst,
                              hipStream_t st)
{
    hipLaunchKernelGGL(mp_far_fill_kernel, dim3(mp_grid(n)), dim3(MP_NT), 0, st, node, n, cff, src, dst);
    return hipGetLastError();
}

}  // namespace fdirw
