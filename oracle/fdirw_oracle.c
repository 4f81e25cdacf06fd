/*
 * fdirw_oracle.c -- plain FP64 CPU oracle of the FDiRW fast-diffusion step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code, header or constant with the HIP
 * path.
 *
 * What it computes (arXiv 2408.11376):
 *   Sec. 3.1, Eqs. (8)-(9): the state after one big step is the superposition
 *     c(t+dt_big) = P c(t); column j of P is the mass that one unit placed at
 *     node j spreads to every node i over the big step.
 *   Sec. 3.1 (text after Eq. 9): that column is obtained by an explicit finite
 *     difference solution of the diffusion equation started from a single unit
 *     point source.
 *   Eq. (1) (diffusion term, D per phase): the diffusivity is a material
 *     property of each phase.
 * The paper does not state the finite-difference scheme.  The reading used
 * here: a conservative 7-point explicit scheme on unit cells of edge h;
 * face diffusivity = harmonic mean 2 Dx Dy / (Dx + Dy) (0 if either side is 0);
 * lambda_f = D_f dt / h^2; no flux through domain walls, through faces touching
 * an impermeable (D = 0) cell, or through the walls of the local window
 * [s - r, s + r]^3 around the source; sub-step dt = 0.9 h^2 / (6 Dmax) unless
 * given.  Every source cell of the grid is a source; the superposition skips
 * sources with c(s) = 0, whose contribution is exactly zero.
 *
 * Every floating-point result is FP64.  Compile with -ffp-contract=off so that
 * the expression order written here is the order evaluated.
 *
 * Layout: cell (x, y, z) of an nx*ny*nz grid has linear index
 * (z*ny + y)*nx + x.  Face arrays lam_x/lam_y/lam_z hold, at the index of a
 * cell, the coefficient of the face to its +x/+y/+z neighbour (0 on the last
 * plane).  Windows are W^3 arrays (W = 2r+1) ordered z, y, x relative to s - r;
 * window cells outside the domain hold 0.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define IDX(x, y, z) (((int64_t)(z) * ny + (y)) * nx + (x))

/* Neumaier-compensated sum (Neumaier 1974, "Rundungsfehleranalyse einiger
 * Verfahren zur Summation endlicher Summen"). */
static double neumaier_sum(const double *v, int64_t n)
{
    double s = 0.0, comp = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double t = s + v[i];
        if (fabs(s) >= fabs(v[i])) comp += (s - t) + v[i];
        else                       comp += (v[i] - t) + s;
        s = t;
    }
    return s + comp;
}

double fo_sum(const double *v, int64_t n) { return neumaier_sum(v, n); }

/* Sub-step length: the given dt if > 0, else 0.9 h^2 / (6 Dmax) with Dmax the
 * largest diffusivity of any cell in the grid.  Returns 0 when dt is not given
 * and every cell is impermeable. */
double fo_resolve_dt(int nx, int ny, int nz, const uint8_t *label,
                     const double *d_phase, double h, double dt)
{
    if (dt > 0.0) return dt;
    double dmax = 0.0;
    int64_t n = (int64_t)nx * ny * nz;
    for (int64_t i = 0; i < n; ++i) {
        double d = d_phase[label[i]];
        if (d > dmax) dmax = d;
    }
    if (dmax <= 0.0) return 0.0;
    return (0.9 * h * h) / (6.0 * dmax);
}

/* Face coefficient between two cells of diffusivities da and db. */
static double face_lambda(double da, double db, double dt, double h)
{
    if (!(da > 0.0 && db > 0.0)) return 0.0;
    double num = (2.0 * da) * db;
    double den = da + db;
    double df = num / den;
    return (df * dt) / (h * h);
}

/* Coefficients: the three owned face coefficients of every cell. */
void fo_coefficients(int nx, int ny, int nz, const uint8_t *label,
                     const double *d_phase, double h, double dt,
                     double *lam_x, double *lam_y, double *lam_z)
{
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                int64_t i = IDX(x, y, z);
                double d0 = d_phase[label[i]];
                lam_x[i] = (x + 1 < nx) ? face_lambda(d0, d_phase[label[IDX(x + 1, y, z)]], dt, h) : 0.0;
                lam_y[i] = (y + 1 < ny) ? face_lambda(d0, d_phase[label[IDX(x, y + 1, z)]], dt, h) : 0.0;
                lam_z[i] = (z + 1 < nz) ? face_lambda(d0, d_phase[label[IDX(x, y, z + 1)]], dt, h) : 0.0;
            }
}

/* Explicit sub-steps on a box [lo, hi] (inclusive, per axis) of the grid with
 * no flux through the box walls.  g holds the box state (z, y, x order) on
 * entry and exit; tmp is scratch of the same size.  Jacobi: every cell reads
 * the state of the previous sub-step.  Neighbour order -x, +x, -y, +y, -z, +z.
 * fixed (may be NULL): grid mask of Dirichlet cells (the far-field boundary of
 * Eq. 8), which hold the value fval after every sub-step.
 * nu_x / nu_y / nu_z (NULL, or all three): signed Courant numbers u dt / h of
 * a steady flow on the owned +x / +y / +z face of each cell (positive towards
 * +x / +y / +z); the advective flux through a face is first-order upwind,
 * nu * (value of the upstream cell), added after the diffusive terms in the
 * same neighbour order (the flow extension of Sec. 5). */
static void box_substeps(int nx, int ny, int nz,
                         const double *lam_x, const double *lam_y, const double *lam_z,
                         const int lo[3], const int hi[3], int n_sub,
                         double *g, double *tmp, const uint8_t *fixed, double fval,
                         const double *nu_x, const double *nu_y, const double *nu_z)
{
    (void)nz;
    int bx = hi[0] - lo[0] + 1, by = hi[1] - lo[1] + 1, bz = hi[2] - lo[2] + 1;
    for (int step = 0; step < n_sub; ++step) {
        for (int k = 0; k < bz; ++k)
            for (int j = 0; j < by; ++j)
                for (int i = 0; i < bx; ++i) {
                    int X = lo[0] + i, Y = lo[1] + j, Z = lo[2] + k;
                    int64_t b = ((int64_t)k * by + j) * bx + i;
                    double gx = g[b];
                    double acc = gx;
                    if (i > 0)      acc += lam_x[IDX(X - 1, Y, Z)] * (g[b - 1] - gx);
                    if (i < bx - 1) acc += lam_x[IDX(X, Y, Z)]     * (g[b + 1] - gx);
                    if (j > 0)      acc += lam_y[IDX(X, Y - 1, Z)] * (g[b - bx] - gx);
                    if (j < by - 1) acc += lam_y[IDX(X, Y, Z)]     * (g[b + bx] - gx);
                    if (k > 0)      acc += lam_z[IDX(X, Y, Z - 1)] * (g[b - (int64_t)bx * by] - gx);
                    if (k < bz - 1) acc += lam_z[IDX(X, Y, Z)]     * (g[b + (int64_t)bx * by] - gx);
                    if (nu_x) {
                        /* inflow through the lower face, outflow through the upper face */
                        double v;
                        if (i > 0)      { v = nu_x[IDX(X - 1, Y, Z)]; acc += v > 0.0 ? v * g[b - 1] : v * gx; }
                        if (i < bx - 1) { v = nu_x[IDX(X, Y, Z)];     acc -= v > 0.0 ? v * gx : v * g[b + 1]; }
                        if (j > 0)      { v = nu_y[IDX(X, Y - 1, Z)]; acc += v > 0.0 ? v * g[b - bx] : v * gx; }
                        if (j < by - 1) { v = nu_y[IDX(X, Y, Z)];     acc -= v > 0.0 ? v * gx : v * g[b + bx]; }
                        if (k > 0)      { v = nu_z[IDX(X, Y, Z - 1)]; acc += v > 0.0 ? v * g[b - (int64_t)bx * by] : v * gx; }
                        if (k < bz - 1) { v = nu_z[IDX(X, Y, Z)];     acc -= v > 0.0 ? v * gx : v * g[b + (int64_t)bx * by]; }
                    }
                    tmp[b] = (fixed && fixed[IDX(X, Y, Z)]) ? fval : acc;
                }
        memcpy(g, tmp, sizeof(double) * (size_t)bx * by * bz);
    }
}

static void window_box(int nx, int ny, int nz, int r, int sx, int sy, int sz, int lo[3], int hi[3])
{
    int s[3] = {sx, sy, sz}, n[3] = {nx, ny, nz};
    for (int a = 0; a < 3; ++a) {
        lo[a] = s[a] - r < 0 ? 0 : s[a] - r;
        hi[a] = s[a] + r > n[a] - 1 ? n[a] - 1 : s[a] + r;
    }
}

/* Window kernel of one source: the W^3 window kernel G_s (placed relative to
 * s - r, zeros outside the domain) and its mass.  work: 2 * W^3 doubles.
 * fixed (may be NULL): Dirichlet cells held at 0 (they absorb). */
static void kernel_one(int nx, int ny, int nz,
                       const double *lam_x, const double *lam_y, const double *lam_z,
                       int r, int n_sub, int64_t s, double *G, double *mass, double *work,
                       const uint8_t *fixed, const double *nu_x, const double *nu_y, const double *nu_z)
{
    int W = 2 * r + 1;
    int sx = (int)(s % nx), sy = (int)((s / nx) % ny), sz = (int)(s / ((int64_t)nx * ny));
    int lo[3], hi[3];
    window_box(nx, ny, nz, r, sx, sy, sz, lo, hi);
    int bx = hi[0] - lo[0] + 1, by = hi[1] - lo[1] + 1, bz = hi[2] - lo[2] + 1;
    int64_t nb = (int64_t)bx * by * bz;
    double *g = work, *tmp = work + nb;
    memset(g, 0, sizeof(double) * (size_t)nb);
    g[((int64_t)(sz - lo[2]) * by + (sy - lo[1])) * bx + (sx - lo[0])] = 1.0;
    box_substeps(nx, ny, nz, lam_x, lam_y, lam_z, lo, hi, n_sub, g, tmp, fixed, 0.0, nu_x, nu_y, nu_z);
    memset(G, 0, sizeof(double) * (size_t)W * W * W);
    for (int k = 0; k < bz; ++k)
        for (int j = 0; j < by; ++j)
            for (int i = 0; i < bx; ++i) {
                int wz = lo[2] + k - (sz - r), wy = lo[1] + j - (sy - r), wx = lo[0] + i - (sx - r);
                G[((int64_t)wz * W + wy) * W + wx] = g[((int64_t)k * by + j) * bx + i];
            }
    if (mass) *mass = neumaier_sum(g, nb);
}

/* Kernels of a list of sources: G [n_src][W][W][W], mass [n_src]; fixed (may
 * be NULL): Dirichlet cells held at 0; nu_* (may be NULL): flow Courant
 * numbers as in box_substeps. */
void fo_kernels_general(int nx, int ny, int nz,
                        const double *lam_x, const double *lam_y, const double *lam_z,
                        int r, int n_sub, const int64_t *src, int64_t n_src,
                        double *G, double *mass, const uint8_t *fixed,
                        const double *nu_x, const double *nu_y, const double *nu_z)
{
    int64_t W3 = (int64_t)(2 * r + 1) * (2 * r + 1) * (2 * r + 1);
#pragma omp parallel
    {
        double *work = (double *)malloc(sizeof(double) * 2 * W3);
#pragma omp for schedule(dynamic, 16)
        for (int64_t i = 0; i < n_src; ++i)
            kernel_one(nx, ny, nz, lam_x, lam_y, lam_z, r, n_sub, src[i],
                       G + i * W3, mass ? mass + i : NULL, work, fixed, nu_x, nu_y, nu_z);
        free(work);
    }
}

void fo_kernels_fixed(int nx, int ny, int nz,
                      const double *lam_x, const double *lam_y, const double *lam_z,
                      int r, int n_sub, const int64_t *src, int64_t n_src,
                      double *G, double *mass, const uint8_t *fixed)
{
    fo_kernels_general(nx, ny, nz, lam_x, lam_y, lam_z, r, n_sub, src, n_src, G, mass, fixed, NULL, NULL, NULL);
}

void fo_kernels(int nx, int ny, int nz,
                const double *lam_x, const double *lam_y, const double *lam_z,
                int r, int n_sub, const int64_t *src, int64_t n_src,
                double *G, double *mass)
{
    fo_kernels_fixed(nx, ny, nz, lam_x, lam_y, lam_z, r, n_sub, src, n_src, G, mass, NULL);
}

/* Superposition: c_new(x) = sum over sources s (ascending, c_old(s) != 0) of
 * c_old(s) * G_s(x), added in window z, y, x order.  Kernels are generated in
 * parallel in batches and added strictly in ascending source order, so the
 * result does not depend on the thread count.  Optional: kmass_minmax[2] =
 * min / max kernel mass over the sources used.  Returns the number of sources
 * used. */
int64_t fo_step(int nx, int ny, int nz,
                const double *lam_x, const double *lam_y, const double *lam_z,
                int r, int n_sub, const double *c_old, double *c_new,
                double *kmass_minmax)
{
    int64_t n = (int64_t)nx * ny * nz;
    int W = 2 * r + 1;
    int64_t W3 = (int64_t)W * W * W;
    memset(c_new, 0, sizeof(double) * (size_t)n);
    int64_t n_used = 0;
    for (int64_t s = 0; s < n; ++s) if (c_old[s] != 0.0) ++n_used;
    int64_t *src = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_used ? n_used : 1));
    int64_t q = 0;
    for (int64_t s = 0; s < n; ++s) if (c_old[s] != 0.0) src[q++] = s;

    const int64_t batch = 4096;
    double *G = (double *)malloc(sizeof(double) * (size_t)(batch * W3));
    double *mass = (double *)malloc(sizeof(double) * (size_t)batch);
    double mmin = INFINITY, mmax = -INFINITY;
    for (int64_t b0 = 0; b0 < n_used; b0 += batch) {
        int64_t nb = n_used - b0 < batch ? n_used - b0 : batch;
        fo_kernels(nx, ny, nz, lam_x, lam_y, lam_z, r, n_sub, src + b0, nb, G, mass);
        for (int64_t i = 0; i < nb; ++i) {
            int64_t s = src[b0 + i];
            int sx = (int)(s % nx), sy = (int)((s / nx) % ny), sz = (int)(s / ((int64_t)nx * ny));
            double cs = c_old[s];
            const double *g = G + i * W3;
            for (int wz = 0; wz < W; ++wz) {
                int Z = sz - r + wz;
                if (Z < 0 || Z >= nz) continue;
                for (int wy = 0; wy < W; ++wy) {
                    int Y = sy - r + wy;
                    if (Y < 0 || Y >= ny) continue;
                    for (int wx = 0; wx < W; ++wx) {
                        int X = sx - r + wx;
                        if (X < 0 || X >= nx) continue;
                        c_new[IDX(X, Y, Z)] += cs * g[((int64_t)wz * W + wy) * W + wx];
                    }
                }
            }
            if (mass[i] < mmin) mmin = mass[i];
            if (mass[i] > mmax) mmax = mass[i];
        }
    }
    if (kmass_minmax) { kmass_minmax[0] = mmin; kmass_minmax[1] = mmax; }
    free(G); free(mass); free(src);
    return n_used;
}

/* Test-only reference: the same explicit update on the whole domain, started
 * from c, for n_sub sub-steps (no-flux domain walls).  out may not alias c. */
void fo_global_fd(int nx, int ny, int nz,
                  const double *lam_x, const double *lam_y, const double *lam_z,
                  int n_sub, const double *c, double *out)
{
    int64_t n = (int64_t)nx * ny * nz;
    double *tmp = (double *)malloc(sizeof(double) * (size_t)n);
    int lo[3] = {0, 0, 0}, hi[3] = {nx - 1, ny - 1, nz - 1};
    memcpy(out, c, sizeof(double) * (size_t)n);
    box_substeps(nx, ny, nz, lam_x, lam_y, lam_z, lo, hi, n_sub, out, tmp, NULL, 0.0, NULL, NULL, NULL);
    free(tmp);
}

/* The same with Dirichlet cells (mask fixed, may be NULL) holding fval from
 * the start and an optional flow (nu_*, may be NULL). */
void fo_global_fd_general(int nx, int ny, int nz,
                          const double *lam_x, const double *lam_y, const double *lam_z,
                          int n_sub, const double *c, double *out, const uint8_t *fixed, double fval,
                          const double *nu_x, const double *nu_y, const double *nu_z)
{
    int64_t n = (int64_t)nx * ny * nz;
    double *tmp = (double *)malloc(sizeof(double) * (size_t)n);
    int lo[3] = {0, 0, 0}, hi[3] = {nx - 1, ny - 1, nz - 1};
    for (int64_t i = 0; i < n; ++i) out[i] = (fixed && fixed[i]) ? fval : c[i];
    box_substeps(nx, ny, nz, lam_x, lam_y, lam_z, lo, hi, n_sub, out, tmp, fixed, fval, nu_x, nu_y, nu_z);
    free(tmp);
}

void fo_global_fd_fixed(int nx, int ny, int nz,
                        const double *lam_x, const double *lam_y, const double *lam_z,
                        int n_sub, const double *c, double *out, const uint8_t *fixed, double fval)
{
    fo_global_fd_general(nx, ny, nz, lam_x, lam_y, lam_z, n_sub, c, out, fixed, fval, NULL, NULL, NULL);
}

/* Test-only reference: structural support of G_s, i.e. the window cells
 * reachable from s through faces with lambda > 0 inside the (clipped) window in
 * at most n_sub face crossings.  Breadth-first search; out [W^3] uint8. */
void fo_support(int nx, int ny, int nz,
                const double *lam_x, const double *lam_y, const double *lam_z,
                int r, int n_sub, int64_t s, uint8_t *out)
{
    int W = 2 * r + 1;
    int64_t W3 = (int64_t)W * W * W;
    int sx = (int)(s % nx), sy = (int)((s / nx) % ny), sz = (int)(s / ((int64_t)nx * ny));
    int lo[3], hi[3];
    window_box(nx, ny, nz, r, sx, sy, sz, lo, hi);
    int *depth = (int *)malloc(sizeof(int) * (size_t)W3);
    int64_t *queue = (int64_t *)malloc(sizeof(int64_t) * (size_t)W3);
    for (int64_t i = 0; i < W3; ++i) depth[i] = -1;
    memset(out, 0, (size_t)W3);
    int64_t head = 0, tail = 0;
    int64_t c0 = ((int64_t)r * W + r) * W + r;
    depth[c0] = 0;
    queue[tail++] = c0;
    while (head < tail) {
        int64_t w = queue[head++];
        out[w] = 1;
        if (depth[w] == n_sub) continue;
        int wx = (int)(w % W), wy = (int)((w / W) % W), wz = (int)(w / ((int64_t)W * W));
        int X = sx - r + wx, Y = sy - r + wy, Z = sz - r + wz;
        for (int dir = 0; dir < 6; ++dir) {
            int dx = (dir == 0) ? -1 : (dir == 1) ? 1 : 0;
            int dy = (dir == 2) ? -1 : (dir == 3) ? 1 : 0;
            int dz = (dir == 4) ? -1 : (dir == 5) ? 1 : 0;
            int X2 = X + dx, Y2 = Y + dy, Z2 = Z + dz;
            if (X2 < lo[0] || X2 > hi[0] || Y2 < lo[1] || Y2 > hi[1] || Z2 < lo[2] || Z2 > hi[2]) continue;
            double lam;
            if (dx) lam = lam_x[IDX(dx < 0 ? X2 : X, Y, Z)];
            else if (dy) lam = lam_y[IDX(X, dy < 0 ? Y2 : Y, Z)];
            else lam = lam_z[IDX(X, Y, dz < 0 ? Z2 : Z)];
            if (!(lam > 0.0)) continue;
            int64_t w2 = ((int64_t)(wz + dz) * W + (wy + dy)) * W + (wx + dx);
            if (depth[w2] >= 0) continue;
            depth[w2] = depth[w] + 1;
            queue[tail++] = w2;
        }
    }
    free(depth);
    free(queue);
}

int fo_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads used by the OpenMP loops from now on (timing on one core). */
void fo_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
