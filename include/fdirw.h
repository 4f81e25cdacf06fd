/*
 * fdirw.h -- C ABI of the MI355X (gfx950) FDiRW fast-diffusion library.
 *
 * The method (arXiv 2408.11376, Sec. 3.1, Eqs. 8-9): over one big time step
 * the concentration field is advanced by superposition, c(t + dt_big) = P c(t),
 * where column j of the proportion matrix P is the mass that a unit point
 * source at cell j spreads to every other cell.  The paper obtains each column
 * by an explicit finite-difference solution started from that point source
 * (Sec. 3.1, text after Eq. 9) and applies the matrix-vector product on the GPU
 * (Sec. 3.2), optionally with P stored in reduced precision and FP32
 * accumulation (Sec. 3.3).
 *
 * This library computes the columns on the fly, per source cell, on a local
 * window [s - r, s + r]^3 of the fine grid, and scatter-adds c(s) * G_s into
 * the new field:
 *   - explicit 7-point scheme, sub-step dt (given, or 0.9 h^2 / (6 Dmax));
 *   - face coefficient lambda_f = D_f dt / h^2 with D_f the harmonic mean
 *     2 Da Db / (Da + Db) of the two cells (0 if either is 0);
 *   - no flux through domain walls, impermeable (D = 0) cells or the window
 *     walls; cells of the window outside the domain hold 0;
 *   - superposition accumulated in FP64.
 *
 * Conventions for every entry point:
 *   - Grids are [nz][ny][nx] with x fastest; the linear index of (x, y, z) is
 *     (z*ny + y)*nx + x (int64).
 *   - Pointers are DEVICE pointers (memory of the current HIP device) unless
 *     marked (host).  All buffers belong to the caller; the library never frees
 *     them.  The library allocates only internal scratch (per device, grown on
 *     demand, released by fdirw_release()).
 *   - Work is enqueued on the given hipStream_t (NULL = the default stream).
 *     Argument checks that need the device (label range, Dmax) read a few
 *     bytes back, so each call synchronises the stream once at its start;
 *     passing a stats pointer synchronises again at the end.
 *   - Every function returns an fdirw_status and never throws or aborts; on a
 *     non-OK status nothing has been written to the outputs unless stated, and
 *     fdirw_last_error() returns a message (per calling thread).
 */
#ifndef FDIRW_H_
#define FDIRW_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FDIRW_ABI_VERSION 1
#define FDIRW_MAX_RADIUS 8   /* largest window radius r supported (W = 17) */
#define FDIRW_MAX_COARSE_RADIUS 128   /* largest r of the coarse operator (node windows beyond 8) */
#define FDIRW_MAX_COARSE_K 8          /* ... with ceil(r / block) at most this */
#define FDIRW_MAX_ENSEMBLE 4096       /* members of one ensemble coarse product */
#define FDIRW_MAX_PHASES 256

typedef enum fdirw_status {
    FDIRW_OK = 0,
    FDIRW_E_ARG = -1,          /* invalid argument (null, size, label range, aliasing) */
    FDIRW_E_UNSTABLE = -2,     /* 6 Dmax dt / h^2 > 1: explicit scheme unstable */
    FDIRW_E_NOMEM = -3,        /* internal scratch could not be allocated */
    FDIRW_E_DEVICE = -4,       /* a HIP call failed */
    FDIRW_E_UNSUPPORTED = -5,  /* valid request the library does not implement */
    FDIRW_E_NONFINITE = -6     /* non-finite input mass */
} fdirw_status;

/* Precision of the window stencil (Sec. 3.3 for the paper's FP32/FP16 split).
 *   FP64           state, coefficients and exchange in FP64.
 *   FP32           state, coefficients and exchange in FP32; kernels are
 *                  renormalised by their FP64 mass before the superposition
 *                  (FP32 rounding of 1 - sum(lambda) otherwise biases the mass
 *                  by ~1e-6 over 200 sub-steps).
 *   FP16X32/BF16X32  FP32 state and coefficients; neighbours exchange FP16 /
 *                  BF16 copies (round to nearest even) and every face flux is
 *                  formed from the two reduced copies, so the two cells of a
 *                  face see exactly opposite fluxes; kernels are renormalised
 *                  to unit mass before the superposition.
 *   FP16_STATE/BF16_STATE  the state itself is rounded to FP16/BF16 after
 *                  every sub-step (control case); renormalised.
 *   FP16_BANK/BF16_BANK    the kernel is generated in FP32 and rounded once to
 *                  FP16/BF16 (the paper's stored-P split); the superposition
 *                  uses the rounded kernel, scaled by its own mass.
 * In every mode the superposition c(s) * G_s and the mass sums are FP64. */
typedef enum fdirw_prec {
    FDIRW_FP64 = 0,
    FDIRW_FP32 = 1,
    FDIRW_FP16X32 = 2,
    FDIRW_BF16X32 = 3,
    FDIRW_FP16_STATE = 4,
    FDIRW_BF16_STATE = 5,
    FDIRW_FP16_BANK = 6,
    FDIRW_BF16_BANK = 7
} fdirw_prec;

typedef enum fdirw_gen {
    FDIRW_GEN_FD = 0,          /* explicit finite-difference window kernels */
    FDIRW_GEN_NN = 1           /* learned surrogate (fdirw_nn_*), audited against FD */
} fdirw_gen;

/* One domain (a phase map and the parameters of one big step). */
typedef struct fdirw_domain {
    int32_t nx, ny, nz;        /* cells per axis, each >= 1 */
    double h;                  /* grid spacing > 0 */
    const uint8_t *label;      /* N phase labels, each < n_phase */
    const double *d_phase;     /* (host) n_phase diffusivities, finite, >= 0 */
    int32_t n_phase;           /* 1..FDIRW_MAX_PHASES */
    int32_t r;                 /* window radius, 0..FDIRW_MAX_RADIUS (W = 2r + 1) */
    int32_t n_sub;             /* explicit sub-steps per big step, >= 0 (0: identity) */
    double dt;                 /* sub-step; <= 0 selects 0.9 h^2 / (6 Dmax) */
} fdirw_domain;

typedef struct fdirw_opts {
    int32_t prec;              /* fdirw_prec */
    int32_t gen;               /* fdirw_gen */
    const void *nn;            /* surrogate handle from fdirw_nn_create (GEN_NN) */
    double audit_tol;          /* GEN_NN: largest mean per-kernel L1 error accepted; <= 0: 1e-3 */
    int32_t audit_samples;     /* GEN_NN: sources audited per step; <= 0: 1024 */
    int32_t deterministic;     /* 0 or 1.  1: no floating-point atomics anywhere in the step;
                                  fdirw_step / fdirw_run results are a function of the inputs
                                  (bitwise equal on repeat, for n_dom > 1 and n_dom == 1 calls,
                                  and for a run resumed from its intermediate field).  The
                                  fused step then takes the source planes in slabs: per slab
                                  every source line stores its completed output planes to its
                                  own slot of a library-held buffer of W^2 (slab + 2r) nx ny
                                  doubles (slab chosen so that it stays <= 4 GiB, at least one
                                  plane), and a second pass adds the W^2 slots of each cell in
                                  a fixed order.  With n_dom > 1 the domains run in turn through
                                  that step instead of the persistent launch.  GEN_NN:
                                  E_UNSUPPORTED.  0: FP64 atomics (sums of ~1e-16 relative
                                  order-dependence). */
    size_t bank_budget_bytes;  /* fdirw_run: store every kernel once if the bank fits; 0 = never */
    void *stream;              /* hipStream_t, NULL = default stream */
    int32_t tune;              /* launch shape.  n_dom == 1: > 0 = segments per source line,
                                  else automatic; with deterministic = 1, > 0 = source planes
                                  per slab, else automatic.  n_dom > 1: batched shape id, 0..5 = the
                                  640-thread segment layout (item z extent whole / whole / 64 / 32 /
                                  16 / 8 planes; natural order for 0, longest first otherwise), 6..9
                                  = the 256-thread flat layout, FP32 only (one source line per item
                                  at r >= 7, two at r = 5, 6 and r = 3, four at r = 4 and r <= 2;
                                  z extent whole / 64 / 32 / 16, longest first; E_ARG for another
                                  precision), -1 = autotuned (cached per precision,
                                  radius / sub-step mix, size class and device; the cache file is
                                  named by the environment variable FDIRW_TUNE_CACHE) */
} fdirw_opts;

typedef struct fdirw_stats {
    double mass_in;            /* compensated FP64 sum of c_in */
    double mass_out;           /* compensated FP64 sum of c_out */
    double kmass_min;          /* min / max mass of the kernels generated (before any */
    double kmass_max;          /*   renormalisation); +inf / -inf if none */
    double audit_l1;           /* surrogate audit statistic (0 with GEN_FD) */
    double seconds;            /* wall time of the call, synchronised */
    int32_t fallback_used;     /* surrogate fell back to FD (0 with GEN_FD) */
    int32_t tuned_config_id;   /* launch shape used */
    int64_t n_sources;         /* sources processed (cells with c != 0) */
    int32_t bank_used;         /* fdirw_run applied a stored kernel bank */
    int32_t reserved;
    double kernel_seconds;     /* device time of the main kernel of the (last) step,
                                  from HIP events recorded around its launch */
} fdirw_stats;

/* Coefficients.  Writes lam[0*N + i], lam[1*N + i], lam[2*N + i] =
 * the FP64 coefficient of the face from cell i to its +x, +y, +z neighbour
 * (0 on the last plane of that axis and for faces touching an impermeable
 * cell), and *dt_out (host, may be NULL) = the sub-step used.  lam: 3N doubles.
 * Errors: E_ARG (null, sizes, label >= n_phase, negative or non-finite D),
 * E_UNSTABLE. */
int fdirw_coefficients(const fdirw_domain *d, void *stream, double *lam, double *dt_out);

/* The window kernels of n_src sources (Sec. 3.1: column s of P
 * is the response to a unit point source at s).  src: n_src int64 linear
 * indices, each in [0, N).  G: [n_src][W][W][W] ordered z, y, x relative to
 * s - r, doubles for FDIRW_FP64 and floats otherwise; cells outside the domain
 * are 0.  G is the kernel as generated (in the BANK modes: rounded to FP16 /
 * BF16 and widened), before any renormalisation.  mass (may be NULL): n_src
 * doubles, the FP64 sum of each kernel.  Every mode except FP64 superposes
 * G / mass, so fdirw_step with c = e_s yields exactly (1 / mass) * G (FP64
 * product) placed at s.
 * Errors: E_ARG (also: a source index out of range), E_UNSTABLE. */
int fdirw_kernels(const fdirw_domain *d, const fdirw_opts *o, const int64_t *src, int64_t n_src,
                  void *G, double *mass);

/* Window kernels with a steady flow (the extension of P to diffusion with a
 * steady flow, Sec. 5): the explicit update of fdirw_kernels plus a
 * first-order upwind advective flux through every face, Courant number
 * nu_f = u_f dt / h; a face that leaves the window or the domain carries
 * neither diffusion nor flow.  velocity: 3N doubles, u on the face from cell i
 * to its +x, +y, +z neighbour (entries of the last plane of each axis are not
 * read), in units of h per unit time, positive towards +x / +y / +z.  prec:
 * FP64 or FP32 (E_UNSUPPORTED otherwise).  G and mass as in fdirw_kernels;
 * the kernels are not renormalised.  Errors: E_ARG, E_UNSUPPORTED,
 * E_UNSTABLE (also when 6 lambda + the outflow Courant numbers of a cell
 * exceed 1). */
int fdirw_kernels_flow(const fdirw_domain *d, const fdirw_opts *o, const double *velocity, const int64_t *src,
                       int64_t n_src, void *G, double *mass);

/* One big step of the superposition (Eq. 8, column form):
 * c_out[i][x] = sum over s of c_in[i][s] * G_s(x) for each domain i.  d, c_in,
 * c_out and st are (host) arrays of n_dom entries; c_in[i] and c_out[i] point
 * to N_i doubles and must not overlap (E_ARG).  st may be NULL.  n_dom > 1
 * runs all domains in one persistent launch.
 * With gen = GEN_NN (n_dom must be 1, else E_UNSUPPORTED; r and n_sub must
 * match the surrogate, else E_ARG) the kernels come from the surrogate o->nn:
 * first audit_samples seeded sources are generated both ways (surrogate and
 * FP32 FD) and the mean of sum |G_nn - G_fd| over them is compared with
 * audit_tol; above it the step falls back to the FD step in precision o->prec
 * (st->fallback_used = 1); else every kernel is the surrogate's, superposed
 * as G / sum(G) in FP64.  st->audit_l1 holds the audit mean in both cases. */
int fdirw_step(const fdirw_domain *d, int32_t n_dom, const fdirw_opts *o,
               const double *const *c_in, double *const *c_out, fdirw_stats *st);

/* fdirw_step for one domain without allocating: for callers that cannot
 * allocate device memory (code under HIP graph capture, serving loops,
 * harnesses that forbid hipMalloc).  It calls no hipMalloc / hipFree and no
 * allocating library routine, and creates no events.  The result is that of
 * fdirw_step with n_dom = 1 (same kernels and arithmetic; the face
 * coefficients are looked up per phase pair instead of being stored per
 * cell, same values), up to the order of the FP64 atomic additions.
 *
 * Scratch: one statically sized device array of FDIRW_NOALLOC_SCRATCH_BYTES
 * per GPU, held from the library's first use on that GPU until the process
 * ends: flags, counters, reduction partials, the n_phase^2 coefficient table
 * and, when st != NULL, one kernel-mass pair per workgroup.  All calls on one
 * GPU share it and it keeps the last call's contents (every part a call reads
 * is rewritten or cleared by that call first), so calls that overlap in time
 * on one GPU (two host threads, or two streams whose work overlaps) race.
 * The call synchronises o->stream once (label check and Dmax) and again
 * for the statistics.
 *
 * Limits and errors: as fdirw_step (E_ARG, E_UNSTABLE, E_NONFINITE, E_DEVICE);
 * E_UNSUPPORTED for GEN_NN, deterministic = 1, or a precision other than
 * FP64, FP32, FP16X32, BF16X32; E_ARG when st != NULL and the launch has more
 * than FDIRW_NOALLOC_MAX_BLOCKS workgroups (nx * ny * segments per line,
 * i.e. nx * ny above FDIRW_NOALLOC_MAX_BLOCKS), or c_in == c_out.
 * st->kernel_seconds is 0 (no events). */
#define FDIRW_NOALLOC_SCRATCH_BYTES (2 << 20)
#define FDIRW_NOALLOC_MAX_BLOCKS 65536
int fdirw_step_noalloc(const fdirw_domain *d, const fdirw_opts *o, const double *c_in, double *c_out,
                       fdirw_stats *st);

/* n_steps big steps (the time marching of
 * Eq. 8).  c[i] holds the initial field and receives the final one;
 * scratch[i] is a second buffer of N_i doubles (its content is overwritten).
 * With n_dom == 1 and bank_budget_bytes allowing, every kernel is generated
 * once and each step applies the stored bank (P is fixed for a fixed
 * geometry, Sec. 3.1 and 5); n_dom > 1 runs one batched launch per step.
 * st (may be NULL) receives the statistics of the last step, with seconds
 * covering the whole call. */
int fdirw_run(const fdirw_domain *d, int32_t n_dom, const fdirw_opts *o, int32_t n_steps,
              double *const *c, double *const *scratch, fdirw_stats *st);

/* Compensated (Neumaier per thread, two-sum tree) FP64 sum of n
 * doubles, in a fixed order for a given n.  *sum_out is host memory. */
int fdirw_field_sum(const double *c, int64_t n, void *stream, double *sum_out);

/* ------------------------------------------------------------------ surrogate
 * A learned generator of window kernels (an extension: the
 * paper obtains every column of P by FD from a point source, Sec. 3.1).  For a
 * source s with window radius FDIRW_NN_RADIUS (W = 17) the network reads three
 * features per window cell (permeable-and-in-domain flag; (max(log10 D, -12)
 * + 6) / 6 inside the domain, -1 outside; the prior log U / 20, U the FD kernel
 * of an all-permeable window with lambda = 0.15 on every face), applies five
 * 3x3x3 convolutions with zero padding (3 -> 16 -> 16 -> 16 -> 16 -> 1
 * channels, SiLU after the first four; BF16 operands on MFMA, FP32
 * accumulation) and returns G = softmax over the structural support (cells
 * reached from s in at most n_sub crossings of faces whose two cells are in
 * the domain with D > 0) of log U + network output; G is 0 elsewhere.
 * Parameters: one flat FP32 vector of fdirw_nn_num_params() values, per layer
 * w[co][ci][3][3][3] (taps z, y, x) then b[co].
 * A handle belongs to the device current at creation; every call must be made
 * with that device current (E_ARG otherwise).  Handles are not thread-safe
 * against each other's use of the same handle. */
#define FDIRW_NN_RADIUS 8

/* Number of parameters (22,529). */
int64_t fdirw_nn_num_params(void);

/* Creates a surrogate for windows of FDIRW_NN_RADIUS and n_sub sub-steps
 * (the prior and the support depth depend on n_sub).  Parameters start from
 * a deterministic He-normal draw of `seed` (last layer scaled by 0.1, zero
 * biases); Adam moments start at 0.  *nn receives the handle.
 * Errors: E_ARG, E_NOMEM, E_DEVICE. */
int fdirw_nn_create(int32_t n_sub, uint64_t seed, void **nn);

/* Frees the handle and its device memory (NULL is accepted). */
int fdirw_nn_destroy(void *nn);

/* Copies the parameters in / out; theta is (host) memory of
 * fdirw_nn_num_params() floats.  Setting resets nothing else. */
int fdirw_nn_set_params(void *nn, const float *theta);
int fdirw_nn_get_params(const void *nn, float *theta);

/* Surrogate kernels of n_src sources of domain d (d->r must be
 * FDIRW_NN_RADIUS and d->n_sub the handle's).  src: n_src int64 linear
 * indices in [0, N).  Outputs (each may be NULL), [n_src][W][W][W] in z, y, x
 * order relative to s - r: G (float, unit mass up to FP32 rounding),
 * support (uint8 0 / 1), logits (float, log U + network output, every cell).
 * Errors: E_ARG (also: a source or label out of range), E_UNSTABLE. */
int fdirw_nn_forward(void *nn, const fdirw_domain *d, const int64_t *src, int64_t n_src, float *G,
                     uint8_t *support, float *logits, void *stream);

/* Loss and gradient over n_src >= 1 windows: loss = mean over windows of
 * KL(q || G) + sum |q - G| over the support, q = target / sum(target).
 * target: [n_src][W][W][W] floats, or NULL to use the FP32 FD kernels of the
 * sources (generated here).  grad (may be NULL): fdirw_nn_num_params() floats
 * receiving d loss / d parameters; the gradient is also kept in the handle for
 * fdirw_nn_adam.  loss (host, may be NULL): 2 doubles, the mean KL and the
 * mean L1 term.  Synchronises the stream.  Errors as fdirw_nn_forward. */
int fdirw_nn_backward(void *nn, const fdirw_domain *d, const int64_t *src, int64_t n_src, const float *target,
                      float *grad, double *loss, void *stream);

/* One Adam step (Kingma and Ba 2015, bias-corrected) on the FP32 parameters
 * with the gradient of the last fdirw_nn_backward.  Errors: E_ARG. */
int fdirw_nn_adam(void *nn, double lr, double beta1, double beta2, double eps, void *stream);

/* Writes / reads the parameters, Adam moments and step count to / from a
 * little-endian binary file.  load checks the file's n_sub against the
 * handle's.  Errors: E_ARG (I/O, format), E_DEVICE. */
int fdirw_nn_save(const void *nn, const char *path);
int fdirw_nn_load(void *nn, const char *path);

/* ------------------------------------------------------------------ coarse mesh
 * Coarse-mesh FDiRW (Sec. 3.1, Eqs. 10-15): the fine grid is cut into blocks
 * of `block`^3 cells (ragged at the far edges); the grouped cells (those of the
 * fast, liquid phases) of block I form group I with N_I cells, whose
 * representative node carries the mean concentration C_I.  Cells of the other
 * phases keep their value (the paper maps the liquid nodes only).
 * One coarse big step is
 *   mapping (Eq. 13)    C_J = mean of c_in over group J
 *   FDiRW (Eq. 14)      C'_I = sum_J P[I][J] C_J
 *   remapping (Eq. 15)  c_out(i) = C'_I for every cell i of group I
 * with P[I][J] = (1 / N_I) sum over grouped sources j of group J and cells i
 * of group I of G_j(i) / m_j, G_j the fine window kernel of fdirw_kernels
 * (radius d->r, d->n_sub sub-steps) and m_j its mass over the grouped cells:
 * the share of group J's mass that the big step moves into group I, as a
 * concentration ratio (columns conserve mass exactly).  P is
 * nonzero only for |I - J| <= K = ceil(r / block) per axis and is stored
 * offset-major in the precision `prec`; the product and its sum are FP64.
 * With block = 1 and the default grouping the step is the fine step with
 * renormalised kernels.
 * Node windows: for d->r above FDIRW_MAX_RADIUS (up to
 * FDIRW_MAX_COARSE_RADIUS, with K = ceil(r / block) <= FDIRW_MAX_COARSE_K)
 * the column of group J is instead one FD of unit mass on every grouped cell
 * of J, on the window made of J's block and the K blocks around it (clipped
 * at the domain, walls at its faces), scaled to N_J over the grouped cells
 * (not scaled with a far field): by linearity the sum of the point-source
 * kernels of J's cells on that shared window; with block = 1 it is the
 * point-source window of radius r.  Its state lives in HBM (batches of
 * nodes, one launch per sub-step).
 * Far field (Eqs. 7, 8, 10, 14): cells of the reservoir phases are the
 * far-field boundary, Dirichlet cells holding the uniform far-field
 * concentration c_ff.  Their handle builds P from kernels in which those cells
 * absorb (held at 0), not renormalised, and P_BC[I] = the mean over group I
 * of the whole-domain FD response to a unit concentration held on them; a
 * step is C' = P C + P_BC c_ff, the remapping, and then Eq. 7:
 * c_ff' = (m_total - sum of c_out over the other cells) / v_ff.  Without
 * reservoir phases the far-field term is zero (no-flux domain walls). */

/* Builds the coarse operator of domain d (generating every fine kernel once,
 * FP64 for prec = FDIRW_FP64, FP32 otherwise; P stored as FP64, FP32,
 * FP16 (FDIRW_FP16_BANK) or BF16 (FDIRW_BF16_BANK)).  grouped (host, may be
 * NULL): d->n_phase flags, nonzero for the grouped phases; NULL groups every
 * phase with D > 0.  reservoir (host, may be NULL): d->n_phase flags, nonzero
 * for the far-field boundary phases (never grouped).  velocity (may be NULL):
 * a steady flow as in fdirw_kernels_flow; P and P_BC then include it (the
 * kernels are the flow kernels, generated in chunks of sources; r <= 8 only).  block: 1..256.  d->label is read
 * only here.  *handle
 * receives a handle owning device memory of about 4 N + (2K+1)^3 x N_nodes x
 * element bytes (for K >= 5 N_nodes counts only the nodes of the 16-byte z
 * groups of P that hold a grouped cell; the build also holds (2K+1)^3 x
 * N_nodes x 8 bytes for its duration); seconds (host, may be NULL) receives
 * the build time.
 * Synchronises the stream.  The handle belongs to the current device.
 * Errors: E_ARG (also a block outside 1..256, another precision or K above
 * FDIRW_MAX_COARSE_K), E_UNSUPPORTED (a flow with r above FDIRW_MAX_RADIUS),
 * E_UNSTABLE, E_NOMEM, E_DEVICE. */
int fdirw_coarse_create(const fdirw_domain *d, int32_t block, int32_t prec, const uint8_t *grouped,
                        const uint8_t *reservoir, const double *velocity, void *stream, void **handle,
                        double *seconds);

/* Arithmetic of the coarse product (the precisions compared in Sec. 3.3
 * and Table 2; the mapping and remapping stay FP64, the group means are
 * rounded to the C type):
 *   FP64   C, products and sums in FP64 (the default; P of any storage)
 *   FP32   C in FP32, fused FP32 multiply-adds (P stored in FP32)
 *   MIXED  the paper's FP32/FP16 scheme: C rounded to FP32 and then FP16,
 *          each product P[I][J] C_J taken in FP16 (P stored in FP16), the
 *          products accumulated in FP32
 *   FP16   as MIXED with the products accumulated in FP16
 * The far-field term P_BC c_ff is formed as one more product.  The result is
 * widened to FP64 for the remapping. */
enum {
    FDIRW_COARSE_ARITH_FP64 = 0,
    FDIRW_COARSE_ARITH_FP32 = 1,
    FDIRW_COARSE_ARITH_MIXED = 2,
    FDIRW_COARSE_ARITH_FP16 = 3
};

/* Selects the arithmetic of the handle's later steps (allocates the reduced
 * C grid on first use, synchronously).  Errors: E_ARG (unknown id, or a P
 * storage the arithmetic does not take), E_NOMEM, E_DEVICE. */
int fdirw_coarse_set_arith(void *handle, int32_t arith);

/* One coarse big step from c_in to c_out (N doubles each, not overlapping).
 * st (may be NULL) receives mass_in / mass_out (compensated FP64 sums, one
 * synchronisation each), n_sources = number of nodes, tuned_config_id =
 * block and kernel_seconds = device time of mapping + product + remapping.
 * Errors: E_ARG (null, overlap, another device, a handle with a far field),
 * E_DEVICE. */
int fdirw_coarse_step(void *handle, const double *c_in, double *c_out, void *stream, fdirw_stats *st);

/* One coarse big step with the far field (handle created with reservoir
 * phases).  *c_ff (host, in / out): the far-field concentration of the step's
 * start, replaced by the Eq. 7 value, which is also written into the
 * far-field cells of c_out; m_total: the conserved total (sum of c over the
 * cells outside the far field plus c_ff * v_ff at the start of the run);
 * v_ff > 0: the far-field volume in cell units.  st (may be NULL): mass_in =
 * m_total, mass_out = the same total after the step, kernel_seconds.
 * Synchronises the stream.  Errors: E_ARG, E_NONFINITE, E_DEVICE. */
int fdirw_coarse_step_far_field(void *handle, const double *c_in, double *c_out, double *c_ff, double m_total,
                                double v_ff, void *stream, fdirw_stats *st);

/* Ensemble form of the coarse product (Eq. 14 with n_ens right-hand sides,
 * in the mixed FP32/FP16 precision of Sec. 3.3, on the matrix cores):
 * C_out[e] = P C_in[e] for e < n_ens.  C_in, C_out: device, n_ens x n_nodes
 * doubles each, member-major, nodes numbered as in fdirw_coarse_shape; not
 * overlapping.  Every C value is rounded to FP32, scaled by the power of two
 * that brings its member's largest |C| into [2^14, 2^15) and rounded to FP16;
 * P is the handle's FP16 P scaled the same way by its largest entry; scaled
 * operands below 2^-14 (the smallest normal FP16 number) are taken as 0.  Each
 * product of two FP16 numbers is exact and the products of a node are summed
 * in FP32 (in an order the matrix unit fixes; within gamma_n(2^-23) sum |terms|
 * of the exact sum), scaled back exactly and widened to FP64.  Nodes without
 * grouped cells get 0.  A member holding a non-finite value gives non-finite
 * results for that member.  P is read
 * once per call for all members (as matrix fragments built from it on the
 * first call, about 10 KB per 16 nodes at K = 2, kept by the handle); the
 * padded FP16 grids of the members (grown on demand, kept) are written by
 * every call.  Stream-ordered on `stream`; calls on one handle that overlap
 * on different streams race.  kernel_seconds (host, may be NULL): device
 * time of the call (synchronises the stream).
 * Errors: E_ARG (null, overlap, n_ens outside 1..FDIRW_MAX_ENSEMBLE, P not
 * stored in FP16, a handle with a far field, another device), E_UNSUPPORTED
 * (K above 4), E_NOMEM, E_DEVICE. */
int fdirw_coarse_apply_ensemble(void *handle, const double *C_in, double *C_out, int32_t n_ens, void *stream,
                                double *kernel_seconds);

/* Copies P_BC (host, n_nodes doubles; zeros without a far field). */
int fdirw_coarse_pbc(void *handle, double *pbc_host);

/* shape5 (host, may be NULL) = {ncz, ncy, ncx, K, block}; *n_nodes (host,
 * may be NULL) = ncz * ncy * ncx, nodes numbered (bz * ncy + by) * ncx + bx. */
int fdirw_coarse_shape(const void *handle, int32_t *shape5, int64_t *n_nodes);

/* Copies P widened to FP64 into P_host (host, (2K+1)^3 x n_nodes doubles):
 * P_host[o * n_nodes + I] = P[I][J] with J = I - (oz - K, oy - K, ox - K),
 * o = (oz * (2K+1) + oy) * (2K+1) + ox (0 where J is outside the grid or a
 * group is empty).  Synchronous.  Errors: E_ARG, E_DEVICE. */
int fdirw_coarse_matrix(void *handle, double *P_host);

/* Frees the handle (NULL is accepted). */
int fdirw_coarse_destroy(void *handle);

/* ------------------------------------------------------------------ integrated solver
 * The near-field solver of a porous particle in a waste solution (Sec. 2,
 * Eqs. 1-7; flowchart of Sec. 3.4).  Every phase has a role: near-field liquid
 * (fast diffusion), solid (slow diffusion) or far-field liquid (the uniform
 * reservoir of Eq. 7, held in its cells as a Dirichlet boundary).  One field c
 * holds the liquid concentration in liquid cells and the solid concentration
 * in solid cells.  Inside a phase A_m and c_m^eq are constant, so Eq. 1 with
 * Eqs. 2-3 is a diffusion with coefficient D_m A_m / RT; the two media meet
 * only through the interface reaction.  One big step dt = n_sub * d->dt runs,
 * in the flowchart's order:
 *   1. fast diffusion: the coarse far-field step (fdirw_coarse_step_far_field)
 *      of the near-field liquid, its kernels walled by the solid, with
 *      P_BC c_ff of the step's start; solid cells keep their value
 *   2. absorption (Eqs. 4-6): for every face between a near-field liquid cell
 *      and a solid cell, d c_S / dt = k f_L f_S = -d c_L / dt integrated
 *      exactly over dt for the pair: with a = c_L - c_L^eq, b = c_S^eq - c_S
 *      and d = (b - a) k dt / (c_L^eq c_S^eq), the liquid cell gives
 *      a b (e^d - 1) / (b e^d - a) to the solid cell (nothing while a <= 0);
 *      the faces go in six groups in which no cell appears twice: x faces
 *      between cells 2i and 2i+1, then 2i+1 and 2i+2, then y, then z
 *   3. slow diffusion: n_sub_solid explicit sub-steps of dt / n_sub_solid in
 *      the solid, harmonic-mean faces between solid cells, liquid cells walls
 *   4. far field (Eq. 7): c_ff = (m_total - Q_L - Q_S) / v_ff, Q_L and Q_S
 *      the sums of c over the near-field liquid and the solid cells, written
 *      into the far-field cells.
 * Steps run on the stream without host synchronisation (c_ff stays on the
 * device between them). */
enum { FDIRW_ROLE_LIQUID = 0, FDIRW_ROLE_SOLID = 1, FDIRW_ROLE_FAR_FIELD = 2 };

typedef struct {
    const uint8_t *role;       /* (host) d->n_phase roles, FDIRW_ROLE_*                        */
    const double *a_over_rt;   /* (host) d->n_phase values of A_m / RT (Eqs. 2-3), finite and
                                  >= 0; NULL: 1 for every phase                              */
    double k;                  /* rate constant of Eq. 4 (per unit time of d->dt), >= 0     */
    double c_eq_liquid;        /* c_L^eq of Eq. 5, > 0                                      */
    double c_eq_solid;         /* c_S^eq of Eq. 6, > 0                                      */
    int32_t n_sub_solid;       /* explicit solid sub-steps per big step, >= 1               */
    double v_far_field;        /* V_L^far-field of Eq. 7 in cell volumes, > 0               */
} fdirw_mp_params;

/* Builds the solver of domain d: d->d_phase holds D_m per phase, d->dt > 0
 * the fast sub-step, d->n_sub the fast sub-steps of one big step, d->r the
 * window radius of the liquid kernels; block and prec as in
 * fdirw_coarse_create (the liquid's coarse operator, with the near-field
 * liquid phases grouped and the far-field phases as reservoir).  Checks the
 * explicit limits 6 max(D A / RT) d->dt / h^2 <= 1 over the liquid phases and
 * 6 max(D A / RT) (dt / n_sub_solid) / h^2 <= 1 over the solid phases.  Lists
 * once the interface faces, the active cells (near-field liquid and solid)
 * and the solid cells with their face coefficients; a step then touches the
 * active cells only, and the far-field cells once per fdirw_mp_step call.
 * d->label is read only here; N must be below 2^31.  *handle owns about 8 N
 * bytes (a second field) plus 4 bytes per active cell, 88 per solid cell and
 * 8 per interface face besides the coarse operator; seconds (host, may be
 * NULL) receives the build time.  Synchronises the stream.
 * Errors: E_ARG, E_UNSTABLE, E_NOMEM, E_DEVICE. */
int fdirw_mp_create(const fdirw_domain *d, const fdirw_mp_params *p, int32_t block, int32_t prec, void *stream,
                    void **handle, double *seconds);

/* n_steps >= 0 big steps on c (device, N doubles, in place).  *c_ff (host, in /
 * out): the far-field concentration at the start, replaced by the value after
 * the last step; m_total: the conserved total Sum c_{S+L}(t0) of Eq. 7 (sum
 * over the non-far-field cells plus c_ff v_ff at the start of the run).
 * history (host, may be NULL): n_steps rows of {Q_L, Q_S, c_ff} after each
 * step.  st (may be NULL): mass_in = m_total, mass_out = Q_L + Q_S + c_ff v_ff
 * after the last step, kernel_seconds = device time of the steps, seconds.
 * Synchronises the stream once at the end.  The handle's scratch is shared by
 * its calls: calls on one handle must not overlap.
 * Errors: E_ARG (null, another device), E_NONFINITE, E_NOMEM, E_DEVICE. */
int fdirw_mp_step(void *handle, double *c, double *c_ff, double m_total, int32_t n_steps, double *history,
                  void *stream, fdirw_stats *st);

/* Number of interface faces (host, may be NULL) and the coarse handle of the
 * liquid step (owned by the solver; valid while it lives). */
int fdirw_mp_info(const void *handle, int64_t *n_faces, void **coarse);

/* Frees the solver (NULL is accepted). */
int fdirw_mp_destroy(void *handle);

/* Message describing the last non-OK status returned on this thread. */
const char *fdirw_last_error(void);

/* Frees the internal scratch of every device. */
int fdirw_release(void);

int fdirw_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* FDIRW_H_ */
