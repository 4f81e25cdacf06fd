// fdirw_launch.h -- host-visible launchers of the FDiRW kernels (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fdirw {

struct CoefTable {
    double d[256];            // diffusivity per phase label
};

// Coefficients: lx points to 3*n values of the stencil precision laid out as
// [lam_x | lam_y | lam_z], each [nz][ny][nx].
struct LineArgs {
    int nx, ny, nz;
    int64_t n;
    int n_sub;
    int z_begin, z_end;       // source planes of this launch
    int seg_len, n_seg;       // each (x, y) line of sources is cut into n_seg segments
    const void *lx;
    const double *c_in;
    double *c_out;            // null in the deterministic form
    double *wg_kmass;         // [n_blocks][2] min / max kernel mass, or null
    unsigned long long *n_used;
    // Deterministic form (n_seg == 1): instead of adding its completed planes
    // to c_out, the line of source column (sx, sy) stores window column
    // col = cy W + cx of plane Z to part[(col * part_planes + Z - part_z0) *
    // nx ny + y nx + x] (zeros included), one writer per entry.
    double *part;
    int part_z0, part_planes;
    // Coefficients by phase pair (launch_line_labels only): the face between
    // a cell of phase a and its + neighbour of phase b is lam_tab[a * n_phase
    // + b] (double in FP64 mode, float otherwise); lx is not read.
    const uint8_t *label;
    const void *lam_tab;
    int n_phase;
};

// Deterministic superposition, second pass: for every cell of planes
// [z_lo, z_hi) c_out += sum of the W^2 partials whose source line lies in the
// domain, in window-column order.
hipError_t launch_line_reduce(int r, const LineArgs &a, int z_lo, int z_hi, hipStream_t st);
// The fused step reading its coefficients through a.label / a.lam_tab
// (modes FP64, FP32, FP16X32, BF16X32).
hipError_t launch_line_labels(int mode, int r, const LineArgs &a, hipStream_t st);

struct WindowArgs {
    int nx, ny, nz;
    int64_t n;
    int n_sub;
    const void *lx;
    const int64_t *src;       // null: sources 0 .. n_src-1
    int64_t n_src;
    void *G;
    double *mass;
    int normalize;            // renormalising modes: write G / mass instead of G
    int out_lp;               // BANK modes: write the 16-bit rounded values
    int offset_major;         // store as the bank [W^3][z/zb][y][x][z%zb] (zb = 16 B / element):
                              // P[o][s + o] = G_s(o); cells outside the domain are skipped
};

// Apply a stored kernel bank in the row form c'(x) = sum_o P[o][x] c^(x - o).
struct BankArgs {
    int nx, ny, nz;
    int64_t n;
    const void *bank;         // offset-major bank (bank_elems() elements of the bank type)
    const double *mass;       // [N] kernel mass (renormalising modes)
    const double *c_in;
    double *c_out;            // every cell written
    double *chat;             // scratch of bank_chat_elems() doubles
};

// Coarse-mesh FDiRW (fdirw_coarse.hip).
struct CoarseTable {
    uint8_t mobile[256];      // 1 if the phase is grouped (a fast phase)
    uint8_t reservoir[256];   // 1 if the phase is the far-field boundary (Dirichlet cells)
};

// node[] values of the cells that are in no group.
constexpr int COARSE_OUTSIDE = -1;     // keeps its value
constexpr int COARSE_RESERVOIR = -2;   // far-field boundary cell

struct CoarseGenArgs {
    int nx, ny, nz;
    int64_t n;
    int n_sub;
    const void *lx;           // coefficients as in LineArgs
    const int *node;          // [N] node (block) index of a grouped cell, else COARSE_OUTSIDE / _RESERVOIR
    int block, K;             // block edge B, offset reach K = ceil(r / B)
    int ncx, ncy;             // coarse grid (x, y extents)
    int64_t n_nodes;
    double *S;                // [(2K+1)^3][n_nodes] sums of renormalised kernels, 0 at launch
};

// Window kernels with a steady flow (fdirw_flow.hip).
struct FlowArgs {
    int nx, ny, nz;
    int64_t n;
    int n_sub;
    const void *lam;          // [3][N] face coefficients (double for FP64, else float)
    const double *u;          // [3][N] flow on the owned +x, +y, +z faces (h per unit time)
    double dt, h;             // Courant number = u dt / h
    const int64_t *src;       // sources, or null: src_base + 0 .. n_src-1
    int64_t src_base;
    int64_t n_src;
    const int *node;          // coarse node index per cell (skips and far-field sinks), or null
    void *G;                  // [n_src][W^3] of the state type, or null
    double *mass;             // [n_src], or null
};

// Batched persistent launch (fdirw_batched.hip).
struct BatchDom {
    int nx, ny, nz, r, n_sub;
    int64_t n;
    const void *lam;          // [3][n] coefficients of the stencil precision
    const double *c_in;
    double *c_out;
    unsigned long long *n_used;
};

struct BatchItem {
    int dom;                  // domain index
    int line0, nlines;        // source lines (y * nx + x) line0 .. line0 + nlines - 1
    int z0, z1;               // source planes z0 .. z1 - 1
};

struct BatchArgs {
    const BatchDom *doms;
    const BatchItem *items;
    int n_items;
    unsigned *head;           // work counter, 0 at launch
    double *item_kmass;       // [n_items][2] kernel-mass range, or null
};

hipError_t launch_batched(int mode, const BatchArgs &a, int grid, hipStream_t st);
hipError_t batched_occupancy(int mode, int *blocks);
// The batched launch with the flat layout (FP32; items of one line each).
hipError_t launch_batched_flat(const BatchArgs &a, int grid, hipStream_t st);
hipError_t batched_flat_occupancy(int *blocks);
// Source lines one flat-layout workgroup runs side by side at radius r
// (4 at r = 4, 2 at r = 5 and 6, 1 at r = 7 and 8).
int flat_lines_per_group(int r);
int batch_windows_per_group(int r);

hipError_t launch_validate(const uint8_t *label, int64_t n, int n_phase, unsigned *out, hipStream_t st);
// tab[a * n_phase + b] = coefficient of a face between phases a and b
// (t64 and / or t32 may be null).
hipError_t launch_pair_table(const CoefTable &tab, int n_phase, double dt, double h, double *t64, float *t32,
                             hipStream_t st);
hipError_t launch_coef(const uint8_t *label, int nx, int ny, int nz, const CoefTable &tab,
                       double dt, double h, double *lam64, float *lam32, hipStream_t st);
hipError_t launch_line(int mode, int r, const LineArgs &a, hipStream_t st);
// Flat-layout fused step (FP32, r = 4..8, atomic superposition only), with
// the coefficients of a.lx or looked up per phase pair (a.label, a.lam_tab).
hipError_t launch_line_flat(int mode, int r, const LineArgs &a, hipStream_t st);
hipError_t launch_line_flat_labels(int mode, int r, const LineArgs &a, hipStream_t st);
hipError_t launch_window(int mode, int r, const WindowArgs &a, hipStream_t st);
hipError_t launch_bank_apply(int prec, int r, const BankArgs &a, hipStream_t st);
int64_t bank_chat_elems(int nx, int ny, int nz, int r);
hipError_t launch_bank_gather(int prec, int r, const BankArgs &a, hipStream_t st);   // a.chat given
hipError_t launch_coarse_nodes(const uint8_t *label, const CoarseTable &tab, int nx, int ny, int nz, int B,
                               int ncx, int ncy, int *node, double *count, hipStream_t st);
hipError_t launch_coarse_window(int fp64, int sink, int r, const CoarseGenArgs &a, hipStream_t st);
// Node windows of the coarse build (radius beyond the per-source kernels).
struct NodeWinArgs {
    int nx, ny, nz;
    int64_t n;                // cells
    int B, K, ncx, ncy, ncz;
    int64_t n_nodes;
    const void *lx;           // owned face coefficients [3][N], FP64 (fp64) or FP32
    const int *node;
    const int *batch;         // node ids of this batch
    int n_batch;
    int wb;                   // window edge (2K + 1) B
    int sink;                 // far-field cells absorb
};
// S [(2K+1)^3][n_nodes] entries of the batch's nodes are written (not added);
// ga, gb: n_batch * wb^3 elements each; 2K + 1 <= 17
hipError_t launch_nodewin(int fp64, const NodeWinArgs &a, int n_sub, void *ga, void *gb, const double *count,
                          double *S, hipStream_t st);
hipError_t launch_coarse_pbc_fd(int fp64, const void *lam, const int *node, int nx, int ny, int nz, int n_sub,
                                const double *u, double cour, double *a, double *b, double **result, hipStream_t st);
hipError_t launch_coarse_fill_reservoir(const int *node, int64_t n, double v, double *c, hipStream_t st);
// slot null: every chunk at its own index (plane = all chunks x zb); else the
// listed chunks only, chunk c at slot[c] (-1: not stored; plane = list x zb)
hipError_t launch_coarse_finalize(int prec, const double *S, const double *count, int64_t n_nodes, int nb, int ncx,
                                  int ncy, int ncz, const int *slot, int64_t plane, void *P, hipStream_t st);
// The coarse grid padded by K on every side: node (x, y, z) sits at
// (x + K) sx + (y + K) sy + (z + K) sz.  Two layouts, fixed by K: for small
// windows x fastest (the product with one lane per node reads runs along x);
// for K >= COARSE_CHUNK_MIN_K z fastest, with the z extent ncz rounded up to
// 8, plus 2K (the product with one lane per chunk of P's layout reads one
// contiguous, 16-byte aligned z column per offset pair).
constexpr int COARSE_CHUNK_MIN_K = 5;
struct CoarsePad {
    int K;
    int64_t sx, sy, sz, size;
};
__host__ __device__ inline CoarsePad coarse_pad(int ncx, int ncy, int ncz, int K)
{
    CoarsePad p;
    p.K = K;
    const int64_t px = ncx + 2 * K, py = ncy + 2 * K;
    if (K >= COARSE_CHUNK_MIN_K) {
        const int64_t pz = (ncz + 7) / 8 * 8 + 2 * K;
        p.sz = 1;
        p.sy = pz;
        p.sx = py * pz;
        p.size = px * py * pz;
    } else {
        p.sx = 1;
        p.sy = px;
        p.sz = px * py;
        p.size = px * py * (ncz + 2 * K);
    }
    return p;
}
__host__ __device__ inline int64_t coarse_pad_at(const CoarsePad &p, int x, int y, int z)
{
    return (x + p.K) * p.sx + (y + p.K) * p.sy + (z + p.K) * p.sz;
}
// writes the nodes with grouped cells only: cpad must be zeroed once; dense:
// one workgroup per row of blocks (most blocks hold grouped cells), else one
// wave per node
hipError_t launch_coarse_map(const double *c, const int *node, const double *count, int nx, int ny, int nz, int B,
                             int ncx, int ncy, int ncz, int K, double *cpad, hipStream_t st, int dense,
                             const int *used = nullptr, int64_t n_used = 0);   // used: the nodes with cells
hipError_t launch_flow_window(int fp64, int r, const FlowArgs &a, hipStream_t st);
// FP32 flow window kernels in the flat layout (r = 4..8)
hipError_t launch_flow_flat(int r, const FlowArgs &a, hipStream_t st);
hipError_t launch_flow_stability(int fp64, const void *lam, const double *u, int nx, int ny, int nz, double cour,
                                 unsigned long long *out, hipStream_t st);
hipError_t launch_coarse_bin(int fp64, int sink, int r, const CoarseGenArgs &a, const void *G, int64_t src_base,
                             int64_t n_src, hipStream_t st);
// Product C' = P C (+ P_BC c_ff) over the nodes of the listed units of P's
// layout (a chunk: zb = 16 / element size nodes along z at one (x, y)).  K <
// COARSE_CHUNK_MIN_K: list = the 64-position groups holding a node with cells,
// one lane per node; else list = the chunks holding a node with cells, one
// lane per chunk, the offset pairs (oy, ox) split into n_split ranges whose
// partial sums go to part (coarse_apply_part_elems doubles) and are added in
// range order by a second launch.
hipError_t launch_coarse_apply(int prec, const void *P, const double *cpad, int ncx, int ncy, int ncz, int K,
                               const double *pbc_pad, double c_ff, const double *count, double *cnew,
                               hipStream_t st, const double *cff_dev,    // cff_dev set: c_ff read from it
                               const int *list, int64_t n_list, int n_split, double *part);
// Arithmetic of the coarse product (the precisions of Table 2): C and the
// products / sums in FP64, in FP32, in FP16 with FP32 accumulation (the
// mixed scheme of Sec. 3.3), or all in FP16.  The mapping writes the padded
// C in the arithmetic's C type (FP64, FP32, FP16 rounded through FP32).
enum CoarseArithId : int { COARSE_FP64 = 0, COARSE_FP32 = 1, COARSE_MIXED = 2, COARSE_FP16 = 3 };
bool coarse_arith_supported(int arith, int prec);               // P storage the arithmetic takes
size_t coarse_c_bytes(int arith);                               // bytes of one padded C value
hipError_t launch_coarse_map_arith(int arith, const double *c, const int *node, const double *count, int nx, int ny,
                                   int nz, int B, int ncx, int ncy, int ncz, int K, void *cpad, hipStream_t st,
                                   int dense, const int *used = nullptr, int64_t n_used = 0);
hipError_t launch_coarse_apply_arith(int arith, int prec, const void *P, const void *cpad, int ncx, int ncy, int ncz,
                                     int K, const double *pbc_pad, double c_ff, const double *count, double *cnew,
                                     hipStream_t st, const double *cff_dev, const int *list, int64_t n_list,
                                     int n_split, double *part);

// Ensemble product (several coarse fields at once) on the matrix cores, for
// P stored in FP16 with K <= ENSEMBLE_MAX_K: tiles of 4 x 4 nodes in (x, y),
// (2K + 1) z offsets of kst steps of 32 columns; the padded FP16 C grid has
// px x py x pz positions (pad K) for every member.
constexpr int ENSEMBLE_MAX_K = 4;
struct EnsembleShape {
    int ncx, ncy, ncz, K, kw;
    int tx, ty;               // tiles along x and y
    int row;                  // columns per source row (4 + 2K rounded up to 8)
    int kst;                  // 32-column steps per z offset
    int64_t n_tiles;
    int px, py, pz;
    int64_t msize;            // elements of one member's padded grid
};
EnsembleShape ensemble_shape(int ncx, int ncy, int ncz, int K);
int64_t ensemble_frag_bytes(const EnsembleShape &s);
// largest |P| (FP32 bits, into *out) and the power-of-two scale it gives
hipError_t launch_ensemble_pmax(const void *P16, int64_t n, unsigned *out, hipStream_t st);
int ensemble_p_scale(unsigned pmax_bits);
hipError_t launch_ensemble_frags(const void *P16, int64_t plane, const EnsembleShape &s, int sp, void *frag,
                                 hipStream_t st);
// cap: members the padded grid holds (a multiple of 16, >= n_ens; the
// grid is cap x msize halves); cmax: n_ens unsigned of scratch (each
// member's largest |C|)
hipError_t launch_ensemble_pack(const double *C, int n_ens, int64_t n_nodes, const EnsembleShape &s, int cap,
                                unsigned *cmax, void *cpad, hipStream_t st);
hipError_t launch_ensemble_apply(const void *frag, const void *cpad, int n_ens, int64_t n_nodes,
                                 const EnsembleShape &s, int cap, int sp, const unsigned *cmax, double *out,
                                 hipStream_t st);
int coarse_apply_zb(int prec);                                  // nodes per chunk
int coarse_apply_split(int K, int64_t n_chunks);                // the number of pair ranges (1 below the chunk K)
int64_t coarse_apply_part_elems(int prec, int K, int64_t n_chunks);
hipError_t launch_coarse_remap(const double *c_in, const int *node, const double *cnew, int64_t n, double *c_out,
                               hipStream_t st);
// Integrated near-field solver (fdirw_mp.hip).  Cell roles come from the
// coarse node index: >= 0 near-field liquid, COARSE_RESERVOIR far field,
// COARSE_OUTSIDE solid.  Per-phase tables live in device memory, not in
// kernel arguments (every workgroup reads them).
// Tiles of the fused local kernel: MP_TX x MP_TY x MP_TZ cells and a halo of
// MP_H cells on every side in LDS.
constexpr int MP_TX = 16, MP_TY = 8, MP_TZ = 8, MP_H = 3;
constexpr int MP_BX = MP_TX + 2 * MP_H, MP_BY = MP_TY + 2 * MP_H, MP_BZ = MP_TZ + 2 * MP_H;
constexpr int MP_BOX = MP_BX * MP_BY * MP_BZ;
constexpr int MP_PAIR_CAP = 512;      // interface pairs of a tile staged in LDS (the rest read from memory)
constexpr int MP_MAX_SOLID_PHASES = 126;   // solid phases the fused kernel's role byte can tell apart
constexpr int MP_SUM_BLOCKS = 256;    // most workgroups of the balance kernel
constexpr int MP_CHUNK = 1024;        // cells per workgroup of the list kernels
struct MpLocalArgs {
    int nx, ny, nz;
    const int *tiles;                 // tile indices (tz * nty + ty) * ntx + tx
    int64_t n_tiles;
    const int *pair_off;              // [6 n_tiles + 1] start of each tile's pass in pairs
    const uint16_t *pairs;            // interface pairs, (q << 1) | (lower cell solid)
    const int *node;
    const uint8_t *scode;             // [N] compact solid-phase index of every cell (solid cells read)
    const double *dsolc;              // D A / RT of the solid phases, by compact index
    int n_solid;                      // entries of dsolc
    const double *cnew;               // node values after the product
    const double *c_in;               // the step's input field (solid cells)
    double *out;                      // the step's output field (active cells written)
    double c_eq_l, c_eq_s, kappa_dt;
    int solid;                        // 1: one solid sub-step and the Eq. 7 balance
    double dt_s, h;
    double *part;                     // 2 * n_tiles doubles
    double m_total, v_ff;
    double *cff, *hist_row;
};
int64_t mp_tile_count(int nx, int ny, int nz);
hipError_t launch_mp_faces(const int *node, int nx, int ny, int nz, unsigned long long *count, hipStream_t st);
// scode[i] = table256[label[i]]
hipError_t launch_mp_code(const uint8_t *label, int64_t n, const unsigned char *table256, uint8_t *scode,
                          hipStream_t st);
hipError_t launch_mp_tile_flags(const int *node, int nx, int ny, int nz, int *flag, hipStream_t st);
// list null: counts into cnt[6 n_tiles]; else entries at list[off[6 t + p]..]
hipError_t launch_mp_tile_pairs(const int *node, int nx, int ny, int nz, const int *tiles, int64_t n_tiles,
                                const int *off, uint16_t *list, int *cnt, hipStream_t st);
// the fused local kernel, then (a.solid) the Eq. 7 finish from its partials
hipError_t launch_mp_local(const MpLocalArgs &a, hipStream_t st);
// sorted lists: mode 0 active cells (not far field), mode 1 solid cells;
// chunk_count / chunk_off hold ceil(n / MP_CHUNK) entries
hipError_t launch_mp_list_count(const int *node, int64_t n, int mode, int *chunk_count, hipStream_t st);
hipError_t launch_mp_list_write(const int *node, int64_t n, int mode, const int64_t *chunk_off, int *list,
                                hipStream_t st);
// inv: [N] ints preset to -1; lam [6][n_sol] doubles, nb [6][n_sol] ints
// dsol: [256] D A / RT of every solid phase (0 for the others), device memory
hipError_t launch_mp_solid_prep(const int *sol, int64_t n_sol, const uint8_t *label, const double *dsol,
                                int *inv, int nx, int ny, int nz, double dt, double h, double *lam, int *nb,
                                hipStream_t st);
// n_sub sub-steps of the solid cells of field, in place (a, b: n_sol doubles)
hipError_t launch_mp_solid(const int *sol, int64_t n_sol, const double *lam, const int *nb, int nx, int ny,
                           int n_sub, double *field, double *a, double *b, hipStream_t st);
unsigned mp_balance_blocks(int64_t n_act);   // part needs 2 x this many doubles
hipError_t launch_mp_balance(const int *act, int64_t n_act, const int *node, const double *c, double *part,
                             double m_total, double v_ff, double *cff, double *hist_row, hipStream_t st);
hipError_t launch_mp_far_fill(const int *node, int64_t n, const double *cff, const double *src, double *dst,
                              hipStream_t st);
int64_t bank_elems(int nx, int ny, int nz, int r, int elem_bytes);   // offset-major bank, padded
hipError_t launch_fill(double *p, int64_t n, double v, hipStream_t st);
hipError_t launch_fill_u32(unsigned *p, int64_t n, unsigned v, hipStream_t st);
int field_sum_blocks(int64_t n);
hipError_t launch_field_sum(const double *v, int64_t n, double *part, double *out, hipStream_t st);
hipError_t launch_minmax(const double *v, int64_t n, double *out, hipStream_t st);
hipError_t launch_minmax_scalar(const double *v, int64_t n, double *part, double *out, hipStream_t st);
hipError_t launch_src_check(const int64_t *src, int64_t n_src, int64_t n, unsigned *bad, hipStream_t st);

// ----------------------------------------------------------------- surrogate
// (fdirw_nn.hip).  The network runs on windows of radius NN_R; 16-bit values
// are BF16 bit patterns held as uint16_t.

#define NN_R 8
constexpr int NN_W = 2 * NN_R + 1;
constexpr int NN_V = NN_W * NN_W * NN_W;

struct NnFeatArgs {
    int nx, ny, nz;
    int n_sub;
    const int64_t *src;       // [B] source indices
    const uint8_t *label;
    float f1[256];            // log-D feature per phase (-1 for D = 0)
    uint8_t open[256];        // 1 where the phase has D > 0
    const float *prior;       // [V] log of the uniform-D window kernel
    uint16_t *X;              // [B][V][8] features (BF16)
    uint8_t *support;         // [B][V]
};

struct NnConvArgs {
    const uint16_t *in;       // [B][V][CI] BF16 channel-last
    const uint16_t *wpack;    // packed B operands
    const float *bias;        // [16] (modes 0, 1)
    int mode;                 // 0 hidden layer, 1 last layer, 2 input gradient
    float *zpre;              // mode 0: [B][V][16] pre-activation, or null
    uint16_t *hout;           // mode 0: [B][V][16] SiLU output (BF16)
    float *z5;                // mode 1: [B][V]
    float *dh;                // mode 2: [B][V][16]
};

struct NnLossArgs {
    const float *z5;          // [B][V] last-layer output
    const float *prior;       // [V]
    const uint8_t *support;   // [B][V]
    const float *target;      // [B][V] FD kernels (any positive mass), or null
    float *G;                 // [B][V] softmax kernel, or null
    double *mass;             // [B] FP64 sum of G as stored, or null
    float *logits;            // [B][V] prior + z5, or null
    double *loss;             // [B][2] KL and L1 (with target)
    uint16_t *dlog8;          // [B][V][8] d loss / d logits in channel 0 (with target)
    float grad_scale;         // factor on d loss / d logits (1 / batch)
};

struct NnWgradArgs {
    const uint16_t *dz;       // [B][V][COP] gradient at the layer output
    const uint16_t *h;        // [B][V][CI] layer input
    int co_n, ci_n;           // real channel counts
    int n_slab;               // B * slabs per window
    float *part;              // [grid][27][16][16] weight partials
    float *bpart;             // [grid][16] bias partials
};

// Fused inference: one workgroup runs features, support, the five layers
// (activations resident in LDS) and the softmax of one window.
struct NnFusedArgs {
    int nx, ny, nz;
    int n_sub;
    const int64_t *src;       // [B] source indices
    const uint8_t *label;
    float f1[256];
    uint8_t open[256];
    const float *prior;       // [V]
    const uint16_t *wf[5];    // weights in the fused operand layout (nn_launch_fpack)
    const float *bias[5];
    float *G;                 // [B][V] softmax kernel, or null
    double *mass;             // [B] FP64 sum of G as stored, or null
    float *logits;            // [B][V], or null
    uint8_t *support;         // [B][V], or null
    float *z5g;               // [B][V] scratch for the last layer's output (may be G)
};

int nn_slabs_per_window();
int nn_fpack_elems(int layer);
hipError_t nn_launch_fpack(const float *w, int layer, int co_n, int ci_n, uint16_t *out, hipStream_t st);
hipError_t nn_launch_fused(const NnFusedArgs &a, int batch, hipStream_t st);
hipError_t nn_launch_features(const NnFeatArgs &a, int batch, hipStream_t st);
hipError_t nn_launch_pack(const float *w, int co_n, int ci_n, int CI, int flip, uint16_t *out, hipStream_t st);
int nn_pack_chunks(int CI);
hipError_t nn_launch_conv(int CI, const NnConvArgs &a, int batch, hipStream_t st);
hipError_t nn_launch_loss(const NnLossArgs &a, int batch, hipStream_t st);
hipError_t nn_launch_silu_bwd(const float *dh, const float *zpre, uint16_t *dz, int64_t n, hipStream_t st);
hipError_t nn_launch_wgrad(int CI, int COP, const NnWgradArgs &a, int grid, hipStream_t st);
hipError_t nn_launch_wgrad_reduce(const float *part, const float *bpart, int grid, int co_n, int ci_n,
                                  float *gw, float *gb, hipStream_t st);
hipError_t nn_launch_adam(float *w, float *m, float *v, const float *g, int n, float lr, float b1, float b2,
                          float eps, float c1, float c2, hipStream_t st);
hipError_t nn_launch_lines_src(int64_t line0, int nlines, int nx, int ny, int nz, int64_t *src, hipStream_t st);
hipError_t nn_launch_apply(int nx, int ny, int nz, int64_t line0, int nlines, int seg_len, int n_seg,
                           const float *G, const double *mass, const double *c_in, double *c_out,
                           unsigned long long *n_used, hipStream_t st);
hipError_t nn_launch_l1(const float *a, const float *b, int batch, double *out, hipStream_t st);
hipError_t nn_launch_fill_f32(float *p, int64_t n, float v, hipStream_t st);

}  // namespace fdirw
