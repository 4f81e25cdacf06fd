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
    int seg_len, n_seg;       // each (x, y) line of sources is cut into n_seg segments
    const void *lx;
    const double *c_in;
    double *c_out;
    double *wg_kmass;         // [n_blocks][2] min / max kernel mass, or null
    unsigned long long *n_used;
};

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
};

// Apply a stored kernel bank: same line walk as the fused step, kernels read
// from HBM instead of generated.
struct BankArgs {
    int nx, ny, nz;
    int seg_len, n_seg;
    const void *bank;         // [N][W][W][W] of the bank element type
    const double *mass;       // [N] kernel mass (renormalising modes), or null
    const double *c_in;
    double *c_out;
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
int batch_windows_per_group(int r);

hipError_t launch_validate(const uint8_t *label, int64_t n, int n_phase, unsigned *out, hipStream_t st);
hipError_t launch_coef(const uint8_t *label, int nx, int ny, int nz, const CoefTable &tab,
                       double dt, double h, double *lam64, float *lam32, hipStream_t st);
hipError_t launch_line(int mode, int r, const LineArgs &a, hipStream_t st);
hipError_t launch_window(int mode, int r, const WindowArgs &a, hipStream_t st);
hipError_t launch_bank_apply(int prec, int r, const BankArgs &a, hipStream_t st);
hipError_t launch_fill(double *p, int64_t n, double v, hipStream_t st);
hipError_t launch_fill_u32(unsigned *p, int64_t n, unsigned v, hipStream_t st);
int field_sum_blocks(int64_t n);
hipError_t launch_field_sum(const double *v, int64_t n, double *part, double *out, hipStream_t st);
hipError_t launch_minmax(const double *v, int64_t n, double *out, hipStream_t st);
hipError_t launch_src_check(const int64_t *src, int64_t n_src, int64_t n, unsigned *bad, hipStream_t st);

}  // namespace fdirw
