// fdirw_coarse_api.cpp -- host side of the coarse-mesh FDiRW entry points
// (include/fdirw.h; Sec. 3.1 of arXiv 2408.11376, Eqs. 10-15).
//
// A handle owns the coarse operator of one geometry: the node index of every
// cell, the cell count of every node and P in the bank layout of its storage
// precision.  fdirw_coarse_create builds P from the fine window kernels of
// every grouped source (the same FD as fdirw_kernels); fdirw_coarse_step maps,
// applies P (one thread per node) and remaps.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/fdirw.h"
#include "fdirw_host.h"
#include "fdirw_launch.h"

namespace fdirw {

namespace {

struct Coarse {
    int dev = -1;
    int nx = 0, ny = 0, nz = 0;
    int64_t n = 0;
    int B = 1, K = 0, ncx = 0, ncy = 0, ncz = 0;
    int64_t n_nodes = 0;
    int prec = FDIRW_FP64;          // storage of P: FP64, FP32, FP16_BANK or BF16_BANK
    size_t esz = 8;
    int64_t plane = 0;              // elements of one offset plane of P (bank layout; compact for K >= 5)
    std::vector<int> slot;          // K >= 5: chunk -> its place in P's compact layout (-1: not stored)
    void *node = nullptr;           // int [N]
    void *count = nullptr;          // double [n_nodes]
    void *P = nullptr;              // esz * (2K+1)^3 * plane bytes
    void *cpad = nullptr;           // double [coarse_pad(...).size]: the padded coarse grid
    void *cnew = nullptr;           // double [n_nodes]
    void *part = nullptr;           // field-sum partials
    bool far_field = false;         // reservoir (far-field boundary) phases present
    bool dense = true;              // most nodes hold grouped cells (mapping by rows of blocks)
    void *pbc = nullptr;            // double, P_BC on the padded coarse grid (far field only)
    void *list = nullptr;           // int [n_list]: the product's units of P's layout holding a node with cells
    int64_t n_list = 0;             // (64-position groups for K < COARSE_CHUNK_MIN_K, else chunks)
    void *apart = nullptr;          // double: the product's partial sums, n_split ranges of offset pairs
    int n_split = 1;
    void *used = nullptr;           // int [n_used]: the nodes with cells (sparse mapping)
    int64_t n_used = 0;
    int arith = COARSE_FP64;        // arithmetic of the product (fdirw_coarse_set_arith)
    void *cpad_lp = nullptr;        // the padded coarse grid in the arithmetic's C type (FP32 / FP16)
    void *efrag = nullptr;          // ensemble product: P as matrix fragments (built on first use)
    void *ecpad = nullptr;          // ensemble product: padded FP16 grids of ecpad_members members
    void *ecmax = nullptr;          // ensemble product: each member's largest |C| (FP32 bits)
    int64_t ecpad_members = 0;
    int esp = 0;                    // ensemble product: P's power-of-two scale

    ~Coarse()
    {
        for (void *p : {node, count, P, cpad, cnew, part, pbc, list, apart, used, cpad_lp, efrag, ecpad, ecmax})
            if (p) (void)hipFree(p);
    }
    int nb() const { return (2 * K + 1) * (2 * K + 1) * (2 * K + 1); }
};

int coarse_alloc(void **p, size_t bytes)
{
    if (bytes == 0) bytes = 16;
    if (hipMalloc(p, bytes) != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(FDIRW_E_NOMEM, "coarse FDiRW: could not allocate %zu bytes", bytes);
    }
    return FDIRW_OK;
}

int check_handle(const Coarse *h)
{
    if (!h) return fail(FDIRW_E_ARG, "coarse handle is null");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != h->dev)
        return fail(FDIRW_E_ARG, "coarse handle belongs to device %d, current device is %d", h->dev, dev);
    return FDIRW_OK;
}

int field_sum_h(Coarse *h, const double *c, hipStream_t st, double *out)
{
    double *part = (double *)h->part;
    double *res = part + 2 * field_sum_blocks(h->n);
    hipError_t e = launch_field_sum(c, h->n, part, res, st);
    if (e == hipSuccess) e = hipMemcpyAsync(out, res, sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "coarse field sum");
    return FDIRW_OK;
}

}  // namespace

}  // namespace fdirw

using namespace fdirw;

extern "C" {

int fdirw_coarse_create(const fdirw_domain *d, int32_t block, int32_t prec, const uint8_t *grouped,
                        const uint8_t *reservoir, const double *velocity, void *stream, void **handle,
                        double *seconds)
{
    if (!handle) return fail(FDIRW_E_ARG, "handle is null");
    *handle = nullptr;
    int rc = check_domain(d, FDIRW_MAX_COARSE_RADIUS);
    if (rc) return rc;
    if (block < 1 || block > 256) return fail(FDIRW_E_ARG, "block = %d outside 1..256", block);
    const bool node_windows = d->r > FDIRW_MAX_RADIUS;
    if (node_windows && (d->r + block - 1) / block > FDIRW_MAX_COARSE_K)
        return fail(FDIRW_E_ARG, "r = %d needs ceil(r / block) <= %d (block = %d)", d->r, FDIRW_MAX_COARSE_K, block);
    if (node_windows && velocity)
        return fail(FDIRW_E_UNSUPPORTED, "steady flow needs r <= %d (per-source kernels)", FDIRW_MAX_RADIUS);
    if (node_windows) {
        const int64_t wb = (int64_t)(2 * ((d->r + block - 1) / block) + 1) * block;
        if (wb * wb * wb > 0x7fffffffLL)
            return fail(FDIRW_E_ARG, "node window of %lld^3 cells is too large (block %d, r %d)", (long long)wb, block,
                        d->r);
    }
    if (prec != FDIRW_FP64 && prec != FDIRW_FP32 && prec != FDIRW_FP16_BANK && prec != FDIRW_BF16_BANK)
        return fail(FDIRW_E_ARG, "coarse P precision must be FP64, FP32, FP16_BANK or BF16_BANK (got %d)", prec);
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t st = (hipStream_t)stream;
    auto *h = new (std::nothrow) Coarse;
    if (!h) return fail(FDIRW_E_NOMEM, "coarse handle");
    if (hipGetDevice(&h->dev) != hipSuccess) {
        delete h;
        return fail(FDIRW_E_DEVICE, "hipGetDevice failed");
    }
    h->nx = d->nx; h->ny = d->ny; h->nz = d->nz;
    h->n = (int64_t)d->nx * d->ny * d->nz;
    h->B = block;
    h->K = (d->r + block - 1) / block;
    h->ncx = (d->nx + block - 1) / block;
    h->ncy = (d->ny + block - 1) / block;
    h->ncz = (d->nz + block - 1) / block;
    h->n_nodes = (int64_t)h->ncx * h->ncy * h->ncz;
    h->prec = prec;
    h->esz = bank_elem_bytes(prec);
    if (reservoir)
        for (int i = 0; i < d->n_phase; ++i) h->far_field = h->far_field || reservoir[i] != 0;
    const int zb = 16 / (int)h->esz;
    h->plane = (int64_t)((h->ncz + zb - 1) / zb) * h->ncy * h->ncx * zb;
    const int nb = h->nb();
    const int64_t n_pad = coarse_pad(h->ncx, h->ncy, h->ncz, h->K).size;
    double *S = nullptr;
    hipError_t e = hipSuccess;
    {
        std::lock_guard<std::mutex> lk(cache_mutex());
        DevCache &dc = cache_for_current_device();
        Geometry g;
        const void *lam = nullptr;
        rc = coef_buffers(d, prec == FDIRW_FP64 ? FDIRW_FP64 : FDIRW_FP32, st, dc, &g, &lam);
        if (!rc && velocity) rc = flow_stable(d, prec == FDIRW_FP64, lam, velocity, g.dt, st, dc);
        if (!rc) rc = coarse_alloc(&h->node, (size_t)h->n * sizeof(int));
        if (!rc) rc = coarse_alloc(&h->count, (size_t)h->n_nodes * sizeof(double));
        if (!rc) rc = coarse_alloc(&h->cpad, (size_t)n_pad * sizeof(double));
        if (!rc) rc = coarse_alloc(&h->cnew, (size_t)h->n_nodes * sizeof(double));
        if (!rc) rc = coarse_alloc(&h->part, (size_t)(2 * field_sum_blocks(h->n) + 2) * sizeof(double));
        if (!rc) rc = coarse_alloc((void **)&S, (size_t)nb * h->n_nodes * sizeof(double));
        if (!rc && h->far_field) rc = coarse_alloc(&h->pbc, (size_t)n_pad * sizeof(double));
        if (rc) {
            (void)hipFree(S);
            delete h;
            return rc;
        }
        CoarseTable tab;
        std::memset(&tab, 0, sizeof tab);
        for (int i = 0; i < d->n_phase; ++i) {
            tab.mobile[i] = (grouped ? grouped[i] != 0 : d->d_phase[i] > 0.0) ? 1 : 0;
            tab.reservoir[i] = (reservoir && reservoir[i]) ? 1 : 0;
        }
        // P entries of empty nodes and of the padding groups stay 0, and so do
        // the halo and the empty nodes of the padded coarse fields
        e = launch_fill((double *)h->count, h->n_nodes, 0.0, st);
        if (e == hipSuccess) e = launch_fill((double *)h->cpad, n_pad, 0.0, st);
        if (e == hipSuccess && h->pbc) e = launch_fill((double *)h->pbc, n_pad, 0.0, st);
        if (e == hipSuccess) e = launch_fill(S, (int64_t)nb * h->n_nodes, 0.0, st);
        if (e == hipSuccess)
            e = launch_coarse_nodes(d->label, tab, d->nx, d->ny, d->nz, block, h->ncx, h->ncy, (int *)h->node,
                                    (double *)h->count, st);
        if (e == hipSuccess) {
            // the mapping's shape: by rows of blocks when most nodes hold cells
            std::vector<double> hc((size_t)h->n_nodes);
            e = hipMemcpyAsync(hc.data(), h->count, hc.size() * sizeof(double), hipMemcpyDeviceToHost, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            int64_t used = 0;
            for (double v : hc) used += v > 0.0;
            h->dense = 2 * used >= h->n_nodes;
            // the product's units of P's layout that hold a node with cells:
            // chunks (zb nodes along z), or groups of 64 / zb chunks for small K
            if (e == hipSuccess) {
                const int zb = coarse_apply_zb(prec);
                const int64_t n_ch = (int64_t)((h->ncz + zb - 1) / zb) * h->ncy * h->ncx;
                const int64_t per = h->K >= COARSE_CHUNK_MIN_K ? 1 : 64 / zb;    // chunks per unit
                std::vector<int> gl;
                for (int64_t u0 = 0; u0 < n_ch; u0 += per) {
                    bool any = false;
                    for (int64_t ch = u0; ch < u0 + per && ch < n_ch && !any; ++ch) {
                        const int x = (int)(ch % h->ncx), y = (int)((ch / h->ncx) % h->ncy);
                        const int z0 = (int)(ch / ((int64_t)h->ncx * h->ncy)) * zb;
                        for (int z = z0; z < z0 + zb && z < h->ncz && !any; ++z)
                            any = hc[(size_t)(((int64_t)z * h->ncy + y) * h->ncx + x)] > 0.0;
                    }
                    if (any) gl.push_back((int)(u0 / per));
                }
                h->n_list = (int64_t)gl.size();
                h->n_split = coarse_apply_split(h->K, h->n_list);
                std::vector<int> ul;
                for (int64_t I = 0; I < h->n_nodes; ++I)
                    if (hc[(size_t)I] > 0.0) ul.push_back((int)I);
                h->n_used = (int64_t)ul.size();
                // P: every chunk of the grid (K < 5) or the listed chunks only,
                // in list order (K >= 5); entries never written stay 0
                if (h->K >= COARSE_CHUNK_MIN_K) {
                    h->plane = h->n_list * zb;
                    h->slot.assign((size_t)n_ch, -1);
                    for (size_t k = 0; k < gl.size(); ++k) h->slot[(size_t)gl[k]] = (int)k;
                }
                rc = coarse_alloc(&h->P, (size_t)nb * h->plane * h->esz);
                if (!rc && h->plane > 0)
                    e = launch_fill_u32((unsigned *)h->P, (int64_t)((size_t)nb * h->plane * h->esz / 4), 0u, st);
                if (!rc) rc = coarse_alloc(&h->list, gl.size() * sizeof(int));
                if (!rc) rc = coarse_alloc(&h->used, ul.size() * sizeof(int));
                if (!rc)
                    rc = coarse_alloc(&h->apart,
                                      (size_t)coarse_apply_part_elems(prec, h->K, h->n_list) * sizeof(double));
                if (!rc && !gl.empty())
                    e = hipMemcpyAsync(h->list, gl.data(), gl.size() * sizeof(int), hipMemcpyHostToDevice, st);
                if (!rc && e == hipSuccess && !ul.empty())
                    e = hipMemcpyAsync(h->used, ul.data(), ul.size() * sizeof(int), hipMemcpyHostToDevice, st);
                if (e == hipSuccess) e = hipStreamSynchronize(st);
                if (rc) {
                    (void)hipFree(S);
                    delete h;
                    return rc;
                }
            }
            if (node_windows && e == hipSuccess) {
                // node windows: the nodes with cells in batches of at most
                // ~2 GB of window state
                std::vector<int> ids;
                for (int64_t I = 0; I < h->n_nodes; ++I)
                    if (hc[(size_t)I] > 0.0) ids.push_back((int)I);
                const int K = h->K, wb = (2 * K + 1) * block;
                const size_t esz = prec == FDIRW_FP64 ? 8 : 4;
                const size_t per = (size_t)wb * wb * wb * esz * 2;
                int64_t nbat = (int64_t)(((size_t)2 << 30) / per);
                if (nbat < 1) nbat = 1;
                if (nbat > 65535) nbat = 65535;
                if (nbat > (int64_t)ids.size()) nbat = (int64_t)ids.size();
                int *dids = nullptr;
                void *ga = nullptr, *gb = nullptr;
                rc = coarse_alloc((void **)&dids, ids.size() * sizeof(int));
                if (!rc) rc = coarse_alloc(&ga, (size_t)nbat * wb * wb * wb * esz);
                if (!rc) rc = coarse_alloc(&gb, (size_t)nbat * wb * wb * wb * esz);
                if (!rc && !ids.empty())
                    e = hipMemcpyAsync(dids, ids.data(), ids.size() * sizeof(int), hipMemcpyHostToDevice, st);
                NodeWinArgs w;
                w.nx = d->nx; w.ny = d->ny; w.nz = d->nz; w.n = h->n;
                w.B = block; w.K = K; w.ncx = h->ncx; w.ncy = h->ncy; w.ncz = h->ncz;
                w.n_nodes = h->n_nodes;
                w.lx = lam;
                w.node = (const int *)h->node;
                w.wb = wb;
                w.sink = h->far_field ? 1 : 0;
                for (int64_t b0 = 0; !rc && e == hipSuccess && b0 < (int64_t)ids.size(); b0 += nbat) {
                    w.batch = dids + b0;
                    w.n_batch = (int)(b0 + nbat <= (int64_t)ids.size() ? nbat : (int64_t)ids.size() - b0);
                    e = launch_nodewin(prec == FDIRW_FP64, w, d->n_sub, ga, gb, (const double *)h->count, S, st);
                }
                (void)hipStreamSynchronize(st);
                (void)hipFree(dids);
                (void)hipFree(ga);
                (void)hipFree(gb);
                if (rc) {
                    (void)hipFree(S);
                    delete h;
                    return rc;
                }
            }
        }
        if (e == hipSuccess) {
            CoarseGenArgs a;
            a.nx = d->nx; a.ny = d->ny; a.nz = d->nz; a.n = h->n;
            a.n_sub = d->n_sub;
            a.lx = lam;
            a.node = (const int *)h->node;
            a.block = block; a.K = h->K;
            a.ncx = h->ncx; a.ncy = h->ncy;
            a.n_nodes = h->n_nodes;
            a.S = S;
            if (node_windows) {
                // built above
            } else if (!velocity) {
                e = launch_coarse_window(prec == FDIRW_FP64, h->far_field, d->r, a, st);
            } else {
                // flow kernels, generated in chunks of sources into a scratch
                // buffer and binned like the fused build
                const int64_t W = 2 * d->r + 1, W3 = W * W * W;
                const size_t esz = prec == FDIRW_FP64 ? 8 : 4;
                int64_t chunk = (int64_t)((size_t)512 << 20) / (W3 * (int64_t)esz);
                if (chunk < 1) chunk = 1;
                if (chunk > h->n) chunk = h->n;
                void *Gc = nullptr;
                if ((rc = coarse_alloc(&Gc, (size_t)chunk * W3 * esz))) {
                    (void)hipStreamSynchronize(st);
                    (void)hipFree(S);
                    delete h;
                    return rc;
                }
                for (int64_t base = 0; base < h->n && e == hipSuccess; base += chunk) {
                    const int64_t cnt = base + chunk <= h->n ? chunk : h->n - base;
                    FlowArgs f;
                    f.nx = d->nx; f.ny = d->ny; f.nz = d->nz; f.n = h->n;
                    f.n_sub = d->n_sub;
                    f.lam = lam;
                    f.u = velocity;
                    f.dt = g.dt; f.h = d->h;
                    f.src = nullptr; f.src_base = base; f.n_src = cnt;
                    f.node = (const int *)h->node;
                    f.G = Gc; f.mass = nullptr;
                    e = launch_flow_window(prec == FDIRW_FP64, d->r, f, st);
                    if (e == hipSuccess)
                        e = launch_coarse_bin(prec == FDIRW_FP64, h->far_field, d->r, a, Gc, base, cnt, st);
                }
                (void)hipStreamSynchronize(st);
                (void)hipFree(Gc);
            }
        }
        if (e == hipSuccess && h->far_field) {
            // p_BC: the whole-domain FD from 0 with the far-field cells at 1,
            // then its group means on the padded coarse grid
            double *fa = nullptr;
            if ((rc = coarse_alloc((void **)&fa, (size_t)2 * h->n * sizeof(double)))) {
                (void)hipStreamSynchronize(st);
                (void)hipFree(S);
                delete h;
                return rc;
            }
            double *field = nullptr;
            e = launch_coarse_pbc_fd(prec == FDIRW_FP64, lam, (const int *)h->node, d->nx, d->ny, d->nz, d->n_sub,
                                     velocity, g.dt / d->h, fa, fa + h->n, &field, st);
            if (e == hipSuccess)
                e = launch_coarse_map(field, (const int *)h->node, (const double *)h->count, h->nx, h->ny, h->nz,
                                      block, h->ncx, h->ncy, h->ncz, h->K, (double *)h->pbc, st, h->dense,
                                      (const int *)h->used, h->n_used);
            (void)hipStreamSynchronize(st);
            (void)hipFree(fa);
        }
        int *dslot = nullptr;
        if (e == hipSuccess && !h->slot.empty()) {
            if (coarse_alloc((void **)&dslot, h->slot.size() * sizeof(int))) e = hipErrorOutOfMemory;
            if (e == hipSuccess)
                e = hipMemcpyAsync(dslot, h->slot.data(), h->slot.size() * sizeof(int), hipMemcpyHostToDevice, st);
        }
        if (e == hipSuccess)
            e = launch_coarse_finalize(prec, S, (const double *)h->count, h->n_nodes, nb, h->ncx, h->ncy, h->ncz,
                                       dslot, h->plane, h->P, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (dslot) {
            (void)hipStreamSynchronize(st);
            (void)hipFree(dslot);
        }
    }
    (void)hipFree(S);
    if (e != hipSuccess) {
        delete h;
        return hip_fail(e, "coarse operator build");
    }
    if (seconds) *seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    *handle = h;
    return FDIRW_OK;
}

}  // extern "C"

namespace {

// Mapping, product (with P_BC c_ff when pbc is set) and remapping; far-field
// cells of c_out are left at 0.  kernel seconds of the three launches in *ks.
int coarse_apply_all(Coarse *h, const double *c_in, double *c_out, const double *pbc, double c_ff, hipStream_t st,
                     double *ks, const double *cff_dev = nullptr)
{
    EventPair ev;
    hipError_t e = ks ? ev.create() : hipSuccess;
    if (ks && e == hipSuccess) e = hipEventRecord(ev.a, st);
    void *cp = h->arith == COARSE_FP64 ? h->cpad : h->cpad_lp;
    if (e == hipSuccess)
        e = launch_coarse_map_arith(h->arith, c_in, (const int *)h->node, (const double *)h->count, h->nx, h->ny,
                                    h->nz, h->B, h->ncx, h->ncy, h->ncz, h->K, cp, st, h->dense,
                                    (const int *)h->used, h->n_used);
    if (e == hipSuccess)
        e = launch_coarse_apply_arith(h->arith, h->prec, h->P, cp, h->ncx, h->ncy, h->ncz, h->K, pbc, c_ff,
                                      (const double *)h->count, (double *)h->cnew, st, cff_dev,
                                      (const int *)h->list, h->n_list, h->n_split, (double *)h->apart);
    if (e == hipSuccess) e = launch_coarse_remap(c_in, (const int *)h->node, (const double *)h->cnew, h->n, c_out, st);
    if (ks && e == hipSuccess) e = hipEventRecord(ev.b, st);
    if (e != hipSuccess) return hip_fail(e, "coarse step launch");
    if (ks) {
        e = hipEventSynchronize(ev.b);
        if (e != hipSuccess) return hip_fail(e, "coarse step");
        *ks = ev.seconds();
    }
    return FDIRW_OK;
}

}  // namespace

namespace fdirw {

// Mapping and product of the fast step of the integrated solver, with P_BC
// c_ff read from device memory (far-field handles); *cnew receives the node
// values C' (the caller remaps).
int coarse_map_apply(void *handle, const double *c_in, const double *cff_dev, hipStream_t st, const double **cnew)
{
    Coarse *h = (Coarse *)handle;
    int rc = check_handle(h);
    if (rc) return rc;
    void *cp = h->arith == COARSE_FP64 ? h->cpad : h->cpad_lp;
    hipError_t e = launch_coarse_map_arith(h->arith, c_in, (const int *)h->node, (const double *)h->count, h->nx,
                                           h->ny, h->nz, h->B, h->ncx, h->ncy, h->ncz, h->K, cp, st, h->dense,
                                           (const int *)h->used, h->n_used);
    if (e == hipSuccess)
        e = launch_coarse_apply_arith(h->arith, h->prec, h->P, cp, h->ncx, h->ncy, h->ncz, h->K,
                                      h->far_field ? (const double *)h->pbc : nullptr, 0.0, (const double *)h->count,
                                      (double *)h->cnew, st, h->far_field ? cff_dev : nullptr,
                                      (const int *)h->list, h->n_list, h->n_split, (double *)h->apart);
    if (e != hipSuccess) return hip_fail(e, "coarse mapping / product launch");
    *cnew = (const double *)h->cnew;
    return FDIRW_OK;
}

const int *coarse_node(const void *handle) { return (const int *)((const Coarse *)handle)->node; }

}  // namespace fdirw

extern "C" {

int fdirw_coarse_set_arith(void *handle, int32_t arith)
{
    Coarse *h = (Coarse *)handle;
    int rc = check_handle(h);
    if (rc) return rc;
    if (arith < FDIRW_COARSE_ARITH_FP64 || arith > FDIRW_COARSE_ARITH_FP16)
        return fail(FDIRW_E_ARG, "unknown coarse arithmetic %d", arith);
    static_assert(FDIRW_COARSE_ARITH_FP64 == COARSE_FP64 && FDIRW_COARSE_ARITH_FP32 == COARSE_FP32 &&
                      FDIRW_COARSE_ARITH_MIXED == COARSE_MIXED && FDIRW_COARSE_ARITH_FP16 == COARSE_FP16,
                  "arithmetic ids");
    if (!coarse_arith_supported(arith, h->prec))
        return fail(FDIRW_E_ARG, "coarse arithmetic %d needs P stored in %s (the handle stores precision %d)", arith,
                    arith == FDIRW_COARSE_ARITH_FP32 ? "FP32" : "FP16", h->prec);
    if (arith != COARSE_FP64 && !h->cpad_lp) {
        // the largest C type (FP32) for either reduced arithmetic; halo and
        // empty nodes stay 0
        const size_t bytes = (size_t)coarse_pad(h->ncx, h->ncy, h->ncz, h->K).size * sizeof(float) + 16;
        if ((rc = coarse_alloc(&h->cpad_lp, bytes))) return rc;
        hipError_t e = hipMemset(h->cpad_lp, 0, bytes);
        if (e != hipSuccess) return hip_fail(e, "coarse C clear");
    } else if (arith != COARSE_FP64 && arith != h->arith) {
        const size_t bytes = (size_t)coarse_pad(h->ncx, h->ncy, h->ncz, h->K).size * sizeof(float) + 16;
        hipError_t e = hipMemset(h->cpad_lp, 0, bytes);
        if (e != hipSuccess) return hip_fail(e, "coarse C clear");
    }
    h->arith = arith;
    return FDIRW_OK;
}

int fdirw_coarse_step(void *handle, const double *c_in, double *c_out, void *stream, fdirw_stats *stats)
{
    Coarse *h = (Coarse *)handle;
    int rc = check_handle(h);
    if (rc) return rc;
    if (h->far_field) return fail(FDIRW_E_ARG, "the handle has far-field phases: use fdirw_coarse_step_far_field");
    if (!c_in || !c_out) return fail(FDIRW_E_ARG, "c_in and c_out must not be null");
    if (c_in == c_out) return fail(FDIRW_E_ARG, "c_in and c_out must not overlap");
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t st = (hipStream_t)stream;
    fdirw_stats loc;
    std::memset(&loc, 0, sizeof loc);
    if (stats && (rc = field_sum_h(h, c_in, st, &loc.mass_in))) return rc;
    if ((rc = coarse_apply_all(h, c_in, c_out, nullptr, 0.0, st, stats ? &loc.kernel_seconds : nullptr))) return rc;
    if (stats) {
        if ((rc = field_sum_h(h, c_out, st, &loc.mass_out))) return rc;
        loc.kmass_min = INFINITY;
        loc.kmass_max = -INFINITY;
        loc.n_sources = h->n_nodes;
        loc.tuned_config_id = h->B;
        loc.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        *stats = loc;
    }
    return FDIRW_OK;
}

int fdirw_coarse_step_far_field(void *handle, const double *c_in, double *c_out, double *c_ff, double m_total,
                                double v_ff, void *stream, fdirw_stats *stats)
{
    Coarse *h = (Coarse *)handle;
    int rc = check_handle(h);
    if (rc) return rc;
    if (!h->far_field) return fail(FDIRW_E_ARG, "the handle has no far-field phase");
    if (!c_in || !c_out || !c_ff) return fail(FDIRW_E_ARG, "c_in, c_out and c_ff must not be null");
    if (c_in == c_out) return fail(FDIRW_E_ARG, "c_in and c_out must not overlap");
    if (!(v_ff > 0.0) || !std::isfinite(v_ff)) return fail(FDIRW_E_ARG, "v_ff must be finite and > 0");
    if (!std::isfinite(*c_ff) || !std::isfinite(m_total)) return fail(FDIRW_E_NONFINITE, "c_ff and m_total must be finite");
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t st = (hipStream_t)stream;
    double ks = 0.0;
    if ((rc = coarse_apply_all(h, c_in, c_out, (const double *)h->pbc, *c_ff, st, stats ? &ks : nullptr))) return rc;
    // Eq. 7: the far field holds what the near field does not
    double near = 0.0;
    if ((rc = field_sum_h(h, c_out, st, &near))) return rc;
    const double cff = (m_total - near) / v_ff;
    hipError_t e = launch_coarse_fill_reservoir((const int *)h->node, h->n, cff, c_out, st);
    if (e != hipSuccess) return hip_fail(e, "far-field fill");
    *c_ff = cff;
    if (stats) {
        fdirw_stats loc;
        std::memset(&loc, 0, sizeof loc);
        loc.mass_in = m_total;
        loc.mass_out = near + cff * v_ff;
        loc.kmass_min = INFINITY;
        loc.kmass_max = -INFINITY;
        loc.n_sources = h->n_nodes;
        loc.tuned_config_id = h->B;
        loc.kernel_seconds = ks;
        e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(e, "far-field step");
        loc.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        *stats = loc;
    }
    return FDIRW_OK;
}

int fdirw_coarse_apply_ensemble(void *handle, const double *C_in, double *C_out, int32_t n_ens, void *stream,
                                double *kernel_seconds)
{
    Coarse *h = (Coarse *)handle;
    int rc = check_handle(h);
    if (rc) return rc;
    if (!C_in || !C_out) return fail(FDIRW_E_ARG, "C_in and C_out must not be null");
    if (n_ens < 1 || n_ens > FDIRW_MAX_ENSEMBLE)
        return fail(FDIRW_E_ARG, "n_ens = %d outside 1..%d", n_ens, FDIRW_MAX_ENSEMBLE);
    if (h->prec != FDIRW_FP16_BANK)
        return fail(FDIRW_E_ARG, "the ensemble product needs P stored in FP16 (the handle stores precision %d)",
                    h->prec);
    if (h->far_field) return fail(FDIRW_E_ARG, "the ensemble product takes handles without a far field");
    if (h->K > ENSEMBLE_MAX_K)
        return fail(FDIRW_E_UNSUPPORTED, "the ensemble product needs K <= %d (the handle has K = %d)", ENSEMBLE_MAX_K,
                    h->K);
    const size_t bytes = (size_t)n_ens * h->n_nodes * sizeof(double);
    const char *a0 = (const char *)C_in, *b0 = (const char *)C_out;
    if (a0 < b0 + bytes && b0 < a0 + bytes) return fail(FDIRW_E_ARG, "C_in and C_out must not overlap");
    hipStream_t st = (hipStream_t)stream;
    const EnsembleShape s = ensemble_shape(h->ncx, h->ncy, h->ncz, h->K);
    if (s.n_tiles >= ((int64_t)1 << 31) || (int64_t)h->ncy * h->ncz >= ((int64_t)1 << 31))
        return fail(FDIRW_E_UNSUPPORTED, "coarse grid too large for the ensemble product");
    hipError_t e = hipSuccess;
    if (!h->efrag) {
        // P's scale from its largest entry (once per handle), then the fragments
        void *pm = nullptr;
        if ((rc = coarse_alloc(&pm, 16))) return rc;
        unsigned bits = 0;
        e = launch_ensemble_pmax(h->P, (int64_t)h->nb() * h->plane, (unsigned *)pm, st);
        if (e == hipSuccess) e = hipMemcpyAsync(&bits, pm, sizeof bits, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        (void)hipFree(pm);
        if (e != hipSuccess) return hip_fail(e, "ensemble P scale");
        h->esp = ensemble_p_scale(bits);
        if ((rc = coarse_alloc(&h->efrag, (size_t)ensemble_frag_bytes(s)))) return rc;
        e = launch_ensemble_frags(h->P, h->plane, s, h->esp, h->efrag, st);
        if (e != hipSuccess) return hip_fail(e, "ensemble fragments");
    }
    const int64_t members = ((int64_t)n_ens + 15) / 16 * 16;
    if (members > h->ecpad_members) {
        // the halo rows stay zero; interior rows are written by every call
        e = hipStreamSynchronize(st);                         // earlier calls may still read the old grids
        if (e != hipSuccess) return hip_fail(e, "ensemble grid");
        if (h->ecpad) (void)hipFree(h->ecpad);
        if (h->ecmax) (void)hipFree(h->ecmax);
        h->ecpad = h->ecmax = nullptr;
        h->ecpad_members = 0;
        const size_t gb = (size_t)members * s.msize * sizeof(_Float16);
        if ((rc = coarse_alloc(&h->ecmax, (size_t)members * sizeof(unsigned)))) return rc;
        if ((rc = coarse_alloc(&h->ecpad, gb))) return rc;
        e = launch_fill_u32((unsigned *)h->ecpad, (int64_t)(gb / 4), 0u, st);
        if (e != hipSuccess) return hip_fail(e, "ensemble grid clear");
        h->ecpad_members = members;
    }
    EventPair ev;
    if (kernel_seconds) {
        e = ev.create();
        if (e == hipSuccess) e = hipEventRecord(ev.a, st);
    }
    const int cap = (int)h->ecpad_members;
    if (e == hipSuccess)
        e = launch_ensemble_pack(C_in, n_ens, h->n_nodes, s, cap, (unsigned *)h->ecmax, h->ecpad, st);
    if (e == hipSuccess)
        e = launch_ensemble_apply(h->efrag, h->ecpad, n_ens, h->n_nodes, s, cap, h->esp, (const unsigned *)h->ecmax,
                                  C_out, st);
    if (kernel_seconds && e == hipSuccess) e = hipEventRecord(ev.b, st);
    if (e != hipSuccess) return hip_fail(e, "ensemble product launch");
    if (kernel_seconds) {
        e = hipEventSynchronize(ev.b);
        if (e != hipSuccess) return hip_fail(e, "ensemble product");
        *kernel_seconds = ev.seconds();
    }
    return FDIRW_OK;
}

int fdirw_coarse_pbc(void *handle, double *pbc_host)
{
    Coarse *h = (Coarse *)handle;
    int rc = check_handle(h);
    if (rc) return rc;
    if (!pbc_host) return fail(FDIRW_E_ARG, "pbc is null");
    if (!h->far_field) {
        for (int64_t I = 0; I < h->n_nodes; ++I) pbc_host[I] = 0.0;
        return FDIRW_OK;
    }
    const CoarsePad cp = coarse_pad(h->ncx, h->ncy, h->ncz, h->K);
    std::vector<double> pad((size_t)cp.size);
    hipError_t e = hipMemcpy(pad.data(), h->pbc, pad.size() * sizeof(double), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "P_BC copy");
    for (int64_t I = 0; I < h->n_nodes; ++I) {
        const int x = (int)(I % h->ncx), y = (int)((I / h->ncx) % h->ncy), z = (int)(I / ((int64_t)h->ncx * h->ncy));
        pbc_host[I] = pad[(size_t)coarse_pad_at(cp, x, y, z)];
    }
    return FDIRW_OK;
}

int fdirw_coarse_shape(const void *handle, int32_t *shape5, int64_t *n_nodes)
{
    const Coarse *h = (const Coarse *)handle;
    if (!h) return fail(FDIRW_E_ARG, "coarse handle is null");
    if (shape5) {
        shape5[0] = h->ncz; shape5[1] = h->ncy; shape5[2] = h->ncx;
        shape5[3] = h->K; shape5[4] = h->B;
    }
    if (n_nodes) *n_nodes = h->n_nodes;
    return FDIRW_OK;
}

int fdirw_coarse_matrix(void *handle, double *P_host)
{
    Coarse *h = (Coarse *)handle;
    int rc = check_handle(h);
    if (rc) return rc;
    if (!P_host) return fail(FDIRW_E_ARG, "P is null");
    const int nb = h->nb();
    std::vector<unsigned char> raw((size_t)nb * h->plane * h->esz);
    hipError_t e = hipMemcpy(raw.data(), h->P, raw.size(), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "coarse matrix copy");
    const int zb = 16 / (int)h->esz;
    for (int o = 0; o < nb; ++o)
        for (int64_t I = 0; I < h->n_nodes; ++I) {
            const int x = (int)(I % h->ncx), y = (int)((I / h->ncx) % h->ncy);
            const int z = (int)(I / ((int64_t)h->ncx * h->ncy));
            const size_t ch = ((size_t)(z / zb) * h->ncy + y) * h->ncx + x;
            const int64_t at = h->slot.empty() ? (int64_t)ch : h->slot[ch];
            if (at < 0) {                                         // not stored: a node without cells
                P_host[(size_t)o * h->n_nodes + I] = 0.0;
                continue;
            }
            const size_t k = (size_t)o * h->plane + (size_t)at * zb + z % zb;
            double v;
            if (h->prec == FDIRW_FP64) {
                std::memcpy(&v, raw.data() + k * 8, 8);
            } else if (h->prec == FDIRW_FP32) {
                float f;
                std::memcpy(&f, raw.data() + k * 4, 4);
                v = f;
            } else {
                uint16_t u;
                std::memcpy(&u, raw.data() + k * 2, 2);
                if (h->prec == FDIRW_BF16_BANK) {
                    const uint32_t w = (uint32_t)u << 16;
                    float f;
                    std::memcpy(&f, &w, 4);
                    v = f;
                } else {
                    _Float16 hv;
                    std::memcpy(&hv, &u, 2);
                    v = (double)(float)hv;
                }
            }
            P_host[(size_t)o * h->n_nodes + I] = v;
        }
    return FDIRW_OK;
}

int fdirw_coarse_destroy(void *handle)
{
    Coarse *h = (Coarse *)handle;
    if (!h) return FDIRW_OK;
    int dev = -1;
    (void)hipGetDevice(&dev);
    const int own = h->dev;
    if (dev != own) (void)hipSetDevice(own);
    delete h;
    if (dev != own && dev >= 0) (void)hipSetDevice(dev);
    return FDIRW_OK;
}

}  // extern "C"
