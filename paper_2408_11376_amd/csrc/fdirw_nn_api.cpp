// fdirw_nn_api.cpp -- host side of the learned window-kernel generator:
// the model handle, features / forward / backward / Adam on the device, and
// the surrogate big step (GEN_NN) with its FD audit and fallback.
//
// The surrogate replaces the per-source explicit FD of Sec. 3.1 (the columns
// of P) by a CNN evaluated on MFMA; the superposition of Eq. 8 is unchanged.
// Parameter layout (flat FP32): for each layer l = 0..4, w[co][ci][3][3][3]
// (tap order z, y, x) then b[co], channels 3, 16, 16, 16, 16, 1.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "fdirw_host.h"
#include "fdirw_launch.h"

namespace fdirw {

static const int kChan[6] = {3, 16, 16, 16, 16, 1};
static const int kStoreCI[5] = {8, 16, 16, 16, 16};     // input channels as stored (BF16 vectors of 8)
static const int kMbTrain = 128;                          // windows per training micro-batch
static const int kMbInfer = 4096;                         // windows per inference chunk
static const int kWgradGrid = 512;

static int64_t layer_w_off(int l)
{
    int64_t o = 0;
    for (int i = 0; i < l; ++i) o += (int64_t)kChan[i + 1] * kChan[i] * 27 + kChan[i + 1];
    return o;
}
static int64_t layer_b_off(int l) { return layer_w_off(l) + (int64_t)kChan[l + 1] * kChan[l] * 27; }
static int64_t num_params() { return layer_w_off(5); }

struct NnWork {
    int cap = 0;              // windows
    Buf src, X, S, h[4], zpre[4], z5, G, mass, targ, tmass, loss, dlog8, dh, dz, part, bpart, l1, kmm;
};

struct NnModel {
    int dev = -1;
    int n_sub = 0;
    int64_t t = 0;            // Adam steps taken
    bool dirty = true;        // training operand layouts out of date
    bool dirty_fused = true;  // fused inference layout out of date
    Buf theta, grad, m, v, prior, wp[5], wpf[5], wfu[5];
    NnWork ws;
    double last_loss[2] = {0.0, 0.0};
};

static void free_buf(Buf &b)
{
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.cap = 0;
}

static void free_model(NnModel *m)
{
    for (Buf *b : {&m->theta, &m->grad, &m->m, &m->v, &m->prior}) free_buf(*b);
    for (int l = 0; l < 5; ++l) { free_buf(m->wp[l]); free_buf(m->wpf[l]); free_buf(m->wfu[l]); }
    NnWork &w = m->ws;
    for (Buf *b : {&w.src, &w.X, &w.S, &w.z5, &w.G, &w.mass, &w.targ, &w.tmass, &w.loss, &w.dlog8, &w.dh, &w.dz,
                   &w.part, &w.bpart, &w.l1, &w.kmm})
        free_buf(*b);
    for (int l = 0; l < 4; ++l) { free_buf(w.h[l]); free_buf(w.zpre[l]); }
}

// SplitMix64 (Steele, Lea, Flood 2014) and Box-Muller normals for the
// default initialisation.
static uint64_t splitmix64(uint64_t x)
{
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

static double uniform01(uint64_t seed, uint64_t i)
{
    return ((double)(splitmix64(seed + (i + 1) * 0x9E3779B97F4A7C15ull) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

static int check_model(const void *h, NnModel **out)
{
    if (!h) return fail(FDIRW_E_ARG, "surrogate handle is null");
    NnModel *m = (NnModel *)h;
    int dev = -1;
    (void)hipGetDevice(&dev);
    if (dev != m->dev) return fail(FDIRW_E_ARG, "surrogate lives on device %d, current device is %d", m->dev, dev);
    *out = m;
    return FDIRW_OK;
}

static int nn_domain_check(const NnModel *m, const fdirw_domain *d)
{
    int rc = check_domain(d);
    if (rc) return rc;
    if (d->r != FDIRW_NN_RADIUS) return fail(FDIRW_E_ARG, "the surrogate needs r = %d (got %d)", FDIRW_NN_RADIUS, d->r);
    if (d->n_sub != m->n_sub)
        return fail(FDIRW_E_ARG, "the surrogate was built for n_sub = %d (got %d)", m->n_sub, d->n_sub);
    return FDIRW_OK;
}

// Work buffers for cap windows.  Inference (fused kernel) needs the source
// list, G, masses and the audit's FD targets; training adds every activation.
static int ensure_work(NnModel *m, int cap, bool train)
{
    NnWork &w = m->ws;
    const size_t V = NN_V;
    int rc;
    if ((rc = ensure(w.src, (size_t)cap * 8))) return rc;
    if ((rc = ensure(w.G, (size_t)cap * V * 4))) return rc;
    if ((rc = ensure(w.mass, (size_t)cap * 8))) return rc;
    if ((rc = ensure(w.targ, (size_t)cap * V * 4))) return rc;
    if ((rc = ensure(w.tmass, (size_t)cap * 8))) return rc;
    if ((rc = ensure(w.l1, (size_t)cap * 8))) return rc;
    if (train) {
        if ((rc = ensure(w.X, (size_t)cap * V * 8 * 2))) return rc;
        if ((rc = ensure(w.S, (size_t)cap * V))) return rc;
        if ((rc = ensure(w.z5, (size_t)cap * V * 4))) return rc;
        for (int l = 0; l < 4; ++l) {
            if ((rc = ensure(w.h[l], (size_t)cap * V * 16 * 2))) return rc;
            if ((rc = ensure(w.zpre[l], (size_t)cap * V * 16 * 4))) return rc;
        }
        if ((rc = ensure(w.loss, (size_t)cap * 16))) return rc;
        if ((rc = ensure(w.dlog8, (size_t)cap * V * 8 * 2))) return rc;
        if ((rc = ensure(w.dh, (size_t)cap * V * 16 * 4))) return rc;
        if ((rc = ensure(w.dz, (size_t)cap * V * 16 * 2))) return rc;
        if ((rc = ensure(w.part, (size_t)kWgradGrid * 27 * 256 * 4))) return rc;
        if ((rc = ensure(w.bpart, (size_t)kWgradGrid * 16 * 4))) return rc;
    }
    w.cap = cap;
    return FDIRW_OK;
}

// Packs the BF16 MFMA operands from the FP32 parameters when they changed:
// the training layouts (forward and input-gradient) or the fused inference
// layout, whichever the caller is about to use.
static int pack_weights(NnModel *m, hipStream_t st, bool fused)
{
    const float *th = (const float *)m->theta.p;
    hipError_t e = hipSuccess;
    if (fused && m->dirty_fused) {
        for (int l = 0; l < 5 && e == hipSuccess; ++l)
            e = nn_launch_fpack(th + layer_w_off(l), l, kChan[l + 1], kChan[l], (uint16_t *)m->wfu[l].p, st);
        if (e == hipSuccess) m->dirty_fused = false;
    }
    if (!fused && m->dirty) {
        for (int l = 0; l < 5 && e == hipSuccess; ++l) {
            e = nn_launch_pack(th + layer_w_off(l), kChan[l + 1], kChan[l], kStoreCI[l], 0, (uint16_t *)m->wp[l].p, st);
            // input-gradient weights: input channels = this layer's outputs (8 slots for the last layer)
            if (e == hipSuccess && l >= 1)
                e = nn_launch_pack(th + layer_w_off(l), kChan[l + 1], kChan[l], l == 4 ? 8 : 16, 1,
                                   (uint16_t *)m->wpf[l].p, st);
        }
        if (e == hipSuccess) m->dirty = false;
    }
    return e == hipSuccess ? FDIRW_OK : hip_fail(e, "weight packing");
}

static void feature_tables(const fdirw_domain *d, NnFeatArgs &a)
{
    for (int p = 0; p < 256; ++p) {
        const double D = p < d->n_phase ? d->d_phase[p] : 0.0;
        a.open[p] = D > 0.0 ? 1 : 0;
        a.f1[p] = D > 0.0 ? (float)(std::fmax(std::log10(D), -12.0) / 6.0 + 1.0) : -1.0f;
    }
}

// Features and support for n windows whose sources are in ws.src.
static int run_features(NnModel *m, const fdirw_domain *d, int n, hipStream_t st)
{
    NnFeatArgs a;
    a.nx = d->nx; a.ny = d->ny; a.nz = d->nz;
    a.n_sub = d->n_sub;
    a.src = (const int64_t *)m->ws.src.p;
    a.label = d->label;
    feature_tables(d, a);
    a.prior = (const float *)m->prior.p;
    a.X = (uint16_t *)m->ws.X.p;
    a.support = (uint8_t *)m->ws.S.p;
    hipError_t e = nn_launch_features(a, n, st);
    return e == hipSuccess ? FDIRW_OK : hip_fail(e, "feature launch");
}

// Layer-by-layer forward pass of n windows for training: keeps every
// activation and pre-activation for the backward pass.
static int run_forward(NnModel *m, int n, bool train, hipStream_t st)
{
    NnWork &w = m->ws;
    const float *th = (const float *)m->theta.p;
    const uint16_t *in = (const uint16_t *)w.X.p;
    hipError_t e = hipSuccess;
    for (int l = 0; l < 5 && e == hipSuccess; ++l) {
        NnConvArgs a;
        a.in = in;
        a.wpack = (const uint16_t *)m->wp[l].p;
        a.bias = th + layer_b_off(l);
        a.zpre = nullptr; a.hout = nullptr; a.z5 = nullptr; a.dh = nullptr;
        if (l < 4) {
            a.mode = 0;
            uint16_t *out = (uint16_t *)(train ? w.h[l].p : w.h[l & 1].p);
            a.hout = out;
            if (train) a.zpre = (float *)w.zpre[l].p;
            e = nn_launch_conv(kStoreCI[l], a, n, st);
            in = out;
        } else {
            a.mode = 1;
            a.z5 = (float *)w.z5.p;
            e = nn_launch_conv(16, a, n, st);
        }
    }
    return e == hipSuccess ? FDIRW_OK : hip_fail(e, "forward launch");
}

// Backward pass of n windows after run_forward(train) and the loss kernel
// (which wrote d loss / d logits into dlog8); accumulates into grad.
static int run_backward(NnModel *m, int n, hipStream_t st)
{
    NnWork &w = m->ws;
    float *g = (float *)m->grad.p;
    const int nslab = n * nn_slabs_per_window();
    const int grid = nslab < kWgradGrid ? nslab : kWgradGrid;
    const int64_t nel = (int64_t)n * NN_V * 16;
    hipError_t e = hipSuccess;
    const uint16_t *dz = (const uint16_t *)w.dlog8.p;     // gradient at the output of layer l
    int cop = 8;
    for (int l = 4; l >= 0 && e == hipSuccess; --l) {
        NnWgradArgs wa;
        wa.dz = dz;
        wa.h = (const uint16_t *)(l == 0 ? w.X.p : w.h[l - 1].p);
        wa.co_n = kChan[l + 1];
        wa.ci_n = kChan[l];
        wa.n_slab = nslab;
        wa.part = (float *)w.part.p;
        wa.bpart = (float *)w.bpart.p;
        e = nn_launch_wgrad(kStoreCI[l], cop, wa, grid, st);
        if (e == hipSuccess)
            e = nn_launch_wgrad_reduce(wa.part, wa.bpart, grid, kChan[l + 1], kChan[l], g + layer_w_off(l),
                                       g + layer_b_off(l), st);
        if (l == 0 || e != hipSuccess) break;
        // gradient at the input of layer l = output of layer l - 1 (FP32), then
        // through that layer's SiLU into BF16
        NnConvArgs ca;
        ca.in = dz;
        ca.wpack = (const uint16_t *)m->wpf[l].p;
        ca.bias = nullptr;
        ca.mode = 2;
        ca.zpre = nullptr; ca.hout = nullptr; ca.z5 = nullptr;
        ca.dh = (float *)w.dh.p;
        e = nn_launch_conv(cop, ca, n, st);
        if (e == hipSuccess) e = nn_launch_silu_bwd((const float *)w.dh.p, (const float *)w.zpre[l - 1].p,
                                                    (uint16_t *)w.dz.p, nel, st);
        dz = (const uint16_t *)w.dz.p;
        cop = 16;
    }
    return e == hipSuccess ? FDIRW_OK : hip_fail(e, "backward launch");
}

static int check_sources(const int64_t *src, int64_t n_src, int64_t n, DevCache &dc, hipStream_t st)
{
    int rc;
    if ((rc = ensure(dc.flags, 16 * sizeof(unsigned)))) return rc;
    unsigned *bad = (unsigned *)dc.flags.p + 12;
    hipError_t e = launch_src_check(src, n_src, n, bad, st);
    unsigned h_bad = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&h_bad, bad, sizeof h_bad, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "source check");
    if (h_bad) return fail(FDIRW_E_ARG, "a source index is outside [0, %lld)", (long long)n);
    return FDIRW_OK;
}

// FD targets (FP32, unit mass) of the n windows whose sources are in ws.src.
static int fd_targets(NnModel *m, const fdirw_domain *d, const void *lam32, int n, hipStream_t st)
{
    WindowArgs a;
    a.nx = d->nx; a.ny = d->ny; a.nz = d->nz;
    a.n = (int64_t)d->nx * d->ny * d->nz;
    a.n_sub = d->n_sub;
    a.lx = lam32;
    a.src = (const int64_t *)m->ws.src.p;
    a.n_src = n;
    a.G = m->ws.targ.p;
    a.mass = (double *)m->ws.tmass.p;
    a.normalize = 1;
    a.out_lp = 0;
    a.offset_major = 0;
    hipError_t e = launch_window(FDIRW_FP32, NN_R, a, st);
    return e == hipSuccess ? FDIRW_OK : hip_fail(e, "FD target launch");
}

// Fused inference of n windows whose sources are in ws.src: G, mass and the
// optional logits / support outputs.
static int run_fused(NnModel *m, const fdirw_domain *d, int n, float *G, double *mass, float *logits,
                     uint8_t *support, hipStream_t st)
{
    NnFusedArgs a;
    a.nx = d->nx; a.ny = d->ny; a.nz = d->nz;
    a.n_sub = d->n_sub;
    a.src = (const int64_t *)m->ws.src.p;
    a.label = d->label;
    NnFeatArgs t;
    feature_tables(d, t);
    for (int i = 0; i < 256; ++i) { a.f1[i] = t.f1[i]; a.open[i] = t.open[i]; }
    a.prior = (const float *)m->prior.p;
    const float *th = (const float *)m->theta.p;
    for (int l = 0; l < 5; ++l) {
        a.wf[l] = (const uint16_t *)m->wfu[l].p;
        a.bias[l] = th + layer_b_off(l);
    }
    a.G = G; a.mass = mass; a.logits = logits; a.support = support;
    a.z5g = G ? G : (float *)m->ws.G.p;
    hipError_t e = nn_launch_fused(a, n, st);
    return e == hipSuccess ? FDIRW_OK : hip_fail(e, "fused surrogate launch");
}

// ----------------------------------------------------------------- surrogate step

static uint64_t audit_index(uint64_t k, uint64_t n) { return splitmix64(0xA0D17ull + k) % n; }

int step_nn(const fdirw_domain *d, const fdirw_opts *o, const double *c_in, double *c_out, fdirw_stats *st,
            DevCache &dc, hipStream_t stream)
{
    NnModel *m = nullptr;
    int rc;
    if ((rc = check_model(o->nn, &m))) return rc;
    if ((rc = nn_domain_check(m, d))) return rc;
    Geometry geo;
    const void *lam32 = nullptr;
    if ((rc = coef_buffers(d, FDIRW_FP32, stream, dc, &geo, &lam32))) return rc;
    const int64_t n = geo.n;
    if ((rc = ensure_work(m, kMbInfer > d->nz ? kMbInfer : d->nz, false))) return rc;
    if ((rc = pack_weights(m, stream, true))) return rc;
    NnWork &w = m->ws;

    // audit: K seeded sources, mean per-kernel L1 of the surrogate against FD
    int64_t K = o->audit_samples > 0 ? o->audit_samples : 1024;
    if (K > n) K = n;
    const double tol = o->audit_tol > 0.0 ? o->audit_tol : 1e-3;
    double l1_sum = 0.0;
    std::vector<int64_t> hsrc;
    std::vector<double> hl1;
    for (int64_t k0 = 0; k0 < K; k0 += w.cap) {
        const int nb = (int)((K - k0) < w.cap ? (K - k0) : w.cap);
        hsrc.resize(nb);
        hl1.resize(nb);
        for (int i = 0; i < nb; ++i) hsrc[i] = (int64_t)audit_index((uint64_t)(k0 + i), (uint64_t)n);
        hipError_t e = hipMemcpyAsync(w.src.p, hsrc.data(), (size_t)nb * 8, hipMemcpyHostToDevice, stream);
        if (e != hipSuccess) return hip_fail(e, "audit sources");
        if ((rc = run_fused(m, d, nb, (float *)w.G.p, (double *)w.mass.p, nullptr, nullptr, stream))) return rc;
        if ((rc = fd_targets(m, d, lam32, nb, stream))) return rc;
        e = nn_launch_l1((const float *)w.G.p, (const float *)w.targ.p, nb, (double *)w.l1.p, stream);
        if (e == hipSuccess) e = hipMemcpyAsync(hl1.data(), w.l1.p, (size_t)nb * 8, hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return hip_fail(e, "audit");
        for (int i = 0; i < nb; ++i) l1_sum += hl1[i];
    }
    const double audit_l1 = K > 0 ? l1_sum / (double)K : 0.0;
    if (!(audit_l1 <= tol)) {
        // the surrogate is not accurate enough on this geometry: plain FD step
        fdirw_opts fo = *o;
        fo.gen = FDIRW_GEN_FD;
        if ((rc = step_one(d, &fo, c_in, c_out, st, dc, stream, false, nullptr, nullptr))) return rc;
        if (st) {
            st->audit_l1 = audit_l1;
            st->fallback_used = 1;
        }
        return FDIRW_OK;
    }

    if (st) {
        if ((rc = field_sum_dev(c_in, n, stream, dc, &st->mass_in))) return rc;
        if (!std::isfinite(st->mass_in)) return fail(FDIRW_E_NONFINITE, "input mass is not finite");
    }
    const int nz = d->nz;
    const int64_t lines = (int64_t)d->nx * d->ny;
    const int per = w.cap / nz > 0 ? w.cap / nz : 1;        // lines per chunk
    const int64_t n_chunks = (lines + per - 1) / per;
    if ((rc = ensure(w.kmm, (size_t)n_chunks * 16))) return rc;
    if ((rc = ensure(dc.small, 64))) return rc;
    unsigned long long *used = (unsigned long long *)dc.small.p;
    hipError_t e = launch_fill(c_out, n, 0.0, stream);
    if (e == hipSuccess) e = launch_fill_u32((unsigned *)used, 2, 0u, stream);
    if (e != hipSuccess) return hip_fail(e, "output clear");
    EventPair ev;
    if (st && (e = ev.create()) != hipSuccess) return hip_fail(e, "event create");
    if (st) (void)hipEventRecord(ev.a, stream);
    int64_t ci = 0;
    for (int64_t l0 = 0; l0 < lines; l0 += per, ++ci) {
        const int nl = (int)((lines - l0) < per ? (lines - l0) : per);
        const int nb = nl * nz;
        e = nn_launch_lines_src(l0, nl, d->nx, d->ny, nz, (int64_t *)w.src.p, stream);
        if (e != hipSuccess) return hip_fail(e, "source list");
        if ((rc = run_fused(m, d, nb, (float *)w.G.p, (double *)w.mass.p, nullptr, nullptr, stream))) return rc;
        int n_seg = (int)((1024 + nl - 1) / nl);
        if (n_seg > nz) n_seg = nz;
        const int seg_len = (nz + n_seg - 1) / n_seg;
        n_seg = (nz + seg_len - 1) / seg_len;
        e = nn_launch_apply(d->nx, d->ny, nz, l0, nl, seg_len, n_seg, (const float *)w.G.p,
                            (const double *)w.mass.p, c_in, c_out, used, stream);
        if (e == hipSuccess && st)
            e = launch_minmax_scalar((const double *)w.mass.p, nb, nullptr, (double *)w.kmm.p + 2 * ci, stream);
        if (e != hipSuccess) return hip_fail(e, "surrogate superposition");
    }
    if (st) (void)hipEventRecord(ev.b, stream);
    if (st) {
        if ((rc = field_sum_dev(c_out, n, stream, dc, &st->mass_out))) return rc;
        double *mm = (double *)dc.small.p + 2;
        e = launch_minmax((const double *)w.kmm.p, n_chunks, mm, stream);
        double h_mm[2];
        unsigned long long h_used = 0;
        if (e == hipSuccess) e = hipMemcpyAsync(h_mm, mm, sizeof h_mm, hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipMemcpyAsync(&h_used, used, sizeof h_used, hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return hip_fail(e, "step statistics");
        st->kmass_min = h_mm[0];
        st->kmass_max = h_mm[1];
        st->n_sources = (int64_t)h_used;
        st->kernel_seconds = ev.seconds();
        st->audit_l1 = audit_l1;
        st->fallback_used = 0;
        st->bank_used = 0;
        st->tuned_config_id = 0;
    }
    return FDIRW_OK;
}

}  // namespace fdirw

using namespace fdirw;

extern "C" {

int64_t fdirw_nn_num_params(void) { return num_params(); }

int fdirw_nn_create(int32_t n_sub, uint64_t seed, void **nn)
{
    if (!nn) return fail(FDIRW_E_ARG, "nn is null");
    *nn = nullptr;
    if (n_sub < 0) return fail(FDIRW_E_ARG, "n_sub = %d must be >= 0", n_sub);
    std::lock_guard<std::mutex> lk(cache_mutex());
    NnModel *m = new (std::nothrow) NnModel;
    if (!m) return fail(FDIRW_E_NOMEM, "host allocation failed");
    (void)hipGetDevice(&m->dev);
    m->n_sub = n_sub;
    const int64_t np = num_params();
    int rc = FDIRW_OK;
    for (Buf *b : {&m->theta, &m->grad, &m->m, &m->v})
        if (!rc) rc = ensure(*b, (size_t)np * 4);
    if (!rc) rc = ensure(m->prior, (size_t)NN_V * 4);
    for (int l = 0; l < 5 && !rc; ++l) {
        rc = ensure(m->wp[l], (size_t)nn_pack_chunks(kStoreCI[l]) * 512 * 2);
        if (!rc) rc = ensure(m->wpf[l], (size_t)nn_pack_chunks(16) * 512 * 2);
        if (!rc) rc = ensure(m->wfu[l], (size_t)nn_fpack_elems(l) * 2);
    }
    // default parameters: He-normal for the SiLU layers, a tenth of that for
    // the last layer (so an untrained model starts at the prior), zero biases
    std::vector<float> th((size_t)np, 0.0f);
    for (int l = 0; l < 5; ++l) {
        const int64_t nw = (int64_t)kChan[l + 1] * kChan[l] * 27;
        const double std = std::sqrt(2.0 / (kChan[l] * 27.0)) * (l == 4 ? 0.1 : 1.0);
        for (int64_t i = 0; i < nw; ++i) {
            const uint64_t key = seed * 16 + (uint64_t)l;
            const double u1 = uniform01(key, 2 * (uint64_t)i), u2 = uniform01(key, 2 * (uint64_t)i + 1);
            th[(size_t)(layer_w_off(l) + i)] = (float)(std * std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2));
        }
    }
    // prior: log of the FD kernel of an all-permeable W^3 window with D = 1,
    // h = 1 and dt = 0.9 / 6 (lambda = 0.15 on every face), in FP64
    uint8_t *lab = nullptr;
    int64_t *src = nullptr;
    double *G = nullptr, *mass = nullptr;
    hipStream_t st = nullptr;
    std::vector<double> hG(NN_V);
    if (!rc) {
        hipError_t e = hipMalloc(&lab, NN_V);
        if (e == hipSuccess) e = hipMalloc(&src, 8);
        if (e == hipSuccess) e = hipMalloc(&G, (size_t)NN_V * 8);
        if (e == hipSuccess) e = hipMalloc(&mass, 8);
        const int64_t centre = ((int64_t)NN_R * NN_W + NN_R) * NN_W + NN_R;
        if (e == hipSuccess) e = hipMemset(lab, 0, NN_V);
        if (e == hipSuccess) e = hipMemcpy(src, &centre, 8, hipMemcpyHostToDevice);
        if (e != hipSuccess) rc = hip_fail(e, "prior set-up");
    }
    if (!rc) {
        DevCache &dc = cache_for_current_device();
        const double one = 1.0;
        fdirw_domain pd;
        pd.nx = pd.ny = pd.nz = NN_W;
        pd.h = 1.0;
        pd.label = lab;
        pd.d_phase = &one;
        pd.n_phase = 1;
        pd.r = NN_R;
        pd.n_sub = n_sub;
        pd.dt = 0.0;
        Geometry g;
        const void *lam = nullptr;
        rc = coef_buffers(&pd, FDIRW_FP64, st, dc, &g, &lam);
        if (!rc) {
            WindowArgs a;
            a.nx = a.ny = a.nz = NN_W;
            a.n = NN_V;
            a.n_sub = n_sub;
            a.lx = lam;
            a.src = src; a.n_src = 1;
            a.G = G; a.mass = mass;
            a.normalize = 0;
            a.out_lp = 0;
            a.offset_major = 0;
            hipError_t e = launch_window(FDIRW_FP64, NN_R, a, st);
            if (e == hipSuccess) e = hipMemcpy(hG.data(), G, (size_t)NN_V * 8, hipMemcpyDeviceToHost);
            if (e != hipSuccess) rc = hip_fail(e, "prior kernel");
        }
    }
    if (lab) (void)hipFree(lab);
    if (src) (void)hipFree(src);
    if (G) (void)hipFree(G);
    if (mass) (void)hipFree(mass);
    if (!rc) {
        std::vector<float> pr(NN_V);
        for (int i = 0; i < NN_V; ++i) pr[i] = (float)std::log(std::fmax(hG[i], 1e-30));
        hipError_t e = hipMemcpy(m->prior.p, pr.data(), (size_t)NN_V * 4, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(m->theta.p, th.data(), (size_t)np * 4, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemset(m->m.p, 0, (size_t)np * 4);
        if (e == hipSuccess) e = hipMemset(m->v.p, 0, (size_t)np * 4);
        if (e == hipSuccess) e = hipMemset(m->grad.p, 0, (size_t)np * 4);
        if (e != hipSuccess) rc = hip_fail(e, "parameter upload");
    }
    if (rc) {
        free_model(m);
        delete m;
        return rc;
    }
    *nn = m;
    return FDIRW_OK;
}

int fdirw_nn_destroy(void *nn)
{
    if (!nn) return FDIRW_OK;
    std::lock_guard<std::mutex> lk(cache_mutex());
    NnModel *m = (NnModel *)nn;
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(m->dev);
    free_model(m);
    (void)hipSetDevice(prev);
    delete m;
    return FDIRW_OK;
}

int fdirw_nn_set_params(void *nn, const float *theta)
{
    NnModel *m = nullptr;
    int rc = check_model(nn, &m);
    if (rc) return rc;
    if (!theta) return fail(FDIRW_E_ARG, "theta is null");
    std::lock_guard<std::mutex> lk(cache_mutex());
    hipError_t e = hipMemcpy(m->theta.p, theta, (size_t)num_params() * 4, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "parameter upload");
    m->dirty = m->dirty_fused = true;
    return FDIRW_OK;
}

int fdirw_nn_get_params(const void *nn, float *theta)
{
    NnModel *m = nullptr;
    int rc = check_model(nn, &m);
    if (rc) return rc;
    if (!theta) return fail(FDIRW_E_ARG, "theta is null");
    std::lock_guard<std::mutex> lk(cache_mutex());
    hipError_t e = hipMemcpy(theta, m->theta.p, (size_t)num_params() * 4, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "parameter download");
    return FDIRW_OK;
}

int fdirw_nn_forward(void *nn, const fdirw_domain *d, const int64_t *src, int64_t n_src, float *G,
                     uint8_t *support, float *logits, void *stream)
{
    NnModel *m = nullptr;
    int rc = check_model(nn, &m);
    if (rc) return rc;
    if ((rc = nn_domain_check(m, d))) return rc;
    if (n_src < 0) return fail(FDIRW_E_ARG, "n_src < 0");
    if (n_src == 0) return FDIRW_OK;
    if (!src) return fail(FDIRW_E_ARG, "src is null");
    std::lock_guard<std::mutex> lk(cache_mutex());
    DevCache &dc = cache_for_current_device();
    hipStream_t st = (hipStream_t)stream;
    const int64_t n = (int64_t)d->nx * d->ny * d->nz;
    if ((rc = check_sources(src, n_src, n, dc, st))) return rc;
    Geometry geo;
    const void *lam32 = nullptr;
    if ((rc = coef_buffers(d, FDIRW_FP32, st, dc, &geo, &lam32))) return rc;   // validates labels
    if ((rc = ensure_work(m, kMbInfer, false))) return rc;
    if ((rc = pack_weights(m, st, true))) return rc;
    NnWork &w = m->ws;
    for (int64_t k0 = 0; k0 < n_src; k0 += w.cap) {
        const int nb = (int)((n_src - k0) < w.cap ? (n_src - k0) : w.cap);
        hipError_t e = hipMemcpyAsync(w.src.p, src + k0, (size_t)nb * 8, hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return hip_fail(e, "source copy");
        if ((rc = run_fused(m, d, nb, G ? G + k0 * NN_V : nullptr, (double *)w.mass.p,
                            logits ? logits + k0 * NN_V : nullptr, support ? support + k0 * NN_V : nullptr, st)))
            return rc;
    }
    return FDIRW_OK;
}

int fdirw_nn_backward(void *nn, const fdirw_domain *d, const int64_t *src, int64_t n_src, const float *target,
                      float *grad, double *loss, void *stream)
{
    NnModel *m = nullptr;
    int rc = check_model(nn, &m);
    if (rc) return rc;
    if ((rc = nn_domain_check(m, d))) return rc;
    if (n_src < 1) return fail(FDIRW_E_ARG, "n_src = %lld must be >= 1", (long long)n_src);
    if (!src) return fail(FDIRW_E_ARG, "src is null");
    std::lock_guard<std::mutex> lk(cache_mutex());
    DevCache &dc = cache_for_current_device();
    hipStream_t st = (hipStream_t)stream;
    const int64_t n = (int64_t)d->nx * d->ny * d->nz;
    if ((rc = check_sources(src, n_src, n, dc, st))) return rc;
    Geometry geo;
    const void *lam32 = nullptr;
    if ((rc = coef_buffers(d, FDIRW_FP32, st, dc, &geo, &lam32))) return rc;
    if ((rc = ensure_work(m, kMbTrain, true))) return rc;
    if ((rc = pack_weights(m, st, false))) return rc;
    NnWork &w = m->ws;
    const int64_t np = num_params();
    hipError_t e = nn_launch_fill_f32((float *)m->grad.p, np, 0.0f, st);
    if (e != hipSuccess) return hip_fail(e, "gradient clear");
    const float scale = (float)(1.0 / (double)n_src);
    double kl = 0.0, l1 = 0.0;
    std::vector<double> hl((size_t)2 * kMbTrain);
    for (int64_t k0 = 0; k0 < n_src; k0 += kMbTrain) {
        const int nb = (int)((n_src - k0) < kMbTrain ? (n_src - k0) : kMbTrain);
        e = hipMemcpyAsync(w.src.p, src + k0, (size_t)nb * 8, hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return hip_fail(e, "source copy");
        if ((rc = run_features(m, d, nb, st))) return rc;
        const float *tg = target ? target + k0 * NN_V : (const float *)w.targ.p;
        if (!target && (rc = fd_targets(m, d, lam32, nb, st))) return rc;
        if ((rc = run_forward(m, nb, true, st))) return rc;
        NnLossArgs la;
        la.z5 = (const float *)w.z5.p;
        la.prior = (const float *)m->prior.p;
        la.support = (const uint8_t *)w.S.p;
        la.target = tg;
        la.G = nullptr;
        la.mass = nullptr;
        la.logits = nullptr;
        la.loss = (double *)w.loss.p;
        la.dlog8 = (uint16_t *)w.dlog8.p;
        la.grad_scale = scale;
        e = nn_launch_loss(la, nb, st);
        if (e != hipSuccess) return hip_fail(e, "loss launch");
        if ((rc = run_backward(m, nb, st))) return rc;
        e = hipMemcpyAsync(hl.data(), w.loss.p, (size_t)nb * 16, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(e, "loss readback");
        for (int i = 0; i < nb; ++i) { kl += hl[2 * i]; l1 += hl[2 * i + 1]; }
    }
    if (grad) {
        e = hipMemcpyAsync(grad, m->grad.p, (size_t)np * 4, hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return hip_fail(e, "gradient copy");
    }
    m->last_loss[0] = kl / (double)n_src;
    m->last_loss[1] = l1 / (double)n_src;
    if (loss) { loss[0] = m->last_loss[0]; loss[1] = m->last_loss[1]; }
    return FDIRW_OK;
}

int fdirw_nn_adam(void *nn, double lr, double beta1, double beta2, double eps, void *stream)
{
    NnModel *m = nullptr;
    int rc = check_model(nn, &m);
    if (rc) return rc;
    if (!(lr >= 0.0) || !(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0) || !(eps > 0.0))
        return fail(FDIRW_E_ARG, "Adam needs lr >= 0, 0 <= beta < 1, eps > 0");
    std::lock_guard<std::mutex> lk(cache_mutex());
    m->t += 1;
    const double c1 = 1.0 - std::pow(beta1, (double)m->t), c2 = 1.0 - std::pow(beta2, (double)m->t);
    hipError_t e = nn_launch_adam((float *)m->theta.p, (float *)m->m.p, (float *)m->v.p, (const float *)m->grad.p,
                                  (int)num_params(), (float)lr, (float)beta1, (float)beta2, (float)eps, (float)c1,
                                  (float)c2, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "Adam launch");
    m->dirty = m->dirty_fused = true;
    return FDIRW_OK;
}

static const char kMagic[8] = {'F', 'D', 'I', 'R', 'W', 'N', 'N', '1'};

int fdirw_nn_save(const void *nn, const char *path)
{
    NnModel *m = nullptr;
    int rc = check_model(nn, &m);
    if (rc) return rc;
    if (!path) return fail(FDIRW_E_ARG, "path is null");
    std::lock_guard<std::mutex> lk(cache_mutex());
    const int64_t np = num_params();
    std::vector<float> buf((size_t)np * 3);
    hipError_t e = hipMemcpy(buf.data(), m->theta.p, (size_t)np * 4, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(buf.data() + np, m->m.p, (size_t)np * 4, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(buf.data() + 2 * np, m->v.p, (size_t)np * 4, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "parameter download");
    FILE *f = std::fopen(path, "wb");
    if (!f) return fail(FDIRW_E_ARG, "cannot open %s for writing", path);
    const int32_t hdr[2] = {m->n_sub, 0};
    const int64_t nums[2] = {np, m->t};
    bool ok = std::fwrite(kMagic, 1, 8, f) == 8 && std::fwrite(hdr, 4, 2, f) == 2 && std::fwrite(nums, 8, 2, f) == 2 &&
              std::fwrite(buf.data(), 4, buf.size(), f) == buf.size();
    ok = (std::fclose(f) == 0) && ok;
    return ok ? FDIRW_OK : fail(FDIRW_E_ARG, "write to %s failed", path);
}

int fdirw_nn_load(void *nn, const char *path)
{
    NnModel *m = nullptr;
    int rc = check_model(nn, &m);
    if (rc) return rc;
    if (!path) return fail(FDIRW_E_ARG, "path is null");
    std::lock_guard<std::mutex> lk(cache_mutex());
    FILE *f = std::fopen(path, "rb");
    if (!f) return fail(FDIRW_E_ARG, "cannot open %s", path);
    char magic[8];
    int32_t hdr[2];
    int64_t nums[2];
    const int64_t np = num_params();
    std::vector<float> buf((size_t)np * 3);
    bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, kMagic, 8) == 0 && std::fread(hdr, 4, 2, f) == 2 &&
              std::fread(nums, 8, 2, f) == 2 && nums[0] == np && hdr[0] == m->n_sub &&
              std::fread(buf.data(), 4, buf.size(), f) == buf.size();
    std::fclose(f);
    if (!ok) return fail(FDIRW_E_ARG, "%s is not a surrogate file for n_sub = %d", path, m->n_sub);
    hipError_t e = hipMemcpy(m->theta.p, buf.data(), (size_t)np * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m->m.p, buf.data() + np, (size_t)np * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m->v.p, buf.data() + 2 * np, (size_t)np * 4, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "parameter upload");
    m->t = nums[1];
    m->dirty = m->dirty_fused = true;
    return FDIRW_OK;
}

}  // extern "C"
