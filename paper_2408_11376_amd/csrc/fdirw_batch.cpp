// fdirw_batch.cpp -- host side of the batched persistent launch and of its
// autotuner (fdirw_step / fdirw_run with n_dom > 1).
//
// Work items: a domain, a group of consecutive source lines (as many as the
// radius lets one workgroup hold) and a range of source planes.  Launch shape
// choices the tuner explores: the workgroup layout (the 640-thread segment
// layout, which packs several small windows per workgroup, or the 256-thread
// flat layout of the single-domain FP32 step, one to four windows per
// workgroup by radius and two workgroups per CU), the z extent of an item (long items amortise the
// per-item LDS setup; short items balance the load at the end of the queue)
// and the queue order (natural, or longest-processing-time first).  The tuner
// times each candidate on an evenly spaced sample of the real items, with HIP
// events, normalised by the sample's modelled cost (windows x cells x
// sub-steps), and caches the winner per (precision, radii / sub-step mix, size
// class, device); the cache can be kept in a text file named by the
// environment variable FDIRW_TUNE_CACHE.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <string>
#include <vector>

#include "fdirw_host.h"
#include "fdirw_launch.h"

namespace fdirw {

struct BatchConfig {
    int zlen;       // planes per item, 0 = whole column of sources
    int lpt;        // 1 = longest item first
    int flat;       // 1 = flat layout (FP32 only): flat_lines_per_group(r) lines per item
};

static const BatchConfig kConfigs[] = {
    {0, 0, 0}, {0, 1, 0}, {64, 1, 0}, {32, 1, 0}, {16, 1, 0}, {8, 1, 0},
    {0, 1, 1}, {64, 1, 1}, {32, 1, 1}, {16, 1, 1},
};

static bool config_valid(int id, int prec) { return !kConfigs[id].flat || prec == FDIRW_FP32; }
static const int kNumConfigs = (int)(sizeof(kConfigs) / sizeof(kConfigs[0]));

int batch_config_count() { return kNumConfigs; }

static std::map<std::string, int> g_tune_cache;
static bool g_tune_loaded = false;

static void load_tune_file()
{
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char *path = std::getenv("FDIRW_TUNE_CACHE");
    if (!path) return;
    FILE *f = std::fopen(path, "r");
    if (!f) return;
    char key[512];
    int id;
    while (std::fscanf(f, "%511s %d", key, &id) == 2)
        if (id >= 0 && id < kNumConfigs) g_tune_cache[key] = id;
    std::fclose(f);
}

static void store_tune_file()
{
    const char *path = std::getenv("FDIRW_TUNE_CACHE");
    if (!path) return;
    FILE *f = std::fopen(path, "w");
    if (!f) return;
    for (auto &kv : g_tune_cache) std::fprintf(f, "%s %d\n", kv.first.c_str(), kv.second);
    std::fclose(f);
}

static std::string tune_key(const fdirw_domain *d, int n_dom, int prec)
{
    std::vector<std::pair<int, int>> rn;
    double cells = 0.0;
    for (int i = 0; i < n_dom; ++i) {
        rn.push_back({d[i].r, d[i].n_sub});
        cells += (double)d[i].nx * d[i].ny * d[i].nz;
    }
    std::sort(rn.begin(), rn.end());
    rn.erase(std::unique(rn.begin(), rn.end()), rn.end());
    int dev = 0;
    (void)hipGetDevice(&dev);
    hipDeviceProp_t prop;
    std::string arch = "gfx";
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
    for (char &ch : arch)
        if (ch == ':') ch = '_';
    std::string k = arch + "|p" + std::to_string(prec) + "|c" + std::to_string((int)std::log2(cells + 1.0));
    for (auto &x : rn) k += "|r" + std::to_string(x.first) + "n" + std::to_string(x.second);
    return k;
}

static int lines_per_item(const BatchConfig &cfg, int r)
{
    return cfg.flat ? flat_lines_per_group(r) : batch_windows_per_group(r);
}

static double item_cost(const fdirw_domain &d, const BatchItem &it, const BatchConfig &cfg)
{
    const double W = 2.0 * d.r + 1.0;
    const int ng = lines_per_item(cfg, d.r);
    return (double)ng * (it.z1 - it.z0) * W * W * W * (d.n_sub > 0 ? d.n_sub : 1);
}

static void build_items(const fdirw_domain *d, int n_dom, const BatchConfig &cfg, std::vector<BatchItem> &items)
{
    items.clear();
    for (int i = 0; i < n_dom; ++i) {
        const int lines = d[i].nx * d[i].ny;
        const int ng = lines_per_item(cfg, d[i].r);
        const int zl = cfg.zlen > 0 ? cfg.zlen : d[i].nz;
        for (int l0 = 0; l0 < lines; l0 += ng)
            for (int z0 = 0; z0 < d[i].nz; z0 += zl) {
                BatchItem it;
                it.dom = i;
                it.line0 = l0;
                it.nlines = std::min(ng, lines - l0);
                it.z0 = z0;
                it.z1 = std::min(d[i].nz, z0 + zl);
                items.push_back(it);
            }
    }
    if (cfg.lpt) {
        std::stable_sort(items.begin(), items.end(), [&](const BatchItem &a, const BatchItem &b) {
            return item_cost(d[a.dom], a, cfg) > item_cost(d[b.dom], b, cfg);
        });
    }
}

static int batch_grid(int prec, int flat, int *grid)
{
    int dev = 0, cus = 0, occ = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = flat ? batched_flat_occupancy(&occ) : batched_occupancy(prec, &occ);
    if (e != hipSuccess) return hip_fail(e, "batched occupancy");
    if (occ < 1) occ = 1;
    *grid = cus * occ;
    return FDIRW_OK;
}

// Launch the items (already on the device) after clearing the queue counter.
static int launch_items(int prec, int flat, const BatchDom *ddoms, const BatchItem *ditems, int n_items,
                        double *kmass, DevCache &dc, int grid, hipStream_t st)
{
    unsigned *head = (unsigned *)dc.small.p + 14;
    hipError_t e = launch_fill_u32(head, 1, 0u, st);
    BatchArgs a;
    a.doms = ddoms;
    a.items = ditems;
    a.n_items = n_items;
    a.head = head;
    a.item_kmass = kmass;
    if (e == hipSuccess) e = flat ? launch_batched_flat(a, grid, st) : launch_batched(prec, a, grid, st);
    if (e != hipSuccess) return hip_fail(e, "batched launch");
    return FDIRW_OK;
}

// Times every candidate on a sample of its own items; returns the best id.
static int autotune(const fdirw_domain *d, int n_dom, int prec, const BatchDom *ddoms, double *const *c_out,
                    DevCache &dc, hipStream_t st, int *best_out)
{
    int rc;
    double best_t = INFINITY;
    int best = 1;
    std::vector<BatchItem> items, sample;
    EventPair ev;
    hipError_t e = ev.create();
    if (e != hipSuccess) return hip_fail(e, "event create");
    for (int id = 1; id < kNumConfigs; ++id) {
        if (!config_valid(id, prec)) continue;
        int grid = 0;
        if ((rc = batch_grid(prec, kConfigs[id].flat, &grid))) return rc;
        build_items(d, n_dom, kConfigs[id], items);
        const size_t want = (size_t)grid * 3;
        const size_t step = std::max<size_t>(1, items.size() / want);
        sample.clear();
        double cost = 0.0;
        for (size_t i = 0; i < items.size(); i += step) {
            sample.push_back(items[i]);
            cost += item_cost(d[items[i].dom], items[i], kConfigs[id]);
        }
        if ((rc = ensure(dc.bitems, sample.size() * sizeof(BatchItem)))) return rc;
        e = hipMemcpyAsync(dc.bitems.p, sample.data(), sample.size() * sizeof(BatchItem), hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return hip_fail(e, "tuner item upload");
        // warm the kernel once, then time it
        for (int rep = 0; rep < 2; ++rep) {
            if (rep == 1 && (e = hipEventRecord(ev.a, st)) != hipSuccess) return hip_fail(e, "event");
            if ((rc = launch_items(prec, kConfigs[id].flat, ddoms, (const BatchItem *)dc.bitems.p,
                                   (int)sample.size(), nullptr, dc, grid, st)))
                return rc;
            if (rep == 1 && (e = hipEventRecord(ev.b, st)) != hipSuccess) return hip_fail(e, "event");
        }
        if ((e = hipEventSynchronize(ev.b)) != hipSuccess) return hip_fail(e, "tuner sync");
        const double t = ev.seconds() / cost;
        if (t < best_t) {
            best_t = t;
            best = id;
        }
    }
    (void)c_out;
    *best_out = best;
    return FDIRW_OK;
}

int step_batched(const fdirw_domain *d, int n_dom, const fdirw_opts *o, const double *const *c_in,
                 double *const *c_out, fdirw_stats *st, DevCache &dc, hipStream_t stream)
{
    int rc;
    if (o->deterministic) {
        // the persistent launch adds with FP64 atomics; the deterministic
        // form takes the domains in order through the single-domain
        // deterministic step, so each domain's result is bitwise that of a
        // call with n_dom = 1
        for (int i = 0; i < n_dom; ++i)
            if ((rc = step_one(&d[i], o, c_in[i], c_out[i], st ? &st[i] : nullptr, dc, stream, false, nullptr,
                               nullptr)))
                return rc;
        return FDIRW_OK;
    }
    const bool f64 = o->prec == FDIRW_FP64;
    const size_t esz = f64 ? 8 : 4;
    std::vector<int64_t> off(n_dom + 1, 0);
    for (int i = 0; i < n_dom; ++i) off[i + 1] = off[i] + 3 * (int64_t)d[i].nx * d[i].ny * d[i].nz;
    if ((rc = ensure(dc.blam, (size_t)off[n_dom] * esz))) return rc;
    if ((rc = ensure(dc.bsmall, (size_t)n_dom * sizeof(unsigned long long) + 64))) return rc;
    if ((rc = ensure(dc.small, 64))) return rc;
    unsigned long long *used = (unsigned long long *)dc.bsmall.p;
    std::vector<BatchDom> hd(n_dom);
    for (int i = 0; i < n_dom; ++i) {
        Geometry g;
        char *lam = (char *)dc.blam.p + off[i] * esz;
        rc = prepare_geometry(&d[i], stream, dc, f64 ? (double *)lam : nullptr, f64 ? nullptr : (float *)lam, &g);
        if (rc) return rc;
        const int64_t n = (int64_t)d[i].nx * d[i].ny * d[i].nz;
        if (st) {
            if ((rc = field_sum_dev(c_in[i], n, stream, dc, &st[i].mass_in))) return rc;
            if (!std::isfinite(st[i].mass_in)) return fail(FDIRW_E_NONFINITE, "input mass of domain %d is not finite", i);
        }
        hd[i].nx = d[i].nx; hd[i].ny = d[i].ny; hd[i].nz = d[i].nz;
        hd[i].r = d[i].r; hd[i].n_sub = d[i].n_sub;
        hd[i].n = n;
        hd[i].lam = lam;
        hd[i].c_in = c_in[i];
        hd[i].c_out = c_out[i];
        hd[i].n_used = used + i;
    }
    if ((rc = ensure(dc.bdoms, (size_t)n_dom * sizeof(BatchDom)))) return rc;
    hipError_t e = hipMemcpyAsync(dc.bdoms.p, hd.data(), n_dom * sizeof(BatchDom), hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return hip_fail(e, "domain upload");
    int cfg = o->tune;
    if (cfg >= kNumConfigs || (cfg >= 0 && !config_valid(cfg, o->prec)))
        return fail(FDIRW_E_ARG, "batched shape %d is not available for precision %d", cfg, o->prec);
    if (cfg < 0) {
        load_tune_file();
        const std::string key = tune_key(d, n_dom, o->prec);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            cfg = it->second;
        } else {
            if ((rc = autotune(d, n_dom, o->prec, (const BatchDom *)dc.bdoms.p, c_out, dc, stream, &cfg)))
                return rc;
            g_tune_cache[key] = cfg;
            store_tune_file();
        }
    }
    int grid = 0;
    if ((rc = batch_grid(o->prec, kConfigs[cfg].flat, &grid))) return rc;
    std::vector<BatchItem> items;
    build_items(d, n_dom, kConfigs[cfg], items);
    if ((rc = ensure(dc.bitems, items.size() * sizeof(BatchItem)))) return rc;
    if ((rc = ensure(dc.wgk, items.size() * 2 * sizeof(double)))) return rc;
    e = hipMemcpyAsync(dc.bitems.p, items.data(), items.size() * sizeof(BatchItem), hipMemcpyHostToDevice, stream);
    for (int i = 0; i < n_dom && e == hipSuccess; ++i)
        e = launch_fill(c_out[i], (int64_t)d[i].nx * d[i].ny * d[i].nz, 0.0, stream);
    if (e == hipSuccess) e = launch_fill_u32((unsigned *)used, 2 * (int64_t)n_dom, 0u, stream);
    if (e != hipSuccess) return hip_fail(e, "batched setup");
    EventPair ev;
    if (st && (e = ev.create()) != hipSuccess) return hip_fail(e, "event create");
    if (st) (void)hipEventRecord(ev.a, stream);
    if ((rc = launch_items(o->prec, kConfigs[cfg].flat, (const BatchDom *)dc.bdoms.p, (const BatchItem *)dc.bitems.p,
                           (int)items.size(), (double *)dc.wgk.p, dc, grid, stream)))
        return rc;
    if (st) (void)hipEventRecord(ev.b, stream);
    if (st) {
        std::vector<double> km(items.size() * 2);
        std::vector<unsigned long long> hu(n_dom);
        e = hipMemcpyAsync(km.data(), dc.wgk.p, km.size() * sizeof(double), hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(hu.data(), used, n_dom * sizeof(unsigned long long), hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return hip_fail(e, "batched statistics");
        for (int i = 0; i < n_dom; ++i) {
            st[i].kmass_min = INFINITY;
            st[i].kmass_max = -INFINITY;
        }
        for (size_t q = 0; q < items.size(); ++q) {
            fdirw_stats &s = st[items[q].dom];
            s.kmass_min = std::fmin(s.kmass_min, km[2 * q]);
            s.kmass_max = std::fmax(s.kmass_max, km[2 * q + 1]);
        }
        const double ks = ev.seconds();
        for (int i = 0; i < n_dom; ++i) {
            const int64_t n = (int64_t)d[i].nx * d[i].ny * d[i].nz;
            if ((rc = field_sum_dev(c_out[i], n, stream, dc, &st[i].mass_out))) return rc;
            st[i].n_sources = (int64_t)hu[i];
            st[i].audit_l1 = 0.0;
            st[i].fallback_used = 0;
            st[i].bank_used = 0;
            st[i].tuned_config_id = cfg;
            st[i].kernel_seconds = ks;
        }
    }
    return FDIRW_OK;
}

}  // namespace fdirw
