// The C ABI: argument checking, contexts and budgets, lattice handles, per-call
// tile maps, and the rigid EM driver (Sec. 3.1: E-step, M-step, repeat).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstring>

#include <mutex>

#include "fr_internal.h"

namespace fr {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

void clear_error() { g_err[0] = '\0'; }

static thread_local hipStream_t tls_stream = nullptr;

hipStream_t current_stream() { return tls_stream; }
StreamScope::StreamScope(hipStream_t st) : prev(tls_stream) { tls_stream = st; }
StreamScope::~StreamScope() { tls_stream = prev; }

// Sizes are rounded so that freed blocks fit later requests of similar size:
// powers of two up to 1 MiB, multiples of 2 MiB above.
// Size classes of the block cache: powers of two up to 1 MiB, then four
// classes per octave (2^k times 1, 1.25, 1.5, 1.75), so that blocks freed by
// calls of similar size -- a serving engine's lattice builds -- fit later
// ones, and the cache holds few distinct sizes; at most 25% is unused.
static size_t round_alloc(size_t b)
{
    if (b == 0) b = 16;
    if (b <= ((size_t)1 << 20)) {
        size_t r = 512;
        while (r < b) r <<= 1;
        return r;
    }
    size_t oct = (size_t)1 << 20;   // the largest power of two below b
    while (oct * 2 < b) oct <<= 1;
    for (int q = 1; q < 4; ++q) {
        const size_t c = oct + oct / 4 * (size_t)q;
        if (b <= c) return c;
    }
    return oct * 2;
}

static void recycle_event(fr_ctx *ctx, hipEvent_t ev)
{
    if (ev) ctx->spare_events.push_back(ev);
}

// Free cached blocks back to HIP: those whose last use has finished, or with
// wait == true all of them (waiting for their streams first).
static void trim_cache(fr_ctx *ctx, bool wait)
{
    std::vector<fr_ctx::Block> keep;
    for (const fr_ctx::Block &b : ctx->cache) {
        bool idle = b.done == nullptr || hipEventQuery(b.done) == hipSuccess;
        if (!idle && wait) idle = hipEventSynchronize(b.done) == hipSuccess;
        if (!idle) {
            keep.push_back(b);
            continue;
        }
        (void)hipFree(b.p);
        ctx->cached -= b.bytes;
        recycle_event(ctx, b.done);
    }
    (void)hipGetLastError();
    ctx->cache.swap(keep);
}

fr_status dev_alloc(fr_ctx *ctx, void **p, size_t bytes)
{
    *p = nullptr;
    const size_t rb = round_alloc(bytes);
    const hipStream_t st = current_stream();
    // best fit among cached blocks of this size class that this stream may use now
    int best = -1;
    const size_t slack = 0;   // one size class
    for (int i = 0; i < (int)ctx->cache.size(); ++i) {
        const fr_ctx::Block &b = ctx->cache[i];
        if (b.bytes < rb || b.bytes > rb + slack) continue;
        if (best >= 0 && b.bytes >= ctx->cache[best].bytes) continue;
        if (b.done != nullptr && b.stream != st && hipEventQuery(b.done) != hipSuccess) continue;
        best = i;
    }
    (void)hipGetLastError();
    if (best >= 0) {
        const fr_ctx::Block b = ctx->cache[best];
        ctx->cache.erase(ctx->cache.begin() + best);
        ctx->cached -= b.bytes;
        ctx->in_use += b.bytes;
        recycle_event(ctx, b.done);
        *p = b.p;
        return FR_OK;
    }
    if (ctx->budget != 0 && ctx->in_use + ctx->cached + rb > ctx->budget) trim_cache(ctx, false);
    if (ctx->budget != 0 && ctx->in_use + ctx->cached + rb > ctx->budget) trim_cache(ctx, true);
    if (ctx->budget != 0 && ctx->in_use + rb > ctx->budget) {
        set_error("HBM budget exceeded: %zu in use + %zu requested > %zu", ctx->in_use, rb, ctx->budget);
        return FR_EBUDGET;
    }
    hipError_t e = hipMalloc(p, rb);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        trim_cache(ctx, true);
        e = hipMalloc(p, rb);
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        set_error("hipMalloc(%zu) failed: %s", rb, hipGetErrorString(e));
        return FR_ENOMEM;
    }
    ctx->in_use += rb;
    return FR_OK;
}

fr_status stage_h2d(fr_ctx *ctx, void *dst, const void *src, size_t n, hipStream_t st)
{
    if (n == 0) return FR_OK;
    const size_t need = (n + 63) & ~(size_t)63;
    if (ctx->stage_used + need > ctx->stage_cap) {
        // the arena is reused from its start once every copy out of it has run
        for (hipEvent_t ev : ctx->stage_ev) {
            (void)hipEventSynchronize(ev);
            recycle_event(ctx, ev);
        }
        ctx->stage_ev.clear();
        ctx->stage_used = 0;
        if (need > ctx->stage_cap) {
            if (ctx->stage != nullptr) FR_HIP(hipHostFree(ctx->stage));
            ctx->stage = nullptr;
            ctx->stage_cap = 0;
            const size_t cap = std::max<size_t>(need, (size_t)1 << 20);
            FR_HIP(hipHostMalloc(reinterpret_cast<void **>(&ctx->stage), cap, hipHostMallocDefault));
            ctx->stage_cap = cap;
        }
    }
    char *buf = ctx->stage + ctx->stage_used;
    std::memcpy(buf, src, n);
    FR_HIP(hipMemcpyAsync(dst, buf, n, hipMemcpyHostToDevice, st));
    hipEvent_t ev = nullptr;
    if (!ctx->spare_events.empty()) {
        ev = ctx->spare_events.back();
        ctx->spare_events.pop_back();
    } else {
        FR_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    }
    FR_HIP(hipEventRecord(ev, st));
    ctx->stage_ev.push_back(ev);
    ctx->stage_used += need;
    // drop the events of copies that have run (keeps the list short)
    if (ctx->stage_ev.size() > 64) {
        std::vector<hipEvent_t> live;
        for (hipEvent_t e : ctx->stage_ev) {
            if (hipEventQuery(e) == hipSuccess) recycle_event(ctx, e);
            else live.push_back(e);
        }
        (void)hipGetLastError();
        ctx->stage_ev.swap(live);
    }
    return FR_OK;
}

fr_status build_readback(fr_ctx *ctx, size_t n, void **out)
{
    if (ctx->pin_build_n < n) {
        if (ctx->pin_build) FR_HIP(hipHostFree(ctx->pin_build));
        ctx->pin_build = nullptr;
        ctx->pin_build_n = 0;
        const size_t cap = std::max<size_t>(n, 4096);
        FR_HIP(hipHostMalloc(reinterpret_cast<void **>(&ctx->pin_build), cap, hipHostMallocDefault));
        ctx->pin_build_n = cap;
    }
    *out = ctx->pin_build;
    return FR_OK;
}

void dev_free(fr_ctx *ctx, void *p, size_t bytes, hipStream_t st, bool idle)
{
    if (!p) return;
    const size_t rb = round_alloc(bytes);
    hipEvent_t ev = nullptr;
    if (!idle) {
        if (!ctx->spare_events.empty()) {
            ev = ctx->spare_events.back();
            ctx->spare_events.pop_back();
        } else if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
            ev = nullptr;
        }
        if (ev == nullptr || hipEventRecord(ev, st) != hipSuccess) {
            // no event: fall back to waiting for the device
            (void)hipGetLastError();
            (void)hipDeviceSynchronize();
            recycle_event(ctx, ev);
            ev = nullptr;
        }
    }
    ctx->cache.push_back(fr_ctx::Block{p, rb, st, ev});
    ctx->in_use -= std::min(ctx->in_use, rb);
    ctx->cached += rb;
}

void dev_release_cache(fr_ctx *ctx)
{
    (void)hipDeviceSynchronize();
    trim_cache(ctx, true);
    for (hipEvent_t ev : ctx->spare_events) (void)hipEventDestroy(ev);
    ctx->spare_events.clear();
}

fr_status check_cloud(const fr_cloud *c, bool need_normals, const char *what)
{
    if (c == nullptr || c->offsets == nullptr || c->n_sets < 1) {
        set_error("%s: cloud is NULL, has no offsets, or n_sets < 1", what);
        return FR_EINVAL;
    }
    if (c->offsets[0] != 0) {
        set_error("%s: offsets[0] must be 0", what);
        return FR_EINVAL;
    }
    for (int32_t s = 0; s < c->n_sets; ++s)
        if (c->offsets[s + 1] < c->offsets[s]) {
            set_error("%s: offsets must be non-decreasing (set %d)", what, s);
            return FR_EINVAL;
        }
    const int64_t n = c->offsets[c->n_sets];
    if (n > 0 && (c->x == nullptr || c->y == nullptr || c->z == nullptr)) {
        set_error("%s: x/y/z must be non-NULL", what);
        return FR_EINVAL;
    }
    if (need_normals && n > 0 && (c->nx == nullptr || c->ny == nullptr || c->nz == nullptr)) {
        set_error("%s: normals are required (feat 6 or point-to-plane)", what);
        return FR_EINVAL;
    }
    if (n >= (int64_t)1 << 31) {
        set_error("%s: %lld points exceed 2^31", what, (long long)n);
        return FR_EINVAL;
    }
    return FR_OK;
}

fr_status plan_layout(const fr_cloud *cloud, const fr_xform *xf, int32_t tile, const double *c_seg_host, Plan &plan,
                      std::vector<char> &image)
{
    plan.tile = tile;
    plan.n_sets = cloud->n_sets;
    const bool seg = xf != nullptr && xf->kind == FR_XF_SEGMENTED;
    if (seg) {
        plan.n_seg = xf->n_seg;
        plan.seg_off.assign(xf->seg_offsets, xf->seg_offsets + xf->n_seg + 1);
        plan.seg_set.assign(xf->n_seg, 0);
        int32_t set = 0;
        for (int32_t s = 0; s < xf->n_seg; ++s) {
            const int64_t a = plan.seg_off[s], b = plan.seg_off[s + 1];
            while (set < cloud->n_sets && cloud->offsets[set + 1] <= a && !(a == b && cloud->offsets[set + 1] == a))
                ++set;
            if (set >= cloud->n_sets || a < cloud->offsets[set] || b > cloud->offsets[set + 1]) {
                set_error("fr_xform: segment %d [%lld, %lld) does not lie inside one set", s, (long long)a,
                          (long long)b);
                return FR_EINVAL;
            }
            plan.seg_set[s] = set;
        }
    } else {
        plan.n_seg = cloud->n_sets;
        plan.seg_off.assign(cloud->offsets, cloud->offsets + cloud->n_sets + 1);
        plan.seg_set.resize(cloud->n_sets);
        for (int32_t s = 0; s < cloud->n_sets; ++s) plan.seg_set[s] = s;
    }
    plan.seg_tile.assign(plan.n_seg + 1, 0);
    for (int32_t s = 0; s < plan.n_seg; ++s)
        plan.seg_tile[s + 1] = plan.seg_tile[s] + (int32_t)((plan.seg_off[s + 1] - plan.seg_off[s] + tile - 1) / tile);
    plan.n_tiles = plan.seg_tile[plan.n_seg];
    // XCD-contiguous tile order pays off once the launch is several waves of the chip deep
    int32_t chunk = 0, grid = plan.n_tiles;
    if (plan.n_tiles >= 8 * 64) {
        chunk = (plan.n_tiles + 7) / 8;
        grid = chunk * 8;
    }
    plan.grid = grid;
    plan.tm.n_seg = plan.n_seg;
    plan.tm.n_tiles = plan.n_tiles;
    plan.tm.tile = tile;
    plan.tm.xcd_chunk = chunk;
    std::vector<float> cseg(plan.n_seg, 0.0f);
    if (c_seg_host)
        for (int32_t s = 0; s < plan.n_seg; ++s) cseg[s] = (float)c_seg_host[plan.seg_set[s]];
    const size_t b_off = sizeof(int64_t) * (plan.n_seg + 1);
    const size_t b_tile = sizeof(int32_t) * (plan.n_seg + 1);
    const size_t b_set = sizeof(int32_t) * plan.n_seg;
    const size_t b_c = sizeof(float) * plan.n_seg;
    image.assign(b_off + b_tile + b_set + b_c, 0);
    std::memcpy(image.data(), plan.seg_off.data(), b_off);
    std::memcpy(image.data() + b_off, plan.seg_tile.data(), b_tile);
    std::memcpy(image.data() + b_off + b_tile, plan.seg_set.data(), b_set);
    std::memcpy(image.data() + b_off + b_tile + b_set, cseg.data(), b_c);
    return FR_OK;
}

void plan_bind(Plan &plan, const void *dev_image)
{
    const size_t b_off = sizeof(int64_t) * (plan.n_seg + 1);
    const size_t b_tile = sizeof(int32_t) * (plan.n_seg + 1);
    const size_t b_set = sizeof(int32_t) * plan.n_seg;
    const char *p = static_cast<const char *>(dev_image);
    plan.tm.seg_off = reinterpret_cast<const int64_t *>(p);
    plan.tm.seg_end = plan.tm.seg_off + 1;
    plan.tm.seg_tile = reinterpret_cast<const int32_t *>(p + b_off);
    plan.tm.seg_set = reinterpret_cast<const int32_t *>(p + b_off + b_tile);
    plan.seg_c = reinterpret_cast<const float *>(p + b_off + b_tile + b_set);
}

fr_status make_plan(fr_ctx *ctx, const fr_cloud *cloud, const fr_xform *xf, int32_t tile, const double *c_seg_host,
                    hipStream_t st, Plan &plan)
{
    plan.ctx = ctx;
    plan.slice = ctx->slice_mode;
    std::vector<char> host;
    FR_TRY(plan_layout(cloud, xf, tile, c_seg_host, plan, host));
    FR_TRY(plan.meta.alloc(ctx, host.size()));
    FR_HIP(hipMemcpyAsync(plan.meta.p, host.data(), host.size(), hipMemcpyHostToDevice, st));
    FR_HIP(hipStreamSynchronize(st));
    plan_bind(plan, plan.meta.p);
    return FR_OK;
}

bool ctx_ok(const fr_ctx *c) { return c != nullptr && c->magic == kCtxMagic; }
static bool lat_ok(const fr_lattice *l) { return l != nullptr && l->magic == kLatMagic; }

// Integral over feature space of the lattice kernel of one observation,
// K(x, y) = sum_v b_v(x) b_v(y) (splat and slice of Sec. 4.2), for d feature
// dimensions of widths sig[0..d-1].  The vertex hats sum to one everywhere and
// are congruent, so each integrates to the volume per vertex, and so does K
// over x: the vertices form the scaled lattice (d+1) A*_d, (d+1)^(d - 1/2) of
// volume per point, reached from the normalised features by a uniform stretch
// of sqrt(2/3) (d+1); hence (3/2)^(d/2) / sqrt(d+1) prod sig_i.  The blur of
// the uncustomised filter keeps the vertex mass and scales the output by
// 1 / (1 + 2^-d).
static double kernel_mass(int d, const double *sig, bool blurred)
{
    double h = std::pow(1.5, 0.5 * d) / std::sqrt(d + 1.0);
    for (int i = 0; i < d; ++i) h *= sig[i];
    return blurred ? h / (1.0 + std::ldexp(1.0, -d)) : h;
}

// Outlier constant c of Eq. 7 in the units of the lattice sums: Eq. 4 sets the
// uniform component beside Gaussian PDFs of unit mass, and c = w/(1-w) N/M is
// taken against their sum; M0 sums a kernel of mass kernel_mass per
// observation instead, so the weight M0 / (M0 + c) keeps its meaning with c
// scaled by that mass (every feature dimension: position and, for d = 6,
// normal widths).
double outlier_constant(const fr_lattice_params &lp, double w, double c_override, double Ms, double Ns, bool blurred)
{
    if (c_override >= 0.0) return c_override;
    if (!(Ms > 0) || !(w > 0.0)) return 0.0;
    double sig[6] = {lp.sigma[0], lp.sigma[1], lp.sigma[2], lp.sigma_n, lp.sigma_n, lp.sigma_n};
    return w / (1.0 - w) * (Ns / Ms) * kernel_mass(lp.feat == 6 ? 6 : 3, sig, blurred);
}

fr_status check_lattice_params(const fr_lattice_params *p)
{
    if (p == nullptr) {
        set_error("lattice params are NULL");
        return FR_EINVAL;
    }
    if (p->feat != 3 && p->feat != 6) {
        set_error("feat must be 3 or 6 (got %d)", p->feat);
        return FR_EINVAL;
    }
    if (p->values != 4 && p->values != 5 && p->values != 7 && p->values != 8) {
        set_error("values must be FR_VAL_PT2PT, FR_VAL_PT2PT_M2, FR_VAL_PT2PL or FR_VAL_PT2PL_M2");
        return FR_EINVAL;
    }
    for (int i = 0; i < 3; ++i)
        if (!(p->sigma[i] > 0.0) || !std::isfinite(p->sigma[i])) {
            set_error("sigma[%d] must be finite and > 0", i);
            return FR_EINVAL;
        }
    if (p->feat == 6 && (!(p->sigma_n > 0.0) || !std::isfinite(p->sigma_n))) {
        set_error("sigma_n must be finite and > 0 for feat 6");
        return FR_EINVAL;
    }
    if (p->splat != FR_SPLAT_SORTED && p->splat != FR_SPLAT_ATOMIC) {
        set_error("splat must be FR_SPLAT_SORTED or FR_SPLAT_ATOMIC");
        return FR_EINVAL;
    }
    if (p->reserved != 0) {
        set_error("reserved must be 0");
        return FR_EINVAL;
    }
    return FR_OK;
}

void free_lattice(fr_lattice *lat, hipStream_t st, bool idle)
{
    if (lat->tab) dev_free(lat->ctx, lat->tab, lat->tab_bytes, st, idle);
    if (lat->sets_d) dev_free(lat->ctx, lat->sets_d, lat->sets_h.size() * sizeof(SetTable), st, idle);
    if (lat->vkey) dev_free(lat->ctx, lat->vkey, lat->vert_bytes, st, idle);
    if (lat->err_d) dev_free(lat->ctx, lat->err_d, sizeof(int32_t), st, idle);
    if (lat->kfeat_d) dev_free(lat->ctx, lat->kfeat_d, lat->kfeat.size() * sizeof(float), st, idle);
    lat->kfeat_d = nullptr;
    lat->tab = nullptr;
    lat->sets_d = nullptr;
    lat->vkey = nullptr;
    lat->err_d = nullptr;
}

// Lattice scale per feature dimension: sqrt(2/3) (d+1) / (sigma_i sqrt((i+1)(i+2))),
// rounded once to binary32 (the feature normalisation of Sec. 4.1 folded into
// the permutohedral lattice scale).
void scale_factors(const fr_lattice_params *p, float *k)
{
    const int d = p->feat;
    for (int i = 0; i < 8; ++i) k[i] = 0.0f;
    for (int i = 0; i < d; ++i) {
        const double sig = (i < 3) ? p->sigma[i] : p->sigma_n;
        k[i] = (float)(std::sqrt(2.0 / 3.0) * (double)(d + 1) / (sig * std::sqrt((double)((i + 1) * (i + 2)))));
    }
}

fr_status lattice_build_impl(fr_ctx *ctx, const fr_cloud *obs, const fr_lattice_params *params, hipStream_t st,
                             fr_lattice **out, const double *sigma_set, const fr_cloud *joint_model,
                             const float *joint_mats, bool wait_end)
{
    fr_lattice *lat = new (std::nothrow) fr_lattice();
    if (!lat) {
        set_error("out of host memory");
        return FR_ENOMEM;
    }
    lat->ctx = ctx;
    lat->d = params->feat;
    lat->V = params->values;
    lat->KW = (params->feat + 2) / 3;
    lat->n_sets = obs->n_sets;
    lat->splat = params->splat;
    lat->n_points_total = cloud_points(obs) + (joint_model ? cloud_points(joint_model) : 0);
    scale_factors(params, lat->k);
    lat->kset.resize((size_t)8 * obs->n_sets);
    for (int32_t q = 0; q < obs->n_sets; ++q) {
        if (sigma_set) {
            fr_lattice_params ps = *params;
            ps.sigma[0] = ps.sigma[1] = ps.sigma[2] = sigma_set[q];
            scale_factors(&ps, lat->kset.data() + 8 * (size_t)q);
        } else {
            std::memcpy(lat->kset.data() + 8 * (size_t)q, lat->k, sizeof(lat->k));
        }
    }
    fr_status s = dev_alloc(ctx, reinterpret_cast<void **>(&lat->err_d), sizeof(int32_t));
    if (s == FR_OK)
        s = joint_model ? build_joint_lattice(ctx, obs, joint_model, joint_mats, params, st, lat)
                        : build_lattice(ctx, obs, params, st, lat, nullptr, wait_end);
    if (s != FR_OK) {
        free_lattice(lat, st, false);
        lat->magic = kDeadMagic;
        delete lat;
        return s;
    }
    *out = lat;
    return FR_OK;
}

// Descriptor lattice of Eq. 8: d = dim, values [1, y], one isotropic width
// sigma_f for every descriptor dimension (the scale factors of scale_factors()
// with sigma_i = sigma_f).
static fr_status feature_lattice_impl(fr_ctx *ctx, const fr_cloud *obs, const float *obs_feat, int32_t dim,
                                      double sigma_f, int32_t splat, hipStream_t st, fr_lattice **out)
{
    fr_lattice *lat = new (std::nothrow) fr_lattice();
    if (!lat) {
        set_error("out of host memory");
        return FR_ENOMEM;
    }
    lat->ctx = ctx;
    lat->d = dim;
    lat->V = FR_VAL_PT2PT;
    lat->KW = (dim + 2) / 3;
    lat->n_sets = obs->n_sets;
    lat->splat = splat;
    lat->n_points_total = cloud_points(obs);
    lat->kfeat.resize(dim);
    for (int i = 0; i < dim; ++i)
        lat->kfeat[i] = (float)(std::sqrt(2.0 / 3.0) * (double)(dim + 1) /
                                (sigma_f * std::sqrt((double)((i + 1) * (i + 2)))));
    for (int i = 0; i < 8; ++i) lat->k[i] = lat->kfeat[i];
    lat->kset.resize((size_t)8 * obs->n_sets);
    for (int32_t q = 0; q < obs->n_sets; ++q) std::memcpy(lat->kset.data() + 8 * (size_t)q, lat->k, sizeof(lat->k));
    fr_status s = dev_alloc(ctx, reinterpret_cast<void **>(&lat->err_d), sizeof(int32_t));
    if (s == FR_OK) s = dev_alloc(ctx, reinterpret_cast<void **>(&lat->kfeat_d), dim * sizeof(float));
    if (s == FR_OK) {
        const hipError_t e = hipMemcpyAsync(lat->kfeat_d, lat->kfeat.data(), dim * sizeof(float),
                                            hipMemcpyHostToDevice, st);
        if (e != hipSuccess) {
            set_error("hipMemcpyAsync: %s", hipGetErrorString(e));
            s = FR_EDEVICE;
        }
    }
    if (s == FR_OK) s = build_feature_lattice(ctx, obs, obs_feat, st, lat);
    if (s != FR_OK) {
        free_lattice(lat, st, false);
        lat->magic = kDeadMagic;
        delete lat;
        return s;
    }
    *out = lat;
    return FR_OK;
}

// c of Eq. 7 for a kernel over dim descriptor dimensions of width sigma_f:
// the rule of outlier_constant with the descriptor lattice's kernel mass.
static double feature_outlier_constant(double w, double c_override, double Ms, double Ns, double sigma_f, int dim)
{
    if (c_override >= 0.0) return c_override;
    if (!(Ms > 0) || !(w > 0.0)) return 0.0;
    double sig[64];
    for (int i = 0; i < dim; ++i) sig[i] = sigma_f;
    return w / (1.0 - w) * (Ns / Ms) * kernel_mass(dim, sig, false);
}

static fr_status check_features(const float *feat, int32_t dim, const char *what)
{
    if (feat == nullptr || !feature_dim_supported(dim)) {
        set_error("%s: descriptors must be non-NULL with dimension 8, 16 or 32 (got %d)", what, dim);
        return FR_EINVAL;
    }
    if ((reinterpret_cast<uintptr_t>(feat) & 15u) != 0) {
        set_error("%s: descriptor rows must be 16-byte aligned", what);
        return FR_EINVAL;
    }
    return FR_OK;
}

static fr_status check_xform(const fr_xform *xf, const fr_cloud *cloud, const char *what)
{
    if (xf == nullptr) return FR_OK;
    if (xf->kind == FR_XF_NONE) return FR_OK;
    if (xf->kind != FR_XF_RIGID && xf->kind != FR_XF_SEGMENTED) {
        set_error("%s: unknown xform kind %d", what, xf->kind);
        return FR_EINVAL;
    }
    if (xf->mats == nullptr) {
        set_error("%s: xform mats is NULL", what);
        return FR_EINVAL;
    }
    if (xf->kind == FR_XF_RIGID && xf->n_seg != 0 && xf->n_seg != cloud->n_sets) {
        set_error("%s: rigid xform needs one matrix per set", what);
        return FR_EINVAL;
    }
    if (xf->kind == FR_XF_SEGMENTED) {
        if (xf->seg_offsets == nullptr || xf->n_seg < 1) {
            set_error("%s: segmented xform needs seg_offsets and n_seg >= 1", what);
            return FR_EINVAL;
        }
        if (xf->seg_offsets[0] != 0 || xf->seg_offsets[xf->n_seg] != cloud_points(cloud)) {
            set_error("%s: seg_offsets must partition [0, M)", what);
            return FR_EINVAL;
        }
        for (int32_t s = 0; s < xf->n_seg; ++s)
            if (xf->seg_offsets[s + 1] < xf->seg_offsets[s]) {
                set_error("%s: seg_offsets must be non-decreasing", what);
                return FR_EINVAL;
            }
    }
    return FR_OK;
}

}  // namespace fr

using namespace fr;

// ===========================================================================
// extern "C"
// ===========================================================================
extern "C" {

int32_t fr_version(void) { return 100; }

const char *fr_last_error(void) { return g_err; }

fr_status fr_ctx_create(int32_t device, size_t hbm_budget_bytes, fr_ctx **out)
{
    clear_error();
    if (out == nullptr) {
        set_error("fr_ctx_create: out is NULL");
        return FR_EINVAL;
    }
    *out = nullptr;
    int n = 0;
    FR_HIP(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) {
        set_error("fr_ctx_create: device %d not in [0, %d)", device, n);
        return FR_EINVAL;
    }
    FR_HIP(hipSetDevice(device));
    fr_ctx *c = new (std::nothrow) fr_ctx();
    if (!c) {
        set_error("out of host memory");
        return FR_ENOMEM;
    }
    c->device = device;
    c->budget = hbm_budget_bytes;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
        c->cu_count = cus;
    *out = c;
    return FR_OK;
}

fr_status fr_ctx_destroy(fr_ctx *ctx)
{
    clear_error();
    if (!ctx_ok(ctx)) {
        set_error("fr_ctx_destroy: invalid or destroyed context");
        return FR_EINVAL;
    }
    (void)hipSetDevice(ctx->device);
    dev_release_cache(ctx);
    if (ctx->graph_stream) (void)hipStreamDestroy(ctx->graph_stream);
    ctx->graph_stream = nullptr;
    if (ctx->pin_flags) (void)hipHostFree(ctx->pin_flags);
    ctx->pin_flags = nullptr;
    for (hipEvent_t ev : ctx->stage_ev) (void)hipEventDestroy(ev);
    ctx->stage_ev.clear();
    if (ctx->stage) (void)hipHostFree(ctx->stage);
    ctx->stage = nullptr;
    if (ctx->pin_build) (void)hipHostFree(ctx->pin_build);
    ctx->pin_build = nullptr;
    ctx->magic = kDeadMagic;
    delete ctx;
    return FR_OK;
}

fr_status fr_ctx_usage(const fr_ctx *ctx, size_t *bytes)
{
    clear_error();
    if (!ctx_ok(ctx) || bytes == nullptr) {
        set_error("fr_ctx_usage: invalid argument");
        return FR_EINVAL;
    }
    *bytes = ctx->in_use;
    return FR_OK;
}

fr_status fr_lattice_records(const fr_lattice *lat, int64_t *incidences, int64_t *partial_records)
{
    clear_error();
    if (!lat_ok(lat) || incidences == nullptr || partial_records == nullptr) {
        set_error("fr_lattice_records: invalid argument");
        return FR_EINVAL;
    }
    *incidences = lat->n_points_total * (lat->d + 1);
    *partial_records = lat->n_partials;
    return FR_OK;
}

fr_status fr_lattice_build_times(const fr_lattice *lat, double *stage_ms_h)
{
    clear_error();
    if (!lat_ok(lat) || stage_ms_h == nullptr) {
        set_error("fr_lattice_build_times: invalid argument");
        return FR_EINVAL;
    }
    for (int i = 0; i < 4; ++i) stage_ms_h[i] = (double)lat->stage_ms[i];
    return FR_OK;
}

fr_status fr_ctx_set_tuning(fr_ctx *ctx, const fr_tuning *t)
{
    clear_error();
    if (!ctx_ok(ctx) || t == nullptr) {
        set_error("fr_ctx_set_tuning: invalid argument");
        return FR_EINVAL;
    }
    if (t->slice != FR_SLICE_AUTO && t->slice != FR_SLICE_PLAIN && t->slice != FR_SLICE_SHARED) {
        set_error("fr_ctx_set_tuning: slice %d is not an FR_SLICE_* value", t->slice);
        return FR_EINVAL;
    }
    ctx->slice_mode = t->slice;
    return FR_OK;
}

fr_status fr_ctx_tuning_table(const fr_ctx *ctx, fr_tuning_entry *out_h, int32_t cap, int32_t *n)
{
    clear_error();
    if (!ctx_ok(ctx) || n == nullptr || cap < 0 || (cap > 0 && out_h == nullptr)) {
        set_error("fr_ctx_tuning_table: invalid argument");
        return FR_EINVAL;
    }
    *n = (int32_t)ctx->tuned.size();
    for (int32_t i = 0; i < cap && i < *n; ++i) out_h[i] = ctx->tuned[i];
    return FR_OK;
}

fr_status fr_lattice_build(fr_ctx *ctx, const fr_cloud *obs, const fr_lattice_params *params, void *stream,
                           fr_lattice **out)
{
    clear_error();
    if (!ctx_ok(ctx) || out == nullptr) {
        set_error("fr_lattice_build: invalid context or out pointer");
        return FR_EINVAL;
    }
    *out = nullptr;
    FR_TRY(check_lattice_params(params));
    FR_TRY(check_cloud(obs, params->feat == 6 || params->values >= 7, "fr_lattice_build"));
    FR_HIP(hipSetDevice(ctx->device));
    StreamScope scope(static_cast<hipStream_t>(stream));
    return lattice_build_impl(ctx, obs, params, static_cast<hipStream_t>(stream), out);
}

// Per-set scale factors of `p` with set s's position scale sigma_set_h[s] (or p's).
static void set_scale_factors(const fr_lattice_params &p, int32_t n_sets, const double *sigma_set_h, float *k)
{
    for (int32_t s = 0; s < n_sets; ++s) {
        fr_lattice_params ps = p;
        if (sigma_set_h != nullptr) ps.sigma[0] = ps.sigma[1] = ps.sigma[2] = sigma_set_h[s];
        scale_factors(&ps, k + 8 * (size_t)s);
    }
}

static fr_status check_set_sigmas(const double *sigma_set_h, int32_t n_sets, const char *what)
{
    for (int32_t s = 0; sigma_set_h != nullptr && s < n_sets; ++s)
        if (!(sigma_set_h[s] > 0.0) || !std::isfinite(sigma_set_h[s])) {
            set_error("%s: sigma of set %d must be finite and > 0", what, s);
            return FR_EINVAL;
        }
    return FR_OK;
}

fr_status fr_lattice_build_inplace(fr_ctx *ctx, const fr_cloud *obs, const fr_lattice_params *params,
                                   const double *sigma_set_h, void *stream, fr_lattice **out)
{
    clear_error();
    if (!ctx_ok(ctx) || out == nullptr) {
        set_error("fr_lattice_build_inplace: invalid context or out pointer");
        return FR_EINVAL;
    }
    *out = nullptr;
    FR_TRY(check_lattice_params(params));
    FR_TRY(check_cloud(obs, params->feat == 6 || params->values >= 7, "fr_lattice_build_inplace"));
    FR_TRY(check_set_sigmas(sigma_set_h, obs->n_sets, "fr_lattice_build_inplace"));
    FR_HIP(hipSetDevice(ctx->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    StreamScope scope(st);
    ResidentBuild *rb = nullptr;
    FR_TRY(resident_create(ctx, obs, params, st, &rb));
    fr_lattice *lat = resident_lattice(rb);
    scale_factors(params, lat->k);
    lat->kset.assign(8 * (size_t)obs->n_sets, 0.0f);
    set_scale_factors(*params, obs->n_sets, sigma_set_h, lat->kset.data());
    fr_status s = resident_build_host(rb, lat->kset.data(), st);
    if (s == FR_OK) s = fr_sync_status(lat);
    if (s != FR_OK) {
        const std::string msg = fr_last_error();
        (void)hipStreamSynchronize(st);
        resident_destroy(rb, st, true);
        set_error("%s", msg.c_str());
        return s;
    }
    *out = lat;
    return FR_OK;
}

fr_status fr_lattice_rebuild(fr_lattice *lat, const double *sigma_set_h, void *stream)
{
    clear_error();
    if (!lat_ok(lat) || lat->resident == nullptr || sigma_set_h == nullptr) {
        set_error("fr_lattice_rebuild: a lattice from fr_lattice_build_inplace and per-set sigmas are required");
        return FR_EINVAL;
    }
    FR_TRY(check_set_sigmas(sigma_set_h, lat->n_sets, "fr_lattice_rebuild"));
    FR_HIP(hipSetDevice(lat->ctx->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    StreamScope scope(st);
    set_scale_factors(lat->params, lat->n_sets, sigma_set_h, lat->kset.data());
    return resident_build_host(lat->resident, lat->kset.data(), st);
}

fr_status fr_lattice_build_joint(fr_ctx *ctx, const fr_cloud *obs, const fr_cloud *model_ref, const fr_xform *xf,
                                 const fr_lattice_params *params, void *stream, fr_lattice **out)
{
    clear_error();
    if (!ctx_ok(ctx) || out == nullptr) {
        set_error("fr_lattice_build_joint: invalid context or out pointer");
        return FR_EINVAL;
    }
    *out = nullptr;
    FR_TRY(check_lattice_params(params));
    if (params->values != FR_VAL_PT2PT && params->values != FR_VAL_PT2PL) {
        set_error("fr_lattice_build_joint: values must be FR_VAL_PT2PT or FR_VAL_PT2PL");
        return FR_EINVAL;
    }
    FR_TRY(check_cloud(obs, params->feat == 6 || params->values >= 7, "fr_lattice_build_joint(obs)"));
    FR_TRY(check_cloud(model_ref, params->feat == 6, "fr_lattice_build_joint(model)"));
    if (model_ref->n_sets != obs->n_sets) {
        set_error("fr_lattice_build_joint: model has %d sets, observation %d", model_ref->n_sets, obs->n_sets);
        return FR_EINVAL;
    }
    if (xf != nullptr && xf->kind != FR_XF_NONE &&
        (xf->kind != FR_XF_RIGID || xf->mats == nullptr || (xf->n_seg != 0 && xf->n_seg != obs->n_sets))) {
        set_error("fr_lattice_build_joint: xform must be FR_XF_NONE or FR_XF_RIGID with one matrix per set");
        return FR_EINVAL;
    }
    FR_HIP(hipSetDevice(ctx->device));
    StreamScope scope(static_cast<hipStream_t>(stream));
    const float *mats = (xf != nullptr && xf->kind == FR_XF_RIGID) ? xf->mats : nullptr;
    return lattice_build_impl(ctx, obs, params, static_cast<hipStream_t>(stream), out, nullptr, model_ref, mats);
}

fr_status fr_lattice_build_features(fr_ctx *ctx, const fr_cloud *obs, const float *obs_feat, int32_t dim,
                                    double sigma_f, int32_t splat, void *stream, fr_lattice **out)
{
    clear_error();
    if (!ctx_ok(ctx) || out == nullptr) {
        set_error("fr_lattice_build_features: invalid context or out pointer");
        return FR_EINVAL;
    }
    *out = nullptr;
    FR_TRY(check_features(obs_feat, dim, "fr_lattice_build_features"));
    if (!(sigma_f > 0.0) || !std::isfinite(sigma_f) || (splat != FR_SPLAT_SORTED && splat != FR_SPLAT_ATOMIC)) {
        set_error("fr_lattice_build_features: sigma_f must be finite and > 0, splat sorted or atomic");
        return FR_EINVAL;
    }
    FR_TRY(check_cloud(obs, false, "fr_lattice_build_features"));
    FR_HIP(hipSetDevice(ctx->device));
    StreamScope scope(static_cast<hipStream_t>(stream));
    return feature_lattice_impl(ctx, obs, obs_feat, dim, sigma_f, splat, static_cast<hipStream_t>(stream), out);
}

fr_status fr_estep_features(const fr_lattice *lat, const fr_cloud *model_ref, const float *model_feat, float *m0,
                            float *m1, void *stream)
{
    clear_error();
    if (!lat_ok(lat) || lat->kfeat_d == nullptr) {
        set_error("fr_estep_features: invalid lattice (build it with fr_lattice_build_features)");
        return FR_EINVAL;
    }
    FR_TRY(check_features(model_feat, lat->d, "fr_estep_features"));
    FR_TRY(check_cloud(model_ref, false, "fr_estep_features"));
    if (model_ref->n_sets != lat->n_sets) {
        set_error("fr_estep_features: model has %d sets, lattice has %d", model_ref->n_sets, lat->n_sets);
        return FR_EINVAL;
    }
    const int64_t M = cloud_points(model_ref);
    if (M > 0 && (m0 == nullptr || m1 == nullptr)) {
        set_error("fr_estep_features: m0/m1 must be non-NULL");
        return FR_EINVAL;
    }
    if (M == 0) return FR_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    StreamScope scope(st);
    FR_HIP(hipSetDevice(lat->ctx->device));
    Plan plan;
    FR_TRY(make_plan(lat->ctx, model_ref, nullptr, kEstepTile, nullptr, st, plan));
    return launch_estep_features(lat, model_ref, plan, model_feat, m0, m1, st);
}

fr_status fr_lattice_blur(fr_lattice *lat, void *stream)
{
    clear_error();
    if (!lat_ok(lat) || lat->resident != nullptr) {
        set_error("fr_lattice_blur: invalid lattice (a lattice rebuilt in place cannot be blurred)");
        return FR_EINVAL;
    }
    FR_HIP(hipSetDevice(lat->ctx->device));
    StreamScope scope(static_cast<hipStream_t>(stream));
    return blur_lattice(lat, static_cast<hipStream_t>(stream));
}

fr_status fr_lattice_destroy(fr_lattice *lat)
{
    clear_error();
    if (!lat_ok(lat)) {
        set_error("fr_lattice_destroy: invalid or destroyed lattice");
        return FR_EINVAL;
    }
    (void)hipSetDevice(lat->ctx->device);
    // kernels queued on any stream may still read the lattice
    (void)hipDeviceSynchronize();
    if (lat->resident != nullptr) {
        resident_destroy(lat->resident, nullptr, true);
        return FR_OK;
    }
    free_lattice(lat, nullptr, true);
    lat->magic = kDeadMagic;
    delete lat;
    return FR_OK;
}

fr_status fr_sync_status(const fr_lattice *lat)
{
    clear_error();
    if (!lat_ok(lat)) {
        set_error("fr_sync_status: invalid lattice");
        return FR_EINVAL;
    }
    FR_HIP(hipSetDevice(lat->ctx->device));
    FR_HIP(hipDeviceSynchronize());
    int32_t e = 0;
    FR_HIP(hipMemcpy(&e, lat->err_d, sizeof(int32_t), hipMemcpyDeviceToHost));
    if (e != 0) {
        FR_HIP(hipMemset(lat->err_d, 0, sizeof(int32_t)));
        set_error("a lattice coordinate left [-2^20, 2^20) in an earlier call");
        return FR_ERANGE;
    }
    if (lat->resident != nullptr) {
        uint32_t f[2] = {0u, 0u};
        FR_HIP(hipMemcpy(f, resident_fail_words(lat->resident), sizeof(f), hipMemcpyDeviceToHost));
        if (f[0] != 0u || f[1] != 0u) {
            set_error("the last in-place rebuild overflowed its %s table; the lattice is not valid",
                      f[0] != 0u ? "provisional" : "cuckoo");
            return FR_EDEVICE;
        }
    }
    return FR_OK;
}

fr_status fr_lattice_stats(const fr_lattice *lat, int32_t set, int64_t *n_vertices, int64_t *capacity,
                           int64_t *device_bytes)
{
    clear_error();
    if (!lat_ok(lat) || set < 0 || set >= lat->n_sets || lat->resident != nullptr) {
        set_error("fr_lattice_stats: invalid lattice or set (not available on a lattice rebuilt in place)");
        return FR_EINVAL;
    }
    FR_TRY(fr_sync_status(lat));
    const SetTable &st = lat->sets_h[set];
    const int KW = lat->KW;
    const int VP = lat->V <= 4 ? 4 : 8;
    if (n_vertices) *n_vertices = st.n_vertices;
    if (capacity) *capacity = (int64_t)st.cap;
    if (device_bytes)
        *device_bytes = (int64_t)st.cap * slot_bytes(KW, VP) +
                        (int64_t)st.n_vertices * (KW * 8 + 4 + 4 * lat->V);
    return FR_OK;
}

fr_status fr_lattice_export(const fr_lattice *lat, int32_t set, int32_t *keys_h, int32_t *occ_h, float *vals_h)
{
    clear_error();
    if (!lat_ok(lat) || set < 0 || set >= lat->n_sets || lat->resident != nullptr) {
        set_error("fr_lattice_export: invalid lattice or set (not available on a lattice rebuilt in place)");
        return FR_EINVAL;
    }
    FR_TRY(fr_sync_status(lat));
    const int64_t v0 = lat->vbase[set], nv = lat->vbase[set + 1] - v0, NV = lat->n_vertices_total;
    if (nv == 0) return FR_OK;
    if (!keys_h || !occ_h || !vals_h) {
        set_error("fr_lattice_export: NULL output");
        return FR_EINVAL;
    }
    const int KW = lat->KW, V = lat->V, d = lat->d;
    std::vector<uint64_t> key((size_t)KW * nv);
    std::vector<uint32_t> occ(nv);
    std::vector<float> val((size_t)V * nv);
    for (int w = 0; w < KW; ++w)
        FR_HIP(hipMemcpy(key.data() + (size_t)w * nv, lat->vkey + (size_t)w * NV + v0, nv * sizeof(uint64_t),
                         hipMemcpyDeviceToHost));
    FR_HIP(hipMemcpy(occ.data(), lat->vocc + v0, nv * sizeof(uint32_t), hipMemcpyDeviceToHost));
    for (int c = 0; c < V; ++c)
        FR_HIP(hipMemcpy(val.data() + (size_t)c * nv, lat->vval + (size_t)c * NV + v0, nv * sizeof(float),
                         hipMemcpyDeviceToHost));
    // packed keys order lexicographically by coordinates (coordinate 0 in the top bits of word 0)
    std::vector<int64_t> order(nv);
    for (int64_t i = 0; i < nv; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
        for (int w = 0; w < KW; ++w) {
            const uint64_t ka = key[(size_t)w * nv + a], kb = key[(size_t)w * nv + b];
            if (ka != kb) return ka < kb;
        }
        return false;
    });
    for (int64_t o = 0; o < nv; ++o) {
        const int64_t i = order[o];
        uint64_t words[12] = {0};
        for (int w = 0; w < KW; ++w) words[w] = key[(size_t)w * nv + i];
        for (int j = 0; j < d; ++j) keys_h[o * d + j] = unpack_coord(words, j);
        occ_h[o] = (int32_t)occ[i];
        for (int c = 0; c < V; ++c) vals_h[o * V + c] = val[(size_t)c * nv + i];
    }
    return FR_OK;
}

static fr_status estep_impl(const fr_lattice *lat, const fr_cloud *model_ref, const fr_xform *xf, float *m0,
                            float *m1, float *nsum, float *m2, void *stream, const char *what)
{
    clear_error();
    if (!lat_ok(lat)) {
        set_error("%s: invalid lattice", what);
        return FR_EINVAL;
    }
    FR_TRY(check_cloud(model_ref, lat->d == 6, what));
    if (model_ref->n_sets != lat->n_sets) {
        set_error("%s: model has %d sets, lattice has %d", what, model_ref->n_sets, lat->n_sets);
        return FR_EINVAL;
    }
    FR_TRY(check_xform(xf, model_ref, what));
    const int64_t M = cloud_points(model_ref);
    if (M > 0 && (m0 == nullptr || m1 == nullptr)) {
        set_error("%s: m0/m1 must be non-NULL", what);
        return FR_EINVAL;
    }
    if (M == 0) return FR_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    StreamScope scope(st);
    FR_HIP(hipSetDevice(lat->ctx->device));
    Plan plan;
    FR_TRY(make_plan(lat->ctx, model_ref, xf, kEstepTile, nullptr, st, plan));
    const int kind = xf ? xf->kind : FR_XF_NONE;
    // the plan's device table goes back to the block cache ordered after the launch
    return launch_estep(lat, model_ref, plan, kind, kind == FR_XF_NONE ? nullptr : xf->mats, m0, m1,
                        lat->V >= 7 ? nsum : nullptr, nullptr, st, (lat->V == 5 || lat->V == 8) ? m2 : nullptr);
}

fr_status fr_estep(const fr_lattice *lat, const fr_cloud *model_ref, const fr_xform *xf, float *m0, float *m1,
                   float *nsum, void *stream)
{
    return estep_impl(lat, model_ref, xf, m0, m1, nsum, nullptr, stream, "fr_estep");
}

fr_status fr_estep_m2(const fr_lattice *lat, const fr_cloud *model_ref, const fr_xform *xf, float *m0, float *m1,
                      float *nsum, float *m2, void *stream)
{
    if (lat_ok(lat) && (lat->V == 5 || lat->V == 8) && m2 == nullptr && cloud_points(model_ref) > 0) {
        set_error("fr_estep_m2: m2 must be non-NULL");
        return FR_EINVAL;
    }
    if (lat_ok(lat) && lat->V != 5 && lat->V != 8) {
        set_error("fr_estep_m2: the lattice has no |y|^2 channel (values FR_VAL_PT2PT_M2 or FR_VAL_PT2PL_M2)");
        return FR_EINVAL;
    }
    return estep_impl(lat, model_ref, xf, m0, m1, nsum, m2, stream, "fr_estep_m2");
}

fr_status fr_estep_touched(const fr_lattice *lat, const fr_cloud *model_ref, const fr_xform *xf, int32_t set,
                           int64_t *n_touched)
{
    clear_error();
    if (!lat_ok(lat) || n_touched == nullptr || set < 0 || set >= lat->n_sets) {
        set_error("fr_estep_touched: invalid argument");
        return FR_EINVAL;
    }
    FR_TRY(check_cloud(model_ref, lat->d == 6, "fr_estep_touched"));
    if (model_ref->n_sets != lat->n_sets) {
        set_error("fr_estep_touched: set count mismatch");
        return FR_EINVAL;
    }
    FR_TRY(check_xform(xf, model_ref, "fr_estep_touched"));
    FR_HIP(hipSetDevice(lat->ctx->device));
    hipStream_t st = nullptr;
    const SetTable &t = lat->sets_h[set];
    const size_t total_slots = (size_t)lat->n_slots;
    DevBuf flags;
    FR_TRY(flags.alloc(lat->ctx, total_slots * sizeof(uint32_t)));
    FR_HIP(hipMemset(flags.p, 0, total_slots * sizeof(uint32_t)));
    Plan plan;
    FR_TRY(make_plan(lat->ctx, model_ref, xf, kEstepTile, nullptr, st, plan));
    const int kind = xf ? xf->kind : FR_XF_NONE;
    FR_TRY(launch_estep(lat, model_ref, plan, kind, kind == FR_XF_NONE ? nullptr : xf->mats, nullptr, nullptr,
                        nullptr, flags.as<uint32_t>(), st));
    FR_HIP(hipDeviceSynchronize());
    std::vector<uint32_t> h((size_t)t.cap);
    FR_HIP(hipMemcpy(h.data(), flags.as<uint32_t>() + t.slot_base, h.size() * sizeof(uint32_t),
                     hipMemcpyDeviceToHost));
    int64_t n = 0;
    for (uint32_t v : h) n += v != 0u;
    *n_touched = n;
    return FR_OK;
}

fr_status fr_mstep_reduce(const fr_cloud *model_ref, const fr_xform *xf, const float *m0, const float *m1,
                          const float *nsum, const fr_mstep_params *params, double *jtj, double *jtr, double *stats,
                          void *stream)
{
    clear_error();
    FR_TRY(check_cloud(model_ref, false, "fr_mstep_reduce"));
    FR_TRY(check_xform(xf, model_ref, "fr_mstep_reduce"));
    if (params == nullptr || (params->residual != FR_PT2PT && params->residual != FR_PT2PL) ||
        !(params->sigma > 0.0) || !(params->c >= 0.0)) {
        set_error("fr_mstep_reduce: residual must be PT2PT/PT2PL, sigma > 0, c >= 0");
        return FR_EINVAL;
    }
    if (jtj == nullptr || jtr == nullptr || stats == nullptr) {
        set_error("fr_mstep_reduce: outputs must be non-NULL");
        return FR_EINVAL;
    }
    const int64_t M = cloud_points(model_ref);
    if (M > 0 && (m0 == nullptr || m1 == nullptr || (params->residual == FR_PT2PL && nsum == nullptr))) {
        set_error("fr_mstep_reduce: m0/m1 (and nsum for point-to-plane) must be non-NULL");
        return FR_EINVAL;
    }
    int dev = 0;
    FR_HIP(hipGetDevice(&dev));
    fr_ctx tmp_ctx;
    tmp_ctx.device = dev;
    hipStream_t st = static_cast<hipStream_t>(stream);
    StreamScope scope(st);
    std::vector<double> cset(model_ref->n_sets, params->c);
    if (params->c_per_set)
        for (int32_t s = 0; s < model_ref->n_sets; ++s) cset[s] = params->c_per_set[s];
    Plan plan;
    FR_TRY(make_plan(&tmp_ctx, model_ref, xf, 1024, cset.data(), st, plan));
    DevBuf part;
    FR_TRY(part.alloc(&tmp_ctx, reduce_partials_floats(plan) * sizeof(float)));
    const int kind = xf ? xf->kind : FR_XF_NONE;
    FR_TRY(launch_reduce(model_ref, plan, kind, kind == FR_XF_NONE ? nullptr : xf->mats, m0, m1, nsum,
                         params->residual, params->normalize_n, params->sigma, jtj, jtr, stats, part.as<float>(),
                         st));
    FR_HIP(hipStreamSynchronize(st));
    return FR_OK;
}

// ---------------------------------------------------------------------------
// fr_mstep_reduce without allocation: the tile map and the per-tile partial
// rows of the reduction live in one file-scope device array.  Each GPU the
// library runs on holds its own copy until the process ends; host code only
// ever uses the address hipGetSymbolAddress returns for it on that device.
// ---------------------------------------------------------------------------
static __device__ __attribute__((aligned(256))) unsigned char scratch[FR_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per device.
static fr_status scratch_address(void **out)
{
    int dev = 0;
    FR_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("fr_mstep_reduce_noalloc: device %d beyond the %d the library tracks", dev, kMaxDevices);
        return FR_EINVAL;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_dev[dev] == nullptr) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr) {
            set_error("fr_mstep_reduce_noalloc: hipGetSymbolAddress of the scratch array failed: %s",
                      hipGetErrorString(e));
            return FR_EDEVICE;
        }
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return FR_OK;
}

fr_status fr_mstep_reduce_noalloc(const fr_cloud *model_ref, const fr_xform *xf, const float *m0, const float *m1,
                                  const float *nsum, const fr_mstep_params *params, double *jtj, double *jtr,
                                  double *stats, void *stream)
{
    clear_error();
    FR_TRY(check_cloud(model_ref, false, "fr_mstep_reduce_noalloc"));
    FR_TRY(check_xform(xf, model_ref, "fr_mstep_reduce_noalloc"));
    if (params == nullptr || (params->residual != FR_PT2PT && params->residual != FR_PT2PL) ||
        !(params->sigma > 0.0) || !(params->c >= 0.0)) {
        set_error("fr_mstep_reduce_noalloc: residual must be PT2PT/PT2PL, sigma > 0, c >= 0");
        return FR_EINVAL;
    }
    if (jtj == nullptr || jtr == nullptr || stats == nullptr) {
        set_error("fr_mstep_reduce_noalloc: outputs must be non-NULL");
        return FR_EINVAL;
    }
    const int64_t M = cloud_points(model_ref);
    if (M > 0 && (m0 == nullptr || m1 == nullptr || (params->residual == FR_PT2PL && nsum == nullptr))) {
        set_error("fr_mstep_reduce_noalloc: m0/m1 (and nsum for point-to-plane) must be non-NULL");
        return FR_EINVAL;
    }
    std::vector<double> cset(model_ref->n_sets, params->c);
    if (params->c_per_set)
        for (int32_t s = 0; s < model_ref->n_sets; ++s) cset[s] = params->c_per_set[s];
    Plan plan;
    std::vector<char> image;
    FR_TRY(plan_layout(model_ref, xf, 1024, cset.data(), plan, image));
    // scratch = [tile map image | partial rows], the rows 256-byte aligned
    const size_t rows_off = (image.size() + 255) / 256 * 256;
    const size_t need = rows_off + reduce_partials_floats(plan) * sizeof(float);
    if (need > (size_t)FR_NOALLOC_SCRATCH_BYTES) {
        set_error("fr_mstep_reduce_noalloc: %zu bytes of tile map and partial rows (%d segments, %d tiles of 1024 "
                  "points) exceed its %d-byte scratch; use fr_mstep_reduce",
                  need, plan.n_seg, plan.n_tiles, (int)FR_NOALLOC_SCRATCH_BYTES);
        return FR_EINVAL;
    }
    void *base = nullptr;
    FR_TRY(scratch_address(&base));
    hipStream_t st = static_cast<hipStream_t>(stream);
    char *sp = static_cast<char *>(base);
    if (!image.empty()) FR_HIP(hipMemcpyAsync(sp, image.data(), image.size(), hipMemcpyHostToDevice, st));
    plan_bind(plan, sp);
    // every tile rewrites its whole partial row before the final sum reads it: nothing to clear
    const int kind = xf ? xf->kind : FR_XF_NONE;
    FR_TRY(launch_reduce(model_ref, plan, kind, kind == FR_XF_NONE ? nullptr : xf->mats, m0, m1, nsum,
                         params->residual, params->normalize_n, params->sigma, jtj, jtr, stats,
                         reinterpret_cast<float *>(sp + rows_off), st));
    FR_HIP(hipStreamSynchronize(st));   // the host image and the scratch are free for the next call
    return FR_OK;
}

fr_status fr_solve_rigid(int32_t n, const double *jtj, const double *jtr, double *poses, float *mats,
                         double *twist_norm, int32_t *status, const int32_t *active, void *stream)
{
    clear_error();
    if (n < 0 || (n > 0 && (!jtj || !jtr || !poses || !mats || !twist_norm || !status))) {
        set_error("fr_solve_rigid: invalid argument");
        return FR_EINVAL;
    }
    return launch_solve_rigid(n, jtj, jtr, poses, mats, twist_norm, status, active,
                              static_cast<hipStream_t>(stream));
}

// The context's capture stream (created on first use, default priority,
// non-blocking); graphs are captured and replayed on it.
static fr_status graph_stream(fr_ctx *ctx, hipStream_t &gs)
{
    if (ctx->graph_stream == nullptr) FR_HIP(hipStreamCreateWithFlags(&ctx->graph_stream, hipStreamNonBlocking));
    gs = ctx->graph_stream;
    return FR_OK;
}

// Pinned host memory for n words of stop flags (kept by the context; the
// previous contents are not needed once the caller's stream is idle).
static fr_status pinned_flags(fr_ctx *ctx, size_t n, int32_t *&out)
{
    if (ctx->pin_flags_n < n) {
        if (ctx->pin_flags) FR_HIP(hipHostFree(ctx->pin_flags));
        ctx->pin_flags = nullptr;
        ctx->pin_flags_n = 0;
        FR_HIP(hipHostMalloc(reinterpret_cast<void **>(&ctx->pin_flags), n * sizeof(int32_t), hipHostMallocDefault));
        ctx->pin_flags_n = n;
    }
    out = ctx->pin_flags;
    return FR_OK;
}

struct GraphGuard {
    hipGraph_t g = nullptr;
    hipGraphExec_t e = nullptr;
    ~GraphGuard()
    {
        if (e) (void)hipGraphExecDestroy(e);
        if (g) (void)hipGraphDestroy(g);
    }
};

// Stream-ordered release of a lattice the caller's loop no longer reads.
static void release_lattice(fr_lattice *lat, hipStream_t st)
{
    free_lattice(lat, st, false);
    lat->magic = kDeadMagic;
    delete lat;
}

fr_status fr_register(fr_ctx *ctx, const fr_cloud *model_ref, const fr_cloud *obs, const fr_register_params *params,
                      double *theta_inout_h, int32_t *status_h, fr_report *report_h, void *stream)
{
    clear_error();
    using clk = std::chrono::steady_clock;
    if (!ctx_ok(ctx) || params == nullptr || theta_inout_h == nullptr) {
        set_error("fr_register: invalid context, params or theta");
        return FR_EINVAL;
    }
    FR_TRY(check_lattice_params(&params->lattice));
    if (params->residual != FR_PT2PT && params->residual != FR_PT2PL) {
        set_error("fr_register: residual must be FR_PT2PT or FR_PT2PL");
        return FR_EINVAL;
    }
    if (params->residual == FR_PT2PL && params->lattice.values != FR_VAL_PT2PL) {
        set_error("fr_register: point-to-plane needs a lattice with values = FR_VAL_PT2PL");
        return FR_EINVAL;
    }
    if (params->lattice.values != FR_VAL_PT2PT && params->lattice.values != FR_VAL_PT2PL) {
        set_error("fr_register: values must be FR_VAL_PT2PT or FR_VAL_PT2PL (the |y|^2 layouts serve "
                  "fr_register_sigma)");
        return FR_EINVAL;
    }
    if (params->max_iters < 0 || params->kinematics != FR_KIN_RIGID || !(params->w >= 0.0 && params->w < 1.0)) {
        set_error("fr_register: max_iters >= 0, rigid kinematics and 0 <= w < 1 are required");
        return FR_EINVAL;
    }
    const bool blurred = (params->flags & FR_BLURRED) != 0;
    if (blurred && (params->flags & FR_FUSED) != 0) {
        set_error("fr_register: FR_BLURRED and FR_FUSED cannot be combined");
        return FR_EINVAL;
    }
    FR_TRY(check_cloud(model_ref, params->lattice.feat == 6, "fr_register(model)"));
    FR_TRY(check_cloud(obs, params->lattice.feat == 6 || params->lattice.values >= 7, "fr_register(obs)"));
    if (model_ref->n_sets != obs->n_sets) {
        set_error("fr_register: model has %d sets, observation %d", model_ref->n_sets, obs->n_sets);
        return FR_EINVAL;
    }
    FR_HIP(hipSetDevice(ctx->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    StreamScope scope(st);
    const int32_t S = model_ref->n_sets;
    const int64_t M = cloud_points(model_ref);
    fr_report rep{};

    auto t0 = clk::now();
    fr_lattice *lat = nullptr;
    // the uncustomised filter's lattice depends on the pose: built in the loop
    if (!blurred) FR_TRY(lattice_build_impl(ctx, obs, &params->lattice, st, &lat));
    struct LatGuard {
        fr_lattice *l;
        ~LatGuard()
        {
            if (l) fr_lattice_destroy(l);
        }
    } guard{lat};
    auto t1 = clk::now();
    rep.build_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();

    // per-set outlier constant (Eq. 7 in the units of the lattice sums)
    std::vector<double> cset(S, 0.0);
    for (int32_t s = 0; s < S; ++s)
        cset[s] = outlier_constant(params->lattice, params->w, params->c_override,
                                   (double)(model_ref->offsets[s + 1] - model_ref->offsets[s]),
                                   (double)(obs->offsets[s + 1] - obs->offsets[s]), blurred);
    const double sig_m = (params->lattice.sigma[0] + params->lattice.sigma[1] + params->lattice.sigma[2]) / 3.0;

    const bool fused = (params->flags & FR_FUSED) != 0;
    Plan pe, pr;
    FR_TRY(make_plan(ctx, model_ref, nullptr, kEstepTile, cset.data(), st, pe));
    if (!fused) FR_TRY(make_plan(ctx, model_ref, nullptr, 1024, cset.data(), st, pr));
    // The uncustomised filter rebuilds its joint lattice every iteration: in
    // place (storage sized once, no host wait) for joint clouds of up to 2^20
    // incidences, with a fall-back to the host-sized build for the rest of the
    // call if a rebuild overflows.  Larger ones keep the host-sized build:
    // there the storage's bounds (every incidence a vertex) cost the blur's
    // passes over the bound of the slots more than the waits they save (one
    // 640x480 frame: 1.1 against 0.94 ms per rebuild).
    constexpr int64_t kInplaceJointMax = (int64_t)1 << 20;
    ResidentBuild *rbj = nullptr;
    DevBuf kset_j;
    const int64_t joint_incidences = (cloud_points(obs) + M) * (params->lattice.feat + 1);
    if (blurred && joint_incidences > 0 && joint_incidences <= kInplaceJointMax) {
        FR_TRY(resident_create_joint(ctx, obs, model_ref, &params->lattice, st, &rbj));
        std::vector<float> k8((size_t)S * 8);
        set_scale_factors(params->lattice, S, nullptr, k8.data());
        FR_TRY(kset_j.alloc(ctx, k8.size() * sizeof(float)));
        FR_TRY(stage_h2d(ctx, kset_j.p, k8.data(), k8.size() * sizeof(float), st));
    }
    struct RbGuard {
        ResidentBuild *rb;
        hipStream_t st;
        ~RbGuard() { resident_destroy(rb, st); }
    } rbj_guard{rbj, st};
    const bool pl = params->residual == FR_PT2PL;
    const size_t nM = (size_t)std::max<int64_t>(M, 1);
    DevBuf wm0, wm1, wns, part, wjtj, wjtr, wstat, wpose, wmats, wtn, wstatus, wactive, witers;
    if (!fused) {
        FR_TRY(wm0.alloc(ctx, nM * sizeof(float)));
        FR_TRY(wm1.alloc(ctx, 3 * nM * sizeof(float)));
        if (pl || params->lattice.values == 7) FR_TRY(wns.alloc(ctx, 3 * nM * sizeof(float)));
    }
    FR_TRY(part.alloc(ctx, reduce_partials_floats(fused ? pe : pr) * sizeof(float)));
    FR_TRY(wjtj.alloc(ctx, S * 21 * sizeof(double)));
    FR_TRY(wjtr.alloc(ctx, S * 6 * sizeof(double)));
    FR_TRY(wstat.alloc(ctx, S * 4 * sizeof(double)));
    FR_TRY(wpose.alloc(ctx, S * 16 * sizeof(double)));
    FR_TRY(wmats.alloc(ctx, S * 12 * sizeof(float)));
    FR_TRY(wtn.alloc(ctx, S * 2 * sizeof(double)));
    FR_TRY(wstatus.alloc(ctx, S * sizeof(int32_t)));
    FR_TRY(wactive.alloc(ctx, S * sizeof(int32_t)));
    FR_TRY(witers.alloc(ctx, S * sizeof(int32_t)));
    // the loop's state as saved at the start of a block of in-place rebuilds
    DevBuf ckpt;
    const size_t ck_pose = 0, ck_mats = 16 * (size_t)S * 8, ck_tn = ck_mats + 12 * (size_t)S * 4;
    const size_t ck_status = ck_tn + 2 * (size_t)S * 8, ck_act = ck_status + (size_t)S * 4;
    const size_t ck_iters = ck_act + (size_t)S * 4, ck_bytes = ck_iters + (size_t)S * 4;
    if (rbj != nullptr) FR_TRY(ckpt.alloc(ctx, ck_bytes));
    std::vector<float> mats_h((size_t)S * 12);
    for (int32_t s = 0; s < S; ++s)
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 4; ++j) mats_h[(size_t)s * 12 + 4 * i + j] = (float)theta_inout_h[(size_t)s * 16 + 4 * i + j];
    std::vector<int32_t> active_h(S, 1), status_v(S, FR_OK), iters_v(S, 0);
    FR_HIP(hipMemcpyAsync(wpose.p, theta_inout_h, S * 16 * sizeof(double), hipMemcpyHostToDevice, st));
    FR_HIP(hipMemcpyAsync(wmats.p, mats_h.data(), S * 12 * sizeof(float), hipMemcpyHostToDevice, st));
    FR_HIP(hipMemcpyAsync(wactive.p, active_h.data(), S * sizeof(int32_t), hipMemcpyHostToDevice, st));
    FR_HIP(hipMemcpyAsync(wstatus.p, status_v.data(), S * sizeof(int32_t), hipMemcpyHostToDevice, st));
    FR_HIP(hipMemcpyAsync(witers.p, iters_v.data(), S * sizeof(int32_t), hipMemcpyHostToDevice, st));
    FR_HIP(hipStreamSynchronize(st));

    const bool prof = (params->flags & FR_PROFILE_EVENTS) != 0;
    const bool fixed = (params->flags & FR_FIXED_ITERS) != 0;
    const int max_it = params->max_iters;
    // Iteration control on the device: every solve clears the active flag of
    // a set whose step degenerated or, without FR_FIXED_ITERS, fell below the
    // twist tolerance (Sec. 6.1), and the kernels of later iterations skip that
    // set.  The host never waits for an iteration: it enqueues blocks of 4 and,
    // once the block before the last one has finished, reads its copy of the
    // flags and stops enqueuing when no set is left.
    const double tol = fixed ? -1.0 : params->twist_tol;
    int32_t *act = wactive.as<int32_t>();
    std::vector<hipEvent_t> ev;
    if (prof) {
        ev.resize(3 * (size_t)max_it + 1);
        for (auto &e : ev) FR_HIP(hipEventCreate(&e));
    }
    struct EventPair {
        hipEvent_t e[2] = {nullptr, nullptr};
        ~EventPair()
        {
            for (hipEvent_t x : e)
                if (x) (void)hipEventDestroy(x);
        }
    } bev;
    int32_t *pin = nullptr;
    if (!fixed || rbj != nullptr) FR_TRY(pinned_flags(ctx, std::max<size_t>(2 * (size_t)S, (size_t)S + 3), pin));
    if (!fixed)
        for (hipEvent_t &x : bev.e) FR_HIP(hipEventCreateWithFlags(&x, hipEventDisableTiming));
    int n_blocks = 0;
    // after a block of iterations on stream q: copy the flags; false once the previous block's copy
    // shows that every set has stopped
    auto block_done = [&](hipStream_t q, bool &more) -> fr_status {
        more = true;
        if (fixed) return FR_OK;
        const int b = n_blocks & 1;
        FR_HIP(hipMemcpyAsync(pin + (size_t)b * S, act, S * sizeof(int32_t), hipMemcpyDeviceToHost, q));
        FR_HIP(hipEventRecord(bev.e[b], q));
        if (n_blocks > 0) {
            FR_HIP(hipEventSynchronize(bev.e[b ^ 1]));
            const int32_t *f = pin + (size_t)(b ^ 1) * S;
            int32_t any = 0;
            for (int32_t s = 0; s < S; ++s) any |= f[s];
            more = any != 0;
        }
        ++n_blocks;
        return FR_OK;
    };
    // one EM iteration on stream q (without the profiling events)
    auto enqueue_iter = [&](hipStream_t q) -> fr_status {
        if (fused) {
            FR_TRY(launch_estep_fused(lat->d, lat->V, lat->sets_d, lat->err_d, 0, model_ref, pe, wmats.as<float>(),
                                      params->residual, 0, part.as<float>(), q, act));
            FR_TRY(launch_reduce_final(pe, part.as<float>(), sig_m, wjtj.as<double>(), wjtr.as<double>(),
                                       wstat.as<double>(), q));
        } else {
            FR_TRY(launch_estep(lat, model_ref, pe, FR_XF_RIGID, wmats.as<float>(), wm0.as<float>(),
                                wm1.as<float>(), lat->V == 7 ? wns.as<float>() : nullptr, nullptr, q, nullptr, act));
            FR_TRY(launch_reduce(model_ref, pr, FR_XF_RIGID, wmats.as<float>(), wm0.as<float>(), wm1.as<float>(),
                                 pl ? wns.as<float>() : nullptr, params->residual, 0, sig_m, wjtj.as<double>(),
                                 wjtr.as<double>(), wstat.as<double>(), part.as<float>(), q, nullptr, nullptr, act));
        }
        return launch_solve_rigid(S, wjtj.as<double>(), wjtr.as<double>(), wpose.as<double>(), wmats.as<float>(),
                                  wtn.as<double>(), wstatus.as<int32_t>(), act, q, act, tol, witers.as<int32_t>());
    };
    auto t2 = clk::now();
    int it = 0;
    constexpr int kBlock = 4;
    if ((params->flags & FR_GRAPH) != 0 && !prof && !blurred && max_it > 0) {
        // The iterations of a block (up to 32 with fixed iterations, 4 otherwise) are captured once
        // into a HIP graph and replayed: one launch per block instead of three or four per
        // iteration.  Capture needs a stream of its own (the caller's may be the null stream); the
        // caller's stream is idle here, and the blocks are waited for below.
        hipStream_t gs = nullptr;
        FR_TRY(graph_stream(ctx, gs));
        const int blk = fixed ? std::min(max_it, 32) : kBlock;   // bounded graph size; a remainder runs eagerly
        GraphGuard gg;
        FR_HIP(hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal));
        fr_status cs = FR_OK;
        for (int k = 0; k < blk && cs == FR_OK; ++k) cs = enqueue_iter(gs);
        const hipError_t ce = hipStreamEndCapture(gs, &gg.g);
        FR_TRY(cs);
        if (ce != hipSuccess) {
            set_error("fr_register: graph capture failed: %s", hipGetErrorString(ce));
            return FR_EDEVICE;
        }
        FR_HIP(hipGraphInstantiate(&gg.e, gg.g, nullptr, nullptr, 0));
        while (it < max_it) {
            const int n = std::min(blk, max_it - it);
            if (n == blk) {
                FR_HIP(hipGraphLaunch(gg.e, gs));
            } else {
                for (int k = 0; k < n; ++k) FR_TRY(enqueue_iter(gs));
            }
            it += n;
            bool more = true;
            if (it < max_it) FR_TRY(block_done(gs, more));
            if (!more) break;
        }
        FR_HIP(hipStreamSynchronize(gs));
    } else {
        // in-place rebuilds: the state copies of a block, and the block's check (one wait)
        char *ck = ckpt.as<char>();
        auto state_copy = [&](bool save) -> fr_status {
            const struct {
                void *dev;
                size_t off, bytes;
            } parts[] = {{wpose.p, ck_pose, 16 * (size_t)S * 8}, {wmats.p, ck_mats, 12 * (size_t)S * 4},
                         {wtn.p, ck_tn, 2 * (size_t)S * 8},       {wstatus.p, ck_status, (size_t)S * 4},
                         {wactive.p, ck_act, (size_t)S * 4},      {witers.p, ck_iters, (size_t)S * 4}};
            for (const auto &q : parts)
                FR_HIP(hipMemcpyAsync(save ? ck + q.off : q.dev, save ? q.dev : ck + q.off, q.bytes,
                                      hipMemcpyDeviceToDevice, st));
            return FR_OK;
        };
        const fr_lattice *elat = lat;   // the lattice the iteration slices
        int block_start = 0;
        std::vector<hipEvent_t> bev2;
        struct BuildEvents {
            std::vector<hipEvent_t> &e;
            ~BuildEvents()
            {
                for (auto &x : e)
                    if (x) (void)hipEventDestroy(x);
            }
        } bev2_guard{bev2};
        if (prof && rbj != nullptr) {
            bev2.assign(2 * (size_t)max_it, nullptr);
            for (auto &e : bev2) FR_HIP(hipEventCreate(&e));
        }
        while (it < max_it) {
            if (rbj != nullptr && it % kBlock == 0) {
                FR_TRY(state_copy(true));
                block_start = it;
            }
            if (blurred && rbj != nullptr) {
                if (prof) FR_HIP(hipEventRecord(bev2[2 * (size_t)it], st));
                FR_TRY(resident_build_joint(rbj, wmats.as<float>(), kset_j.as<float>(), st));
                if (prof) FR_HIP(hipEventRecord(bev2[2 * (size_t)it + 1], st));
                elat = resident_lattice(rbj);
            } else if (blurred) {
                auto tb = clk::now();
                if (lat != nullptr) {
                    release_lattice(lat, st);
                    lat = guard.l = nullptr;
                }
                FR_TRY(lattice_build_impl(ctx, obs, &params->lattice, st, &lat, nullptr, model_ref,
                                          wmats.as<float>()));
                guard.l = lat;
                FR_TRY(blur_lattice(lat, st));
                rep.build_ms += std::chrono::duration<double, std::milli>(clk::now() - tb).count();
                elat = lat;
            }
            if (prof) FR_HIP(hipEventRecord(ev[3 * it], st));
            if (fused) {
                FR_TRY(launch_estep_fused(elat->d, elat->V, elat->sets_d, elat->err_d, 0, model_ref, pe,
                                          wmats.as<float>(), params->residual, 0, part.as<float>(), st, act));
                if (prof) FR_HIP(hipEventRecord(ev[3 * it + 1], st));
                FR_TRY(launch_reduce_final(pe, part.as<float>(), sig_m, wjtj.as<double>(), wjtr.as<double>(),
                                           wstat.as<double>(), st));
            } else {
                FR_TRY(launch_estep(elat, model_ref, pe, FR_XF_RIGID, wmats.as<float>(), wm0.as<float>(),
                                    wm1.as<float>(), elat->V == 7 ? wns.as<float>() : nullptr, nullptr, st, nullptr,
                                    act));
                if (prof) FR_HIP(hipEventRecord(ev[3 * it + 1], st));
                FR_TRY(launch_reduce(model_ref, pr, FR_XF_RIGID, wmats.as<float>(), wm0.as<float>(),
                                     wm1.as<float>(), pl ? wns.as<float>() : nullptr, params->residual, 0, sig_m,
                                     wjtj.as<double>(), wjtr.as<double>(), wstat.as<double>(), part.as<float>(), st,
                                     nullptr, nullptr, act));
            }
            FR_TRY(launch_solve_rigid(S, wjtj.as<double>(), wjtr.as<double>(), wpose.as<double>(),
                                      wmats.as<float>(), wtn.as<double>(), wstatus.as<int32_t>(), act, st, act, tol,
                                      witers.as<int32_t>()));
            if (prof) FR_HIP(hipEventRecord(ev[3 * it + 2], st));
            ++it;
            if (rbj != nullptr && (it % kBlock == 0 || it == max_it)) {
                // the block's check: a rebuild that overflowed a table sends the block back to its start,
                // and the rest of the call to the host-sized build
                FR_HIP(hipMemcpyAsync(pin, act, S * sizeof(int32_t), hipMemcpyDeviceToHost, st));
                FR_HIP(hipMemcpyAsync(pin + S, resident_fail_words(rbj), 2 * sizeof(uint32_t),
                                      hipMemcpyDeviceToHost, st));
                FR_HIP(hipMemcpyAsync(pin + S + 2, resident_lattice(rbj)->err_d, sizeof(int32_t),
                                      hipMemcpyDeviceToHost, st));
                FR_HIP(hipStreamSynchronize(st));
                if (pin[S + 2] != 0) {
                    set_error("fr_register: a lattice coordinate left [-2^20, 2^20); increase sigma or centre the "
                              "cloud");
                    return FR_ERANGE;
                }
                if (pin[S] != 0 || pin[S + 1] != 0) {
                    FR_TRY(state_copy(false));
                    it = block_start;
                    elat = nullptr;
                    FR_HIP(hipStreamSynchronize(st));
                    resident_destroy(rbj, st, true);
                    rbj = rbj_guard.rb = nullptr;
                    continue;
                }
                int32_t any = 0;
                for (int32_t s2 = 0; s2 < S; ++s2) any |= pin[s2];
                if (any == 0) break;
                continue;
            }
            bool more = true;
            if (it % kBlock == 0 && it < max_it) FR_TRY(block_done(st, more));
            if (!more) break;
        }
        if (prof && !bev2.empty()) {
            FR_HIP(hipStreamSynchronize(st));
            for (int i = 0; i < it; ++i) {
                float b = 0.0f;
                FR_HIP(hipEventElapsedTime(&b, bev2[2 * (size_t)i], bev2[2 * (size_t)i + 1]));
                rep.build_ms += b;
            }
        }
    }    FR_HIP(hipMemcpyAsync(iters_v.data(), witers.p, S * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    FR_HIP(hipMemcpyAsync(theta_inout_h, wpose.p, S * 16 * sizeof(double), hipMemcpyDeviceToHost, st));
    FR_HIP(hipMemcpyAsync(status_v.data(), wstatus.p, S * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    FR_HIP(hipStreamSynchronize(st));
    auto t3 = clk::now();
    rep.iterations = 0;
    for (int32_t s = 0; s < S; ++s) rep.iterations = std::max(rep.iterations, iters_v[s]);
    rep.em_ms = std::chrono::duration<double, std::milli>(t3 - t2).count();
    if (prof) {
        for (int i = 0; i < it; ++i) {
            float a = 0.0f, b = 0.0f;
            FR_HIP(hipEventElapsedTime(&a, ev[3 * i], ev[3 * i + 1]));
            FR_HIP(hipEventElapsedTime(&b, ev[3 * i + 1], ev[3 * i + 2]));
            rep.estep_ms += a;
            rep.mstep_ms += b;
        }
        rep.estep_launches = it;
        for (auto &e : ev) (void)hipEventDestroy(e);
    }
    int32_t n_deg = 0;
    for (int32_t s = 0; s < S; ++s) {
        if (status_v[s] != FR_OK) ++n_deg;
        if (status_h) status_h[s] = status_v[s];
    }
    rep.n_degenerate = n_deg;
    if (blurred) rep.em_ms -= rep.build_ms - std::chrono::duration<double, std::milli>(t1 - t0).count();
    if (report_h) *report_h = rep;
    if (lat != nullptr) FR_TRY(fr_sync_status(lat));
    if (n_deg > 0) {
        set_error("fr_register: %d set(s) had a degenerate normal-equation system", n_deg);
        return FR_EDEGENERATE;
    }
    return FR_OK;
}


// The splat/slice kernel K(x, y) = sum_v b_v(x) b_v(y) of a lattice of scale s
// has per-axis variance s^2 / 4: a vertex's linear hat has second moment
// d (d+1)^2 / 12 (trace, isotropic) in lattice units, the position-averaged
// kernel is the hat's autocorrelation (twice that moment), and a position
// offset r is r (d+1) sqrt(2/3) / s lattice units.
constexpr double kKernelAxisVar = 0.25;

// Rigid EM with the isotropic variance as a decision variable.  The lattice
// depends on sigma, so each iteration rebuilds it from the observation with
// every set's current scale s; one E-step pass gives the Gauss-Newton terms and
// the posterior-weighted squared distance V = sum_i w_i (|x_i - t_i|^2 +
// m2_i / m0_i) (m2 taken about the target t_i).  V / (3 sum_i w_i) is the
// variance of the Gaussian the kernel stands for, so
// s^2 <- V / (3 sum_i w_i) / kKernelAxisVar after the pose step.
fr_status fr_register_sigma(fr_ctx *ctx, const fr_cloud *model_ref, const fr_cloud *obs,
                            const fr_register_params *params, double sigma_min, double *theta_inout_h,
                            double *sigma_inout_h, int32_t *status_h, fr_report *report_h, void *stream)
{
    clear_error();
    using clk = std::chrono::steady_clock;
    if (!ctx_ok(ctx) || params == nullptr || theta_inout_h == nullptr || sigma_inout_h == nullptr) {
        set_error("fr_register_sigma: invalid context, params, theta or sigma");
        return FR_EINVAL;
    }
    FR_TRY(check_lattice_params(&params->lattice));
    const int32_t want = params->residual == FR_PT2PL ? FR_VAL_PT2PL_M2 : FR_VAL_PT2PT_M2;
    if ((params->residual != FR_PT2PT && params->residual != FR_PT2PL) || params->lattice.values != want) {
        set_error("fr_register_sigma: residual FR_PT2PT needs values FR_VAL_PT2PT_M2, FR_PT2PL needs "
                  "FR_VAL_PT2PL_M2");
        return FR_EINVAL;
    }
    if (params->max_iters < 0 || params->kinematics != FR_KIN_RIGID || !(params->w >= 0.0 && params->w < 1.0) ||
        (params->flags & FR_FUSED) != 0 || !(sigma_min > 0.0)) {
        set_error("fr_register_sigma: max_iters >= 0, rigid kinematics, 0 <= w < 1, sigma_min > 0 and no "
                  "FR_FUSED are required");
        return FR_EINVAL;
    }
    FR_TRY(check_cloud(model_ref, params->lattice.feat == 6, "fr_register_sigma(model)"));
    FR_TRY(check_cloud(obs, params->lattice.feat == 6 || params->lattice.values >= 7, "fr_register_sigma(obs)"));
    if (model_ref->n_sets != obs->n_sets) {
        set_error("fr_register_sigma: model has %d sets, observation %d", model_ref->n_sets, obs->n_sets);
        return FR_EINVAL;
    }
    const int32_t S = model_ref->n_sets;
    for (int32_t s = 0; s < S; ++s)
        if (!(sigma_inout_h[s] > 0.0) || !std::isfinite(sigma_inout_h[s])) {
            set_error("fr_register_sigma: sigma of set %d must be finite and > 0", s);
            return FR_EINVAL;
        }
    FR_HIP(hipSetDevice(ctx->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    StreamScope scope(st);
    const int64_t M = cloud_points(model_ref);
    fr_report rep{};

    Plan pe, pr;
    FR_TRY(make_plan(ctx, model_ref, nullptr, kEstepTile, nullptr, st, pe));
    FR_TRY(make_plan(ctx, model_ref, nullptr, 1024, nullptr, st, pr));
    if (pr.n_seg != S) {
        set_error("fr_register_sigma: internal error (a plan of %d segments for %d sets)", pr.n_seg, S);
        return FR_EDEVICE;
    }
    const bool pl = params->residual == FR_PT2PL;
    const size_t nM = (size_t)std::max<int64_t>(M, 1);
    DevBuf wm0, wm1, wns, wm2, part, wjtj, wjtr, wstat, wvar, state, ckpt;
    FR_TRY(wm0.alloc(ctx, nM * sizeof(float)));
    FR_TRY(wm1.alloc(ctx, 3 * nM * sizeof(float)));
    FR_TRY(wm2.alloc(ctx, nM * sizeof(float)));
    if (pl) FR_TRY(wns.alloc(ctx, 3 * nM * sizeof(float)));
    FR_TRY(part.alloc(ctx, reduce_partials_floats(pr) * sizeof(float)));
    FR_TRY(wjtj.alloc(ctx, S * 21 * sizeof(double)));
    FR_TRY(wjtr.alloc(ctx, S * 6 * sizeof(double)));
    FR_TRY(wstat.alloc(ctx, S * 4 * sizeof(double)));
    FR_TRY(wvar.alloc(ctx, S * sizeof(double)));

    // The loop's state in one block (one copy saves or restores it): poses,
    // twist norms, scales s, the outlier constants' scale-free factors, the
    // binary32 transforms, lattice scale factors and outlier constants of the
    // current s, status, active flags, iteration counts and which sets the last
    // solve ran for.
    const size_t o_pose = 0, o_tn = o_pose + 16 * (size_t)S * 8, o_sig = o_tn + 2 * (size_t)S * 8;
    const size_t o_cpre = o_sig + (size_t)S * 8, o_mats = o_cpre + (size_t)S * 8;
    const size_t o_kset = o_mats + 12 * (size_t)S * 4, o_segc = o_kset + 8 * (size_t)S * 4;
    const size_t o_status = o_segc + (size_t)S * 4, o_act = o_status + (size_t)S * 4;
    const size_t o_iters = o_act + (size_t)S * 4, o_ran = o_iters + (size_t)S * 4;
    const size_t state_bytes = o_ran + (size_t)S * 4;
    std::vector<char> img(state_bytes, 0);
    {
        auto put = [&](size_t off, const void *src, size_t bytes) { std::memcpy(img.data() + off, src, bytes); };
        put(o_pose, theta_inout_h, (size_t)S * 16 * sizeof(double));
        put(o_sig, sigma_inout_h, (size_t)S * sizeof(double));
        for (int32_t s = 0; s < S; ++s) {
            const double Ms = (double)(model_ref->offsets[s + 1] - model_ref->offsets[s]);
            const double Ns = (double)(obs->offsets[s + 1] - obs->offsets[s]);
            // outlier_constant's factor ahead of the kernel mass, in its order of operations
            const double w = params->w;
            const double pre = (!(Ms > 0) || !(w > 0.0)) ? 0.0 : w / (1.0 - w) * (Ns / Ms);
            put(o_cpre + (size_t)s * 8, &pre, 8);
            float m12[12];
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 4; ++j) m12[4 * i + j] = (float)theta_inout_h[(size_t)s * 16 + 4 * i + j];
            put(o_mats + (size_t)s * 48, m12, 48);
            fr_lattice_params ls = params->lattice;
            ls.sigma[0] = ls.sigma[1] = ls.sigma[2] = sigma_inout_h[s];
            float k8[8];
            scale_factors(&ls, k8);
            put(o_kset + (size_t)s * 32, k8, 32);
            const float c = (float)outlier_constant(ls, params->w, params->c_override, Ms, Ns);
            put(o_segc + (size_t)s * 4, &c, 4);
            const int32_t ok = FR_OK, one = 1, zero = 0;
            put(o_status + (size_t)s * 4, &ok, 4);
            put(o_act + (size_t)s * 4, &one, 4);
            put(o_iters + (size_t)s * 4, &zero, 4);
        }
    }
    FR_TRY(state.alloc(ctx, state_bytes));
    FR_TRY(ckpt.alloc(ctx, state_bytes));
    FR_HIP(hipMemcpyAsync(state.p, img.data(), state_bytes, hipMemcpyHostToDevice, st));
    char *sb = state.as<char>();
    double *wpose = reinterpret_cast<double *>(sb + o_pose), *wtn = reinterpret_cast<double *>(sb + o_tn);
    double *wsig = reinterpret_cast<double *>(sb + o_sig);
    float *wmats = reinterpret_cast<float *>(sb + o_mats), *wkset = reinterpret_cast<float *>(sb + o_kset);
    float *wsegc = reinterpret_cast<float *>(sb + o_segc);
    int32_t *wstatus = reinterpret_cast<int32_t *>(sb + o_status), *act = reinterpret_cast<int32_t *>(sb + o_act);
    int32_t *witers = reinterpret_cast<int32_t *>(sb + o_iters), *wran = reinterpret_cast<int32_t *>(sb + o_ran);
    pr.seg_c = wsegc;   // the reduction reads the constants the variance update writes

    SigmaRule rule;
    {
        const int d = params->lattice.feat;
        rule.feat = d;
        rule.sigma_min = sigma_min;
        rule.sigma_n = params->lattice.sigma_n;
        rule.kernel_axis_var = kKernelAxisVar;
        rule.scale_num = std::sqrt(2.0 / 3.0) * (double)(d + 1);
        for (int i = 0; i < d; ++i) rule.scale_den[i] = std::sqrt((double)((i + 1) * (i + 2)));
        rule.mass0 = std::pow(1.5, 0.5 * d) / std::sqrt(d + 1.0);
        rule.c_override = params->c_override >= 0.0 ? params->c_override : -1.0;
        rule.c_pre = reinterpret_cast<const double *>(sb + o_cpre);
    }

    // The lattice is rebuilt in place every iteration (no host wait); a
    // rebuild whose provisional table overflowed or whose cuckoo insertion
    // gave up is caught at the end of its block, which is then run again
    // from the saved state with the build that sizes its tables on the host.
    ResidentBuild *rb = nullptr;
    if (cloud_points(obs) > 0) FR_TRY(resident_create(ctx, obs, &params->lattice, st, &rb));
    struct RbGuard {
        ResidentBuild *rb;
        hipStream_t st;
        ~RbGuard() { resident_destroy(rb, st); }
    } rb_guard{rb, st};
    int32_t *pin = nullptr;
    FR_TRY(pinned_flags(ctx, 3 * (size_t)S + 3, pin));

    const bool prof = (params->flags & FR_PROFILE_EVENTS) != 0;
    const bool fixed = (params->flags & FR_FIXED_ITERS) != 0;
    const double tol = fixed ? -1.0 : params->twist_tol;
    const int max_it = params->max_iters;
    std::vector<hipEvent_t> ev;
    struct EventsGuard {
        std::vector<hipEvent_t> &e;
        ~EventsGuard()
        {
            for (auto &x : e)
                if (x) (void)hipEventDestroy(x);
        }
    } ev_guard{ev};
    if (prof) {
        ev.assign(4 * (size_t)max_it, nullptr);
        for (auto &e : ev) FR_HIP(hipEventCreate(&e));
    }
    hipStream_t q = st;
    // E-step, reduction, solve and variance update of iteration j on a built lattice
    auto iter_kernels = [&](const fr_lattice *lat, int j) -> fr_status {
        if (prof) FR_HIP(hipEventRecord(ev[4 * (size_t)j + 1], q));
        FR_TRY(launch_estep(lat, model_ref, pe, FR_XF_RIGID, wmats, wm0.as<float>(), wm1.as<float>(),
                            pl ? wns.as<float>() : nullptr, nullptr, q, wm2.as<float>(), act));
        if (prof) FR_HIP(hipEventRecord(ev[4 * (size_t)j + 2], q));
        // the Gauss-Newton step does not depend on the residual scale: reduce at sigma = 1
        FR_TRY(launch_reduce(model_ref, pr, FR_XF_RIGID, wmats, wm0.as<float>(), wm1.as<float>(),
                             pl ? wns.as<float>() : nullptr, params->residual, 0, 1.0, wjtj.as<double>(),
                             wjtr.as<double>(), wstat.as<double>(), part.as<float>(), q, wm2.as<float>(),
                             wvar.as<double>(), act));
        FR_TRY(launch_solve_rigid(S, wjtj.as<double>(), wjtr.as<double>(), wpose, wmats, wtn, wstatus, act, q, act,
                                  tol, witers, wran));
        FR_TRY(launch_sigma_update(S, wran, wstatus, wstat.as<double>(), wvar.as<double>(), rule, wsig, wkset, wsegc,
                                   q));
        if (prof) FR_HIP(hipEventRecord(ev[4 * (size_t)j + 3], q));
        return FR_OK;
    };
    std::vector<double> sig_h(S);
    // iteration j with the build that sizes its tables on the host (waits)
    auto iter_waiting = [&](int j) -> fr_status {
        FR_HIP(hipMemcpyAsync(sig_h.data(), wsig, S * sizeof(double), hipMemcpyDeviceToHost, q));
        FR_HIP(hipStreamSynchronize(q));
        if (prof) FR_HIP(hipEventRecord(ev[4 * (size_t)j], q));
        fr_lattice *lat = nullptr;
        FR_TRY(lattice_build_impl(ctx, obs, &params->lattice, q, &lat, sig_h.data()));
        struct LatGuard {
            fr_lattice *l;
            ~LatGuard() { fr_lattice_destroy(l); }
        } guard{lat};
        FR_TRY(iter_kernels(lat, j));
        return fr_sync_status(lat);
    };
    // a block of iterations with in-place rebuilds (replaying a captured graph of
    // it measured slower here: the launches are short and the capture is per call)
    constexpr int kBlock = 4;
    auto enqueue_block = [&](int it0, int n) -> fr_status {
        for (int k = 0; k < n; ++k) {
            if (prof) FR_HIP(hipEventRecord(ev[4 * (size_t)(it0 + k)], q));
            FR_TRY(resident_build(rb, wkset, q));
            FR_TRY(iter_kernels(resident_lattice(rb), it0 + k));
        }
        return FR_OK;
    };
    const size_t flag_bytes = 3 * (size_t)S * sizeof(int32_t);   // status, active, iterations
    auto t_em = clk::now();
    int it = 0;
    while (it < max_it) {
        const int n = std::min(kBlock, max_it - it);
        bool redo = rb == nullptr;
        if (rb != nullptr) {
            FR_HIP(hipMemcpyAsync(ckpt.p, state.p, state_bytes, hipMemcpyDeviceToDevice, q));
            FR_TRY(enqueue_block(it, n));
            FR_HIP(hipMemcpyAsync(pin, wstatus, flag_bytes, hipMemcpyDeviceToHost, q));
            FR_HIP(hipMemcpyAsync(pin + 3 * S, resident_fail_words(rb), 2 * sizeof(uint32_t), hipMemcpyDeviceToHost,
                                  q));
            FR_HIP(hipMemcpyAsync(pin + 3 * S + 2, resident_lattice(rb)->err_d, sizeof(int32_t),
                                  hipMemcpyDeviceToHost, q));
            FR_HIP(hipStreamSynchronize(q));
            if (pin[3 * S + 2] != 0) {
                set_error("fr_register_sigma: a lattice coordinate left [-2^20, 2^20); increase sigma_min or "
                          "centre the cloud");
                return FR_ERANGE;
            }
            if (pin[3 * S] != 0 || pin[3 * S + 1] != 0) {
                FR_HIP(hipMemcpyAsync(state.p, ckpt.p, state_bytes, hipMemcpyDeviceToDevice, q));
                redo = true;
            }
        }
        if (redo) {
            for (int k = 0; k < n; ++k) FR_TRY(iter_waiting(it + k));
            FR_HIP(hipMemcpyAsync(pin, wstatus, flag_bytes, hipMemcpyDeviceToHost, q));
            FR_HIP(hipStreamSynchronize(q));
        }
        it += n;
        int32_t any = 0;
        for (int32_t s = 0; s < S; ++s) any |= pin[S + s];
        if (any == 0) break;
    }
    FR_HIP(hipStreamSynchronize(q));
    std::vector<int32_t> status_v(S), iters_v(S);
    std::vector<double> sig(S);
    FR_HIP(hipMemcpyAsync(theta_inout_h, wpose, S * 16 * sizeof(double), hipMemcpyDeviceToHost, st));
    FR_HIP(hipMemcpyAsync(sig.data(), wsig, S * sizeof(double), hipMemcpyDeviceToHost, st));
    FR_HIP(hipMemcpyAsync(status_v.data(), wstatus, S * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    FR_HIP(hipMemcpyAsync(iters_v.data(), witers, S * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    FR_HIP(hipStreamSynchronize(st));
    rep.iterations = 0;
    for (int32_t s = 0; s < S; ++s) rep.iterations = std::max(rep.iterations, iters_v[s]);
    rep.em_ms = std::chrono::duration<double, std::milli>(clk::now() - t_em).count();
    if (prof) {
        for (int i = 0; i < it; ++i) {
            float a = 0.0f, b = 0.0f, c = 0.0f;
            FR_HIP(hipEventElapsedTime(&a, ev[4 * (size_t)i], ev[4 * (size_t)i + 1]));
            FR_HIP(hipEventElapsedTime(&b, ev[4 * (size_t)i + 1], ev[4 * (size_t)i + 2]));
            FR_HIP(hipEventElapsedTime(&c, ev[4 * (size_t)i + 2], ev[4 * (size_t)i + 3]));
            rep.build_ms += a;
            rep.estep_ms += b;
            rep.mstep_ms += c;
        }
        rep.estep_launches = it;
        rep.em_ms -= rep.build_ms;
    }
    int32_t n_deg = 0;
    for (int32_t s = 0; s < S; ++s) {
        if (status_v[s] != FR_OK) ++n_deg;
        if (status_h) status_h[s] = status_v[s];
        sigma_inout_h[s] = sig[s];
    }
    rep.n_degenerate = n_deg;
    if (report_h) *report_h = rep;
    if (n_deg > 0) {
        set_error("fr_register_sigma: %d set(s) had a degenerate normal-equation system", n_deg);
        return FR_EDEGENERATE;
    }
    return FR_OK;
}


fr_status fr_register_features(fr_ctx *ctx, const fr_cloud *model_ref, const float *model_feat, const fr_cloud *obs,
                               const float *obs_feat, int32_t dim, double sigma_f, const fr_register_params *params,
                               double *theta_inout_h, int32_t *status_h, fr_report *report_h, void *stream)
{
    clear_error();
    using clk = std::chrono::steady_clock;
    if (!ctx_ok(ctx) || params == nullptr || theta_inout_h == nullptr) {
        set_error("fr_register_features: invalid context, params or theta");
        return FR_EINVAL;
    }
    FR_TRY(check_features(model_feat, dim, "fr_register_features(model)"));
    FR_TRY(check_features(obs_feat, dim, "fr_register_features(obs)"));
    if (params->residual != FR_PT2PT || params->max_iters < 0 || params->kinematics != FR_KIN_RIGID ||
        !(params->w >= 0.0 && params->w < 1.0) || (params->flags & (FR_FUSED | FR_BLURRED)) != 0 ||
        !(sigma_f > 0.0) || !std::isfinite(sigma_f) ||
        (params->lattice.splat != FR_SPLAT_SORTED && params->lattice.splat != FR_SPLAT_ATOMIC)) {
        set_error("fr_register_features: point-to-point residual, rigid kinematics, max_iters >= 0, 0 <= w < 1, "
                  "sigma_f > 0, no FR_FUSED / FR_BLURRED are required");
        return FR_EINVAL;
    }
    FR_TRY(check_cloud(model_ref, false, "fr_register_features(model)"));
    FR_TRY(check_cloud(obs, false, "fr_register_features(obs)"));
    if (model_ref->n_sets != obs->n_sets) {
        set_error("fr_register_features: model has %d sets, observation %d", model_ref->n_sets, obs->n_sets);
        return FR_EINVAL;
    }
    FR_HIP(hipSetDevice(ctx->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    StreamScope scope(st);
    const int32_t S = model_ref->n_sets;
    const int64_t M = cloud_points(model_ref);
    fr_report rep{};
    auto t0 = clk::now();
    fr_lattice *lat = nullptr;
    FR_TRY(feature_lattice_impl(ctx, obs, obs_feat, dim, sigma_f, params->lattice.splat, st, &lat));
    struct LatGuard {
        fr_lattice *l;
        ~LatGuard()
        {
            if (l) fr_lattice_destroy(l);
        }
    } guard{lat};
    rep.build_ms = std::chrono::duration<double, std::milli>(clk::now() - t0).count();
    std::vector<double> cset(S);
    for (int32_t s = 0; s < S; ++s)
        cset[s] = feature_outlier_constant(params->w, params->c_override,
                                           (double)(model_ref->offsets[s + 1] - model_ref->offsets[s]),
                                           (double)(obs->offsets[s + 1] - obs->offsets[s]), sigma_f, dim);
    Plan pe, pr;
    FR_TRY(make_plan(ctx, model_ref, nullptr, kEstepTile, nullptr, st, pe));
    FR_TRY(make_plan(ctx, model_ref, nullptr, 1024, cset.data(), st, pr));
    const size_t nM = (size_t)std::max<int64_t>(M, 1);
    DevBuf wm0, wm1, part, wjtj, wjtr, wstat, wpose, wmats, wtn, wstatus, wactive;
    FR_TRY(wm0.alloc(ctx, nM * sizeof(float)));
    FR_TRY(wm1.alloc(ctx, 3 * nM * sizeof(float)));
    FR_TRY(part.alloc(ctx, reduce_partials_floats(pr) * sizeof(float)));
    FR_TRY(wjtj.alloc(ctx, S * 21 * sizeof(double)));
    FR_TRY(wjtr.alloc(ctx, S * 6 * sizeof(double)));
    FR_TRY(wstat.alloc(ctx, S * 4 * sizeof(double)));
    FR_TRY(wpose.alloc(ctx, S * 16 * sizeof(double)));
    FR_TRY(wmats.alloc(ctx, S * 12 * sizeof(float)));
    FR_TRY(wtn.alloc(ctx, S * 2 * sizeof(double)));
    FR_TRY(wstatus.alloc(ctx, S * sizeof(int32_t)));
    FR_TRY(wactive.alloc(ctx, S * sizeof(int32_t)));
    std::vector<float> mats_h((size_t)S * 12);
    for (int32_t s = 0; s < S; ++s)
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 4; ++j) mats_h[(size_t)s * 12 + 4 * i + j] = (float)theta_inout_h[(size_t)s * 16 + 4 * i + j];
    std::vector<int32_t> active_h(S, 1), status_v(S, FR_OK);
    FR_HIP(hipMemcpyAsync(wpose.p, theta_inout_h, S * 16 * sizeof(double), hipMemcpyHostToDevice, st));
    FR_HIP(hipMemcpyAsync(wmats.p, mats_h.data(), S * 12 * sizeof(float), hipMemcpyHostToDevice, st));
    FR_HIP(hipMemcpyAsync(wactive.p, active_h.data(), S * sizeof(int32_t), hipMemcpyHostToDevice, st));
    FR_HIP(hipMemcpyAsync(wstatus.p, status_v.data(), S * sizeof(int32_t), hipMemcpyHostToDevice, st));
    auto t2 = clk::now();
    // the kernel involves the descriptors only: one E-step fixes targets and weights
    struct Events {
        hipEvent_t a = nullptr, b = nullptr;
        ~Events()
        {
            if (a) (void)hipEventDestroy(a);
            if (b) (void)hipEventDestroy(b);
        }
    } ev;
    const bool prof = (params->flags & FR_PROFILE_EVENTS) != 0;
    if (prof) {
        FR_HIP(hipEventCreate(&ev.a));
        FR_HIP(hipEventCreate(&ev.b));
        FR_HIP(hipEventRecord(ev.a, st));
    }
    FR_TRY(launch_estep_features(lat, model_ref, pe, model_feat, wm0.as<float>(), wm1.as<float>(), st));
    if (prof) FR_HIP(hipEventRecord(ev.b, st));
    const bool fixed = (params->flags & FR_FIXED_ITERS) != 0;
    const int max_it = params->max_iters;
    int it = 0;
    for (; it < max_it; ++it) {
        FR_TRY(launch_reduce(model_ref, pr, FR_XF_RIGID, wmats.as<float>(), wm0.as<float>(), wm1.as<float>(), nullptr,
                             FR_PT2PT, 0, 1.0, wjtj.as<double>(), wjtr.as<double>(), wstat.as<double>(),
                             part.as<float>(), st));
        FR_TRY(launch_solve_rigid(S, wjtj.as<double>(), wjtr.as<double>(), wpose.as<double>(), wmats.as<float>(),
                                  wtn.as<double>(), wstatus.as<int32_t>(), wactive.as<int32_t>(), st));
        if (!fixed && ((it + 1) % 4 == 0 || it + 1 == max_it)) {
            std::vector<double> tn((size_t)S * 2);
            FR_HIP(hipMemcpyAsync(tn.data(), wtn.p, S * 2 * sizeof(double), hipMemcpyDeviceToHost, st));
            FR_HIP(hipMemcpyAsync(status_v.data(), wstatus.p, S * sizeof(int32_t), hipMemcpyDeviceToHost, st));
            FR_HIP(hipStreamSynchronize(st));
            int n_active = 0;
            for (int32_t s = 0; s < S; ++s) {
                if (status_v[s] != FR_OK || (tn[2 * s] < params->twist_tol && tn[2 * s + 1] < params->twist_tol))
                    active_h[s] = 0;
                n_active += active_h[s];
            }
            FR_HIP(hipMemcpyAsync(wactive.p, active_h.data(), S * sizeof(int32_t), hipMemcpyHostToDevice, st));
            if (n_active == 0) {
                ++it;
                break;
            }
        }
    }
    FR_HIP(hipMemcpyAsync(theta_inout_h, wpose.p, S * 16 * sizeof(double), hipMemcpyDeviceToHost, st));
    FR_HIP(hipMemcpyAsync(status_v.data(), wstatus.p, S * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    FR_HIP(hipStreamSynchronize(st));
    rep.iterations = it;
    rep.em_ms = std::chrono::duration<double, std::milli>(clk::now() - t2).count();
    if (prof) {
        float a = 0.0f;
        FR_HIP(hipEventElapsedTime(&a, ev.a, ev.b));
        rep.estep_ms = a;
        rep.estep_launches = 1;
    }
    int32_t n_deg = 0;
    for (int32_t s = 0; s < S; ++s) {
        if (status_v[s] != FR_OK) ++n_deg;
        if (status_h) status_h[s] = status_v[s];
    }
    rep.n_degenerate = n_deg;
    if (report_h) *report_h = rep;
    FR_TRY(fr_sync_status(lat));
    if (n_deg > 0) {
        set_error("fr_register_features: %d set(s) had a degenerate normal-equation system", n_deg);
        return FR_EDEGENERATE;
    }
    return FR_OK;
}

fr_status fr_articulated_step(fr_ctx *ctx, const fr_kinematic_tree *tree, const double *jtj, const double *jtr,
                              double *theta, float *mats, int32_t *status, void *stream)
{
    clear_error();
    if (!ctx_ok(ctx) || tree == nullptr || theta == nullptr || mats == nullptr || ((jtj == nullptr) != (jtr == nullptr))) {
        set_error("fr_articulated_step: invalid argument");
        return FR_EINVAL;
    }
    FR_HIP(hipSetDevice(ctx->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    StreamScope scope(st);
    ArtTreeHost t;
    FR_TRY(upload_tree(ctx, tree, st, t));
    FR_TRY(launch_articulated_step(t, jtj ? 1 : 0, jtj, jtr, theta, mats, nullptr, status, st));
    FR_HIP(hipStreamSynchronize(st));
    return FR_OK;
}

fr_status fr_register_articulated(fr_ctx *ctx, const fr_cloud *model_ref, const int64_t *body_offsets,
                                  const fr_cloud *obs, const fr_kinematic_tree *tree,
                                  const fr_register_params *params, double *theta_inout_h, fr_report *report_h,
                                  void *stream)
{
    clear_error();
    using clk = std::chrono::steady_clock;
    if (!ctx_ok(ctx) || params == nullptr || theta_inout_h == nullptr || tree == nullptr || body_offsets == nullptr) {
        set_error("fr_register_articulated: invalid context, params, tree, body offsets or theta");
        return FR_EINVAL;
    }
    FR_TRY(check_lattice_params(&params->lattice));
    if ((params->residual != FR_PT2PT && params->residual != FR_PT2PL) ||
        (params->residual == FR_PT2PL && params->lattice.values != FR_VAL_PT2PL) || params->max_iters < 0 ||
        (params->lattice.values != FR_VAL_PT2PT && params->lattice.values != FR_VAL_PT2PL) ||
        !(params->w >= 0.0 && params->w < 1.0)) {
        set_error("fr_register_articulated: bad residual/values, max_iters or w");
        return FR_EINVAL;
    }
    FR_TRY(check_cloud(model_ref, params->lattice.feat == 6, "fr_register_articulated(model)"));
    FR_TRY(check_cloud(obs, params->lattice.feat == 6 || params->lattice.values >= 7, "fr_register_articulated(obs)"));
    if (model_ref->n_sets != 1 || obs->n_sets != 1) {
        set_error("fr_register_articulated: one model set and one observation set");
        return FR_EINVAL;
    }
    const int32_t B = tree->n_bodies;
    const int64_t M = cloud_points(model_ref);
    fr_xform xf{FR_XF_SEGMENTED, B, nullptr, body_offsets};
    if (B < 1 || body_offsets[0] != 0 || body_offsets[B] != M) {
        set_error("fr_register_articulated: body_offsets must partition [0, M)");
        return FR_EINVAL;
    }
    for (int32_t b = 0; b < B; ++b)
        if (body_offsets[b + 1] < body_offsets[b]) {
            set_error("fr_register_articulated: body_offsets must be non-decreasing");
            return FR_EINVAL;
        }
    FR_HIP(hipSetDevice(ctx->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    StreamScope scope(st);
    ArtTreeHost t;
    FR_TRY(upload_tree(ctx, tree, st, t));
    const int32_t n = t.n_dof;
    fr_report rep{};

    auto t0 = clk::now();
    fr_lattice *lat = nullptr;
    FR_TRY(lattice_build_impl(ctx, obs, &params->lattice, st, &lat));
    struct LatGuard {
        fr_lattice *l;
        ~LatGuard()
        {
            if (l) fr_lattice_destroy(l);
        }
    } guard{lat};
    auto t1 = clk::now();
    rep.build_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();

    const double c = outlier_constant(params->lattice, params->w, params->c_override, (double)M,
                                      (double)cloud_points(obs));
    const double sig_m = (params->lattice.sigma[0] + params->lattice.sigma[1] + params->lattice.sigma[2]) / 3.0;

    Plan pe, pr;
    FR_TRY(make_plan(ctx, model_ref, &xf, kEstepTile, nullptr, st, pe));
    FR_TRY(make_plan(ctx, model_ref, &xf, 1024, &c, st, pr));
    const bool pl = params->residual == FR_PT2PL;
    const size_t nM = (size_t)std::max<int64_t>(M, 1);
    DevBuf wm0, wm1, wns, part, wjtj, wjtr, wstat, wth, wmats, wnorm, wstatus;
    FR_TRY(wm0.alloc(ctx, nM * sizeof(float)));
    FR_TRY(wm1.alloc(ctx, 3 * nM * sizeof(float)));
    if (lat->V == 7) FR_TRY(wns.alloc(ctx, 3 * nM * sizeof(float)));
    FR_TRY(part.alloc(ctx, reduce_partials_floats(pr) * sizeof(float)));
    FR_TRY(wjtj.alloc(ctx, B * 21 * sizeof(double)));
    FR_TRY(wjtr.alloc(ctx, B * 6 * sizeof(double)));
    FR_TRY(wstat.alloc(ctx, B * 4 * sizeof(double)));
    FR_TRY(wth.alloc(ctx, n * sizeof(double)));
    FR_TRY(wmats.alloc(ctx, B * 12 * sizeof(float)));
    FR_TRY(wnorm.alloc(ctx, sizeof(double)));
    FR_TRY(wstatus.alloc(ctx, sizeof(int32_t)));
    int32_t status_h = FR_OK;
    FR_HIP(hipMemcpyAsync(wth.p, theta_inout_h, n * sizeof(double), hipMemcpyHostToDevice, st));
    FR_HIP(hipMemcpyAsync(wstatus.p, &status_h, sizeof(int32_t), hipMemcpyHostToDevice, st));
    FR_TRY(launch_articulated_step(t, 0, nullptr, nullptr, wth.as<double>(), wmats.as<float>(), nullptr, nullptr, st));
    FR_HIP(hipStreamSynchronize(st));

    const bool fixed = (params->flags & FR_FIXED_ITERS) != 0;
    auto t2 = clk::now();
    int it = 0;
    for (; it < params->max_iters; ++it) {
        FR_TRY(launch_estep(lat, model_ref, pe, FR_XF_SEGMENTED, wmats.as<float>(), wm0.as<float>(), wm1.as<float>(),
                            lat->V == 7 ? wns.as<float>() : nullptr, nullptr, st));
        FR_TRY(launch_reduce(model_ref, pr, FR_XF_SEGMENTED, wmats.as<float>(), wm0.as<float>(), wm1.as<float>(),
                             pl ? wns.as<float>() : nullptr, params->residual, 0, sig_m, wjtj.as<double>(),
                             wjtr.as<double>(), wstat.as<double>(), part.as<float>(), st));
        FR_TRY(launch_articulated_step(t, 1, wjtj.as<double>(), wjtr.as<double>(), wth.as<double>(),
                                       wmats.as<float>(), wnorm.as<double>(), wstatus.as<int32_t>(), st));
        if (!fixed || it + 1 == params->max_iters) {
            double nrm = 0.0;
            FR_HIP(hipMemcpyAsync(&nrm, wnorm.p, sizeof(double), hipMemcpyDeviceToHost, st));
            FR_HIP(hipMemcpyAsync(&status_h, wstatus.p, sizeof(int32_t), hipMemcpyDeviceToHost, st));
            FR_HIP(hipStreamSynchronize(st));
            if (status_h != FR_OK || (!fixed && nrm < params->twist_tol)) {
                ++it;
                break;
            }
        }
    }
    FR_HIP(hipMemcpyAsync(theta_inout_h, wth.p, n * sizeof(double), hipMemcpyDeviceToHost, st));
    FR_HIP(hipMemcpyAsync(&status_h, wstatus.p, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    FR_HIP(hipStreamSynchronize(st));
    rep.iterations = it;
    rep.em_ms = std::chrono::duration<double, std::milli>(clk::now() - t2).count();
    rep.n_degenerate = status_h != FR_OK ? 1 : 0;
    if (report_h) *report_h = rep;
    FR_TRY(fr_sync_status(lat));
    if (status_h != FR_OK) {
        set_error("fr_register_articulated: degenerate normal equations");
        return FR_EDEGENERATE;
    }
    return FR_OK;
}


static fr_status check_graph(const fr_node_graph *graph, int64_t M, const char *what)
{
    const int32_t K = graph->n_nodes;
    if (K < 1 || graph->nodes == nullptr || (M > 0 && (graph->skin_idx == nullptr || graph->skin_w == nullptr)) ||
        graph->n_edges < 0 || (graph->n_edges > 0 && graph->edges == nullptr) || !(graph->lambda >= 0.0)) {
        set_error("%s: graph needs nodes, skinning arrays, edges and lambda >= 0", what);
        return FR_EINVAL;
    }
    for (int64_t i = 0; i < 4 * M; ++i)
        if (graph->skin_idx[i] < 0 || graph->skin_idx[i] >= K) {
            set_error("%s: skin index %d out of [0, %d)", what, graph->skin_idx[i], K);
            return FR_EINVAL;
        }
    for (int32_t q = 0; q < 2 * graph->n_edges; ++q)
        if (graph->edges[q] < 0 || graph->edges[q] >= K) {
            set_error("%s: edge node out of range", what);
            return FR_EINVAL;
        }
    return FR_OK;
}

// The node-graph M-step alone (the reduction fr_register_nodegraph runs every
// iteration, without the solve): block structure from the graph, per-point
// terms at the moved points, ordered binary64 block sums, regulariser at the
// given node transforms, assembly; then copies of the blocks and the
// right-hand side into the caller's arrays.
fr_status fr_mstep_reduce_nodes(fr_ctx *ctx, const fr_cloud *x, const float *m0, const float *m1, const float *nsum,
                                const fr_node_graph *graph, const double *node_T_h, const fr_mstep_params *params,
                                int64_t *n_blocks, int32_t *block_nodes_h, double *blocks, double *rhs, void *stream)
{
    clear_error();
    if (!ctx_ok(ctx) || x == nullptr || graph == nullptr || node_T_h == nullptr || params == nullptr ||
        n_blocks == nullptr) {
        set_error("fr_mstep_reduce_nodes: invalid context, cloud, graph, node transforms, params or n_blocks");
        return FR_EINVAL;
    }
    FR_TRY(check_cloud(x, false, "fr_mstep_reduce_nodes(x)"));
    if (x->n_sets != 1 || (params->residual != FR_PT2PT && params->residual != FR_PT2PL) ||
        params->normalize_n != 0 || !(params->sigma > 0.0) || !(params->c >= 0.0)) {
        set_error("fr_mstep_reduce_nodes: one set, residual FR_PT2PT or FR_PT2PL, normalize_n 0, sigma > 0, c >= 0");
        return FR_EINVAL;
    }
    const int64_t M = cloud_points(x);
    if (M > 0 && (m0 == nullptr || m1 == nullptr || (params->residual == FR_PT2PL && nsum == nullptr))) {
        set_error("fr_mstep_reduce_nodes: m0, m1 (and nsum for point-to-plane) are required");
        return FR_EINVAL;
    }
    FR_TRY(check_graph(graph, M, "fr_mstep_reduce_nodes"));
    FR_HIP(hipSetDevice(ctx->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    StreamScope scope(st);
    NodeGraphDev d;
    FR_TRY(ng_setup(ctx, graph, M, st, d));
    *n_blocks = d.n_blocks;
    if (blocks == nullptr) return FR_OK;
    if (rhs == nullptr || block_nodes_h == nullptr) {
        set_error("fr_mstep_reduce_nodes: blocks, rhs and block_nodes_h are required together");
        return FR_EINVAL;
    }
    const int32_t K = graph->n_nodes;
    std::vector<double> T12((size_t)12 * K);
    for (int32_t k = 0; k < K; ++k)
        for (int j = 0; j < 12; ++j) T12[(size_t)12 * k + j] = node_T_h[(size_t)16 * k + j];
    FR_HIP(hipMemcpyAsync(d.T, T12.data(), T12.size() * sizeof(double), hipMemcpyHostToDevice, st));
    FR_TRY(ng_reduce(d, x->x, x->y, x->z, m0, m1, nsum, params->residual, params->c, params->sigma, graph->lambda, st));
    FR_HIP(hipMemcpyAsync(blocks, d.A, (size_t)36 * d.n_blocks * sizeof(double), hipMemcpyDeviceToDevice, st));
    FR_HIP(hipMemcpyAsync(rhs, d.rhs, (size_t)6 * K * sizeof(double), hipMemcpyDeviceToDevice, st));
    for (int32_t b = 0; b < d.n_blocks; ++b) {
        block_nodes_h[2 * b] = (int32_t)(d.block_keys[b] / K);
        block_nodes_h[2 * b + 1] = (int32_t)(d.block_keys[b] % K);
    }
    FR_HIP(hipStreamSynchronize(st));
    return FR_OK;
}

fr_status fr_register_nodegraph(fr_ctx *ctx, const fr_cloud *model_ref, const fr_cloud *obs, const fr_node_graph *graph,
                                const fr_register_params *params, double *node_T_inout_h, fr_report *report_h,
                                void *stream)
{
    clear_error();
    using clk = std::chrono::steady_clock;
    if (!ctx_ok(ctx) || params == nullptr || node_T_inout_h == nullptr || graph == nullptr) {
        set_error("fr_register_nodegraph: invalid context, params, graph or node transforms");
        return FR_EINVAL;
    }
    FR_TRY(check_lattice_params(&params->lattice));
    if ((params->residual != FR_PT2PT && params->residual != FR_PT2PL) ||
        (params->residual == FR_PT2PL && params->lattice.values != FR_VAL_PT2PL) || params->max_iters < 0 ||
        (params->lattice.values != FR_VAL_PT2PT && params->lattice.values != FR_VAL_PT2PL) ||
        !(params->w >= 0.0 && params->w < 1.0)) {
        set_error("fr_register_nodegraph: bad residual/values, max_iters or w");
        return FR_EINVAL;
    }
    FR_TRY(check_cloud(model_ref, params->lattice.feat == 6, "fr_register_nodegraph(model)"));
    FR_TRY(check_cloud(obs, params->lattice.feat == 6 || params->lattice.values >= 7, "fr_register_nodegraph(obs)"));
    if (model_ref->n_sets != 1 || obs->n_sets != 1) {
        set_error("fr_register_nodegraph: one model set and one observation set");
        return FR_EINVAL;
    }
    const int64_t M = cloud_points(model_ref);
    const int32_t K = graph->n_nodes;
    FR_TRY(check_graph(graph, M, "fr_register_nodegraph"));
    FR_HIP(hipSetDevice(ctx->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    StreamScope scope(st);
    fr_report rep{};
    auto t0 = clk::now();
    fr_lattice *lat = nullptr;
    FR_TRY(lattice_build_impl(ctx, obs, &params->lattice, st, &lat));
    struct LatGuard {
        fr_lattice *l;
        ~LatGuard()
        {
            if (l) fr_lattice_destroy(l);
        }
    } guard{lat};
    rep.build_ms = std::chrono::duration<double, std::milli>(clk::now() - t0).count();

    NodeGraphDev d;
    FR_TRY(ng_setup(ctx, graph, M, st, d));
    std::vector<double> T12((size_t)12 * K);
    for (int32_t k = 0; k < K; ++k)
        for (int j = 0; j < 12; ++j) T12[(size_t)12 * k + j] = node_T_inout_h[(size_t)16 * k + j];
    FR_HIP(hipMemcpyAsync(d.T, T12.data(), T12.size() * sizeof(double), hipMemcpyHostToDevice, st));

    const double c = outlier_constant(params->lattice, params->w, params->c_override, (double)M,
                                      (double)cloud_points(obs));
    const double sig_m = (params->lattice.sigma[0] + params->lattice.sigma[1] + params->lattice.sigma[2]) / 3.0;
    const bool normals = params->lattice.feat == 6;
    const size_t nM = (size_t)std::max<int64_t>(M, 1);
    DevBuf wpts, wm0, wm1, wns;
    FR_TRY(wpts.alloc(ctx, (normals ? 6 : 3) * nM * sizeof(float)));
    FR_TRY(wm0.alloc(ctx, nM * sizeof(float)));
    FR_TRY(wm1.alloc(ctx, 3 * nM * sizeof(float)));
    if (lat->V == 7) FR_TRY(wns.alloc(ctx, 3 * nM * sizeof(float)));
    float *wp = wpts.as<float>();
    float *const outs[6] = {wp, wp + nM, wp + 2 * nM, normals ? wp + 3 * nM : nullptr, normals ? wp + 4 * nM : nullptr,
                            normals ? wp + 5 * nM : nullptr};
    int64_t offs[2] = {0, M};
    fr_cloud warped{outs[0], outs[1], outs[2], outs[3], outs[4], outs[5], offs, 1};
    Plan pe;
    FR_TRY(make_plan(ctx, &warped, nullptr, kEstepTile, nullptr, st, pe));
    auto t2 = clk::now();
    int it = 0;
    double info[2] = {0.0, 0.0};
    int32_t bad = 0;
    for (; it < params->max_iters; ++it) {
        FR_TRY(ng_warp(d, model_ref, outs, st));
        FR_TRY(launch_estep(lat, &warped, pe, FR_XF_NONE, nullptr, wm0.as<float>(), wm1.as<float>(),
                            lat->V == 7 ? wns.as<float>() : nullptr, nullptr, st));
        FR_TRY(ng_step(d, outs[0], outs[1], outs[2], wm0.as<float>(), wm1.as<float>(),
                       lat->V == 7 ? wns.as<float>() : nullptr, params->residual, c, sig_m, graph->lambda, 1e-10, 2000,
                       st));
        FR_HIP(hipMemcpyAsync(info, d.info, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
        FR_HIP(hipMemcpyAsync(&bad, d.bad, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        FR_HIP(hipStreamSynchronize(st));
        if (bad) {
            ++it;
            break;
        }
    }
    FR_HIP(hipMemcpyAsync(T12.data(), d.T, T12.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    FR_HIP(hipStreamSynchronize(st));
    for (int32_t k = 0; k < K; ++k)
        for (int j = 0; j < 12; ++j) node_T_inout_h[(size_t)16 * k + j] = T12[(size_t)12 * k + j];
    rep.iterations = it;
    rep.em_ms = std::chrono::duration<double, std::milli>(clk::now() - t2).count();
    rep.solver_iters = (int32_t)info[0];
    rep.solver_residual = info[1];
    rep.n_degenerate = bad ? 1 : 0;
    if (report_h) *report_h = rep;
    FR_TRY(fr_sync_status(lat));
    if (bad) {
        set_error("fr_register_nodegraph: a node's diagonal block is singular");
        return FR_EDEGENERATE;
    }
    return FR_OK;
}

}  // extern "C"
