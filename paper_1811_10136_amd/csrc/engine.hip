// Serving engine: continuous batching of rigid registrations.
//
// A slot holds one registration (an observation/model pair) resident on the
// device: its model points in the engine's point arena, the lattice of its
// observation (built once per pair, Sec. 3.2), its binary64 pose and binary32
// [R | t].  One step runs one EM iteration (Sec. 3.1: E-step slice, M-step
// reduction, Gauss-Newton solve and twist update of Sec. 5) of any subset of
// the slots with the same three kernels fr_register uses; the segments of the
// launch are the slots, so a slot that is not stepped is an empty segment.
// Each slot's arithmetic is that of the pair alone: tiles never straddle a
// segment and every per-slot sum runs in a fixed order, so a result does not
// depend on which other requests share the launch.
//
// Memory: a request costs its arena range (model in, M0/M1/N work) plus its
// lattice; lattices come from the context's block cache and go back to it
// ordered after the steps that read them, so admission and retirement never
// synchronise the device.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "fr_internal.h"

namespace fr {

constexpr uint32_t kEngMagic = 0xF17E0E61u;
constexpr int kEngRing = 4;            // plan uploads in flight
constexpr int32_t kEngMaxSlots = 4096;

struct AdmitRec {
    double T[16];
    SetTable tab;
    int32_t slot;
    int32_t pad;
};

__global__ void __launch_bounds__(64) k_engine_admit(int32_t n, const AdmitRec *recs, double *poses, float *mats,
                                                      int32_t *status, int32_t *err, SetTable *tables, int32_t *run,
                                                      int32_t *iters)
{
    const int32_t j = blockIdx.x * 64 + threadIdx.x;
    if (j >= n) return;
    const AdmitRec r = recs[j];
    const int32_t s = r.slot;
    for (int i = 0; i < 16; ++i) poses[(size_t)s * 16 + i] = r.T[i];
    for (int i = 0; i < 3; ++i)
        for (int c = 0; c < 4; ++c) mats[(size_t)s * 12 + 4 * i + c] = (float)r.T[4 * i + c];
    status[s] = FR_OK;
    err[s] = 0;
    tables[s] = r.tab;
    run[s] = 1;
    iters[s] = 0;
}

// State of every slot for the host: a range error of the slot's E-step wins
// over the solve's status.
__global__ void __launch_bounds__(256) k_engine_state(int32_t n, const int32_t *status, const int32_t *err,
                                                       const int32_t *run, const int32_t *iters, fr_slot_state *out)
{
    const int32_t s = blockIdx.x * 256 + threadIdx.x;
    if (s < n) {
        fr_slot_state v;
        v.status = err[s] ? FR_ERANGE : status[s];
        v.iterations = iters[s];
        v.stopped = run[s] == 0 ? 1 : 0;
        v.reserved = 0;
        out[s] = v;
    }
}

}  // namespace fr

using namespace fr;

struct fr_engine {
    uint32_t magic = kEngMagic;
    fr_ctx *ctx = nullptr;
    fr_engine_params prm{};
    int d = 3, V = 4;
    bool fused = false;
    double sig_m = 1.0;
    int32_t S = 0;
    int64_t P = 0;
    hipStream_t st = nullptr;     // the caller's stream: steps, reads, releases
    hipStream_t bst = nullptr;    // the engine's build stream
    DevBuf arena, state, plan_d, partials, admit_d;
    float *x = nullptr, *y = nullptr, *z = nullptr, *nx = nullptr, *ny = nullptr, *nz = nullptr;
    float *m0 = nullptr, *m1 = nullptr, *ns = nullptr;
    double *poses = nullptr, *jtj = nullptr, *jtr = nullptr, *stats = nullptr, *twist = nullptr;
    float *mats = nullptr;
    int32_t *status = nullptr, *err = nullptr;
    int32_t *run = nullptr;           // per slot: 1 while the slot runs, cleared by the solve when it stops
    int32_t *iters = nullptr;         // per slot: solves since admission
    fr_slot_state *state_out = nullptr;
    double tol = -1.0;
    SetTable *tables = nullptr;
    int64_t offsets_h[2] = {0, 0};  // the arena as a one-set cloud
    // pinned staging: kEngRing plan images, then the admission records
    char *pin = nullptr;
    size_t plan_bytes = 0, pin_bytes = 0;
    hipEvent_t ring_ev[kEngRing] = {};
    int ring = 0;
    hipEvent_t admit_ev = nullptr;
    std::vector<hipEvent_t> pending;  // admissions the engine stream has not waited for yet
    // FR_GRAPH: the kernels of a step captured once per plan ring entry and replayed
    bool graph = false;
    bool captured = false;
    hipGraphExec_t gexec[kEngRing] = {};
    int32_t graph_slice = FR_SLICE_PLAIN;
    struct Slot {
        int32_t used = 0;
        int64_t begin = 0, m = 0;
        int32_t group = -1;
        float c = 0.0f;
    };
    std::vector<Slot> slots;
    struct Group {
        fr_lattice *lat = nullptr;
        int32_t refs = 0;
    };
    std::vector<Group> groups;
    std::vector<int32_t> mark;
};

static bool eng_ok(const fr_engine *e) { return e != nullptr && e->magic == kEngMagic; }

// Plan image layout (S segments): seg_off i64[S] | seg_end i64[S] | E-step
// tiles i32[S+1] | tiles of 1024 i32[S+1] | seg_set i32[S] | active i32[S] | c f32[S]
static size_t plan_image_bytes(int32_t S) { return ((size_t)36 * S + 8 + 255) / 256 * 256; }

static void engine_free(fr_engine *e)
{
    if (e->bst) (void)hipStreamSynchronize(e->bst);
    (void)hipStreamSynchronize(e->st);
    for (auto &g : e->groups)
        if (g.lat) {
            free_lattice(g.lat, nullptr, true);   // both streams have drained
            g.lat->magic = kDeadMagic;
            delete g.lat;
            g.lat = nullptr;
        }
    e->arena.reset();
    e->state.reset();
    e->plan_d.reset();
    e->partials.reset();
    e->admit_d.reset();
    for (hipEvent_t &ev : e->ring_ev)
        if (ev) (void)hipEventDestroy(ev);
    if (e->admit_ev) (void)hipEventDestroy(e->admit_ev);
    for (hipEvent_t ev : e->pending) (void)hipEventDestroy(ev);
    e->pending.clear();
    for (hipGraphExec_t &g : e->gexec)
        if (g) (void)hipGraphExecDestroy(g);
    if (e->pin) (void)hipHostFree(e->pin);
    if (e->bst) (void)hipStreamDestroy(e->bst);
    e->pin = nullptr;
    e->bst = nullptr;
}

fr_status fr_engine_create(fr_ctx *ctx, const fr_engine_params *params, void *stream, fr_engine **out)
{
    clear_error();
    if (!ctx_ok(ctx) || params == nullptr || out == nullptr) {
        set_error("fr_engine_create: invalid context, params or out pointer");
        return FR_EINVAL;
    }
    *out = nullptr;
    FR_TRY(check_lattice_params(&params->lattice));
    const fr_engine_params &p = *params;
    if (p.residual != FR_PT2PT && p.residual != FR_PT2PL) {
        set_error("fr_engine_create: residual must be FR_PT2PT or FR_PT2PL");
        return FR_EINVAL;
    }
    if (p.residual == FR_PT2PL && p.lattice.values != FR_VAL_PT2PL) {
        set_error("fr_engine_create: point-to-plane needs values = FR_VAL_PT2PL");
        return FR_EINVAL;
    }
    if (p.lattice.values != FR_VAL_PT2PT && p.lattice.values != FR_VAL_PT2PL) {
        set_error("fr_engine_create: values must be FR_VAL_PT2PT or FR_VAL_PT2PL");
        return FR_EINVAL;
    }
    if (p.max_slots < 1 || p.max_slots > kEngMaxSlots || p.arena_points < 1 || p.arena_points >= ((int64_t)1 << 31)) {
        set_error("fr_engine_create: 1 <= max_slots <= %d and 1 <= arena_points < 2^31 required", kEngMaxSlots);
        return FR_EINVAL;
    }
    if (!(p.w >= 0.0 && p.w < 1.0)) {
        set_error("fr_engine_create: 0 <= w < 1 required");
        return FR_EINVAL;
    }
    if ((p.flags & ~(FR_FUSED | FR_GRAPH)) != 0 || p.reserved != 0 ||
        ((p.flags & FR_FUSED) && (p.flags & FR_GRAPH))) {
        set_error("fr_engine_create: flags may hold FR_FUSED or FR_GRAPH (not both) and reserved must be 0");
        return FR_EINVAL;
    }
    FR_HIP(hipSetDevice(ctx->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    StreamScope scope(st);
    fr_engine *e = new (std::nothrow) fr_engine();
    if (!e) {
        set_error("out of host memory");
        return FR_ENOMEM;
    }
    e->ctx = ctx;
    e->prm = p;
    e->graph = (p.flags & FR_GRAPH) != 0;
    e->d = p.lattice.feat;
    e->V = p.lattice.values;
    e->S = p.max_slots;
    e->P = p.arena_points;
    e->st = st;
    e->offsets_h[1] = e->P;
    e->sig_m = (p.lattice.sigma[0] + p.lattice.sigma[1] + p.lattice.sigma[2]) / 3.0;
    e->tol = p.twist_tol > 0.0 ? p.twist_tol : -1.0;
    const int64_t P = e->P, S = e->S;
    auto fail = [&](fr_status s) {
        engine_free(e);
        e->magic = kDeadMagic;
        delete e;
        return s;
    };
    const bool normals = e->d == 6;
    const int n_in = normals ? 6 : 3;
    e->fused = (p.flags & FR_FUSED) != 0;
    const size_t arena_floats = (size_t)P * (n_in + (e->fused ? 0 : 4 + (e->V == 7 ? 3 : 0)));
    fr_status s = e->arena.alloc(ctx, arena_floats * sizeof(float));
    if (s != FR_OK) return fail(s);
    float *a = e->arena.as<float>();
    e->x = a;
    e->y = a + P;
    e->z = a + 2 * P;
    if (normals) {
        e->nx = a + 3 * P;
        e->ny = a + 4 * P;
        e->nz = a + 5 * P;
    }
    if (!e->fused) {
        e->m0 = a + n_in * P;
        e->m1 = e->m0 + P;
        if (e->V == 7) e->ns = e->m1 + 3 * P;
    }
    // per-slot state
    const size_t b_pose = S * 16 * sizeof(double), b_jtj = S * 21 * sizeof(double), b_jtr = S * 6 * sizeof(double);
    const size_t b_stat = S * 4 * sizeof(double), b_tw = S * 2 * sizeof(double), b_mats = S * 12 * sizeof(float);
    const size_t b_i32 = S * sizeof(int32_t), b_tab = S * sizeof(SetTable), b_st = S * sizeof(fr_slot_state);
    s = e->state.alloc(ctx, b_pose + b_jtj + b_jtr + b_stat + b_tw + b_mats + 4 * b_i32 + b_st + b_tab + 64);
    if (s != FR_OK) return fail(s);
    char *q = e->state.as<char>();
    e->poses = reinterpret_cast<double *>(q);
    q += b_pose;
    e->jtj = reinterpret_cast<double *>(q);
    q += b_jtj;
    e->jtr = reinterpret_cast<double *>(q);
    q += b_jtr;
    e->stats = reinterpret_cast<double *>(q);
    q += b_stat;
    e->twist = reinterpret_cast<double *>(q);
    q += b_tw;
    e->tables = reinterpret_cast<SetTable *>(q);
    q += b_tab;
    e->mats = reinterpret_cast<float *>(q);
    q += b_mats;
    e->status = reinterpret_cast<int32_t *>(q);
    q += b_i32;
    e->err = reinterpret_cast<int32_t *>(q);
    q += b_i32;
    e->run = reinterpret_cast<int32_t *>(q);
    q += b_i32;
    e->iters = reinterpret_cast<int32_t *>(q);
    q += b_i32;
    e->state_out = reinterpret_cast<fr_slot_state *>(q);
    if (hipMemsetAsync(e->state.p, 0, e->state.bytes, st) != hipSuccess) return fail(FR_EDEVICE);
    e->plan_bytes = plan_image_bytes(e->S);
    s = e->plan_d.alloc(ctx, e->plan_bytes);
    if (s != FR_OK) return fail(s);
    // reduction partials: at most one tile per slot beyond P / tile
    s = e->partials.alloc(ctx, ((size_t)(P / std::min(1024, kEstepTile) + S + 2)) * 32 * sizeof(float));
    if (s != FR_OK) return fail(s);
    s = e->admit_d.alloc(ctx, S * sizeof(AdmitRec));
    if (s != FR_OK) return fail(s);
    e->pin_bytes = kEngRing * e->plan_bytes + S * sizeof(AdmitRec);
    if (hipHostMalloc(reinterpret_cast<void **>(&e->pin), e->pin_bytes, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        e->pin = nullptr;
        set_error("fr_engine_create: pinned host allocation of %zu bytes failed", e->pin_bytes);
        return fail(FR_ENOMEM);
    }
    for (hipEvent_t &ev : e->ring_ev)
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) return fail(FR_EDEVICE);
    if (hipEventCreateWithFlags(&e->admit_ev, hipEventDisableTiming) != hipSuccess) return fail(FR_EDEVICE);
    if (hipStreamCreateWithFlags(&e->bst, hipStreamNonBlocking) != hipSuccess) {
        e->bst = nullptr;
        return fail(FR_EDEVICE);
    }
    e->slots.assign(S, fr_engine::Slot{});
    e->mark.assign(S, 0);
    if (hipStreamSynchronize(st) != hipSuccess) return fail(FR_EDEVICE);
    *out = e;
    return FR_OK;
}

fr_status fr_engine_destroy(fr_engine *e)
{
    clear_error();
    if (!eng_ok(e)) {
        set_error("fr_engine_destroy: invalid or destroyed engine");
        return FR_EINVAL;
    }
    (void)hipSetDevice(e->ctx->device);
    StreamScope scope(e->st);
    engine_free(e);
    e->magic = kDeadMagic;
    delete e;
    return FR_OK;
}

// Check that slots_h lists n distinct slots, occupied (want_used) or free.
static fr_status check_slots(fr_engine *e, int32_t n, const int32_t *slots_h, bool want_used, const char *what)
{
    if (n < 0 || n > e->S || (n > 0 && slots_h == nullptr)) {
        set_error("%s: need 0 <= n <= max_slots and a slot list", what);
        return FR_EINVAL;
    }
    fr_status s = FR_OK;
    int32_t j = 0;
    for (; j < n; ++j) {
        const int32_t k = slots_h[j];
        if (k < 0 || k >= e->S || e->mark[k] || (e->slots[k].used != 0) != want_used) {
            set_error("%s: slot %d is out of range, repeated or %s", what, k, want_used ? "free" : "occupied");
            s = FR_EINVAL;
            break;
        }
        e->mark[k] = 1;
    }
    for (int32_t i = 0; i < j; ++i) e->mark[slots_h[i]] = 0;
    return s;
}

fr_status fr_engine_admit(fr_engine *e, int32_t n, const int32_t *slots_h, const fr_cloud *model_ref,
                          const fr_cloud *obs, const int64_t *arena_begin_h, const double *T0_h)
{
    clear_error();
    if (!eng_ok(e) || n < 1 || arena_begin_h == nullptr || T0_h == nullptr) {
        set_error("fr_engine_admit: invalid engine, n < 1, or missing arena_begin / T0");
        return FR_EINVAL;
    }
    FR_TRY(check_slots(e, n, slots_h, false, "fr_engine_admit"));
    const fr_lattice_params &lp = e->prm.lattice;
    FR_TRY(check_cloud(model_ref, e->d == 6, "fr_engine_admit(model)"));
    FR_TRY(check_cloud(obs, e->d == 6 || e->V >= 7, "fr_engine_admit(obs)"));
    if (model_ref->n_sets != n || obs->n_sets != n) {
        set_error("fr_engine_admit: model and observation must hold n = %d sets", n);
        return FR_EINVAL;
    }
    // arena ranges: inside the arena, disjoint from each other and from occupied slots
    std::vector<std::pair<int64_t, int64_t>> ranges;
    for (int32_t s = 0; s < e->S; ++s)
        if (e->slots[s].used && e->slots[s].m > 0) ranges.push_back({e->slots[s].begin, e->slots[s].m});
    for (int32_t j = 0; j < n; ++j) {
        const int64_t m = model_ref->offsets[j + 1] - model_ref->offsets[j];
        const int64_t b = arena_begin_h[j];
        if (b < 0 || b > e->P || m > e->P - b) {
            set_error("fr_engine_admit: request %d needs arena [%lld, %lld) beyond %lld points", j, (long long)b,
                      (long long)(b + m), (long long)e->P);
            return FR_EINVAL;
        }
        if (m > 0) ranges.push_back({b, m});
    }
    std::sort(ranges.begin(), ranges.end());
    for (size_t i = 1; i < ranges.size(); ++i)
        if (ranges[i - 1].first + ranges[i - 1].second > ranges[i].first) {
            set_error("fr_engine_admit: arena ranges overlap at point %lld", (long long)ranges[i].first);
            return FR_EINVAL;
        }
    FR_HIP(hipSetDevice(e->ctx->device));
    StreamScope scope(e->bst);

    // lattices of the n observations: one build on the build stream
    // (the build reports a key-range overflow itself, FR_ERANGE, from the wait for its record
    // counts; its last kernels need no wait: the steps are ordered after the build on the device)
    fr_lattice *lat = nullptr;
    FR_TRY(lattice_build_impl(e->ctx, obs, &lp, e->bst, &lat, nullptr, nullptr, nullptr, false));
    int32_t g = 0;
    while (g < (int32_t)e->groups.size() && e->groups[g].lat != nullptr) ++g;
    if (g == (int32_t)e->groups.size()) e->groups.push_back(fr_engine::Group{});
    e->groups[g].lat = lat;
    e->groups[g].refs = n;

    // the arena ranges and slot state may still be read by steps queued on the
    // engine stream: order the copies after them
    hipEvent_t here = nullptr;
    FR_HIP(hipEventCreateWithFlags(&here, hipEventDisableTiming));
    FR_HIP(hipEventRecord(here, e->st));
    FR_HIP(hipStreamWaitEvent(e->bst, here, 0));
    (void)hipEventDestroy(here);
    const float *src[6] = {model_ref->x, model_ref->y, model_ref->z, model_ref->nx, model_ref->ny, model_ref->nz};
    float *dst[6] = {e->x, e->y, e->z, e->nx, e->ny, e->nz};
    const int n_in = e->d == 6 ? 6 : 3;
    for (int32_t j = 0; j < n; ++j) {
        const int64_t o = model_ref->offsets[j], m = model_ref->offsets[j + 1] - o;
        if (m == 0) continue;
        for (int a = 0; a < n_in; ++a)
            FR_HIP(hipMemcpyAsync(dst[a] + arena_begin_h[j], src[a] + o, m * sizeof(float), hipMemcpyDeviceToDevice,
                                  e->bst));
    }
    // slot state: pose, [R | t], status, range flag, lattice table
    FR_HIP(hipEventSynchronize(e->admit_ev));   // the previous admission's records were consumed
    AdmitRec *rec = reinterpret_cast<AdmitRec *>(e->pin + kEngRing * e->plan_bytes);
    for (int32_t j = 0; j < n; ++j) {
        std::memcpy(rec[j].T, T0_h + 16 * (size_t)j, 16 * sizeof(double));
        rec[j].tab = lat->sets_h[j];
        rec[j].slot = slots_h[j];
        rec[j].pad = 0;
    }
    FR_HIP(hipMemcpyAsync(e->admit_d.p, rec, n * sizeof(AdmitRec), hipMemcpyHostToDevice, e->bst));
    k_engine_admit<<<(n + 63) / 64, 64, 0, e->bst>>>(n, e->admit_d.as<AdmitRec>(), e->poses, e->mats, e->status,
                                                     e->err, e->tables, e->run, e->iters);
    FR_HIP(hipGetLastError());
    FR_HIP(hipEventRecord(e->admit_ev, e->bst));
    hipEvent_t built = nullptr;
    FR_HIP(hipEventCreateWithFlags(&built, hipEventDisableTiming));
    FR_HIP(hipEventRecord(built, e->bst));
    e->pending.push_back(built);

    for (int32_t j = 0; j < n; ++j) {
        fr_engine::Slot &sl = e->slots[slots_h[j]];
        sl.used = 1;
        sl.begin = arena_begin_h[j];
        sl.m = model_ref->offsets[j + 1] - model_ref->offsets[j];
        sl.group = g;
        sl.c = (float)outlier_constant(lp, e->prm.w, e->prm.c_override, (double)sl.m,
                                       (double)(obs->offsets[j + 1] - obs->offsets[j]));
    }
    return FR_OK;
}

// Make the engine stream wait, on the device, for every admission so far.
static fr_status join_pending(fr_engine *e)
{
    for (hipEvent_t ev : e->pending) {
        FR_HIP(hipStreamWaitEvent(e->st, ev, 0));
        (void)hipEventDestroy(ev);
    }
    e->pending.clear();
    return FR_OK;
}

static fr_status enqueue_step_kernels(fr_engine *e, int32_t e_tiles, int32_t r_tiles, int persist_e, int persist_r,
                                      hipStream_t st);
static fr_status capture_steps(fr_engine *e);

fr_status fr_engine_step(fr_engine *e, int32_t n, const int32_t *slots_h)
{
    clear_error();
    if (!eng_ok(e)) {
        set_error("fr_engine_step: invalid or destroyed engine");
        return FR_EINVAL;
    }
    FR_TRY(check_slots(e, n, slots_h, true, "fr_engine_step"));
    if (n == 0) return FR_OK;
    FR_HIP(hipSetDevice(e->ctx->device));
    StreamScope scope(e->st);
    FR_TRY(join_pending(e));
    const int32_t S = e->S;

    // plan image in the next pinned ring entry (waiting only if the host is
    // kEngRing steps ahead of the device)
    const int r = e->ring;
    e->ring = (e->ring + 1) % kEngRing;
    FR_HIP(hipEventSynchronize(e->ring_ev[r]));
    char *img = e->pin + (size_t)r * e->plan_bytes;
    int64_t *off = reinterpret_cast<int64_t *>(img);
    int64_t *end = off + S;
    int32_t *te = reinterpret_cast<int32_t *>(end + S);
    int32_t *tr = te + (S + 1);
    int32_t *set = tr + (S + 1);
    int32_t *act = set + S;
    float *cs = reinterpret_cast<float *>(act + S);
    for (int32_t j = 0; j < n; ++j) e->mark[slots_h[j]] = 1;
    te[0] = 0;
    tr[0] = 0;
    for (int32_t s = 0; s < S; ++s) {
        const fr_engine::Slot &sl = e->slots[s];
        const bool on = e->mark[s] != 0;
        off[s] = sl.begin;
        end[s] = on ? sl.begin + sl.m : sl.begin;
        const int64_t m = on ? sl.m : 0;
        te[s + 1] = te[s] + (int32_t)((m + kEstepTile - 1) / kEstepTile);
        tr[s + 1] = tr[s] + (int32_t)((m + 1023) / 1024);
        set[s] = s;
        act[s] = on ? 1 : 0;
        cs[s] = sl.c;
    }
    for (int32_t j = 0; j < n; ++j) e->mark[slots_h[j]] = 0;
    if (e->graph) {
        if (!e->captured) FR_TRY(capture_steps(e));
        // the graph copies this ring entry's plan image to the device, then runs the step's kernels
        FR_HIP(hipGraphLaunch(e->gexec[r], e->st));
        FR_HIP(hipEventRecord(e->ring_ev[r], e->st));
        return FR_OK;
    }
    FR_HIP(hipMemcpyAsync(e->plan_d.p, img, e->plan_bytes, hipMemcpyHostToDevice, e->st));
    FR_HIP(hipEventRecord(e->ring_ev[r], e->st));
    return enqueue_step_kernels(e, te[S], tr[S], 0, 0, e->st);
}

// The kernels of one step on `st`, reading the plan at plan_d: with
// persist_e > 0 the persistent E-step and reduction on persist_e / persist_r
// workgroups, their tile counts read from the plan on the device.
static fr_status enqueue_step_kernels(fr_engine *e, int32_t e_tiles, int32_t r_tiles, int persist_e, int persist_r,
                                      hipStream_t st)
{
    const int32_t S = e->S;
    const char *pd = e->plan_d.as<char>();
    const int64_t *d_off = reinterpret_cast<const int64_t *>(pd);
    const int64_t *d_end = d_off + S;
    const int32_t *d_te = reinterpret_cast<const int32_t *>(d_end + S);
    const int32_t *d_tr = d_te + (S + 1);
    const int32_t *d_set = d_tr + (S + 1);
    const int32_t *d_act = d_set + S;
    const float *d_c = reinterpret_cast<const float *>(d_act + S);
    auto make = [&](const int32_t *d_tiles, int32_t n_tiles, int32_t tile, Plan &p) {
        p.tile = tile;
        p.n_seg = S;
        p.n_sets = S;
        p.n_tiles = n_tiles;
        int32_t chunk = 0, grid = n_tiles;
        if (n_tiles >= 8 * 64) {
            chunk = (n_tiles + 7) / 8;
            grid = chunk * 8;
        }
        p.grid = grid;
        p.tm.seg_off = d_off;
        p.tm.seg_end = d_end;
        p.tm.seg_tile = d_tiles;
        p.tm.seg_set = d_set;
        p.tm.n_seg = S;
        p.tm.n_tiles = n_tiles;
        p.tm.tile = tile;
        p.tm.xcd_chunk = chunk;
        p.seg_c = d_c;
        p.ctx = e->ctx;
        p.slice = e->ctx->slice_mode;
        p.tune_new_classes = false;   // the resident set changes size every step: reuse the nearest tuned class
    };
    Plan pe, pr;
    make(d_te, e_tiles, kEstepTile, pe);
    make(d_tr, r_tiles, 1024, pr);
    if (persist_e > 0) {
        pe.persist_grid = persist_e;
        pe.slice = e->graph_slice;
        pr.persist_grid = persist_r;
    }
    fr_cloud arena{e->x, e->y, e->z, e->nx, e->ny, e->nz, e->offsets_h, 1};
    // slots that have stopped on the device (twist below tolerance, or degenerate) are skipped by
    // every kernel: a step that still lists them leaves them unchanged
    if (e->fused) {
        FR_TRY(launch_estep_fused(e->d, e->V, e->tables, e->err, 1, &arena, pe, e->mats, e->prm.residual, 0,
                                  e->partials.as<float>(), st, e->run));
        FR_TRY(launch_reduce_final(pe, e->partials.as<float>(), e->sig_m, e->jtj, e->jtr, e->stats, st));
    } else {
        FR_TRY(launch_estep_sets(e->d, e->V, e->tables, e->err, 1, &arena, e->P, pe, FR_XF_RIGID, e->mats,
                                 e->m0, e->m1, e->V == 7 ? e->ns : nullptr, nullptr, nullptr, st, e->run));
        FR_TRY(launch_reduce(&arena, pr, FR_XF_RIGID, e->mats, e->m0, e->m1,
                             e->prm.residual == FR_PT2PL ? e->ns : nullptr, e->prm.residual, 0, e->sig_m, e->jtj,
                             e->jtr, e->stats, e->partials.as<float>(), st, nullptr, nullptr, e->run));
    }
    FR_TRY(launch_solve_rigid(S, e->jtj, e->jtr, e->poses, e->mats, e->twist, e->status, d_act, st, e->run,
                              e->tol, e->iters));
    return FR_OK;
}

// FR_GRAPH: one graph per plan ring entry -- the copy of that entry's pinned
// plan image to the device, the persistent E-step and reduction, the final
// sums and the solve -- captured on a stream of its own and instantiated
// once.  Launch shapes do not depend on the plan, so every later step only
// fills the ring entry and replays its graph.  The slice form is the one the
// autotuner's table gives for the largest resident set (no timing).
static fr_status capture_steps(fr_engine *e)
{
    const int pe = estep_persistent_grid(e->d, e->V, FR_SLICE_PLAIN);
    e->graph_slice = tuned_slice_nearest(e->ctx, e->d, e->V, FR_XF_RIGID, e->P);
    const int pes = e->graph_slice == FR_SLICE_SHARED ? estep_persistent_grid(e->d, e->V, FR_SLICE_SHARED) : pe;
    const int pr = reduce_persistent_grid(e->prm.residual);
    if (pes <= 0 || pr <= 0) {
        set_error("fr_engine_step: no persistent launch shape for d=%d V=%d", e->d, e->V);
        return FR_EINVAL;
    }
    hipStream_t cs = nullptr;
    FR_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    fr_status rc = FR_OK;
    for (int r = 0; r < kEngRing && rc == FR_OK; ++r) {
        hipGraph_t g = nullptr;
        if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            rc = FR_EDEVICE;
            break;
        }
        hipError_t he = hipMemcpyAsync(e->plan_d.p, e->pin + (size_t)r * e->plan_bytes, e->plan_bytes,
                                       hipMemcpyHostToDevice, cs);
        fr_status ks = he == hipSuccess ? enqueue_step_kernels(e, 0, 0, pes, pr, cs) : FR_EDEVICE;
        const hipError_t ee = hipStreamEndCapture(cs, &g);
        if (ks != FR_OK || ee != hipSuccess || g == nullptr) {
            rc = ks != FR_OK ? ks : FR_EDEVICE;
        } else if (hipGraphInstantiate(&e->gexec[r], g, nullptr, nullptr, 0) != hipSuccess) {
            rc = FR_EDEVICE;
        }
        if (g) (void)hipGraphDestroy(g);
    }
    (void)hipStreamDestroy(cs);
    if (rc != FR_OK) {
        for (hipGraphExec_t &x : e->gexec)
            if (x) (void)hipGraphExecDestroy(x), x = nullptr;
        if (rc == FR_EDEVICE) set_error("fr_engine_step: capturing the step graph failed");
        return rc;
    }
    e->captured = true;
    return FR_OK;
}

fr_status fr_engine_read(fr_engine *e, double *poses_h, fr_slot_state *state_h)
{
    clear_error();
    if (!eng_ok(e) || state_h == nullptr) {
        set_error("fr_engine_read: invalid engine or output");
        return FR_EINVAL;
    }
    FR_HIP(hipSetDevice(e->ctx->device));
    StreamScope scope(e->st);
    FR_TRY(join_pending(e));
    k_engine_state<<<(e->S + 255) / 256, 256, 0, e->st>>>(e->S, e->status, e->err, e->run, e->iters, e->state_out);
    FR_HIP(hipGetLastError());
    if (poses_h != nullptr)
        FR_HIP(hipMemcpyAsync(poses_h, e->poses, (size_t)e->S * 16 * sizeof(double), hipMemcpyDeviceToHost, e->st));
    FR_HIP(hipMemcpyAsync(state_h, e->state_out, (size_t)e->S * sizeof(fr_slot_state), hipMemcpyDeviceToHost,
                          e->st));
    return FR_OK;
}

fr_status fr_engine_release(fr_engine *e, int32_t n, const int32_t *slots_h)
{
    clear_error();
    if (!eng_ok(e)) {
        set_error("fr_engine_release: invalid or destroyed engine");
        return FR_EINVAL;
    }
    FR_TRY(check_slots(e, n, slots_h, true, "fr_engine_release"));
    FR_HIP(hipSetDevice(e->ctx->device));
    StreamScope scope(e->st);
    for (int32_t j = 0; j < n; ++j) {
        fr_engine::Slot &sl = e->slots[slots_h[j]];
        fr_engine::Group &g = e->groups[sl.group];
        sl = fr_engine::Slot{};
        if (--g.refs == 0) {
            // steps already queued on the engine stream may still slice this lattice
            free_lattice(g.lat, e->st, false);
            g.lat->magic = kDeadMagic;
            delete g.lat;
            g.lat = nullptr;
        }
    }
    return FR_OK;
}
