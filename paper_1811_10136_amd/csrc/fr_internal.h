// Host-side internals shared by the translation units of the library:
// context and lattice objects, error reporting, budgeted device allocation,
// per-call tile maps and the kernel launchers of each .hip file.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/filterreg.h"
#include "fr_device.h"

namespace fr {

constexpr uint32_t kCtxMagic = 0xF17E0C7Cu;
constexpr uint32_t kLatMagic = 0xF17E1A77u;
constexpr uint32_t kDeadMagic = 0xDEADDEADu;

// --- errors ---------------------------------------------------------------
void set_error(const char *fmt, ...);
void clear_error();

struct Status {
    fr_status code = FR_OK;
    bool ok() const { return code == FR_OK; }
};

#define FR_HIP(call)                                                                          \
    do {                                                                                      \
        hipError_t _e = (call);                                                               \
        if (_e != hipSuccess) {                                                               \
            ::fr::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(_e), __FILE__, \
                            __LINE__);                                                        \
            return FR_EDEVICE;                                                                \
        }                                                                                     \
    } while (0)

#define FR_TRY(expr)                    \
    do {                                \
        fr_status _s = (expr);          \
        if (_s != FR_OK) return _s;     \
    } while (0)

}  // namespace fr

// --- handles (global namespace: they complete the ABI's opaque types) ------
struct fr_ctx {
    uint32_t magic = fr::kCtxMagic;
    int32_t device = 0;
    size_t budget = 0;       // 0 = unlimited; covers live and cached blocks
    size_t in_use = 0;       // bytes of live allocations
    size_t cached = 0;       // bytes of freed blocks kept for reuse
    int cu_count = 256;
    // A freed block is reused at once by allocations on the stream that last
    // used it (stream order makes that safe), elsewhere once `done` -- an event
    // recorded on that stream at the free -- has completed.  done == nullptr
    // marks a block freed with the device idle.
    struct Block {
        void *p;
        size_t bytes;
        hipStream_t stream;
        hipEvent_t done;
    };
    std::vector<Block> cache;
    std::vector<hipEvent_t> spare_events;
    hipStream_t graph_stream = nullptr;   // capture/replay stream of fr_register's graphs
    // pinned host words the EM loops read the device's per-set stop flags into
    int32_t *pin_flags = nullptr;
    size_t pin_flags_n = 0;
    // Pinned staging of small host -> device copies (tile maps, set tables,
    // scale factors): a bump arena, reset once the copies out of it have
    // completed (their events), so such a copy never makes the host wait for
    // the stream as a copy from pageable memory does.
    char *stage = nullptr;
    size_t stage_cap = 0, stage_used = 0;
    std::vector<hipEvent_t> stage_ev;
    // pinned host memory the lattice build reads its sizes back into
    char *pin_build = nullptr;
    size_t pin_build_n = 0;
    // vertices per splat record of the context's last lattice build: sizes the
    // first provisional table of the next one (loops that rebuild at a
    // shrinking scale see most records carry keys of their own)
    double vertex_ratio = 0.0;
    // kernel choices: the fixed choice (fr_ctx_set_tuning) and the autotuner's table
    int32_t slice_mode = FR_SLICE_AUTO;
    std::vector<fr_tuning_entry> tuned;
};

namespace fr {
struct ResidentBuild;
}

struct fr_lattice {
    uint32_t magic = fr::kLatMagic;
    fr_ctx *ctx = nullptr;
    int32_t d = 3, V = 4, KW = 1;
    int32_t n_sets = 0;
    int32_t splat = FR_SPLAT_SORTED;
    float k[8] = {0};               // scale factors of the lattice parameters
    std::vector<float> kset;        // n_sets x 8: scale factors of each set (per-set sigma)
    int64_t n_points_total = 0;
    int64_t n_partials = 0;           // partial records of the last build (runs of shared vertices)
    float stage_ms[4] = {-1.0f, -1.0f, -1.0f, -1.0f};   // build stages: embed, insert + ids, values, tables
    // bucketed cuckoo tables of all sets, back to back: slot_bytes(KW, VP) per
    // slot, the key words then the padded values
    uint64_t *tab = nullptr;
    size_t tab_bytes = 0;
    uint64_t n_slots = 0;
    fr::SetTable *sets_d = nullptr;   // device copy of sets_h
    std::vector<fr::SetTable> sets_h;
    // vertex arrays (for export), vertices of set s are [vbase[s], vbase[s+1])
    uint64_t *vkey = nullptr;         // KW words per vertex, word-major: vkey[w * nv + v]
    uint32_t *vocc = nullptr;
    float *vval = nullptr;            // V per vertex, channel-major: vval[c * nv + v]
    int64_t n_vertices_total = 0;
    std::vector<int64_t> vbase;
    size_t vert_bytes = 0;
    int32_t *err_d = nullptr;         // latched device fault bits
    // descriptor lattices (d = feature dimension): the d binary32 scale factors
    float *kfeat_d = nullptr;
    std::vector<float> kfeat;
    // lattices rebuilt in place: the storage and state of the rebuilds
    fr::ResidentBuild *resident = nullptr;
    fr_lattice_params params{};
};

namespace fr {

// --- budgeted allocation ---------------------------------------------------
// Stream of the API call running on this thread (set by StreamScope at each
// entry point); allocations remember it so that their release is stream-ordered.
hipStream_t current_stream();
struct StreamScope {
    hipStream_t prev;
    explicit StreamScope(hipStream_t st);
    ~StreamScope();
};

// Budgeted allocation through the context's block cache.  dev_free keeps the
// block for reuse: ordered after the work queued so far on `st`, or, with
// idle == true, after work the caller has already waited for.
fr_status dev_alloc(fr_ctx *ctx, void **p, size_t bytes);
void free_lattice(fr_lattice *lat, hipStream_t st, bool idle);
bool ctx_ok(const fr_ctx *c);
fr_status check_lattice_params(const fr_lattice_params *p);
// sigma_set (host, n_sets, may be NULL): an isotropic position sigma per set
// in place of params->sigma (the normal sigma stays params->sigma_n).
// joint_model (may be NULL): build the uncustomised filter's joint lattice of
// the observation and the model moved by joint_mats (device, n_sets x 12, or
// NULL for the identity); the model points carry no value.
fr_status lattice_build_impl(fr_ctx *ctx, const fr_cloud *obs, const fr_lattice_params *params, hipStream_t st,
                             fr_lattice **out, const double *sigma_set = nullptr,
                             const fr_cloud *joint_model = nullptr, const float *joint_mats = nullptr,
                             bool wait_end = true);
void scale_factors(const fr_lattice_params *p, float *k);
// c of Eq. 7 in the units of the lattice sums (w/(1-w) N/M times the kernel's
// mass over feature space; blurred: the uncustomised filter's kernel).
double outlier_constant(const fr_lattice_params &lp, double w, double c_override, double Ms, double Ns,
                        bool blurred = false);
void dev_free(fr_ctx *ctx, void *p, size_t bytes, hipStream_t st, bool idle = false);
void dev_release_cache(fr_ctx *ctx);

// RAII temporary device buffer charged to the context.
struct DevBuf {
    fr_ctx *ctx = nullptr;
    void *p = nullptr;
    size_t bytes = 0;
    hipStream_t stream = nullptr;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { reset(); }
    fr_status alloc(fr_ctx *c, size_t b)
    {
        reset();
        ctx = c;
        bytes = b < 16 ? 16 : b;
        stream = current_stream();
        fr_status s = dev_alloc(ctx, &p, bytes);
        if (s != FR_OK) { p = nullptr; bytes = 0; }
        return s;
    }
    void reset()
    {
        if (p) dev_free(ctx, p, bytes, stream);
        p = nullptr;
        bytes = 0;
    }
    template <class T> T *as() const { return reinterpret_cast<T *>(p); }
};

// --- per-call tile maps ----------------------------------------------------
// Device copy of the segment table of a cloud (segments are the sets, or the
// segments of an fr_xform), split into tiles of `tile` points.
struct Plan {
    int32_t n_seg = 0, n_sets = 0, tile = 256, n_tiles = 0, grid = 0;
    std::vector<int64_t> seg_off;   // host copies
    std::vector<int32_t> seg_tile, seg_set;
    DevBuf meta;                    // device: seg_off | seg_tile | seg_set | seg_c | mats of NONE
    TileMap tm{};
    const float *seg_c = nullptr;   // device, per segment outlier constant (reduce only)
    int32_t slice = FR_SLICE_AUTO;  // E-step slice kernel (FR_SLICE_*; AUTO: the context's autotuner)
    fr_ctx *ctx = nullptr;          // context of the plan (autotuner table)
    // false: an untuned size class takes the choice of the nearest tuned class of the same (d, V,
    // transform) instead of timing (the serving engine, whose launches change size every step)
    bool tune_new_classes = true;
    // > 0: launch the persistent E-step / reduction kernels on this many workgroups (a multiple of
    // 8), reading the tile count from the device plan (graph replay with any resident set)
    int32_t persist_grid = 0;
};

// Build a plan for `model_ref` segmented per `xf` (NULL = per set).
fr_status make_plan(fr_ctx *ctx, const fr_cloud *cloud, const fr_xform *xf, int32_t tile, const double *c_seg_host,
                    hipStream_t stream, Plan &plan);
// The host half of make_plan: segments, tiles and launch shape of the plan,
// and the byte image of its device tables (seg_off | seg_tile | seg_set |
// seg_c) in `image`; plan_bind points the plan's tile map at a device copy
// of that image.
fr_status plan_layout(const fr_cloud *cloud, const fr_xform *xf, int32_t tile, const double *c_seg_host, Plan &plan,
                      std::vector<char> &image);
void plan_bind(Plan &plan, const void *dev_image);

inline int64_t cloud_points(const fr_cloud *c) { return c->offsets[c->n_sets]; }
fr_status check_cloud(const fr_cloud *c, bool need_normals, const char *what);

// --- launchers ---------------------------------------------------------------
// lattice_build.hip
// wait_end == false: return once the last kernel is enqueued (the build still
// waits for its own sizes on the way); later work must be ordered after it on
// the device, and the stage times are not read.
fr_status build_lattice(fr_ctx *ctx, const fr_cloud *obs, const fr_lattice_params *prm, hipStream_t st,
                        fr_lattice *lat, const int64_t *valued_end = nullptr, bool wait_end = true);
// Joint splat of each set's observation (valued) and its model moved by mats
// (device, n_sets x 12 [R | t], or NULL), for the uncustomised filter.
fr_status build_joint_lattice(fr_ctx *ctx, const fr_cloud *obs, const fr_cloud *model, const float *mats,
                              const fr_lattice_params *prm, hipStream_t st, fr_lattice *lat);
// d+1 passes of [1/4, 1/2, 1/4] along the lattice directions, then the output
// scale 1 / (1 + 2^-d); table and vertex values are replaced.
fr_status blur_lattice(fr_lattice *lat, hipStream_t st);
// Descriptor lattice (Eq. 8): keys from feat (device, N x dim row-major
// binary32) scaled by lat->kfeat_d, values [1, y] from the points of obs.
// dim is 8, 16 or 32.
fr_status build_feature_lattice(fr_ctx *ctx, const fr_cloud *obs, const float *feat, hipStream_t st,
                                fr_lattice *lat);
bool feature_dim_supported(int dim);

// A lattice of one observation cloud rebuilt in place at any per-set scale:
// storage sized once (resident_create waits once for its set-up), and each
// resident_build only enqueues kernels on `st` -- no host wait, no allocation
// -- reading the per-set scale factors (n_sets x 8 binary32) from the device.
// resident_fail_words: two device words, a provisional-table overflow and a
// cuckoo insertion that gave up in the last rebuild (its tables are then not
// valid); range errors latch in the lattice's err_d as for build_lattice.
// The optimised-sigma loop's variance rule and the constants of the scale
// factors and outlier constant that follow sigma (host-computed once).
struct SigmaRule {
    int32_t feat = 3;
    double sigma_min = 0.0, sigma_n = 1.0, kernel_axis_var = 0.25;
    double scale_num = 0.0;         // sqrt(2/3) (d + 1)
    double scale_den[8] = {0};      // sqrt((i + 1)(i + 2))
    double mass0 = 0.0;             // (3/2)^(d/2) / sqrt(d + 1)
    double c_override = -1.0;       // >= 0: the outlier constant itself
    const double *c_pre = nullptr;  // device, per set: w / (1 - w) N_s / M_s (0: no outlier term)
};
// ran: per set, 1 where the solve just before ran (launch_solve_rigid's `ran`).
fr_status launch_sigma_update(int32_t n, const int32_t *ran, const int32_t *status, const double *stats,
                              const double *var, const SigmaRule &rule, double *sig, float *kset, float *seg_c,
                              hipStream_t st);

struct ResidentBuild;
fr_status resident_create(fr_ctx *ctx, const fr_cloud *obs, const fr_lattice_params *prm, hipStream_t st,
                          ResidentBuild **out);
fr_status resident_build(ResidentBuild *rb, const float *kset, hipStream_t st);
// The same with the scale factors from host memory (copied through a pinned
// buffer of the build, after the previous rebuild's copy has been read).
fr_status resident_build_host(ResidentBuild *rb, const float *kset_h, hipStream_t st);
fr_lattice *resident_lattice(ResidentBuild *rb);
// The uncustomised filter's joint lattice rebuilt in place: per set the
// observation points (valued) then the model points moved by the set's
// [R | t] (valueless), built and blurred by resident_build_joint; its
// arrays, tile maps, offsets and blur buffers are allocated once here.
fr_status resident_create_joint(fr_ctx *ctx, const fr_cloud *obs, const fr_cloud *model,
                                const fr_lattice_params *prm, hipStream_t st, ResidentBuild **out);
fr_status resident_build_joint(ResidentBuild *rb, const float *mats, const float *kset, hipStream_t st);
const uint32_t *resident_fail_words(const ResidentBuild *rb);
// Frees the storage and the lattice; idle: the device has finished every use
// (else the release is ordered after the work queued on st).
void resident_destroy(ResidentBuild *rb, hipStream_t st, bool idle = false);

// estep.hip
// active (device, per set, may be NULL): tiles of a set with active == 0 do
// nothing (a set that has stopped on its twist or degenerated).
fr_status launch_estep_sets(int d, int V, const SetTable *sets, int32_t *err, int32_t err_stride,
                            const fr_cloud *model, int64_t M, const Plan &plan, int xf_kind, const float *mats,
                            float *m0, float *m1, float *nsum, float *m2, uint32_t *touched, hipStream_t st,
                            const int32_t *active = nullptr);
fr_status launch_estep(const fr_lattice *lat, const fr_cloud *model, const Plan &plan, int xf_kind, const float *mats,
                       float *m0, float *m1, float *nsum, uint32_t *touched, hipStream_t st, float *m2 = nullptr,
                       const int32_t *active = nullptr);
// Persistent launches (graph replay): workgroups the device holds at once,
// a multiple of 8; the slice form the autotuner's table gives without timing
// (nearest tuned size class, else FR_SLICE_PLAIN).
int estep_persistent_grid(int d, int V, int slice);
int reduce_persistent_grid(int residual);
int tuned_slice_nearest(const fr_ctx *ctx, int d, int V, int xf_kind, int64_t pts);
// Descriptor E-step (Eq. 8): slice lat at feat (device, M x lat->d) -> m0, m1.
fr_status launch_estep_features(const fr_lattice *lat, const fr_cloud *model, const Plan &plan, const float *feat,
                                float *m0, float *m1, hipStream_t st);

// mstep.hip
fr_status launch_reduce(const fr_cloud *model, const Plan &plan, int xf_kind, const float *mats, const float *m0,
                        const float *m1, const float *nsum, int residual, int normalize_n, double sigma, double *jtj,
                        double *jtr, double *stats, float *partials, hipStream_t st, const float *m2 = nullptr,
                        double *var_stat = nullptr, const int32_t *active = nullptr);
size_t reduce_partials_floats(const Plan &plan);
fr_status launch_reduce_final(const Plan &plan, const float *partials, double sigma, double *jtj, double *jtr,
                              double *stats, hipStream_t st, double *var_stat = nullptr);
// Fused slice + reduction (E-step and M-step terms of every point in one
// pass): one partial row per E-step tile, then launch_reduce_final on `plan`.
fr_status launch_estep_fused(int d, int V, const SetTable *sets, int32_t *err, int32_t err_stride,
                             const fr_cloud *model, const Plan &plan, const float *mats, int residual,
                             int normalize_n, float *partials, hipStream_t st, const int32_t *active = nullptr);

// solve.hip
// Sets with active[i] == 0 or stop[i] == 0 are skipped (either may be NULL).
// After a set's solve, stop[i] is cleared when the step degenerated or both
// twist norms are below twist_tol (twist_tol < 0: only when it degenerated);
// iters (may be NULL) counts the solves of every set.
fr_status launch_solve_rigid(int32_t n, const double *jtj, const double *jtr, double *poses, float *mats,
                             double *twist_norm, int32_t *status, const int32_t *active, hipStream_t stream,
                             int32_t *stop = nullptr, double twist_tol = -1.0, int32_t *iters = nullptr,
                             int32_t *ran = nullptr);

// articulated.hip
struct ArtTreeHost {
    int32_t n_bodies = 0, n_dof = 0, n_levels = 0;
    const int32_t *parent = nullptr, *dof_off = nullptr;
    const int32_t *level_off = nullptr, *level_body = nullptr;   // bodies grouped by depth in the tree
    const double *origin = nullptr, *axis = nullptr;
    const uint64_t *moved_by = nullptr;
    DevBuf buf;
};
fr_status upload_tree(fr_ctx *ctx, const fr_kinematic_tree *tree, hipStream_t stream, ArtTreeHost &out);
fr_status launch_articulated_step(const ArtTreeHost &tree, int mode, const double *jtj, const double *jtr,
                                  double *theta, float *mats, double *step_norm, int32_t *status, hipStream_t stream);

// nodegraph.hip
struct NodeGraphDev {
    int32_t K = 0, E = 0, n_blocks = 0;
    int64_t M = 0;
    DevBuf meta, work;
    const double *nodes = nullptr;
    const int32_t *edges = nullptr;
    const int4 *skin_idx = nullptr;
    const float4 *skin_w = nullptr;
    const int32_t *blk_off = nullptr, *blk_pts = nullptr, *rhs_off = nullptr, *rhs_pts = nullptr;
    const float *blk_w = nullptr, *rhs_w = nullptr;
    const int32_t *reg_off = nullptr, *reg_ref = nullptr, *nreg_off = nullptr, *nreg_ref = nullptr;
    const int32_t *row_off = nullptr, *row_blk = nullptr, *row_col = nullptr, *diag_blk = nullptr;
    double *T = nullptr, *dq = nullptr, *data21 = nullptr, *bdata = nullptr, *edge_terms = nullptr, *A = nullptr,
           *minv = nullptr, *rhs = nullptr, *x = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr,
           *s = nullptr, *info = nullptr, *part = nullptr;
    float *terms = nullptr;
    int32_t *bad = nullptr;
    std::vector<int64_t> block_keys;   // block b holds rows of node key / K, columns of node key % K
};
fr_status ng_setup(fr_ctx *ctx, const fr_node_graph *g, int64_t M, hipStream_t stream, NodeGraphDev &d);
fr_status ng_warp(const NodeGraphDev &d, const fr_cloud *ref, float *const out[6], hipStream_t stream);
// The node system of one EM iteration (data blocks, regulariser, right-hand
// side) into d.A (n_blocks x 36, row-major, scaled by 1 / sigma^2) and d.rhs (6K).
fr_status ng_reduce(NodeGraphDev &d, const float *x, const float *y, const float *z, const float *m0, const float *m1,
                    const float *ns, int residual, double c, double sigma, double lambda, hipStream_t stream);
fr_status ng_step(NodeGraphDev &d, const float *x, const float *y, const float *z, const float *m0, const float *m1,
                  const float *ns, int residual, double c, double sigma, double lambda, double tol, int32_t max_it,
                  hipStream_t stream);

// scan / sort helpers (lattice_build.hip)
// Asynchronous copy of n host bytes to device memory through the context's
// pinned staging arena: the host bytes may change as soon as it returns.
fr_status stage_h2d(fr_ctx *ctx, void *dst, const void *src, size_t n, hipStream_t st);
// Pinned host memory of at least n bytes for the lattice build's read-backs
// (one per context; its contents are the caller's until the next call).
fr_status build_readback(fr_ctx *ctx, size_t n, void **out);

// ws: NULL (temporaries from the context), or scan_ws_words(n) words the caller keeps until the scan has run.
fr_status scan_exclusive_u32(fr_ctx *ctx, const uint32_t *in, uint32_t *out, size_t n, int mode, hipStream_t stream,
                             uint32_t *ws = nullptr);
size_t scan_ws_words(size_t n);

}  // namespace fr
