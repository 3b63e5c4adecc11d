/*
 * filterreg.h -- C ABI of the MI355X FilterReg hot path.
 *
 * FilterReg (Gao & Tedrake, CVPR 2019) registers a model point set X, moved by
 * a motion parameter theta, onto a fixed observation Y (Sec. 3.1).  Its E-step
 * is a Gaussian transform evaluated with a permutohedral lattice built once
 * from Y (Sec. 3.2, Sec. 4); its M-step is a Gauss-Newton step in the twist
 * parameterisation (Sec. 5).  This library runs both on one gfx950 GPU.
 *
 * Conventions shared by every call
 *  - Every array argument named "device" is GPU memory owned by the caller and
 *    must stay valid until the work queued on `stream` has finished.  Arrays
 *    named "host" are read (or written) before the call returns.
 *  - Point clouds are structure-of-arrays binary32.  A cloud may hold several
 *    independent sets (registration pairs) back to back; `offsets` (host,
 *    n_sets + 1 entries, offsets[0] == 0, non-decreasing) delimits them.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Calls that take a stream only enqueue work and return; device-side faults
 *    they detect (key range overflow) are latched in the handle and returned by
 *    the next synchronising call (fr_lattice_stats, fr_lattice_export,
 *    fr_register, fr_sync_status).
 *  - Every call returns fr_status; FR_OK is 0.  fr_last_error() gives a
 *    thread-local message for the last failure.  No C++ exception crosses the
 *    ABI.  Argument errors are reported before anything is enqueued.
 *  - Opaque handles (fr_ctx, fr_lattice) are owned by the library and freed
 *    only by their destroy call; destroying a handle twice returns FR_EINVAL.
 *  - A context is used by one host thread at a time.
 */
#ifndef FILTERREG_H
#define FILTERREG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t fr_status;
enum {
    FR_OK = 0,
    FR_EINVAL = 1,       /* bad argument (NULL, size, sigma <= 0, unsupported d, mismatched sets) */
    FR_ENOMEM = 2,       /* device allocation failed */
    FR_EBUDGET = 3,      /* the context's HBM budget would be exceeded */
    FR_ERANGE = 4,       /* a lattice coordinate left the packed key range [-2^20, 2^20) */
    FR_EDEGENERATE = 5,  /* normal equations singular (see fr_solve_rigid), or no model point has support */
    FR_EDEVICE = 6       /* a HIP runtime call failed */
};

enum { FR_FEAT_POS = 3, FR_FEAT_POS_NORMAL = 6 };         /* feature dimension d */
/* value channels V of the lattice: [1, y], [1, y, n_y]; the _M2 layouts add |y|^2 (variance update) */
enum { FR_VAL_PT2PT = 4, FR_VAL_PT2PT_M2 = 5, FR_VAL_PT2PL = 7, FR_VAL_PT2PL_M2 = 8 };
enum { FR_SPLAT_SORTED = 0, FR_SPLAT_ATOMIC = 1 };
enum { FR_XF_NONE = 0, FR_XF_RIGID = 1, FR_XF_SEGMENTED = 2 };
enum { FR_PT2PT = 0, FR_PT2PL = 1 };
enum { FR_KIN_RIGID = 0, FR_KIN_ARTICULATED = 1, FR_KIN_NODEGRAPH = 2 };
enum { FR_FIXED_ITERS = 1, FR_PROFILE_EVENTS = 2, FR_FUSED = 4, FR_BLURRED = 8, FR_GRAPH = 16 };

typedef struct fr_ctx fr_ctx;
typedef struct fr_lattice fr_lattice;

/* Library version (major * 10000 + minor * 100 + patch). */
int32_t fr_version(void);

/* Thread-local message of the last failed call on this thread ("" if none). */
const char *fr_last_error(void);

/*
 * Create a context on HIP device `device`.  Every device allocation the
 * library makes through this context is charged to `hbm_budget_bytes`
 * (0 = no limit); a call that would exceed it fails with FR_EBUDGET.
 */
fr_status fr_ctx_create(int32_t device, size_t hbm_budget_bytes, fr_ctx **out);
fr_status fr_ctx_destroy(fr_ctx *ctx);
/* Bytes currently charged to the context's budget. */
fr_status fr_ctx_usage(const fr_ctx *ctx, size_t *bytes_in_use);

/*
 * Kernel choices of a context (tuning only: every choice gives bitwise the
 * same results).  The slice of Sec. 4.2 interpolates the lattice at each model
 * point from the d+1 vertices of its simplex:
 *   FR_SLICE_PLAIN   each model point looks its d+1 vertices up in the
 *                    lattice table (any point order);
 *   FR_SLICE_SHARED  a wavefront of 64 consecutive model points looks each
 *                    distinct vertex up once: neighbouring points of a
 *                    range-image scan share most of their vertices;
 *   FR_SLICE_AUTO    (the default) an autotuner times both on the first E-step
 *                    launch of each (d, V, transform kind, size class) the
 *                    context meets -- the launches compute the same outputs,
 *                    so they are that E-step -- and keeps the faster.  The
 *                    timing waits for the stream once; a launch enqueued while
 *                    the stream is being captured into a graph is not timed
 *                    (it takes FR_SLICE_PLAIN until a later launch tunes).
 *                    The serving engine times only when the table has no
 *                    entry for its (d, V, transform kind) yet; otherwise a
 *                    new size class takes the nearest tuned class's choice.
 * size class = floor(log2(model points of the launch)).
 */
enum { FR_SLICE_AUTO = 0, FR_SLICE_PLAIN = 1, FR_SLICE_SHARED = 2 };
typedef struct {
    int32_t slice;         /* FR_SLICE_* */
} fr_tuning;
fr_status fr_ctx_set_tuning(fr_ctx *ctx, const fr_tuning *tuning);

/* One choice of the autotuner: the mean launch times it measured (us).
 * xf_kind: the E-step's transform (FR_XF_*), or 16 + it for the fused slice
 * and reduction (FR_FUSED). */
typedef struct {
    int32_t d, V, xf_kind, size_class;
    int32_t slice;         /* FR_SLICE_PLAIN or FR_SLICE_SHARED */
    float us_plain, us_shared;
} fr_tuning_entry;
/* Copies up to `cap` entries of the context's autotuner table to out_h (host)
 * and their total count to *n (host). */
fr_status fr_ctx_tuning_table(const fr_ctx *ctx, fr_tuning_entry *out_h, int32_t cap, int32_t *n);

/* A point cloud of n_sets sets (see the conventions above). */
typedef struct {
    const float *x, *y, *z;        /* device, offsets[n_sets] entries each */
    const float *nx, *ny, *nz;     /* device, same length, or all NULL */
    const int64_t *offsets;        /* host, n_sets + 1 */
    int32_t n_sets;
} fr_cloud;

/*
 * Lattice parameters.  Features are normalised to identity covariance
 * (Sec. 4.1): position / sigma[axis], and for feat == 6 also the normal /
 * sigma_n (the feature extension of Sec. 3.3, Eq. 8).  Values splatted per
 * observation point are [1, y] (Eq. 6) or [1, y, n_y] (Eq. 9).
 */
typedef struct {
    int32_t feat;          /* FR_FEAT_POS or FR_FEAT_POS_NORMAL */
    int32_t values;        /* FR_VAL_PT2PT, FR_VAL_PT2PL or their _M2 layouts */
    double sigma[3];       /* > 0 */
    double sigma_n;        /* > 0 when feat == 6 */
    int32_t splat;         /* FR_SPLAT_SORTED: bitwise deterministic; FR_SPLAT_ATOMIC: float atomics */
    int32_t reserved;      /* must be 0 */
} fr_lattice_params;

/*
 * Build the lattice of every set of `obs` (Sec. 3.2: built once per
 * observation when the variance is fixed; Sec. 4.2: splat of the
 * permutohedral filter, no blur).  Each observation point adds b_k * value to
 * the d+1 vertices of its enclosing simplex; occupancy counts incidences.
 * Normals are required when feat == 6 or values is FR_VAL_PT2PL(_M2).
 * Synchronises once with the stream (vertex counts size the tables).
 * A set with no points gets an empty lattice.  On success *out owns all
 * device memory of the lattice (charged to ctx).
 */
fr_status fr_lattice_build(fr_ctx *ctx, const fr_cloud *obs, const fr_lattice_params *params, void *stream,
                           fr_lattice **out);
fr_status fr_lattice_destroy(fr_lattice *lat);

/*
 * A lattice rebuilt in place (for loops that rebuild it every iteration, as
 * the optimised variance of Sec. 3.3 does; Sec. 3.1 notes that the index is
 * built once only while the variance is fixed).  fr_lattice_build_inplace
 * sizes every array once from `obs` with bounds that hold at any scale -- a
 * set of n points has at most (feat+1) n incidences, partial records and
 * vertices -- and builds the lattice at the scales of `params`, with the
 * position scale of set s replaced by sigma_set_h[s] (host, n_sets float64,
 * or NULL).  Synchronises; returns FR_EDEVICE if a table overflowed (not
 * seen at these bounds, not ruled out).  fr_lattice_rebuild rebuilds it from
 * the same `obs` (its device arrays must stay valid and unchanged) at new
 * per-set position scales (sigma_set_h as above, required): it only enqueues
 * kernels on `stream` -- no allocation, no host wait -- and its tables are
 * those fr_lattice_build would make at the same scales (the same slices,
 * bitwise with FR_SPLAT_SORTED).  A failed rebuild leaves the lattice invalid
 * and is reported by fr_sync_status (FR_EDEVICE) until a rebuild succeeds.
 * Memory: tables for (feat+1) vertices per observation point, several times
 * what fr_lattice_build allocates.  fr_lattice_stats and fr_lattice_export
 * are not available on such a lattice (FR_EINVAL); fr_lattice_destroy frees it.
 */
fr_status fr_lattice_build_inplace(fr_ctx *ctx, const fr_cloud *obs, const fr_lattice_params *params,
                                   const double *sigma_set_h, void *stream, fr_lattice **out);
fr_status fr_lattice_rebuild(fr_lattice *lat, const double *sigma_set_h, void *stream);

/* Vertex count, hash capacity (slots) and device bytes of set `set`; synchronises. */
fr_status fr_lattice_stats(const fr_lattice *lat, int32_t set, int64_t *n_vertices, int64_t *capacity,
                           int64_t *device_bytes);

/*
 * Copy set `set` of the lattice to host arrays, vertices in lexicographic key
 * order: keys_h n_v x d int32 (the first d of the d+1 lattice coordinates),
 * occ_h n_v int32, vals_h n_v x V binary32.  Synchronises.
 */
fr_status fr_lattice_export(const fr_lattice *lat, int32_t set, int32_t *keys_h, int32_t *occ_h, float *vals_h);

/*
 * Splat records of the lattice's build (all sets): *incidences (host) = D N,
 * one per observation point and simplex vertex (Eq. 14's splat), and
 * *partial_records (host) = the runs of shared vertices the build inserted,
 * sorted and summed in their place (neighbouring points of a scan share most
 * vertices; descriptor lattices insert every incidence).
 */
fr_status fr_lattice_records(const fr_lattice *lat, int64_t *incidences, int64_t *partial_records);

/*
 * Device time of the build's stages, from HIP events on the build stream
 * (host, 4 doubles, ms; -1 where not measured): [0] embedding and partial
 * records, [1] insertion into the provisional tables and vertex numbering,
 * [2] the vertex values (radix sort and binary64 sums, or the atomic sums),
 * [3] the final bucketed tables.  The stages include the build's waits for
 * its sizes (the host round trips between them).
 */
fr_status fr_lattice_build_times(const fr_lattice *lat, double *stage_ms_h);

/*
 * Motion applied to model reference points before the E-step (Eq. 15,
 * x_i = T_i x_ref_i).  mats is device memory, one row-major [R | t] of 12
 * binary32 per segment.  FR_XF_RIGID: one matrix per set.  FR_XF_SEGMENTED:
 * seg_offsets (host, n_seg + 1) partitions the cloud's points into segments
 * that each lie inside one set (e.g. the rigid bodies of Sec. 5.1).
 * FR_XF_NONE: points are used as given.  The transform is evaluated in
 * binary32 as ((R0 x + R1 y) + R2 z) + t with no fused multiply-add; normals
 * are rotated the same way without t.
 */
typedef struct {
    int32_t kind;
    int32_t n_seg;
    const float *mats;
    const int64_t *seg_offsets;
} fr_xform;

/*
 * The uncustomised permutohedral filter (the cited Adams et al. method that
 * Sec. 4.2 customises; Sec. 3.1: with it the index depends on X and is rebuilt
 * every EM iteration).  fr_lattice_build_joint splats, per set, the
 * observation points with their values [1, y(, n_y)] together with the model
 * points moved by `xf` (FR_XF_NONE, or FR_XF_RIGID with one binary32 [R | t]
 * per set in device memory) with no value, so that every simplex the E-step
 * will read at those model points exists; occupancy counts the incidences of
 * both.  values must be FR_VAL_PT2PT or FR_VAL_PT2PL.  Synchronises like
 * fr_lattice_build.
 */
fr_status fr_lattice_build_joint(fr_ctx *ctx, const fr_cloud *obs, const fr_cloud *model_ref, const fr_xform *xf,
                                 const fr_lattice_params *params, void *stream, fr_lattice **out);

/*
 * Descriptor lattices (Sec. 3.3 "Features", Eq. 8): the kernel is
 * N(f_x; f_y, sigma_f^2 I) over dim-dimensional descriptors (dim = 8, 16 or
 * 32) instead of positions.  fr_lattice_build_features splats, per set, the
 * values [1, y] of the observation points (positions from `obs`) at their
 * descriptors obs_feat (device, N x dim row-major binary32, rows 16-byte
 * aligned), with scale factors sqrt(2/3)(dim+1) / (sigma_f sqrt((i+1)(i+2)))
 * (no blur, as fr_lattice_build).  fr_estep_features slices it at the model
 * descriptors model_feat (device, M x dim) -> m0 (device, M) and m1 (device,
 * 3M channel-major); only the set offsets of `model_ref` are used, since the
 * descriptors do not depend on the pose.  Build synchronises like
 * fr_lattice_build; FR_EINVAL for other dimensions.
 */
fr_status fr_lattice_build_features(fr_ctx *ctx, const fr_cloud *obs, const float *obs_feat, int32_t dim,
                                    double sigma_f, int32_t splat, void *stream, fr_lattice **out);
fr_status fr_estep_features(const fr_lattice *lat, const fr_cloud *model_ref, const float *model_feat, float *m0,
                            float *m1, void *stream);

/*
 * Blur of the uncustomised filter, in place: for each lattice direction j =
 * 0..d in turn (every coordinate +1, coordinate j -d), every vertex takes 1/2
 * its value plus 1/4 of each of its two neighbours along j from the previous
 * pass (absent neighbours read as 0, none are created); the result is scaled
 * by 1 / (1 + 2^-d) (the published filter's output scale).  A slice of the
 * blurred lattice (fr_estep) is the filter's output.  Table and exported
 * vertex values are replaced; keys and occupancy are kept.  FR_EINVAL for the
 * |y|^2 layouts.
 */
fr_status fr_lattice_blur(fr_lattice *lat, void *stream);

/*
 * E-step through the lattice (Eq. 6, Eq. 9 via Eq. 11): for every model point
 * of every set, slice the set's lattice at the transformed point's feature:
 *   m0[i]           = sum_k b_k value_0[v_k]                  (device, M)
 *   m1[c * M + i]   = sum_k b_k value_(1+c)[v_k], c = 0..2    (device, 3M)
 *   nsum[c * M + i] = sum_k b_k value_(4+c)[v_k]              (device, 3M; NULL unless V = 7)
 * where M = offsets[n_sets] of `model_ref`; vertices absent from the lattice
 * contribute nothing, so points without support get m0 = 0.  `model_ref`
 * must have the lattice's n_sets, and normals when the lattice has feat 6.
 */
fr_status fr_estep(const fr_lattice *lat, const fr_cloud *model_ref, const fr_xform *xf, float *m0, float *m1,
                   float *nsum, void *stream);

/*
 * fr_estep on a lattice built with a |y|^2 channel (values FR_VAL_PT2PT_M2 or
 * FR_VAL_PT2PL_M2): also m2 (device, M float32), the second moment about the
 * target t_i = M1_i / M0_i,
 *   m2_i = sum_k K(x_i, y_k) |y_k - t_i|^2  (= M2_i - |M1_i|^2 / M0_i, 0 without support),
 * which the variance update of Sec. 3.3 (optimised variance, the closed form
 * of the Coherent Point Drift M-step) needs next to M0 and M1.  Each vertex
 * keeps the scatter of its observations about its own mean, so the result
 * is not a difference of |y|^2-sized binary32 numbers.  nsum is written for
 * FR_VAL_PT2PL_M2.  fr_lattice_export returns that per-vertex scatter as the
 * last channel.  FR_EINVAL on a lattice without the channel.
 */
fr_status fr_estep_m2(const fr_lattice *lat, const fr_cloud *model_ref, const fr_xform *xf, float *m0, float *m1,
                      float *nsum, float *m2, void *stream);

/*
 * Diagnostic: number of distinct lattice vertices the E-step of set `set`
 * reads (found by at least one lookup).  Synchronises.
 */
fr_status fr_estep_touched(const fr_lattice *lat, const fr_cloud *model_ref, const fr_xform *xf, int32_t set,
                           int64_t *n_touched);

/*
 * M-step terms (Eq. 7 point-to-point, Eq. 10 point-to-plane) linearised in
 * the twist of each point's transform (Eq. 16, with d x / d omega = -[x]_x) and
 * reduced per segment into the Gauss-Newton normal equations (Eq. 17-18):
 *   w_i = m0_i / (m0_i + c), target = m1_i / m0_i, n_i = nsum_i / m0_i,
 *   pt2pt: r = (x_i - target) / sigma,        J = [-[x_i]_x, I] / sigma
 *   pt2pl: r = n_i . (x_i - target) / sigma,  J = [x_i x n_i, n_i] / sigma
 *   jtj[s] = sum w J^T J (21 doubles: upper triangle, row-major),
 *   jtr[s] = sum w J^T r (6 doubles), stats[s] = [sum w, sum w r^2, n_support, sum m0]
 * over the points of segment s (device outputs).  Points with m0 = 0 are
 * skipped.  x_i is the model point moved by `xf` (segments of `xf` are the
 * reduction segments; FR_XF_NONE/RIGID reduce per set).  Per-point terms are
 * accumulated in binary32 per tile, tiles are summed in binary64 in a fixed
 * order (bitwise reproducible).  c_per_set (host, n_sets) overrides c.
 */
typedef struct {
    int32_t residual;      /* FR_PT2PT or FR_PT2PL */
    int32_t normalize_n;   /* 1: use n_i / |n_i| */
    double c;              /* outlier constant of Eq. 7 in the units of the lattice sums, >= 0 */
    double sigma;          /* residual scale (Sigma^-1/2 of Eq. 7), > 0 */
    const double *c_per_set;
} fr_mstep_params;

fr_status fr_mstep_reduce(const fr_cloud *model_ref, const fr_xform *xf, const float *m0, const float *m1,
                          const float *nsum, const fr_mstep_params *params, double *jtj, double *jtr,
                          double *stats, void *stream);

/*
 * fr_mstep_reduce for callers that cannot allocate device memory (code that
 * must not call hipMalloc: tight serving loops, harnesses that forbid it).
 * Same arguments, kernels and results (bitwise) as fr_mstep_reduce; it
 * allocates nothing.  Its tile map and per-tile partial rows live in a
 * device array of FR_NOALLOC_SCRATCH_BYTES inside the library, one per GPU,
 * held until the process ends.  A call needs 20 bytes per segment plus
 * 128 bytes per 1024 points (about 67 M points in one segment); a larger one
 * fails with FR_EINVAL before anything is enqueued.  Every call on a GPU
 * shares that GPU's array: calls that overlap on one GPU (from several host
 * threads, or on several streams) race and must be serialised by the caller.
 * Synchronises `stream` before returning, like fr_mstep_reduce.
 */
#define FR_NOALLOC_SCRATCH_BYTES (8 << 20)
fr_status fr_mstep_reduce_noalloc(const fr_cloud *model_ref, const fr_xform *xf, const float *m0, const float *m1,
                                  const float *nsum, const fr_mstep_params *params, double *jtj, double *jtr,
                                  double *stats, void *stream);

/*
 * Rigid Gauss-Newton update on the device in binary64 (Eq. 17 and the
 * left-multiplied update of Eq. 16): for each of n sets,
 *   dzeta = -A^-1 b (Cholesky), T <- Exp(dzeta) T,
 * poses (device, n x 16 row-major float64) are updated in place, mats
 * (device, n x 12) receive the binary32 [R | t], twist_norm (device, n x 2)
 * receives |omega| and |v| of dzeta, status (device, n int32) receives FR_OK
 * or FR_EDEGENERATE (pose left unchanged) per set.  A is taken as singular
 * when a Cholesky pivot is at most 1e-4 times its diagonal entry (a
 * numerical-rank test: A is summed from binary32 terms over tiles of 1024
 * points, whose rounding reaches about 6.1e-5 of the diagonal scale, so a
 * smaller pivot cannot be told from zero -- e.g. every supported point on one
 * plane under point-to-plane, rank 3).  Sets with active[i] == 0 are skipped
 * (active may be NULL).
 */
fr_status fr_solve_rigid(int32_t n, const double *jtj, const double *jtr, double *poses, float *mats,
                         double *twist_norm, int32_t *status, const int32_t *active, void *stream);

/* Registration parameters (Sec. 3.1 EM loop; termination on a small twist, Sec. 6.1). */
typedef struct {
    fr_lattice_params lattice;
    int32_t residual;      /* FR_PT2PT or FR_PT2PL */
    int32_t max_iters;     /* EM iterations (exact count with FR_FIXED_ITERS) */
    double w;              /* outlier ratio of Eq. 4 in [0, 1); c derived per set as w/(1-w) N/M
                              (Eq. 7) times the mass of the lattice kernel over feature space,
                              (3/2)^(d/2) / sqrt(d+1) times the product of the d feature widths
                              (sigma_x sigma_y sigma_z, and sigma_n^3 when feat == 6; divided by
                              1 + 2^-d with FR_BLURRED): Eq. 7's c is taken against Gaussian PDFs
                              of unit mass, M0 sums this kernel instead */
    double c_override;     /* >= 0: use this c for every set instead; < 0: derive from w */
    double twist_tol;      /* stop a set when |omega| and |v| of its step are below this */
    int32_t flags;         /* FR_FIXED_ITERS | FR_PROFILE_EVENTS | FR_FUSED (slice and reduction in one
                              kernel: same terms, binary32 partial sums taken in another order) |
                              FR_BLURRED (the uncustomised filter: every iteration builds the joint
                              lattice of the observation and the moved model and blurs it, as
                              fr_lattice_build_joint + fr_lattice_blur; not with FR_FUSED) |
                              FR_GRAPH (capture the kernels of up to 32 iterations -- 4, between
                              the convergence checks, without FR_FIXED_ITERS -- into a HIP graph
                              on a stream of the context and replay it; same results bitwise;
                              ignored with FR_PROFILE_EVENTS or FR_BLURRED.  The capture costs
                              more than it saves when the call is short) */
    int32_t kinematics;    /* FR_KIN_RIGID */
} fr_register_params;

typedef struct {
    int32_t iterations;        /* EM iterations run */
    int32_t n_degenerate;      /* sets that stopped on a degenerate system */
    double build_ms;           /* lattice build (host clock) */
    double em_ms;              /* EM loop incl. final copy (host clock) */
    double estep_ms;           /* sum of E-step kernel times (FR_PROFILE_EVENTS) */
    double mstep_ms;           /* sum of reduce + solve times (FR_PROFILE_EVENTS) */
    int64_t estep_launches;
    int32_t solver_iters;      /* node graph: conjugate-gradient iterations of the last solve */
    double solver_residual;    /* node graph: relative residual of the last solve */
} fr_report;

/*
 * Rigid registration of every set of `model_ref` onto the same set of `obs`
 * (Sec. 3.1 with the rigid kinematics of Sec. 5): build the lattices once,
 * then per EM iteration E-step, reduce and FP64 solve/update, all on the
 * device.  theta_inout_h (host, n_sets x 16 float64, row-major 4x4) holds the
 * start poses and receives the results; status_h (host, n_sets int32, may be
 * NULL) receives each set's status.  Synchronous.  Returns FR_EDEGENERATE if
 * any set degenerated (its pose is left at the last good value).
 */
fr_status fr_register(fr_ctx *ctx, const fr_cloud *model_ref, const fr_cloud *obs, const fr_register_params *params,
                      double *theta_inout_h, int32_t *status_h, fr_report *report_h, void *stream);

/*
 * Rigid registration with an optimised isotropic variance per set (Sec. 3.3,
 * Sigma_xyz = sigma^2 I as a decision variable; Tab. 1 "updated sigma").  The
 * closed form is that of the Coherent Point Drift M-step: with the posterior
 * P_ik = K(x_i, y_k) / (M0_i + c) of Eq. 4-5,
 *   var = sum_ik P_ik |x_i - y_k|^2 / (3 sum_ik P_ik)
 *       = sum_i w_i (|x_i - t_i|^2 + m2_i / M0_i) / (3 sum_i w_i)
 * (t_i and m2_i as in fr_estep_m2), evaluated at the pose the E-step used.  sigma here is the lattice scale s,
 * as in fr_lattice_params; the splat/slice kernel of scale s has per-axis
 * variance s^2 / 4, so the Gaussian it stands for has variance s^2 / 4 and the
 * update is s^2 <- 4 var, floored at sigma_min.  The lattice depends on s, so
 * every iteration rebuilds it from `obs` with each set's s (the normal
 * features keep lattice.sigma_n), and c of Eq. 7 follows s as in fr_register.
 * params->lattice.values must be FR_VAL_PT2PT_M2 for FR_PT2PT and
 * FR_VAL_PT2PL_M2 for FR_PT2PL; lattice.sigma is not used (it must still be
 * valid); FR_FUSED is rejected.  sigma_inout_h (host, n_sets float64, > 0)
 * holds the start scales and receives the scale each set would use next.
 * theta_inout_h, status_h, report_h and the return value as fr_register
 * (with FR_PROFILE_EVENTS report_h->build_ms sums the rebuilds' device time
 * and em_ms excludes it; without, build_ms is 0).  The lattice is rebuilt in
 * place in storage sized once from `obs`, and the scale update, lattice scale
 * factors and outlier constants stay on the device, so the host waits once
 * every 4 iterations; a rebuild whose tables overflow is caught there and its
 * 4 iterations are run again with a build sized on the host.
 */
fr_status fr_register_sigma(fr_ctx *ctx, const fr_cloud *model_ref, const fr_cloud *obs,
                            const fr_register_params *params, double sigma_min, double *theta_inout_h,
                            double *sigma_inout_h, int32_t *status_h, fr_report *report_h, void *stream);

/*
 * Rigid registration by descriptors alone (Sec. 3.3 "Features" with Eq. 8;
 * the global registration of Sec. 6.3): the kernel does not involve the pose,
 * so one E-step (fr_estep_features) fixes the targets M1/M0 and the weights
 * M0/(M0 + c), c = w/(1-w) N/M (3/2)^(dim/2) / sqrt(dim+1) sigma_f^dim (the
 * kernel mass rule of fr_register_params.w; c_override if >= 0), and each EM iteration is one point-to-point Gauss-Newton step toward
 * them (Eq. 17; residual scale 1).  params: residual FR_PT2PT, lattice.splat
 * selects the splat (the other lattice fields are not used), max_iters, w,
 * c_override, twist_tol, FR_FIXED_ITERS and
 * FR_PROFILE_EVENTS as fr_register; FR_FUSED and FR_BLURRED are rejected.
 * theta_inout_h, status_h, report_h and the return value as fr_register.
 */
fr_status fr_register_features(fr_ctx *ctx, const fr_cloud *model_ref, const float *model_feat, const fr_cloud *obs,
                               const float *obs_feat, int32_t dim, double sigma_f, const fr_register_params *params,
                               double *theta_inout_h, int32_t *status_h, fr_report *report_h, void *stream);

/*
 * Kinematic tree of an articulated model (Sec. 5.1).  Body b (0 <= b < n_bodies)
 * hangs from parent[b] < b (-1 = world) at the joint origin origin[3b..3b+2]
 * given in the parent's frame, and owns the revolute DOFs
 * [dof_offset[b], dof_offset[b+1]).  Its frame is
 *   T_b = T_parent . Trans(origin_b) . Rot(axis_k0, theta_k0) . Rot(axis_k1, theta_k1) ...
 * with each unit axis[3k..3k+2] given in the frame left by the preceding
 * rotations.  All arrays are host memory; at most 128 bodies and 64 DOFs.
 */
typedef struct {
    int32_t n_bodies;
    const int32_t *parent;
    const int32_t *dof_offset;
    const double *origin;
    const double *axis;
} fr_kinematic_tree;

/*
 * Articulated Gauss-Newton step on the device in binary64 (Eq. 19-20, the
 * assembly and solve of Alg. 1): given per-body sums jtj (device, n_bodies x 21, upper triangle
 * row-major) and jtr (device, n_bodies x 6) from fr_mstep_reduce segmented by
 * body at the current angles, builds the spatial velocity Jacobian of every
 * body by forward kinematics (DOF k moves the bodies below its joint with the
 * twist (w_k, q_k x w_k) of its world axis w_k through the joint point q_k),
 * assembles A = sum_b J_b^T jtj_b J_b and b = sum_b J_b^T jtr_b, solves
 * A dtheta = -b by Cholesky (a DOF whose row of A is zero -- it moves no
 * supported point -- is held at its value; a pivot at most 1e-4 of its
 * diagonal entry is refused as in fr_solve_rigid), updates theta (device, n_dof) in place and writes
 * the binary32 [R | t] of every body at the new angles to mats (device,
 * n_bodies x 12).  status (device int32, may be NULL) receives FR_OK or
 * FR_EDEGENERATE (theta unchanged).  jtj/jtr may be NULL for forward
 * kinematics only (theta unchanged, mats written).
 */
fr_status fr_articulated_step(fr_ctx *ctx, const fr_kinematic_tree *tree, const double *jtj, const double *jtr,
                              double *theta, float *mats, int32_t *status, void *stream);

/*
 * Articulated registration (Sec. 3.1 with the kinematics of Sec. 5.1) of one
 * model (one set, points grouped by body: body_offsets host, n_bodies + 1)
 * onto one observation set.  theta_inout_h (host, n_dof) holds the start
 * angles and receives the result.  Synchronous; FR_EDEGENERATE if the
 * normal equations degenerate (theta left at the last good value).
 */
fr_status fr_register_articulated(fr_ctx *ctx, const fr_cloud *model_ref, const int64_t *body_offsets,
                                  const fr_cloud *obs, const fr_kinematic_tree *tree,
                                  const fr_register_params *params, double *theta_inout_h, fr_report *report_h,
                                  void *stream);

/*
 * Node graph of a deformable model (Sec. 5.2, Eq. 21): nodes {p_k, T_k}; model
 * point i moves by the normalised dual-quaternion blend of the transforms of
 * its 4 skinning nodes skin_idx[4i..4i+3] with weights skin_w[4i..4i+3] (sum 1).
 * The point twist is the blend of the node twists, so the node normal
 * equations collect w_ki w_li J_i^T J_i per node pair; lambda weights the
 * regulariser sum over directed edges (j, k) of |(T_j p_k - T_k p_k) / sigma|^2.
 * All arrays are host memory.
 */
typedef struct {
    int32_t n_nodes;
    const double *nodes;        /* 3 x n_nodes reference node positions */
    const int32_t *skin_idx;    /* 4 x M */
    const float *skin_w;        /* 4 x M */
    int32_t n_edges;
    const int32_t *edges;       /* 2 x n_edges */
    double lambda;              /* >= 0 */
} fr_node_graph;

/*
 * Node-graph M-step (Sec. 5.2, Eq. 21: the Gauss-Newton normal equations of
 * Eq. 17 in the node twists) at one EM iteration: x is the model moved by the
 * node graph (one set, device; normals not used), m0/m1/nsum the E-step at it
 * (fr_estep with FR_XF_NONE; nsum for FR_PT2PL only), node_T_h (host,
 * n_nodes x 16 row-major) the node transforms the regulariser is linearised
 * at, params->c/sigma/residual as in fr_mstep_reduce (normalize_n must be 0,
 * c_per_set is not used).  The system is block sparse: a 6x6 block for every
 * node pair (k <= l) that shares a model point's skinning or an edge, and for
 * every node with itself, ordered by k * n_nodes + l.  Block (k, l) holds
 *   sum_i w_ki w_li J_i^T J_i / sigma^2 (+ the regulariser's lambda J^T J terms)
 * and rhs node k holds sum_i w_ki J_i^T r_i / sigma^2 + lambda J_k^T e, with
 * J_i, r_i the rigid twist terms of fr_mstep_reduce at x_i and e the edge
 * residual of fr_node_graph.  With blocks == NULL only *n_blocks is written;
 * otherwise block_nodes_h (host, 2 x n_blocks int32: k, l), blocks (device,
 * n_blocks x 36 float64, row-major, rows of node k) and rhs (device, 6 n_nodes
 * float64) receive the system.  Synchronises.
 */
fr_status fr_mstep_reduce_nodes(fr_ctx *ctx, const fr_cloud *x, const float *m0, const float *m1, const float *nsum,
                                const fr_node_graph *graph, const double *node_T_h, const fr_mstep_params *params,
                                int64_t *n_blocks, int32_t *block_nodes_h, double *blocks, double *rhs, void *stream);

/*
 * Node-graph registration of one model set onto one observation set: per EM
 * iteration the model is warped on the device (binary64 blend, binary32
 * output), sliced, reduced into the block-sparse node system, which is solved
 * by block-Jacobi preconditioned conjugate gradients in binary64 (relative
 * residual 1e-10, at most 2000 iterations), and every node is updated by
 * T_k <- Exp(dzeta_k) T_k.  node_T_inout_h (host, n_nodes x 16 row-major)
 * holds the start transforms and receives the result.  Synchronous.
 * FR_EDEGENERATE when a node's diagonal block is singular (a node that skins
 * no supported point and has no regulariser edge, or lambda = 0); the nodes
 * keep the transforms of the iteration before.
 */
fr_status fr_register_nodegraph(fr_ctx *ctx, const fr_cloud *model_ref, const fr_cloud *obs, const fr_node_graph *graph,
                                const fr_register_params *params, double *node_T_inout_h, fr_report *report_h,
                                void *stream);

/*
 * Serving engine: continuous batching of rigid registrations (the EM loop of
 * Sec. 3.1 with the rigid twist M-step of Sec. 5, one request = one
 * observation/model pair).  An engine keeps up to max_slots registrations
 * resident at once -- each slot holds its model points in the engine's point
 * arena, the lattice of its observation (built once, Sec. 3.2), its binary64
 * pose and binary32 transform -- and fr_engine_step runs one EM iteration of
 * any subset of the occupied slots with one E-step, one reduction and one
 * solve launch.  Requests of different sizes therefore share every launch,
 * and a slot joins or leaves between two steps.
 *
 * Streams: every step, read and release is enqueued on the engine's `stream`
 * (given at creation).  Lattice builds run on a stream of the engine's own,
 * so a build overlaps the steps already queued; a step that includes a newly
 * admitted slot waits for that slot's build on the device, not on the host.
 * Results are bitwise those of fr_register on the same pair alone (sorted
 * splat; same iteration count, twist tolerance and FR_FUSED setting).  A slot
 * stops on the device (twist_tol, or a degenerate step): steps that still list
 * it leave it unchanged, so the host may learn of the stop a few steps late
 * (fr_engine_read) without changing the result.  One host thread at a time per engine.
 */
typedef struct fr_engine fr_engine;

typedef struct {
    fr_lattice_params lattice;  /* shared by every request */
    int32_t residual;           /* FR_PT2PT or FR_PT2PL */
    int32_t max_slots;          /* 1 .. 4096 registrations resident at once */
    int64_t arena_points;       /* model points resident at once (>= 1) */
    double w;                   /* outlier ratio of Eq. 4; c per request as in fr_register_params */
    double c_override;          /* >= 0: this c for every request; < 0: derive from w */
    int32_t flags;              /* FR_FUSED: as fr_register with FR_FUSED;
                                   FR_GRAPH: the first step captures, for each of the engine's pinned plan
                                   buffers, one HIP graph -- the plan's copy to the device, a persistent
                                   E-step and reduction (a fixed grid that walks the plan's tiles, their
                                   count read on the device), the final sums and the solve -- and every step
                                   then fills a plan buffer and replays its graph, whatever the resident
                                   set; same results bitwise (not with FR_FUSED) */
    int32_t reserved;           /* must be 0 */
    double twist_tol;           /* > 0: a slot stops (its later steps do nothing) after a step whose
                                   |omega| and |v| are both below it (Sec. 6.1); <= 0: only a degenerate
                                   step stops a slot */
} fr_engine_params;

/* Create an engine; allocates the point arena (52 bytes per point for d = 6
 * point-to-plane) and the per-slot state from ctx's budget. */
fr_status fr_engine_create(fr_ctx *ctx, const fr_engine_params *params, void *stream, fr_engine **out);
/* Wait for all queued work and free everything the engine holds. */
fr_status fr_engine_destroy(fr_engine *eng);

/*
 * Admit n requests: request j is set j of model_ref (device, normals when
 * feat == 6) and set j of obs; it occupies slot slots_h[j] (must be free) and
 * arena points [arena_begin_h[j], arena_begin_h[j] + M_j) (inside the arena,
 * disjoint from every occupied slot's range and from each other), and starts
 * at pose T0_h[16 j .. 16 j + 15] (host, row-major 4x4).  The n lattices are
 * built in one build on the engine's build stream (the host waits for that
 * build only); the model points are copied into the arena, on the device,
 * once the steps queued so far have finished.  obs may be reused when the
 * call returns; model_ref must stay valid until the engine stream has
 * completed a later fr_engine_step or fr_engine_read (both wait for every
 * earlier admission on the device).
 */
fr_status fr_engine_admit(fr_engine *eng, int32_t n, const int32_t *slots_h, const fr_cloud *model_ref,
                          const fr_cloud *obs, const int64_t *arena_begin_h, const double *T0_h);

/* One EM iteration (E-step, reduction, binary64 solve and pose update) of the
 * n occupied slots listed in slots_h (host), enqueued on the engine stream. */
fr_status fr_engine_step(fr_engine *eng, int32_t n, const int32_t *slots_h);

/* Progress of a slot since its admission. */
typedef struct {
    int32_t status;       /* FR_OK or FR_EDEGENERATE of its last solve, or FR_ERANGE if one of its
                             E-steps saw a lattice coordinate out of range */
    int32_t iterations;   /* EM iterations (solves) the slot has run */
    int32_t stopped;      /* 1: the slot has stopped -- its last step was degenerate or below
                             twist_tol -- and later steps leave it unchanged */
    int32_t reserved;
} fr_slot_state;

/* Enqueue a copy of every slot's pose (poses_h: max_slots x 16 float64,
 * row-major, or NULL to skip) and state (state_h: max_slots entries) into host
 * memory; pinned host memory makes it asynchronous.  The state of a slot is
 * reset when it is admitted. */
fr_status fr_engine_read(fr_engine *eng, double *poses_h, fr_slot_state *state_h);

/* Free n slots.  Their arena ranges may be admitted again at once; a lattice
 * is freed (ordered after the queued steps) when its last slot is released. */
fr_status fr_engine_release(fr_engine *eng, int32_t n, const int32_t *slots_h);

/* Return (and clear) a device fault latched in `lat` by earlier async calls; synchronises. */
fr_status fr_sync_status(const fr_lattice *lat);

/*
 * Roofline probes (measurement only; their buffers are charged to ctx).
 *  fr_probe_atomics: n_atomics binary32 atomic adds without return value, each
 *    to its own word of a power-of-two table of table_bytes (at least
 *    4 n_atomics bytes); scattered != 0 puts neighbouring threads on
 *    different lines (one line per atomic), scattered == 0 on neighbouring
 *    words (a wave's 64 atomics on two lines): atomics per second (*per_s,
 *    host).  The two uncontended ceilings of the atomic splat's vertex sums.
 *  fr_probe_lines: 16-byte loads, lanes_per_line (1, 2, 4 or 8) lanes of a
 *    wave reading the same 128-byte line, lines drawn at random from a table
 *    of table_bytes (L2-resident when small, HBM when large): 128-byte line
 *    accesses per second (*lines_per_s, host).  A hash lookup with one lane
 *    per key costs one line access per 16-byte load.
 * Both time a few launches with HIP events on `stream` and wait for them.
 */
fr_status fr_probe_atomics(fr_ctx *ctx, int64_t n_atomics, size_t table_bytes, int32_t scattered, double *per_s,
                           void *stream);
fr_status fr_probe_lines(fr_ctx *ctx, int32_t lanes_per_line, size_t table_bytes, double *lines_per_s, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* FILTERREG_H */
