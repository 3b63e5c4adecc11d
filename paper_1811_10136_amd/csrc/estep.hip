// E-step slice (Eq. 6, Eq. 9 through the general Gaussian transform Eq. 11):
// one thread per model point moves the point (Eq. 15), embeds its feature in
// the lattice, looks the D = d + 1 vertices of its simplex up in the set's
// cuckoo table (all 2D candidate key slots are read at once, then the value
// slots of the vertices found) and accumulates b_k * [1, y, n_y] into M0, M1
// and the normal sum.
//
// Memory behaviour: model points and outputs are streamed once (structure of
// arrays, coalesced, non-temporal so they do not evict the table from L2);
// the table of the set being sliced is read through L2, and the logical tile
// order keeps one set's tiles on one XCD.
#include "fr_internal.h"
#include "fr_mstep.h"

namespace fr {

struct EstepArgs {
    const float *x, *y, *z, *nx, *ny, *nz;
    const float *mats;            // per segment [R | t], or NULL for no transform
    const SetTable *sets;
    TileMap tm;
    float k[8];
    float *m0, *m1, *ns;          // outputs (m1/ns channel-major, stride M)
    int64_t M;
    uint32_t *touched;            // optional: per-slot "was found" flags
    int32_t *err;                 // range-error flag: one word, or one per segment
    int32_t err_stride;           // 0: one word; 1: err[segment]
    // fused slice + reduction only
    const float *seg_c;           // outlier constant per segment
    float *partials;              // one row of kRedStride floats per tile
    int32_t normalize_n;
};

template <typename T>
__device__ __forceinline__ T ld_stream(const T *p) { return __builtin_nontemporal_load(p); }
template <typename T>
__device__ __forceinline__ void st_stream(T *p, T v) { __builtin_nontemporal_store(v, p); }

// Each thread slices kEstepPP consecutive points of its segment.  Model
// points arrive in scan order, so neighbouring points mostly share simplex
// vertices (three in four for depth frames): a vertex whose key equals one of
// the previous point's takes that point's table slot and lookup result, and
// only the remaining vertices are hashed into the table.  The block first
// stages its tile of points through LDS so that the HBM reads stay coalesced.
// The arithmetic of every point -- its embedding, its weights and the order
// of its sum over vertices -- is the same as for a point sliced on its own.
template <int d>
struct Stage {
    static constexpr int NIN = d == 6 ? 6 : 3;
    static constexpr int ROW = 256 * (kEstepPP + 1);   // padded: point j of the tile sits at j + j / PP
    float v[NIN][ROW];
};

// Slice the tile of segment s starting at point `first` (n_here points);
// emit(i, x, y, z, acc) receives every point's index, moved position and
// slice sums.
template <int d, int V, bool XF, class Emit>
__device__ __forceinline__ void slice_tile(const EstepArgs &a, int32_t s, int64_t first, int32_t n_here,
                                           Stage<d> &sg, Emit &&emit)
{
    constexpr int D = d + 1;
    constexpr int KW = KeyWords<d>::value;
    constexpr int PP = kEstepPP;
    constexpr int NIN = Stage<d>::NIN;
    auto &stage = sg.v;
    const SetTable st = a.sets[a.tm.seg_set[s]];

    const float *src[6] = {a.x, a.y, a.z, a.nx, a.ny, a.nz};
#pragma unroll
    for (int q = 0; q < PP; ++q) {
        const int32_t j = q * 256 + (int32_t)threadIdx.x;
        if (j < n_here) {
#pragma unroll
            for (int c = 0; c < NIN; ++c) stage[c][j + j / PP] = ld_stream(src[c] + first + j);
        }
    }
    __syncthreads();

    float m[12];
    if constexpr (XF) {
#pragma unroll
        for (int j = 0; j < 12; ++j) m[j] = a.mats[12 * s + j];
    }
    float kk[d];
#pragma unroll
    for (int j = 0; j < d; ++j) kk[j] = a.k[j];

    uint64_t pk[D][KW];          // previous point's vertex keys (kKeyEmpty: none)
    uint32_t pslot[D];           // and their value-slot byte offsets
    uint32_t pfound = 0;         // bit v: previous vertex v is in the table
#pragma unroll
    for (int v = 0; v < D; ++v) {
#pragma unroll
        for (int w = 0; w < KW; ++w) pk[v][w] = kKeyEmpty;
        pslot[v] = 0;
    }
    constexpr uint32_t VB = (uint32_t)(ValPad<V>::value * sizeof(float));
    const int32_t base = (int32_t)threadIdx.x * PP;
    for (int q = 0; q < PP; ++q) {
        const int32_t j = base + q;
        if (j >= n_here) break;
        const int32_t sj = j + j / PP;
        float p[d];
        if constexpr (XF) {
            xform_point(m, stage[0][sj], stage[1][sj], stage[2][sj], p[0], p[1], p[2]);
            if constexpr (d == 6) xform_normal(m, stage[3][sj], stage[4][sj], stage[5][sj], p[3], p[4], p[5]);
        } else {
#pragma unroll
            for (int c = 0; c < d; ++c) p[c] = stage[c][sj];
        }
        uint64_t keys[D][KW];
        float b[D];
        if (!embed<d>(p, kk, keys, b)) atomicOr(a.err + a.err_stride * s, 1);

        // vertices shared with the previous point
        uint32_t slot[D];
        uint32_t found = 0, known = 0;
#pragma unroll
        for (int v = 0; v < D; ++v) {
            slot[v] = 0;
#pragma unroll
            for (int u = 0; u < D; ++u) {
                const bool eq = key_equal<KW>(keys[v], pk[u]);
                slot[v] = eq ? pslot[u] : slot[v];
                found |= eq ? ((pfound >> u) & 1u) << v : 0u;
                known |= eq ? 1u << v : 0u;
            }
        }
        // the others through the table: both candidate key slots, read only by
        // lanes that need them
        uint32_t p1[D], p2[D];
        uint64_t ka[D][KW], kc[D][KW];
#pragma unroll
        for (int v = 0; v < D; ++v) {
            cuckoo_slots(hash_key<KW>(keys[v], st.seed), st.cap, p1[v], p2[v]);
#pragma unroll
            for (int w = 0; w < KW; ++w) {
                ka[v][w] = kKeyEmpty;
                kc[v][w] = kKeyEmpty;
            }
            if (!((known >> v) & 1u)) {
                load_key<KW>(st.keys, p1[v], ka[v]);
                load_key<KW>(st.keys, p2[v], kc[v]);
            }
        }
#pragma unroll
        for (int v = 0; v < D; ++v) {
            if (!((known >> v) & 1u)) {
                const bool in1 = key_equal<KW>(ka[v], keys[v]);
                const bool in2 = key_equal<KW>(kc[v], keys[v]);
                slot[v] = (in1 ? p1[v] : p2[v]) * VB;
                found |= (in1 || in2) ? 1u << v : 0u;
            }
        }
        float acc[V];
#pragma unroll
        for (int c = 0; c < V; ++c) acc[c] = 0.0f;
#pragma unroll
        for (int v = 0; v < D; ++v) {
            const bool f = (found >> v) & 1u;
            const float w = f ? b[v] : 0.0f;
            u32x4 q0 = {0u, 0u, 0u, 0u}, q1 = q0;
            if (f) {
                q0 = load_at<u32x4>(st.vals, slot[v]);
                if constexpr (V > 4) q1 = load_at<u32x4>(st.vals, slot[v] + 16u);
            }
            const float val[8] = {__uint_as_float(q0.x), __uint_as_float(q0.y), __uint_as_float(q0.z),
                                  __uint_as_float(q0.w), __uint_as_float(q1.x), __uint_as_float(q1.y),
                                  __uint_as_float(q1.z), __uint_as_float(q1.w)};
#pragma unroll
            for (int c = 0; c < V; ++c) acc[c] = fmaf(w, val[c], acc[c]);
        }
        emit(first + j, p[0], p[1], p[2], acc);
#pragma unroll
        for (int v = 0; v < D; ++v) {
#pragma unroll
            for (int w = 0; w < KW; ++w) pk[v][w] = keys[v][w];
            pslot[v] = slot[v];
        }
        pfound = found;
    }
}

template <int d, int V, bool XF>
__global__ void __launch_bounds__(256) k_estep(EstepArgs a)
{
    __shared__ Stage<d> sg;
    const int32_t t = logical_tile(a.tm);
    if (t >= a.tm.n_tiles) return;
    const int32_t s = tile_segment(a.tm, t);
    const int64_t first = a.tm.seg_off[s] + (int64_t)(t - a.tm.seg_tile[s]) * a.tm.tile;
    const int32_t n_here = (int32_t)min((int64_t)a.tm.tile, a.tm.seg_end[s] - first);
    slice_tile<d, V, XF>(a, s, first, n_here, sg, [&](int64_t i, float, float, float, const float (&acc)[V]) {
        a.m0[i] = acc[0];
        a.m1[i] = acc[1];
        a.m1[a.M + i] = acc[2];
        a.m1[2 * a.M + i] = acc[3];
        if constexpr (V == 7) {
            if (a.ns != nullptr) {
                a.ns[i] = acc[4];
                a.ns[a.M + i] = acc[5];
                a.ns[2 * a.M + i] = acc[6];
            }
        }
    });
}

// Fused slice + reduction: every point's M-step terms (Eq. 7 / Eq. 10 in the
// twist of Eq. 16) are accumulated right after its slice, and the block writes
// one partial row of the normal equations per tile; M0, M1 and N never leave
// the chip.
template <int d, int V, bool XF, int RES>
__global__ void __launch_bounds__(256) k_estep_fused(EstepArgs a)
{
    __shared__ Stage<d> sg;
    __shared__ float part[4][kRedStride];
    const int32_t t = logical_tile(a.tm);
    if (t >= a.tm.n_tiles) return;
    const int32_t s = tile_segment(a.tm, t);
    const int64_t first = a.tm.seg_off[s] + (int64_t)(t - a.tm.seg_tile[s]) * a.tm.tile;
    const int32_t n_here = (int32_t)min((int64_t)a.tm.tile, a.tm.seg_end[s] - first);
    const float c = a.seg_c[s];
    float red[kRedVals];
#pragma unroll
    for (int j = 0; j < kRedVals; ++j) red[j] = 0.0f;
    slice_tile<d, V, XF>(a, s, first, n_here, sg, [&](int64_t, float x, float y, float z, const float (&acc)[V]) {
        if constexpr (RES == FR_PT2PL)
            mstep_point<RES>(red, x, y, z, acc[0], acc[1], acc[2], acc[3], acc[4], acc[5], acc[6], c, a.normalize_n);
        else
            mstep_point<RES>(red, x, y, z, acc[0], acc[1], acc[2], acc[3], 0.0f, 0.0f, 0.0f, c, a.normalize_n);
    });
    block_partials(red, part, a.partials + (size_t)t * kRedStride);
}

// Diagnostic twin of k_estep: marks every table slot a lookup finds.
template <int d, int V, bool XF>
__global__ void __launch_bounds__(256) k_estep_touch(EstepArgs a)
{
    constexpr int D = d + 1;
    constexpr int KW = KeyWords<d>::value;
    const int32_t t = logical_tile(a.tm);
    if (t >= a.tm.n_tiles) return;
    const int32_t s = tile_segment(a.tm, t);
    const SetTable st = a.sets[a.tm.seg_set[s]];
    const int64_t first = a.tm.seg_off[s] + (int64_t)(t - a.tm.seg_tile[s]) * a.tm.tile;
    for (int q = 0; q < kEstepPP; ++q) {
        const int64_t i = first + q * 256 + threadIdx.x;
        if (i >= a.tm.seg_end[s]) break;
        float p[d];
        if constexpr (XF) {
            float m[12];
#pragma unroll
            for (int j = 0; j < 12; ++j) m[j] = a.mats[12 * s + j];
            xform_point(m, a.x[i], a.y[i], a.z[i], p[0], p[1], p[2]);
            if constexpr (d == 6) xform_normal(m, a.nx[i], a.ny[i], a.nz[i], p[3], p[4], p[5]);
        } else {
            p[0] = a.x[i];
            p[1] = a.y[i];
            p[2] = a.z[i];
            if constexpr (d == 6) {
                p[3] = a.nx[i];
                p[4] = a.ny[i];
                p[5] = a.nz[i];
            }
        }
        float kk[d];
#pragma unroll
        for (int j = 0; j < d; ++j) kk[j] = a.k[j];
        uint64_t keys[D][KW];
        float b[D];
        embed<d>(p, kk, keys, b);
#pragma unroll
        for (int v = 0; v < D; ++v) {
            const int64_t slot = find_slot<KW>(st.keys, st, keys[v]);
            if (slot >= 0) a.touched[st.slot_base + slot] = 1u;
        }
    }
}

template <int d, int V>
static void launch_dv(const EstepArgs &a, bool xf, bool touch, int grid, hipStream_t st)
{
    if (touch) {
        if (xf) k_estep_touch<d, V, true><<<grid, 256, 0, st>>>(a);
        else k_estep_touch<d, V, false><<<grid, 256, 0, st>>>(a);
    } else {
        if (xf) k_estep<d, V, true><<<grid, 256, 0, st>>>(a);
        else k_estep<d, V, false><<<grid, 256, 0, st>>>(a);
    }
}

fr_status launch_estep_sets(int d, int V, const float *k, const SetTable *sets, int32_t *err, int32_t err_stride,
                            const fr_cloud *model, int64_t M, const Plan &plan, int xf_kind, const float *mats,
                            float *m0, float *m1, float *nsum, uint32_t *touched, hipStream_t st)
{
    if (plan.grid == 0) return FR_OK;
    EstepArgs a{};
    a.x = model->x;
    a.y = model->y;
    a.z = model->z;
    a.nx = model->nx;
    a.ny = model->ny;
    a.nz = model->nz;
    a.mats = mats;
    a.sets = sets;
    a.tm = plan.tm;
    for (int j = 0; j < 8; ++j) a.k[j] = k[j];
    a.m0 = m0;
    a.m1 = m1;
    a.ns = nsum;
    a.M = M;
    a.touched = touched;
    a.err = err;
    a.err_stride = err_stride;
    const bool xf = xf_kind != FR_XF_NONE;
    const bool touch = touched != nullptr;
    if (d == 3 && V == 4) launch_dv<3, 4>(a, xf, touch, plan.grid, st);
    else if (d == 3 && V == 7) launch_dv<3, 7>(a, xf, touch, plan.grid, st);
    else if (d == 6 && V == 4) launch_dv<6, 4>(a, xf, touch, plan.grid, st);
    else if (d == 6 && V == 7) launch_dv<6, 7>(a, xf, touch, plan.grid, st);
    else {
        set_error("fr_estep: unsupported lattice d=%d V=%d", d, V);
        return FR_EINVAL;
    }
    FR_HIP(hipGetLastError());
    return FR_OK;
}

template <int d, int V>
static void launch_fused_dv(const EstepArgs &a, int residual, int grid, hipStream_t st)
{
    if constexpr (V == 7) {
        if (residual == FR_PT2PL) {
            k_estep_fused<d, V, true, FR_PT2PL><<<grid, 256, 0, st>>>(a);
            return;
        }
    }
    k_estep_fused<d, V, true, FR_PT2PT><<<grid, 256, 0, st>>>(a);
}

fr_status launch_estep_fused(int d, int V, const float *k, const SetTable *sets, int32_t *err, int32_t err_stride,
                             const fr_cloud *model, const Plan &plan, const float *mats, int residual,
                             int normalize_n, float *partials, hipStream_t st)
{
    if (plan.grid == 0) return FR_OK;
    if (residual == FR_PT2PL && V != 7) {
        set_error("fused E-step: point-to-plane needs V = 7");
        return FR_EINVAL;
    }
    EstepArgs a{};
    a.x = model->x;
    a.y = model->y;
    a.z = model->z;
    a.nx = model->nx;
    a.ny = model->ny;
    a.nz = model->nz;
    a.mats = mats;
    a.sets = sets;
    a.tm = plan.tm;
    for (int j = 0; j < 8; ++j) a.k[j] = k[j];
    a.M = cloud_points(model);
    a.err = err;
    a.err_stride = err_stride;
    a.seg_c = plan.seg_c;
    a.partials = partials;
    a.normalize_n = normalize_n;
    if (d == 3 && V == 4) launch_fused_dv<3, 4>(a, residual, plan.grid, st);
    else if (d == 3 && V == 7) launch_fused_dv<3, 7>(a, residual, plan.grid, st);
    else if (d == 6 && V == 4) launch_fused_dv<6, 4>(a, residual, plan.grid, st);
    else if (d == 6 && V == 7) launch_fused_dv<6, 7>(a, residual, plan.grid, st);
    else {
        set_error("fused E-step: unsupported lattice d=%d V=%d", d, V);
        return FR_EINVAL;
    }
    FR_HIP(hipGetLastError());
    return FR_OK;
}

fr_status launch_estep(const fr_lattice *lat, const fr_cloud *model, const Plan &plan, int xf_kind, const float *mats,
                       float *m0, float *m1, float *nsum, uint32_t *touched, hipStream_t st)
{
    return launch_estep_sets(lat->d, lat->V, lat->k, lat->sets_d, lat->err_d, 0, model, cloud_points(model), plan,
                             xf_kind, mats, m0, m1, nsum, touched, st);
}

}  // namespace fr
