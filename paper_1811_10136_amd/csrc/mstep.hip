// M-step reduction (Eq. 7 / Eq. 10 linearised in the twist, Eq. 16, summed
// into the Gauss-Newton normal equations of Eq. 17-18).
//
// k_reduce: one block per tile of 1024 model points of one segment.  Each
// thread accumulates w J^T J (21 upper entries), w J^T r (6) and 4 statistics
// in binary32 registers over its points; the block reduces the 32 values with
// halving lane exchanges and an LDS exchange between its 4 waves and writes
// one partial row per tile.  k_reduce_final: one block per segment sums its
// tiles' partial rows in binary64 in a fixed order (bitwise reproducible)
// and applies the 1/sigma^2 of the residual scaling.
#include "fr_internal.h"
#include "fr_mstep.h"

namespace fr {

constexpr int kRedThreads = 256;   // a tile of 1024 points: 4 per thread
struct ReduceArgs {
    const float *x, *y, *z;
    const float *mats;
    TileMap tm;
    const float *m0, *m1, *ns, *m2;
    int64_t M;
    const float *seg_c;
    float *partials;
    int normalize_n;
    const int32_t *active;        // per set: 0 = stopped, its tiles do nothing (or NULL)
};

template <int RES, bool XF, bool M2>
__device__ __forceinline__ void reduce_tile(const ReduceArgs &a, int32_t t, float (&part)[kRedThreads / 64][kRedStride])
{
    const int32_t s = tile_segment(a.tm, t);
    if (a.active != nullptr && a.active[a.tm.seg_set[s]] == 0) return;   // no partial row: the set is not solved
    const int64_t start = a.tm.seg_off[s] + (int64_t)(t - a.tm.seg_tile[s]) * a.tm.tile;
    const int64_t stop = min(start + (int64_t)a.tm.tile, a.tm.seg_end[s]);
    const float c = a.seg_c[s];
    float m[12];
    if constexpr (XF) {
#pragma unroll
        for (int j = 0; j < 12; ++j) m[j] = a.mats[12 * s + j];
    }
    float acc[kRedVals];
#pragma unroll
    for (int j = 0; j < kRedVals; ++j) acc[j] = 0.0f;

    for (int64_t i = start + threadIdx.x; i < stop; i += kRedThreads) {
        float x = __builtin_nontemporal_load(a.x + i);
        float y = __builtin_nontemporal_load(a.y + i);
        float z = __builtin_nontemporal_load(a.z + i);
        if constexpr (XF) {
            float ox, oy, oz;
            xform_point(m, x, y, z, ox, oy, oz);
            x = ox;
            y = oy;
            z = oz;
        }
        const float m0 = __builtin_nontemporal_load(a.m0 + i);
        if (!(m0 > 0.0f)) continue;
        float nsx = 0.0f, nsy = 0.0f, nsz = 0.0f;
        if constexpr (RES == FR_PT2PL) {
            nsx = __builtin_nontemporal_load(a.ns + i);
            nsy = __builtin_nontemporal_load(a.ns + a.M + i);
            nsz = __builtin_nontemporal_load(a.ns + 2 * a.M + i);
        }
        mstep_point<RES, M2>(acc, x, y, z, m0, __builtin_nontemporal_load(a.m1 + i),
                             __builtin_nontemporal_load(a.m1 + a.M + i),
                             __builtin_nontemporal_load(a.m1 + 2 * a.M + i), nsx, nsy, nsz, c, a.normalize_n,
                             M2 ? __builtin_nontemporal_load(a.m2 + i) : 0.0f);
    }
    block_partials(acc, &part[0][0], kRedStride, a.partials + (size_t)t * kRedStride);
}

template <int RES, bool XF, bool M2, bool PERSIST>
__global__ void __launch_bounds__(kRedThreads) k_reduce(ReduceArgs a)
{
    __shared__ float part[kRedThreads / 64][kRedStride];
    if constexpr (PERSIST) {
        for_each_tile_persistent(a.tm, [&](int32_t t) {
            __syncthreads();   // the previous tile's partial row has been read out of LDS
            reduce_tile<RES, XF, M2>(a, t, part);
        });
    } else {
        const int32_t t = logical_tile(a.tm);
        if (t >= a.tm.n_tiles) return;
        reduce_tile<RES, XF, M2>(a, t, part);
    }
}

// One block per segment.  Thread (g, j) of the 32 x 32 threads sums value j
// of tiles g, g + 32, g + 64, ... in binary64 -- four interleaved chains
// (tiles g + 128 k + 32 u for chain u), added in chain order at the end, so
// four loads are in flight per thread -- and the 32 group sums are then added
// in group order: a fixed order, reproducible, and one wave reads two whole
// partial rows per load.
constexpr int kFinalGroups = 32;
constexpr int kFinalChains = 4;

__global__ void __launch_bounds__(kFinalGroups * kRedVals) k_reduce_final(TileMap tm, const float *partials,
                                                                          double inv_s2, double *jtj, double *jtr,
                                                                          double *stats, double *var_stat)
{
    __shared__ double group_sum[kFinalGroups][kRedVals];
    const int32_t s = blockIdx.x;
    const int j = threadIdx.x % kRedVals;
    const int g = threadIdx.x / kRedVals;
    const int32_t t0 = tm.seg_tile[s], t1 = tm.seg_tile[s + 1];
    double acc[kFinalChains];
#pragma unroll
    for (int u = 0; u < kFinalChains; ++u) acc[u] = 0.0;
    constexpr int32_t kStep = kFinalGroups * kFinalChains;
    for (int32_t t = t0 + g; t < t1; t += kStep) {
        float v[kFinalChains];
#pragma unroll
        for (int u = 0; u < kFinalChains; ++u) {
            const int32_t tu = t + u * kFinalGroups;
            v[u] = tu < t1 ? partials[(size_t)tu * kRedStride + j] : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < kFinalChains; ++u) acc[u] += (double)v[u];
    }
    double sum = 0.0;
#pragma unroll
    for (int u = 0; u < kFinalChains; ++u) sum += acc[u];
    group_sum[g][j] = sum;
    __syncthreads();
    if (threadIdx.x < kRedVals) {
        const int jj = threadIdx.x;
        double tot = 0.0;
#pragma unroll
        for (int q = 0; q < kFinalGroups; ++q) tot += group_sum[q][jj];
        if (jj < 21) jtj[(size_t)s * 21 + jj] = tot * inv_s2;
        else if (jj < 27) jtr[(size_t)s * 6 + (jj - 21)] = tot * inv_s2;
        else if (jj < 31) stats[(size_t)s * 4 + (jj - 27)] = (jj == 28) ? tot * inv_s2 : tot;
        else if (var_stat != nullptr) var_stat[s] = tot;
    }
}

size_t reduce_partials_floats(const Plan &plan) { return (size_t)(plan.n_tiles + 1) * kRedStride; }

fr_status launch_reduce_final(const Plan &plan, const float *partials, double sigma, double *jtj, double *jtr,
                              double *stats, hipStream_t st, double *var_stat)
{
    if (plan.n_seg == 0) return FR_OK;
    k_reduce_final<<<plan.n_seg, kFinalGroups * kRedVals, 0, st>>>(plan.tm, partials, 1.0 / (sigma * sigma), jtj,
                                                                     jtr, stats, var_stat);
    FR_HIP(hipGetLastError());
    return FR_OK;
}

template <int RES, bool M2>
static void launch_reduce_rm(const ReduceArgs &a, bool xf, int grid, int persist_grid, hipStream_t st)
{
    if (persist_grid > 0) {
        if (xf) k_reduce<RES, true, M2, true><<<persist_grid, kRedThreads, 0, st>>>(a);
        else k_reduce<RES, false, M2, true><<<persist_grid, kRedThreads, 0, st>>>(a);
    } else {
        if (xf) k_reduce<RES, true, M2, false><<<grid, kRedThreads, 0, st>>>(a);
        else k_reduce<RES, false, M2, false><<<grid, kRedThreads, 0, st>>>(a);
    }
}

int reduce_persistent_grid(int residual)
{
    int per_cu = 0, dev = 0, cus = 0;
    const void *f = residual == FR_PT2PL ? reinterpret_cast<const void *>(k_reduce<FR_PT2PL, true, false, true>)
                                         : reinterpret_cast<const void *>(k_reduce<FR_PT2PT, true, false, true>);
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, kRedThreads, 0);
    (void)hipGetLastError();
    const int g = per_cu * cus / 8 * 8;
    return g > 8 ? g : 8;
}

fr_status launch_reduce(const fr_cloud *model, const Plan &plan, int xf_kind, const float *mats, const float *m0,
                        const float *m1, const float *nsum, int residual, int normalize_n, double sigma, double *jtj,
                        double *jtr, double *stats, float *partials, hipStream_t st, const float *m2,
                        double *var_stat, const int32_t *active)
{
    if (plan.n_seg == 0) return FR_OK;
    ReduceArgs a{};
    a.active = active;
    a.x = model->x;
    a.y = model->y;
    a.z = model->z;
    a.mats = mats;
    a.tm = plan.tm;
    a.m0 = m0;
    a.m1 = m1;
    a.ns = nsum;
    a.m2 = m2;
    a.M = cloud_points(model);
    a.seg_c = plan.seg_c;
    a.partials = partials;
    a.normalize_n = normalize_n;
    const bool xf = xf_kind != FR_XF_NONE;
    if (plan.grid > 0 || plan.persist_grid > 0) {
        const int pg = plan.persist_grid;
        if (residual == FR_PT2PT) {
            if (m2) launch_reduce_rm<FR_PT2PT, true>(a, xf, plan.grid, pg, st);
            else launch_reduce_rm<FR_PT2PT, false>(a, xf, plan.grid, pg, st);
        } else {
            if (m2) launch_reduce_rm<FR_PT2PL, true>(a, xf, plan.grid, pg, st);
            else launch_reduce_rm<FR_PT2PL, false>(a, xf, plan.grid, pg, st);
        }
        FR_HIP(hipGetLastError());
    }
    return launch_reduce_final(plan, partials, sigma, jtj, jtr, stats, st, var_stat);
}

}  // namespace fr
