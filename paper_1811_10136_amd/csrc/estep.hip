// E-step slice (Eq. 6, Eq. 9 through the general Gaussian transform Eq. 11):
// one thread per model point moves the point (Eq. 15), embeds its feature in
// the lattice, looks the D = d + 1 vertices of its simplex up in the set's
// bucketed cuckoo table (the first buckets of all D vertices at once, second
// buckets where needed, then the values of the vertices found, from the lines
// just read) and accumulates b_k * [1, y, n_y] into M0, M1 and the normal sum.
//
// Memory behaviour: model points and outputs are streamed once (structure of
// arrays, coalesced, non-temporal so they do not evict the table from L2);
// the table of the set being sliced is read through L2, and the logical tile
// order keeps one set's tiles on one XCD.
#include <algorithm>
#include <cstdlib>

#include "fr_internal.h"
#include "fr_mstep.h"

namespace fr {

struct EstepArgs {
    const float *x, *y, *z, *nx, *ny, *nz;
    const float *mats;            // per segment [R | t], or NULL for no transform
    const SetTable *sets;
    TileMap tm;
    float *m0, *m1, *ns;          // outputs (m1/ns channel-major, stride M)
    float *m2;                    // output sum b |y|^2 (value layouts with that channel), or NULL
    int64_t M;
    uint32_t *touched;            // optional: per-slot "was found" flags
    int32_t *err;                 // range-error flag: one word, or one per segment
    int32_t err_stride;           // 0: one word; 1: err[segment]
    const int32_t *active;        // per set: 0 = the set has stopped, its tiles do nothing (or NULL)
    // fused slice + reduction only
    const float *seg_c;           // outlier constant per segment
    float *partials;              // one row of kRedStride floats per tile
    int32_t normalize_n;
};

template <typename T>
__device__ __forceinline__ T ld_stream(const T *p) { return __builtin_nontemporal_load(p); }
template <typename T>
__device__ __forceinline__ void st_stream(T *p, T v) { __builtin_nontemporal_store(v, p); }

// Slice model point i of segment s: its moved position (x[0..2]) and the
// slice sums acc = sum_k b_k [1, y, n_y] over the vertices found.
template <int d, int V, bool XF>
__device__ __forceinline__ void slice_point(const EstepArgs &a, int32_t s, int64_t i, const SetTable &st,
                                            float (&x)[3], float (&acc)[V])
{
    constexpr int D = d + 1;
    constexpr int KW = KeyWords<d>::value;
    float px = ld_stream(a.x + i), py = ld_stream(a.y + i), pz = ld_stream(a.z + i);
    float p[d];
    if constexpr (XF) {
        float m[12];
#pragma unroll
        for (int j = 0; j < 12; ++j) m[j] = a.mats[12 * s + j];
        xform_point(m, px, py, pz, p[0], p[1], p[2]);
        if constexpr (d == 6) {
            xform_normal(m, ld_stream(a.nx + i), ld_stream(a.ny + i), ld_stream(a.nz + i), p[3], p[4], p[5]);
        }
    } else {
        p[0] = px;
        p[1] = py;
        p[2] = pz;
        if constexpr (d == 6) {
            p[3] = ld_stream(a.nx + i);
            p[4] = ld_stream(a.ny + i);
            p[5] = ld_stream(a.nz + i);
        }
    }
    float kk[d];
#pragma unroll
    for (int j = 0; j < d; ++j) kk[j] = st.k[j];

    uint64_t keys[D][KW];
    float b[D];
    if (!embed<d>(p, kk, keys, b)) atomicOr(a.err + a.err_stride * s, 1);

#pragma unroll
    for (int c = 0; c < V; ++c) acc[c] = 0.0f;
    slice_simplex<KW, V, D>(st, keys, b, acc);
    x[0] = p[0];
    x[1] = p[1];
    x[2] = p[2];
}

template <int d, int V, bool XF>
__device__ __forceinline__ void estep_tile(const EstepArgs &a, int32_t t)
{
    const int32_t s = tile_segment(a.tm, t);
    if (a.active != nullptr && a.active[a.tm.seg_set[s]] == 0) return;
    const int64_t i = a.tm.seg_off[s] + (int64_t)(t - a.tm.seg_tile[s]) * a.tm.tile + threadIdx.x;
    if (i >= a.tm.seg_end[s]) return;
    const SetTable st = a.sets[a.tm.seg_set[s]];
    float x[3], acc[V];
    slice_point<d, V, XF>(a, s, i, st, x, acc);
    st_stream(a.m0 + i, acc[0]);
    st_stream(a.m1 + i, acc[1]);
    st_stream(a.m1 + a.M + i, acc[2]);
    st_stream(a.m1 + 2 * a.M + i, acc[3]);
    if constexpr (ValLayout<V>::normals) {
        if (a.ns != nullptr) {
            st_stream(a.ns + i, acc[4]);
            st_stream(a.ns + a.M + i, acc[5]);
            st_stream(a.ns + 2 * a.M + i, acc[6]);
        }
    }
    if constexpr (ValLayout<V>::m2) {
        if (a.m2 != nullptr) st_stream(a.m2 + i, acc[V - 1]);
    }
}

template <int d, int V, bool XF, bool PERSIST>
__global__ void __launch_bounds__(256) k_estep(EstepArgs a)
{
    if constexpr (PERSIST) {
        for_each_tile_persistent(a.tm, [&](int32_t t) { estep_tile<d, V, XF>(a, t); });
    } else {
        const int32_t t = logical_tile(a.tm);
        if (t >= a.tm.n_tiles) return;
        estep_tile<d, V, XF>(a, t);
    }
}

// ---------------------------------------------------------------------------
// Slice with the lookups of a wave shared (k_estep_dedup).
//
// On a 640 x 480 depth frame about one vertex in four of a wave's 64 points
// starts a run of shared vertices (wave_runs).  A wave therefore
//   1. embeds its 64 points and finds its runs;
//   2. looks each run's key up once (64 runs per round, one per lane, with the
//      same bucket probes as the plain slice) and parks the values in LDS;
//   3. gives every point the values of its D vertices from LDS and sums them
//      in vertex order m = 0..d with the plain slice's arithmetic, so the
//      result is bitwise that of k_estep.
// A wave with more runs than its LDS holds (points in no particular order)
// takes the plain slice.  LDS is private to each wave: no barrier across the
// workgroup.
// ---------------------------------------------------------------------------
template <int d, int V> struct DedupGeom {
    static constexpr int D = d + 1;
    static constexpr int KW = KeyWords<d>::value;
    static constexpr int VP = ValPad<V>::value;
    static constexpr int key_bytes = WaveKeys<d>::bytes;        // keys of the wave, [lane][class]
    static constexpr int by_vals = key_bytes / (VP * 4) / 64 * 64;
    static constexpr int C0 = by_vals < 64 * D ? by_vals : 64 * D;
    static constexpr int C = C0 < 192 ? C0 : 192;               // runs a wave can hold (entries fit a byte)
    static constexpr int NL = C / 64;                           // lookups per lane
    static constexpr int region = key_bytes > C * VP * 4 ? key_bytes : C * VP * 4;
    static constexpr int src_off = region;                      // u16 per entry: (lane << 3) | class
    static constexpr int ent_off = src_off + 2 * C;             // u8 per (lane, vertex): its entry
    static constexpr int fnd_off = ent_off + 64 * D;            // u8 per entry: found
    static constexpr int wave_bytes = (fnd_off + C + 15) / 16 * 16;
    static_assert(NL >= 1, "a wave must hold at least one round of lookups");
};

// The lookups of a wave's distinct keys by lane pairs.  Lanes 2i and 2i+1
// take entries e = 64 j + 32 h + i (h = 0, 1) and read the two slots of the
// entry's bucket side by side, lane parity = slot: one load instruction
// covers 32 buckets, two lanes per line, where a lane reading both key slots
// and then the values of its own key touches a line per lane and piece.  The
// lane whose slot holds the key (told by a lane swap) tells the pair which slot
// to read the values from; as in lookup_keys the second bucket is read only
// when the first is full without the key.  Three dependent rounds: first-
// bucket keys; second-bucket keys (skipped by a wave none of whose keys needs
// them); the values, from the bucket that holds each key.  Keys are read from
// the wave's LDS key region (src[e] names the lane and class that hold entry
// e's key), which the values overwrite once every key read is done.  fnd[e] =
// 1 found; absent keys get zero values.
template <int d, int V, int NL>
__device__ __forceinline__ void lookup_pairs(const SetTable &st, const char *kreg, const uint16_t *src, int32_t U,
                                             float *vreg, uint8_t *fnd)
{
    constexpr int D = d + 1;
    constexpr int KW = KeyWords<d>::value;
    constexpr int KB = 8 * KW;
    using SG = SlotGeom<KW, V>;
    constexpr int VP = ValPad<V>::value;
    constexpr int VU = VP / 4;   // 16-byte value pieces of a slot
    constexpr int NE = 2 * NL;   // entries per lane pair
    static_assert(KB <= 16 && 2 * SG::bytes <= 128 && VU <= 2, "a key fits one piece, a bucket one line");
    const int lane = (int)(threadIdx.x & 63u);
    const uint32_t half = (uint32_t)(lane & 1), pi = (uint32_t)(lane >> 1);
    const uint32_t nb = st.cap >> 1;
    const uint64_t *kb = st.keys;
    auto entry = [&](int q) { return (int32_t)(64 * (q >> 1) + 32 * (q & 1) + (int)pi); };
    auto key_of = [&](int32_t e, uint64_t(&k)[KW]) {
        const uint32_t sc = src[e];
        lds_get_key<KW>(kreg + ((int32_t)(sc >> 3) * D + (int32_t)(sc & 7u)) * KB, k);
    };
    auto matches = [&](const u32x4 &qv, const uint64_t(&k)[KW]) {
        bool m = qv.x == (uint32_t)k[0] && qv.y == (uint32_t)(k[0] >> 32);
        if constexpr (KW == 2) m = m && qv.z == (uint32_t)k[1] && qv.w == (uint32_t)(k[1] >> 32);
        return m;
    };
    auto taken = [](const u32x4 &qv) { return !(qv.x == 0xFFFFFFFFu && qv.y == 0xFFFFFFFFu); };
    // the other lane of the pair: quad_perm [1, 0, 3, 2] (every lane runs it)
    auto swap_pair = [](uint32_t v) { return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false); };
    auto partner = [&](bool b) { return swap_pair(b ? 1u : 0u) != 0u; };
    const u32x4 zero = {0u, 0u, 0u, 0u};

    // bucket offsets: of entries q = 2j and 2j+1 each lane of a pair hashes
    // the one of its parity and takes the other from its partner
    uint32_t bo1[NE], bo2[NE];
#pragma unroll
    for (int j = 0; j < NL; ++j) {
        const int32_t e = entry(2 * j + (int)half);
        uint32_t o1 = 0u, o2 = 0u;
        if (e < U) {
            uint64_t k[KW];
            key_of(e, k);
            uint32_t b1, b2;
            key_buckets<KW>(k, st.seed, nb, b1, b2);
            o1 = b1 * SG::bucket;
            o2 = b2 * SG::bucket;
        }
        const uint32_t p1 = swap_pair(o1), p2 = swap_pair(o2);
        bo1[2 * j] = half ? p1 : o1;
        bo1[2 * j + 1] = half ? o1 : p1;
        bo2[2 * j] = half ? p2 : o2;
        bo2[2 * j + 1] = half ? o2 : p2;
    }
    // round 1: each lane's slot key of the first buckets
    u32x4 kq[NE];
#pragma unroll
    for (int q = 0; q < NE; ++q) {
        kq[q] = zero;
        if (entry(q) < U) kq[q] = load_at<u32x4>(kb, bo1[q] + half * SG::bytes);
    }
    // state: bit 0 found, bit 1 the slot holding the key, bit 2 second bucket next, bit 3 found there
    uint32_t state[NE];
#pragma unroll
    for (int q = 0; q < NE; ++q) {
        const int32_t e = entry(q);
        const bool live = e < U;
        uint64_t k[KW];
#pragma unroll
        for (int w = 0; w < KW; ++w) k[w] = 0;
        if (live) key_of(e, k);
        const bool eq = live && matches(kq[q], k);
        const bool tk = live && taken(kq[q]);
        const bool pe = partner(eq), pt = partner(tk);
        const bool found = eq || pe;
        const uint32_t slot = eq ? half : half ^ 1u;
        const bool second = live && !found && tk && pt;
        state[q] = (found ? 1u : 0u) | (slot << 1) | (second ? 4u : 0u);
    }
    // round 2 (if a wave's key needs it): each lane's slot key of the second buckets
    bool any_second = false;
#pragma unroll
    for (int q = 0; q < NE; ++q) any_second = any_second || (state[q] & 4u) != 0u;
    if (__ballot(any_second) != 0ull) {
#pragma unroll
        for (int q = 0; q < NE; ++q) {
            kq[q] = zero;
            if (state[q] & 4u) kq[q] = load_at<u32x4>(kb, bo2[q] + half * SG::bytes);
        }
#pragma unroll
        for (int q = 0; q < NE; ++q) {
            const bool sec = (state[q] & 4u) != 0u;
            uint64_t k[KW];
#pragma unroll
            for (int w = 0; w < KW; ++w) k[w] = 0;
            if (sec) key_of(entry(q), k);
            const bool eq = sec && matches(kq[q], k);
            const bool pe = partner(eq);
            if (sec) state[q] = (eq || pe) ? (1u | ((eq ? half : half ^ 1u) << 1) | 8u) : 0u;
        }
    }
    // round 3: the values of every key found, from the bucket that holds it
#pragma unroll
    for (int q = 0; q < NE; ++q) {
        kq[q] = zero;
        if ((state[q] & 1u) && half < (uint32_t)VU)
            kq[q] = load_at<u32x4>(kb, ((state[q] & 8u) ? bo2[q] : bo1[q]) + ((state[q] >> 1) & 1u) * SG::bytes +
                                           SG::val_off + 16u * half);
    }
    wave_sync();   // every key read: the values may overwrite the key region now
#pragma unroll
    for (int q = 0; q < NE; ++q) {
        const int32_t e = entry(q);
        if (e < U) {
            if (half < (uint32_t)VU)
                reinterpret_cast<float4 *>(vreg + e * VP)[half] = make_float4(
                    __uint_as_float(kq[q].x), __uint_as_float(kq[q].y), __uint_as_float(kq[q].z),
                    __uint_as_float(kq[q].w));
            if (half == 0u) fnd[e] = (state[q] & 1u) ? 1 : 0;
        }
    }
}

// Slice of a wave's points with shared lookups.  live: the lane has a point
// (dead lanes form the tail of the wave).  Returns acc for live lanes.
template <int d, int V>
__device__ __forceinline__ void slice_wave_dedup(const SetTable &st, const uint64_t (&keys)[d + 1][KeyWords<d>::value],
                                                 const float (&b)[d + 1], int32_t sdiv, bool live, char *lds,
                                                 float (&acc)[V])
{
    using G = DedupGeom<d, V>;
    using SG = SlotGeom<KeyWords<d>::value, V>;
    constexpr int D = G::D;
    constexpr int KW = G::KW;
    constexpr int VP = G::VP;
    const int lane = (int)(threadIdx.x & 63u);
    const int32_t r = class_shift<D>(sdiv);
    char *kreg = lds;
    uint16_t *src = reinterpret_cast<uint16_t *>(lds + G::src_off);
    uint8_t *ent = reinterpret_cast<uint8_t *>(lds + G::ent_off) + lane * D;
    uint8_t *fnd = reinterpret_cast<uint8_t *>(lds + G::fnd_off);
    constexpr int KB = 8 * KW;
    const int32_t U = wave_runs<d>(keys, r, live, kreg, src, G::C, ent, nullptr);
#pragma unroll
    for (int c = 0; c < V; ++c) acc[c] = 0.0f;
    if (U > G::C) {
        // more runs than the wave's LDS holds (points in no particular order)
        if (!live) return;
        if constexpr (ValLayout<V>::m2) {
            slice_simplex<KW, V, D>(st, keys, b, acc);
        } else {
            // one vertex at a time (few registers), the plain slice's arithmetic and order
#pragma unroll
            for (int m = 0; m < D; ++m) {
                const int64_t slot = find_slot<KW, V>(st, keys[m]);
                float val[8];
#pragma unroll
                for (int c = 0; c < 8; ++c) val[c] = 0.0f;
                if (slot >= 0) load_vals<V>(st.vals, (uint32_t)slot * SG::bytes, val);
                const float w = slot >= 0 ? b[m] : 0.0f;
#pragma unroll
                for (int c = 0; c < V; ++c) acc[c] = fmaf(w, val[c], acc[c]);
            }
        }
        return;
    }
    wave_sync();
    // look every distinct key up once
    float *vreg = reinterpret_cast<float *>(lds);
    lookup_pairs<d, V, G::NL>(st, kreg, src, U, vreg, fnd);
    wave_sync();
    if (!live) return;
    if constexpr (ValLayout<V>::m2) {
        float val[D][8];
        bool fv[D];
#pragma unroll
        for (int m = 0; m < D; ++m) {
            const int32_t e = ent[m];
            fv[m] = fnd[e] != 0;
            const float4 *q = reinterpret_cast<const float4 *>(vreg + e * VP);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const float4 f = (h < VP / 4) ? q[h] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                val[m][4 * h] = f.x;
                val[m][4 * h + 1] = f.y;
                val[m][4 * h + 2] = f.z;
                val[m][4 * h + 3] = f.w;
            }
        }
        accumulate_simplex<V, D>(val, fv, b, acc);
    } else {
        // the sums of accumulate_simplex, one vertex at a time from LDS
#pragma unroll
        for (int m = 0; m < D; ++m) {
            const int32_t e = ent[m];
            const float w = fnd[e] != 0 ? b[m] : 0.0f;
            const float4 *q = reinterpret_cast<const float4 *>(vreg + e * VP);
            float val[8];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const float4 f = (h < VP / 4) ? q[h] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                val[4 * h] = f.x;
                val[4 * h + 1] = f.y;
                val[4 * h + 2] = f.z;
                val[4 * h + 3] = f.w;
            }
#pragma unroll
            for (int c = 0; c < V; ++c) acc[c] = fmaf(w, val[c], acc[c]);
        }
    }
}

// The shared-lookup slice of this thread's point of tile t (segment s): x =
// the moved point, acc = its sums; false for a lane without a point.  The
// lanes of a wave with a point in the segment all take part (run detection
// and lookups are wave-wide); a wave wholly past the segment does nothing.
template <int d, int V, bool XF>
__device__ __forceinline__ bool dedup_point(const EstepArgs &a, int32_t s, int32_t t, char *lds, int64_t &i,
                                            float (&x)[3], float (&acc)[V])
{
    constexpr int D = d + 1;
    constexpr int KW = KeyWords<d>::value;
    const int64_t i0 = a.tm.seg_off[s] + (int64_t)(t - a.tm.seg_tile[s]) * a.tm.tile;
    i = i0 + threadIdx.x;
    const int64_t end = a.tm.seg_end[s];
    if (i0 + (int64_t)(threadIdx.x & ~63u) >= end) return false;   // the whole wave is past the segment
    const bool live = i < end;
    const SetTable st = a.sets[a.tm.seg_set[s]];
    float p[d];
#pragma unroll
    for (int j = 0; j < d; ++j) p[j] = 0.0f;
    if (live) {
        const float px = ld_stream(a.x + i), py = ld_stream(a.y + i), pz = ld_stream(a.z + i);
        if constexpr (XF) {
            float m[12];
#pragma unroll
            for (int j = 0; j < 12; ++j) m[j] = a.mats[12 * s + j];
            xform_point(m, px, py, pz, p[0], p[1], p[2]);
            if constexpr (d == 6)
                xform_normal(m, ld_stream(a.nx + i), ld_stream(a.ny + i), ld_stream(a.nz + i), p[3], p[4], p[5]);
        } else {
            p[0] = px;
            p[1] = py;
            p[2] = pz;
            if constexpr (d == 6) {
                p[3] = ld_stream(a.nx + i);
                p[4] = ld_stream(a.ny + i);
                p[5] = ld_stream(a.nz + i);
            }
        }
    }
    float kk[d];
#pragma unroll
    for (int j = 0; j < d; ++j) kk[j] = st.k[j];
    uint64_t keys[D][KW];
    float b[D];
    int32_t sdiv = 0;
    const bool ok = embed<d>(p, kk, keys, b, &sdiv);
    if (live && !ok) atomicOr(a.err + a.err_stride * s, 1);
    slice_wave_dedup<d, V>(st, keys, b, sdiv, live, lds, acc);
    x[0] = p[0];
    x[1] = p[1];
    x[2] = p[2];
    return live;
}

template <int d, int V, bool XF>
__device__ __forceinline__ void estep_dedup_tile(const EstepArgs &a, int32_t t, char *lds)
{
    const int32_t s = tile_segment(a.tm, t);
    if (a.active != nullptr && a.active[a.tm.seg_set[s]] == 0) return;
    int64_t i = 0;
    float x[3], acc[V];
    if (!dedup_point<d, V, XF>(a, s, t, lds, i, x, acc)) return;
    st_stream(a.m0 + i, acc[0]);
    st_stream(a.m1 + i, acc[1]);
    st_stream(a.m1 + a.M + i, acc[2]);
    st_stream(a.m1 + 2 * a.M + i, acc[3]);
    if constexpr (ValLayout<V>::normals) {
        if (a.ns != nullptr) {
            st_stream(a.ns + i, acc[4]);
            st_stream(a.ns + a.M + i, acc[5]);
            st_stream(a.ns + 2 * a.M + i, acc[6]);
        }
    }
    if constexpr (ValLayout<V>::m2) {
        if (a.m2 != nullptr) st_stream(a.m2 + i, acc[V - 1]);
    }
}

template <int d, int V, bool XF, bool PERSIST>
__global__ void __launch_bounds__(256) k_estep_dedup(EstepArgs a)
{
    using G = DedupGeom<d, V>;
    __shared__ __attribute__((aligned(16))) char lds[4 * G::wave_bytes];
    char *wl = lds + (threadIdx.x >> 6) * G::wave_bytes;
    if constexpr (PERSIST) {
        for_each_tile_persistent(a.tm, [&](int32_t t) {
            wave_sync();   // the wave's LDS reads of the previous tile are done before it is written again
            estep_dedup_tile<d, V, XF>(a, t, wl);
        });
    } else {
        const int32_t t = logical_tile(a.tm);
        if (t >= a.tm.n_tiles) return;
        estep_dedup_tile<d, V, XF>(a, t, wl);
    }
}

// Fused slice + reduction: every point's M-step terms (Eq. 7 / Eq. 10 in the
// twist of Eq. 16) are formed right after its slice and the block writes one
// partial row of the normal equations per tile; M0, M1 and N never leave the
// chip.  SHARED: the shared-lookup slice (its per-wave LDS region holds the
// wave's sums once its slice is done), else the per-point slice.
template <int d, int V, bool XF, int RES, bool SHARED>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(SHARED ? 5 : 1))) k_estep_fused(EstepArgs a)
{
    using G = DedupGeom<d, V>;
    constexpr int kWaveLds = SHARED ? G::wave_bytes : kRedStride * (int)sizeof(float);
    __shared__ __attribute__((aligned(16))) char lds[4 * kWaveLds];
    const int32_t t = logical_tile(a.tm);
    if (t >= a.tm.n_tiles) return;
    const int32_t s = tile_segment(a.tm, t);
    if (a.active != nullptr && a.active[a.tm.seg_set[s]] == 0) return;   // no partial row: the set is not solved
    const int wave = threadIdx.x >> 6;
    float red[kRedVals];
#pragma unroll
    for (int j = 0; j < kRedVals; ++j) red[j] = 0.0f;
    float x[3] = {0.0f, 0.0f, 0.0f}, acc[V];
#pragma unroll
    for (int c = 0; c < V; ++c) acc[c] = 0.0f;
    bool live;
    if constexpr (SHARED) {
        int64_t i = 0;
        live = dedup_point<d, V, XF>(a, s, t, lds + wave * kWaveLds, i, x, acc);
    } else {
        const int64_t i = a.tm.seg_off[s] + (int64_t)(t - a.tm.seg_tile[s]) * a.tm.tile + threadIdx.x;
        live = i < a.tm.seg_end[s];
        if (live) slice_point<d, V, XF>(a, s, i, a.sets[a.tm.seg_set[s]], x, acc);
    }
    {
        // one branch (m0 > 0 in mstep_point): a lane without a point passes m0 = 0 and adds nothing,
        // so the accumulators' zeros are not set up again for each of two nested branches
        const float c = a.seg_c[s];
        const float m0 = live ? acc[0] : 0.0f;
        if constexpr (RES == FR_PT2PL)
            mstep_point<RES>(red, x[0], x[1], x[2], m0, acc[1], acc[2], acc[3], acc[4], acc[5], acc[6], c,
                             a.normalize_n);
        else
            mstep_point<RES>(red, x[0], x[1], x[2], m0, acc[1], acc[2], acc[3], 0.0f, 0.0f, 0.0f, c,
                             a.normalize_n);
    }
    wave_sync();   // the wave's slice has read its LDS region
    block_partials(red, reinterpret_cast<float *>(lds), kWaveLds / (int)sizeof(float),
                   a.partials + (size_t)t * kRedStride);
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
    const int64_t i = a.tm.seg_off[s] + (int64_t)(t - a.tm.seg_tile[s]) * a.tm.tile + threadIdx.x;
    if (i >= a.tm.seg_end[s]) return;
    const SetTable st = a.sets[a.tm.seg_set[s]];
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
    for (int j = 0; j < d; ++j) kk[j] = st.k[j];
    uint64_t keys[D][KW];
    float b[D];
    embed<d>(p, kk, keys, b);
#pragma unroll
    for (int v = 0; v < D; ++v) {
        const int64_t slot = find_slot<KW, V>(st, keys[v]);
        if (slot >= 0) a.touched[st.slot_base + slot] = 1u;
    }
}

template <int d, int V, bool P>
static void launch_dvp(const EstepArgs &a, bool xf, bool touch, int slice, int grid, hipStream_t st)
{
    if (touch) {
        if (xf) k_estep_touch<d, V, true><<<grid, 256, 0, st>>>(a);
        else k_estep_touch<d, V, false><<<grid, 256, 0, st>>>(a);
    } else if (slice == FR_SLICE_SHARED) {
        if (xf) k_estep_dedup<d, V, true, P><<<grid, 256, 0, st>>>(a);
        else k_estep_dedup<d, V, false, P><<<grid, 256, 0, st>>>(a);
    } else {
        if (xf) k_estep<d, V, true, P><<<grid, 256, 0, st>>>(a);
        else k_estep<d, V, false, P><<<grid, 256, 0, st>>>(a);
    }
}

// persist_grid > 0: the persistent kernels on that many workgroups (tile count from the device)
template <int d, int V>
static void launch_dv(const EstepArgs &a, bool xf, bool touch, int slice, int grid, int persist_grid, hipStream_t st)
{
    if (persist_grid > 0 && !touch) launch_dvp<d, V, true>(a, xf, false, slice, persist_grid, st);
    else launch_dvp<d, V, false>(a, xf, touch, slice, grid, st);
}

// The slice autotuner: the first launch of each (d, V, transform kind, size
// class) a context meets is timed in both forms -- they compute the same
// outputs, so the timing launches are that E-step -- and the faster form is
// kept in the context's table.  One wait for the stream; nothing is timed
// while the stream is being captured into a graph.
// Autotuner entries of the fused slice + reduction carry this plus the transform kind.
constexpr int kTuneFused = 16;

template <class Launch>
static fr_status autotune_slice(fr_ctx *ctx, int d, int V, int xf_kind, int64_t pts, bool tune_new, hipStream_t st,
                                Launch &launch, int &slice)
{
    slice = FR_SLICE_PLAIN;
    if (ctx == nullptr) return FR_OK;
    int32_t cls = 0;
    while (cls < 62 && (2ll << cls) <= pts) ++cls;
    const fr_tuning_entry *near = nullptr;
    for (const fr_tuning_entry &e : ctx->tuned) {
        if (e.d != d || e.V != V || e.xf_kind != xf_kind) continue;
        if (e.size_class == cls) {
            slice = e.slice;
            return FR_OK;
        }
        if (near == nullptr || std::abs(e.size_class - cls) < std::abs(near->size_class - cls)) near = &e;
    }
    if (!tune_new && near != nullptr) {
        slice = near->slice;
        return FR_OK;
    }
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    FR_HIP(hipStreamIsCapturing(st, &cs));
    if (cs != hipStreamCaptureStatusNone) return FR_OK;
    constexpr int kReps = 4;
    const int cand[2] = {FR_SLICE_PLAIN, FR_SLICE_SHARED};
    float us[2] = {0.0f, 0.0f};
    hipEvent_t ev[2];
    FR_HIP(hipEventCreate(&ev[0]));
    FR_HIP(hipEventCreate(&ev[1]));
    fr_status rc = FR_OK;
    for (int c = 0; c < 2 && rc == FR_OK; ++c) {
        rc = launch(cand[c]);   // warm-up
        if (rc != FR_OK) break;
        if (hipEventRecord(ev[0], st) != hipSuccess) rc = FR_EDEVICE;
        for (int r = 0; r < kReps && rc == FR_OK; ++r) rc = launch(cand[c]);
        if (rc == FR_OK && (hipEventRecord(ev[1], st) != hipSuccess || hipEventSynchronize(ev[1]) != hipSuccess ||
                            hipEventElapsedTime(&us[c], ev[0], ev[1]) != hipSuccess))
            rc = FR_EDEVICE;
        us[c] *= 1000.0f / kReps;
    }
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    if (rc != FR_OK) {
        if (rc == FR_EDEVICE) set_error("slice autotuner: timing events failed");
        return rc;
    }
    fr_tuning_entry e{};
    e.d = d;
    e.V = V;
    e.xf_kind = xf_kind;
    e.size_class = cls;
    e.slice = us[1] < us[0] ? FR_SLICE_SHARED : FR_SLICE_PLAIN;
    e.us_plain = us[0];
    e.us_shared = us[1];
    ctx->tuned.push_back(e);
    slice = e.slice;
    return FR_OK;
}

int tuned_slice_nearest(const fr_ctx *ctx, int d, int V, int xf_kind, int64_t pts)
{
    if (ctx == nullptr) return FR_SLICE_PLAIN;
    if (ctx->slice_mode != FR_SLICE_AUTO) return ctx->slice_mode;
    int32_t cls = 0;
    while (cls < 62 && (2ll << cls) <= pts) ++cls;
    const fr_tuning_entry *near = nullptr;
    for (const fr_tuning_entry &e : ctx->tuned)
        if (e.d == d && e.V == V && e.xf_kind == xf_kind &&
            (near == nullptr || std::abs(e.size_class - cls) < std::abs(near->size_class - cls)))
            near = &e;
    return near != nullptr ? near->slice : FR_SLICE_PLAIN;
}

fr_status launch_estep_sets(int d, int V, const SetTable *sets, int32_t *err, int32_t err_stride,
                            const fr_cloud *model, int64_t M, const Plan &plan, int xf_kind, const float *mats,
                            float *m0, float *m1, float *nsum, float *m2, uint32_t *touched, hipStream_t st,
                            const int32_t *active)
{
    if (plan.grid == 0 && plan.persist_grid == 0) return FR_OK;
    EstepArgs a{};
    a.active = active;
    a.x = model->x;
    a.y = model->y;
    a.z = model->z;
    a.nx = model->nx;
    a.ny = model->ny;
    a.nz = model->nz;
    a.mats = mats;
    a.sets = sets;
    a.tm = plan.tm;
    a.m0 = m0;
    a.m1 = m1;
    a.ns = nsum;
    a.m2 = m2;
    a.M = M;
    a.touched = touched;
    a.err = err;
    a.err_stride = err_stride;
    const bool xf = xf_kind != FR_XF_NONE;
    const bool touch = touched != nullptr;
    auto launch = [&](int slice) -> fr_status {
        if (d == 3 && V == 4) launch_dv<3, 4>(a, xf, touch, slice, plan.grid, plan.persist_grid, st);
        else if (d == 3 && V == 7) launch_dv<3, 7>(a, xf, touch, slice, plan.grid, plan.persist_grid, st);
        else if (d == 6 && V == 4) launch_dv<6, 4>(a, xf, touch, slice, plan.grid, plan.persist_grid, st);
        else if (d == 6 && V == 7) launch_dv<6, 7>(a, xf, touch, slice, plan.grid, plan.persist_grid, st);
        else if (d == 3 && V == 5) launch_dv<3, 5>(a, xf, touch, slice, plan.grid, plan.persist_grid, st);
        else if (d == 3 && V == 8) launch_dv<3, 8>(a, xf, touch, slice, plan.grid, plan.persist_grid, st);
        else if (d == 6 && V == 5) launch_dv<6, 5>(a, xf, touch, slice, plan.grid, plan.persist_grid, st);
        else if (d == 6 && V == 8) launch_dv<6, 8>(a, xf, touch, slice, plan.grid, plan.persist_grid, st);
        else {
            set_error("fr_estep: unsupported lattice d=%d V=%d", d, V);
            return FR_EINVAL;
        }
        FR_HIP(hipGetLastError());
        return FR_OK;
    };
    int slice = touch ? FR_SLICE_PLAIN : plan.slice;
    if (slice == FR_SLICE_AUTO)
        FR_TRY(autotune_slice(plan.ctx, d, V, xf_kind, (int64_t)plan.n_tiles * plan.tile, plan.tune_new_classes, st,
                              launch, slice));
    return launch(slice);
}

// Workgroups of a persistent E-step launch: what the device holds at once
// (occupancy per CU times the CUs), a multiple of 8.
template <int d, int V>
static int persistent_grid_dv(int slice)
{
    int per_cu = 0, dev = 0, cus = 0;
    const void *f = slice == FR_SLICE_SHARED ? reinterpret_cast<const void *>(k_estep_dedup<d, V, true, true>)
                                             : reinterpret_cast<const void *>(k_estep<d, V, true, true>);
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, 256, 0);
    (void)hipGetLastError();
    return std::max(8, per_cu * cus / 8 * 8);
}

int estep_persistent_grid(int d, int V, int slice)
{
    if (d == 3 && V == 4) return persistent_grid_dv<3, 4>(slice);
    if (d == 3 && V == 7) return persistent_grid_dv<3, 7>(slice);
    if (d == 6 && V == 4) return persistent_grid_dv<6, 4>(slice);
    if (d == 6 && V == 7) return persistent_grid_dv<6, 7>(slice);
    return 0;
}

template <int d, int V, bool SHARED>
static void launch_fused_dvs(const EstepArgs &a, int residual, int grid, hipStream_t st)
{
    if constexpr (V == 7) {
        if (residual == FR_PT2PL) {
            k_estep_fused<d, V, true, FR_PT2PL, SHARED><<<grid, 256, 0, st>>>(a);
            return;
        }
    }
    k_estep_fused<d, V, true, FR_PT2PT, SHARED><<<grid, 256, 0, st>>>(a);
}

template <int d, int V>
static void launch_fused_dv(const EstepArgs &a, int residual, int slice, int grid, hipStream_t st)
{
    if (slice == FR_SLICE_SHARED) launch_fused_dvs<d, V, true>(a, residual, grid, st);
    else launch_fused_dvs<d, V, false>(a, residual, grid, st);
}

fr_status launch_estep_fused(int d, int V, const SetTable *sets, int32_t *err, int32_t err_stride,
                             const fr_cloud *model, const Plan &plan, const float *mats, int residual,
                             int normalize_n, float *partials, hipStream_t st, const int32_t *active)
{
    if (plan.grid == 0) return FR_OK;
    if ((residual == FR_PT2PL && V != 7) || (V != 4 && V != 7)) {
        set_error("fused E-step: V = 4 or 7 (7 for point-to-plane)");
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
    a.M = cloud_points(model);
    a.err = err;
    a.err_stride = err_stride;
    a.seg_c = plan.seg_c;
    a.partials = partials;
    a.normalize_n = normalize_n;
    a.active = active;
    if (!((d == 3 || d == 6) && (V == 4 || V == 7))) {
        set_error("fused E-step: unsupported lattice d=%d V=%d", d, V);
        return FR_EINVAL;
    }
    auto launch = [&](int slice) -> fr_status {
        if (d == 3 && V == 4) launch_fused_dv<3, 4>(a, residual, slice, plan.grid, st);
        else if (d == 3 && V == 7) launch_fused_dv<3, 7>(a, residual, slice, plan.grid, st);
        else if (d == 6 && V == 4) launch_fused_dv<6, 4>(a, residual, slice, plan.grid, st);
        else launch_fused_dv<6, 7>(a, residual, slice, plan.grid, st);
        FR_HIP(hipGetLastError());
        return FR_OK;
    };
    int slice = plan.slice;
    if (slice == FR_SLICE_AUTO)
        FR_TRY(autotune_slice(plan.ctx, d, V, kTuneFused + FR_XF_RIGID, (int64_t)plan.n_tiles * plan.tile,
                              plan.tune_new_classes, st, launch, slice));
    return launch(slice);
}

// Descriptor E-step (Eq. 8 with the features alone): one model point per
// thread reads its descriptor row, walks the d+1 vertices of its simplex one at
// a time (key, its bucket or two, the values of the slot found) and sums
// b * [1, y].
struct FeatArgs {
    const float *feat;        // M x d row-major
    const float *kf;          // d scale factors
    const SetTable *sets;
    TileMap tm;
    float *m0, *m1;
    int64_t M;
    int32_t *err;
};

template <int d>
__global__ void __launch_bounds__(256) k_estep_feat(FeatArgs a)
{
    constexpr int D = d + 1;
    constexpr int KW = KeyWords<d>::value;
    const int32_t t = logical_tile(a.tm);
    if (t >= a.tm.n_tiles) return;
    const int32_t s = tile_segment(a.tm, t);
    const int64_t i = a.tm.seg_off[s] + (int64_t)(t - a.tm.seg_tile[s]) * a.tm.tile + threadIdx.x;
    if (i >= a.tm.seg_end[s]) return;
    const SetTable st = a.sets[a.tm.seg_set[s]];
    float p[d], kk[d];
    const float4 *row = reinterpret_cast<const float4 *>(a.feat + (size_t)i * d);
#pragma unroll
    for (int q = 0; q < d / 4; ++q) {
        const float4 v = row[q];
        p[4 * q] = v.x;
        p[4 * q + 1] = v.y;
        p[4 * q + 2] = v.z;
        p[4 * q + 3] = v.w;
    }
#pragma unroll
    for (int j = 0; j < d; ++j) kk[j] = a.kf[j];
    HdEmbed<d> h;
    embed_hd_init<d>(p, kk, h);
    if (!h.ok) atomicOr(a.err, 1);
    float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll 1
    for (int m = 0; m < D; ++m) {   // one vertex at a time: keeps the key walk in registers
        const float b = embed_hd_next<d>(h, m);
        const int64_t r = find_slot<KW, 4>(st, h.P);
        if (r >= 0) {
            const u32x4 q = load_at<u32x4>(st.vals, (uint32_t)r * SlotGeom<KW, 4>::bytes);
            acc[0] = fmaf(b, __uint_as_float(q.x), acc[0]);
            acc[1] = fmaf(b, __uint_as_float(q.y), acc[1]);
            acc[2] = fmaf(b, __uint_as_float(q.z), acc[2]);
            acc[3] = fmaf(b, __uint_as_float(q.w), acc[3]);
        }
    }
    a.m0[i] = acc[0];
    a.m1[i] = acc[1];
    a.m1[a.M + i] = acc[2];
    a.m1[2 * a.M + i] = acc[3];
}

fr_status launch_estep_features(const fr_lattice *lat, const fr_cloud *model, const Plan &plan, const float *feat,
                                float *m0, float *m1, hipStream_t st)
{
    if (plan.grid == 0) return FR_OK;
    FeatArgs a{feat, lat->kfeat_d, lat->sets_d, plan.tm, m0, m1, cloud_points(model), lat->err_d};
    if (lat->d == 8) k_estep_feat<8><<<plan.grid, 256, 0, st>>>(a);
    else if (lat->d == 16) k_estep_feat<16><<<plan.grid, 256, 0, st>>>(a);
    else if (lat->d == 32) k_estep_feat<32><<<plan.grid, 256, 0, st>>>(a);
    else {
        set_error("descriptor E-step: dimension %d not supported", lat->d);
        return FR_EINVAL;
    }
    FR_HIP(hipGetLastError());
    return FR_OK;
}

fr_status launch_estep(const fr_lattice *lat, const fr_cloud *model, const Plan &plan, int xf_kind, const float *mats,
                       float *m0, float *m1, float *nsum, uint32_t *touched, hipStream_t st, float *m2,
                       const int32_t *active)
{
    return launch_estep_sets(lat->d, lat->V, lat->sets_d, lat->err_d, 0, model, cloud_points(model), plan,
                             xf_kind, mats, m0, m1, nsum, m2, touched, st, active);
}

}  // namespace fr
