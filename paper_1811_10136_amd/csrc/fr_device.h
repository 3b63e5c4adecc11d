// Device building blocks of the lattice E-step: the permutohedral embedding in
// pinned binary32 arithmetic, packed lattice keys, the hash and the slot layout
// of the lattice table, and the tile -> segment mapping shared by all kernels.
//
// Every translation unit that includes this file is compiled with
// -ffp-contract=off: the key of a point is an integer decided by floating
// point, so the key path is a fixed sequence of IEEE binary32 operations.
// Multiply-adds that are wanted elsewhere are written as explicit fmaf.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fr {

constexpr int kKeyBits = 21;                       // bits per packed lattice coordinate
constexpr int32_t kKeyBias = 1 << 20;              // coordinates live in [-2^20, 2^20)
constexpr uint64_t kKeyEmpty = ~0ull;              // never a packed key: bit 63 of a key is 0
constexpr uint32_t kOwnerEmpty = 0xFFFFFFFFu;

// E-step tiling: one model point per thread, 256 threads per block.
constexpr int kEstepTile = 256;

template <int d> struct KeyWords { static constexpr int value = (d + 2) / 3; };   // 3 coordinates per u64

// The lattice table of one set is a bucketed two-choice cuckoo hash: a
// bucket is two slots side by side, every vertex key sits in a slot of one of
// its two buckets b1(key), b2(key), and a slot holds the key's KW packed words
// (word 0 == kKeyEmpty marks a free slot) followed, at a 16-byte aligned
// offset, by its V binary32 values padded to VP = 4 or 8.  A key goes to b2
// only when b1 is full, and a filled slot is never emptied, so a lookup reads
// b1 (one cache line holding both keys and their values), stops there if it
// found the key or saw a free slot, and reads b2 otherwise.
template <int V> struct ValPad { static constexpr int value = V <= 4 ? 4 : 8; };

// Bytes of a slot (a power of two >= 32) and the byte offset of its values.
__host__ __device__ constexpr uint32_t slot_value_offset(int kw) { return (uint32_t)((8 * kw + 15) / 16 * 16); }
__host__ __device__ constexpr uint32_t slot_bytes(int kw, int vp)
{
    return slot_value_offset(kw) + 4u * vp <= 32u    ? 32u
           : slot_value_offset(kw) + 4u * vp <= 64u  ? 64u
           : slot_value_offset(kw) + 4u * vp <= 128u ? 128u
                                                     : 256u;
}
constexpr int kBucketSlots = 2;
template <int KW, int V> struct SlotGeom {
    static constexpr uint32_t bytes = slot_bytes(KW, ValPad<V>::value);
    static constexpr uint32_t val_off = slot_value_offset(KW);
    static constexpr uint32_t bucket = kBucketSlots * bytes;
};

// Value channels splatted per observation point: [1, y] (V = 4), [1, y, |y|^2]
// (V = 5), [1, y, n_y] (V = 7), [1, y, n_y, |y|^2] (V = 8).  |y|^2 feeds the
// variance update; it is always the last channel, and a vertex stores it as
// the scatter about its own mean, S_v = sum b |y - mu_v|^2 with mu_v = M1_v / W_v,
// so that no |y|^2-sized numbers are subtracted after rounding to binary32.
template <int V> struct ValLayout {
    static constexpr bool normals = V >= 7;
    static constexpr bool m2 = V == 5 || V == 8;
};

// Per-set view of the lattice table.  keys points at the set's first slot and
// vals at the values of that slot (keys + slot_value_offset bytes); slot i of
// the set starts slot_bytes * i bytes further.  Absolute pointers, so one
// launch can slice sets of lattices that were built separately.
struct SetTable {
    const uint64_t *keys; // first slot of the set
    const float *vals;    // values of the first slot
    uint64_t slot_base;   // first slot of the set in its lattice's table
    uint32_t cap;         // slots of the set (even, >= 16; cap / 2 buckets)
    uint32_t n_vertices;
    uint32_t seed;        // hash seed (changed when a cuckoo insertion has to be redone)
    uint32_t mask;        // cap - 1 for the power-of-two tables of the build
    float k[8];           // lattice scale of the set's features (binary32, see embed)
};

// Tiles of points grouped by segment; a segment lies inside one set.
struct TileMap {
    const int64_t *seg_off;    // n_seg first points
    const int64_t *seg_end;    // n_seg end points (seg_off + 1 for a partition)
    const int32_t *seg_tile;   // n_seg + 1 tile prefix
    const int32_t *seg_set;    // n_seg
    int32_t n_seg;
    int32_t n_tiles;
    int32_t tile;              // points per tile
    int32_t xcd_chunk;         // logical tiles per XCD (0 = identity mapping)
};

// Launches are dispatched round-robin over the 8 XCDs (block b runs on XCD
// b % 8).  Mapping block b to logical tile (b % 8) * chunk + b / 8 hands each
// XCD a contiguous run of tiles, so consecutive tiles of one set -- which read
// the same lattice -- share that XCD's L2.
__device__ __forceinline__ int32_t logical_tile(const TileMap &tm)
{
    const int32_t b = (int32_t)blockIdx.x;
    if (tm.xcd_chunk <= 0) return b;
    return (b & 7) * tm.xcd_chunk + (b >> 3);
}

// Persistent launches (a fixed grid, a multiple of 8 workgroups): the tile
// count comes from the device (seg_tile[n_seg]), XCD x = block % 8 takes the
// x-th of 8 contiguous runs of tiles, and its workgroups walk that run with a
// stride of grid / 8 -- the same XCD-contiguous order as logical_tile, for a
// grid that does not depend on the plan (a captured graph replays it for any
// set of resident requests).
template <class Body>
__device__ __forceinline__ void for_each_tile_persistent(const TileMap &tm, Body &&body)
{
    const int32_t n = tm.seg_tile[tm.n_seg];
    const int32_t chunk = (n + 7) / 8;
    const int32_t x = (int32_t)(blockIdx.x & 7u);
    const int32_t hi = min((x + 1) * chunk, n);
    const int32_t stride = (int32_t)(gridDim.x >> 3);
    for (int32_t t = x * chunk + (int32_t)(blockIdx.x >> 3); t < hi; t += stride) body(t);
}

// Segment of a logical tile: last s with seg_tile[s] <= t (uniform per block).
__device__ __forceinline__ int32_t tile_segment(const TileMap &tm, int32_t t)
{
    int32_t lo = 0, hi = tm.n_seg - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (tm.seg_tile[mid] <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ uint32_t fmix32(uint32_t h)
{
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return h;
}

// Hash of the packed key words.  The seed enters first and every later step
// mixes it non-linearly, so keys that collide under one seed do not collide
// under the next (a multiply-add chain is affine in the words: its collisions
// would not depend on the seed, and a rebuild with a new seed could never
// separate three colliding keys).  Position keys (KW <= 2, the slice's and the
// build's hot path) fold each 32-bit half in with one multiply and one shift
// and end with the finaliser of MurmurHash3: 6 integer multiplies, which run
// at a quarter of the vector rate, against 14 for the full block mix.
// Descriptor keys (KW > 2: up to 11 words, millions of vertices per set) take
// the block mix and finaliser of MurmurHash3 (x86, 32-bit).
__device__ __forceinline__ uint32_t rotl32(uint32_t x, int r) { return (x << r) | (x >> (32 - r)); }

template <int KW>
__device__ __forceinline__ uint32_t hash_key(const uint64_t (&w)[KW], uint32_t seed)
{
    if constexpr (KW <= 2) {
        uint32_t h = seed ^ 0x9E3779B9u;
#pragma unroll
        for (int i = 0; i < 2 * KW; ++i) {
            const uint32_t x = (i & 1) ? (uint32_t)(w[i / 2] >> 32) : (uint32_t)w[i / 2];
            h = (h ^ x) * 0xCC9E2D51u;
            h ^= h >> 16;
        }
        return fmix32(h ^ (uint32_t)(8 * KW));
    }
    uint32_t h = seed;
#pragma unroll
    for (int i = 0; i < 2 * KW; ++i) {
        uint32_t k = (i & 1) ? (uint32_t)(w[i / 2] >> 32) : (uint32_t)w[i / 2];
        k *= 0xCC9E2D51u;
        k = rotl32(k, 15);
        k *= 0x1B873593u;
        h ^= k;
        h = rotl32(h, 13);
        h = h * 5u + 0xE6546B64u;
    }
    h ^= (uint32_t)(8 * KW);
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return h;
}

// The two candidate buckets of a key in a table of `nb` buckets: two hashes
// mapped to [0, nb) by a multiply-high range reduction (no power-of-two size
// needed); the second moves on by one if it coincides with the first.
__device__ __forceinline__ void cuckoo_buckets(uint32_t h, uint32_t nb, uint32_t &b1, uint32_t &b2)
{
    b1 = __umulhi(h, nb);
    const uint32_t h2 = (h ^ (h >> 16)) * 0x7FEB352Du;
    b2 = __umulhi(h2, nb);
    b2 = (b2 == b1) ? ((b1 + 1u == nb) ? 0u : b1 + 1u) : b2;
}

// Both candidate buckets of a key.  Positions (KW <= 2) take them from one
// 32-bit hash.  Descriptor lattices hold millions of vertices per set, where
// several keys share a 32-bit hash and, with it, both buckets (five such keys
// cannot be placed); their second bucket comes from a second hash with
// another seed, so a shared first hash no longer implies a shared pair.
template <int KW>
__device__ __forceinline__ void key_buckets(const uint64_t (&key)[KW], uint32_t seed, uint32_t nb, uint32_t &b1,
                                            uint32_t &b2)
{
    const uint32_t h = hash_key<KW>(key, seed);
    if constexpr (KW <= 2) {
        cuckoo_buckets(h, nb, b1, b2);
    } else {
        b1 = __umulhi(h, nb);
        b2 = __umulhi(hash_key<KW>(key, seed * 0x2545F491u + 0x9E3779B9u), nb);
        b2 = (b2 == b1) ? ((b1 + 1u == nb) ? 0u : b1 + 1u) : b2;
    }
}

// Loads from a uniform table base with a 32-bit byte offset (a set's table
// is below 4 GiB; the build checks).
// The base is cast to the global address space: table pointers arrive through
// memory (the per-set table), where the compiler cannot infer it, and a
// generic pointer would turn every lookup into a flat load with 64-bit address
// arithmetic instead of the scalar-base + vector-offset global form.
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) const char global_cchar;

template <typename T>
__device__ __forceinline__ T load_at(const void *__restrict__ base, uint32_t byte_off)
{
    typedef __attribute__((address_space(1))) const T global_T;
    return *(global_T *)((global_cchar *)base + byte_off);
}

// The key words of the slot that starts `base` bytes into the table.
template <int KW>
__device__ __forceinline__ void load_key(const uint64_t *__restrict__ keys, uint32_t base, uint64_t (&k)[KW])
{
    if constexpr (KW == 2) {
        const u32x4 q = load_at<u32x4>(keys, base);
        k[0] = (uint64_t)q.x | ((uint64_t)q.y << 32);
        k[1] = (uint64_t)q.z | ((uint64_t)q.w << 32);
    } else if constexpr (KW == 1) {
        const u32x2 q = load_at<u32x2>(keys, base);
        k[0] = (uint64_t)q.x | ((uint64_t)q.y << 32);
    } else {
        // descriptor lattices: KW words of 8 bytes
#pragma unroll
        for (int w = 0; w < KW; ++w) {
            const u32x2 q = load_at<u32x2>(keys, base + 8u * w);
            k[w] = (uint64_t)q.x | ((uint64_t)q.y << 32);
        }
    }
}

template <int KW>
__device__ __forceinline__ bool key_equal(const uint64_t (&a)[KW], const uint64_t (&b)[KW])
{
    bool eq = true;
#pragma unroll
    for (int w = 0; w < KW; ++w) eq = eq && (a[w] == b[w]);
    return eq;
}

// The permutohedral embedding of one point (the lattice method the paper uses
// for its filter, Sec. 4.2; features normalised by sigma, Sec. 4.1):
//   cf_i = p_i k_i; e_j = (cf_j + ... + cf_(d-1)) - j cf_(j-1), e_0 = sum cf;
//   g_j = nearest multiple of D = d+1 to e_j (ties to the lower one);
//   rank_j = #{i: delta_i > delta_j} + #{i < j: delta_i == delta_j}, delta = e - g;
//   s = sum(g) / D.
// The enclosing simplex is usually written after a correction that adds s to
// every rank and moves the coordinates whose rank wraps by -/+D.  That
// correction only relabels the simplex: its vertex k is vertex (k + s) mod D of
// the uncorrected simplex moved by -s in every coordinate, with the same
// weight.  So, with no correction step, vertex m (m = 0..d) is
//   v_m[j] = g_j - s + m - D [rank_j > d - m],
// with weight b_0 = 1 + (u_(d) - u_(0)), b_m = u_(d-m) - u_(d-m+1), where u_(r)
// is the r-th largest delta / D.  Vertex order is immaterial to splat and
// slice, which sum over all d + 1 vertices.
// All key-path arithmetic is binary32 in this exact order (no contraction).
// Keys: 21-bit biased coordinates packed 3 per u64 (coordinate 0 in the top
// field of word 0); vertex m's key is vertex m-1's plus +1 in every field and
// -D in the field of the coordinate of rank d - m + 1.  Returns false if a
// coordinate leaves the packed range.
// s_out receives s: every coordinate of vertex m is congruent to m - s
// modulo D, so equal keys of two points sit at vertex indices that differ by
// the difference of their s (mod D).
template <int d>
__device__ __forceinline__ bool embed(const float (&p)[d], const float (&k)[d],
                                      uint64_t (&keys)[d + 1][KeyWords<d>::value], float (&b)[d + 1],
                                      int32_t *s_out = nullptr)
{
    constexpr int D = d + 1;
    constexpr int KW = KeyWords<d>::value;
    constexpr float invD = (float)(1.0 / (double)D);
    constexpr float fD = (float)D;

    float e[D];
    float S = 0.0f;
#pragma unroll
    for (int j = d; j >= 1; --j) {
        const float cf = p[j - 1] * k[j - 1];
        const float jc = (float)j * cf;
        e[j] = S - jc;
        S = S + cf;
    }
    e[0] = S;

    // nearest multiple of D: floor(v) D or the next one (up = floor(v) D + D
    // equals ceil(v) D unless v is integral, where e is within rounding of the
    // lower one and the lower one wins either way)
    int32_t g[D];
    float delta[D];
    int32_t sum_g = 0;
#pragma unroll
    for (int j = 0; j < D; ++j) {
        const float v = e[j] * invD;
        const float dn = floorf(v) * fD;
        const float up = dn + fD;
        const float du = up - e[j];
        const float dd = e[j] - dn;
        const float gf = (du < dd) ? up : dn;
        g[j] = (int32_t)gf;
        delta[j] = e[j] - gf;
        sum_g += g[j];
    }
    const int32_t s = sum_g / D;
    if (s_out != nullptr) *s_out = s;

    int32_t rank[D];
#pragma unroll
    for (int j = 0; j < D; ++j) rank[j] = 0;
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = i + 1; j < D; ++j) {
            // the larger delta ranks first; on a tie the lower index ranks first
            const int32_t c = delta[i] < delta[j] ? 1 : 0;
            rank[i] += c;
            rank[j] += 1 - c;
        }

    // deltas in descending order (odd-even transposition network)
    float us[D];
#pragma unroll
    for (int j = 0; j < D; ++j) us[j] = delta[j];
#pragma unroll
    for (int r = 0; r < D; ++r)
#pragma unroll
        for (int i = r & 1; i + 1 < D; i += 2) {
            const float hi = fmaxf(us[i], us[i + 1]);
            const float lo = fminf(us[i], us[i + 1]);
            us[i] = hi;
            us[i + 1] = lo;
        }
    b[0] = 1.0f + (us[d] - us[0]) * invD;
#pragma unroll
    for (int m = 1; m <= d; ++m) b[m] = (us[d - m] - us[d - m + 1]) * invD;

    bool ok = true;
    uint64_t P[KW];
#pragma unroll
    for (int w = 0; w < KW; ++w) P[w] = 0;
#pragma unroll
    for (int j = 0; j < d; ++j) {
        const int32_t c = g[j] - s;
        ok = ok && (c >= -kKeyBias + D) && (c < kKeyBias - D);
        P[j / 3] |= (uint64_t)((uint32_t)(c + kKeyBias) & ((1u << kKeyBits) - 1u)) << (kKeyBits * (2 - (j % 3)));
    }
#pragma unroll
    for (int w = 0; w < KW; ++w) keys[0][w] = P[w];
#pragma unroll
    for (int m = 1; m <= d; ++m) {
        const int32_t t = d - m + 1;
#pragma unroll
        for (int w = 0; w < KW; ++w) {
            uint64_t ones = 0, down = 0;
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                const int j = 3 * w + f;
                if (j < d) {
                    const uint64_t unit = 1ull << (kKeyBits * (2 - f));
                    ones += unit;
                    down = (rank[j] == t) ? (uint64_t)D * unit : down;
                }
            }
            P[w] += ones - down;
            keys[m][w] = P[w];
        }
    }
    return ok;
}

// The same embedding for descriptor spaces of dozens of dimensions, where the
// d+1 keys do not fit in registers at once: embed_hd_init does the elevation,
// rounding and ranking (the arithmetic of embed<d>, in the same binary32
// order) and packs vertex 0's key; embed_hd_next then gives the weight of
// vertex m and moves the key to it (vertices in order m = 0, 1, ..., d).  The
// deltas of a given rank are found by scanning the d+1 coordinates, so that
// nothing is indexed by a runtime value.
template <int d> struct HdEmbed {
    float delta[d + 1];
    int32_t rank[d + 1];
    float u_first, u_last;               // largest and smallest delta
    uint64_t P[KeyWords<d>::value];      // key of the current vertex
    bool ok;
};

template <int d>
__device__ __forceinline__ void embed_hd_init(const float *p, const float *k, HdEmbed<d> &h)
{
    constexpr int D = d + 1;
    constexpr int KW = KeyWords<d>::value;
    constexpr float invD = (float)(1.0 / (double)D);
    constexpr float fD = (float)D;
    float e[D];
    float S = 0.0f;
#pragma unroll
    for (int j = d; j >= 1; --j) {
        const float cf = p[j - 1] * k[j - 1];
        const float jc = (float)j * cf;
        e[j] = S - jc;
        S = S + cf;
    }
    e[0] = S;
    int32_t g[D];
    int32_t sum_g = 0;
#pragma unroll
    for (int j = 0; j < D; ++j) {
        const float v = e[j] * invD;
        const float dn = floorf(v) * fD;
        const float up = dn + fD;
        const float du = up - e[j];
        const float dd = e[j] - dn;
        const float gf = (du < dd) ? up : dn;
        g[j] = (int32_t)gf;
        h.delta[j] = e[j] - gf;
        sum_g += g[j];
    }
    const int32_t s = sum_g / D;
#pragma unroll
    for (int j = 0; j < D; ++j) h.rank[j] = 0;
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = i + 1; j < D; ++j) {
            const int32_t c = h.delta[i] < h.delta[j] ? 1 : 0;
            h.rank[i] += c;
            h.rank[j] += 1 - c;
        }
    h.u_first = 0.0f;
    h.u_last = 0.0f;
#pragma unroll
    for (int j = 0; j < D; ++j) {
        h.u_first = h.rank[j] == 0 ? h.delta[j] : h.u_first;
        h.u_last = h.rank[j] == d ? h.delta[j] : h.u_last;
    }
    h.ok = true;
#pragma unroll
    for (int w = 0; w < KW; ++w) h.P[w] = 0;
#pragma unroll
    for (int j = 0; j < d; ++j) {
        const int32_t c = g[j] - s;
        h.ok = h.ok && (c >= -kKeyBias + D) && (c < kKeyBias - D);
        h.P[j / 3] |= (uint64_t)((uint32_t)(c + kKeyBias) & ((1u << kKeyBits) - 1u)) << (kKeyBits * (2 - (j % 3)));
    }
}

// Weight of vertex m; for m >= 1 first steps the key from vertex m-1 to m
// (+1 in every coordinate, -D in the coordinate of rank d - m + 1).
template <int d>
__device__ __forceinline__ float embed_hd_next(HdEmbed<d> &h, int m)
{
    constexpr int D = d + 1;
    constexpr int KW = KeyWords<d>::value;
    constexpr float invD = (float)(1.0 / (double)D);
    if (m == 0) return 1.0f + (h.u_last - h.u_first) * invD;
    const int32_t t = d - m + 1;
    float ua = 0.0f, ub = 0.0f;
    uint64_t down[KW];
#pragma unroll
    for (int w = 0; w < KW; ++w) down[w] = 0;
#pragma unroll
    for (int j = 0; j < D; ++j) {
        ua = h.rank[j] == t - 1 ? h.delta[j] : ua;
        ub = h.rank[j] == t ? h.delta[j] : ub;
        if (j < d) {
            const uint64_t unit = 1ull << (kKeyBits * (2 - (j % 3)));
            down[j / 3] = h.rank[j] == t ? (uint64_t)D * unit : down[j / 3];
        }
    }
#pragma unroll
    for (int w = 0; w < KW; ++w) {
        uint64_t ones = 0;
#pragma unroll
        for (int f = 0; f < 3; ++f)
            if (3 * w + f < d) ones += 1ull << (kKeyBits * (2 - f));
        h.P[w] += ones - down[w];
    }
    return (ua - ub) * invD;
}

// Unpack coordinate j of a packed key (for export).
__host__ __device__ inline int32_t unpack_coord(const uint64_t *words, int j)
{
    const uint64_t w = words[j / 3];
    const uint32_t f = (uint32_t)((w >> (kKeyBits * (2 - (j % 3)))) & ((1u << kKeyBits) - 1u));
    return (int32_t)f - kKeyBias;
}

// Pinned binary32 rigid transform ((R0 x + R1 y) + R2 z) + t, no contraction.
__device__ __forceinline__ void xform_point(const float *m, float x, float y, float z, float &ox, float &oy, float &oz)
{
    ox = ((m[0] * x + m[1] * y) + m[2] * z) + m[3];
    oy = ((m[4] * x + m[5] * y) + m[6] * z) + m[7];
    oz = ((m[8] * x + m[9] * y) + m[10] * z) + m[11];
}

__device__ __forceinline__ void xform_normal(const float *m, float x, float y, float z, float &ox, float &oy, float &oz)
{
    ox = (m[0] * x + m[1] * y) + m[2] * z;
    oy = (m[4] * x + m[5] * y) + m[6] * z;
    oz = (m[8] * x + m[9] * y) + m[10] * z;
}

// The values of the slot whose values start `off` bytes after vb.
template <int V>
__device__ __forceinline__ void load_vals(const float *__restrict__ vb, uint32_t off, float (&val)[8])
{
    constexpr int VP = ValPad<V>::value;
    const u32x4 q0 = load_at<u32x4>(vb, off);
    u32x4 q1 = {0u, 0u, 0u, 0u};
    if constexpr (VP == 8) q1 = load_at<u32x4>(vb, off + 16u);
    val[0] = __uint_as_float(q0.x);
    val[1] = __uint_as_float(q0.y);
    val[2] = __uint_as_float(q0.z);
    val[3] = __uint_as_float(q0.w);
    val[4] = __uint_as_float(q1.x);
    val[5] = __uint_as_float(q1.y);
    val[6] = __uint_as_float(q1.z);
    val[7] = __uint_as_float(q1.w);
}

// Lookup of NL keys (live[v] == false: no key, nothing read).  Level 1 reads
// both key slots of every key's first bucket (one line each); level 2, where
// a first bucket is full without the key, both key slots of the second
// bucket.  off[v] is the byte offset of the slot found (found[v]).
template <int KW, int V, int NL>
__device__ __forceinline__ void lookup_keys(const SetTable &st, const uint64_t (&keys)[NL][KW], const bool (&live)[NL],
                                            uint32_t (&off)[NL], bool (&found)[NL])
{
    using G = SlotGeom<KW, V>;
    const uint64_t *__restrict__ kb = st.keys;
    const uint32_t nb = st.cap >> 1;
    uint32_t alt[NL];
    uint64_t k0[NL][KW], k1[NL][KW];
    bool second[NL];
#pragma unroll
    for (int v = 0; v < NL; ++v) {
        off[v] = 0u;
        alt[v] = 0u;
        if (live[v]) {
            uint32_t b1, b2;
            key_buckets<KW>(keys[v], st.seed, nb, b1, b2);
            off[v] = b1 * G::bucket;
            alt[v] = b2 * G::bucket;
            load_key<KW>(kb, off[v], k0[v]);
            load_key<KW>(kb, off[v] + G::bytes, k1[v]);
        }
    }
#pragma unroll
    for (int v = 0; v < NL; ++v) {
        found[v] = false;
        second[v] = false;
        if (live[v]) {
            const bool e0 = key_equal<KW>(k0[v], keys[v]);
            const bool e1 = key_equal<KW>(k1[v], keys[v]);
            found[v] = e0 || e1;
            second[v] = !found[v] && k0[v][0] != kKeyEmpty && k1[v][0] != kKeyEmpty;
            off[v] += e1 ? G::bytes : 0u;
            if (second[v]) {
                load_key<KW>(kb, alt[v], k0[v]);
                load_key<KW>(kb, alt[v] + G::bytes, k1[v]);
            }
        }
    }
#pragma unroll
    for (int v = 0; v < NL; ++v) {
        if (second[v]) {
            const bool e0 = key_equal<KW>(k0[v], keys[v]);
            const bool e1 = key_equal<KW>(k1[v], keys[v]);
            found[v] = e0 || e1;
            off[v] = alt[v] + (e1 ? G::bytes : 0u);
        }
    }
}

// Slice sums of one point from the values of its D vertices (val[v] = 0 and
// found[v] == false for a vertex absent from the lattice): vertices
// accumulate in order v = 0..d, each as w * value with w = b or 0.  For the
// |y|^2 layouts the last channel comes out as the second moment about the
// target, sum_k K |y_k - t|^2 with t = M1 / M0 (0 without support).
template <int V, int D>
__device__ __forceinline__ void accumulate_simplex(const float (&val)[D][8], const bool (&found)[D],
                                                   const float (&b)[D], float (&acc)[V])
{
    float vw[D];
#pragma unroll
    for (int v = 0; v < D; ++v) {
        const float w = found[v] ? b[v] : 0.0f;
        vw[v] = w;
#pragma unroll
        for (int c = 0; c < V; ++c) acc[c] = fmaf(w, val[v][c], acc[c]);
    }
    if constexpr (ValLayout<V>::m2) {
        // second moment about the target t = M1 / M0:
        //   sum_k K |y_k - t|^2 = sum_v b_v (S_v + W_v |mu_v - t|^2)
        if (acc[0] > 0.0f) {
            const float inv = 1.0f / acc[0];
            const float tx = acc[1] * inv, ty = acc[2] * inv, tz = acc[3] * inv;
#pragma unroll
            for (int v = 0; v < D; ++v) {
                const float W = val[v][0];
                const float iw = W > 0.0f ? 1.0f / W : 0.0f;
                const float dx = val[v][1] * iw - tx, dy = val[v][2] * iw - ty, dz = val[v][3] * iw - tz;
                acc[V - 1] = fmaf(vw[v] * W, fmaf(dx, dx, fmaf(dy, dy, dz * dz)), acc[V - 1]);
            }
        }
    }
}

// Slice one point: look its D vertices up (all first buckets at once, then
// the second buckets needed), read the values of the vertices found from the
// lines just fetched, and accumulate.  A vertex absent from the lattice
// contributes nothing.
template <int KW, int V, int D>
__device__ __forceinline__ void slice_simplex(const SetTable &st, const uint64_t (&keys)[D][KW], const float (&b)[D],
                                              float (&acc)[V])
{
    const float *__restrict__ vb = st.vals;
    bool live[D];
#pragma unroll
    for (int v = 0; v < D; ++v) live[v] = true;
    uint32_t off[D];
    bool found[D];
    lookup_keys<KW, V, D>(st, keys, live, off, found);
    float val[D][8];
#pragma unroll
    for (int v = 0; v < D; ++v) {
#pragma unroll
        for (int c = 0; c < 8; ++c) val[v][c] = 0.0f;
        if (found[v]) load_vals<V>(vb, off[v], val[v]);
    }
    accumulate_simplex<V, D>(val, found, b, acc);
}

// ---------------------------------------------------------------------------
// Runs of shared vertices along a wavefront.
//
// Consecutive points of a range-image scan lie side by side on the surface,
// so their simplices share most vertices.  Vertex m of a point has every
// coordinate congruent to m - s (mod D) (see embed), so its key can only equal
// the previous point's vertex of the same class c = (m - s) mod D.  Along the
// 64 lanes of a wave (lane = point), the vertices of one class form runs of
// equal keys; a run starts at a lane whose class-c key differs from the
// previous lane's (lane 0 starts a run in every class).  Runs are numbered
// class by class, and by start lane within a class: entry e of the wave.
// ---------------------------------------------------------------------------

// Orders the LDS accesses of the lanes of one wave (no workgroup barrier).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int KW>
__device__ __forceinline__ void lds_put_key(char *p, const uint64_t (&k)[KW])
{
#pragma unroll
    for (int w = 0; w < KW; ++w) reinterpret_cast<uint64_t *>(p)[w] = k[w];
}
template <int KW>
__device__ __forceinline__ void lds_get_key(const char *p, uint64_t (&k)[KW])
{
#pragma unroll
    for (int w = 0; w < KW; ++w) k[w] = reinterpret_cast<const uint64_t *>(p)[w];
}

// Bytes of the key region of a wave: 64 lanes x D classes x KW words.
template <int d> struct WaveKeys {
    static constexpr int D = d + 1;
    static constexpr int KW = KeyWords<d>::value;
    static constexpr int bytes = 64 * D * KW * 8;
};

// Class of vertex m: (m - r) mod D with r = s mod D.
template <int D>
__device__ __forceinline__ int32_t class_shift(int32_t sdiv)
{
    int32_t r = sdiv % D;
    return r + (r < 0 ? D : 0);
}

// Finds the runs of the wave.  live: the lane has a point (dead lanes form
// the tail of the wave).  kreg (LDS, WaveKeys<d>::bytes) receives every live
// lane's keys at [lane][class].  Each run start writes (lane << 3) | class at
// src[e] if e < src_cap; with ent != NULL every live lane writes the entry of
// the run holding its vertex m at ent[m] (valid when U <= 256, the only case
// its callers read it); with hc != NULL lane 0 writes the
// run-start mask of class c at hc[c].  Returns the number of runs U (uniform).
template <int d>
__device__ __forceinline__ int32_t wave_runs(const uint64_t (&keys)[d + 1][KeyWords<d>::value], int32_t r, bool live,
                                             char *kreg, uint16_t *src, int32_t src_cap, uint8_t *ent,
                                             uint64_t *hc)
{
    constexpr int D = d + 1;
    constexpr int KW = KeyWords<d>::value;
    constexpr int KB = 8 * KW;
    const int lane = (int)(threadIdx.x & 63u);
    if (live) {
#pragma unroll
        for (int m = 0; m < D; ++m) {
            int32_t c = m - r;
            c += c < 0 ? D : 0;
            lds_put_key<KW>(kreg + (lane * D + c) * KB, keys[m]);
        }
    }
    wave_sync();
    uint32_t hmask = 0;
    if (live) {
        if (lane == 0) {
            hmask = (1u << D) - 1u;
        } else {
#pragma unroll
            for (int m = 0; m < D; ++m) {
                int32_t c = m - r;
                c += c < 0 ? D : 0;
                uint64_t pk[KW];
                lds_get_key<KW>(kreg + ((lane - 1) * D + c) * KB, pk);
                hmask |= key_equal<KW>(pk, keys[m]) ? 0u : (1u << m);
            }
        }
    }
    int32_t U = 0;
#pragma unroll
    for (int c = 0; c < D; ++c) {
        int32_t mc = c + r;
        mc -= mc >= D ? D : 0;
        const bool bit = live && ((hmask >> mc) & 1u);
        const uint64_t H = __ballot(bit);
        const int32_t below = (int32_t)__builtin_amdgcn_mbcnt_hi((uint32_t)(H >> 32),
                                                                __builtin_amdgcn_mbcnt_lo((uint32_t)H, 0u));
        if (bit && U + below < src_cap) src[U + below] = (uint16_t)((lane << 3) | c);
        if (ent != nullptr && live) ent[mc] = (uint8_t)(U + below + (bit ? 0 : -1));
        if (hc != nullptr && lane == 0) hc[c] = H;
        U += (int32_t)__popcll(H);
    }
    return U;
}

// Slot of a key in a set's table (relative to the set's first slot), or -1.
template <int KW, int V>
__device__ __forceinline__ int64_t find_slot(const SetTable &st, const uint64_t (&key)[KW])
{
    using G = SlotGeom<KW, V>;
    uint32_t bk[2];
    key_buckets<KW>(key, st.seed, st.cap >> 1, bk[0], bk[1]);
#pragma unroll 1
    for (int i = 0; i < 2; ++i) {
        uint64_t k0[KW], k1[KW];
        load_key<KW>(st.keys, bk[i] * G::bucket, k0);
        load_key<KW>(st.keys, bk[i] * G::bucket + G::bytes, k1);
        if (key_equal<KW>(k0, key)) return (int64_t)kBucketSlots * bk[i];
        if (key_equal<KW>(k1, key)) return (int64_t)kBucketSlots * bk[i] + 1;
        if (k0[0] == kKeyEmpty || k1[0] == kKeyEmpty) return -1;   // the key never moved past a free slot
    }
    return -1;
}

}  // namespace fr
