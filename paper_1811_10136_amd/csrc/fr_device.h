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

template <int d> struct KeyWords { static constexpr int value = (d + 2) / 3; };   // 3 coordinates per u64

// Slot of the lattice table: packed key words, then V binary32 values,
// padded to whole 16-byte quads so one slot is read with NQ dwordx4 loads.
template <int KW, int V> struct SlotLayout {
    static constexpr int kWords = 2 * KW + V;
    static constexpr int kNQ = (kWords + 3) / 4;
    static constexpr int kBytes = 16 * kNQ;
};

// Per-set view of the lattice table.
struct SetTable {
    uint64_t slot_base;   // first slot of the set in the shared table
    uint32_t mask;        // capacity - 1 (capacity is a power of two)
    uint32_t n_vertices;
};

// Tiles of points grouped by segment; a segment lies inside one set.
struct TileMap {
    const int64_t *seg_off;    // n_seg + 1 point offsets
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

template <int KW>
__device__ __forceinline__ uint32_t hash_key(const uint64_t (&w)[KW])
{
    uint32_t h = 0x9E3779B9u;
#pragma unroll
    for (int i = 0; i < KW; ++i) {
        h = (h ^ (uint32_t)w[i]) * 0x01000193u;
        h = (h ^ (uint32_t)(w[i] >> 32)) * 0x27D4EB2Fu;
    }
    return fmix32(h);
}

// The permutohedral embedding of one point (the lattice method the paper uses
// for its filter, Sec. 4.2; features normalised by sigma, Sec. 4.1):
//   cf_i = p_i k_i; e_j = (cf_j + ... + cf_(d-1)) - j cf_(j-1), e_0 = sum cf;
//   g_j = nearest multiple of D = d+1 (ties to the lower); ranks of e - g with
//   ties broken by index; the sum of g / D shifts the ranks, and a rank that
//   wraps moves g_j by -/+ D; weights are differences of the rank-sorted
//   (e - g) / D; vertex k has coordinates g_j + k - D [rank_j > d - k].
// All key-path arithmetic is binary32 in this exact order (no contraction).
// Outputs: packed keys of the D vertices and their weights; returns false if a
// coordinate leaves the packed range.
template <int d>
__device__ __forceinline__ bool embed(const float (&p)[d], const float (&k)[d],
                                      uint64_t (&keys)[d + 1][KeyWords<d>::value], float (&b)[d + 1])
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
        const float up = ceilf(v) * fD;
        const float dn = floorf(v) * fD;
        const float du = up - e[j];
        const float dd = e[j] - dn;
        g[j] = (du < dd) ? (int32_t)up : (int32_t)dn;
        sum_g += g[j];
    }
    const int32_t s = sum_g / D;

    float delta[D];
#pragma unroll
    for (int j = 0; j < D; ++j) delta[j] = e[j] - (float)g[j];

    int32_t rank[D];
#pragma unroll
    for (int j = 0; j < D; ++j) rank[j] = 0;
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = i + 1; j < D; ++j) {
            // rank_j counts larger deltas and equal deltas of lower index
            if (delta[i] < delta[j]) rank[i]++; else rank[j]++;
        }

#pragma unroll
    for (int j = 0; j < D; ++j) {
        rank[j] += s;
        if (rank[j] < 0) { rank[j] += D; g[j] += D; }
        else if (rank[j] > d) { rank[j] -= D; g[j] -= D; }
    }

    // u by rank, gathered with selects (no dynamic register indexing)
    float ur[D];
#pragma unroll
    for (int r = 0; r < D; ++r) {
        float acc = 0.0f;
#pragma unroll
        for (int j = 0; j < D; ++j) acc = (rank[j] == r) ? (e[j] - (float)g[j]) * invD : acc;
        ur[r] = acc;
    }
    b[0] = (1.0f + ur[d]) - ur[0];
#pragma unroll
    for (int kk = 1; kk <= d; ++kk) b[kk] = ur[d - kk] - ur[d - kk + 1];

    bool ok = true;
#pragma unroll
    for (int kk = 0; kk < D; ++kk) {
#pragma unroll
        for (int w = 0; w < KW; ++w) keys[kk][w] = 0;
#pragma unroll
        for (int j = 0; j < d; ++j) {
            const int32_t c = g[j] + kk - ((rank[j] > d - kk) ? D : 0);
            ok = ok && (c >= -kKeyBias) && (c < kKeyBias);
            const uint64_t field = (uint64_t)((uint32_t)(c + kKeyBias) & ((1u << kKeyBits) - 1u));
            keys[kk][j / 3] |= field << (kKeyBits * (2 - (j % 3)));
        }
    }
    return ok;
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

// Look a packed key up in one set's table; on a hit add b * values to acc.
// The table always has an empty slot (load factor <= 1/2), so probing ends at
// the key or at an empty slot; the probe count is bounded by the capacity.
template <int KW, int V>
__device__ __forceinline__ bool probe_accumulate(const uint4 *__restrict__ table, const SetTable &st,
                                                 const uint64_t (&key)[KW], float bw, float (&acc)[V])
{
    using L = SlotLayout<KW, V>;
    uint32_t h = hash_key<KW>(key) & st.mask;
    const uint4 *base = table + st.slot_base * L::kNQ;
    for (uint32_t n = 0; n <= st.mask; ++n) {
        uint4 q[L::kNQ];
#pragma unroll
        for (int i = 0; i < L::kNQ; ++i) q[i] = base[(size_t)h * L::kNQ + i];
        const uint64_t w0 = (uint64_t)q[0].x | ((uint64_t)q[0].y << 32);
        if (w0 == kKeyEmpty) return false;
        bool eq = (w0 == key[0]);
        if constexpr (KW >= 2) eq = eq && (((uint64_t)q[0].z | ((uint64_t)q[0].w << 32)) == key[1]);
        if (eq) {
            uint32_t words[4 * L::kNQ];
#pragma unroll
            for (int i = 0; i < L::kNQ; ++i) {
                words[4 * i + 0] = q[i].x;
                words[4 * i + 1] = q[i].y;
                words[4 * i + 2] = q[i].z;
                words[4 * i + 3] = q[i].w;
            }
#pragma unroll
            for (int c = 0; c < V; ++c) acc[c] = fmaf(bw, __uint_as_float(words[2 * KW + c]), acc[c]);
            return true;
        }
        h = (h + 1) & st.mask;
    }
    return false;
}

}  // namespace fr
