// Lattice build (splat of the observation, Sec. 3.2 / Sec. 4.2).
//
// Pipeline for all sets of a cloud at once:
//   1. embed      one thread per observation point: D vertex keys + weights
//                 written as records r = point * D + k.
//   2. insert     one thread per record: insert the key into a provisional
//                 open-addressing table of the record's set (32-bit owner CAS,
//                 keys compared through the owner record, so keys of any
//                 width work); count incidences per slot.
//   3. compact    exclusive scan of occupied slots -> vertex ids; per-vertex
//                 key and occupancy.
//   4. values     sorted mode: stable LSD radix sort of the records by vertex
//                 id (records start in point order, so each vertex's records
//                 stay in point order), then one thread per vertex sums
//                 b * [1, y, n_y] in that order in binary64 -> bitwise
//                 deterministic.  Atomic mode: binary32 hardware atomics.
//   5. final      per set, a table of capacity pow2 >= 2 n_v whose slots hold
//                 the packed key and the binary32 values inline, so that a
//                 lookup in the E-step is one 32/48-byte read.
#include "fr_internal.h"

namespace fr {

// ---------------------------------------------------------------------------
// Device-wide exclusive scan of u32 (optionally of the flags x != 0)
// ---------------------------------------------------------------------------
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t t = __shfl_up(v, off, 64);
        if (lane >= off) v += t;
    }
    return v;
}

template <bool FLAGS>
__global__ void __launch_bounds__(kScanThreads) k_scan_tile(const uint32_t *in, uint32_t *out, uint32_t *bsum, size_t n)
{
    __shared__ uint32_t wsum[kScanThreads / 64];
    const size_t base = (size_t)blockIdx.x * kScanTile + (size_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t tot = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const size_t idx = base + i;
        uint32_t x = idx < n ? in[idx] : 0u;
        if (FLAGS) x = x != 0u;
        v[i] = tot;
        tot += x;
    }
    const uint32_t incl = wave_inclusive_scan(tot);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    uint32_t wpre = 0;
    for (int w = 0; w < wave; ++w) wpre += wsum[w];
    const uint32_t excl = wpre + incl - tot;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i)
        if (base + i < n) out[base + i] = excl + v[i];
    if (bsum != nullptr && threadIdx.x == kScanThreads - 1) bsum[blockIdx.x] = excl + tot;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_add(uint32_t *out, const uint32_t *bsum, size_t n)
{
    const uint32_t add = bsum[blockIdx.x];
    const size_t base = (size_t)blockIdx.x * kScanTile;
    for (int i = threadIdx.x; i < kScanTile; i += kScanThreads) {
        const size_t idx = base + i;
        if (idx < n) out[idx] += add;
    }
}

fr_status scan_exclusive_u32(fr_ctx *ctx, const uint32_t *in, uint32_t *out, size_t n, bool flags, hipStream_t st)
{
    if (n == 0) return FR_OK;
    const size_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb == 1) {
        if (flags) k_scan_tile<true><<<1, kScanThreads, 0, st>>>(in, out, nullptr, n);
        else k_scan_tile<false><<<1, kScanThreads, 0, st>>>(in, out, nullptr, n);
        FR_HIP(hipGetLastError());
        return FR_OK;
    }
    DevBuf bs;
    FR_TRY(bs.alloc(ctx, nb * sizeof(uint32_t)));
    if (flags) k_scan_tile<true><<<(unsigned)nb, kScanThreads, 0, st>>>(in, out, bs.as<uint32_t>(), n);
    else k_scan_tile<false><<<(unsigned)nb, kScanThreads, 0, st>>>(in, out, bs.as<uint32_t>(), n);
    FR_HIP(hipGetLastError());
    FR_TRY(scan_exclusive_u32(ctx, bs.as<uint32_t>(), bs.as<uint32_t>(), nb, false, st));
    k_scan_add<<<(unsigned)nb, kScanThreads, 0, st>>>(out, bs.as<uint32_t>(), n);
    FR_HIP(hipGetLastError());
    // bs is freed by the destructor: DevBuf frees after a stream sync (see dev_free).
    FR_HIP(hipStreamSynchronize(st));
    return FR_OK;
}

// ---------------------------------------------------------------------------
// Stable LSD radix sort of (u32 key, u32 value) pairs, 8-bit digits.
// ---------------------------------------------------------------------------
constexpr int kRsThreads = 256;
constexpr int kRsRounds = 16;                        // rounds of 64 items per wave
constexpr int kRsWaves = kRsThreads / 64;
constexpr int kRsTile = kRsThreads * kRsRounds;      // 4096 items per block

__global__ void __launch_bounds__(kRsThreads) k_rs_hist(const uint32_t *keys, size_t n, int shift, uint32_t *hist,
                                                        uint32_t nblocks)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const size_t base = (size_t)blockIdx.x * kRsTile;
    for (int i = threadIdx.x; i < kRsTile; i += kRsThreads) {
        const size_t idx = base + i;
        if (idx < n) atomicAdd(&h[(keys[idx] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(size_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// Each wave ranks its contiguous 1024 items in 16 rounds of 64 (lane order =
// item order): lanes with equal digits are found with 8 ballots, and a
// per-wave LDS counter per digit carries the running count between rounds.
// Waves are then ordered by a per-digit exclusive prefix, so the rank of an
// item among equal digits of the block follows item order (stability).
__global__ void __launch_bounds__(kRsThreads) k_rs_scatter(const uint32_t *kin, const uint32_t *vin, uint32_t *kout,
                                                           uint32_t *vout, size_t n, int shift,
                                                           const uint32_t *hist_scan, uint32_t nblocks)
{
    __shared__ uint32_t wcnt[kRsWaves][256];
    __shared__ uint32_t gbase[256];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int w = 0; w < kRsWaves; ++w) wcnt[w][threadIdx.x] = 0;
    gbase[threadIdx.x] = hist_scan[(size_t)threadIdx.x * nblocks + blockIdx.x];
    __syncthreads();

    const size_t base = (size_t)blockIdx.x * kRsTile + (size_t)wave * (64 * kRsRounds);
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint32_t key[kRsRounds], val[kRsRounds], lrank[kRsRounds];
#pragma unroll
    for (int r = 0; r < kRsRounds; ++r) {
        const size_t idx = base + (size_t)r * 64 + lane;
        const bool valid = idx < n;
        key[r] = valid ? kin[idx] : 0u;
        val[r] = valid ? vin[idx] : 0u;
        const uint32_t digit = (key[r] >> shift) & 255u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const bool on = (digit >> bit) & 1u;
            const uint64_t m = __ballot(on);
            peers &= on ? m : ~m;
        }
        const uint32_t before = wcnt[wave][digit];
        lrank[r] = before + (uint32_t)__popcll(peers & lt);
        __builtin_amdgcn_wave_barrier();
        if (valid && (__ffsll((long long)peers) - 1) == lane) wcnt[wave][digit] = before + (uint32_t)__popcll(peers);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    {
        uint32_t run = 0;
#pragma unroll
        for (int w = 0; w < kRsWaves; ++w) {
            const uint32_t t = wcnt[w][threadIdx.x];
            wcnt[w][threadIdx.x] = run;
            run += t;
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kRsRounds; ++r) {
        const size_t idx = base + (size_t)r * 64 + lane;
        if (idx < n) {
            const uint32_t digit = (key[r] >> shift) & 255u;
            const size_t pos = (size_t)gbase[digit] + wcnt[wave][digit] + lrank[r];
            kout[pos] = key[r];
            vout[pos] = val[r];
        }
    }
}

// Sorts keys/vals in place (ping-pong through tk/tv) by the low `bits` bits.
static fr_status radix_sort_pairs(fr_ctx *ctx, uint32_t *keys, uint32_t *vals, uint32_t *tk, uint32_t *tv, size_t n,
                                  int bits, hipStream_t st)
{
    if (n <= 1 || bits <= 0) return FR_OK;
    const uint32_t nb = (uint32_t)((n + kRsTile - 1) / kRsTile);
    DevBuf hist;
    FR_TRY(hist.alloc(ctx, (size_t)256 * nb * sizeof(uint32_t)));
    uint32_t *ka = keys, *va = vals, *kb = tk, *vb = tv;
    int passes = 0;
    for (int shift = 0; shift < bits; shift += 8, ++passes) {
        k_rs_hist<<<nb, kRsThreads, 0, st>>>(ka, n, shift, hist.as<uint32_t>(), nb);
        FR_HIP(hipGetLastError());
        FR_TRY(scan_exclusive_u32(ctx, hist.as<uint32_t>(), hist.as<uint32_t>(), (size_t)256 * nb, false, st));
        k_rs_scatter<<<nb, kRsThreads, 0, st>>>(ka, va, kb, vb, n, shift, hist.as<uint32_t>(), nb);
        FR_HIP(hipGetLastError());
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    if (ka != keys) {
        FR_HIP(hipMemcpyAsync(keys, ka, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, st));
        FR_HIP(hipMemcpyAsync(vals, va, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, st));
    }
    FR_HIP(hipStreamSynchronize(st));
    return FR_OK;
}

// ---------------------------------------------------------------------------
// Build kernels
// ---------------------------------------------------------------------------
struct Pts {
    const float *x, *y, *z, *nx, *ny, *nz;
};

template <int d>
__global__ void __launch_bounds__(256) k_embed_obs(Pts pts, TileMap tm, float4 k0, float4 k1, uint64_t *rec_key,
                                                  float *rec_b, size_t R, int32_t *err)
{
    constexpr int D = d + 1;
    constexpr int KW = KeyWords<d>::value;
    const int32_t t = logical_tile(tm);
    if (t >= tm.n_tiles) return;
    const int32_t s = tile_segment(tm, t);
    const int64_t i = tm.seg_off[s] + (int64_t)(t - tm.seg_tile[s]) * tm.tile + threadIdx.x;
    if (i >= tm.seg_off[s + 1]) return;
    float p[d];
    float kk[d];
    const float kall[8] = {k0.x, k0.y, k0.z, k0.w, k1.x, k1.y, k1.z, k1.w};
#pragma unroll
    for (int j = 0; j < d; ++j) kk[j] = kall[j];
    p[0] = pts.x[i];
    p[1] = pts.y[i];
    p[2] = pts.z[i];
    if constexpr (d == 6) {
        p[3] = pts.nx[i];
        p[4] = pts.ny[i];
        p[5] = pts.nz[i];
    }
    uint64_t keys[D][KW];
    float b[D];
    if (!embed<d>(p, kk, keys, b)) atomicOr(err, 1);
#pragma unroll
    for (int v = 0; v < D; ++v) {
        const size_t r = (size_t)i * D + v;
#pragma unroll
        for (int w = 0; w < KW; ++w) rec_key[(size_t)w * R + r] = keys[v][w];
        rec_b[r] = b[v];
    }
}

// One thread per record: find or claim the record's key in the provisional table.
template <int KW>
__global__ void __launch_bounds__(256) k_insert_records(TileMap tm, const SetTable *tables, const uint64_t *rec_key,
                                                       size_t R, uint32_t *own, uint32_t *occ, uint32_t *rec_slot)
{
    const int32_t t = logical_tile(tm);
    if (t >= tm.n_tiles) return;
    const int32_t s = tile_segment(tm, t);
    const int64_t r = tm.seg_off[s] + (int64_t)(t - tm.seg_tile[s]) * tm.tile + threadIdx.x;
    if (r >= tm.seg_off[s + 1]) return;
    uint64_t key[KW];
#pragma unroll
    for (int w = 0; w < KW; ++w) key[w] = rec_key[(size_t)w * R + r];
    const SetTable st = tables[s];
    uint32_t h = hash_key<KW>(key) & st.mask;
    for (uint32_t n = 0; n <= st.mask; ++n) {
        const size_t slot = st.slot_base + h;
        const uint32_t old = atomicCAS(&own[slot], kOwnerEmpty, (uint32_t)r);
        bool mine = (old == kOwnerEmpty);
        if (!mine) {
            mine = true;
#pragma unroll
            for (int w = 0; w < KW; ++w) mine = mine && (rec_key[(size_t)w * R + old] == key[w]);
        }
        if (mine) {
            rec_slot[r] = (uint32_t)slot;
            atomicAdd(&occ[slot], 1u);
            return;
        }
        h = (h + 1) & st.mask;
    }
}

// Per-set vertex counts from the scanned occupancy flags (one thread per set).
__global__ void k_set_counts(const SetTable *tables, int32_t n_sets, const uint32_t *vid, const uint32_t *occ,
                             size_t n_slots, uint32_t *counts)
{
    const int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_sets) return;
    const size_t b0 = tables[s].slot_base;
    const size_t b1 = b0 + (size_t)tables[s].mask + 1;
    const uint32_t total_end = (b1 < n_slots) ? vid[b1] : (vid[n_slots - 1] + (occ[n_slots - 1] != 0u ? 1u : 0u));
    counts[s] = total_end - vid[b0];
}

template <int KW>
__global__ void __launch_bounds__(256) k_compact_slots(size_t n_slots, const uint32_t *occ, const uint32_t *own,
                                                      const uint32_t *vid, const uint64_t *rec_key, size_t R,
                                                      uint64_t *vkey, uint32_t *vocc, size_t NV)
{
    const size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n_slots) return;
    const uint32_t c = occ[j];
    if (c == 0u) return;
    const uint32_t v = vid[j];
    const uint32_t r = own[j];
#pragma unroll
    for (int w = 0; w < KW; ++w) vkey[(size_t)w * NV + v] = rec_key[(size_t)w * R + r];
    vocc[v] = c;
}

__global__ void __launch_bounds__(256) k_record_vertex(size_t R, const uint32_t *rec_slot, const uint32_t *vid,
                                                      uint32_t *rvid, uint32_t *rid)
{
    const size_t r = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    rvid[r] = vid[rec_slot[r]];
    rid[r] = (uint32_t)r;
}

// Sorted mode: ordered binary64 sums per vertex.
template <int D, int V>
__global__ void __launch_bounds__(256) k_vertex_sum_sorted(size_t NV, const uint32_t *voff, const uint32_t *vocc,
                                                          const uint32_t *rid_sorted, const float *rec_b, Pts pts,
                                                          float *vval)
{
    const size_t v = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= NV) return;
    double acc[V];
#pragma unroll
    for (int c = 0; c < V; ++c) acc[c] = 0.0;
    const uint32_t q0 = voff[v], q1 = q0 + vocc[v];
    for (uint32_t q = q0; q < q1; ++q) {
        const uint32_t r = rid_sorted[q];
        const uint32_t i = r / D;
        const double bw = (double)rec_b[r];
        acc[0] += bw;
        acc[1] += bw * (double)pts.x[i];
        acc[2] += bw * (double)pts.y[i];
        acc[3] += bw * (double)pts.z[i];
        if constexpr (V == 7) {
            acc[4] += bw * (double)pts.nx[i];
            acc[5] += bw * (double)pts.ny[i];
            acc[6] += bw * (double)pts.nz[i];
        }
    }
#pragma unroll
    for (int c = 0; c < V; ++c) vval[(size_t)c * NV + v] = (float)acc[c];
}

// Atomic mode: one thread per record, binary32 hardware atomics.
template <int D, int V>
__global__ void __launch_bounds__(256) k_vertex_sum_atomic(size_t R, const uint32_t *rec_slot, const uint32_t *vid,
                                                          const float *rec_b, Pts pts, float *vval, size_t NV)
{
    const size_t r = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    const uint32_t v = vid[rec_slot[r]];
    const size_t i = r / D;
    const float bw = rec_b[r];
    unsafeAtomicAdd(&vval[v], bw);
    unsafeAtomicAdd(&vval[NV + v], bw * pts.x[i]);
    unsafeAtomicAdd(&vval[2 * NV + v], bw * pts.y[i]);
    unsafeAtomicAdd(&vval[3 * NV + v], bw * pts.z[i]);
    if constexpr (V == 7) {
        unsafeAtomicAdd(&vval[4 * NV + v], bw * pts.nx[i]);
        unsafeAtomicAdd(&vval[5 * NV + v], bw * pts.ny[i]);
        unsafeAtomicAdd(&vval[6 * NV + v], bw * pts.nz[i]);
    }
}

// One thread per vertex: claim a slot of the set's final table and write the
// packed key and values inline.  Keys are unique, so a claimed slot is never
// compared.
template <int KW, int V>
__global__ void __launch_bounds__(256) k_final_insert(TileMap tm, const SetTable *tables, const uint64_t *vkey,
                                                     const float *vval, size_t NV, uint32_t *own, uint4 *table)
{
    using L = SlotLayout<KW, V>;
    const int32_t t = logical_tile(tm);
    if (t >= tm.n_tiles) return;
    const int32_t s = tile_segment(tm, t);
    const int64_t v = tm.seg_off[s] + (int64_t)(t - tm.seg_tile[s]) * tm.tile + threadIdx.x;
    if (v >= tm.seg_off[s + 1]) return;
    uint64_t key[KW];
#pragma unroll
    for (int w = 0; w < KW; ++w) key[w] = vkey[(size_t)w * NV + v];
    const SetTable st = tables[s];
    uint32_t h = hash_key<KW>(key) & st.mask;
    for (uint32_t n = 0; n <= st.mask; ++n) {
        const size_t slot = st.slot_base + h;
        if (atomicCAS(&own[slot], kOwnerEmpty, (uint32_t)v) == kOwnerEmpty) {
            uint32_t words[4 * L::kNQ];
#pragma unroll
            for (int i = 0; i < 4 * L::kNQ; ++i) words[i] = 0u;
#pragma unroll
            for (int w = 0; w < KW; ++w) {
                words[2 * w] = (uint32_t)key[w];
                words[2 * w + 1] = (uint32_t)(key[w] >> 32);
            }
#pragma unroll
            for (int c = 0; c < V; ++c) words[2 * KW + c] = __float_as_uint(vval[(size_t)c * NV + v]);
#pragma unroll
            for (int i = 0; i < L::kNQ; ++i)
                table[slot * L::kNQ + i] = make_uint4(words[4 * i], words[4 * i + 1], words[4 * i + 2], words[4 * i + 3]);
            return;
        }
        h = (h + 1) & st.mask;
    }
}

// ---------------------------------------------------------------------------
// Host driver
// ---------------------------------------------------------------------------
static uint32_t next_pow2(uint64_t x)
{
    uint64_t p = 16;
    while (p < x) p <<= 1;
    return (uint32_t)p;
}

static inline unsigned blocks_for(size_t n, int threads) { return (unsigned)((n + threads - 1) / threads); }

// Tile map over explicit offsets (device copy kept in `buf`).
static fr_status make_offset_map(fr_ctx *ctx, const std::vector<int64_t> &off, int32_t tile, hipStream_t st,
                                 DevBuf &buf, TileMap &tm)
{
    const int32_t n = (int32_t)off.size() - 1;
    std::vector<int32_t> tiles(n + 1, 0), sets(n);
    for (int32_t s = 0; s < n; ++s) {
        tiles[s + 1] = tiles[s] + (int32_t)((off[s + 1] - off[s] + tile - 1) / tile);
        sets[s] = s;
    }
    const size_t b_off = sizeof(int64_t) * (n + 1), b_tile = sizeof(int32_t) * (n + 1), b_set = sizeof(int32_t) * n;
    FR_TRY(buf.alloc(ctx, b_off + b_tile + b_set));
    char *p = buf.as<char>();
    FR_HIP(hipMemcpyAsync(p, off.data(), b_off, hipMemcpyHostToDevice, st));
    FR_HIP(hipMemcpyAsync(p + b_off, tiles.data(), b_tile, hipMemcpyHostToDevice, st));
    FR_HIP(hipMemcpyAsync(p + b_off + b_tile, sets.data(), b_set, hipMemcpyHostToDevice, st));
    tm.seg_off = reinterpret_cast<const int64_t *>(p);
    tm.seg_tile = reinterpret_cast<const int32_t *>(p + b_off);
    tm.seg_set = reinterpret_cast<const int32_t *>(p + b_off + b_tile);
    tm.n_seg = n;
    tm.n_tiles = tiles[n];
    tm.tile = tile;
    tm.xcd_chunk = 0;
    FR_HIP(hipStreamSynchronize(st));   // host vectors go out of scope
    return FR_OK;
}

template <int d, int V>
static fr_status build_impl(fr_ctx *ctx, const fr_cloud *obs, hipStream_t st, fr_lattice *lat)
{
    constexpr int D = d + 1;
    constexpr int KW = KeyWords<d>::value;
    const int32_t S = obs->n_sets;
    const int64_t N = cloud_points(obs);
    const size_t R = (size_t)N * D;
    if (R >= 0xFFFFFFF0ull) {
        set_error("fr_lattice_build: %lld records exceed the 32-bit record index", (long long)R);
        return FR_EINVAL;
    }
    Pts pts{obs->x, obs->y, obs->z, obs->nx, obs->ny, obs->nz};

    // provisional tables: capacity pow2 >= 2 * records of the set
    std::vector<SetTable> t1(S);
    uint64_t n1 = 0;
    for (int32_t s = 0; s < S; ++s) {
        const uint64_t rs = (uint64_t)(obs->offsets[s + 1] - obs->offsets[s]) * D;
        const uint32_t cap = next_pow2(2 * rs);
        t1[s] = SetTable{n1, cap - 1, 0};
        n1 += cap;
    }
    if (n1 >= 0xFFFFFFF0ull) {
        set_error("fr_lattice_build: provisional table too large");
        return FR_EINVAL;
    }

    DevBuf rec_key, rec_b, rec_slot, own1, occ1, vid, t1_d, ptmap, rtmap;
    FR_TRY(rec_key.alloc(ctx, R * KW * sizeof(uint64_t)));
    FR_TRY(rec_b.alloc(ctx, R * sizeof(float)));
    FR_TRY(rec_slot.alloc(ctx, R * sizeof(uint32_t)));
    FR_TRY(own1.alloc(ctx, n1 * sizeof(uint32_t)));
    FR_TRY(occ1.alloc(ctx, n1 * sizeof(uint32_t)));
    FR_TRY(vid.alloc(ctx, n1 * sizeof(uint32_t)));
    FR_TRY(t1_d.alloc(ctx, S * sizeof(SetTable)));
    FR_HIP(hipMemcpyAsync(t1_d.p, t1.data(), S * sizeof(SetTable), hipMemcpyHostToDevice, st));
    FR_HIP(hipMemsetAsync(own1.p, 0xFF, n1 * sizeof(uint32_t), st));
    FR_HIP(hipMemsetAsync(occ1.p, 0, n1 * sizeof(uint32_t), st));
    FR_HIP(hipMemsetAsync(lat->err_d, 0, sizeof(int32_t), st));

    // 1. embed
    std::vector<int64_t> poff(obs->offsets, obs->offsets + S + 1);
    TileMap ptm{}, rtm{};
    FR_TRY(make_offset_map(ctx, poff, 256, st, ptmap, ptm));
    const float4 k0 = make_float4(lat->k[0], lat->k[1], lat->k[2], lat->k[3]);
    const float4 k1 = make_float4(lat->k[4], lat->k[5], lat->k[6], lat->k[7]);
    if (ptm.n_tiles > 0) {
        k_embed_obs<d><<<ptm.n_tiles, 256, 0, st>>>(pts, ptm, k0, k1, rec_key.as<uint64_t>(), rec_b.as<float>(), R,
                                                    lat->err_d);
        FR_HIP(hipGetLastError());
    }
    // 2. insert
    std::vector<int64_t> roff(S + 1);
    for (int32_t s = 0; s <= S; ++s) roff[s] = obs->offsets[s] * D;
    FR_TRY(make_offset_map(ctx, roff, 256, st, rtmap, rtm));
    if (rtm.n_tiles > 0) {
        k_insert_records<KW><<<rtm.n_tiles, 256, 0, st>>>(rtm, t1_d.as<SetTable>(), rec_key.as<uint64_t>(), R,
                                                          own1.as<uint32_t>(), occ1.as<uint32_t>(),
                                                          rec_slot.as<uint32_t>());
        FR_HIP(hipGetLastError());
    }
    // 3. compact
    FR_TRY(scan_exclusive_u32(ctx, occ1.as<uint32_t>(), vid.as<uint32_t>(), n1, true, st));
    DevBuf counts_d;
    FR_TRY(counts_d.alloc(ctx, S * sizeof(uint32_t)));
    k_set_counts<<<blocks_for(S, 64), 64, 0, st>>>(t1_d.as<SetTable>(), S, vid.as<uint32_t>(), occ1.as<uint32_t>(),
                                                    n1, counts_d.as<uint32_t>());
    FR_HIP(hipGetLastError());
    std::vector<uint32_t> counts(S);
    int32_t err_h = 0;
    FR_HIP(hipMemcpyAsync(counts.data(), counts_d.p, S * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    FR_HIP(hipMemcpyAsync(&err_h, lat->err_d, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    FR_HIP(hipStreamSynchronize(st));
    if (err_h != 0) {
        set_error("fr_lattice_build: a lattice coordinate left [-2^20, 2^20); increase sigma or centre the cloud");
        return FR_ERANGE;
    }
    lat->vbase.assign(S + 1, 0);
    for (int32_t s = 0; s < S; ++s) lat->vbase[s + 1] = lat->vbase[s] + counts[s];
    const size_t NV = (size_t)lat->vbase[S];
    lat->n_vertices_total = (int64_t)NV;

    // vertex arrays (kept for export)
    lat->vert_bytes = NV * (KW * sizeof(uint64_t) + sizeof(uint32_t) + V * sizeof(float)) + 64;
    {
        void *p = nullptr;
        FR_TRY(dev_alloc(ctx, &p, lat->vert_bytes));
        lat->charged += lat->vert_bytes;
        char *c = static_cast<char *>(p);
        lat->vkey = reinterpret_cast<uint64_t *>(c);
        lat->vval = reinterpret_cast<float *>(c + NV * KW * sizeof(uint64_t));
        lat->vocc = reinterpret_cast<uint32_t *>(c + NV * (KW * sizeof(uint64_t) + V * sizeof(float)));
    }
    if (NV > 0) {
        k_compact_slots<KW><<<blocks_for(n1, 256), 256, 0, st>>>(n1, occ1.as<uint32_t>(), own1.as<uint32_t>(),
                                                                 vid.as<uint32_t>(), rec_key.as<uint64_t>(), R,
                                                                 lat->vkey, lat->vocc, NV);
        FR_HIP(hipGetLastError());
    }

    // 4. values
    if (NV > 0) {
        if (lat->splat == FR_SPLAT_SORTED) {
            DevBuf rvid, rid, tk, tv, voff;
            FR_TRY(rvid.alloc(ctx, R * sizeof(uint32_t)));
            FR_TRY(rid.alloc(ctx, R * sizeof(uint32_t)));
            FR_TRY(tk.alloc(ctx, R * sizeof(uint32_t)));
            FR_TRY(tv.alloc(ctx, R * sizeof(uint32_t)));
            FR_TRY(voff.alloc(ctx, NV * sizeof(uint32_t)));
            k_record_vertex<<<blocks_for(R, 256), 256, 0, st>>>(R, rec_slot.as<uint32_t>(), vid.as<uint32_t>(),
                                                                 rvid.as<uint32_t>(), rid.as<uint32_t>());
            FR_HIP(hipGetLastError());
            int bits = 0;
            while (bits < 32 && (NV - 1) >> bits) ++bits;
            FR_TRY(radix_sort_pairs(ctx, rvid.as<uint32_t>(), rid.as<uint32_t>(), tk.as<uint32_t>(),
                                    tv.as<uint32_t>(), R, bits, st));
            FR_TRY(scan_exclusive_u32(ctx, lat->vocc, voff.as<uint32_t>(), NV, false, st));
            k_vertex_sum_sorted<D, V><<<blocks_for(NV, 256), 256, 0, st>>>(
                NV, voff.as<uint32_t>(), lat->vocc, rid.as<uint32_t>(), rec_b.as<float>(), pts, lat->vval);
            FR_HIP(hipGetLastError());
            FR_HIP(hipStreamSynchronize(st));
        } else {
            FR_HIP(hipMemsetAsync(lat->vval, 0, NV * V * sizeof(float), st));
            k_vertex_sum_atomic<D, V><<<blocks_for(R, 256), 256, 0, st>>>(R, rec_slot.as<uint32_t>(),
                                                                           vid.as<uint32_t>(), rec_b.as<float>(), pts,
                                                                           lat->vval, NV);
            FR_HIP(hipGetLastError());
        }
    }

    // 5. final tables
    using L = SlotLayout<KW, V>;
    lat->sets_h.resize(S);
    uint64_t n2 = 0;
    for (int32_t s = 0; s < S; ++s) {
        const uint32_t cap = next_pow2(2 * (uint64_t)counts[s]);
        lat->sets_h[s] = SetTable{n2, cap - 1, counts[s]};
        n2 += cap;
    }
    lat->table_bytes = n2 * L::kBytes;
    FR_TRY(dev_alloc(ctx, &lat->table, lat->table_bytes));
    lat->charged += lat->table_bytes;
    FR_TRY(dev_alloc(ctx, reinterpret_cast<void **>(&lat->sets_d), S * sizeof(SetTable)));
    lat->charged += S * sizeof(SetTable);
    FR_HIP(hipMemcpyAsync(lat->sets_d, lat->sets_h.data(), S * sizeof(SetTable), hipMemcpyHostToDevice, st));
    FR_HIP(hipMemsetAsync(lat->table, 0xFF, lat->table_bytes, st));
    if (NV > 0) {
        DevBuf own2, vtmap;
        FR_TRY(own2.alloc(ctx, n2 * sizeof(uint32_t)));
        FR_HIP(hipMemsetAsync(own2.p, 0xFF, n2 * sizeof(uint32_t), st));
        TileMap vtm{};
        FR_TRY(make_offset_map(ctx, lat->vbase, 256, st, vtmap, vtm));
        k_final_insert<KW, V><<<vtm.n_tiles, 256, 0, st>>>(vtm, lat->sets_d, lat->vkey, lat->vval, NV,
                                                           own2.as<uint32_t>(), static_cast<uint4 *>(lat->table));
        FR_HIP(hipGetLastError());
        FR_HIP(hipStreamSynchronize(st));
    }
    FR_HIP(hipStreamSynchronize(st));
    return FR_OK;
}

fr_status build_lattice(fr_ctx *ctx, const fr_cloud *obs, const fr_lattice_params *prm, hipStream_t st,
                        fr_lattice *lat)
{
    if (prm->feat == 3 && prm->values == 4) return build_impl<3, 4>(ctx, obs, st, lat);
    if (prm->feat == 3 && prm->values == 7) return build_impl<3, 7>(ctx, obs, st, lat);
    if (prm->feat == 6 && prm->values == 4) return build_impl<6, 4>(ctx, obs, st, lat);
    if (prm->feat == 6 && prm->values == 7) return build_impl<6, 7>(ctx, obs, st, lat);
    set_error("fr_lattice_build: unsupported feat=%d values=%d", prm->feat, prm->values);
    return FR_EINVAL;
}

}  // namespace fr
