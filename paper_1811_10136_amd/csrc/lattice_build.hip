// Lattice build (splat of the observation, Sec. 3.2 / Sec. 4.2).
//
// Pipeline for all sets of a cloud at once:
//   1. embed      one thread per observation point: D vertex keys + weights
//                 written as records r = point * D + k.
//   2. insert     one thread per record: the records of a tile are merged by
//                 key in LDS, then one record per distinct key inserts it
//                 into a provisional open-addressing table of the record's
//                 set (32-bit owner CAS, keys compared through the owner
//                 record, so keys of any width work).
//   3. vertices   the record that owns each slot defines a vertex; an
//                 exclusive scan over records numbers the vertices in owner
//                 order (so vertex ids follow point order) and gives each
//                 set's contiguous vertex range.
//   4. values     sorted mode: stable LSD radix sort of the records by vertex
//                 id (records start in point order, so each vertex's records
//                 stay in point order); segment lengths give the occupancy
//                 and one thread per vertex sums b * [1, y, n_y] in that
//                 order in binary64 -> bitwise deterministic.  Atomic mode:
//                 binary32 hardware atomics and an occupancy counter.
//   5. final      per set, a bucketed two-choice cuckoo table (load factor
//                 <= 0.5, two slots of key + values per bucket): an E-step
//                 lookup reads one bucket line, and a second one only when
//                 the first bucket is full without the key.
#include <algorithm>

#include <cstring>

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

// MODE 0: scan the values; 1: scan (x != 0); 2: scan (x != 0xFFFFFFFF).
template <int MODE>
__global__ void __launch_bounds__(kScanThreads) k_scan_tile(const uint32_t *in, uint32_t *out, uint32_t *bsum, size_t n)
{
    __shared__ uint32_t wsum[kScanThreads / 64];
    const size_t base = (size_t)blockIdx.x * kScanTile + (size_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t tot = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const size_t idx = base + i;
        uint32_t x = idx < n ? in[idx] : (MODE == 2 ? kOwnerEmpty : 0u);
        if (MODE == 1) x = x != 0u;
        if (MODE == 2) x = x != kOwnerEmpty;
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

// One workgroup scans up to kScanSmall values in tiles, carrying the running
// total: one launch instead of three for the short scans of small builds
// (longer inputs are faster spread over workgroups: about 2 us per tile here).
constexpr size_t kScanSmall = 8 * (size_t)kScanTile;

__global__ void __launch_bounds__(kScanThreads) k_scan_small(const uint32_t *in, uint32_t *out, size_t n)
{
    __shared__ uint32_t wsum[kScanThreads / 64];
    __shared__ uint32_t carry;
    if (threadIdx.x == 0) carry = 0u;
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (size_t t0 = 0; t0 < n; t0 += kScanTile) {
        const size_t base = t0 + (size_t)threadIdx.x * kScanItems;
        uint32_t v[kScanItems];
        uint32_t tot = 0;
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            const uint32_t x = base + i < n ? in[base + i] : 0u;
            v[i] = tot;
            tot += x;
        }
        const uint32_t incl = wave_inclusive_scan(tot);
        if (lane == 63) wsum[wave] = incl;
        __syncthreads();
        uint32_t pre = carry;
        for (int w = 0; w < wave; ++w) pre += wsum[w];
        const uint32_t excl = pre + incl - tot;
#pragma unroll
        for (int i = 0; i < kScanItems; ++i)
            if (base + i < n) out[base + i] = excl + v[i];
        __syncthreads();   // every thread has read carry and wsum
        if (threadIdx.x == kScanThreads - 1) carry = excl + tot;
        __syncthreads();
    }
}

size_t scan_ws_words(size_t n)
{
    size_t words = 0;
    while (n > (size_t)kScanTile) {
        n = (n + kScanTile - 1) / kScanTile;
        words += n;
    }
    return words;
}

fr_status scan_exclusive_u32(fr_ctx *ctx, const uint32_t *in, uint32_t *out, size_t n, int mode, hipStream_t st,
                             uint32_t *ws)
{
    if (n == 0) return FR_OK;
    const size_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb > 1 && n <= kScanSmall && mode == 0) {
        k_scan_small<<<1, kScanThreads, 0, st>>>(in, out, n);
        FR_HIP(hipGetLastError());
        return FR_OK;
    }
    if (nb == 1) {
        if (mode == 1) k_scan_tile<1><<<1, kScanThreads, 0, st>>>(in, out, nullptr, n);
        else if (mode == 2) k_scan_tile<2><<<1, kScanThreads, 0, st>>>(in, out, nullptr, n);
        else k_scan_tile<0><<<1, kScanThreads, 0, st>>>(in, out, nullptr, n);
        FR_HIP(hipGetLastError());
        return FR_OK;
    }
    DevBuf bs;
    uint32_t *bsum = ws;
    if (bsum == nullptr) {
        FR_TRY(bs.alloc(ctx, nb * sizeof(uint32_t)));
        bs.stream = st;   // freed in the order of st: no wait here
        bsum = bs.as<uint32_t>();
    }
    if (mode == 1) k_scan_tile<1><<<(unsigned)nb, kScanThreads, 0, st>>>(in, out, bsum, n);
    else if (mode == 2) k_scan_tile<2><<<(unsigned)nb, kScanThreads, 0, st>>>(in, out, bsum, n);
    else k_scan_tile<0><<<(unsigned)nb, kScanThreads, 0, st>>>(in, out, bsum, n);
    FR_HIP(hipGetLastError());
    FR_TRY(scan_exclusive_u32(ctx, bsum, bsum, nb, 0, st, ws != nullptr ? ws + nb : nullptr));
    k_scan_add<<<(unsigned)nb, kScanThreads, 0, st>>>(out, bsum, n);
    FR_HIP(hipGetLastError());
    return FR_OK;
}

// ---------------------------------------------------------------------------
// Stable LSD radix sort of (u32 key, u32 value) pairs, 8-bit digits.
// ---------------------------------------------------------------------------
constexpr int kRsThreads = 256;
constexpr int kRsRounds = 16;                        // rounds of 64 items per wave
constexpr int kRsWaves = kRsThreads / 64;
constexpr int kRsTile = kRsThreads * kRsRounds;      // 4096 items per block

// n_dev (or NULL): a device count that bounds n (blocks past it count nothing).
__device__ __forceinline__ size_t dev_count(size_t n, const uint32_t *n_dev)
{
    return n_dev != nullptr ? min(n, (size_t)*n_dev) : n;
}

// A rebuild in place runs its kernels without reading failures back in
// between; a kernel whose inputs an earlier failure left partly unset (record
// slots of an overflowed insertion, vertex slots of a cuckoo pass that gave
// up) is given the failure word and returns at once when it is set.
__device__ __forceinline__ bool aborted(const uint32_t *fail) { return fail != nullptr && *fail != 0u; }

__global__ void __launch_bounds__(kRsThreads) k_rs_hist(const uint32_t *keys, size_t n, const uint32_t *n_dev,
                                                        int shift, uint32_t *hist, uint32_t nblocks)
{
    __shared__ uint32_t h[256];
    n = dev_count(n, n_dev);
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
// item among equal digits of the block follows item order (stability).  The
// block's items are placed in LDS in digit order and written out from there,
// so consecutive threads write consecutive places of each digit's run.
__global__ void __launch_bounds__(kRsThreads) k_rs_scatter(const uint32_t *kin, const uint32_t *vin, uint32_t *kout,
                                                           uint32_t *vout, size_t n, const uint32_t *n_dev, int shift,
                                                           const uint32_t *hist_scan, uint32_t nblocks)
{
    n = dev_count(n, n_dev);
    if ((size_t)blockIdx.x * kRsTile >= n) return;   // uniform: no items, nothing to place
    __shared__ uint32_t wcnt[kRsWaves][256];
    __shared__ uint32_t gbase[256];
    __shared__ uint32_t dstart[256];      // first place of each digit among the block's items
    __shared__ uint32_t wsum[kRsWaves];
    __shared__ uint32_t skey[kRsTile], sval[kRsTile];
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
    uint32_t run = 0;   // items of digit threadIdx.x in the block
#pragma unroll
    for (int w = 0; w < kRsWaves; ++w) {
        const uint32_t t = wcnt[w][threadIdx.x];
        wcnt[w][threadIdx.x] = run;
        run += t;
    }
    // exclusive prefix of the digit counts over the block: per wave, then across waves
    uint32_t inc = run;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t o = __shfl_up(inc, off, 64);
        if (lane >= off) inc += o;
    }
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    uint32_t before = 0;
    for (int w = 0; w < wave; ++w) before += wsum[w];
    dstart[threadIdx.x] = before + inc - run;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kRsRounds; ++r) {
        const size_t idx = base + (size_t)r * 64 + lane;
        if (idx < n) {
            const uint32_t digit = (key[r] >> shift) & 255u;
            const uint32_t lpos = dstart[digit] + wcnt[wave][digit] + lrank[r];
            skey[lpos] = key[r];
            sval[lpos] = val[r];
        }
    }
    __syncthreads();
    const size_t first = (size_t)blockIdx.x * kRsTile;
    const uint32_t count = (uint32_t)min((size_t)kRsTile, n - first);
    for (uint32_t i = threadIdx.x; i < count; i += kRsThreads) {
        const uint32_t k = skey[i];
        const uint32_t digit = (k >> shift) & 255u;
        const size_t pos = (size_t)gbase[digit] + (i - dstart[digit]);
        kout[pos] = k;
        vout[pos] = sval[i];
    }
}

// Sorts keys/vals by the low `bits` bits, ping-ponging through tk/tv; on
// return *keys_out / *vals_out name the pair of arrays that holds the result.
// n_dev (or NULL): the device count of items (at most n) -- the launches are
// sized for n.  ws (or NULL): radix_ws_words(n) words kept by the caller.
static size_t radix_ws_words(size_t n)
{
    const size_t nb = (n + kRsTile - 1) / kRsTile;
    return 256 * nb + scan_ws_words(256 * nb);
}

static fr_status radix_sort_pairs(fr_ctx *ctx, uint32_t *keys, uint32_t *vals, uint32_t *tk, uint32_t *tv, size_t n,
                                  int bits, hipStream_t st, uint32_t **keys_out, uint32_t **vals_out,
                                  const uint32_t *n_dev = nullptr, uint32_t *ws = nullptr)
{
    *keys_out = keys;
    *vals_out = vals;
    if (n <= 1 || bits <= 0) return FR_OK;
    const uint32_t nb = (uint32_t)((n + kRsTile - 1) / kRsTile);
    DevBuf hbuf;
    uint32_t *hist = ws;
    if (hist == nullptr) {
        FR_TRY(hbuf.alloc(ctx, (size_t)256 * nb * sizeof(uint32_t)));
        hbuf.stream = st;
        hist = hbuf.as<uint32_t>();
    }
    uint32_t *scan_ws = ws != nullptr ? ws + (size_t)256 * nb : nullptr;
    uint32_t *ka = keys, *va = vals, *kb = tk, *vb = tv;
    int passes = 0;
    for (int shift = 0; shift < bits; shift += 8, ++passes) {
        k_rs_hist<<<nb, kRsThreads, 0, st>>>(ka, n, n_dev, shift, hist, nb);
        FR_HIP(hipGetLastError());
        FR_TRY(scan_exclusive_u32(ctx, hist, hist, (size_t)256 * nb, 0, st, scan_ws));
        k_rs_scatter<<<nb, kRsThreads, 0, st>>>(ka, va, kb, vb, n, n_dev, shift, hist, nb);
        FR_HIP(hipGetLastError());
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    *keys_out = ka;
    *vals_out = va;
    return FR_OK;
}

// ---------------------------------------------------------------------------
// Sorted splat of a one-shot build: the records of each set (a contiguous
// range) are ordered by vertex id, stably, with a segmented LSD radix sort
// of the id less the set's first vertex id, in 9-bit digits -- sets of up to
// 2^18 vertices take two passes, where the global ids of many sets would
// take three 8-bit ones.  Tiles of kRsTile records never straddle two sets,
// and a histogram entry of (set s, digit g, tile j of s) sits at
// kSrDigits * tile0(s) + g * tiles(s) + j: one exclusive scan over all of
// them then gives each (tile, digit) its first place inside its set's range.
// Keys stay the global ids (the digits are taken from the local ones).
// ---------------------------------------------------------------------------
constexpr int kSrBits = 9;
constexpr uint32_t kSrDigits = 1u << kSrBits;

__device__ __forceinline__ size_t sr_hist_index(const TileMap &tm, int32_t s, int32_t t, uint32_t digit)
{
    const int32_t t0 = tm.seg_tile[s];
    return (size_t)kSrDigits * t0 + (size_t)digit * (size_t)(tm.seg_tile[s + 1] - t0) + (size_t)(t - t0);
}

// keys (or NULL): the items' keys; with NULL, pass 0 -- each record's vertex
// id is taken through its owner record (ovid[rec_own[r]]) and
// written to keys_out.
__global__ void __launch_bounds__(kRsThreads) k_sr_hist(TileMap tm, const uint32_t *vbase, const uint32_t *keys,
                                                        const uint32_t *rec_own, const uint32_t *ovid,
                                                        uint32_t *keys_out, int shift, uint32_t *hist)
{
    __shared__ uint32_t h[kSrDigits];
    const int32_t t = logical_tile(tm);
    if (t >= tm.n_tiles) return;   // uniform over the workgroup
    const int32_t s = tile_segment(tm, t);
    for (uint32_t i = threadIdx.x; i < kSrDigits; i += kRsThreads) h[i] = 0;
    __syncthreads();
    const int64_t first = tm.seg_off[s] + (int64_t)(t - tm.seg_tile[s]) * tm.tile;
    const int64_t end = min(first + (int64_t)tm.tile, tm.seg_end[s]);
    const uint32_t vb = vbase[s];
    for (int64_t r = first + threadIdx.x; r < end; r += kRsThreads) {
        uint32_t k;
        if (keys == nullptr) {
            k = ovid[rec_own[r]];
            keys_out[r] = k;
        } else {
            k = keys[r];
        }
        atomicAdd(&h[((k - vb) >> shift) & (kSrDigits - 1)], 1u);
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < kSrDigits; i += kRsThreads) hist[sr_hist_index(tm, s, t, i)] = h[i];
}

// The ranking of k_rs_scatter with 9-bit digits (each thread keeps two digits
// in the block prefix).  vin (or NULL): the values; with NULL each item's
// value is its own index (pass 0).
__global__ void __launch_bounds__(kRsThreads) k_sr_scatter(TileMap tm, const uint32_t *vbase, const uint32_t *kin,
                                                           const uint32_t *vin, uint32_t *kout, uint32_t *vout,
                                                           int shift, const uint32_t *hist_scan)
{
    __shared__ uint32_t wcnt[kRsWaves][kSrDigits];
    __shared__ uint32_t gbase[kSrDigits];
    __shared__ uint32_t dstart[kSrDigits];
    __shared__ uint32_t wsum[kRsWaves];
    __shared__ uint32_t skey[kRsTile], sval[kRsTile];
    const int32_t t = logical_tile(tm);
    if (t >= tm.n_tiles) return;   // uniform over the workgroup
    const int32_t s = tile_segment(tm, t);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (uint32_t i = threadIdx.x; i < kSrDigits; i += kRsThreads) {
#pragma unroll
        for (int w = 0; w < kRsWaves; ++w) wcnt[w][i] = 0;
        gbase[i] = hist_scan[sr_hist_index(tm, s, t, i)];
    }
    __syncthreads();

    const int64_t first = tm.seg_off[s] + (int64_t)(t - tm.seg_tile[s]) * tm.tile;
    const int64_t end = min(first + (int64_t)tm.tile, tm.seg_end[s]);
    const uint32_t vb = vbase[s];
    const int64_t base = first + (int64_t)wave * (64 * kRsRounds);
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint32_t key[kRsRounds], val[kRsRounds], lrank[kRsRounds];
#pragma unroll
    for (int r = 0; r < kRsRounds; ++r) {
        const int64_t idx = base + (int64_t)r * 64 + lane;
        const bool valid = idx < end;
        key[r] = valid ? kin[idx] : vb;
        val[r] = valid ? (vin != nullptr ? vin[idx] : (uint32_t)idx) : 0u;
        const uint32_t digit = ((key[r] - vb) >> shift) & (kSrDigits - 1);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < kSrBits; ++bit) {
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
    // digits 2i and 2i+1 of thread i: per-wave offsets, then the block prefix
    uint32_t run[2] = {0u, 0u};
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const uint32_t g = 2u * threadIdx.x + (uint32_t)j;
#pragma unroll
        for (int w = 0; w < kRsWaves; ++w) {
            const uint32_t c = wcnt[w][g];
            wcnt[w][g] = run[j];
            run[j] += c;
        }
    }
    const uint32_t pair = run[0] + run[1];
    uint32_t inc = pair;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t o = __shfl_up(inc, off, 64);
        if (lane >= off) inc += o;
    }
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    uint32_t before = 0;
    for (int w = 0; w < wave; ++w) before += wsum[w];
    dstart[2 * threadIdx.x] = before + inc - pair;
    dstart[2 * threadIdx.x + 1] = before + inc - pair + run[0];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kRsRounds; ++r) {
        const int64_t idx = base + (int64_t)r * 64 + lane;
        if (idx < end) {
            const uint32_t digit = ((key[r] - vb) >> shift) & (kSrDigits - 1);
            const uint32_t lpos = dstart[digit] + wcnt[wave][digit] + lrank[r];
            skey[lpos] = key[r];
            sval[lpos] = val[r];
        }
    }
    __syncthreads();
    const uint32_t count = (uint32_t)(end - first);
    for (uint32_t i = threadIdx.x; i < count; i += kRsThreads) {
        const uint32_t k = skey[i];
        const uint32_t digit = ((k - vb) >> shift) & (kSrDigits - 1);
        const size_t pos = (size_t)gbase[digit] + (i - dstart[digit]);
        kout[pos] = k;
        vout[pos] = sval[i];
    }
}

// Sorts the records of a one-shot build by vertex id (stable).  tm: tiles of
// kRsTile records over the sets' record ranges; vbase: the sets' first
// vertex ids (device); local_bits: bits of the largest local vertex id.
// Pass 0 takes the ids through the owner records, so keys0 needs no
// input.  On return *keys_out / *vals_out name the arrays holding the result
// (sorted vertex ids and record indices); keys0/vals0 and keys1/vals1 are the
// two ping-pong pairs, each of n entries.
static fr_status segmented_sort_records(fr_ctx *ctx, const TileMap &tm, const uint32_t *vbase,
                                        const uint32_t *rec_own, const uint32_t *ovid, uint32_t *keys0,
                                        uint32_t *vals0, uint32_t *keys1, uint32_t *vals1, size_t n, int local_bits,
                                        hipStream_t st, uint32_t **keys_out, uint32_t **vals_out)
{
    *keys_out = keys0;
    *vals_out = vals0;
    if (n == 0 || tm.n_tiles == 0) return FR_OK;
    if (tm.tile != kRsTile) {
        set_error("segmented sort: tiles of %d records, the kernels take %d", tm.tile, kRsTile);
        return FR_EINVAL;
    }
    const int passes = std::max(1, (local_bits + kSrBits - 1) / kSrBits);
    const size_t n_hist = (size_t)kSrDigits * tm.n_tiles;
    DevBuf hbuf;
    FR_TRY(hbuf.alloc(ctx, n_hist * sizeof(uint32_t)));
    hbuf.stream = st;
    uint32_t *hist = hbuf.as<uint32_t>();
    // pass p reads (ka, va) and writes (kb, vb); pass 0 writes the ids into keys0 first
    uint32_t *ka = keys0, *va = nullptr, *kb = keys1, *vb = vals1;
    const unsigned grid = (unsigned)(tm.xcd_chunk > 0 ? tm.xcd_chunk * 8 : tm.n_tiles);
    for (int p = 0; p < passes; ++p) {
        const int shift = p * kSrBits;
        k_sr_hist<<<grid, kRsThreads, 0, st>>>(tm, vbase, p == 0 ? nullptr : ka, rec_own, ovid, keys0, shift,
                                               hist);
        FR_HIP(hipGetLastError());
        FR_TRY(scan_exclusive_u32(ctx, hist, hist, n_hist, 0, st));
        k_sr_scatter<<<grid, kRsThreads, 0, st>>>(tm, vbase, ka, va, kb, vb, shift, hist);
        FR_HIP(hipGetLastError());
        // next pass reads what this one wrote and writes the other pair
        uint32_t *kn = (kb == keys1) ? keys0 : keys1, *vn = (vb == vals1) ? vals0 : vals1;
        ka = kb;
        va = vb;
        kb = kn;
        vb = vn;
    }
    *keys_out = ka;
    *vals_out = va;
    return FR_OK;
}

// ---------------------------------------------------------------------------
// Build kernels
// ---------------------------------------------------------------------------
struct Pts {
    const float *x, *y, *z, *nx, *ny, *nz;
};

// Partial records (d <= 6).  Neighbouring observation points of a scan share
// most simplex vertices; a wave of 64 points finds its runs of shared
// vertices (wave_runs) and emits one partial record per run: the key, the
// number of incidences (the run's length) and the sums over the run's points,
// in lane order and binary64, of b [1, y, n_y] (and b |y|^2 for the variance
// layouts).  A depth frame has about one run per four incidences, so the
// insertion, sort and sums that follow handle a quarter of the D N records.
// Partials are numbered wave by wave (run order within a wave), so that their
// order -- and with it every sum -- is fixed by the input alone.
template <int V> struct PartialType { using T = float; };
template <> struct PartialType<5> { using T = double; };   // |y|^2 layouts: the scatter about the
template <> struct PartialType<8> { using T = double; };   // mean is formed after the sums

// A partial record's values are one row: the V sums, then the incidence count
// (exact in T), padded to whole 16-byte chunks, so a gather reads one or two
// lines per record instead of one per channel.  Keys are rows of KW words.
template <int V> struct PartialRow {
    using T = typename PartialType<V>::T;
    static constexpr int S = (int)((((V + 1) * sizeof(T)) + 15) / 16 * 16 / sizeof(T));   // elements per row
    static constexpr int Q = (int)(S * sizeof(T) / 16);                                   // 16-byte chunks
};

template <int V>
__device__ __forceinline__ void store_row(typename PartialRow<V>::T *rows, size_t q,
                                          const typename PartialRow<V>::T (&v)[PartialRow<V>::S])
{
    using R = PartialRow<V>;
    uint4 *dst = reinterpret_cast<uint4 *>(rows + q * R::S);
    const uint4 *src = reinterpret_cast<const uint4 *>(v);
#pragma unroll
    for (int c = 0; c < R::Q; ++c) dst[c] = src[c];
}

template <int V>
__device__ __forceinline__ void load_row(const typename PartialRow<V>::T *rows, size_t q,
                                         typename PartialRow<V>::T (&v)[PartialRow<V>::S])
{
    using R = PartialRow<V>;
    const uint4 *src = reinterpret_cast<const uint4 *>(rows + q * R::S);
    uint4 *dst = reinterpret_cast<uint4 *>(v);
#pragma unroll
    for (int c = 0; c < R::Q; ++c) dst[c] = src[c];
}

template <int d>
__device__ __forceinline__ void load_feature(const Pts &pts, int64_t i, float (&p)[d])
{
    p[0] = pts.x[i];
    p[1] = pts.y[i];
    p[2] = pts.z[i];
    if constexpr (d == 6) {
        p[3] = pts.nx[i];
        p[4] = pts.ny[i];
        p[5] = pts.nz[i];
    }
}

// Count pass: the runs of every wave (4 waves per tile of 256 points; a wave
// past its set's end counts 0).
template <int d>
__global__ void __launch_bounds__(256) k_build_count(Pts pts, TileMap tm, const float *kset, uint32_t *wave_cnt,
                                                    int32_t *err)
{
    constexpr int D = d + 1;
    constexpr int KW = KeyWords<d>::value;
    __shared__ __attribute__((aligned(16))) char lds[4][WaveKeys<d>::bytes];
    __shared__ uint16_t no_src[4];
    const int32_t t = logical_tile(tm);
    if (t >= tm.n_tiles) return;
    const int32_t s = tile_segment(tm, t);
    const int wv = (int)(threadIdx.x >> 6);
    const int64_t i0 = tm.seg_off[s] + (int64_t)(t - tm.seg_tile[s]) * tm.tile + 64 * wv;
    const int64_t end = tm.seg_end[s];
    const int64_t i = i0 + (threadIdx.x & 63u);
    if (i0 >= end) {
        if ((threadIdx.x & 63u) == 0) wave_cnt[4 * (size_t)t + wv] = 0;
        return;
    }
    const bool live = i < end;
    float p[d], kk[d];
#pragma unroll
    for (int j = 0; j < d; ++j) {
        kk[j] = kset[8 * s + j];
        p[j] = 0.0f;
    }
    if (live) load_feature<d>(pts, i, p);
    uint64_t keys[D][KW];
    float b[D];
    int32_t sdiv = 0;
    if (!embed<d>(p, kk, keys, b, &sdiv) && live) atomicOr(err, 1);
    const int32_t U = wave_runs<d>(keys, class_shift<D>(sdiv), live, lds[wv], no_src, 0, nullptr, nullptr);
    if ((threadIdx.x & 63u) == 0) wave_cnt[4 * (size_t)t + wv] = (uint32_t)U;
}

// Partial pass: the same runs, their sums, written at the wave's offset
// (exclusive scan of the counts).  Points past valued_end[s] create their
// vertices but carry no value.
template <int d, int V> struct PartialLds {
    static constexpr int D = d + 1;
    static constexpr int NCH = ValLayout<V>::normals ? 6 : 3;   // point values after the 1: y (and n_y)
    static constexpr int keys = WaveKeys<d>::bytes;
    static constexpr int src = keys;                           // u16 per run, up to 64 D
    static constexpr int hc = src + ((2 * 64 * D + 7) / 8) * 8; // u64 per class
    static constexpr int bw = hc + 8 * D;                      // float [lane][class]: b
    static constexpr int pv = bw + 4 * 64 * D;                 // float [lane][NCH]: y, n_y
    static constexpr int bytes = pv + 4 * 64 * NCH;
};

// poff (or NULL): workgroup 0 also writes each set's first partial (set
// n_seg: the partial count, also to *p_count) as int64 -- what a tile map of
// the partials reads on the device.
template <int d, int V>
__global__ void __launch_bounds__(256) k_build_partials(Pts pts, TileMap tm, const float *kset,
                                                       const uint32_t *wave_off, uint64_t *pkey,
                                                       typename PartialType<V>::T *prow, size_t P,
                                                       const int64_t *valued_end, int64_t *poff = nullptr,
                                                       uint32_t *p_count = nullptr)
{
    if (poff != nullptr && blockIdx.x == 0)
        for (int32_t s = (int32_t)threadIdx.x; s <= tm.n_seg; s += (int32_t)blockDim.x) {
            const uint32_t q = wave_off[4 * (size_t)tm.seg_tile[s]];
            poff[s] = (int64_t)q;
            if (s == tm.n_seg) *p_count = q;
        }
    using T = typename PartialType<V>::T;
    using L = PartialLds<d, V>;
    constexpr int D = d + 1;
    constexpr int KW = KeyWords<d>::value;
    constexpr int NCH = L::NCH;
    __shared__ __attribute__((aligned(16))) char lds_all[4][L::bytes];
    const int32_t t = logical_tile(tm);
    if (t >= tm.n_tiles) return;
    const int32_t s = tile_segment(tm, t);
    const int wv = (int)(threadIdx.x >> 6);
    const int lane = (int)(threadIdx.x & 63u);
    const int64_t i0 = tm.seg_off[s] + (int64_t)(t - tm.seg_tile[s]) * tm.tile + 64 * wv;
    const int64_t end = tm.seg_end[s];
    if (i0 >= end) return;
    const int64_t i = i0 + lane;
    const bool live = i < end;
    char *lds = lds_all[wv];
    uint16_t *src = reinterpret_cast<uint16_t *>(lds + L::src);
    uint64_t *hc = reinterpret_cast<uint64_t *>(lds + L::hc);
    float *bw = reinterpret_cast<float *>(lds + L::bw);
    float *pv = reinterpret_cast<float *>(lds + L::pv);
    float p[d], kk[d];
#pragma unroll
    for (int j = 0; j < d; ++j) {
        kk[j] = kset[8 * s + j];
        p[j] = 0.0f;
    }
    float val[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) val[c] = 0.0f;
    if (live) {
        load_feature<d>(pts, i, p);
        val[0] = pts.x[i];
        val[1] = pts.y[i];
        val[2] = pts.z[i];
        if constexpr (NCH == 6) {
            val[3] = pts.nx[i];
            val[4] = pts.ny[i];
            val[5] = pts.nz[i];
        }
    }
    uint64_t keys[D][KW];
    float b[D];
    int32_t sdiv = 0;
    embed<d>(p, kk, keys, b, &sdiv);   // range errors were raised by the count pass
    const int32_t r = class_shift<D>(sdiv);
    if (live) {
        const float keep = (valued_end == nullptr || i < valued_end[s]) ? 1.0f : 0.0f;
#pragma unroll
        for (int m = 0; m < D; ++m) {
            int32_t c = m - r;
            c += c < 0 ? D : 0;
            bw[lane * D + c] = b[m] * keep;
        }
#pragma unroll
        for (int c = 0; c < NCH; ++c) pv[lane * NCH + c] = val[c];
    }
    const int32_t U = wave_runs<d>(keys, r, live, lds, src, 64 * D, nullptr, hc);
    wave_sync();
    const int32_t n_live = (int32_t)__popcll(__ballot(live));
    const size_t base = wave_off[4 * (size_t)t + wv];
    for (int32_t e = lane; e < U; e += 64) {
        const uint32_t sc = src[e];
        const int32_t o = (int32_t)(sc >> 3), c = (int32_t)(sc & 7u);
        const uint64_t above = hc[c] & ~((2ull << o) - 1ull);   // run starts of class c after lane o
        const int32_t stop = above != 0ull ? (int32_t)__builtin_ctzll(above) : n_live;
        double acc[V];
#pragma unroll
        for (int q = 0; q < V; ++q) acc[q] = 0.0;
        for (int32_t l = o; l < stop; ++l) {
            const double w = (double)bw[l * D + c];
            acc[0] += w;
            double y2 = 0.0;
#pragma unroll
            for (int q = 0; q < NCH; ++q) {
                const double y = (double)pv[l * NCH + q];
                acc[1 + q] += w * y;
                if (q < 3) y2 += y * y;
            }
            if constexpr (ValLayout<V>::m2) acc[V - 1] += w * y2;
        }
        uint64_t key[KW];
        lds_get_key<KW>(lds + (o * D + c) * 8 * KW, key);
        const size_t q = base + (size_t)e;
#pragma unroll
        for (int w = 0; w < KW; ++w) pkey[q * KW + w] = key[w];
        alignas(16) T row[PartialRow<V>::S];
#pragma unroll
        for (int ch = 0; ch < PartialRow<V>::S; ++ch) row[ch] = ch < V ? (T)acc[ch] : (T)0;
        row[V] = (T)(stop - o);
        store_row<V>(prow, q, row);
    }
}

// Set boundaries of the partials: the offset of each set's first wave.
__global__ void k_set_partial_off(int32_t n_sets, const int32_t *seg_tile, const uint32_t *wave_off,
                                  uint32_t *set_off)
{
    const int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s > n_sets) return;
    set_off[s] = wave_off[4 * (size_t)seg_tile[s]];
}

// Descriptor lattices: one thread per observation point writes its D records
// straight to memory (D * KW words are too many to stage in LDS), producing the
// vertices one at a time; each record is a partial of one incidence, values
// b [1, y] (binary32 products).
template <int d>
__global__ void __launch_bounds__(256) k_embed_feat(const float *feat, const float *kf, TileMap tm, Pts pts,
                                                   uint64_t *rec_key, float *rec_row, size_t R, int32_t *err)
{
    constexpr int D = d + 1;
    constexpr int KW = KeyWords<d>::value;
    const int32_t t = logical_tile(tm);
    if (t >= tm.n_tiles) return;
    const int32_t s = tile_segment(tm, t);
    const int64_t i = tm.seg_off[s] + (int64_t)(t - tm.seg_tile[s]) * tm.tile + threadIdx.x;
    if (i >= tm.seg_end[s]) return;
    float p[d], kk[d];
    const float4 *row = reinterpret_cast<const float4 *>(feat + (size_t)i * d);
#pragma unroll
    for (int q = 0; q < d / 4; ++q) {
        const float4 v = row[q];
        p[4 * q] = v.x;
        p[4 * q + 1] = v.y;
        p[4 * q + 2] = v.z;
        p[4 * q + 3] = v.w;
    }
#pragma unroll
    for (int j = 0; j < d; ++j) kk[j] = kf[j];
    HdEmbed<d> h;
    embed_hd_init<d>(p, kk, h);
    if (!h.ok) atomicOr(err, 1);
    const size_t r0 = (size_t)i * D;
    const float y0 = pts.x[i], y1 = pts.y[i], y2 = pts.z[i];
#pragma unroll 1
    for (int m = 0; m < D; ++m) {   // one vertex at a time: keeps the key walk in registers
        const float b = embed_hd_next<d>(h, m);
#pragma unroll
        for (int w = 0; w < KW; ++w) rec_key[(r0 + m) * KW + w] = h.P[w];
        alignas(16) float row[PartialRow<4>::S] = {b, b * y0, b * y1, b * y2, 1.0f, 0.0f, 0.0f, 0.0f};
        store_row<4>(rec_row, r0 + m, row);
    }
}

// Key words of record r (rows of KW words; one 16-byte load for KW = 2).
template <int KW>
__device__ __forceinline__ void load_key_row(const uint64_t *rec_key, size_t r, uint64_t (&k)[KW])
{
    if constexpr (KW == 2) {
        const uint4 q = *reinterpret_cast<const uint4 *>(rec_key + 2 * r);
        k[0] = (uint64_t)q.x | ((uint64_t)q.y << 32);
        k[1] = (uint64_t)q.z | ((uint64_t)q.w << 32);
    } else {
#pragma unroll
        for (int w = 0; w < KW; ++w) k[w] = rec_key[r * KW + w];
    }
}

// One thread per record: find or claim the record's key in the provisional
// linear-probing table of its set.  Neighbouring observation points share most
// of their vertices, so the records of a tile (TILE records of one set) are
// first merged in LDS: each record finds or claims its key in a small
// open-addressing table of the workgroup, and only the record that claimed a
// key (its representative) probes the global table; the others take the
// representative's result (MERGE; without it every record probes).  In the
// global table a slot holds a fingerprint of its key above its owner record;
// a slot read as taken is compared by fingerprint, then by the owner's key;
// only free slots are claimed with a CAS; owner_flag[r] = 1 marks the record
// whose CAS claimed the slot (the owner of its vertex), and rec_own[r] is the
// owner record of r's key.  An owner lies near the records of its vertex (they
// come from neighbouring points), so later passes that go from a record to
// its vertex id through rec_own read a few nearby lines, where the slot would
// send them to a random one.  Probing stops after kMaxProbe slots and raises
// `fail` (the host then retries with a larger table).
constexpr uint32_t kMaxProbe = 128;
constexpr unsigned long long kSlotEmpty = ~0ull;   // a free provisional slot

// TILE records per workgroup (one per thread): a wider tile merges more of
// the records of a key before they reach the global table (1024 for the
// one-shot build: its insertion 0.08 ms faster than with 256 on 64 depth frames).
template <int KW, bool MERGE, int TILE = 256>
__global__ void __launch_bounds__(TILE) k_insert_records(TileMap tm, const SetTable *tables, const uint64_t *rec_key,
                                                        size_t R, unsigned long long *own, uint32_t *rec_own,
                                                        uint32_t *owner_flag, int32_t *fail)
{
    constexpr uint32_t kTileKeySlots = 2 * TILE;   // LDS table of a tile: load <= 1/2
    __shared__ uint64_t lkey[MERGE ? KW : 1][MERGE ? TILE : 1];
    __shared__ uint32_t lown[MERGE ? kTileKeySlots : 1];
    __shared__ uint32_t lslot[MERGE ? TILE : 1];
    const int32_t t = logical_tile(tm);
    if (t >= tm.n_tiles) return;   // uniform over the workgroup
    const int32_t s = tile_segment(tm, t);
    const uint32_t tid = threadIdx.x;
    const int64_t r = tm.seg_off[s] + (int64_t)(t - tm.seg_tile[s]) * tm.tile + tid;
    const bool active = r < tm.seg_end[s];
    if constexpr (MERGE)
        for (uint32_t j = tid; j < kTileKeySlots; j += blockDim.x) lown[j] = kOwnerEmpty;
    uint64_t key[KW];
    if (active) {
        load_key_row<KW>(rec_key, (size_t)r, key);
        if constexpr (MERGE)
#pragma unroll
            for (int w = 0; w < KW; ++w) lkey[w][tid] = key[w];
    }
    if constexpr (MERGE) __syncthreads();
    uint32_t rep = tid;
    if (MERGE && active) {
        uint32_t h = hash_key<KW>(key, 0x9E3779B9u) & (kTileKeySlots - 1);
        for (uint32_t n = 0; n < kTileKeySlots; ++n) {   // ends: fewer keys than slots
            const uint32_t o = atomicCAS(&lown[h], kOwnerEmpty, tid);
            if (o == kOwnerEmpty) break;
            bool same = true;
#pragma unroll
            for (int w = 0; w < KW; ++w) same = same && (lkey[w][o] == key[w]);
            if (same) {
                rep = o;
                break;
            }
            h = (h + 1) & (kTileKeySlots - 1);
        }
    }
    bool won = false;
    if (active && rep == tid) {
        const SetTable st = tables[s];
        uint32_t h = hash_key<KW>(key, 0u) & st.mask;
        // a slot holds (fingerprint << 32) | owner record; the fingerprint, a second hash of the key,
        // lets a probe pass slots of other keys without reading their owner's key
        const uint32_t fp = hash_key<KW>(key, 0x51ED270Bu);
        const unsigned long long mine64 = ((unsigned long long)fp << 32) | (uint32_t)r;
        const uint32_t limit = min(st.mask + 1u, kMaxProbe);
        uint32_t found = kOwnerEmpty;
        for (uint32_t n = 0; n < limit; ++n) {
            const size_t slot = st.slot_base + h;
            unsigned long long o = __hip_atomic_load(&own[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (o == kSlotEmpty) o = atomicCAS(&own[slot], kSlotEmpty, mine64);
            won = (o == kSlotEmpty);
            bool match = won;
            if (!match && (uint32_t)(o >> 32) == fp) {
                uint64_t ok[KW];
                load_key_row<KW>(rec_key, (size_t)(uint32_t)o, ok);
                match = key_equal<KW>(ok, key);
            }
            if (match) {
                found = won ? (uint32_t)r : (uint32_t)o;   // the owner record of the key
                break;
            }
            h = (h + 1) & st.mask;
        }
        if (found == kOwnerEmpty) atomicOr(fail, 1);
        if constexpr (MERGE) {
            lslot[tid] = found;
        } else {
            if (found != kOwnerEmpty) rec_own[r] = found;
            owner_flag[r] = won ? 1u : 0u;
        }
    }
    if constexpr (MERGE) {
        __syncthreads();
        if (active) {
            const uint32_t o = lslot[rep];
            if (o != kOwnerEmpty) rec_own[r] = o;
            owner_flag[r] = won ? 1u : 0u;
        }
    }
}

// Vertex ids in owner-record order: `ovid` holds the exclusive scan of the
// owner flags over R + 1 entries (the flag past the last record is 0, so
// ovid[R] is the vertex count, and a record's vertex id is ovid[rec_own[r]]);
// owners -- the records whose id the scan steps past -- write their vertex's
// key (word-major, `stride` vertices per word).
// rec_off (or NULL; n_sets + 1 record offsets): workgroup 0 also writes each
// set's first vertex as k_set_vbase does (vbase64, and the count to *nv).
template <int KW>
__global__ void __launch_bounds__(256) k_owner_emit(size_t R, const uint32_t *ovid, const uint64_t *rec_key,
                                                   uint64_t *vkey, size_t stride, int32_t n_sets = 0,
                                                   const int64_t *rec_off = nullptr, int64_t *vbase64 = nullptr,
                                                   uint32_t *nv = nullptr)
{
    if (rec_off != nullptr && blockIdx.x == 0)
        for (int32_t s = (int32_t)threadIdx.x; s <= n_sets; s += (int32_t)blockDim.x) {
            const uint32_t v = ovid[rec_off[s]];
            vbase64[s] = (int64_t)v;
            if (s == n_sets) *nv = v;
        }
    const size_t r = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    const uint32_t v = ovid[r];
    if (ovid[r + 1] == v) return;
#pragma unroll
    for (int w = 0; w < KW; ++w) vkey[(size_t)w * stride + v] = rec_key[(size_t)r * KW + w];
}

// First vertex of each set (set n_sets: the vertex count): owners of a set's
// records form one contiguous id range, so it is the scanned flag at the set's
// first record (rec_off[n_sets] = the record count).  vbase64 and nv (or
// NULL): the same as int64 (a tile map's offsets) and the count alone.
__global__ void k_set_vbase(int32_t n_sets, const int64_t *rec_off, const uint32_t *ovid, uint32_t *vbase,
                            int64_t *vbase64, uint32_t *nv)
{
    const int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s > n_sets) return;
    const uint32_t v = ovid[rec_off[s]];
    if (vbase != nullptr) vbase[s] = v;
    if (vbase64 != nullptr) vbase64[s] = (int64_t)v;
    if (nv != nullptr && s == n_sets) *nv = v;
}

__global__ void __launch_bounds__(256) k_record_vertex(size_t R, const uint32_t *n_dev, const uint32_t *fail,
                                                      const uint32_t *rec_own, const uint32_t *ovid,
                                                      uint32_t *rvid, uint32_t *rid)
{
    const size_t r = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= dev_count(R, n_dev) || aborted(fail)) return;
    rvid[r] = ovid[rec_own[r]];
    rid[r] = (uint32_t)r;
}

// Sorted mode: segment starts and lengths of the vertex-sorted partials.
__global__ void __launch_bounds__(256) k_segment_heads(size_t R, const uint32_t *n_dev, const uint32_t *fail,
                                                       const uint32_t *rvid_sorted, uint32_t *voff)
{
    const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= dev_count(R, n_dev) || aborted(fail)) return;
    const uint32_t v = rvid_sorted[q];
    if (q == 0 || rvid_sorted[q - 1] != v) voff[v] = (uint32_t)q;
}

// Sorted mode: per vertex, the partials in partial order summed in binary64
// (occupancy = the sum of their incidence counts) -> bitwise deterministic.
// Vertex arrays are channel-major with `stride` vertices per channel; nv_dev
// and p_dev (or NULL) are device counts bounding NV and P.
template <int V>
__global__ void __launch_bounds__(256) k_vertex_sum_sorted(size_t NV, const uint32_t *nv_dev, size_t stride, size_t P,
                                                          const uint32_t *p_dev, const uint32_t *fail,
                                                          const uint32_t *voff,
                                                          const uint32_t *rid_sorted,
                                                          const typename PartialRow<V>::T *prow, float *vval,
                                                          uint32_t *vocc)
{
    using R = PartialRow<V>;
    using T = typename R::T;
    NV = dev_count(NV, nv_dev);
    P = dev_count(P, p_dev);
    const size_t v = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= NV || aborted(fail)) return;
    double acc[V];
#pragma unroll
    for (int c = 0; c < V; ++c) acc[c] = 0.0;
    uint32_t occ = 0;
    const uint32_t q0 = voff[v], q1 = v + 1 < NV ? voff[v + 1] : (uint32_t)P;
    for (uint32_t q = q0; q < q1; q += 2) {
        // two rows in flight
        uint32_t r[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) r[u] = (q + u < q1) ? rid_sorted[q + u] : rid_sorted[q0];
        alignas(16) T row[2][R::S];
#pragma unroll
        for (int u = 0; u < 2; ++u) load_row<V>(prow, r[u], row[u]);
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            if (q + u >= q1) break;
            occ += (uint32_t)row[u][V];
#pragma unroll
            for (int c = 0; c < V; ++c) acc[c] += (double)row[u][c];
        }
    }
    if constexpr (ValLayout<V>::m2) {
        // keep the scatter about the vertex mean, sum b |y - mu|^2 = sum b |y|^2 - |M1|^2 / W:
        // the slice then never subtracts |y|^2-sized numbers stored in binary32
        const double q = acc[0] > 0.0 ? (acc[1] * acc[1] + acc[2] * acc[2] + acc[3] * acc[3]) / acc[0] : 0.0;
        acc[V - 1] = fmax(acc[V - 1] - q, 0.0);
    }
    vocc[v] = occ;
#pragma unroll
    for (int c = 0; c < V; ++c) vval[(size_t)c * stride + v] = (float)acc[c];
}

// Sorted mode without the sort, for rebuilds of at most kListMax partials
// (in place, where the launches of a radix sort cost more than its work):
// each partial finds its vertex and takes a place in the vertex's list by an
// atomic counter (k_list_count, an exclusive scan, k_list_place); a vertex's
// thread then walks its list in increasing partial order (k_vertex_sum_list),
// so the sums are those of k_vertex_sum_sorted, bitwise, whatever order the
// atomics gave the places.
constexpr size_t kListMax = (size_t)1 << 17;

__global__ void __launch_bounds__(256) k_list_count(size_t P, const uint32_t *p_dev, const uint32_t *fail,
                                                   const uint32_t *rec_own, const uint32_t *ovid, uint32_t *rvid,
                                                   uint32_t *vcount)
{
    const size_t r = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= dev_count(P, p_dev) || aborted(fail)) return;
    const uint32_t v = ovid[rec_own[r]];
    rvid[r] = v;
    atomicAdd(&vcount[v], 1u);
}

// vfill: per vertex, places taken so far (zero before the launch)
__global__ void __launch_bounds__(256) k_list_place(size_t P, const uint32_t *p_dev, const uint32_t *fail,
                                                   const uint32_t *rvid, const uint32_t *voff, uint32_t *vfill,
                                                   uint32_t *list)
{
    const size_t r = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= dev_count(P, p_dev) || aborted(fail)) return;
    const uint32_t v = rvid[r];
    list[voff[v] + atomicAdd(&vfill[v], 1u)] = (uint32_t)r;
}

template <int V>
__global__ void __launch_bounds__(256) k_vertex_sum_list(size_t NV, const uint32_t *nv_dev, size_t stride,
                                                        const uint32_t *fail, const uint32_t *voff,
                                                        const uint32_t *vcount, const uint32_t *list,
                                                        const typename PartialRow<V>::T *prow, float *vval,
                                                        uint32_t *vocc)
{
    using R = PartialRow<V>;
    using T = typename R::T;
    const size_t v = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= dev_count(NV, nv_dev) || aborted(fail)) return;
    const uint32_t *l = list + voff[v];
    const uint32_t n = vcount[v];
    double acc[V];
#pragma unroll
    for (int c = 0; c < V; ++c) acc[c] = 0.0;
    uint32_t occ = 0;
    // the list's entries in increasing order: each step takes the least entry above the last one
    uint32_t last = 0, first = 1;
    for (uint32_t k = 0; k < n; ++k) {
        uint32_t q = 0xFFFFFFFFu;
        for (uint32_t i = 0; i < n; ++i) {
            const uint32_t e = l[i];
            if ((first || e > last) && e < q) q = e;
        }
        first = 0;
        last = q;
        alignas(16) T row[R::S];
        load_row<V>(prow, q, row);
        occ += (uint32_t)row[V];
#pragma unroll
        for (int c = 0; c < V; ++c) acc[c] += (double)row[c];
    }
    if constexpr (ValLayout<V>::m2) {
        const double q = acc[0] > 0.0 ? (acc[1] * acc[1] + acc[2] * acc[2] + acc[3] * acc[3]) / acc[0] : 0.0;
        acc[V - 1] = fmax(acc[V - 1] - q, 0.0);
    }
    vocc[v] = occ;
#pragma unroll
    for (int c = 0; c < V; ++c) vval[(size_t)c * stride + v] = (float)acc[c];
}

// Atomic mode: one thread per partial, binary32 hardware atomics of its sums;
// occupancy by integer atomics.  The |y|^2 channel waits for the second pass.
template <int V>
__global__ void __launch_bounds__(256) k_vertex_sum_atomic(size_t P, const uint32_t *p_dev, const uint32_t *fail,
                                                          const uint32_t *rec_own, const uint32_t *ovid,
                                                          const typename PartialRow<V>::T *prow, float *vval,
                                                          uint32_t *vocc, size_t NV)
{
    using R = PartialRow<V>;
    const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= dev_count(P, p_dev) || aborted(fail)) return;
    const uint32_t v = ovid[rec_own[q]];
    alignas(16) typename R::T row[R::S];
    load_row<V>(prow, q, row);
    atomicAdd(&vocc[v], (uint32_t)row[V]);
    constexpr int NL = ValLayout<V>::m2 ? V - 1 : V;
#pragma unroll
    for (int c = 0; c < NL; ++c) unsafeAtomicAdd(&vval[(size_t)c * NV + v], (float)row[c]);
}

// Atomic mode, |y|^2 layouts: second pass once the means are complete.  A
// partial p adds its own scatter S_p = Q_p - |M1_p|^2 / W_p plus
// W_p |mu_p - mu_v|^2 about the vertex mean mu_v = M1_v / W_v (the parallel
// form of the scatter; about a mean rounded to binary32 it is larger by
// W |mu - mu'|^2, far below the binary32 resolution of the sum).
template <int V>
__global__ void __launch_bounds__(256) k_vertex_scatter_atomic(size_t P, const uint32_t *p_dev, const uint32_t *fail,
                                                              const uint32_t *rec_own, const uint32_t *ovid,
                                                              const typename PartialRow<V>::T *prow, float *vval,
                                                              size_t NV)
{
    using R = PartialRow<V>;
    const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= dev_count(P, p_dev) || aborted(fail)) return;
    const uint32_t v = ovid[rec_own[q]];
    alignas(16) typename R::T row[R::S];
    load_row<V>(prow, q, row);
    const double W = (double)row[0];
    if (!(W > 0.0)) return;
    const double m1x = (double)row[1], m1y = (double)row[2], m1z = (double)row[3];
    const double own = fmax((double)row[V - 1] - (m1x * m1x + m1y * m1y + m1z * m1z) / W, 0.0);
    const float Wv = vval[v];
    const double iv = Wv > 0.0f ? 1.0 / (double)Wv : 0.0;
    const double dx = m1x / W - (double)vval[NV + v] * iv;
    const double dy = m1y / W - (double)vval[2 * NV + v] * iv;
    const double dz = m1z / W - (double)vval[3 * NV + v] * iv;
    unsafeAtomicAdd(&vval[(size_t)(V - 1) * NV + v], (float)(own + W * (dx * dx + dy * dy + dz * dz)));
}

// Bucketed two-choice cuckoo insertion of the vertices of each set (one
// thread per vertex).  A thread holds exactly one vertex at a time.  A new
// vertex takes a free slot of its first bucket, else of its second; with both
// full it swaps itself into the first and carries the vertex it displaced
// toward that vertex's other bucket, where the same happens: a free slot ends
// the walk, a full bucket gives up one of its slots in turn.  A slot, once
// filled, is never empty again, and a vertex reaches its second bucket only
// when its first is full -- the property a lookup relies on to stop at a
// first bucket with a free slot.  A thread that gives up after kMaxKicks
// raises `fail` and the host rebuilds the table with another seed.
constexpr int kMaxKicks = 512;

template <int KW>
__device__ __forceinline__ void vertex_key(const uint64_t *vkey, size_t NV, uint32_t v, uint64_t (&key)[KW])
{
#pragma unroll
    for (int w = 0; w < KW; ++w) key[w] = vkey[(size_t)w * NV + v];
}

__device__ __forceinline__ bool claim_free(uint32_t *own, uint32_t bucket, uint32_t v)
{
#pragma unroll
    for (int j = 0; j < kBucketSlots; ++j)
        if (atomicCAS(&own[kBucketSlots * bucket + j], kOwnerEmpty, v) == kOwnerEmpty) return true;
    return false;
}

// Vertex keys are word-major with NV (the stride) vertices per word.
template <int KW>
__global__ void __launch_bounds__(256) k_cuckoo_insert(TileMap tm, const SetTable *tables, const uint64_t *vkey,
                                                      size_t NV, uint32_t *own, int32_t *fail)
{
    const int32_t t = logical_tile(tm);
    if (t >= tm.n_tiles) return;
    const int32_t s = tile_segment(tm, t);
    const int64_t v = tm.seg_off[s] + (int64_t)(t - tm.seg_tile[s]) * tm.tile + threadIdx.x;
    if (v >= tm.seg_end[s]) return;
    const SetTable st = tables[s];
    const uint32_t nb = st.cap >> 1;
    uint32_t *o = own + st.slot_base;
    uint32_t cur = (uint32_t)v;
    uint64_t key[KW];
    vertex_key<KW>(vkey, NV, cur, key);
    uint32_t b1, b2;
    key_buckets<KW>(key, st.seed, nb, b1, b2);
    if (claim_free(o, b1, cur) || claim_free(o, b2, cur)) return;
    uint32_t bk = b1;   // full: displace a vertex of the first bucket
    for (int it = 0; it < kMaxKicks; ++it) {
        const uint32_t old = atomicExch(&o[kBucketSlots * bk + (uint32_t)(it % kBucketSlots)], cur);
        if (old == kOwnerEmpty) return;
        cur = old;
        vertex_key<KW>(vkey, NV, cur, key);
        key_buckets<KW>(key, st.seed, nb, b1, b2);
        bk = (bk == b1) ? b2 : b1;
        if (claim_free(o, bk, cur)) return;
    }
    atomicOr(fail, 1);
}

// Filling the table without a slot -> vertex map: free slots get the empty
// key (one thread per slot), and each vertex (one thread per vertex, over the
// cuckoo pass's tile map) finds its own slot among the four of its two
// buckets -- two random 8-byte reads instead of the map's random 4-byte
// writes and its read-back -- and writes its key and padded values there.  A
// vertex the cuckoo pass failed to place writes nothing (the pass is redone).
// One whole slot -- key, values padded to VP, zeros in the padding -- in
// 16-byte stores: every byte of the slot is written, so no sector of the
// table is written in part (a 16-byte key alone in a 64-byte slot wrote at
// well under half the rate of whole slots).
template <int KW, int V>
__device__ __forceinline__ void store_slot(char *dst, const uint64_t (&key)[KW], const float (&val)[ValPad<V>::value])
{
    using G = SlotGeom<KW, V>;
    constexpr uint32_t VP = ValPad<V>::value;
    constexpr uint32_t kUnits = G::bytes / 16;
    uint4 *d = reinterpret_cast<uint4 *>(dst);
#pragma unroll
    for (uint32_t u = 0; u < kUnits; ++u) {
        uint32_t w[4];
#pragma unroll
        for (uint32_t j = 0; j < 4; ++j) {
            const uint32_t byte = 16u * u + 4u * j;
            uint32_t x = 0u;
            if (byte < 8u * KW) {
                const uint64_t k = key[byte / 8u];
                x = (byte % 8u == 0u) ? (uint32_t)k : (uint32_t)(k >> 32);
            } else if (byte >= G::val_off && byte < G::val_off + 4u * VP) {
                x = __float_as_uint(val[(byte - G::val_off) / 4u]);
            }
            w[j] = x;
        }
        d[u] = make_uint4(w[0], w[1], w[2], w[3]);
    }
}

template <int KW, int V>
__global__ void __launch_bounds__(256) k_slot_empty(size_t n_slots, const uint32_t *n_dev, const uint32_t *own,
                                                   char *table)
{
    using G = SlotGeom<KW, V>;
    const size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= dev_count(n_slots, n_dev) || own[j] != kOwnerEmpty) return;
    uint64_t key[KW];
#pragma unroll
    for (int w = 0; w < KW; ++w) key[w] = kKeyEmpty;
    float val[ValPad<V>::value];
#pragma unroll
    for (int c = 0; c < ValPad<V>::value; ++c) val[c] = 0.0f;
    store_slot<KW, V>(table + (size_t)G::bytes * j, key, val);
}

template <int KW, int V>
__global__ void __launch_bounds__(256) k_vertex_place(TileMap tm, const SetTable *tables, const uint32_t *own,
                                                     const uint64_t *vkey, const float *vval, size_t stride,
                                                     const uint32_t *fail, char *table)
{
    using G = SlotGeom<KW, V>;
    constexpr int VP = ValPad<V>::value;
    const int32_t t = logical_tile(tm);
    if (t >= tm.n_tiles || aborted(fail)) return;
    const int32_t s = tile_segment(tm, t);
    const int64_t v = tm.seg_off[s] + (int64_t)(t - tm.seg_tile[s]) * tm.tile + threadIdx.x;
    if (v >= tm.seg_end[s]) return;
    const SetTable st = tables[s];
    uint64_t key[KW];
    vertex_key<KW>(vkey, stride, (uint32_t)v, key);
    uint32_t b1, b2;
    key_buckets<KW>(key, st.seed, st.cap >> 1, b1, b2);
    const uint2 o1 = *reinterpret_cast<const uint2 *>(own + st.slot_base + (size_t)kBucketSlots * b1);
    const uint2 o2 = *reinterpret_cast<const uint2 *>(own + st.slot_base + (size_t)kBucketSlots * b2);
    const uint32_t u = (uint32_t)v;
    int64_t slot = -1;
    if (o1.x == u) slot = (int64_t)kBucketSlots * b1;
    else if (o1.y == u) slot = (int64_t)kBucketSlots * b1 + 1;
    else if (o2.x == u) slot = (int64_t)kBucketSlots * b2;
    else if (o2.y == u) slot = (int64_t)kBucketSlots * b2 + 1;
    if (slot < 0) return;
    float val[VP];
#pragma unroll
    for (int c = 0; c < VP; ++c) val[c] = c < V ? vval[(size_t)c * stride + v] : 0.0f;
    store_slot<KW, V>(table + (size_t)G::bytes * (st.slot_base + (uint64_t)slot), key, val);
}

// ---------------------------------------------------------------------------
// Host driver
// ---------------------------------------------------------------------------
// Smallest power of two >= max(x, 16), capped at 2^31 (callers check the
// capacity they get against what they need).
static uint32_t next_pow2(uint64_t x)
{
    uint64_t p = 16;
    while (p < x && p < (1ull << 31)) p <<= 1;
    return (uint32_t)p;
}

static inline unsigned blocks_for(size_t n, int threads) { return (unsigned)((n + threads - 1) / threads); }

// Tile map over explicit offsets (device copy kept in `buf`).
// Blocks to launch for a tile map: with XCD chunks, 8 whole chunks (the blocks
// past the last tile return at once).
static unsigned grid_of(const TileMap &tm) { return (unsigned)(tm.xcd_chunk > 0 ? tm.xcd_chunk * 8 : tm.n_tiles); }

// The device image goes through the context's pinned staging (no wait).
static fr_status make_offset_map(fr_ctx *ctx, const std::vector<int64_t> &off, int32_t tile, hipStream_t st,
                                 DevBuf &buf, TileMap &tm, bool xcd = false)
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
    std::vector<char> image(b_off + b_tile + b_set);
    std::memcpy(image.data(), off.data(), b_off);
    std::memcpy(image.data() + b_off, tiles.data(), b_tile);
    std::memcpy(image.data() + b_off + b_tile, sets.data(), b_set);
    FR_TRY(stage_h2d(ctx, p, image.data(), image.size(), st));
    tm.seg_off = reinterpret_cast<const int64_t *>(p);
    tm.seg_end = tm.seg_off + 1;
    tm.seg_tile = reinterpret_cast<const int32_t *>(p + b_off);
    tm.seg_set = reinterpret_cast<const int32_t *>(p + b_off + b_tile);
    tm.n_seg = n;
    tm.n_tiles = tiles[n];
    tm.tile = tile;
    // XCD-contiguous tiles: a set's tiles run on one XCD, so the set's tables stay in that XCD's L2
    tm.xcd_chunk = (xcd && tm.n_tiles >= 8 * 64) ? (tm.n_tiles + 7) / 8 : 0;
    return FR_OK;
}

// HIP events at the boundaries of the build's stages (embed | insert and
// vertex ids | values | final tables), read after the build's last wait.
struct StageEvents {
    hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    bool ok = true;
    StageEvents()
    {
        for (auto &e : ev) ok = ok && hipEventCreate(&e) == hipSuccess;
    }
    ~StageEvents()
    {
        for (auto &e : ev)
            if (e) (void)hipEventDestroy(e);
    }
    void mark(int i, hipStream_t st)
    {
        if (ok) ok = hipEventRecord(ev[i], st) == hipSuccess;
    }
    void read(float (&ms)[4]) const
    {
        for (int i = 0; i < 4; ++i) {
            ms[i] = -1.0f;
            if (ok) (void)hipEventElapsedTime(&ms[i], ev[i], ev[i + 1]);
        }
    }
};

template <int d, int V>
static fr_status build_impl(fr_ctx *ctx, const fr_cloud *obs, hipStream_t st, fr_lattice *lat,
                            const int64_t *valued_end, const float *feat = nullptr, bool wait_end = true)
{
    constexpr int D = d + 1;
    constexpr int KW = KeyWords<d>::value;
    StreamScope scope(st);   // temporaries are freed in the order of st
    const int32_t S = obs->n_sets;
    const int64_t N = cloud_points(obs);
    const size_t R = (size_t)N * D;
    const bool sorted = lat->splat == FR_SPLAT_SORTED;
    if (R >= 0xFFFFFFF0ull) {
        set_error("fr_lattice_build: %lld records exceed the 32-bit record index", (long long)R);
        return FR_EINVAL;
    }
    Pts pts{obs->x, obs->y, obs->z, obs->nx, obs->ny, obs->nz};
    using T = typename PartialType<V>::T;

    DevBuf rec_key, rec_row, rec_own, own1, t1_d, ptmap, rtmap, fail;
    FR_TRY(fail.alloc(ctx, sizeof(int32_t)));
    FR_TRY(t1_d.alloc(ctx, S * sizeof(SetTable)));
    StageEvents stage;
    stage.mark(0, st);
    FR_HIP(hipMemsetAsync(lat->err_d, 0, sizeof(int32_t), st));

    // 1. embed: partial records (the runs of each wave, d <= 6; one per
    //    incidence for descriptors); roff = the partials of each set
    std::vector<int64_t> poff(obs->offsets, obs->offsets + S + 1);
    TileMap ptm{}, rtm{};
    FR_TRY(make_offset_map(ctx, poff, 256, st, ptmap, ptm, false));
    DevBuf kset_d;
    FR_TRY(kset_d.alloc(ctx, lat->kset.size() * sizeof(float)));
    FR_TRY(stage_h2d(ctx, kset_d.p, lat->kset.data(), lat->kset.size() * sizeof(float), st));
    std::vector<int64_t> roff(S + 1);
    size_t P = 0;   // partial records
    if constexpr (d > 6) {
        P = R;
        for (int32_t s = 0; s <= S; ++s) roff[s] = obs->offsets[s] * D;
        FR_TRY(rec_key.alloc(ctx, P * KW * sizeof(uint64_t)));
        FR_TRY(rec_row.alloc(ctx, P * PartialRow<V>::S * sizeof(T)));
        if (ptm.n_tiles > 0) {
            k_embed_feat<d><<<ptm.n_tiles, 256, 0, st>>>(feat, lat->kfeat_d, ptm, pts, rec_key.as<uint64_t>(),
                                                         rec_row.as<float>(), P, lat->err_d);
            FR_HIP(hipGetLastError());
        }
    } else {
        const size_t n_waves = (size_t)ptm.n_tiles * 4;
        DevBuf wave_cnt, set_off;
        FR_TRY(wave_cnt.alloc(ctx, (n_waves + 1) * sizeof(uint32_t)));
        FR_TRY(set_off.alloc(ctx, (S + 1) * sizeof(uint32_t)));
        FR_HIP(hipMemsetAsync(wave_cnt.as<uint32_t>() + n_waves, 0, sizeof(uint32_t), st));
        if (ptm.n_tiles > 0) {
            k_build_count<d><<<ptm.n_tiles, 256, 0, st>>>(pts, ptm, kset_d.as<float>(), wave_cnt.as<uint32_t>(),
                                                          lat->err_d);
            FR_HIP(hipGetLastError());
        }
        FR_TRY(scan_exclusive_u32(ctx, wave_cnt.as<uint32_t>(), wave_cnt.as<uint32_t>(), n_waves + 1, 0, st));
        k_set_partial_off<<<blocks_for(S + 1, 64), 64, 0, st>>>(S, ptm.seg_tile, wave_cnt.as<uint32_t>(),
                                                                set_off.as<uint32_t>());
        FR_HIP(hipGetLastError());
        uint32_t *rb = nullptr;   // pinned: [set offsets S + 1 | range error]
        FR_TRY(build_readback(ctx, (S + 2) * sizeof(uint32_t), reinterpret_cast<void **>(&rb)));
        FR_HIP(hipMemcpyAsync(rb, set_off.p, (S + 1) * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
        FR_HIP(hipMemcpyAsync(rb + S + 1, lat->err_d, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        FR_HIP(hipStreamSynchronize(st));
        const std::vector<uint32_t> so(rb, rb + S + 1);
        if (rb[S + 1] != 0) {
            set_error("fr_lattice_build: a lattice coordinate left [-2^20, 2^20); increase sigma or centre the cloud");
            return FR_ERANGE;
        }
        for (int32_t s = 0; s <= S; ++s) roff[s] = so[s];
        P = so[S];
        FR_TRY(rec_key.alloc(ctx, P * KW * sizeof(uint64_t)));
        FR_TRY(rec_row.alloc(ctx, P * PartialRow<V>::S * sizeof(T)));
        if (ptm.n_tiles > 0 && P > 0) {
            k_build_partials<d, V><<<ptm.n_tiles, 256, 0, st>>>(pts, ptm, kset_d.as<float>(),
                                                                wave_cnt.as<uint32_t>(), rec_key.as<uint64_t>(),
                                                                rec_row.as<T>(), P, valued_end);
            FR_HIP(hipGetLastError());
        }
    }
    FR_TRY(rec_own.alloc(ctx, P * sizeof(uint32_t)));
    lat->n_partials = (int64_t)P;

    stage.mark(1, st);
    // 2. insert into provisional tables (pow2 >= R_set / 2 first, or four times
    //    the vertices the last build's vertices-per-record ratio predicts if that
    //    is more; 2 R_set if that overflows; R_set = the set's partial records)
    constexpr int kInsertTile = 1024;
    FR_TRY(make_offset_map(ctx, roff, kInsertTile, st, rtmap, rtm, true));
    uint64_t n1 = 0;
    DevBuf ovid, vb_d;
    FR_TRY(ovid.alloc(ctx, (P + 1) * sizeof(uint32_t)));   // owner flags (and a 0), then their exclusive scan
    FR_TRY(vb_d.alloc(ctx, (S + 1) * sizeof(uint32_t)));
    std::vector<uint32_t> vb_h(S + 1);
    int32_t err_h = 0;
    for (int attempt = 0; attempt < 2; ++attempt) {
        std::vector<SetTable> t1(S);
        n1 = 0;
        for (int32_t s = 0; s < S; ++s) {
            const uint64_t rs = (uint64_t)(roff[s + 1] - roff[s]);
            const uint64_t guess = (uint64_t)(4.0 * std::min(ctx->vertex_ratio, 1.0) * (double)rs);
            const uint32_t cap = next_pow2(attempt == 0 ? std::max<uint64_t>(rs / 2, guess) : 2 * rs);
            if (2 * rs > (1ull << 31) && attempt == 1) {
                set_error("fr_lattice_build: set %d has too many partial records (%llu)", s, (unsigned long long)rs);
                return FR_EINVAL;
            }
            t1[s] = SetTable{nullptr, nullptr, n1, cap, 0, 0, cap - 1, {}};
            n1 += cap;
        }
        if (n1 >= 0xFFFFFFF0ull) {
            set_error("fr_lattice_build: provisional table too large");
            return FR_EINVAL;
        }
        FR_TRY(own1.alloc(ctx, n1 * sizeof(unsigned long long)));
        FR_TRY(stage_h2d(ctx, t1_d.p, t1.data(), S * sizeof(SetTable), st));
        FR_HIP(hipMemsetAsync(own1.p, 0xFF, n1 * sizeof(unsigned long long), st));
        FR_HIP(hipMemsetAsync(fail.p, 0, sizeof(int32_t), st));
        if (rtm.n_tiles > 0) {
            k_insert_records<KW, true, kInsertTile><<<grid_of(rtm), kInsertTile, 0, st>>>(
                rtm, t1_d.as<SetTable>(), rec_key.as<uint64_t>(), P, own1.as<unsigned long long>(),
                rec_own.as<uint32_t>(), ovid.as<uint32_t>(), fail.as<int32_t>());
            FR_HIP(hipGetLastError());
        }
        // 3. vertex ids in owner-record order and per-set ranges, enqueued before the
        //    overflow check (one wait for both; redone if the insertion overflowed)
        FR_HIP(hipMemsetAsync(ovid.as<uint32_t>() + P, 0, sizeof(uint32_t), st));
        FR_TRY(scan_exclusive_u32(ctx, ovid.as<uint32_t>(), ovid.as<uint32_t>(), P + 1, 0, st));
        k_set_vbase<<<blocks_for(S + 1, 64), 64, 0, st>>>(S, rtm.seg_off, ovid.as<uint32_t>(), vb_d.as<uint32_t>(),
                                                          nullptr, nullptr);
        FR_HIP(hipGetLastError());
        uint32_t *rb = nullptr;   // pinned: [vertex bases S + 1 | overflow | range error]
        FR_TRY(build_readback(ctx, (S + 3) * sizeof(uint32_t), reinterpret_cast<void **>(&rb)));
        FR_HIP(hipMemcpyAsync(rb, vb_d.p, (S + 1) * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
        FR_HIP(hipMemcpyAsync(rb + S + 1, fail.p, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        FR_HIP(hipMemcpyAsync(rb + S + 2, lat->err_d, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        FR_HIP(hipStreamSynchronize(st));
        std::copy(rb, rb + S + 1, vb_h.begin());
        const uint32_t failed = rb[S + 1];
        err_h = (int32_t)rb[S + 2];
        if (!failed) break;
        if (attempt == 1) {
            set_error("fr_lattice_build: provisional table overflow");
            return FR_EDEVICE;
        }
    }
    const uint32_t nv_total = vb_h[S];
    if (err_h != 0) {
        set_error("fr_lattice_build: a lattice coordinate left [-2^20, 2^20); increase sigma or centre the cloud");
        return FR_ERANGE;
    }
    lat->vbase.assign(S + 1, 0);
    std::vector<uint32_t> counts(S);
    for (int32_t s = 0; s < S; ++s) {
        lat->vbase[s + 1] = vb_h[s + 1];
        counts[s] = vb_h[s + 1] - vb_h[s];
    }
    const size_t NV = nv_total;
    lat->n_vertices_total = (int64_t)NV;
    if (P > 0) ctx->vertex_ratio = (double)NV / (double)P;

    // vertex arrays (kept for export)
    lat->vert_bytes = NV * (KW * sizeof(uint64_t) + sizeof(uint32_t) + V * sizeof(float)) + 64;
    {
        void *p = nullptr;
        FR_TRY(dev_alloc(ctx, &p, lat->vert_bytes));
        char *c = static_cast<char *>(p);
        lat->vkey = reinterpret_cast<uint64_t *>(c);
        lat->vval = reinterpret_cast<float *>(c + NV * KW * sizeof(uint64_t));
        lat->vocc = reinterpret_cast<uint32_t *>(c + NV * (KW * sizeof(uint64_t) + V * sizeof(float)));
    }
    if (NV > 0) {
        k_owner_emit<KW><<<blocks_for(P, 256), 256, 0, st>>>(P, ovid.as<uint32_t>(), rec_key.as<uint64_t>(),
                                                             lat->vkey, NV);
        FR_HIP(hipGetLastError());
    }

    // 4. values
    stage.mark(2, st);
    if (NV > 0) {
        if (sorted) {
            DevBuf rvid, rid, tk, tv, voff, stmap;
            FR_TRY(rvid.alloc(ctx, P * sizeof(uint32_t)));
            FR_TRY(rid.alloc(ctx, P * sizeof(uint32_t)));
            FR_TRY(tk.alloc(ctx, P * sizeof(uint32_t)));
            FR_TRY(tv.alloc(ctx, P * sizeof(uint32_t)));
            FR_TRY(voff.alloc(ctx, NV * sizeof(uint32_t)));
            // sort each set's records by their vertex id less the set's first one
            uint32_t max_local = 0;
            for (int32_t s = 0; s < S; ++s) max_local = std::max(max_local, counts[s] > 0 ? counts[s] - 1 : 0u);
            int bits = 0;
            while (bits < 32 && (max_local >> bits) != 0) ++bits;
            TileMap srtm{};
            FR_TRY(make_offset_map(ctx, roff, kRsTile, st, stmap, srtm, true));
            uint32_t *svid = nullptr, *srid = nullptr;   // the sorted pairs
            FR_TRY(segmented_sort_records(ctx, srtm, vb_d.as<uint32_t>(), rec_own.as<uint32_t>(),
                                          ovid.as<uint32_t>(), rvid.as<uint32_t>(), rid.as<uint32_t>(),
                                          tk.as<uint32_t>(), tv.as<uint32_t>(), P, bits, st, &svid, &srid));
            k_segment_heads<<<blocks_for(P, 256), 256, 0, st>>>(P, nullptr, nullptr, svid, voff.as<uint32_t>());
            FR_HIP(hipGetLastError());
            k_vertex_sum_sorted<V><<<blocks_for(NV, 256), 256, 0, st>>>(NV, nullptr, NV, P, nullptr, nullptr,
                                                                        voff.as<uint32_t>(), srid, rec_row.as<T>(),
                                                                        lat->vval, lat->vocc);
            FR_HIP(hipGetLastError());
        } else {
            FR_HIP(hipMemsetAsync(lat->vval, 0, NV * V * sizeof(float), st));
            FR_HIP(hipMemsetAsync(lat->vocc, 0, NV * sizeof(uint32_t), st));
            k_vertex_sum_atomic<V><<<blocks_for(P, 256), 256, 0, st>>>(P, nullptr, nullptr, rec_own.as<uint32_t>(),
                                                                        ovid.as<uint32_t>(), rec_row.as<T>(),
                                                                        lat->vval, lat->vocc, NV);
            FR_HIP(hipGetLastError());
            if constexpr (ValLayout<V>::m2) {
                k_vertex_scatter_atomic<V><<<blocks_for(P, 256), 256, 0, st>>>(
                    P, nullptr, nullptr, rec_own.as<uint32_t>(), ovid.as<uint32_t>(), rec_row.as<T>(), lat->vval,
                    NV);
                FR_HIP(hipGetLastError());
            }
        }
    }
    // the provisional table and records are no longer needed
    rec_key.reset();
    rec_row.reset();
    rec_own.reset();
    own1.reset();
    ovid.reset();

    stage.mark(3, st);
    // 5. final bucketed two-choice cuckoo tables, load factor 0.5 (a bucket per
    //    vertex; loads up to 0.6 measured no slower to slice, 0.7 fails to insert)
    constexpr uint32_t SB = SlotGeom<KW, V>::bytes;
    lat->sets_h.resize(S);
    uint64_t n2 = 0;
    for (int32_t s = 0; s < S; ++s) {
        const uint64_t nb = std::max<uint64_t>(8, (uint64_t)counts[s]);
        if (nb * kBucketSlots * SB > 0xFFFFFFFFull) {
            set_error("fr_lattice_build: set %d has %u vertices, more than one table of 4 GiB holds", s, counts[s]);
            return FR_ENOMEM;
        }
        const uint32_t cap = (uint32_t)(kBucketSlots * nb);
        lat->sets_h[s] = SetTable{nullptr, nullptr, n2, cap, counts[s], 0x2545F491u * (uint32_t)(s + 1), 0, {}};
        std::memcpy(lat->sets_h[s].k, lat->kset.data() + 8 * (size_t)s, sizeof(lat->sets_h[s].k));
        n2 += cap;
    }
    lat->n_slots = n2;
    lat->tab_bytes = n2 * SB;
    FR_TRY(dev_alloc(ctx, reinterpret_cast<void **>(&lat->tab), lat->tab_bytes));
    FR_TRY(dev_alloc(ctx, reinterpret_cast<void **>(&lat->sets_d), S * sizeof(SetTable)));
    for (int32_t s = 0; s < S; ++s) {
        char *first = reinterpret_cast<char *>(lat->tab) + lat->sets_h[s].slot_base * SB;
        lat->sets_h[s].keys = reinterpret_cast<const uint64_t *>(first);
        lat->sets_h[s].vals = reinterpret_cast<const float *>(first + SlotGeom<KW, V>::val_off);
    }
    DevBuf own2, vtmap;
    FR_TRY(own2.alloc(ctx, n2 * sizeof(uint32_t)));
    TileMap vtm{};
    FR_TRY(make_offset_map(ctx, lat->vbase, 256, st, vtmap, vtm, true));
    char *table = reinterpret_cast<char *>(lat->tab);
    const uint32_t *fail_word = reinterpret_cast<const uint32_t *>(fail.p);
    // the slots: keys of free slots, then each vertex's key and values (the fill
    // returns at once if the cuckoo pass gave up)
    auto fill_table = [&]() -> fr_status {
        if (n2 == 0) return FR_OK;
        k_slot_empty<KW, V><<<blocks_for(n2, 256), 256, 0, st>>>(n2, nullptr, own2.as<uint32_t>(), table);
        FR_HIP(hipGetLastError());
        if (vtm.n_tiles > 0) {
            k_vertex_place<KW, V><<<grid_of(vtm), 256, 0, st>>>(vtm, lat->sets_d, own2.as<uint32_t>(), lat->vkey,
                                                               lat->vval, NV, fail_word, table);
            FR_HIP(hipGetLastError());
        }
        return FR_OK;
    };
    // A caller that waits for the build gets the table filled behind the cuckoo
    // pass and one wait for both; a cuckoo pass that gave up is redone with
    // another seed and its own wait before the fill.
    for (int attempt = 0;; ++attempt) {
        FR_TRY(stage_h2d(ctx, lat->sets_d, lat->sets_h.data(), S * sizeof(SetTable), st));
        FR_HIP(hipMemsetAsync(own2.p, 0xFF, n2 * sizeof(uint32_t), st));
        FR_HIP(hipMemsetAsync(fail.p, 0, sizeof(int32_t), st));
        if (vtm.n_tiles > 0) {
            k_cuckoo_insert<KW><<<grid_of(vtm), 256, 0, st>>>(vtm, lat->sets_d, lat->vkey, NV, own2.as<uint32_t>(),
                                                             fail.as<int32_t>());
            FR_HIP(hipGetLastError());
        }
        const bool fill_now = wait_end && attempt == 0;
        if (fill_now) {
            FR_TRY(fill_table());
            stage.mark(4, st);
        }
        int32_t *rb = nullptr;
        FR_TRY(build_readback(ctx, sizeof(int32_t), reinterpret_cast<void **>(&rb)));
        FR_HIP(hipMemcpyAsync(rb, fail.p, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        FR_HIP(hipStreamSynchronize(st));
        if (!rb[0]) {
            if (fill_now) {
                stage.read(lat->stage_ms);
                return FR_OK;
            }
            break;
        }
        if (attempt >= 16) {
            set_error("fr_lattice_build: cuckoo insertion did not converge after %d seeds", attempt + 1);
            return FR_EDEVICE;
        }
        for (int32_t s = 0; s < S; ++s) lat->sets_h[s].seed = lat->sets_h[s].seed * 0x9E3779B1u + 0x7F4A7C15u;
    }
    FR_TRY(fill_table());
    stage.mark(4, st);
    if (!wait_end) return FR_OK;   // the caller orders later work after the build on the device
    FR_HIP(hipStreamSynchronize(st));
    stage.read(lat->stage_ms);
    return FR_OK;
}

fr_status build_lattice(fr_ctx *ctx, const fr_cloud *obs, const fr_lattice_params *prm, hipStream_t st,
                        fr_lattice *lat, const int64_t *valued_end, bool wait_end)
{
    const int64_t *ve = valued_end;
    const bool w = wait_end;
    if (prm->feat == 3 && prm->values == 4) return build_impl<3, 4>(ctx, obs, st, lat, ve, nullptr, w);
    if (prm->feat == 3 && prm->values == 7) return build_impl<3, 7>(ctx, obs, st, lat, ve, nullptr, w);
    if (prm->feat == 6 && prm->values == 4) return build_impl<6, 4>(ctx, obs, st, lat, ve, nullptr, w);
    if (prm->feat == 6 && prm->values == 7) return build_impl<6, 7>(ctx, obs, st, lat, ve, nullptr, w);
    if (prm->feat == 3 && prm->values == 5) return build_impl<3, 5>(ctx, obs, st, lat, ve, nullptr, w);
    if (prm->feat == 3 && prm->values == 8) return build_impl<3, 8>(ctx, obs, st, lat, ve, nullptr, w);
    if (prm->feat == 6 && prm->values == 5) return build_impl<6, 5>(ctx, obs, st, lat, ve, nullptr, w);
    if (prm->feat == 6 && prm->values == 8) return build_impl<6, 8>(ctx, obs, st, lat, ve, nullptr, w);
    set_error("fr_lattice_build: unsupported feat=%d values=%d", prm->feat, prm->values);
    return FR_EINVAL;
}

// ---------------------------------------------------------------------------
// Rebuilds in place: storage sized once from the observation cloud
// ---------------------------------------------------------------------------
// A loop that rebuilds the lattice of one observation cloud every iteration
// (the optimised variance of Sec. 3.3 changes the lattice scale each time)
// cannot afford the host waits of build_impl, which sizes its arrays from
// counts it reads back.  Here every array is sized once from bounds that hold
// for any scale: a set of n points has at most R_s = (d+1) n incidences,
// hence at most R_s partial records and R_s vertices.  The provisional table
// of a set has the next power of two >= 2 R_s slots (load <= 1/2), the final
// tables room for the 2 slots per vertex of build_impl's sizing at R_s
// vertices.  The counts themselves stay on the device (cnt words), the tile
// maps of the insertion and of the cuckoo pass take their set offsets from
// device arrays and cover the bounds (tiles past a set's count return), and
// the final tables' layout is written by a kernel from the vertex counts, so
// the tables of a rebuild are those of build_impl for the same scale.  A
// provisional overflow or a cuckoo insertion that gives up raises a word in
// cnt, which the caller reads at its own waits.
namespace {
constexpr int kResP = 0, kResNV = 1, kResSlots = 2, kResFailInsert = 3, kResFailCuckoo = 4, kResWords = 8;
}

struct ResidentBuild {
    fr_ctx *ctx = nullptr;
    fr_lattice *lat = nullptr;
    int32_t d = 3, V = 4, S = 0;
    bool sorted = true;
    Pts pts{};
    size_t R = 0, n1 = 0, n2max = 0, n_waves = 0;
    int bits = 0;
    TileMap ptm{}, rtm{}, vtm{};
    DevBuf ptmap, rtmap, vtmap;   // tile-map arrays
    DevBuf offs;                  // int64: partial offsets [S + 1], then vertex offsets [S + 1]
    DevBuf wave_cnt, rec_key, rec_row, rec_own, ovid, own1, t1;
    DevBuf rvid, rid, tk, tv, voff, own2, ws, cnt;
    // valued points of each set end here (device, n_sets; NULL: all valued)
    const int64_t *valued_end = nullptr;
    // joint rebuilds (the uncustomised filter): the joint cloud, its tile map
    // and offsets, the kernel arguments that assemble it; the blur's slot
    // offsets per set (written by k_set_tables), tile map and value buffers
    bool joint = false, blur = false, jnormals = false;
    DevBuf jpts, joff, jtmap, soff, stmap, bufa, bufb;
    TileMap jtm{}, stm{};
    Pts obs_pts{}, model_pts{};
    size_t jn = 0;   // points per array of the joint cloud
    // scale factors of rebuilds from host values: a device copy, its pinned
    // staging buffer and the event after the last copy out of it
    DevBuf kset_d;
    float *kset_pin = nullptr;
    hipEvent_t kset_ev = nullptr;
    ~ResidentBuild()
    {
        if (kset_ev != nullptr) {
            (void)hipEventSynchronize(kset_ev);
            (void)hipEventDestroy(kset_ev);
        }
        if (kset_pin != nullptr) (void)hipHostFree(kset_pin);
    }
};

// The clears a rebuild starts with, in one launch: the count and failure
// words, the wave scan's last entry, the provisional table (all ones) and the
// owner flags (R + 1 zeros).
__global__ void k_res_clear(uint32_t *cnt, uint32_t *wave_tail, uint32_t *own1, size_t n_own1, uint32_t *ovid,
                            size_t n_ovid, uint32_t *zero_a, uint32_t *zero_b, size_t n_zero)
{
    const size_t i0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x, step = (size_t)gridDim.x * blockDim.x;
    if (i0 < kResWords) cnt[i0] = 0u;
    if (i0 == 0) *wave_tail = 0u;
    for (size_t i = i0; i < n_own1; i += step) own1[i] = 0xFFFFFFFFu;
    for (size_t i = i0; i < n_ovid; i += step) ovid[i] = 0u;
    for (size_t i = i0; i < n_zero; i += step) {
        zero_a[i] = 0u;
        zero_b[i] = 0u;
    }
}

__global__ void k_fill_u32(uint32_t *p, uint32_t v, size_t n, const uint32_t *n_dev)
{
    n = dev_count(n, n_dev);
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Final tables of every set from its vertex count, with build_impl's sizing
// (max(8, n) buckets), slots back to back in set order, the
// set's seed and lattice scale: one workgroup, sets in chunks of 256.
// slot_off (or NULL): each set's first slot as int64 (set n_sets: the total).
template <int KW, int V>
__global__ void __launch_bounds__(256) k_set_tables(int32_t n_sets, const int64_t *vbase, const float *kset,
                                                   char *tab, SetTable *sets, uint32_t *n_slots,
                                                   int64_t *slot_off)
{
    using G = SlotGeom<KW, V>;
    __shared__ uint32_t wsum[4];
    __shared__ uint32_t carry;
    if (threadIdx.x == 0) carry = 0u;
    __syncthreads();
    const int lane = (int)(threadIdx.x & 63u), wave = (int)(threadIdx.x >> 6);
    for (int32_t base = 0; base < n_sets; base += 256) {
        const int32_t s = base + (int32_t)threadIdx.x;
        uint32_t count = 0u, cap = 0u;
        if (s < n_sets) {
            count = (uint32_t)(vbase[s + 1] - vbase[s]);
            const uint32_t nb = max(8u, count);
            cap = (uint32_t)kBucketSlots * nb;
        }
        const uint32_t incl = wave_inclusive_scan(cap);
        if (lane == 63) wsum[wave] = incl;
        __syncthreads();
        uint32_t before = carry;
        for (int w = 0; w < wave; ++w) before += wsum[w];
        const uint32_t first = before + incl - cap;
        if (s < n_sets) {
            SetTable t;
            char *p = tab + (size_t)G::bytes * first;
            t.keys = reinterpret_cast<const uint64_t *>(p);
            t.vals = reinterpret_cast<const float *>(p + G::val_off);
            t.slot_base = first;
            t.cap = cap;
            t.n_vertices = count;
            t.seed = 0x2545F491u * (uint32_t)(s + 1);
            t.mask = 0u;
#pragma unroll
            for (int i = 0; i < 8; ++i) t.k[i] = kset[8 * (size_t)s + i];
            sets[s] = t;
            if (slot_off != nullptr) slot_off[s] = (int64_t)first;
        }
        __syncthreads();
        if (threadIdx.x == 255) carry = first + cap;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        *n_slots = carry;
        if (slot_off != nullptr) slot_off[n_sets] = (int64_t)carry;
    }
}

// Tile map over sets whose offsets are a device array (n_sets + 1 entries) and
// whose sizes are bounded by `bound`: the tiles of the bounds, XCD-contiguous.
static fr_status make_bound_map(fr_ctx *ctx, const int64_t *dev_off, const std::vector<uint64_t> &bound, int32_t tile,
                                hipStream_t st, DevBuf &buf, TileMap &tm)
{
    const int32_t n = (int32_t)bound.size();
    std::vector<int32_t> tiles(n + 1, 0), sets(n);
    for (int32_t s = 0; s < n; ++s) {
        const uint64_t t = tiles[s] + (bound[s] + tile - 1) / tile;
        if (t >= (1ull << 31)) {
            set_error("fr_lattice_build: too many tiles");
            return FR_EINVAL;
        }
        tiles[s + 1] = (int32_t)t;
        sets[s] = s;
    }
    std::vector<char> image(sizeof(int32_t) * (2 * n + 1));
    std::memcpy(image.data(), tiles.data(), sizeof(int32_t) * (n + 1));
    std::memcpy(image.data() + sizeof(int32_t) * (n + 1), sets.data(), sizeof(int32_t) * n);
    FR_TRY(buf.alloc(ctx, image.size()));
    FR_TRY(stage_h2d(ctx, buf.p, image.data(), image.size(), st));
    tm.seg_off = dev_off;
    tm.seg_end = dev_off + 1;
    tm.seg_tile = buf.as<int32_t>();
    tm.seg_set = buf.as<int32_t>() + n + 1;
    tm.n_seg = n;
    tm.n_tiles = tiles[n];
    tm.tile = tile;
    tm.xcd_chunk = tm.n_tiles >= 8 * 64 ? (tm.n_tiles + 7) / 8 : 0;
    return FR_OK;
}

template <int d, int V>
static fr_status resident_blur(ResidentBuild *rb, hipStream_t st);

template <int d, int V>
static fr_status resident_enqueue(ResidentBuild *rb, const float *kset, hipStream_t st)
{
    constexpr int KW = KeyWords<d>::value;
    using T = typename PartialType<V>::T;
    fr_ctx *ctx = rb->ctx;
    fr_lattice *lat = rb->lat;
    const int32_t S = rb->S;
    const size_t R = rb->R;
    uint32_t *cnt = rb->cnt.as<uint32_t>();
    uint32_t *ws = rb->ws.as<uint32_t>();
    uint32_t *wave_cnt = rb->wave_cnt.as<uint32_t>();
    int64_t *poff = rb->offs.as<int64_t>(), *voff64 = poff + S + 1;
    // counts, failure words, the wave scan's last entry, the provisional table and the owner flags
    // (and, for the sums by vertex lists, the per-vertex counters)
    const bool lists = rb->sorted && R <= kListMax;
    k_res_clear<<<blocks_for(std::max<size_t>(2 * rb->n1, R + 1), 256), 256, 0, st>>>(
        cnt, wave_cnt + rb->n_waves, rb->own1.as<uint32_t>(), 2 * rb->n1, rb->ovid.as<uint32_t>(), R + 1,
        lists ? rb->voff.as<uint32_t>() : nullptr, lists ? rb->tk.as<uint32_t>() : nullptr, lists ? R : 0);
    // 1. partial records
    k_build_count<d><<<rb->ptm.n_tiles, 256, 0, st>>>(rb->pts, rb->ptm, kset, wave_cnt, lat->err_d);
    FR_HIP(hipGetLastError());
    FR_TRY(scan_exclusive_u32(ctx, wave_cnt, wave_cnt, rb->n_waves + 1, 0, st, ws));
    k_build_partials<d, V><<<rb->ptm.n_tiles, 256, 0, st>>>(rb->pts, rb->ptm, kset, wave_cnt,
                                                            rb->rec_key.as<uint64_t>(), rb->rec_row.as<T>(), R,
                                                            rb->valued_end, poff, cnt + kResP);
    FR_HIP(hipGetLastError());
    // 2.-3. provisional tables, vertex ids and per-set vertex offsets
    k_insert_records<KW, true><<<grid_of(rb->rtm), 256, 0, st>>>(rb->rtm, rb->t1.as<SetTable>(),
                                                                rb->rec_key.as<uint64_t>(), R,
                                                                rb->own1.as<unsigned long long>(),
                                                                rb->rec_own.as<uint32_t>(), rb->ovid.as<uint32_t>(),
                                                                reinterpret_cast<int32_t *>(cnt + kResFailInsert));
    FR_HIP(hipGetLastError());
    FR_TRY(scan_exclusive_u32(ctx, rb->ovid.as<uint32_t>(), rb->ovid.as<uint32_t>(), R + 1, 0, st, ws));
    k_owner_emit<KW><<<blocks_for(R, 256), 256, 0, st>>>(R, rb->ovid.as<uint32_t>(), rb->rec_key.as<uint64_t>(),
                                                         lat->vkey, R, S, poff, voff64, cnt + kResNV);
    FR_HIP(hipGetLastError());
    // 4. values
    if (rb->sorted && R <= kListMax) {
        const uint32_t *fail_ins = cnt + kResFailInsert;
        uint32_t *vcount = rb->voff.as<uint32_t>(), *vfill = rb->tk.as<uint32_t>();   // zeroed by k_res_clear
        k_list_count<<<blocks_for(R, 256), 256, 0, st>>>(R, cnt + kResP, fail_ins, rb->rec_own.as<uint32_t>(),
                                                          rb->ovid.as<uint32_t>(), rb->rvid.as<uint32_t>(),
                                                          vcount);
        FR_TRY(scan_exclusive_u32(ctx, vcount, rb->rid.as<uint32_t>(), R, 0, st, ws));
        k_list_place<<<blocks_for(R, 256), 256, 0, st>>>(R, cnt + kResP, fail_ins, rb->rvid.as<uint32_t>(),
                                                          rb->rid.as<uint32_t>(), vfill, rb->tv.as<uint32_t>());
        k_vertex_sum_list<V><<<blocks_for(R, 256), 256, 0, st>>>(R, cnt + kResNV, R, fail_ins,
                                                                  rb->rid.as<uint32_t>(), vcount,
                                                                  rb->tv.as<uint32_t>(), rb->rec_row.as<T>(),
                                                                  lat->vval, lat->vocc);
        FR_HIP(hipGetLastError());
    } else if (rb->sorted) {
        const uint32_t *fail_ins = cnt + kResFailInsert;
        k_record_vertex<<<blocks_for(R, 256), 256, 0, st>>>(R, cnt + kResP, fail_ins, rb->rec_own.as<uint32_t>(),
                                                             rb->ovid.as<uint32_t>(), rb->rvid.as<uint32_t>(),
                                                             rb->rid.as<uint32_t>());
        uint32_t *svid = nullptr, *srid = nullptr;
        FR_TRY(radix_sort_pairs(ctx, rb->rvid.as<uint32_t>(), rb->rid.as<uint32_t>(), rb->tk.as<uint32_t>(),
                                rb->tv.as<uint32_t>(), R, rb->bits, st, &svid, &srid, cnt + kResP, ws));
        k_segment_heads<<<blocks_for(R, 256), 256, 0, st>>>(R, cnt + kResP, fail_ins, svid, rb->voff.as<uint32_t>());
        k_vertex_sum_sorted<V><<<blocks_for(R, 256), 256, 0, st>>>(R, cnt + kResNV, R, R, cnt + kResP, fail_ins,
                                                                    rb->voff.as<uint32_t>(), srid,
                                                                    rb->rec_row.as<T>(), lat->vval, lat->vocc);
        FR_HIP(hipGetLastError());
    } else {
        k_fill_u32<<<blocks_for((size_t)V * R, 256), 256, 0, st>>>(reinterpret_cast<uint32_t *>(lat->vval), 0u,
                                                                    (size_t)V * R, nullptr);
        k_fill_u32<<<blocks_for(R, 256), 256, 0, st>>>(lat->vocc, 0u, R, nullptr);
        k_vertex_sum_atomic<V><<<blocks_for(R, 256), 256, 0, st>>>(R, cnt + kResP, cnt + kResFailInsert,
                                                                    rb->rec_own.as<uint32_t>(),
                                                                    rb->ovid.as<uint32_t>(), rb->rec_row.as<T>(),
                                                                    lat->vval, lat->vocc, R);
        if constexpr (ValLayout<V>::m2)
            k_vertex_scatter_atomic<V><<<blocks_for(R, 256), 256, 0, st>>>(
                R, cnt + kResP, cnt + kResFailInsert, rb->rec_own.as<uint32_t>(), rb->ovid.as<uint32_t>(),
                rb->rec_row.as<T>(), lat->vval, R);
        FR_HIP(hipGetLastError());
    }
    // 5. final tables
    char *table = reinterpret_cast<char *>(lat->tab);
    k_set_tables<KW, V><<<1, 256, 0, st>>>(S, voff64, kset, table, lat->sets_d, cnt + kResSlots,
                                           rb->blur ? rb->soff.as<int64_t>() : nullptr);
    k_fill_u32<<<blocks_for(rb->n2max, 256), 256, 0, st>>>(rb->own2.as<uint32_t>(), kOwnerEmpty, rb->n2max,
                                                           cnt + kResSlots);
    k_cuckoo_insert<KW><<<grid_of(rb->vtm), 256, 0, st>>>(rb->vtm, lat->sets_d, lat->vkey, R,
                                                         rb->own2.as<uint32_t>(),
                                                         reinterpret_cast<int32_t *>(cnt + kResFailCuckoo));
    k_slot_empty<KW, V><<<blocks_for(rb->n2max, 256), 256, 0, st>>>(rb->n2max, cnt + kResSlots,
                                                                   rb->own2.as<uint32_t>(), table);
    k_vertex_place<KW, V><<<grid_of(rb->vtm), 256, 0, st>>>(rb->vtm, lat->sets_d, rb->own2.as<uint32_t>(), lat->vkey,
                                                           lat->vval, R, cnt + kResFailCuckoo, table);
    FR_HIP(hipGetLastError());
    if constexpr (V == 4 || V == 7)
        if (rb->blur) FR_TRY((resident_blur<d, V>(rb, st)));
    return FR_OK;
}

template <int d, int V>
static fr_status resident_setup(ResidentBuild *rb, const fr_cloud *obs, hipStream_t st)
{
    constexpr int D = d + 1;
    constexpr int KW = KeyWords<d>::value;
    using T = typename PartialType<V>::T;
    constexpr uint32_t SB = SlotGeom<KW, V>::bytes;
    fr_ctx *ctx = rb->ctx;
    fr_lattice *lat = rb->lat;
    const int32_t S = obs->n_sets;
    const size_t R = rb->R;
    std::vector<int64_t> off(obs->offsets, obs->offsets + S + 1);
    FR_TRY(make_offset_map(ctx, off, 256, st, rb->ptmap, rb->ptm, false));
    rb->n_waves = (size_t)rb->ptm.n_tiles * 4;
    std::vector<uint64_t> bound(S);
    std::vector<SetTable> t1(S);
    uint64_t n1 = 0, n2 = 0;
    for (int32_t s = 0; s < S; ++s) {
        const uint64_t rs = (uint64_t)(obs->offsets[s + 1] - obs->offsets[s]) * D;
        bound[s] = rs;
        const uint32_t cap = next_pow2(2 * rs);
        if (2 * rs > (1ull << 31)) {
            set_error("fr_lattice_build: set %d has too many incidences (%llu)", s, (unsigned long long)rs);
            return FR_EINVAL;
        }
        t1[s] = SetTable{nullptr, nullptr, n1, cap, 0, 0, cap - 1, {}};
        n1 += cap;
        const uint64_t slots = (uint64_t)kBucketSlots * std::max<uint64_t>(8, rs);
        if (slots * SB > 0xFFFFFFFFull) {
            set_error("fr_lattice_build: set %d may need more than one table of 4 GiB", s);
            return FR_ENOMEM;
        }
        n2 += slots;
    }
    if (n1 >= 0xFFFFFFF0ull || n2 >= 0xFFFFFFF0ull || R + 1 >= 0xFFFFFFF0ull) {
        set_error("fr_lattice_build: tables too large for an in-place rebuild");
        return FR_EINVAL;
    }
    rb->n1 = n1;
    rb->n2max = n2;
    int bits = 0;
    while (bits < 32 && (R - 1) >> bits) ++bits;
    rb->bits = bits;
    FR_TRY(rb->offs.alloc(ctx, 2 * (S + 1) * sizeof(int64_t)));
    FR_TRY(make_bound_map(ctx, rb->offs.as<int64_t>(), bound, 256, st, rb->rtmap, rb->rtm));
    FR_TRY(make_bound_map(ctx, rb->offs.as<int64_t>() + S + 1, bound, 256, st, rb->vtmap, rb->vtm));
    FR_TRY(rb->wave_cnt.alloc(ctx, (rb->n_waves + 1) * sizeof(uint32_t)));
    FR_TRY(rb->rec_key.alloc(ctx, R * KW * sizeof(uint64_t)));
    FR_TRY(rb->rec_row.alloc(ctx, R * PartialRow<V>::S * sizeof(T)));
    FR_TRY(rb->rec_own.alloc(ctx, R * sizeof(uint32_t)));
    FR_TRY(rb->ovid.alloc(ctx, (R + 1) * sizeof(uint32_t)));
    FR_TRY(rb->own1.alloc(ctx, n1 * sizeof(unsigned long long)));
    FR_TRY(rb->t1.alloc(ctx, S * sizeof(SetTable)));
    if (rb->sorted) {
        FR_TRY(rb->rvid.alloc(ctx, R * sizeof(uint32_t)));
        FR_TRY(rb->rid.alloc(ctx, R * sizeof(uint32_t)));
        FR_TRY(rb->tk.alloc(ctx, R * sizeof(uint32_t)));
        FR_TRY(rb->tv.alloc(ctx, R * sizeof(uint32_t)));
        FR_TRY(rb->voff.alloc(ctx, R * sizeof(uint32_t)));
    }
    FR_TRY(rb->own2.alloc(ctx, n2 * sizeof(uint32_t)));
    const size_t ws = std::max({scan_ws_words(rb->n_waves + 1), scan_ws_words(R + 1), radix_ws_words(R)});
    FR_TRY(rb->ws.alloc(ctx, std::max<size_t>(ws, 1) * sizeof(uint32_t)));
    FR_TRY(rb->cnt.alloc(ctx, kResWords * sizeof(uint32_t)));
    FR_TRY(stage_h2d(ctx, rb->t1.p, t1.data(), S * sizeof(SetTable), st));
    // the lattice the rebuilds fill: tables at their bound, vertex arrays of R vertices
    lat->n_slots = n2;
    lat->tab_bytes = n2 * SB;
    FR_TRY(dev_alloc(ctx, reinterpret_cast<void **>(&lat->tab), lat->tab_bytes));
    lat->sets_h.assign(S, SetTable{});
    FR_TRY(dev_alloc(ctx, reinterpret_cast<void **>(&lat->sets_d), S * sizeof(SetTable)));
    lat->vert_bytes = R * (KW * sizeof(uint64_t) + sizeof(uint32_t) + V * sizeof(float)) + 64;
    {
        void *p = nullptr;
        FR_TRY(dev_alloc(ctx, &p, lat->vert_bytes));
        char *c = static_cast<char *>(p);
        lat->vkey = reinterpret_cast<uint64_t *>(c);
        lat->vval = reinterpret_cast<float *>(c + R * KW * sizeof(uint64_t));
        lat->vocc = reinterpret_cast<uint32_t *>(c + R * (KW * sizeof(uint64_t) + V * sizeof(float)));
    }
    return FR_OK;
}

fr_status resident_create(fr_ctx *ctx, const fr_cloud *obs, const fr_lattice_params *prm, hipStream_t st,
                          ResidentBuild **out)
{
    *out = nullptr;
    const int64_t N = cloud_points(obs);
    const size_t R = (size_t)N * (prm->feat + 1);
    if (N <= 0 || prm->feat > 6) {
        set_error("fr_lattice_build: an in-place rebuild needs observation points and d <= 6");
        return FR_EINVAL;
    }
    if (R >= 0xFFFFFFF0ull) {
        set_error("fr_lattice_build: %llu incidences exceed the 32-bit record index", (unsigned long long)R);
        return FR_EINVAL;
    }
    ResidentBuild *rb = new (std::nothrow) ResidentBuild();
    fr_lattice *lat = new (std::nothrow) fr_lattice();
    if (rb == nullptr || lat == nullptr) {
        delete rb;
        delete lat;
        set_error("out of host memory");
        return FR_ENOMEM;
    }
    rb->ctx = ctx;
    rb->lat = lat;
    rb->d = prm->feat;
    rb->V = prm->values;
    rb->S = obs->n_sets;
    rb->R = R;
    rb->sorted = prm->splat == FR_SPLAT_SORTED;
    rb->pts = Pts{obs->x, obs->y, obs->z, obs->nx, obs->ny, obs->nz};
    lat->resident = rb;
    lat->params = *prm;
    lat->ctx = ctx;
    lat->d = prm->feat;
    lat->V = prm->values;
    lat->KW = (prm->feat + 2) / 3;
    lat->n_sets = obs->n_sets;
    lat->splat = prm->splat;
    lat->n_points_total = N;
    fr_status s = dev_alloc(ctx, reinterpret_cast<void **>(&lat->err_d), sizeof(int32_t));
    if (s == FR_OK) {
        const hipError_t e = hipMemsetAsync(lat->err_d, 0, sizeof(int32_t), st);
        if (e != hipSuccess) {
            set_error("HIP error: %s", hipGetErrorString(e));
            s = FR_EDEVICE;
        }
    }
    if (s == FR_OK) {
        const int f = prm->feat, v = prm->values;
        if (f == 3 && v == 4) s = resident_setup<3, 4>(rb, obs, st);
        else if (f == 3 && v == 5) s = resident_setup<3, 5>(rb, obs, st);
        else if (f == 3 && v == 7) s = resident_setup<3, 7>(rb, obs, st);
        else if (f == 3 && v == 8) s = resident_setup<3, 8>(rb, obs, st);
        else if (f == 6 && v == 4) s = resident_setup<6, 4>(rb, obs, st);
        else if (f == 6 && v == 5) s = resident_setup<6, 5>(rb, obs, st);
        else if (f == 6 && v == 7) s = resident_setup<6, 7>(rb, obs, st);
        else if (f == 6 && v == 8) s = resident_setup<6, 8>(rb, obs, st);
        else {
            set_error("fr_lattice_build: unsupported feat=%d values=%d", f, v);
            s = FR_EINVAL;
        }
    }
    if (s != FR_OK) {
        resident_destroy(rb, st);
        return s;
    }
    *out = rb;
    return FR_OK;
}

fr_status resident_build(ResidentBuild *rb, const float *kset, hipStream_t st)
{
    const int d = rb->d, v = rb->V;
    if (d == 3 && v == 4) return resident_enqueue<3, 4>(rb, kset, st);
    if (d == 3 && v == 5) return resident_enqueue<3, 5>(rb, kset, st);
    if (d == 3 && v == 7) return resident_enqueue<3, 7>(rb, kset, st);
    if (d == 3 && v == 8) return resident_enqueue<3, 8>(rb, kset, st);
    if (d == 6 && v == 4) return resident_enqueue<6, 4>(rb, kset, st);
    if (d == 6 && v == 5) return resident_enqueue<6, 5>(rb, kset, st);
    if (d == 6 && v == 7) return resident_enqueue<6, 7>(rb, kset, st);
    return resident_enqueue<6, 8>(rb, kset, st);
}

fr_status resident_build_host(ResidentBuild *rb, const float *kset_h, hipStream_t st)
{
    const size_t bytes = 8 * (size_t)rb->S * sizeof(float);
    if (rb->kset_pin == nullptr) {
        FR_TRY(rb->kset_d.alloc(rb->ctx, bytes));
        FR_HIP(hipHostMalloc(reinterpret_cast<void **>(&rb->kset_pin), bytes, hipHostMallocDefault));
        FR_HIP(hipEventCreateWithFlags(&rb->kset_ev, hipEventDisableTiming));
    } else {
        FR_HIP(hipEventSynchronize(rb->kset_ev));   // the last rebuild's copy has left the staging buffer
    }
    std::memcpy(rb->kset_pin, kset_h, bytes);
    FR_HIP(hipMemcpyAsync(rb->kset_d.p, rb->kset_pin, bytes, hipMemcpyHostToDevice, st));
    FR_HIP(hipEventRecord(rb->kset_ev, st));
    return resident_build(rb, rb->kset_d.as<float>(), st);
}

fr_lattice *resident_lattice(ResidentBuild *rb) { return rb->lat; }

const uint32_t *resident_fail_words(const ResidentBuild *rb) { return rb->cnt.as<uint32_t>() + kResFailInsert; }

void resident_destroy(ResidentBuild *rb, hipStream_t st, bool idle)
{
    if (rb == nullptr) return;
    if (rb->lat != nullptr) {
        free_lattice(rb->lat, st, idle);
        rb->lat->magic = kDeadMagic;
        delete rb->lat;
    }
    delete rb;   // the DevBufs release in the order of their streams
}

bool feature_dim_supported(int dim) { return dim == 8 || dim == 16 || dim == 32; }

fr_status build_feature_lattice(fr_ctx *ctx, const fr_cloud *obs, const float *feat, hipStream_t st,
                                fr_lattice *lat)
{
    if (lat->d == 8) return build_impl<8, 4>(ctx, obs, st, lat, nullptr, feat);
    if (lat->d == 16) return build_impl<16, 4>(ctx, obs, st, lat, nullptr, feat);
    if (lat->d == 32) return build_impl<32, 4>(ctx, obs, st, lat, nullptr, feat);
    set_error("descriptor dimension %d not supported (8, 16 or 32)", lat->d);
    return FR_EINVAL;
}

// ---------------------------------------------------------------------------
// Uncustomised filter: joint splat of [Y, X] and the blur of the cited
// permutohedral method
// ---------------------------------------------------------------------------

// One thread per point of the joint cloud: set s holds its observation points
// first (copied) and then its model points moved by the set's [R | t] (the
// E-step's own pinned transform, so the slice finds the same simplices).
struct JointArgs {
    TileMap tm;                       // segments = sets of the joint cloud
    const int64_t *obs_off, *model_off;
    Pts obs, model;
    const float *mats;                // n_sets x 12, or NULL (identity)
    float *x, *y, *z, *nx, *ny, *nz;  // joint cloud (normals may be NULL)
};

__global__ void __launch_bounds__(256) k_joint_points(JointArgs a)
{
    const int32_t t = logical_tile(a.tm);
    if (t >= a.tm.n_tiles) return;
    const int32_t s = tile_segment(a.tm, t);
    const int64_t i = a.tm.seg_off[s] + (int64_t)(t - a.tm.seg_tile[s]) * a.tm.tile + threadIdx.x;
    if (i >= a.tm.seg_end[s]) return;
    const int64_t local = i - a.tm.seg_off[s];
    const int64_t n_obs = a.obs_off[s + 1] - a.obs_off[s];
    float px, py, pz, qx = 0.0f, qy = 0.0f, qz = 0.0f;
    if (local < n_obs) {
        const int64_t j = a.obs_off[s] + local;
        px = a.obs.x[j];
        py = a.obs.y[j];
        pz = a.obs.z[j];
        if (a.obs.nx != nullptr) {
            qx = a.obs.nx[j];
            qy = a.obs.ny[j];
            qz = a.obs.nz[j];
        }
    } else {
        const int64_t j = a.model_off[s] + local - n_obs;
        px = a.model.x[j];
        py = a.model.y[j];
        pz = a.model.z[j];
        if (a.model.nx != nullptr) {
            qx = a.model.nx[j];
            qy = a.model.ny[j];
            qz = a.model.nz[j];
        }
        if (a.mats != nullptr) {
            const float *m = a.mats + 12 * (size_t)s;
            xform_point(m, px, py, pz, px, py, pz);
            xform_normal(m, qx, qy, qz, qx, qy, qz);
        }
    }
    a.x[i] = px;
    a.y[i] = py;
    a.z[i] = pz;
    if (a.nx != nullptr) {
        a.nx[i] = qx;
        a.ny[i] = qy;
        a.nz[i] = qz;
    }
}

fr_status build_joint_lattice(fr_ctx *ctx, const fr_cloud *obs, const fr_cloud *model, const float *mats,
                              const fr_lattice_params *prm, hipStream_t st, fr_lattice *lat)
{
    const int32_t S = obs->n_sets;
    std::vector<int64_t> off(S + 1, 0), vend(S);
    for (int32_t s = 0; s < S; ++s) {
        const int64_t no = obs->offsets[s + 1] - obs->offsets[s], nm = model->offsets[s + 1] - model->offsets[s];
        off[s + 1] = off[s] + no + nm;
        vend[s] = off[s] + no;
    }
    const int64_t T = off[S];
    const bool normals = obs->nx != nullptr;
    DevBuf pts, offs, tmap;
    FR_TRY(pts.alloc(ctx, std::max<int64_t>(T, 1) * (normals ? 6 : 3) * sizeof(float)));
    FR_TRY(offs.alloc(ctx, (3 * (size_t)S + 2) * sizeof(int64_t)));
    int64_t *od = offs.as<int64_t>();
    FR_TRY(stage_h2d(ctx, od, obs->offsets, (S + 1) * sizeof(int64_t), st));
    FR_TRY(stage_h2d(ctx, od + S + 1, model->offsets, (S + 1) * sizeof(int64_t), st));
    FR_TRY(stage_h2d(ctx, od + 2 * S + 2, vend.data(), S * sizeof(int64_t), st));
    TileMap tm{};
    FR_TRY(make_offset_map(ctx, off, 256, st, tmap, tm));
    float *base = pts.as<float>();
    const size_t n = (size_t)std::max<int64_t>(T, 1);
    JointArgs a{tm, od, od + S + 1, Pts{obs->x, obs->y, obs->z, obs->nx, obs->ny, obs->nz},
                Pts{model->x, model->y, model->z, model->nx, model->ny, model->nz}, mats, base, base + n,
                base + 2 * n, normals ? base + 3 * n : nullptr, normals ? base + 4 * n : nullptr,
                normals ? base + 5 * n : nullptr};
    if (tm.n_tiles > 0) {
        k_joint_points<<<tm.n_tiles, 256, 0, st>>>(a);
        FR_HIP(hipGetLastError());
    }
    fr_cloud joint{a.x, a.y, a.z, a.nx, a.ny, a.nz, off.data(), S};
    return build_lattice(ctx, &joint, prm, st, lat, od + 2 * S + 2);
}

// Neighbour of a packed key along lattice direction j (0 <= j <= d): every
// coordinate +sgn, coordinate j (stored only for j < d) -sgn d.  False when a
// coordinate would leave the packed range (such a vertex cannot exist).
template <int d>
__device__ __forceinline__ bool neighbour_key(const uint64_t (&key)[KeyWords<d>::value], int j, int sgn,
                                              uint64_t (&out)[KeyWords<d>::value])
{
    constexpr int KW = KeyWords<d>::value;
    bool ok = true;
#pragma unroll
    for (int w = 0; w < KW; ++w) out[w] = 0;
#pragma unroll
    for (int i = 0; i < d; ++i) {
        const int32_t c = unpack_coord(key, i) + (i == j ? -sgn * d : sgn);
        ok = ok && c >= -kKeyBias && c < kKeyBias;
        out[i / 3] |= (uint64_t)((uint32_t)(c + kKeyBias) & ((1u << kKeyBits) - 1u)) << (kKeyBits * (2 - (i % 3)));
    }
    return ok;
}

// One blur pass along direction `dir`: every slot of every set (one thread per
// slot) takes 1/2 its own values plus 1/4 of each neighbour's, read from `tin`
// (VP binary32 per slot, slots in table order); absent neighbours read as
// zero; empty slots stay zero.  `scale` multiplies the result (the filter's
// output scale on the last pass, 1 before).  Keys come from the table.
template <int d, int V>
__global__ void __launch_bounds__(256) k_blur_pass(TileMap tm, const SetTable *sets, int dir, const float *tin,
                                                  float *tout, float scale)
{
    constexpr int KW = KeyWords<d>::value;
    constexpr int VP = ValPad<V>::value;
    using G = SlotGeom<KW, V>;
    const int32_t t = logical_tile(tm);
    if (t >= tm.n_tiles) return;
    const int32_t s = tile_segment(tm, t);
    const int64_t q = tm.seg_off[s] + (int64_t)(t - tm.seg_tile[s]) * tm.tile + threadIdx.x;
    if (q >= tm.seg_end[s]) return;
    const SetTable st = sets[tm.seg_set[s]];
    uint64_t key[KW];
    load_key<KW>(st.keys, (uint32_t)(q - (int64_t)st.slot_base) * G::bytes, key);
    float acc[VP];
#pragma unroll
    for (int c = 0; c < VP; ++c) acc[c] = 0.0f;
    if (key[0] != kKeyEmpty) {
#pragma unroll
        for (int c = 0; c < V; ++c) acc[c] = 0.5f * tin[(size_t)VP * q + c];
#pragma unroll
        for (int sgn = -1; sgn <= 1; sgn += 2) {
            uint64_t nk[KW];
            if (!neighbour_key<d>(key, dir, sgn, nk)) continue;
            const int64_t r = find_slot<KW, V>(st, nk);
            if (r < 0) continue;
            const float *src = tin + (size_t)VP * (st.slot_base + (uint64_t)r);
#pragma unroll
            for (int c = 0; c < V; ++c) acc[c] = fmaf(0.25f, src[c], acc[c]);
        }
#pragma unroll
        for (int c = 0; c < V; ++c) acc[c] *= scale;
    }
    float4 *dst = reinterpret_cast<float4 *>(tout + (size_t)VP * q);
    dst[0] = make_float4(acc[0], acc[1], acc[2], acc[3]);
    if constexpr (VP == 8) dst[1] = make_float4(acc[4], acc[5], acc[6], acc[7]);
}

// Copy the values of every slot between the table and a plain array of VP
// binary32 per slot (to_table false: out of the table, zeros for a free slot,
// whose values the fill leaves unwritten; true: back in).
template <int KW, int V>
__global__ void __launch_bounds__(256) k_slot_values(size_t n_slots, const uint32_t *n_dev, char *table, float *plain,
                                                    bool to_table)
{
    using G = SlotGeom<KW, V>;
    constexpr int VP = ValPad<V>::value;
    const size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= dev_count(n_slots, n_dev)) return;
    const bool free_slot = reinterpret_cast<const uint64_t *>(table + G::bytes * j)[0] == kKeyEmpty;
    float4 *tv = reinterpret_cast<float4 *>(table + G::bytes * j + G::val_off);
    float4 *pv = reinterpret_cast<float4 *>(plain + (size_t)VP * j);
#pragma unroll
    for (int c = 0; c < VP / 4; ++c) {
        if (to_table)
            tv[c] = pv[c];
        else
            pv[c] = free_slot ? make_float4(0.0f, 0.0f, 0.0f, 0.0f) : tv[c];
    }
}

// Copy the table values back to the vertex arrays (export reads those).
template <int d, int V>
__global__ void __launch_bounds__(256) k_table_to_vertices(TileMap tm, const SetTable *sets, const uint64_t *vkey,
                                                          size_t NV, float *vval)
{
    constexpr int KW = KeyWords<d>::value;
    using G = SlotGeom<KW, V>;
    const int32_t t = logical_tile(tm);
    if (t >= tm.n_tiles) return;
    const int32_t s = tile_segment(tm, t);
    const int64_t v = tm.seg_off[s] + (int64_t)(t - tm.seg_tile[s]) * tm.tile + threadIdx.x;
    if (v >= tm.seg_end[s]) return;
    const SetTable st = sets[tm.seg_set[s]];
    uint64_t key[KW];
#pragma unroll
    for (int w = 0; w < KW; ++w) key[w] = vkey[(size_t)w * NV + v];
    const int64_t r = find_slot<KW, V>(st, key);
    if (r < 0) return;   // cannot happen: every vertex sits in its set's table
    float val[8];
    load_vals<V>(st.vals, (uint32_t)r * G::bytes, val);
#pragma unroll
    for (int c = 0; c < V; ++c) vval[(size_t)c * NV + v] = val[c];
}

template <int d, int V>
static fr_status blur_impl(fr_lattice *lat, hipStream_t st)
{
    constexpr int KW = KeyWords<d>::value;
    constexpr int VP = ValPad<V>::value;
    fr_ctx *ctx = lat->ctx;
    StreamScope scope(st);   // temporaries are freed in the order of st
    const int32_t S = lat->n_sets;
    std::vector<int64_t> soff(S + 1, 0);
    for (int32_t s = 0; s < S; ++s) soff[s + 1] = soff[s] + lat->sets_h[s].cap;
    DevBuf bufa, bufb, smap, vmap;
    TileMap stm{}, vtm{};
    FR_TRY(make_offset_map(ctx, soff, 256, st, smap, stm));
    FR_TRY(make_offset_map(ctx, lat->vbase, 256, st, vmap, vtm));
    const size_t n = (size_t)lat->n_slots;
    if (n == 0) return FR_OK;
    FR_TRY(bufa.alloc(ctx, n * VP * sizeof(float)));
    FR_TRY(bufb.alloc(ctx, n * VP * sizeof(float)));
    char *table = reinterpret_cast<char *>(lat->tab);
    float *bufs[2] = {bufa.as<float>(), bufb.as<float>()};
    k_slot_values<KW, V><<<blocks_for(n, 256), 256, 0, st>>>(n, nullptr, table, bufs[0], false);
    FR_HIP(hipGetLastError());
    const float scale = (float)(1.0 / (1.0 + std::ldexp(1.0, -d)));
    for (int j = 0; j <= d; ++j) {
        k_blur_pass<d, V><<<stm.n_tiles, 256, 0, st>>>(stm, lat->sets_d, j, bufs[j & 1], bufs[(j + 1) & 1],
                                                       j == d ? scale : 1.0f);
        FR_HIP(hipGetLastError());
    }
    k_slot_values<KW, V><<<blocks_for(n, 256), 256, 0, st>>>(n, nullptr, table, bufs[(d + 1) & 1], true);
    FR_HIP(hipGetLastError());
    if (vtm.n_tiles > 0) {
        k_table_to_vertices<d, V><<<vtm.n_tiles, 256, 0, st>>>(vtm, lat->sets_d, lat->vkey,
                                                               (size_t)lat->n_vertices_total, lat->vval);
        FR_HIP(hipGetLastError());
    }
    return FR_OK;
}

// The blur of a lattice rebuilt in place: the slots of set s start at the
// device offset k_set_tables wrote; the tile map covers each set's bound and
// the value buffers the bound of all slots.
template <int d, int V>
static fr_status resident_blur(ResidentBuild *rb, hipStream_t st)
{
    constexpr int KW = KeyWords<d>::value;
    fr_lattice *lat = rb->lat;
    uint32_t *cnt = rb->cnt.as<uint32_t>();
    const size_t n = rb->n2max;
    char *table = reinterpret_cast<char *>(lat->tab);
    float *bufs[2] = {rb->bufa.as<float>(), rb->bufb.as<float>()};
    k_slot_values<KW, V><<<blocks_for(n, 256), 256, 0, st>>>(n, cnt + kResSlots, table, bufs[0], false);
    FR_HIP(hipGetLastError());
    const float scale = (float)(1.0 / (1.0 + std::ldexp(1.0, -d)));
    for (int j = 0; j <= d; ++j) {
        k_blur_pass<d, V><<<grid_of(rb->stm), 256, 0, st>>>(rb->stm, lat->sets_d, j, bufs[j & 1], bufs[(j + 1) & 1],
                                                          j == d ? scale : 1.0f);
        FR_HIP(hipGetLastError());
    }
    k_slot_values<KW, V><<<blocks_for(n, 256), 256, 0, st>>>(n, cnt + kResSlots, table, bufs[(d + 1) & 1], true);
    FR_HIP(hipGetLastError());
    return FR_OK;
}

fr_status resident_create_joint(fr_ctx *ctx, const fr_cloud *obs, const fr_cloud *model,
                                const fr_lattice_params *prm, hipStream_t st, ResidentBuild **out)
{
    *out = nullptr;
    if ((prm->values != 4 && prm->values != 7) || prm->feat > 6) {
        set_error("fr_register: the uncustomised filter needs values FR_VAL_PT2PT or FR_VAL_PT2PL");
        return FR_EINVAL;
    }
    const int32_t S = obs->n_sets;
    std::vector<int64_t> off(S + 1, 0), vend(S);
    for (int32_t s = 0; s < S; ++s) {
        const int64_t no = obs->offsets[s + 1] - obs->offsets[s], nm = model->offsets[s + 1] - model->offsets[s];
        off[s + 1] = off[s] + no + nm;
        vend[s] = off[s] + no;
    }
    const int64_t T = off[S];
    const bool normals = obs->nx != nullptr;
    // the joint cloud's layout; its arrays are attached once the build's storage exists
    fr_cloud joint{nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, off.data(), S};
    ResidentBuild *rb = nullptr;
    FR_TRY(resident_create(ctx, &joint, prm, st, &rb));
    auto fail = [&](fr_status s) {
        resident_destroy(rb, st);
        return s;
    };
    const size_t n = (size_t)std::max<int64_t>(T, 1);
    fr_status s = rb->jpts.alloc(ctx, n * (normals ? 6 : 3) * sizeof(float));
    if (s == FR_OK) s = rb->joff.alloc(ctx, (3 * (size_t)S + 2) * sizeof(int64_t));
    if (s != FR_OK) return fail(s);
    int64_t *od = rb->joff.as<int64_t>();
    s = stage_h2d(ctx, od, obs->offsets, (S + 1) * sizeof(int64_t), st);
    if (s == FR_OK) s = stage_h2d(ctx, od + S + 1, model->offsets, (S + 1) * sizeof(int64_t), st);
    if (s == FR_OK) s = stage_h2d(ctx, od + 2 * S + 2, vend.data(), S * sizeof(int64_t), st);
    if (s == FR_OK) s = make_offset_map(ctx, off, 256, st, rb->jtmap, rb->jtm);
    if (s != FR_OK) return fail(s);
    float *base = rb->jpts.as<float>();
    rb->pts = Pts{base, base + n, base + 2 * n, normals ? base + 3 * n : nullptr, normals ? base + 4 * n : nullptr,
                  normals ? base + 5 * n : nullptr};
    rb->obs_pts = Pts{obs->x, obs->y, obs->z, obs->nx, obs->ny, obs->nz};
    rb->model_pts = Pts{model->x, model->y, model->z, model->nx, model->ny, model->nz};
    rb->jn = n;
    rb->jnormals = normals;
    rb->valued_end = od + 2 * S + 2;
    rb->joint = true;
    // the blur's storage: slot offsets, a tile map over each set's bound of slots, two value buffers
    const int D = prm->feat + 1;
    std::vector<uint64_t> slot_bound(S);
    for (int32_t q = 0; q < S; ++q)
        slot_bound[q] = (uint64_t)kBucketSlots * std::max<uint64_t>(8, (uint64_t)(off[q + 1] - off[q]) * D);
    const int VP = prm->values <= 4 ? 4 : 8;
    s = rb->soff.alloc(ctx, (S + 1) * sizeof(int64_t));
    if (s == FR_OK) s = make_bound_map(ctx, rb->soff.as<int64_t>(), slot_bound, 256, st, rb->stmap, rb->stm);
    if (s == FR_OK) s = rb->bufa.alloc(ctx, std::max<size_t>(rb->n2max, 1) * VP * sizeof(float));
    if (s == FR_OK) s = rb->bufb.alloc(ctx, std::max<size_t>(rb->n2max, 1) * VP * sizeof(float));
    if (s != FR_OK) return fail(s);
    rb->blur = true;
    *out = rb;
    return FR_OK;
}

fr_status resident_build_joint(ResidentBuild *rb, const float *mats, const float *kset, hipStream_t st)
{
    const int32_t S = rb->S;
    const int64_t *od = rb->joff.as<int64_t>();
    float *base = rb->jpts.as<float>();
    const size_t n = rb->jn;
    const bool nm = rb->jnormals;
    JointArgs a{rb->jtm, od, od + S + 1, rb->obs_pts, rb->model_pts, mats, base, base + n, base + 2 * n,
                nm ? base + 3 * n : nullptr, nm ? base + 4 * n : nullptr, nm ? base + 5 * n : nullptr};
    if (rb->jtm.n_tiles > 0) {
        k_joint_points<<<rb->jtm.n_tiles, 256, 0, st>>>(a);
        FR_HIP(hipGetLastError());
    }
    return resident_build(rb, kset, st);
}

fr_status blur_lattice(fr_lattice *lat, hipStream_t st)
{
    if (lat->d == 3 && lat->V == 4) return blur_impl<3, 4>(lat, st);
    if (lat->d == 3 && lat->V == 7) return blur_impl<3, 7>(lat, st);
    if (lat->d == 6 && lat->V == 4) return blur_impl<6, 4>(lat, st);
    if (lat->d == 6 && lat->V == 7) return blur_impl<6, 7>(lat, st);
    set_error("fr_lattice_blur: values must be FR_VAL_PT2PT or FR_VAL_PT2PL");
    return FR_EINVAL;
}

}  // namespace fr
