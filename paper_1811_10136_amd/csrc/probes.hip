// Roofline probes: the two hardware rates that bound the lattice kernels
// besides HBM bandwidth.
//
// * Scattered binary32 atomics with no contention: the ceiling of the atomic
//   splat, whose vertex sums are hardware atomics to vertices spread over the
//   value array.
// * Line accesses of 16-byte lane loads: a load instruction costs the vector
//   memory path about one cycle per distinct cache line its lanes touch, so
//   hash lookups -- one lane per key, keys on distinct lines -- run at the
//   rate of line accesses, not of bytes.  The probe loads 16 bytes per lane
//   with `lanes_per_line` lanes of a wave on the same 128-byte line.
#include <algorithm>

#include "fr_internal.h"

namespace fr {

__device__ __forceinline__ uint32_t probe_mix(uint32_t h)
{
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return h;
}

// Thread i adds to word i (packed: the 64 lanes of a wave cover two lines)
// or to word (i * odd) mod n_words (scattered: a bijection of [0, n_words)
// for a power-of-two n_words, neighbouring threads on different lines); no
// two threads share an address either way.
__global__ void __launch_bounds__(256) k_probe_atomics(float *table, uint32_t mask, uint64_t n, int scattered)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t w = scattered ? (uint32_t)(i * 0x9E3779B1ull) & mask : (uint32_t)i & mask;
    unsafeAtomicAdd(&table[w], 1.0f);
}

typedef uint32_t probe_u32x4 __attribute__((ext_vector_type(4)));

template <int G>
__global__ void __launch_bounds__(256) k_probe_lines(const probe_u32x4 *__restrict__ buf, uint32_t n_lines,
                                                    uint32_t *out, uint32_t seed)
{
    constexpr int K = 8;   // independent loads in flight per lane
    const uint32_t tid = blockIdx.x * 256u + threadIdx.x;
    const uint32_t grp = tid / G;
    const uint32_t chunk = (threadIdx.x % G) * (8 / G);
    probe_u32x4 v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const uint32_t line = probe_mix(grp * 131u + (uint32_t)k * 7919u + seed) % n_lines;
        v[k] = buf[(size_t)line * 8 + chunk];
    }
    uint32_t acc = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) acc += v[k].x ^ v[k].y ^ v[k].z ^ v[k].w;
    out[tid] = acc;
}

}  // namespace fr

using namespace fr;

namespace {
// Mean time of `reps` launches after one warm-up, with HIP events on `st`.
template <class Launch>
fr_status time_launches(hipStream_t st, int reps, Launch &&launch, double *sec)
{
    hipEvent_t e0, e1;
    FR_HIP(hipEventCreate(&e0));
    FR_HIP(hipEventCreate(&e1));
    launch(0);
    (void)hipEventRecord(e0, st);
    for (int r = 0; r < reps; ++r) launch(r + 1);
    (void)hipEventRecord(e1, st);
    const hipError_t err = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (err == hipSuccess) (void)hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    FR_HIP(err);
    FR_HIP(hipGetLastError());
    *sec = (double)ms * 1e-3 / reps;
    return FR_OK;
}
}  // namespace

fr_status fr_probe_atomics(fr_ctx *ctx, int64_t n_atomics, size_t table_bytes, int32_t scattered, double *per_s,
                           void *stream)
{
    clear_error();
    if (!ctx_ok(ctx) || per_s == nullptr || n_atomics <= 0 || table_bytes < 1024 ||
        (table_bytes & (table_bytes - 1)) != 0 || table_bytes > ((size_t)1 << 34) ||
        (uint64_t)n_atomics > table_bytes / sizeof(float)) {
        set_error("fr_probe_atomics: a power-of-two table of 1 KiB..16 GiB with a word for each of the n_atomics");
        return FR_EINVAL;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    StreamScope scope(st);
    DevBuf table;
    FR_TRY(table.alloc(ctx, table_bytes));
    FR_HIP(hipMemsetAsync(table.p, 0, table_bytes, st));
    const uint32_t mask = (uint32_t)(table_bytes / sizeof(float) - 1);
    const unsigned grid = (unsigned)((n_atomics + 255) / 256);
    double sec = 0.0;
    FR_TRY(time_launches(st, 5, [&](int) {
        k_probe_atomics<<<grid, 256, 0, st>>>(table.as<float>(), mask, (uint64_t)n_atomics, scattered);
    }, &sec));
    *per_s = (double)n_atomics / sec;
    return FR_OK;
}

fr_status fr_probe_lines(fr_ctx *ctx, int32_t lanes_per_line, size_t table_bytes, double *lines_per_s, void *stream)
{
    clear_error();
    if (!ctx_ok(ctx) || lines_per_s == nullptr ||
        (lanes_per_line != 1 && lanes_per_line != 2 && lanes_per_line != 4 && lanes_per_line != 8) ||
        table_bytes < 128 * 1024 || table_bytes > ((size_t)1 << 34)) {
        set_error("fr_probe_lines: lanes_per_line in {1, 2, 4, 8} and a table of 128 KiB..16 GiB");
        return FR_EINVAL;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    StreamScope scope(st);
    const uint32_t n_lines = (uint32_t)std::min<size_t>(table_bytes / 128, 0xFFFFFFFFull);
    constexpr unsigned kBlocks = 16384;   // 4 M lanes, 8 loads each
    DevBuf buf, out;
    FR_TRY(buf.alloc(ctx, (size_t)n_lines * 128));
    FR_TRY(out.alloc(ctx, (size_t)kBlocks * 256 * sizeof(uint32_t)));
    FR_HIP(hipMemsetAsync(buf.p, 1, (size_t)n_lines * 128, st));
    const probe_u32x4 *b = buf.as<probe_u32x4>();
    uint32_t *o = out.as<uint32_t>();
    double sec = 0.0;
    auto launch = [&](int r) {
        const uint32_t seed = 17u + 1000003u * (uint32_t)r;
        if (lanes_per_line == 1) k_probe_lines<1><<<kBlocks, 256, 0, st>>>(b, n_lines, o, seed);
        else if (lanes_per_line == 2) k_probe_lines<2><<<kBlocks, 256, 0, st>>>(b, n_lines, o, seed);
        else if (lanes_per_line == 4) k_probe_lines<4><<<kBlocks, 256, 0, st>>>(b, n_lines, o, seed);
        else k_probe_lines<8><<<kBlocks, 256, 0, st>>>(b, n_lines, o, seed);
    };
    FR_TRY(time_launches(st, 10, launch, &sec));
    const double lines = (double)kBlocks * 256.0 * 8.0 / lanes_per_line;
    *lines_per_s = lines / sec;
    return FR_OK;
}
