// Per-point M-step terms (Eq. 7 point-to-point, Eq. 10 point-to-plane, both
// linearised in the twist of the point's transform, Eq. 16) and the block
// reduction of their sums.  Shared by the stand-alone reduction and the fused
// slice + reduction, so both evaluate the same expressions.
#pragma once

#include "fr_device.h"

namespace fr {

constexpr int kRedVals = 32;      // 21 JtJ (upper, row-major) + 6 Jtr + 4 statistics + variance term
constexpr int kRedStride = 32;    // floats per partial row

// Numerical-rank rule of the Gauss-Newton solves (Eq. 17 needs an invertible
// A): A is summed from binary32 per-point terms over tiles of 1024 points, so
// an entry carries rounding of up to about 1024 * 2^-24 = 6.1e-5 of the
// diagonal scale; a Cholesky pivot (the part of A_jj the earlier directions do
// not explain) at or below 1e-4 of A_jj is indistinguishable from zero and
// its direction counts as unobservable.
constexpr double kPivotTol = 1e-4;

__host__ __device__ constexpr int ut_index(int a, int b) { return a * 6 - (a * (a - 1)) / 2 + (b - a); }

template <int NR>
__device__ __forceinline__ void accumulate_rows(float (&acc)[kRedVals], const float (&J)[NR][6], const float (&r)[NR],
                                                float w)
{
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        float wj[6];
#pragma unroll
        for (int a = 0; a < 6; ++a) wj[a] = w * J[q][a];
#pragma unroll
        for (int a = 0; a < 6; ++a) {
#pragma unroll
            for (int b = a; b < 6; ++b) acc[ut_index(a, b)] = fmaf(wj[a], J[q][b], acc[ut_index(a, b)]);
            acc[21 + a] = fmaf(wj[a], r[q], acc[21 + a]);
        }
    }
}

// One model point at (moved) position x with slice results m0, m1 = sum b y,
// ns = sum b n_y (and c2 = sum b |y - t|^2): weight w = m0 / (m0 + c), target
// t = m1 / m0, normal ns / m0;
//   pt2pt: r = x - t, J = [-[x]_x, I]
//   pt2pl: r = n . (x - t), J = [x cross n, n]
// adds w J^T J, w J^T r, w, w r^2, 1, m0 to acc, and with M2 the variance
// term w (|x - t|^2 + c2 / m0), the posterior-weighted squared distance of the
// point to the observations.  Points without support (m0 = 0) add nothing.
template <int RES, bool M2 = false>
__device__ __forceinline__ void mstep_point(float (&acc)[kRedVals], float x, float y, float z, float m0, float m1x,
                                            float m1y, float m1z, float nsx, float nsy, float nsz, float c,
                                            int normalize_n, float m2 = 0.0f)
{
    // No branch: a point without support (m0 = 0, or not a number) takes zeros in place of its
    // position, normal, residual and weight, so each of its terms is +0 whatever its inputs, and adding
    // +0 leaves a sum unchanged (a sum that starts at +0 is never -0).  The other points evaluate the
    // same expressions as with a branch.  Without one the accumulators are not set up again for a path
    // that skips the point.
    const bool ok = m0 > 0.0f;
    const float w = ok ? m0 / (m0 + c) : 0.0f;
    const float inv = ok ? 1.0f / m0 : 0.0f;
    const float tx = m1x * inv, ty = m1y * inv, tz = m1z * inv;
    const float dx = ok ? x - tx : 0.0f, dy = ok ? y - ty : 0.0f, dz = ok ? z - tz : 0.0f;
    const float px = ok ? x : 0.0f, py = ok ? y : 0.0f, pz = ok ? z : 0.0f;
    float r2;
    if constexpr (RES == FR_PT2PT) {
        const float J[3][6] = {{0.0f, pz, -py, 1.0f, 0.0f, 0.0f},
                               {-pz, 0.0f, px, 0.0f, 1.0f, 0.0f},
                               {py, -px, 0.0f, 0.0f, 0.0f, 1.0f}};
        const float r[3] = {dx, dy, dz};
        accumulate_rows<3>(acc, J, r, w);
        r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
    } else {
        float nx = nsx * inv, ny = nsy * inv, nz = nsz * inv;
        if (normalize_n) {
            const float nn = sqrtf(fmaf(nx, nx, fmaf(ny, ny, nz * nz)));
            const float in = nn > 0.0f ? 1.0f / nn : 0.0f;
            nx *= in;
            ny *= in;
            nz *= in;
        }
        nx = ok ? nx : 0.0f;
        ny = ok ? ny : 0.0f;
        nz = ok ? nz : 0.0f;
        const float rr = fmaf(nx, dx, fmaf(ny, dy, nz * dz));
        const float J[1][6] = {{py * nz - pz * ny, pz * nx - px * nz, px * ny - py * nx, nx, ny, nz}};
        const float r[1] = {rr};
        accumulate_rows<1>(acc, J, r, w);
        r2 = rr * rr;
    }
    acc[27] += w;
    acc[28] = fmaf(w, r2, acc[28]);
    acc[29] += ok ? 1.0f : 0.0f;
    acc[30] += ok ? m0 : 0.0f;
    if constexpr (M2) {
        const float dd = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
        const float v = fmaf(m2, inv, dd);
        acc[31] = fmaf(w, ok ? v : 0.0f, acc[31]);
    }
}

// One lane's value of another lane `OFF` apart (lane ^ OFF, OFF < 16): DPP
// lane moves where one gives exactly lane ^ OFF (quad permutations
// [1,0,3,2] and [2,3,0,1]; a rotation by 8 within a 16-lane row), a swizzle
// within 32 lanes otherwise.
template <int OFF>
__device__ __forceinline__ float xor_lane(float v)
{
    static_assert(OFF < 16, "wider exchanges use the lane swaps");
    if constexpr (OFF == 1 || OFF == 2 || OFF == 8) {
        constexpr int ctrl = OFF == 1 ? 0xB1 : OFF == 2 ? 0x4E : 0x128;
        return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), ctrl, 0xF, 0xF, false));
    } else {
        return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), (OFF << 10) | 0x1F));
    }
}

template <int OFF, int HALF>
__device__ __forceinline__ void halve(float (&v)[kRedVals], int lane)
{
    if constexpr (OFF == 32 || OFF == 16) {
        // gfx950's lane swaps exchange the upper OFF lanes of each 2 OFF-lane group of the first operand
        // with the lower OFF lanes of the second: the first result holds v[k] in the lower and v[k + HALF]
        // of the lower partner in the upper lanes, the second the partners' values, so their sum is the
        // exchange and addition below with no selects (the same sums: addition commutes)
#pragma unroll
        for (int k = 0; k < HALF; ++k) {
            const uint32_t a = __float_as_uint(v[k]), b = __float_as_uint(v[k + HALF]);
            const auto r = OFF == 32 ? __builtin_amdgcn_permlane32_swap(a, b, false, false)
                                     : __builtin_amdgcn_permlane16_swap(a, b, false, false);
            v[k] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
        }
    } else {
        const bool up = (lane & OFF) != 0;
#pragma unroll
        for (int k = 0; k < HALF; ++k) {
            const float send = up ? v[k] : v[k + HALF];
            const float keep = up ? v[k + HALF] : v[k];
            v[k] = keep + xor_lane<OFF>(send);
        }
    }
}

// Sum acc over the 256 threads of the block and write the block's partial row
// of the normal equations (acc is consumed).  Each wave sums its 32
// terms over its 64 lanes by halving exchanges (a lane keeps the half of its
// values its lane bit selects and adds its partner's sums of that half: five
// rounds leave value lane >> 1, summed over 32 lanes, and one more exchange
// adds the other lane of the pair -- 32 exchanges where one butterfly per
// value takes 192); the even lanes put the wave's sums in `wrow` (32 floats
// of LDS per wave, `stride` floats apart), and the first 32 threads add the
// four waves in order.
__device__ __forceinline__ void block_partials(float (&v)[kRedVals], float *wrow, int stride, float *row)
{
    static_assert(kRedVals == 32, "five halvings of 32 values");
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    halve<32, 16>(v, lane);
    halve<16, 8>(v, lane);
    halve<8, 4>(v, lane);
    halve<4, 2>(v, lane);
    halve<2, 1>(v, lane);
    v[0] += xor_lane<1>(v[0]);
    if ((lane & 1) == 0) wrow[wave * stride + (lane >> 1)] = v[0];
    __syncthreads();
    if (threadIdx.x < kRedVals) {
        float t = 0.0f;
#pragma unroll
        for (int w = 0; w < 4; ++w) t += wrow[w * stride + threadIdx.x];
        row[threadIdx.x] = t;
    }
}

}  // namespace fr
