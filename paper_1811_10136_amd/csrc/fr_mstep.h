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
    if (!(m0 > 0.0f)) return;
    const float w = m0 / (m0 + c);
    const float inv = 1.0f / m0;
    const float tx = m1x * inv, ty = m1y * inv, tz = m1z * inv;
    const float dx = x - tx, dy = y - ty, dz = z - tz;
    float r2;
    if constexpr (RES == FR_PT2PT) {
        const float J[3][6] = {{0.0f, z, -y, 1.0f, 0.0f, 0.0f},
                               {-z, 0.0f, x, 0.0f, 1.0f, 0.0f},
                               {y, -x, 0.0f, 0.0f, 0.0f, 1.0f}};
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
        const float rr = fmaf(nx, dx, fmaf(ny, dy, nz * dz));
        const float J[1][6] = {{y * nz - z * ny, z * nx - x * nz, x * ny - y * nx, nx, ny, nz}};
        const float r[1] = {rr};
        accumulate_rows<1>(acc, J, r, w);
        r2 = rr * rr;
    }
    acc[27] += w;
    acc[28] = fmaf(w, r2, acc[28]);
    acc[29] += 1.0f;
    acc[30] += m0;
    if constexpr (M2) {
        const float dd = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
        acc[31] = fmaf(w, fmaf(m2, inv, dd), acc[31]);
    }
}

// Sum acc over the 256 threads of the block (wavefront butterflies, then the 4
// waves in order through LDS) and write the block's partial row.
__device__ __forceinline__ void block_partials(const float (&acc)[kRedVals], float (&part)[4][kRedStride],
                                               float *row)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int j = 0; j < kRedVals; ++j) {
        float v = acc[j];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) part[wave][j] = v;
    }
    __syncthreads();
    if (threadIdx.x < kRedVals) {
        float v = 0.0f;
#pragma unroll
        for (int w = 0; w < 4; ++w) v += part[w][threadIdx.x];
        row[threadIdx.x] = v;
    }
}

}  // namespace fr
