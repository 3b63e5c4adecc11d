// Node-graph deformable kinematics on the device (Sec. 5.2, Eq. 21).
//
// Nodes {p_k, T_k}; model point i is skinned to 4 nodes with weights w_ki and
// moves by the normalised dual-quaternion blend of their transforms.  The
// point twist is the blend of the node twists (d zeta_i / d zeta_k = w_ki I6,
// exact where the nodes agree), so the normal equations of the node twists
// have data blocks A_kl = sum_i w_ki w_li J_i^T J_i and b_k = sum_i w_ki J_i^T r_i,
// plus an edge regulariser lambda |(T_j p_k - T_k p_k) / sigma|^2 linearised in
// the twists of both ends.  The system (6 K unknowns, block sparse, SPD) is
// solved by block-Jacobi preconditioned conjugate gradients in binary64 and
// the nodes are updated by T_k <- Exp(dzeta_k) T_k.
//
// Kernels:
//   k_ng_dualquat    per node: T_k (binary64) -> unit dual quaternion
//   k_ng_warp        per point: binary64 blend -> binary32 x (and n)
//   k_ng_terms       per point: w J^T J (21) and w J^T r (6), binary32
//   k_ng_blocks      per block: ordered binary64 sums over its point list
//   k_ng_edges       per edge: regulariser blocks and right-hand sides
//   k_ng_assemble    per block / node: data + regulariser in fixed order
//   k_ng_pcg_coop    block-Jacobi PCG to a relative residual over the
//                    workgroups of one cooperative launch (k_ng_pcg: the same
//                    in one workgroup, where cooperative launch is unavailable)
//   k_ng_update      per node: Exp(dzeta_k) T_k and the binary32 copy
// All sums run in a fixed order, so results are bitwise reproducible.
#include <algorithm>
#include <cmath>
#include <cstring>

#include <hip/hip_cooperative_groups.h>

#include "fr_internal.h"

namespace fr {

constexpr int kNgThreads = 256;
constexpr int kPcgThreads = 1024;
constexpr int kCoopThreads = 256;      // threads per workgroup of the grid-wide PCG
constexpr int kCoopMaxBlocks = 32;

// --- dual quaternions (w, x, y, z) --------------------------------------------
__device__ inline void qmul4(const double *a, const double *b, double *o)
{
    o[0] = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
    o[1] = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
    o[2] = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
    o[3] = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
}

// Unit quaternion of a rotation matrix (largest-pivot method) and the dual part t q / 2.
__global__ void k_ng_dualquat(int32_t K, const double *T, double *dq)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    const double *M = T + 12 * k;   // row-major [R | t]
    const double r00 = M[0], r01 = M[1], r02 = M[2], r10 = M[4], r11 = M[5], r12 = M[6], r20 = M[8], r21 = M[9],
                 r22 = M[10];
    double q[4];
    const double tr = r00 + r11 + r22;
    if (tr > 0.0) {
        const double s = sqrt(tr + 1.0) * 2.0;
        q[0] = 0.25 * s;
        q[1] = (r21 - r12) / s;
        q[2] = (r02 - r20) / s;
        q[3] = (r10 - r01) / s;
    } else if (r00 > r11 && r00 > r22) {
        const double s = sqrt(1.0 + r00 - r11 - r22) * 2.0;
        q[0] = (r21 - r12) / s;
        q[1] = 0.25 * s;
        q[2] = (r01 + r10) / s;
        q[3] = (r02 + r20) / s;
    } else if (r11 > r22) {
        const double s = sqrt(1.0 + r11 - r00 - r22) * 2.0;
        q[0] = (r02 - r20) / s;
        q[1] = (r01 + r10) / s;
        q[2] = 0.25 * s;
        q[3] = (r12 + r21) / s;
    } else {
        const double s = sqrt(1.0 + r22 - r00 - r11) * 2.0;
        q[0] = (r10 - r01) / s;
        q[1] = (r02 + r20) / s;
        q[2] = (r12 + r21) / s;
        q[3] = 0.25 * s;
    }
    const double n = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    for (int i = 0; i < 4; ++i) q[i] /= n;
    const double tq[4] = {0.0, M[3], M[7], M[11]};
    double d[4];
    qmul4(tq, q, d);
    for (int i = 0; i < 4; ++i) {
        dq[8 * k + i] = q[i];
        dq[8 * k + 4 + i] = 0.5 * d[i];
    }
}

// Blend the 4 skinning nodes of each point (signs aligned with the first node),
// normalise, and move the reference point (and normal) in binary64.
__global__ void __launch_bounds__(kNgThreads) k_ng_warp(int64_t M, const float *xr, const float *yr, const float *zr,
                                                        const float *nxr, const float *nyr, const float *nzr,
                                                        const int4 *skin_idx, const float4 *skin_w, const double *dq,
                                                        float *xo, float *yo, float *zo, float *nxo, float *nyo,
                                                        float *nzo)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    const int4 id = skin_idx[i];
    const float4 wf = skin_w[i];
    const int ids[4] = {id.x, id.y, id.z, id.w};
    const double ws[4] = {wf.x, wf.y, wf.z, wf.w};
    const double *ref = dq + 8 * ids[0];
    double br[4] = {0, 0, 0, 0}, bd[4] = {0, 0, 0, 0};
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const double *q = dq + 8 * ids[a];
        const double dot = q[0] * ref[0] + q[1] * ref[1] + q[2] * ref[2] + q[3] * ref[3];
        const double w = dot >= 0.0 ? ws[a] : -ws[a];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            br[c] += w * q[c];
            bd[c] += w * q[4 + c];
        }
    }
    const double nrm = sqrt(br[0] * br[0] + br[1] * br[1] + br[2] * br[2] + br[3] * br[3]);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        br[c] /= nrm;
        bd[c] /= nrm;
    }
    const double w = br[0], x = br[1], y = br[2], z = br[3];
    const double R[3][3] = {{1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)},
                            {2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)},
                            {2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)}};
    const double conj[4] = {br[0], -br[1], -br[2], -br[3]};
    double tq[4];
    qmul4(bd, conj, tq);
    const double t[3] = {2.0 * tq[1], 2.0 * tq[2], 2.0 * tq[3]};
    const double p[3] = {xr[i], yr[i], zr[i]};
    xo[i] = (float)(R[0][0] * p[0] + R[0][1] * p[1] + R[0][2] * p[2] + t[0]);
    yo[i] = (float)(R[1][0] * p[0] + R[1][1] * p[1] + R[1][2] * p[2] + t[1]);
    zo[i] = (float)(R[2][0] * p[0] + R[2][1] * p[1] + R[2][2] * p[2] + t[2]);
    if (nxo != nullptr) {
        const double n[3] = {nxr[i], nyr[i], nzr[i]};
        nxo[i] = (float)(R[0][0] * n[0] + R[0][1] * n[1] + R[0][2] * n[2]);
        nyo[i] = (float)(R[1][0] * n[0] + R[1][1] * n[1] + R[1][2] * n[2]);
        nzo[i] = (float)(R[2][0] * n[0] + R[2][1] * n[1] + R[2][2] * n[2]);
    }
}

// Per-point w J^T J (21, upper triangle row-major) and w J^T r (6), unscaled by sigma.
template <int RES>
__global__ void __launch_bounds__(kNgThreads) k_ng_terms(int64_t M, const float *x, const float *y, const float *z,
                                                         const float *m0, const float *m1, const float *ns, float c,
                                                         float *terms)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    float acc[27];
#pragma unroll
    for (int j = 0; j < 27; ++j) acc[j] = 0.0f;
    const float a0 = m0[i];
    if (a0 > 0.0f) {
        const float px = x[i], py = y[i], pz = z[i];
        const float w = a0 / (a0 + c), inv = 1.0f / a0;
        const float dx = px - m1[i] * inv, dy = py - m1[M + i] * inv, dz = pz - m1[2 * M + i] * inv;
        auto add_row = [&](const float (&J)[6], float r) {
            int idx = 0;
#pragma unroll
            for (int a = 0; a < 6; ++a) {
                const float wj = w * J[a];
#pragma unroll
                for (int b = a; b < 6; ++b) {
                    acc[idx] = fmaf(wj, J[b], acc[idx]);
                    ++idx;
                }
                acc[21 + a] = fmaf(wj, r, acc[21 + a]);
            }
        };
        if constexpr (RES == FR_PT2PT) {
            const float J0[6] = {0.0f, pz, -py, 1.0f, 0.0f, 0.0f};
            const float J1[6] = {-pz, 0.0f, px, 0.0f, 1.0f, 0.0f};
            const float J2[6] = {py, -px, 0.0f, 0.0f, 0.0f, 1.0f};
            add_row(J0, dx);
            add_row(J1, dy);
            add_row(J2, dz);
        } else {
            const float nx = ns[i] * inv, ny = ns[M + i] * inv, nz = ns[2 * M + i] * inv;
            const float rr = fmaf(nx, dx, fmaf(ny, dy, nz * dz));
            const float J[6] = {py * nz - pz * ny, pz * nx - px * nz, px * ny - py * nx, nx, ny, nz};
            add_row(J, rr);
        }
    }
#pragma unroll
    for (int j = 0; j < 27; ++j) terms[27 * i + j] = acc[j];
}

// One wave per data block: sum weight * J^T J over the block's (point, weight)
// list (CSR, point order) in binary64; lanes take every 64th entry and the
// wave reduces in a fixed butterfly order.  Node right-hand sides use the same
// kernel with the J^T r part (mode 1).
template <int MODE>
__global__ void __launch_bounds__(kNgThreads) k_ng_blocks(int32_t n_rows, const int32_t *row_off, const int32_t *pts,
                                                          const float *wts, const float *terms, double *out)
{
    constexpr int nv = MODE == 0 ? 21 : 6;
    constexpr int base = MODE == 0 ? 0 : 21;
    const int lane = threadIdx.x & 63;
    const int row = (int)(((size_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    if (row >= n_rows) return;
    double acc[nv];
#pragma unroll
    for (int j = 0; j < nv; ++j) acc[j] = 0.0;
    for (int e = row_off[row] + lane; e < row_off[row + 1]; e += 64) {
        const double w = wts[e];
        const float *t = terms + 27 * (size_t)pts[e] + base;
#pragma unroll
        for (int j = 0; j < nv; ++j) acc[j] += w * (double)t[j];
    }
#pragma unroll
    for (int j = 0; j < nv; ++j) {
        double v = acc[j];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) out[(size_t)row * nv + j] = v;
    }
}

// Regulariser of directed edge (j, k): e = (T_j p_k - T_k p_k) / sigma,
// J_j = [-[x_j]_x, I] / sigma, J_k = -[-[x_k]_x, I] / sigma; outputs (per edge)
// lambda J_j^T J_j, lambda J_k^T J_k, lambda J_j^T J_k (full 6x6 each, row-major)
// and lambda J_j^T e, lambda J_k^T e.
__global__ void k_ng_edges(int32_t E, const int32_t *edges, const double *nodes, const double *T, double inv_sigma,
                           double lambda, double *out)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= E) return;
    const int j = edges[2 * q], k = edges[2 * q + 1];
    const double *p = nodes + 3 * k;
    double xj[3], xk[3];
    for (int r = 0; r < 3; ++r) {
        xj[r] = T[12 * j + 4 * r] * p[0] + T[12 * j + 4 * r + 1] * p[1] + T[12 * j + 4 * r + 2] * p[2] + T[12 * j + 4 * r + 3];
        xk[r] = T[12 * k + 4 * r] * p[0] + T[12 * k + 4 * r + 1] * p[1] + T[12 * k + 4 * r + 2] * p[2] + T[12 * k + 4 * r + 3];
    }
    double Jj[3][6], Jk[3][6], e[3];
    for (int r = 0; r < 3; ++r) e[r] = (xj[r] - xk[r]) * inv_sigma;
    // -[x]_x rows: (0, z, -y), (-z, 0, x), (y, -x, 0)
    const double sj[3][3] = {{0.0, xj[2], -xj[1]}, {-xj[2], 0.0, xj[0]}, {xj[1], -xj[0], 0.0}};
    const double sk[3][3] = {{0.0, xk[2], -xk[1]}, {-xk[2], 0.0, xk[0]}, {xk[1], -xk[0], 0.0}};
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            Jj[r][c] = sj[r][c] * inv_sigma;
            Jj[r][3 + c] = (r == c ? 1.0 : 0.0) * inv_sigma;
            Jk[r][c] = -sk[r][c] * inv_sigma;
            Jk[r][3 + c] = -(r == c ? 1.0 : 0.0) * inv_sigma;
        }
    double *o = out + (size_t)120 * q;
    for (int a = 0; a < 6; ++a)
        for (int b = 0; b < 6; ++b) {
            double jj = 0.0, kk = 0.0, jk = 0.0;
            for (int r = 0; r < 3; ++r) {
                jj += Jj[r][a] * Jj[r][b];
                kk += Jk[r][a] * Jk[r][b];
                jk += Jj[r][a] * Jk[r][b];
            }
            o[6 * a + b] = lambda * jj;
            o[36 + 6 * a + b] = lambda * kk;
            o[72 + 6 * a + b] = lambda * jk;
        }
    for (int a = 0; a < 6; ++a) {
        double bj = 0.0, bk = 0.0;
        for (int r = 0; r < 3; ++r) {
            bj += Jj[r][a] * e[r];
            bk += Jk[r][a] * e[r];
        }
        o[108 + a] = lambda * bj;
        o[114 + a] = lambda * bk;
    }
}

// Assemble block b (row-major 6x6, rows of node kb[b], columns of node lb[b],
// kb <= lb) = data (21, symmetric) + regulariser terms listed in reg_off/reg_ref
// (ref = 3 * edge + part; part 0: J_j^T J_j, 1: J_k^T J_k, 2: J_j^T J_k, 3: its
// transpose) in list order.  Threads 0..K-1 of the same launch also assemble
// the node right-hand sides.
__global__ void k_ng_assemble(int32_t n_blocks, const double *data21, const int32_t *reg_off, const int32_t *reg_ref,
                              const double *edge_terms, double inv_s2, double *A, int32_t K, const double *b_data,
                              const int32_t *rhs_off, const int32_t *rhs_ref, double *rhs)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n_blocks) {
        double B[36];
        int idx = 0;
        for (int a = 0; a < 6; ++a)
            for (int b = a; b < 6; ++b) {
                const double v = data21[(size_t)21 * q + idx++] * inv_s2;
                B[6 * a + b] = v;
                B[6 * b + a] = v;
            }
        for (int e = reg_off[q]; e < reg_off[q + 1]; ++e) {
            const int ref = reg_ref[e];
            const int edge = ref >> 2, part = ref & 3;
            const double *t = edge_terms + (size_t)120 * edge + 36 * (part == 3 ? 2 : part);
            for (int a = 0; a < 6; ++a)
                for (int b = 0; b < 6; ++b) B[6 * a + b] += part == 3 ? t[6 * b + a] : t[6 * a + b];
        }
        for (int j = 0; j < 36; ++j) A[(size_t)36 * q + j] = B[j];
    }
    if (q < K) {
        double r[6];
        for (int a = 0; a < 6; ++a) r[a] = b_data[6 * q + a] * inv_s2;
        for (int e = rhs_off[q]; e < rhs_off[q + 1]; ++e) {
            const int ref = rhs_ref[e];
            const double *t = edge_terms + (size_t)120 * (ref >> 1) + 108 + 6 * (ref & 1);
            for (int a = 0; a < 6; ++a) r[a] += t[a];
        }
        for (int a = 0; a < 6; ++a) rhs[6 * q + a] = r[a];
    }
}

// Deterministic block-wide sum of one double per thread.
__device__ double block_sum(double v, double *red)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < kPcgThreads / 64; ++w) s += red[w];
    __syncthreads();
    return s;
}

// y = A p for the block-sparse symmetric A: row node k sums its row entries
// (block id, transposed) in list order.  One thread per unknown.
__device__ void spmv(int32_t n, const int32_t *row_off, const int32_t *row_blk, const int32_t *row_col,
                     const double *A, const double *p, double *y)
{
    for (int u = threadIdx.x; u < n; u += kPcgThreads) {
        const int k = u / 6, a = u % 6;
        double acc = 0.0;
        for (int e = row_off[k]; e < row_off[k + 1]; ++e) {
            const int ref = row_blk[e];
            const int blk = ref >> 1;
            const bool tr = ref & 1;
            const double *B = A + (size_t)36 * blk;
            const double *pl = p + 6 * row_col[e];
            if (!tr)
                for (int b = 0; b < 6; ++b) acc += B[6 * a + b] * pl[b];
            else
                for (int b = 0; b < 6; ++b) acc += B[6 * b + a] * pl[b];
        }
        y[u] = acc;
    }
}

// Block-Jacobi PCG for A x = -rhs in one workgroup.  minv holds the inverse of
// each 6x6 diagonal block (row-major).  Stops when |r| <= tol |rhs| or after
// max_it iterations; writes the iteration count and final relative residual.
__global__ void __launch_bounds__(kPcgThreads) k_ng_pcg(int32_t K, const int32_t *row_off, const int32_t *row_blk,
                                                        const int32_t *row_col, const double *A, const double *minv,
                                                        const double *rhs, double *x, double *r, double *z, double *p,
                                                        double *q, double tol, int32_t max_it, double *info)
{
    __shared__ double red[kPcgThreads / 64];
    const int n = 6 * K;
    double rr_loc = 0.0;
    for (int u = threadIdx.x; u < n; u += kPcgThreads) {
        x[u] = 0.0;
        r[u] = -rhs[u];
        rr_loc += rhs[u] * rhs[u];
    }
    const double bnorm = sqrt(block_sum(rr_loc, red));
    auto precond = [&]() {
        for (int u = threadIdx.x; u < n; u += kPcgThreads) {
            const int k = u / 6, a = u % 6;
            const double *Mi = minv + 36 * k;
            double v = 0.0;
            for (int b = 0; b < 6; ++b) v += Mi[6 * a + b] * r[6 * k + b];
            z[u] = v;
        }
    };
    __syncthreads();
    precond();
    __syncthreads();
    double loc = 0.0;
    for (int u = threadIdx.x; u < n; u += kPcgThreads) {
        p[u] = z[u];
        loc += r[u] * z[u];
    }
    double rz = block_sum(loc, red);
    int it = 0;
    double rel = bnorm > 0.0 ? 1.0 : 0.0;
    while (it < max_it && bnorm > 0.0) {
        __syncthreads();
        spmv(n, row_off, row_blk, row_col, A, p, q);
        __syncthreads();
        loc = 0.0;
        for (int u = threadIdx.x; u < n; u += kPcgThreads) loc += p[u] * q[u];
        const double pq = block_sum(loc, red);
        if (!(pq > 0.0)) break;
        const double alpha = rz / pq;
        loc = 0.0;
        for (int u = threadIdx.x; u < n; u += kPcgThreads) {
            x[u] += alpha * p[u];
            r[u] -= alpha * q[u];
            loc += r[u] * r[u];
        }
        const double rn = sqrt(block_sum(loc, red));
        ++it;
        rel = rn / bnorm;
        if (rel <= tol) break;
        precond();
        __syncthreads();
        loc = 0.0;
        for (int u = threadIdx.x; u < n; u += kPcgThreads) loc += r[u] * z[u];
        const double rz_new = block_sum(loc, red);
        const double beta = rz_new / rz;
        rz = rz_new;
        for (int u = threadIdx.x; u < n; u += kPcgThreads) p[u] = z[u] + beta * p[u];
    }
    if (threadIdx.x == 0) {
        info[0] = it;
        info[1] = rel;
    }
}

// The same block-Jacobi PCG spread over G workgroups of one cooperative
// launch: workgroup g owns a contiguous range of nodes (their rows of A, x, r,
// u, w, p, s).  The iteration is the single-reduction form of Chronopoulos and
// Gear (1989): with u = M^-1 r and w = A u, the three sums (r, r), (r, u) and
// (w, u) of an iteration are taken together, s = A p is carried by the
// recurrence s <- w + beta s, and the step length follows from
// alpha = gamma / (delta - beta gamma / alpha_old).  In exact arithmetic the
// iterates are those of the textbook PCG.  Per iteration two grid-wide
// barriers: one before the product (u of every workgroup complete), one for
// the sums.  The sums are taken per workgroup in a fixed order, exchanged
// through `part` and added in workgroup order, so every workgroup takes the
// same decisions and the result is reproducible.
struct PcgArgs {
    int32_t K;
    const int32_t *row_off, *row_blk, *row_col;
    const double *A, *minv, *rhs;
    double *x, *r, *u, *w, *p, *s;
    double *part;           // 2 x 3 x gridDim.x partial sums
    double tol;
    int32_t max_it;
    double *info;
};

// Block sums of three values at once (one pass through LDS).
__device__ void coop_block_sum3(double v[3], double *red)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) v[i] += __shfl_xor(v[i], off, 64);
        if (lane == 0) red[3 * wave + i] = v[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        double t = 0.0;
        for (int w = 0; w < kCoopThreads / 64; ++w) t += red[3 * w + i];
        v[i] = t;
    }
    __syncthreads();
}

__global__ void __launch_bounds__(kCoopThreads) k_ng_pcg_coop(PcgArgs a)
{
    namespace cg = cooperative_groups;
    cg::grid_group grid = cg::this_grid();
    __shared__ double red[3 * (kCoopThreads / 64)];
    __shared__ double lanes[kCoopThreads];
    const int G = gridDim.x, g = blockIdx.x, tid = threadIdx.x;
    const int kb = (a.K + G - 1) / G;
    const int k0 = min(a.K, g * kb), k1 = min(a.K, k0 + kb);
    const int u0 = 6 * k0, u1 = 6 * k1, R = u1 - u0;
    const int L = R > 0 ? max(1, min(8, kCoopThreads / R)) : 1;   // lanes per SpMV row
    // grid-wide sums of three values per workgroup through the partial slots
    // set*3 .. set*3+2 (sets alternate between successive sums)
    // The G partials are read one per lane (one round trip instead of G
    // dependent ones) and added by a fixed xor-shuffle tree within the first
    // wave, so every workgroup adds the same values in the same order.
    auto grid_sum3 = [&](double v[3], int set) {
        coop_block_sum3(v, red);
        if (tid == 0)
            for (int i = 0; i < 3; ++i) a.part[(3 * set + i) * G + g] = v[i];
        __threadfence();
        grid.sync();
        if (tid < 64) {
            double t[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) t[i] = tid < G ? a.part[(3 * set + i) * G + tid] : 0.0;
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1)
#pragma unroll
                for (int i = 0; i < 3; ++i) t[i] += __shfl_xor(t[i], off, 64);
            if (tid == 0)
                for (int i = 0; i < 3; ++i) red[i] = t[i];
        }
        __syncthreads();
        for (int i = 0; i < 3; ++i) v[i] = red[i];
        __syncthreads();
    };
    // u = M^-1 r over the owned nodes; returns the owned parts of (r, u)
    auto precond = [&]() {
        double ru = 0.0;
        for (int q = u0 + tid; q < u1; q += kCoopThreads) {
            const int k = q / 6, c = q % 6;
            const double *Mi = a.minv + 36 * k;
            double v = 0.0;
            for (int b = 0; b < 6; ++b) v += Mi[6 * c + b] * a.r[6 * k + b];
            a.u[q] = v;
            ru += a.r[q] * v;
        }
        return ru;
    };
    // w = A u for the owned rows, L lanes per row summing every L-th entry;
    // returns the owned part of (w, u)
    auto spmv = [&]() {
        double wu = 0.0;
        for (int r0 = 0; r0 < R; r0 += kCoopThreads / L) {
            const int row = r0 + tid / L, lane = tid % L;
            double acc = 0.0;
            const bool on = tid / L < kCoopThreads / L && row < R;
            if (on) {
                const int q = u0 + row, k = q / 6, c = q % 6;
                const int ee = a.row_off[k + 1];
                // four entries at a time: their indices, then all their block
                // and vector loads, then the products in entry order
                for (int e = a.row_off[k] + lane; e < ee; e += 4 * L) {
                    int ref[4], col[4];
                    bool ok[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        ok[j] = e + j * L < ee;
                        ref[j] = ok[j] ? a.row_blk[e + j * L] : 0;
                        col[j] = ok[j] ? a.row_col[e + j * L] : 0;
                    }
                    double bv[4][6], uv[4][6];
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const double *B = a.A + (size_t)36 * (ref[j] >> 1);
                        const double *ul = a.u + 6 * col[j];
#pragma unroll
                        for (int b = 0; b < 6; ++b) {
                            bv[j][b] = ok[j] ? ((ref[j] & 1) ? B[6 * b + c] : B[6 * c + b]) : 0.0;
                            uv[j][b] = ok[j] ? ul[b] : 0.0;
                        }
                    }
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        if (ok[j])
#pragma unroll
                            for (int b = 0; b < 6; ++b) acc += bv[j][b] * uv[j][b];
                }
            }
            lanes[tid] = acc;
            __syncthreads();
            if (on && lane == 0) {
                double y = 0.0;
                for (int l = 0; l < L; ++l) y += lanes[tid + l];
                const int q = u0 + row;
                a.w[q] = y;
                wu += a.u[q] * y;
            }
            __syncthreads();
        }
        return wu;
    };
    double bb = 0.0;
    for (int q = u0 + tid; q < u1; q += kCoopThreads) {
        a.x[q] = 0.0;
        a.r[q] = -a.rhs[q];
        bb += a.rhs[q] * a.rhs[q];
    }
    __syncthreads();   // the preconditioner reads the r of a node's six rows, written by other threads
    const double ru0 = precond();
    grid.sync();       // u of every workgroup complete
    const double wu0 = spmv();
    double v[3] = {bb, ru0, wu0};
    grid_sum3(v, 0);
    const double bnorm = sqrt(v[0]);
    double gamma = v[1], delta = v[2];
    double alpha = delta > 0.0 ? gamma / delta : 0.0;
    for (int q = u0 + tid; q < u1; q += kCoopThreads) {
        a.p[q] = a.u[q];
        a.s[q] = a.w[q];
    }
    int it = 0;
    double rel = bnorm > 0.0 ? 1.0 : 0.0;
    bool go = bnorm > 0.0 && delta > 0.0;
    while (go && it < a.max_it) {
        double rr = 0.0;
        for (int q = u0 + tid; q < u1; q += kCoopThreads) {
            a.x[q] += alpha * a.p[q];
            a.r[q] -= alpha * a.s[q];
            rr += a.r[q] * a.r[q];
        }
        __syncthreads();
        const double ru = precond();
        grid.sync();   // u of every workgroup complete
        const double wu = spmv();
        v[0] = rr;
        v[1] = ru;
        v[2] = wu;
        grid_sum3(v, 1 - (it & 1));
        ++it;
        rel = sqrt(v[0]) / bnorm;
        if (rel <= a.tol) break;
        const double gamma_new = v[1];
        const double beta = gamma_new / gamma;
        const double denom = v[2] - beta * gamma_new / alpha;
        if (!(denom > 0.0)) break;
        alpha = gamma_new / denom;
        gamma = gamma_new;
        for (int q = u0 + tid; q < u1; q += kCoopThreads) {
            a.p[q] = a.u[q] + beta * a.p[q];
            a.s[q] = a.w[q] + beta * a.s[q];
        }
    }
    if (g == 0 && tid == 0) {
        a.info[0] = it;
        a.info[1] = rel;
    }
}

// Inverse of each diagonal 6x6 block by Gauss-Jordan with partial pivoting
// (blocks are SPD); flags a non-positive pivot.
__global__ void __launch_bounds__(64) k_ng_block_inverse(int32_t K, const double *A, const int32_t *diag_blk,
                                                         double *minv, int32_t *bad)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    // every index below is a compile-time constant once the loops are
    // unrolled (the row swap is a select per row), so M stays in registers
    double M[6][12];
    const double *B = A + (size_t)36 * diag_blk[k];
#pragma unroll
    for (int a = 0; a < 6; ++a)
#pragma unroll
        for (int b = 0; b < 12; ++b) M[a][b] = b < 6 ? B[6 * a + b] : (b - 6 == a ? 1.0 : 0.0);
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        int piv = c;
        double best = fabs(M[c][c]);
#pragma unroll
        for (int a = c + 1; a < 6; ++a)
            if (fabs(M[a][c]) > best) {
                best = fabs(M[a][c]);
                piv = a;
            }
        if (!(best > 0.0)) {
            atomicOr(bad, 1);
            for (int a = 0; a < 36; ++a) minv[36 * k + a] = (a % 7 == 0) ? 1.0 : 0.0;
            return;
        }
#pragma unroll
        for (int a = c + 1; a < 6; ++a) {
            const bool sw = (piv == a);
#pragma unroll
            for (int b = 0; b < 12; ++b) {
                const double t = M[c][b];
                M[c][b] = sw ? M[a][b] : t;
                M[a][b] = sw ? t : M[a][b];
            }
        }
        const double inv = 1.0 / M[c][c];
#pragma unroll
        for (int b = 0; b < 12; ++b) M[c][b] *= inv;
#pragma unroll
        for (int a = 0; a < 6; ++a) {
            if (a == c) continue;
            const double f = M[a][c];
#pragma unroll
            for (int b = 0; b < 12; ++b) M[a][b] -= f * M[c][b];
        }
    }
#pragma unroll
    for (int a = 0; a < 6; ++a)
#pragma unroll
        for (int b = 0; b < 6; ++b) minv[36 * k + 6 * a + b] = M[a][6 + b];
}

// Exp of the twist of node k composed on the left of its transform.
__device__ inline void twist_exp(const double *z, double (&E)[3][4])
{
    const double wx = z[0], wy = z[1], wz = z[2];
    const double th2 = wx * wx + wy * wy + wz * wz, th = sqrt(th2);
    double A, B, C;
    if (th < 1e-4) {
        A = 1.0 - th2 / 6.0;
        B = 0.5 - th2 / 24.0;
        C = 1.0 / 6.0 - th2 / 120.0;
    } else {
        A = sin(th) / th;
        B = (1.0 - cos(th)) / th2;
        C = (th - sin(th)) / (th2 * th);
    }
    const double Km[3][3] = {{0.0, -wz, wy}, {wz, 0.0, -wx}, {-wy, wx, 0.0}};
    for (int i = 0; i < 3; ++i) {
        double pv = 0.0;
        for (int j = 0; j < 3; ++j) {
            const double K2 = Km[i][0] * Km[0][j] + Km[i][1] * Km[1][j] + Km[i][2] * Km[2][j];
            const double I = (i == j) ? 1.0 : 0.0;
            E[i][j] = I + A * Km[i][j] + B * K2;
            pv += (I + B * Km[i][j] + C * K2) * z[3 + j];
        }
        E[i][3] = pv;
    }
}

// A singular diagonal block (bad set by the block inverse) leaves every node unchanged.
__global__ void k_ng_update(int32_t K, const double *dz, double *T, const int32_t *bad)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K || *bad != 0) return;
    double E[3][4];
    twist_exp(dz + 6 * k, E);
    double N[3][4];
    const double *M = T + 12 * k;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 4; ++j)
            N[i][j] = E[i][0] * M[j] + E[i][1] * M[4 + j] + E[i][2] * M[8 + j] + (j == 3 ? E[i][3] : 0.0);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 4; ++j) T[12 * k + 4 * i + j] = N[i][j];
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
fr_status ng_setup(fr_ctx *ctx, const fr_node_graph *g, int64_t M, hipStream_t st, NodeGraphDev &d)
{
    const int32_t K = g->n_nodes, E = g->n_edges;
    d.K = K;
    d.E = E;
    d.M = M;
    // blocks: unique (k <= l) pairs from co-skinned nodes and from edges, in key
    // order (key = k K + l); each data block lists its (point, w_k w_l) entries in
    // point order
    auto pair_key = [&](int64_t i, int a, int c, int64_t &key, float &wt) {
        int32_t k = g->skin_idx[4 * i + a], l = g->skin_idx[4 * i + c];
        if (k < 0 || k >= K || l < 0 || l >= K || (a != c && k == l)) return false;
        if (k > l) std::swap(k, l);
        key = (int64_t)k * K + l;
        wt = g->skin_w[4 * i + a] * g->skin_w[4 * i + c];
        return true;
    };
    std::vector<int64_t> ekeys;
    for (int32_t q = 0; q < E; ++q) {
        const int32_t j = g->edges[2 * q], k = g->edges[2 * q + 1];
        ekeys.push_back((int64_t)j * K + j);
        ekeys.push_back((int64_t)k * K + k);
        ekeys.push_back((int64_t)std::min(j, k) * K + std::max(j, k));
    }
    for (int32_t k = 0; k < K; ++k) ekeys.push_back((int64_t)k * K + k);   // every node has a diagonal block
    std::vector<int64_t> all;
    std::vector<int32_t> boff, bpts, diag(K);
    std::vector<float> bw;
    if ((int64_t)K * K <= ((int64_t)1 << 24)) {
        // dense K x K table: count per key, number the keys in order, scatter in point order
        std::vector<int32_t> cnt((size_t)K * K, 0);
        std::vector<uint8_t> used((size_t)K * K, 0);
        for (int64_t i = 0; i < M; ++i)
            for (int a = 0; a < 4; ++a)
                for (int c = a; c < 4; ++c) {
                    int64_t key;
                    float wt;
                    if (pair_key(i, a, c, key, wt)) {
                        ++cnt[(size_t)key];
                        used[(size_t)key] = 1;
                    }
                }
        for (int64_t key : ekeys) used[(size_t)key] = 1;
        std::vector<int32_t> fill((size_t)K * K, 0);
        int32_t total = 0;
        for (int64_t key = 0; key < (int64_t)K * K; ++key)
            if (used[(size_t)key]) {
                all.push_back(key);
                boff.push_back(total);
                fill[(size_t)key] = total;
                total += cnt[(size_t)key];
            }
        boff.push_back(total);
        bpts.resize(total);
        bw.resize(total);
        for (int64_t i = 0; i < M; ++i)
            for (int a = 0; a < 4; ++a)
                for (int c = a; c < 4; ++c) {
                    int64_t key;
                    float wt;
                    if (pair_key(i, a, c, key, wt)) {
                        const int32_t pos = fill[(size_t)key]++;
                        bpts[pos] = (int32_t)i;
                        bw[pos] = wt;
                    }
                }
    } else {
        // many nodes: a stable sort of the entries by key
        struct Ent {
            int64_t key;
            int32_t pt;
            float w;
        };
        std::vector<Ent> ent;
        ent.reserve((size_t)M * 10);
        for (int64_t i = 0; i < M; ++i)
            for (int a = 0; a < 4; ++a)
                for (int c = a; c < 4; ++c) {
                    int64_t key;
                    float wt;
                    if (pair_key(i, a, c, key, wt)) ent.push_back({key, (int32_t)i, wt});
                }
        std::stable_sort(ent.begin(), ent.end(), [](const Ent &x, const Ent &y) { return x.key < y.key; });
        for (const Ent &e : ent) all.push_back(e.key);
        all.insert(all.end(), ekeys.begin(), ekeys.end());
        std::sort(all.begin(), all.end());
        all.erase(std::unique(all.begin(), all.end()), all.end());
        size_t e = 0;
        for (int64_t key : all) {
            boff.push_back((int32_t)bpts.size());
            for (; e < ent.size() && ent[e].key == key; ++e) {
                bpts.push_back(ent[e].pt);
                bw.push_back(ent[e].w);
            }
        }
        boff.push_back((int32_t)bpts.size());
    }
    const int32_t NB = (int32_t)all.size();
    d.n_blocks = NB;
    d.block_keys = all;
    auto block_of = [&](int64_t key) { return (int32_t)(std::lower_bound(all.begin(), all.end(), key) - all.begin()); };
    for (int32_t k = 0; k < K; ++k) diag[k] = block_of((int64_t)k * K + k);
    // node right-hand side CSR: (point, w_ki) in point order
    std::vector<int32_t> roff(K + 1, 0), rpts;
    std::vector<float> rw;
    {
        // counting sort of (point, weight) by node, point order kept
        for (int64_t i = 0; i < M; ++i)
            for (int a = 0; a < 4; ++a) {
                const int32_t k = g->skin_idx[4 * i + a];
                if (k >= 0 && k < K) ++roff[k + 1];
            }
        for (int32_t k = 0; k < K; ++k) roff[k + 1] += roff[k];
        rpts.resize(roff[K]);
        rw.resize(roff[K]);
        std::vector<int32_t> fill(roff.begin(), roff.end() - 1);
        for (int64_t i = 0; i < M; ++i)
            for (int a = 0; a < 4; ++a) {
                const int32_t k = g->skin_idx[4 * i + a];
                if (k >= 0 && k < K) {
                    rpts[fill[k]] = (int32_t)i;
                    rw[fill[k]++] = g->skin_w[4 * i + a];
                }
            }
    }
    // regulariser references per block and per node (edge order)
    std::vector<std::vector<int32_t>> breg(NB), nreg(K);
    for (int32_t q = 0; q < E; ++q) {
        const int32_t j = g->edges[2 * q], k = g->edges[2 * q + 1];
        breg[diag[j]].push_back(4 * q + 0);
        breg[diag[k]].push_back(4 * q + 1);
        const int32_t ob = block_of((int64_t)std::min(j, k) * K + std::max(j, k));
        if (j != k) breg[ob].push_back(4 * q + (j < k ? 2 : 3));
        nreg[j].push_back(2 * q + 0);
        nreg[k].push_back(2 * q + 1);
    }
    std::vector<int32_t> rgoff(NB + 1, 0), rgref, nroff(K + 1, 0), nrref;
    for (int32_t b = 0; b < NB; ++b) {
        rgoff[b] = (int32_t)rgref.size();
        rgref.insert(rgref.end(), breg[b].begin(), breg[b].end());
    }
    rgoff[NB] = (int32_t)rgref.size();
    for (int32_t k = 0; k < K; ++k) {
        nroff[k] = (int32_t)nrref.size();
        nrref.insert(nrref.end(), nreg[k].begin(), nreg[k].end());
    }
    nroff[K] = (int32_t)nrref.size();
    // SpMV rows: row k lists (block, transposed) for blocks (k, l) and (l, k), in block order
    std::vector<std::vector<std::pair<int32_t, int32_t>>> rows(K);
    for (int32_t b = 0; b < NB; ++b) {
        const int32_t k = (int32_t)(all[b] / K), l = (int32_t)(all[b] % K);
        rows[k].push_back({2 * b + 0, l});
        if (k != l) rows[l].push_back({2 * b + 1, k});
    }
    std::vector<int32_t> sroff(K + 1, 0), srblk, srcol;
    for (int32_t k = 0; k < K; ++k) {
        sroff[k] = (int32_t)srblk.size();
        for (auto &e : rows[k]) {
            srblk.push_back(e.first);
            srcol.push_back(e.second);
        }
    }
    sroff[K] = (int32_t)srblk.size();

    // upload everything into one device buffer
    std::vector<char> host;
    auto put = [&](const void *src, size_t bytes) {
        size_t off = (host.size() + 15) & ~(size_t)15;
        host.resize(off + bytes);
        if (bytes) std::memcpy(host.data() + off, src, bytes);
        return off;
    };
    std::vector<double> nodes(g->nodes, g->nodes + 3 * (size_t)K);
    const size_t o_nodes = put(nodes.data(), nodes.size() * 8);
    const size_t o_edges = put(g->edges, (size_t)2 * E * 4);
    const size_t o_sidx = put(g->skin_idx, (size_t)4 * M * 4);
    const size_t o_sw = put(g->skin_w, (size_t)4 * M * 4);
    const size_t o_boff = put(boff.data(), boff.size() * 4);
    const size_t o_bpts = put(bpts.data(), bpts.size() * 4);
    const size_t o_bw = put(bw.data(), bw.size() * 4);
    const size_t o_roff = put(roff.data(), roff.size() * 4);
    const size_t o_rpts = put(rpts.data(), rpts.size() * 4);
    const size_t o_rw = put(rw.data(), rw.size() * 4);
    const size_t o_rgoff = put(rgoff.data(), rgoff.size() * 4);
    const size_t o_rgref = put(rgref.data(), rgref.size() * 4);
    const size_t o_nroff = put(nroff.data(), nroff.size() * 4);
    const size_t o_nrref = put(nrref.data(), nrref.size() * 4);
    const size_t o_sroff = put(sroff.data(), sroff.size() * 4);
    const size_t o_srblk = put(srblk.data(), srblk.size() * 4);
    const size_t o_srcol = put(srcol.data(), srcol.size() * 4);
    const size_t o_diag = put(diag.data(), diag.size() * 4);
    FR_TRY(d.meta.alloc(ctx, host.size()));
    FR_HIP(hipMemcpyAsync(d.meta.p, host.data(), host.size(), hipMemcpyHostToDevice, st));
    FR_HIP(hipStreamSynchronize(st));
    char *b = d.meta.as<char>();
    d.nodes = reinterpret_cast<const double *>(b + o_nodes);
    d.edges = reinterpret_cast<const int32_t *>(b + o_edges);
    d.skin_idx = reinterpret_cast<const int4 *>(b + o_sidx);
    d.skin_w = reinterpret_cast<const float4 *>(b + o_sw);
    d.blk_off = reinterpret_cast<const int32_t *>(b + o_boff);
    d.blk_pts = reinterpret_cast<const int32_t *>(b + o_bpts);
    d.blk_w = reinterpret_cast<const float *>(b + o_bw);
    d.rhs_off = reinterpret_cast<const int32_t *>(b + o_roff);
    d.rhs_pts = reinterpret_cast<const int32_t *>(b + o_rpts);
    d.rhs_w = reinterpret_cast<const float *>(b + o_rw);
    d.reg_off = reinterpret_cast<const int32_t *>(b + o_rgoff);
    d.reg_ref = reinterpret_cast<const int32_t *>(b + o_rgref);
    d.nreg_off = reinterpret_cast<const int32_t *>(b + o_nroff);
    d.nreg_ref = reinterpret_cast<const int32_t *>(b + o_nrref);
    d.row_off = reinterpret_cast<const int32_t *>(b + o_sroff);
    d.row_blk = reinterpret_cast<const int32_t *>(b + o_srblk);
    d.row_col = reinterpret_cast<const int32_t *>(b + o_srcol);
    d.diag_blk = reinterpret_cast<const int32_t *>(b + o_diag);
    // work arrays
    const size_t n = 6 * (size_t)K;
    FR_TRY(d.work.alloc(ctx, sizeof(double) * (12 * (size_t)K + 8 * (size_t)K + 21 * (size_t)NB + 6 * (size_t)K +
                                               120 * (size_t)std::max(E, 1) + 36 * (size_t)NB + 36 * (size_t)K +
                                               7 * n + 2 + 8 + 6 * (size_t)kCoopMaxBlocks) +
                                sizeof(float) * 27 * (size_t)std::max<int64_t>(M, 1) + sizeof(int32_t) * 4));
    double *w = d.work.as<double>();
    d.T = w;
    w += 12 * (size_t)K;
    d.dq = w;
    w += 8 * (size_t)K;
    d.data21 = w;
    w += 21 * (size_t)NB;
    d.bdata = w;
    w += 6 * (size_t)K;
    d.edge_terms = w;
    w += 120 * (size_t)std::max(E, 1);
    d.A = w;
    w += 36 * (size_t)NB;
    d.minv = w;
    w += 36 * (size_t)K;
    d.rhs = w;
    w += n;
    d.x = w;
    w += n;
    d.r = w;
    w += n;
    d.z = w;
    w += n;
    d.p = w;
    w += n;
    d.q = w;
    w += n;
    d.s = w;
    w += n;
    d.info = w;
    w += 8;
    d.part = w;
    w += 6 * (size_t)kCoopMaxBlocks;
    d.terms = reinterpret_cast<float *>(w);
    d.bad = reinterpret_cast<int32_t *>(d.terms + 27 * (size_t)std::max<int64_t>(M, 1));
    return FR_OK;
}

fr_status ng_warp(const NodeGraphDev &d, const fr_cloud *ref, float *const out[6], hipStream_t st)
{
    k_ng_dualquat<<<(d.K + 63) / 64, 64, 0, st>>>(d.K, d.T, d.dq);
    FR_HIP(hipGetLastError());
    if (d.M > 0) {
        k_ng_warp<<<(unsigned)((d.M + kNgThreads - 1) / kNgThreads), kNgThreads, 0, st>>>(
            d.M, ref->x, ref->y, ref->z, ref->nx, ref->ny, ref->nz, d.skin_idx, d.skin_w, d.dq, out[0], out[1], out[2],
            out[3], out[4], out[5]);
        FR_HIP(hipGetLastError());
    }
    return FR_OK;
}

fr_status ng_reduce(NodeGraphDev &d, const float *x, const float *y, const float *z, const float *m0, const float *m1,
                    const float *ns, int residual, double c, double sigma, double lambda, hipStream_t st)
{
    const unsigned gM = (unsigned)((std::max<int64_t>(d.M, 1) + kNgThreads - 1) / kNgThreads);
    if (d.M > 0) {
        if (residual == FR_PT2PT)
            k_ng_terms<FR_PT2PT><<<gM, kNgThreads, 0, st>>>(d.M, x, y, z, m0, m1, ns, (float)c, d.terms);
        else
            k_ng_terms<FR_PT2PL><<<gM, kNgThreads, 0, st>>>(d.M, x, y, z, m0, m1, ns, (float)c, d.terms);
        FR_HIP(hipGetLastError());
    }
    k_ng_blocks<0><<<(d.n_blocks * 64 + kNgThreads - 1) / kNgThreads, kNgThreads, 0, st>>>(
        d.n_blocks, d.blk_off, d.blk_pts, d.blk_w, d.terms, d.data21);
    FR_HIP(hipGetLastError());
    k_ng_blocks<1><<<(d.K * 64 + kNgThreads - 1) / kNgThreads, kNgThreads, 0, st>>>(d.K, d.rhs_off, d.rhs_pts,
                                                                                     d.rhs_w, d.terms, d.bdata);
    FR_HIP(hipGetLastError());
    if (d.E > 0) {
        k_ng_edges<<<(d.E + 63) / 64, 64, 0, st>>>(d.E, d.edges, d.nodes, d.T, 1.0 / sigma, lambda, d.edge_terms);
        FR_HIP(hipGetLastError());
    }
    const int32_t na = std::max(d.n_blocks, d.K);
    k_ng_assemble<<<(na + 63) / 64, 64, 0, st>>>(d.n_blocks, d.data21, d.reg_off, d.reg_ref, d.edge_terms,
                                                 1.0 / (sigma * sigma), d.A, d.K, d.bdata, d.nreg_off, d.nreg_ref,
                                                 d.rhs);
    FR_HIP(hipGetLastError());
    return FR_OK;
}

fr_status ng_step(NodeGraphDev &d, const float *x, const float *y, const float *z, const float *m0, const float *m1,
                  const float *ns, int residual, double c, double sigma, double lambda, double tol, int32_t max_it,
                  hipStream_t st)
{
    FR_TRY(ng_reduce(d, x, y, z, m0, m1, ns, residual, c, sigma, lambda, st));
    FR_HIP(hipMemsetAsync(d.bad, 0, sizeof(int32_t), st));
    k_ng_block_inverse<<<(d.K + 63) / 64, 64, 0, st>>>(d.K, d.A, d.diag_blk, d.minv, d.bad);
    FR_HIP(hipGetLastError());
    // grid-wide PCG when the device can hold the workgroups of one cooperative
    // launch at once, else the single-workgroup kernel
    int per_cu = 0, dev = 0, cus = 0, coop = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(k_ng_pcg_coop),
                                                        kCoopThreads, 0);
    (void)hipGetLastError();
    const int G = std::min({kCoopMaxBlocks, std::max(1, d.K / 4), per_cu * cus});
    bool done = false;
    if (coop && G >= 8) {
        PcgArgs pa{d.K, d.row_off, d.row_blk, d.row_col, d.A, d.minv, d.rhs, d.x, d.r, d.z, d.q, d.p, d.s,
                   d.part, tol, max_it, d.info};
        void *args[] = {&pa};
        done = hipLaunchCooperativeKernel(reinterpret_cast<const void *>(k_ng_pcg_coop), dim3(G), dim3(kCoopThreads),
                                          args, 0, st) == hipSuccess;
        if (!done) (void)hipGetLastError();
    }
    if (!done) {
        k_ng_pcg<<<1, kPcgThreads, 0, st>>>(d.K, d.row_off, d.row_blk, d.row_col, d.A, d.minv, d.rhs, d.x, d.r, d.z,
                                            d.p, d.q, tol, max_it, d.info);
        FR_HIP(hipGetLastError());
    }
    k_ng_update<<<(d.K + 63) / 64, 64, 0, st>>>(d.K, d.x, d.T, d.bad);
    FR_HIP(hipGetLastError());
    return FR_OK;
}

}  // namespace fr
