// Articulated Gauss-Newton step in binary64 on the device (Sec. 5.1, Eq. 19-20,
// Alg. 1, assembly and solve): one block per kinematic tree.
//
// Inputs are the per-body sums S_b = sum J^T J (6x6) and g_b = sum J^T r of the
// points on body b, reduced by the segmented M-step kernel (the per-body
// accumulation of Alg. 1).
// The block runs forward kinematics at the current joint angles to get, for
// every revolute DOF k, its world axis w_k and a point q_k on it; DOF k moves
// every body below its joint with the twist u_k = (w_k, q_k x w_k) (the twist
// convention of Eq. 16), so the spatial velocity Jacobian of body b has column
// u_k for the DOFs of b and its ancestors.  Then
//   A[k][l] = sum_{b moved by k and l} u_k^T S_b u_l,   rhs[k] = sum_{b moved by k} u_k . g_b,
// a Cholesky solve gives dtheta = -A^-1 rhs, theta += dtheta, and a second
// forward kinematics pass writes the binary32 [R | t] of every body for the
// next E-step.
//
// Tree layout (device, built by the host): parent[B], dof_off[B + 1],
// origin[3B] (joint origin in the parent frame), axis[3 n_dof] (unit axis in
// the frame left by the preceding rotations), moved_by[B] (bit k set if DOF k
// moves body b).  n_dof <= 64.
#include <algorithm>
#include <vector>

#include "fr_internal.h"
#include "fr_mstep.h"

namespace fr {

constexpr int kArtThreads = 256;
constexpr int kArtMaxDof = 64;
constexpr int kArtMaxBodies = 128;

struct ArtTree {
    int32_t n_bodies, n_dof;
    const int32_t *parent;
    const int32_t *dof_off;
    const double *origin;
    const double *axis;
    const uint64_t *moved_by;
    int32_t n_levels;
    const int32_t *level_off;    // n_levels + 1: bodies of depth L are level_body[level_off[L] .. level_off[L+1])
    const int32_t *level_body;
};

// R = exp(angle [a]_x) for a unit axis a (two-term series below |angle| = 1e-4).
__device__ inline void axis_rotation(const double *a, double angle, double (&R)[3][3])
{
    double s, c1;
    const double t2 = angle * angle;
    if (fabs(angle) < 1e-4) {
        s = angle * (1.0 - t2 / 6.0);
        c1 = t2 * (0.5 - t2 / 24.0);
    } else {
        s = sin(angle);
        c1 = 1.0 - cos(angle);
    }
    const double K[3][3] = {{0.0, -a[2], a[1]}, {a[2], 0.0, -a[0]}, {-a[1], a[0], 0.0}};
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const double K2 = K[i][0] * K[0][j] + K[i][1] * K[1][j] + K[i][2] * K[2][j];
            R[i][j] = (i == j ? 1.0 : 0.0) + s * K[i][j] + c1 * K2;
        }
}

// Forward kinematics: body frames (R in bodyR[9b], t in bodyT[3b]) and per-DOF
// world axis w (3k) and point q (3k).  The DOF rotations exp(theta_k [a_k]_x)
// are independent and are formed first, one thread per DOF, into Qs (9 per
// DOF); the frames are then composed level by level down the tree, the bodies
// of a level in parallel (each in the same arithmetic as a serial walk).
// Called by the whole block.
__device__ void forward_kinematics(const ArtTree &t, const double *theta, double *Qs, double *bodyR, double *bodyT,
                                   double *w, double *q)
{
    for (int k = threadIdx.x; k < t.n_dof; k += blockDim.x) {
        double Q[3][3];
        axis_rotation(t.axis + 3 * k, theta[k], Q);
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) Qs[9 * k + 3 * i + j] = Q[i][j];
    }
    __syncthreads();
    for (int L = 0; L < t.n_levels; ++L) {   // a body's parent is one level up, complete
        for (int ib = t.level_off[L] + (int)threadIdx.x; ib < t.level_off[L + 1]; ib += blockDim.x) {
            const int b = t.level_body[ib];
            double R[3][3], p[3];
            const int pa = t.parent[b];
            if (pa < 0) {
                for (int i = 0; i < 3; ++i) {
                    for (int j = 0; j < 3; ++j) R[i][j] = (i == j) ? 1.0 : 0.0;
                    p[i] = 0.0;
                }
            } else {
                for (int i = 0; i < 3; ++i) {
                    for (int j = 0; j < 3; ++j) R[i][j] = bodyR[9 * pa + 3 * i + j];
                    p[i] = bodyT[3 * pa + i];
                }
            }
            // joint origin: F = P . Trans(o)
            double o[3];
            for (int i = 0; i < 3; ++i)
                o[i] = R[i][0] * t.origin[3 * b] + R[i][1] * t.origin[3 * b + 1] + R[i][2] * t.origin[3 * b + 2] + p[i];
            for (int k = t.dof_off[b]; k < t.dof_off[b + 1]; ++k) {
                const double *a = t.axis + 3 * k;
                for (int i = 0; i < 3; ++i) {
                    w[3 * k + i] = R[i][0] * a[0] + R[i][1] * a[1] + R[i][2] * a[2];
                    q[3 * k + i] = o[i];
                }
                const double *Q = Qs + 9 * k;
                double N[3][3];
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j)
                        N[i][j] = R[i][0] * Q[0 * 3 + j] + R[i][1] * Q[1 * 3 + j] + R[i][2] * Q[2 * 3 + j];
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j) R[i][j] = N[i][j];
            }
            for (int i = 0; i < 3; ++i) {
                for (int j = 0; j < 3; ++j) bodyR[9 * b + 3 * i + j] = R[i][j];
                bodyT[3 * b + i] = o[i];
            }
        }
        __syncthreads();
    }
}

// mode 0: forward kinematics only (writes mats); mode 1: Gauss-Newton step + forward kinematics.
__global__ void __launch_bounds__(kArtThreads) k_articulated_step(ArtTree tree, int mode, const double *jtj,
                                                                  const double *jtr, double *theta, float *mats,
                                                                  double *step_norm, int32_t *status)
{
    __shared__ double s_th[kArtMaxDof], s_w[3 * kArtMaxDof], s_q[3 * kArtMaxDof], s_u[6 * kArtMaxDof];
    __shared__ double s_A[kArtMaxDof * kArtMaxDof], s_rhs[kArtMaxDof], s_x[kArtMaxDof], s_dg[kArtMaxDof];
    __shared__ double s_R[9 * kArtMaxBodies], s_T[3 * kArtMaxBodies], s_Q[9 * kArtMaxDof];
    // per-body sums and the DOF masks, staged once: the assembly loops read
    // them for every (DOF, DOF) entry and body
    __shared__ double s_S[21 * kArtMaxBodies], s_g[6 * kArtMaxBodies];
    __shared__ uint64_t s_mb[kArtMaxBodies];
    __shared__ int s_ok;
    const int tid = threadIdx.x;
    const int n = tree.n_dof;
    for (int k = tid; k < n; k += kArtThreads) s_th[k] = theta[k];
    if (tid == 0) s_ok = 1;
    __syncthreads();
    if (mode == 1) {
        for (int i = tid; i < 21 * tree.n_bodies; i += kArtThreads) s_S[i] = jtj[i];
        for (int i = tid; i < 6 * tree.n_bodies; i += kArtThreads) s_g[i] = jtr[i];
        for (int b = tid; b < tree.n_bodies; b += kArtThreads) s_mb[b] = tree.moved_by[b];
        forward_kinematics(tree, s_th, s_Q, s_R, s_T, s_w, s_q);
        for (int k = tid; k < n; k += kArtThreads) {
            const double *w = s_w + 3 * k, *q = s_q + 3 * k;
            s_u[6 * k + 0] = w[0];
            s_u[6 * k + 1] = w[1];
            s_u[6 * k + 2] = w[2];
            s_u[6 * k + 3] = q[1] * w[2] - q[2] * w[1];
            s_u[6 * k + 4] = q[2] * w[0] - q[0] * w[2];
            s_u[6 * k + 5] = q[0] * w[1] - q[1] * w[0];
        }
        __syncthreads();
        // A[k][l] = sum over bodies moved by k and l of u_k^T S_b u_l (upper triangle, then mirrored)
        for (int e = tid; e < n * n; e += kArtThreads) {
            const int k = e / n, l = e % n;
            if (l < k) continue;
            double acc = 0.0;
            for (int b = 0; b < tree.n_bodies; ++b) {
                const uint64_t mb = s_mb[b];
                if (!((mb >> k) & 1ull) || !((mb >> l) & 1ull)) continue;
                const double *S = s_S + 21 * b;
                double Su[6];
                int idx = 0;
                double Sf[6][6];
                for (int i = 0; i < 6; ++i)
                    for (int j = i; j < 6; ++j) {
                        Sf[i][j] = S[idx];
                        Sf[j][i] = S[idx];
                        ++idx;
                    }
                for (int i = 0; i < 6; ++i) {
                    double v = 0.0;
                    for (int j = 0; j < 6; ++j) v += Sf[i][j] * s_u[6 * l + j];
                    Su[i] = v;
                }
                for (int i = 0; i < 6; ++i) acc += s_u[6 * k + i] * Su[i];
            }
            s_A[k * n + l] = acc;
            s_A[l * n + k] = acc;
        }
        for (int k = tid; k < n; k += kArtThreads) {
            double acc = 0.0;
            for (int b = 0; b < tree.n_bodies; ++b) {
                if (!((s_mb[b] >> k) & 1ull)) continue;
                for (int i = 0; i < 6; ++i) acc += s_u[6 * k + i] * s_g[6 * b + i];
            }
            s_rhs[k] = acc;
        }
        __syncthreads();
        // a DOF that moves no supported point has an all-zero row and column: hold it (identity
        // row, zero right-hand side) and solve the others
        for (int k = tid; k < n; k += kArtThreads) {
            if (s_A[k * n + k] == 0.0) {
                s_A[k * n + k] = 1.0;
                s_rhs[k] = 0.0;
            }
            s_dg[k] = s_A[k * n + k];
        }
        __syncthreads();
        // Cholesky A = L L^T in place (lower triangle), right-looking: column j
        // is scaled by its pivot, then the trailing triangle takes its rank-1
        // update; every entry receives its updates in column order, as in the
        // left-looking form
        for (int j = 0; j < n; ++j) {
            if (tid == 0) {
                // a pivot at most kPivotTol of its diagonal entry is a numerically
                // unobservable direction at the precision of the binary32 sums (as
                // the rigid solve)
                double v = s_A[j * n + j];
                if (!(v > kPivotTol * s_dg[j])) {
                    s_ok = 0;
                    v = 1.0;
                }
                s_A[j * n + j] = sqrt(v);
            }
            __syncthreads();
            for (int i = j + 1 + tid; i < n; i += kArtThreads) s_A[i * n + j] = s_A[i * n + j] / s_A[j * n + j];
            __syncthreads();
            const int m = n - j - 1;   // trailing size
            for (int e = tid; e < m * m; e += kArtThreads) {
                const int i = j + 1 + e / m, k = j + 1 + e % m;
                if (k <= i) s_A[i * n + k] -= s_A[i * n + j] * s_A[k * n + j];
            }
            __syncthreads();
        }
        // L y = -rhs (column-oriented: y_k is final once the columns before it
        // have been subtracted), then L^T x = y
        for (int i = tid; i < n; i += kArtThreads) s_x[i] = -s_rhs[i];
        __syncthreads();
        for (int k = 0; k < n; ++k) {
            if (tid == 0) s_x[k] = s_x[k] / s_A[k * n + k];
            __syncthreads();
            for (int i = k + 1 + tid; i < n; i += kArtThreads) s_x[i] -= s_A[i * n + k] * s_x[k];
            __syncthreads();
        }
        for (int k = n - 1; k >= 0; --k) {
            if (tid == 0) s_x[k] = s_x[k] / s_A[k * n + k];
            __syncthreads();
            for (int i = tid; i < k; i += kArtThreads) s_x[i] -= s_A[k * n + i] * s_x[k];
            __syncthreads();
        }
        if (tid == 0) {
            if (s_ok) {
                double nrm = 0.0;
                for (int i = n - 1; i >= 0; --i) nrm += s_x[i] * s_x[i];
                for (int i = 0; i < n; ++i) s_th[i] += s_x[i];
                if (step_norm) *step_norm = sqrt(nrm);
                if (status) *status = FR_OK;
            } else {
                if (step_norm) *step_norm = 0.0;
                if (status) *status = FR_EDEGENERATE;
            }
        }
        __syncthreads();
        for (int k = tid; k < n; k += kArtThreads) theta[k] = s_th[k];
    }
    forward_kinematics(tree, s_th, s_Q, s_R, s_T, s_w, s_q);
    for (int b = tid; b < tree.n_bodies; b += kArtThreads) {
        for (int i = 0; i < 3; ++i) {
            for (int j = 0; j < 3; ++j) mats[12 * b + 4 * i + j] = (float)s_R[9 * b + 3 * i + j];
            mats[12 * b + 4 * i + 3] = (float)s_T[3 * b + i];
        }
    }
}

fr_status launch_articulated_step(const ArtTreeHost &h, int mode, const double *jtj, const double *jtr, double *theta,
                                  float *mats, double *step_norm, int32_t *status, hipStream_t st)
{
    ArtTree t{h.n_bodies, h.n_dof, h.parent, h.dof_off, h.origin, h.axis, h.moved_by, h.n_levels, h.level_off,
              h.level_body};
    k_articulated_step<<<1, kArtThreads, 0, st>>>(t, mode, jtj, jtr, theta, mats, step_norm, status);
    FR_HIP(hipGetLastError());
    return FR_OK;
}

fr_status upload_tree(fr_ctx *ctx, const fr_kinematic_tree *tree, hipStream_t st, ArtTreeHost &out)
{
    const int32_t B = tree->n_bodies;
    if (B < 1 || B > kArtMaxBodies || !tree->parent || !tree->dof_offset || !tree->origin || !tree->axis) {
        set_error("kinematic tree: 1..%d bodies with parent, dof_offset, origin and axis arrays required",
                  kArtMaxBodies);
        return FR_EINVAL;
    }
    const int32_t n = tree->dof_offset[B];
    if (tree->dof_offset[0] != 0 || n < 1 || n > kArtMaxDof) {
        set_error("kinematic tree: dof_offset[0] must be 0 and 1 <= n_dof <= %d", kArtMaxDof);
        return FR_EINVAL;
    }
    std::vector<uint64_t> moved(B, 0);
    std::vector<int32_t> depth(B, 0);
    for (int32_t b = 0; b < B; ++b) {
        if (tree->parent[b] >= b || tree->parent[b] < -1 || tree->dof_offset[b + 1] < tree->dof_offset[b]) {
            set_error("kinematic tree: parent[b] must be in [-1, b) and dof_offset non-decreasing (body %d)", b);
            return FR_EINVAL;
        }
        uint64_t m = tree->parent[b] >= 0 ? moved[tree->parent[b]] : 0ull;
        depth[b] = tree->parent[b] >= 0 ? depth[tree->parent[b]] + 1 : 0;
        for (int32_t k = tree->dof_offset[b]; k < tree->dof_offset[b + 1]; ++k) m |= 1ull << k;
        moved[b] = m;
    }
    // bodies grouped by depth (a parent always has a smaller index, so its depth is known first)
    const int32_t n_levels = *std::max_element(depth.begin(), depth.end()) + 1;
    std::vector<int32_t> level_off(n_levels + 1, 0), level_body;
    for (int32_t L = 0; L < n_levels; ++L) {
        level_off[L] = (int32_t)level_body.size();
        for (int32_t b = 0; b < B; ++b)
            if (depth[b] == L) level_body.push_back(b);
    }
    level_off[n_levels] = B;
    out.n_bodies = B;
    out.n_dof = n;
    out.n_levels = n_levels;
    const size_t bp = sizeof(int32_t) * B, bd = sizeof(int32_t) * (B + 1), bo = sizeof(double) * 3 * B,
                 ba = sizeof(double) * 3 * n, bm = sizeof(uint64_t) * B, bl = sizeof(int32_t) * (n_levels + 1);
    // 8-byte aligned sub-buffers: doubles and masks first
    FR_TRY(out.buf.alloc(ctx, bo + ba + bm + bp + bd + bl + bp));
    char *p = out.buf.as<char>();
    FR_HIP(hipMemcpyAsync(p, tree->origin, bo, hipMemcpyHostToDevice, st));
    FR_HIP(hipMemcpyAsync(p + bo, tree->axis, ba, hipMemcpyHostToDevice, st));
    FR_HIP(hipMemcpyAsync(p + bo + ba, moved.data(), bm, hipMemcpyHostToDevice, st));
    FR_HIP(hipMemcpyAsync(p + bo + ba + bm, tree->parent, bp, hipMemcpyHostToDevice, st));
    FR_HIP(hipMemcpyAsync(p + bo + ba + bm + bp, tree->dof_offset, bd, hipMemcpyHostToDevice, st));
    FR_HIP(hipMemcpyAsync(p + bo + ba + bm + bp + bd, level_off.data(), bl, hipMemcpyHostToDevice, st));
    FR_HIP(hipMemcpyAsync(p + bo + ba + bm + bp + bd + bl, level_body.data(), bp, hipMemcpyHostToDevice, st));
    FR_HIP(hipStreamSynchronize(st));
    out.origin = reinterpret_cast<const double *>(p);
    out.axis = reinterpret_cast<const double *>(p + bo);
    out.moved_by = reinterpret_cast<const uint64_t *>(p + bo + ba);
    out.parent = reinterpret_cast<const int32_t *>(p + bo + ba + bm);
    out.dof_off = reinterpret_cast<const int32_t *>(p + bo + ba + bm + bp);
    out.level_off = reinterpret_cast<const int32_t *>(p + bo + ba + bm + bp + bd);
    out.level_body = reinterpret_cast<const int32_t *>(p + bo + ba + bm + bp + bd + bl);
    return FR_OK;
}

}  // namespace fr
