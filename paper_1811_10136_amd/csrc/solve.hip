// Rigid Gauss-Newton update in binary64 on the device (Eq. 17 and the
// left-multiplied twist update of Eq. 16): one thread per set solves
// A dzeta = -b by Cholesky, maps dzeta through the SE(3) exponential and
// composes it on the left of the set's pose; it also refreshes the binary32
// [R | t] the next E-step reads.
#include "fr_internal.h"
#include "fr_mstep.h"

namespace fr {

// Exp of the twist (w, v): R = I + A [w]x + B [w]x^2, p = (I + B [w]x + C [w]x^2) v,
// A = sin t / t, B = (1 - cos t) / t^2, C = (t - sin t) / t^3, t = |w|; two-term
// series below t = 1e-4.
__device__ inline void se3_exp(const double (&z)[6], double (&E)[3][4])
{
    const double wx = z[0], wy = z[1], wz = z[2];
    const double th2 = wx * wx + wy * wy + wz * wz;
    const double th = sqrt(th2);
    double A, B, C;
    if (th < 1e-4) {
        A = 1.0 - th2 / 6.0;
        B = 0.5 - th2 / 24.0;
        C = 1.0 / 6.0 - th2 / 120.0;
    } else {
        const double sn = sin(th), cs = cos(th);
        A = sn / th;
        B = (1.0 - cs) / th2;
        C = (th - sn) / (th2 * th);
    }
    const double K[3][3] = {{0.0, -wz, wy}, {wz, 0.0, -wx}, {-wy, wx, 0.0}};
    double K2[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) K2[i][j] = K[i][0] * K[0][j] + K[i][1] * K[1][j] + K[i][2] * K[2][j];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        double p = 0.0;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const double I = (i == j) ? 1.0 : 0.0;
            E[i][j] = I + A * K[i][j] + B * K2[i][j];
            p += (I + B * K[i][j] + C * K2[i][j]) * z[3 + j];
        }
        E[i][3] = p;
    }
}


__global__ void __launch_bounds__(64) k_solve_rigid(int32_t n, const double *jtj, const double *jtr, double *poses,
                                                    float *mats, double *twist_norm, int32_t *status,
                                                    const int32_t *active, int32_t *stop, double twist_tol,
                                                    int32_t *iters, int32_t *ran)
{
    const int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const bool run = !((active != nullptr && active[s] == 0) || (stop != nullptr && stop[s] == 0));
    if (ran != nullptr) ran[s] = run ? 1 : 0;
    if (!run) return;
    double A[6][6], b[6];
    {
        int idx = 0;
#pragma unroll
        for (int i = 0; i < 6; ++i)
#pragma unroll
            for (int j = i; j < 6; ++j) {
                const double v = jtj[(size_t)s * 21 + idx++];
                A[i][j] = v;
                A[j][i] = v;
            }
#pragma unroll
        for (int i = 0; i < 6; ++i) b[i] = jtr[(size_t)s * 6 + i];
    }
    // Cholesky A = L L^T (in the lower triangle of A); a pivot at most
    // kPivotTol times its diagonal entry marks A as singular
    double d0[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) d0[j] = A[j][j];
    bool ok = true;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        double sum = A[j][j];
#pragma unroll
        for (int k = 0; k < j; ++k) sum -= A[j][k] * A[j][k];
        ok = ok && (sum > 0.0) && (sum > kPivotTol * d0[j]);
        const double ljj = sqrt(ok ? sum : 1.0);
        A[j][j] = ljj;
#pragma unroll
        for (int i = j + 1; i < 6; ++i) {
            double v = A[i][j];
#pragma unroll
            for (int k = 0; k < j; ++k) v -= A[i][k] * A[j][k];
            A[i][j] = v / ljj;
        }
    }
    if (iters != nullptr) iters[s] += 1;
    if (!ok) {
        status[s] = FR_EDEGENERATE;
        twist_norm[2 * s] = 0.0;
        twist_norm[2 * s + 1] = 0.0;
        if (stop != nullptr) stop[s] = 0;
        return;
    }
    double y[6], z[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        double v = -b[i];
#pragma unroll
        for (int k = 0; k < i; ++k) v -= A[i][k] * y[k];
        y[i] = v / A[i][i];
    }
#pragma unroll
    for (int i = 5; i >= 0; --i) {
        double v = y[i];
#pragma unroll
        for (int k = i + 1; k < 6; ++k) v -= A[k][i] * z[k];
        z[i] = v / A[i][i];
    }
    double E[3][4];
    se3_exp(z, E);
    double T[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) T[i][j] = poses[(size_t)s * 16 + 4 * i + j];
    double N[3][4];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
            N[i][j] = E[i][0] * T[0][j] + E[i][1] * T[1][j] + E[i][2] * T[2][j] + (j == 3 ? E[i][3] : 0.0);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            poses[(size_t)s * 16 + 4 * i + j] = N[i][j];
            mats[(size_t)s * 12 + 4 * i + j] = (float)N[i][j];
        }
    const double tw = sqrt(z[0] * z[0] + z[1] * z[1] + z[2] * z[2]);
    const double tv = sqrt(z[3] * z[3] + z[4] * z[4] + z[5] * z[5]);
    twist_norm[2 * s] = tw;
    twist_norm[2 * s + 1] = tv;
    status[s] = FR_OK;
    // stop on a small twist (Sec. 6.1): the set's later iterations do nothing
    if (stop != nullptr && tw < twist_tol && tv < twist_tol) stop[s] = 0;
}

fr_status launch_solve_rigid(int32_t n, const double *jtj, const double *jtr, double *poses, float *mats,
                             double *twist_norm, int32_t *status, const int32_t *active, hipStream_t st,
                             int32_t *stop, double twist_tol, int32_t *iters, int32_t *ran)
{
    if (n <= 0) return FR_OK;
    k_solve_rigid<<<(n + 63) / 64, 64, 0, st>>>(n, jtj, jtr, poses, mats, twist_norm, status, active, stop,
                                                 twist_tol, iters, ran);
    FR_HIP(hipGetLastError());
    return FR_OK;
}

// Variance update of the optimised-sigma loop on the device, after a solve
// (one thread per set).  A set that the solve ran for (ran[s]) and that did
// not degenerate takes the
// closed-form variance V / (3 sum w) of the reduction, as the kernel's
// per-axis variance s^2 / 4, floored: s = max(s_min, sqrt(V / (3 sum w) / (1/4))).
// Its lattice scale factors and outlier constant follow s with the host's
// arithmetic (scale_factors, outlier_constant) in the same order, so a
// rebuild at the new s matches one sized on the host.
__global__ void __launch_bounds__(64) k_sigma_update(int32_t n, const int32_t *ran, const int32_t *status,
                                                     const double *stats, const double *var, SigmaRule rule,
                                                     double *sig, float *kset, float *seg_c)
{
    const int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n || ran[s] == 0) return;
    if (status[s] != FR_OK || !(stats[4 * (size_t)s] > 0.0)) return;
    const double v = var[s] / (3.0 * stats[4 * (size_t)s]);
    const double sg = fmax(rule.sigma_min, sqrt(fmax(v, 0.0) / rule.kernel_axis_var));
    sig[s] = sg;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        float k = 0.0f;
        if (i < rule.feat) {
            const double sd = i < 3 ? sg : rule.sigma_n;
            k = (float)(rule.scale_num / (sd * rule.scale_den[i]));
        }
        kset[8 * (size_t)s + i] = k;
    }
    double c = rule.c_override;
    if (!(c >= 0.0)) {
        double h = rule.mass0;
        for (int i = 0; i < rule.feat; ++i) h *= i < 3 ? sg : rule.sigma_n;
        c = rule.c_pre[s] * h;
    }
    seg_c[s] = (float)c;
}

fr_status launch_sigma_update(int32_t n, const int32_t *ran, const int32_t *status, const double *stats,
                              const double *var, const SigmaRule &rule, double *sig, float *kset, float *seg_c,
                              hipStream_t st)
{
    if (n <= 0) return FR_OK;
    k_sigma_update<<<(n + 63) / 64, 64, 0, st>>>(n, ran, status, stats, var, rule, sig, kset, seg_c);
    FR_HIP(hipGetLastError());
    return FR_OK;
}

}  // namespace fr
