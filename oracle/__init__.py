"""CPU FP64 oracle of FilterReg's E-step and twist M-step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this package:
only ``tests/``, the smoke check and the CPU-baseline leg of the benchmark do.
It shares no code with the GPU library (``paper_1811_10136_amd``) and neither
package imports the other; the seeded input generators live in ``synth``.

Layout
* ``lattice.c``     -- permutohedral embedding, splat, slice and a brute-force
  kernel sum (binary32 key path, binary64 values), loaded with ctypes.
* this module       -- features, E-step driver, the M-step of Eq. (7)/(10)
  through the twist Jacobian of Eq. (16), the Gauss-Newton step of Eq. (17)-(18),
  the SE(3) exponential and the rigid EM loop, all in float64 NumPy.
* ``articulated.py`` / ``nodegraph.py`` -- the kinematic models of Sec. 5.1/5.2.

Every function names the passage of the paper it follows.
"""
from __future__ import annotations

import ctypes
import time
import math
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = [os.path.join(_HERE, "lattice.c")]
_lib = None

C_FLAGS = ["-O2", "-std=c99", "-Wall", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]


def build(force: bool = True) -> str:
    """Compile the C part of the oracle with gcc (binary32 key path: no FMA contraction)."""
    if force or not os.path.exists(_SO) or any(os.path.getmtime(s) > os.path.getmtime(_SO) for s in _SRC):
        tmp = _SO + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", *C_FLAGS, *_SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _L():
    global _lib
    if _lib is None:
        build(force=False)
        lib = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        ci = ctypes.c_int
        lib.or_scale_factors.argtypes = [ci, P, P]
        lib.or_embed_many.argtypes = [ci, i64, P, P, P, P, P]
        lib.or_lattice_build.argtypes = [ci, ci, i64, P, P, P, P, P, P]
        lib.or_lattice_build.restype = i64
        lib.or_slice.argtypes = [ci, ci, i64, P, P, i64, P, P, P, P]
        lib.or_bf_lattice_sum.argtypes = [ci, ci, i64, P, P, i64, P, P, P]
        lib.or_transform_f32.argtypes = [i64, P, P, P, ci]
        lib.or_blur.argtypes = [ci, ci, i64, P, P, ctypes.c_double]
        lib.or_blur.restype = ci
        _lib = lib
    return _lib


def _p(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


# ---------------------------------------------------------------------------
# Features and embedding (Sec. 3.3 "Features", Sec. 4.1 normalised features)
# ---------------------------------------------------------------------------

def feature_sigmas(feat: int, sigma, sigma_n: float):
    """Per-dimension kernel widths: position axes, then normal axes for d = 6."""
    s = [float(v) for v in sigma]
    if feat == 6:
        s += [float(sigma_n)] * 3
    return np.asarray(s, dtype=np.float64)


def scale_factors(sigmas) -> np.ndarray:
    """k_i = sqrt(2/3)(d+1)/(sigma_i sqrt((i+1)(i+2))) in binary32: feature normalisation
    (Sec. 4.1) folded into the lattice scale of the permutohedral method (Sec. 4.2)."""
    sig = np.ascontiguousarray(sigmas, dtype=np.float64)
    k = np.zeros(len(sig), dtype=np.float32)
    _L().or_scale_factors(len(sig), _p(sig), _p(k))
    return k


def features(points: np.ndarray, normals: Optional[np.ndarray], feat: int) -> np.ndarray:
    """Raw binary32 feature rows: [x, y, z] or [x, y, z, nx, ny, nz] (Eq. 8)."""
    p = np.asarray(points, dtype=np.float32)
    if feat == 3:
        return np.ascontiguousarray(p)
    return np.ascontiguousarray(np.concatenate([p, np.asarray(normals, dtype=np.float32)], axis=1))


def embed(feat_rows: np.ndarray, k: np.ndarray):
    """Permutohedral embedding of each row (Sec. 4.2): keys (n, d+1, d) int32,
    barycentric weights (n, d+1) float64, elevated coordinates (n, d+1) float32."""
    f = np.ascontiguousarray(feat_rows, dtype=np.float32)
    n, d = f.shape
    keys = np.zeros((n, d + 1, d), dtype=np.int32)
    b = np.zeros((n, d + 1), dtype=np.float64)
    e = np.zeros((n, d + 1), dtype=np.float32)
    _L().or_embed_many(d, n, _p(f), _p(np.ascontiguousarray(k, dtype=np.float32)), _p(keys), _p(b), _p(e))
    return keys, b, e


def splat_values(points: np.ndarray, normals: Optional[np.ndarray], residual: str, m2: bool = False) -> np.ndarray:
    """Per-observation values v_y of Eq. (11): [1, y] (Eq. 6) or [1, y, n_y] (Eq. 9); with m2 a last
    column |y|^2, the second moment the optimised variance of Sec. 3.3 needs."""
    y = np.asarray(points, dtype=np.float64)
    cols = [np.ones((len(y), 1)), y]
    if residual == "pt2pl":
        cols.append(np.asarray(normals, dtype=np.float64))
    if m2:
        cols.append(np.sum(y * y, axis=1, keepdims=True))
    return np.ascontiguousarray(np.concatenate(cols, axis=1))


class Lattice:
    """The observation's lattice: sorted keys, occupancy and per-vertex value sums."""

    def __init__(self, keys, occ, vals, k, d):
        self.keys, self.occ, self.vals, self.k, self.d = keys, occ, vals, k, d

    @property
    def n_vertices(self):
        return len(self.occ)


def lattice_build(feat_rows: np.ndarray, vals: np.ndarray, k: np.ndarray) -> Lattice:
    """Splat every observation value onto the d+1 vertices of its simplex (Sec. 4.2, Eq. 14)."""
    f = np.ascontiguousarray(feat_rows, dtype=np.float32)
    v = np.ascontiguousarray(vals, dtype=np.float64)
    n, d = f.shape if f.ndim == 2 else (0, len(k))
    nv = v.shape[1]
    cap = max(1, n * (d + 1))
    keys = np.zeros((cap, d), dtype=np.int32)
    occ = np.zeros(cap, dtype=np.int32)
    out = np.zeros((cap, nv), dtype=np.float64)
    kk = np.ascontiguousarray(k, dtype=np.float32)
    if n == 0:
        return Lattice(keys[:0], occ[:0], out[:0], kk, d)
    nvtx = _L().or_lattice_build(d, nv, n, _p(f), _p(v), _p(kk), _p(keys), _p(occ), _p(out))
    if nvtx < 0:
        raise MemoryError("oracle lattice build: out of memory")
    return Lattice(keys[:nvtx].copy(), occ[:nvtx].copy(), out[:nvtx].copy(), kk, d)


def lattice_slice(lat: Lattice, feat_rows: np.ndarray, return_touched: bool = False):
    """Interpolate the lattice at query features with their barycentric weights (Sec. 4.2)."""
    f = np.ascontiguousarray(feat_rows, dtype=np.float32)
    m = len(f)
    nv = lat.vals.shape[1]
    out = np.zeros((m, nv), dtype=np.float64)
    touched = np.zeros(max(1, lat.n_vertices), dtype=np.uint8)
    if m and lat.n_vertices:
        _L().or_slice(lat.d, nv, lat.n_vertices, _p(lat.keys), _p(lat.vals), m, _p(f), _p(lat.k),
                      _p(out), _p(touched))
    if return_touched:
        return out, int(touched[: lat.n_vertices].sum())
    return out


def blur_output_scale(d: int) -> float:
    """Output scale 1 / (1 + 2^-d) of the published permutohedral filter (the cited Adams et al. method)."""
    return 1.0 / (1.0 + 2.0 ** (-d))


def lattice_blur(lat: Lattice) -> Lattice:
    """The uncustomised filter's blur: d+1 passes of [1/4, 1/2, 1/4] along the lattice directions,
    then the output scale; a new Lattice with the blurred values (keys and occupancy shared)."""
    vals = np.ascontiguousarray(lat.vals, dtype=np.float64).copy()
    if lat.n_vertices:
        if _L().or_blur(lat.d, vals.shape[1], lat.n_vertices, _p(np.ascontiguousarray(lat.keys)), _p(vals),
                        blur_output_scale(lat.d)) != 0:
            raise MemoryError("oracle blur: out of memory")
    return Lattice(lat.keys, lat.occ, vals, lat.k, lat.d)


def joint_lattice(fy: np.ndarray, vals: np.ndarray, fx: np.ndarray, k: np.ndarray) -> Lattice:
    """Splat of the augmented input of the uncustomised filter: the observation's features with its
    values and the query features with zero values, so that the query simplices exist in the lattice."""
    fy = np.asarray(fy, dtype=np.float32)
    fx = np.asarray(fx, dtype=np.float32)
    v = np.asarray(vals, dtype=np.float64)
    rows = np.concatenate([fy.reshape(-1, len(k)), fx.reshape(-1, len(k))])
    allv = np.concatenate([v, np.zeros((len(fx), v.shape[1]))])
    return lattice_build(rows, allv, k)


def estep_blurred(obs, obs_n, x32, n32, feat: int, residual: str, k: np.ndarray):
    """E-step through the uncustomised filter: splat of [Y, X] with values [v_y, 0], blur, slice at X.
    Returns M0, M1 and (point-to-plane) the normal sum, like estep()."""
    lat = joint_lattice(features(obs, obs_n, feat), splat_values(obs, obs_n, residual), features(x32, n32, feat), k)
    g = lattice_slice(lattice_blur(lat), features(x32, n32, feat))
    return g[:, 0].copy(), g[:, 1:4].copy(), (g[:, 4:7].copy() if residual == "pt2pl" else None)


def brute_force_lattice_sum(fy, vals, fx, k):
    """Sum_y K(x, y) v_y with K from pairs of shared simplex vertices; no lattice built."""
    fy = np.ascontiguousarray(fy, dtype=np.float32)
    fx = np.ascontiguousarray(fx, dtype=np.float32)
    v = np.ascontiguousarray(vals, dtype=np.float64)
    n, d = fy.shape
    m = len(fx)
    out = np.zeros((m, v.shape[1]), dtype=np.float64)
    _L().or_bf_lattice_sum(d, v.shape[1], n, _p(fy), _p(v), m, _p(fx),
                           _p(np.ascontiguousarray(k, dtype=np.float32)), _p(out))
    return out


def transform_f32(mat12: np.ndarray, pts: np.ndarray, translate: bool = True) -> np.ndarray:
    """Pinned binary32 rigid transform ((R0 x + R1 y) + R2 z) + t (Eq. 15 with T in binary32)."""
    p = np.ascontiguousarray(pts, dtype=np.float32)
    out = np.zeros_like(p)
    m = np.ascontiguousarray(mat12, dtype=np.float32).reshape(12)
    if len(p):
        _L().or_transform_f32(len(p), _p(m), _p(p), _p(out), 1 if translate else 0)
    return out


def pose_to_mat12(T: np.ndarray) -> np.ndarray:
    """Row-major [R | t] of a float64 pose, each entry rounded once to binary32."""
    return np.ascontiguousarray(np.asarray(T, dtype=np.float64)[:3, :4].astype(np.float32).reshape(12))


# ---------------------------------------------------------------------------
# E-step (Eq. 6, 8, 9) through the lattice
# ---------------------------------------------------------------------------

def estep(lat: Lattice, x32: np.ndarray, n32: Optional[np.ndarray], feat: int, residual: str, m2: bool = False):
    """M0 (M,), M1 (M,3) and, for point-to-plane, the un-normalised normal sum (M,3); with m2 (a lattice
    built from splat_values(..., m2=True)) also M2 = sum_k K |y_k|^2 (M,) as a fourth result."""
    g = lattice_slice(lat, features(x32, n32, feat))
    m0 = g[:, 0].copy()
    m1 = g[:, 1:4].copy()
    ns = g[:, 4:7].copy() if residual == "pt2pl" else None
    if m2:
        return m0, m1, ns, g[:, -1].copy()
    return m0, m1, ns


def kernel_mass(sigmas, blurred: bool = False) -> float:
    """Integral over feature space of the lattice kernel of one observation, K(x, y) = sum_v b_v(x) b_v(y)
    (Sec. 4.2 splat and slice; sigmas: the width of every feature dimension, position and normal).

    The hats b_v of the vertices sum to one everywhere and are congruent, so each integrates to the
    volume per vertex, and so does K over x for any y.  The vertices, the points of the hyperplane
    sum(v) = 0 whose d+1 integer coordinates share one remainder modulo d+1, are the scaled lattice
    (d+1) A*_d, with (d+1)^(d - 1/2) volume per point; the embedding stretches the normalised feature
    f_i / sigma_i by sqrt(2/3) (d+1) in every direction.  Hence (3/2)^(d/2) / sqrt(d+1) prod sigma_i.
    The uncustomised filter's blur keeps the mass of the vertex values ([1/4, 1/2, 1/4] along each
    direction) and scales the output by 1 / (1 + 2^-d)."""
    s = np.asarray(sigmas, dtype=np.float64)
    d = len(s)
    h = 1.5 ** (d / 2.0) / math.sqrt(d + 1.0) * float(np.prod(s))
    return h * blur_output_scale(d) if blurred else h


def outlier_constant(w: float, n_obs: int, n_model: int, sigmas, blurred: bool = False) -> float:
    """c of Eq. (7) in the units of the lattice sums.  Eq. (4) sets the uniform component beside
    Gaussian PDFs of unit mass and Eq. (7) gives c = w/(1-w) N/M against their sum; the lattice
    sum M0 = sum_k K(x, y_k) uses a kernel of mass kernel_mass(sigmas) per observation instead, so
    the posterior weight M0 / (M0 + c) keeps its meaning with c = w/(1-w) N/M kernel_mass.
    sigmas: every feature dimension's width (feature_sigmas)."""
    if n_model == 0 or w <= 0.0:
        return 0.0
    return float(w / (1.0 - w) * (n_obs / n_model) * kernel_mass(sigmas, blurred))


# ---------------------------------------------------------------------------
# M-step: twist Jacobian (Eq. 16) and Gauss-Newton normal equations (Eq. 17-18)
# ---------------------------------------------------------------------------

def skew(v: np.ndarray) -> np.ndarray:
    """[v]_x with [v]_x b = v x b; works on (..., 3)."""
    v = np.asarray(v, dtype=np.float64)
    z = np.zeros(v.shape[:-1])
    return np.stack([
        np.stack([z, -v[..., 2], v[..., 1]], -1),
        np.stack([v[..., 2], z, -v[..., 0]], -1),
        np.stack([-v[..., 1], v[..., 0], z], -1)], -2)


def point_jacobian(x: np.ndarray) -> np.ndarray:
    """d x_new / d zeta at zeta = 0 for x_new = (I + [w]_x) x + t (Eq. 16): [-[x]_x, I] (M, 3, 6).

    The update matrix of Eq. (16) adds w x x, and w x x = -[x]_x w, so the
    rotational block is -[x]_x; the printed [skew(x), I] has the opposite
    sign, and finite differences side with the update matrix."""
    x = np.asarray(x, dtype=np.float64)
    J = np.zeros(x.shape[:-1] + (3, 6))
    J[..., :, :3] = -skew(x)
    J[..., :, 3:] = np.eye(3)
    return J


def residuals_and_jacobians(x, m0, m1, nsum, c, sigma, residual, normalize_n=False):
    """Per-point weight, residual and twist Jacobian of Eq. (7) / Eq. (10).

    Points with M0 = 0 have no target and get weight 0.  Returns
    (w (M,), r (M, k), J (M, k, 6), support mask) with k = 3 (pt2pt) or 1 (pt2pl).
    Residuals are divided by sigma (the Sigma^-1 weighting of Eq. 7).
    """
    x = np.asarray(x, dtype=np.float64)
    m0 = np.asarray(m0, dtype=np.float64)
    sup = m0 > 0
    safe = np.where(sup, m0, 1.0)
    w = np.where(sup, m0 / (m0 + c), 0.0)
    tgt = np.asarray(m1, dtype=np.float64) / safe[:, None]
    Jx = point_jacobian(x)
    if residual == "pt2pt":
        r = (x - tgt) / sigma
        J = Jx / sigma
    else:
        n = np.asarray(nsum, dtype=np.float64) / safe[:, None]
        if normalize_n:
            nn = np.linalg.norm(n, axis=1, keepdims=True)
            n = np.where(nn > 0, n / np.where(nn > 0, nn, 1.0), 0.0)
        r = (np.einsum("ij,ij->i", n, x - tgt) / sigma)[:, None]
        J = np.einsum("ij,ijk->ik", n, Jx)[:, None, :] / sigma
    r = np.where(sup[:, None], r, 0.0)
    J = np.where(sup[:, None, None], J, 0.0)
    return w, r, J, sup


def normal_equations(x, m0, m1, nsum, c, sigma, residual, normalize_n=False):
    """A = sum w J^T J, b = sum w J^T r (Eq. 17-18 with the rigid dzeta/dtheta = I of Sec. 5),
    plus stats [sum w, sum w r^2, n_support, sum M0]."""
    w, r, J, sup = residuals_and_jacobians(x, m0, m1, nsum, c, sigma, residual, normalize_n)
    A = np.einsum("i,ikp,ikq->pq", w, J, J)
    b = np.einsum("i,ikp,ik->p", w, J, r)
    stats = np.array([w.sum(), np.einsum("i,ik,ik->", w, r, r), float(sup.sum()),
                      float(np.asarray(m0, dtype=np.float64).sum())])
    return A, b, stats


def per_point_jtj(x, m0, m1, nsum, c, sigma, residual, normalize_n=False):
    """Per-point w J^T J (M, 6, 6) and w J^T r (M, 6): the per-point summands of Alg. 1."""
    w, r, J, _ = residuals_and_jacobians(x, m0, m1, nsum, c, sigma, residual, normalize_n)
    return np.einsum("i,ikp,ikq->ipq", w, J, J), np.einsum("i,ikp,ik->ip", w, J, r)


def se3_exp(zeta: np.ndarray) -> np.ndarray:
    """Exponential of the twist zeta = (w, v) (Eq. 16 ordering alpha, beta, gamma, a, b, c).

    R = I + A [w]_x + B [w]_x^2, p = (I + B [w]_x + C [w]_x^2) v with
    A = sin t / t, B = (1 - cos t)/t^2, C = (t - sin t)/t^3, t = |w|; below
    t = 1e-4 the leading two terms of each series are used."""
    z = np.asarray(zeta, dtype=np.float64)
    w, v = z[:3], z[3:]
    th = float(np.linalg.norm(w))
    K = skew(w)
    K2 = K @ K
    if th < 1e-4:
        t2 = th * th
        A = 1.0 - t2 / 6.0
        B = 0.5 - t2 / 24.0
        C = 1.0 / 6.0 - t2 / 120.0
    else:
        A = math.sin(th) / th
        B = (1.0 - math.cos(th)) / (th * th)
        C = (th - math.sin(th)) / (th ** 3)
    T = np.eye(4)
    T[:3, :3] = np.eye(3) + A * K + B * K2
    T[:3, 3] = (np.eye(3) + B * K + C * K2) @ v
    return T


class Degenerate(RuntimeError):
    """The normal equations are not positive definite (no support or rank-deficient)."""


# The Gauss-Newton step (Eq. 17) exists only for an invertible A, and invertibility is decided at the
# precision A is known to: its per-point terms are binary32 values summed in binary32 over tiles of 1024
# points, so an entry carries rounding of up to about 1024 * 2^-24 = 6.1e-5 of the diagonal scale.  A
# Cholesky pivot L_jj^2 (the part of A_jj the earlier directions leave unexplained) at or below 1e-4 A_jj
# cannot be told from zero: the direction is numerically unobservable and the system counts as singular.
RIGID_PIVOT_TOL = 1e-4


def gn_step(A: np.ndarray, b: np.ndarray, pivot_tol: float = 0.0) -> np.ndarray:
    """Delta = -A^-1 b (Eq. 17) by Cholesky; raises Degenerate when A is not SPD, or when a pivot
    L_jj^2 is at most pivot_tol * A_jj."""
    try:
        L = np.linalg.cholesky(A)
    except np.linalg.LinAlgError as e:
        raise Degenerate(str(e)) from e
    if pivot_tol > 0.0:
        rel = np.diag(L) ** 2 / np.diag(A)
        if (rel <= pivot_tol).any():
            raise Degenerate(f"relative Cholesky pivot {rel.min():.2e} <= {pivot_tol:g}")
    y = np.linalg.solve(L, -b)
    return np.linalg.solve(L.T, y)


# ---------------------------------------------------------------------------
# Rigid EM loop (Sec. 3.1 with the rigid kinematics of Sec. 5)
# ---------------------------------------------------------------------------

def build_observation_lattice(obs, obs_n, feat, residual, sigma, sigma_n):
    k = scale_factors(feature_sigmas(feat, sigma, sigma_n))
    lat = lattice_build(features(obs, obs_n, feat), splat_values(obs, obs_n, residual), k)
    return lat


def register_rigid(model, model_n, obs, obs_n, *, feat, residual, sigma, sigma_n=0.5, c=None, w=0.1,
                   iters=20, T0=None, lattice: Optional[Lattice] = None, normalize_n=False,
                   history: Optional[list] = None, twist_tol: Optional[float] = None, info: Optional[dict] = None,
                   timings: Optional[dict] = None):
    """Rigid FilterReg: build the observation lattice once, then up to `iters` EM iterations of
    E-step (slice at the pinned binary32 transform of the model) and one Gauss-Newton step
    T <- Exp(-A^-1 b) T.  With twist_tol, the loop ends after the first step whose rotation and
    translation parts both have norm below it (Sec. 6.1 terminates on a small twist); info, if
    given, receives the number of steps taken; timings, if given, the wall-clock seconds of the
    build ("build") and of each iteration's E-step and M-step ("estep", "mstep" lists).  Returns
    the float64 pose."""
    clock = time.perf_counter
    T = np.eye(4) if T0 is None else np.array(T0, dtype=np.float64)
    if c is None:
        c = outlier_constant(w, len(obs), len(model), feature_sigmas(feat, sigma, sigma_n))
    sig_m = float(np.mean(sigma))
    t0 = clock()
    lat = lattice if lattice is not None else build_observation_lattice(obs, obs_n, feat, residual, sigma, sigma_n)
    if timings is not None:
        timings["build"] = clock() - t0
        timings.setdefault("estep", [])
        timings.setdefault("mstep", [])
    model = np.asarray(model, dtype=np.float32)
    for _ in range(iters):
        t0 = clock()
        mat = pose_to_mat12(T)
        x32 = transform_f32(mat, model)
        n32 = transform_f32(mat, model_n, translate=False) if feat == 6 else None
        m0, m1, ns = estep(lat, x32, n32, feat, residual)
        t1 = clock()
        R32 = mat.reshape(3, 4).astype(np.float64)
        x64 = model.astype(np.float64) @ R32[:, :3].T + R32[:, 3]
        A, b, stats = normal_equations(x64, m0, m1, ns, c, sig_m, residual, normalize_n)
        dz = gn_step(A, b, RIGID_PIVOT_TOL)
        T = se3_exp(dz) @ T
        if timings is not None:
            timings["estep"].append(t1 - t0)
            timings["mstep"].append(clock() - t1)
        if history is not None:
            history.append(dict(A=A, b=b, stats=stats, dz=dz, T=T.copy()))
        if info is not None:
            info["iterations"] = info.get("iterations", 0) + 1
        if twist_tol is not None and np.linalg.norm(dz[:3]) < twist_tol and np.linalg.norm(dz[3:]) < twist_tol:
            break
    return T


def variance_terms(x, m0, m1, m2, c):
    """The two sums of the optimised isotropic variance (Sec. 3.3, sigma as a decision variable, in the
    closed form of the Coherent Point Drift M-step): with the posterior P_ik = K_ik / (M0_i + c) of
    Eq. (4)-(5),
        sum_ik P_ik |x_i - y_k|^2 = sum_i (M0_i |x_i|^2 - 2 x_i . M1_i + M2_i) / (M0_i + c),
        sum_ik P_ik               = sum_i M0_i / (M0_i + c),
    and sigma^2 = first / (3 * second).  Points with M0 = 0 contribute nothing."""
    x = np.asarray(x, dtype=np.float64)
    m0 = np.asarray(m0, dtype=np.float64)
    sup = m0 > 0
    den = np.where(sup, m0 + c, 1.0)
    num = m0 * np.sum(x * x, axis=1) - 2.0 * np.sum(x * np.asarray(m1, dtype=np.float64), axis=1) + \
        np.asarray(m2, dtype=np.float64)
    return float(np.sum(np.where(sup, num / den, 0.0))), float(np.sum(np.where(sup, m0 / den, 0.0)))


# Per-axis variance of the lattice's kernel K(x, y) = sum_v b_v(x) b_v(y) (splat and slice, no blur)
# in units of the lattice scale s squared.  Derivation: the piecewise-linear hat of one lattice vertex
# has, in the lattice's own coordinates (the (d+1)-scaled A*_d lattice), a second moment of trace
# d (d+1)^2 / 12 spread evenly over the d directions; averaged over positions the kernel is the hat's
# autocorrelation over the volume per vertex, whose second moment is twice the hat's, (d+1)^2 / 6 per
# direction; the embedding maps a position offset of length r to (d+1) sqrt(2/3) r / s.  Hence
# (d+1)^2 / 6 * s^2 * 3 / (2 (d+1)^2) = s^2 / 4 for every d.
LATTICE_KERNEL_AXIS_VAR = 0.25


def register_rigid_sigma(model, model_n, obs, obs_n, *, feat, residual, sigma0, sigma_min, sigma_n=0.5, w=0.1,
                         iters=20, T0=None, history: Optional[list] = None):
    """Rigid FilterReg with sigma updated every EM iteration (Sec. 3.3 optimised variance; Tab. 1
    "updated sigma").  sigma is the lattice scale s, as everywhere in this module; the lattice filters
    with a kernel of per-axis variance s^2 / 4 (LATTICE_KERNEL_AXIS_VAR), so the Gaussian of Eq. (5) it
    stands for has variance s^2 / 4.  Each iteration builds the lattice at the current s (the index
    depends on it, Sec. 3.1), takes the E-step at the pose and one Gauss-Newton step; the closed form
    then gives that Gaussian's variance from the same E-step and pose, variance_terms first / (3 second),
    and s^2 <- it / LATTICE_KERNEL_AXIS_VAR, floored at sigma_min.  c of Eq. (7) follows s as in the
    fixed-sigma loop.  Returns (pose, s)."""
    T = np.eye(4) if T0 is None else np.array(T0, dtype=np.float64)
    sig = float(sigma0)
    model = np.asarray(model, dtype=np.float32)
    for _ in range(iters):
        sv = [sig, sig, sig]
        lat = lattice_build(features(obs, obs_n, feat), splat_values(obs, obs_n, residual, m2=True),
                            scale_factors(feature_sigmas(feat, sv, sigma_n)))
        c = outlier_constant(w, len(obs), len(model), feature_sigmas(feat, sv, sigma_n))
        mat = pose_to_mat12(T)
        x32 = transform_f32(mat, model)
        n32 = transform_f32(mat, model_n, translate=False) if feat == 6 else None
        m0, m1, ns, m2 = estep(lat, x32, n32, feat, residual, m2=True)
        R32 = mat.reshape(3, 4).astype(np.float64)
        x64 = model.astype(np.float64) @ R32[:, :3].T + R32[:, 3]
        A, b, stats = normal_equations(x64, m0, m1, ns, c, sig, residual)
        dz = gn_step(A, b, RIGID_PIVOT_TOL)
        T = se3_exp(dz) @ T
        vs, ws = variance_terms(x64, m0, m1, m2, c)
        if ws > 0:
            sig = max(sigma_min, math.sqrt(max(vs / (3.0 * ws), 0.0) / LATTICE_KERNEL_AXIS_VAR))
        if history is not None:
            history.append(dict(A=A, b=b, stats=stats, dz=dz, T=T.copy(), sigma=sig, var=vs, sum_w=ws))
    return T, sig


def register_rigid_blurred(model, model_n, obs, obs_n, *, feat, residual, sigma, sigma_n=0.5, c=None, w=0.1,
                           iters=20, T0=None, history: Optional[list] = None):
    """Rigid EM with the uncustomised filter: every iteration splats the observation together with the
    moved model, blurs and slices (the index depends on X, so it is rebuilt each iteration), then one
    Gauss-Newton step as in register_rigid.  Returns the float64 pose."""
    T = np.eye(4) if T0 is None else np.array(T0, dtype=np.float64)
    if c is None:
        c = outlier_constant(w, len(obs), len(model), feature_sigmas(feat, sigma, sigma_n), blurred=True)
    sig_m = float(np.mean(sigma))
    k = scale_factors(feature_sigmas(feat, sigma, sigma_n))
    model = np.asarray(model, dtype=np.float32)
    for _ in range(iters):
        mat = pose_to_mat12(T)
        x32 = transform_f32(mat, model)
        n32 = transform_f32(mat, model_n, translate=False) if feat == 6 else None
        m0, m1, ns = estep_blurred(obs, obs_n, x32, n32, feat, residual, k)
        R32 = mat.reshape(3, 4).astype(np.float64)
        x64 = model.astype(np.float64) @ R32[:, :3].T + R32[:, 3]
        A, b, stats = normal_equations(x64, m0, m1, ns, c, sig_m, residual)
        dz = gn_step(A, b, RIGID_PIVOT_TOL)
        T = se3_exp(dz) @ T
        if history is not None:
            history.append(dict(A=A, b=b, stats=stats, dz=dz, T=T.copy()))
    return T


def feature_outlier_constant(w: float, n_obs: int, n_model: int, sigma_f: float, dim: int) -> float:
    """c of Eq. (7) for a kernel over `dim` descriptor dimensions of width sigma_f (Eq. 8): the rule of
    outlier_constant with the descriptor lattice's kernel mass."""
    return outlier_constant(w, n_obs, n_model, np.full(dim, float(sigma_f)))


def feature_lattice(obs, obs_feat, sigma_f: float) -> Lattice:
    """The observation's lattice over descriptor space (Eq. 8), values [1, y]."""
    f = np.ascontiguousarray(obs_feat, dtype=np.float32)
    k = scale_factors(np.full(f.shape[1], float(sigma_f)))
    return lattice_build(f, splat_values(obs, None, "pt2pt"), k)


def register_rigid_features(model, model_feat, obs, obs_feat, *, sigma_f, w=0.2, c=None, iters=20, T0=None,
                            history: Optional[list] = None):
    """Rigid registration by descriptors (Sec. 3.3 "Features", Eq. 8 with the features alone): the
    kernel does not involve the pose, so one E-step gives fixed targets M1/M0 and weights, and the
    EM iterations are Gauss-Newton steps of Eq. (17) toward them (point-to-point, unit residual
    scale).  Returns the float64 pose."""
    T = np.eye(4) if T0 is None else np.array(T0, dtype=np.float64)
    dim = np.asarray(model_feat).shape[1]
    if c is None:
        c = feature_outlier_constant(w, len(obs), len(model), sigma_f, dim)
    lat = feature_lattice(obs, obs_feat, sigma_f)
    g = lattice_slice(lat, np.ascontiguousarray(model_feat, dtype=np.float32))
    m0, m1 = g[:, 0].copy(), g[:, 1:4].copy()
    model = np.asarray(model, dtype=np.float32)
    for _ in range(iters):
        mat = pose_to_mat12(T)
        R32 = mat.reshape(3, 4).astype(np.float64)
        x64 = model.astype(np.float64) @ R32[:, :3].T + R32[:, 3]
        A, b, stats = normal_equations(x64, m0, m1, None, c, 1.0, "pt2pt")
        dz = gn_step(A, b, RIGID_PIVOT_TOL)
        T = se3_exp(dz) @ T
        if history is not None:
            history.append(dict(A=A, b=b, stats=stats, dz=dz, T=T.copy(), m0=m0, m1=m1))
    return T


def alignment_error(T, T_gt, x_ref) -> float:
    """Eq. (22): mean over reference points of |(T - T_gt) x|_2."""
    x = np.asarray(x_ref, dtype=np.float64)
    D = np.asarray(T) - np.asarray(T_gt)
    return float(np.mean(np.linalg.norm(x @ D[:3, :3].T + D[:3, 3], axis=1)))


def rotation_angle(R: np.ndarray) -> float:
    c = (np.trace(R) - 1.0) / 2.0
    return float(math.acos(max(-1.0, min(1.0, c))))
