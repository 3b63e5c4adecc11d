"""Seeded synthetic workloads for registration pairs.

This module only makes inputs: point clouds, normals, ground-truth motions and
request streams.  It holds none of the registration arithmetic (no lattice, no
E-step, no M-step, no solver).  Both the CPU oracle tests and the GPU tests
draw their inputs from here, so the two sides always see identical float32
arrays.

The paper measures on datasets that are not available here (Stanford bunny,
Stanford Lounge, robot RGBD, a DynamicFusion sequence; Sec. 6).  The
generators below stand in for them with clouds of the same structure:

* ``ellipsoid_pair``  -- rigid point-to-point, 2k points on an ellipsoid plus
  10% uniform outliers (stands in for the bunny robustness test, Sec. 6.1).
* ``depth_pair``      -- rigid point-to-plane, a 640x480 pinhole depth render of
  3 planes + 5 spheres (stands in for RGBD frame-to-frame tracking, Sec. 6.2).
* ``articulated_pair``-- 20 capsule links, 32 revolute DOF (Sec. 5.1 / 6.4).
* ``nodegraph_pair``  -- a displaced-sphere blob skinned to 512 nodes
  (Sec. 5.2 / 6.5).
* ``feature_pair``    -- an object cloud with smooth unit-norm descriptors of
  dimension 8-32, seen from an arbitrary pose with occlusion, noise and
  background clutter (stands in for the learned-feature global registration
  of Sec. 6.3, Tab. 2).
* ``request_stream``  -- Poisson arrivals of depth pairs with log-uniform sizes.

All arrays are row-major ``(n, 3)`` float32 unless stated; poses are 4x4
float64.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np
from scipy.spatial.transform import Rotation

__all__ = [
    "Pair",
    "ellipsoid_pair",
    "depth_pair",
    "random_cloud_pair",
    "separated_pair",
    "articulated_pair",
    "nodegraph_pair",
    "feature_pair",
    "KinTree",
    "random_motion",
    "request_stream",
]


@dataclasses.dataclass
class Pair:
    """One registration problem: move ``model`` onto ``obs``.

    ``model``/``model_n``: reference positions / normals of the model X (M, 3).
    ``obs``/``obs_n``:     observation Y positions / normals (N, 3).
    ``T_gt``:              4x4 motion with ``T_gt @ model ~= obs``.
    ``sigma``:             per-axis kernel width of the position feature.
    ``sigma_n``:           kernel width of the normal feature (d = 6 lifting).
    ``feat``:              3 (position) or 6 (position + normal).
    ``residual``:          "pt2pt" or "pt2pl".
    ``iters``:             fixed EM iteration count of the workload.
    ``w``:                 outlier ratio used for the outlier constant c.
    """

    model: np.ndarray
    obs: np.ndarray
    T_gt: np.ndarray
    sigma: tuple
    feat: int
    residual: str
    iters: int
    model_n: Optional[np.ndarray] = None
    obs_n: Optional[np.ndarray] = None
    sigma_n: float = 0.5
    w: float = 0.1
    name: str = ""
    extra: dict = dataclasses.field(default_factory=dict)


def _f32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


def random_motion(rng, max_angle_rad, max_trans, exact_angle=None):
    """Rotation with a uniform axis on S^2 and an angle U[0, max]; translation U[-t, t]^3."""
    axis = rng.normal(size=3)
    axis /= np.linalg.norm(axis)
    ang = rng.uniform(0.0, max_angle_rad) if exact_angle is None else exact_angle
    T = np.eye(4)
    T[:3, :3] = Rotation.from_rotvec(axis * ang).as_matrix()
    T[:3, 3] = rng.uniform(-max_trans, max_trans, size=3)
    return T


def _apply(T, p):
    return p @ T[:3, :3].T + T[:3, 3]


# ---------------------------------------------------------------------------
# Rigid point-to-point: ellipsoid + outliers
# ---------------------------------------------------------------------------

def _ellipsoid_surface(rng, axes, m):
    """Uniform-by-area samples on an ellipsoid (rejection from the unit sphere).

    The map u -> diag(axes) u scales the sphere's area element by
    sqrt((bc ux)^2 + (ac uy)^2 + (ab uz)^2); accept with that factor / its max.
    """
    a, b, c = axes
    gmax = max(b * c, a * c, a * b)
    out = []
    have = 0
    while have < m:
        u = rng.normal(size=(2 * m, 3))
        u /= np.linalg.norm(u, axis=1, keepdims=True)
        g = np.sqrt((b * c * u[:, 0]) ** 2 + (a * c * u[:, 1]) ** 2 + (a * b * u[:, 2]) ** 2)
        keep = u[rng.uniform(size=len(u)) < g / gmax]
        out.append(keep)
        have += len(keep)
    u = np.concatenate(out)[:m]
    p = u * np.asarray(axes)
    n = p / np.asarray(axes) ** 2
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    return p, n


def ellipsoid_pair(seed: int, m: int = 2000, outlier_frac: float = 0.1, noise: float = 0.005,
                   max_angle_deg: float = 30.0, max_trans: float = 0.1, sigma: float = 0.02,
                   iters: int = 30) -> Pair:
    """Rigid point-to-point workload: ``m`` points on a random ellipsoid.

    Semi-axes U[0.5, 1]; observation = model under a random motion (axis
    uniform, angle U[0, 30 deg], translation U[-0.1, 0.1]^3) with Gaussian noise
    ``noise`` plus ``outlier_frac * m`` uniform outliers in the observation's
    bounding box.  Filter sigma 0.02, 30 EM iterations.
    """
    rng = np.random.default_rng(seed)
    axes = rng.uniform(0.5, 1.0, size=3)
    x, xn = _ellipsoid_surface(rng, axes, m)
    T = random_motion(rng, math.radians(max_angle_deg), max_trans)
    y = _apply(T, x) + rng.normal(scale=noise, size=x.shape)
    yn = xn @ T[:3, :3].T
    n_out = int(round(outlier_frac * m))
    lo, hi = y.min(0), y.max(0)
    yo = rng.uniform(lo, hi, size=(n_out, 3))
    on = rng.normal(size=(n_out, 3))
    on /= np.linalg.norm(on, axis=1, keepdims=True)
    return Pair(model=_f32(x), obs=_f32(np.concatenate([y, yo])), T_gt=T,
                sigma=(sigma, sigma, sigma), feat=3, residual="pt2pt", iters=iters,
                model_n=_f32(xn), obs_n=_f32(np.concatenate([yn, on])), w=outlier_frac,
                name=f"ellipsoid-{m}-seed{seed}")


# ---------------------------------------------------------------------------
# Rigid point-to-plane: pinhole depth render of planes + spheres
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class _Scene:
    planes: list      # (normal (3,), offset o with n.p = o, lo (3,), hi (3,))
    spheres: list     # (center (3,), radius)


def _make_scene(rng) -> _Scene:
    """Room corner (floor, back wall, left wall) and 5 spheres at 1-4 m depth."""
    planes = [
        (np.array([0.0, -1.0, 0.0]), -1.0, np.array([-2.6, 0.99, 0.3]), np.array([2.6, 1.01, 4.6])),   # floor y = 1
        (np.array([0.0, 0.0, -1.0]), -4.6, np.array([-2.6, -1.6, 4.59]), np.array([2.45, 1.01, 4.61])), # back wall z = 4.6
        (np.array([1.0, 0.0, 0.0]), -2.6, np.array([-2.61, -1.6, 0.3]), np.array([-2.59, 1.01, 4.6])), # left wall x = -2.6
    ]
    spheres = []
    for _ in range(5):
        z = rng.uniform(1.0, 4.0)
        r = rng.uniform(0.1, 0.3)
        x = rng.uniform(-0.45, 0.45) * z
        y = rng.uniform(-0.3, 0.3) * z
        spheres.append((np.array([x, min(y, 1.0 - r)]).tolist() + [z], r))
    spheres = [(np.asarray(c, dtype=np.float64), r) for c, r in spheres]
    return _Scene(planes, spheres)


def _render(scene: _Scene, width: int, height: int, f: float, cx: float, cy: float, T_scene=None):
    """Ray-cast the scene (optionally moved by ``T_scene``) from a camera at the origin.

    Returns per-hit camera-frame points (z = depth), unit normals facing the
    camera, and the ray directions (z = 1) of the hit pixels.
    """
    u, v = np.meshgrid(np.arange(width, dtype=np.float64), np.arange(height, dtype=np.float64))
    d = np.stack([(u - cx) / f, (v - cy) / f, np.ones_like(u)], axis=-1).reshape(-1, 3)
    if T_scene is None:
        R = np.eye(3)
        t = np.zeros(3)
    else:
        R, t = T_scene[:3, :3], T_scene[:3, 3]
    # Moving the scene by T equals moving the camera by T^-1: cast rays o' + s d' in scene frame.
    o = -R.T @ t
    ds = d @ R                      # rows: R^T d
    best = np.full(len(d), np.inf)
    nrm = np.zeros((len(d), 3))
    for n, off, lo, hi in scene.planes:
        den = ds @ n
        with np.errstate(divide="ignore", invalid="ignore"):
            s = (off - o @ n) / den
            p = o + s[:, None] * ds
        ok = (s > 1e-6) & np.all((p >= lo) & (p <= hi), axis=1) & (s < best)
        best = np.where(ok, s, best)
        nrm[ok] = n
    for c, r in scene.spheres:
        oc = o - c
        a = np.einsum("ij,ij->i", ds, ds)
        b = 2.0 * ds @ oc
        cc = oc @ oc - r * r
        disc = b * b - 4 * a * cc
        hit = disc > 0
        sq = np.sqrt(np.where(hit, disc, 0.0))
        s = (-b - sq) / (2 * a)
        ok = hit & (s > 1e-6) & (s < best)
        p = o + s[:, None] * ds
        nn = (p - c) / r
        best = np.where(ok, s, best)
        nrm[ok] = nn[ok]
    hit = np.isfinite(best) & (best < 6.0)
    s = best[hit]
    n_cam = nrm[hit] @ R.T
    dd = d[hit]
    # Orient normals toward the camera.
    flip = np.einsum("ij,ij->i", n_cam, dd) > 0
    n_cam[flip] *= -1.0
    return s, dd, n_cam


def depth_pair(seed: int, width: int = 640, height: int = 480, f: float = 525.0,
               max_angle_deg: float = 10.0, max_trans: float = 0.05, depth_noise: float = 0.002,
               dropout: float = 0.05, sigma: float = 0.03, sigma_n: float = 0.5, feat: int = 6,
               iters: int = 20, target_points: Optional[int] = None) -> Pair:
    """Rigid point-to-plane workload: a pinhole depth render of 3 planes + 5 spheres.

    Model = noise-free render of the scene (camera frame, analytic normals).
    Observation = render of the scene after a random rigid motion (<= 10 deg,
    <= 0.05 m per axis), depth noise ``depth_noise`` along each ray and
    ``dropout`` of the pixels removed.  ``target_points`` rescales focal length
    and resolution by sqrt(target / 250k) and subsamples the model to exactly
    ``target_points`` (request streams of uneven size).
    """
    rng = np.random.default_rng(seed)
    scene = _make_scene(rng)
    T = random_motion(rng, math.radians(max_angle_deg), max_trans)
    if target_points is not None:
        scale = math.sqrt(max(target_points, 16) / 250_000.0) * 1.02
        width = max(8, int(round(width * scale)))
        height = max(6, int(round(height * scale)))
        f = f * scale
    cx, cy = (width - 1) / 2.0, (height - 1) / 2.0
    s, d, n = _render(scene, width, height, f, cx, cy)
    x = s[:, None] * d
    so, do, no = _render(scene, width, height, f, cx, cy, T_scene=T)
    so = so + rng.normal(scale=depth_noise, size=so.shape)
    keep = rng.uniform(size=len(so)) >= dropout
    y = (so[:, None] * do)[keep]
    yn = no[keep]
    if target_points is not None:
        if len(x) > target_points:
            idx = np.sort(rng.choice(len(x), size=target_points, replace=False))
            x, n = x[idx], n[idx]
        ny = int(round(target_points * len(y) / max(1, len(s))))
        if 0 < ny < len(y):
            idy = np.sort(rng.choice(len(y), size=ny, replace=False))
            y, yn = y[idy], yn[idy]
    return Pair(model=_f32(x), obs=_f32(y), T_gt=T, sigma=(sigma, sigma, sigma), feat=feat,
                residual="pt2pl", iters=iters, model_n=_f32(n), obs_n=_f32(yn), sigma_n=sigma_n,
                w=0.1, name=f"depth-{len(x)}-seed{seed}")


# ---------------------------------------------------------------------------
# Generic small clouds for parity tests
# ---------------------------------------------------------------------------

def random_cloud_pair(seed: int, m: int, n: int, extent: float = 0.3, sigma: float = 0.02,
                      feat: int = 3, residual: str = "pt2pt", surface: bool = True,
                      max_angle_deg: float = 5.0, max_trans: float = 0.01) -> Pair:
    """Small pair on a wavy surface patch (or a uniform blob) with unit normals.

    Used for parity and edge-case tests: sizes are free, values are bounded by
    ``extent``, and the motion is small so most model points have support.
    """
    rng = np.random.default_rng(seed)

    def sample(k):
        if surface:
            uv = rng.uniform(-extent, extent, size=(k, 2))
            h = 0.15 * extent * np.sin(3.0 * uv[:, 0] / extent) * np.cos(2.0 * uv[:, 1] / extent)
            p = np.column_stack([uv, h])
            gx = 0.15 * 3.0 * np.cos(3.0 * uv[:, 0] / extent) * np.cos(2.0 * uv[:, 1] / extent)
            gy = -0.15 * 2.0 * np.sin(3.0 * uv[:, 0] / extent) * np.sin(2.0 * uv[:, 1] / extent)
            nn = np.column_stack([-gx, -gy, np.ones(k)])
        else:
            p = rng.uniform(-extent, extent, size=(k, 3))
            nn = rng.normal(size=(k, 3))
        nn /= np.linalg.norm(nn, axis=1, keepdims=True)
        return p, nn

    x, xn = sample(m)
    T = random_motion(rng, math.radians(max_angle_deg), max_trans)
    yb, ybn = sample(n)
    y = _apply(T, yb)
    yn = ybn @ T[:3, :3].T
    return Pair(model=_f32(x), obs=_f32(y), T_gt=T, sigma=(sigma, sigma, sigma), feat=feat,
                residual=residual, iters=10, model_n=_f32(xn), obs_n=_f32(yn), w=0.1,
                name=f"cloud-{m}x{n}-seed{seed}")


def separated_pair(seed: int, m: int = 400, sigma: float = 0.02, spacing: float = 4.0, feat: int = 3,
                   residual: str = "pt2pt", start_disp: float = 0.4) -> Pair:
    """Noise-free pair whose points are at least ``spacing - 0.4`` sigma apart.

    Points are a random subset of a grid of pitch ``spacing * sigma`` jittered by
    +-0.2 sigma; normals are random unit vectors; observation = ``T_gt`` applied
    exactly (no noise, no outliers).  ``extra["T0"]`` is a start pose that
    displaces every model point by at most ``start_disp * sigma`` from its
    ground-truth position.
    """
    rng = np.random.default_rng(seed)
    side = int(math.ceil(m ** (1.0 / 3.0))) + 2
    g = np.stack(np.meshgrid(*[np.arange(side)] * 3, indexing="ij"), -1).reshape(-1, 3).astype(np.float64)
    g = g[rng.choice(len(g), size=m, replace=False)]
    x = (g - side / 2.0) * spacing * sigma + rng.uniform(-0.2, 0.2, size=(m, 3)) * sigma
    xn = rng.normal(size=(m, 3))
    xn /= np.linalg.norm(xn, axis=1, keepdims=True)
    T = random_motion(rng, math.radians(20.0), 0.05)
    y = _apply(T, x)
    yn = xn @ T[:3, :3].T
    # start pose: T_gt composed with a small motion about the cloud centre
    radius = float(np.linalg.norm(x - x.mean(0), axis=1).max())
    budget = start_disp * sigma
    ang = 0.5 * budget / max(radius, 1e-9)
    P = random_motion(rng, 0.0, 0.0, exact_angle=ang)
    dirv = rng.normal(size=3)
    P[:3, 3] = 0.5 * budget * dirv / np.linalg.norm(dirv)
    c = x.mean(0)
    P[:3, 3] += c - P[:3, :3] @ c
    T0 = T @ P
    return Pair(model=_f32(x), obs=_f32(y), T_gt=T, sigma=(sigma, sigma, sigma), feat=feat,
                residual=residual, iters=15, model_n=_f32(xn), obs_n=_f32(yn), w=0.0,
                name=f"separated-{m}-seed{seed}", extra={"T0": T0})


# ---------------------------------------------------------------------------
# Feature registration: motion-invariant descriptors
# ---------------------------------------------------------------------------

def feature_pair(seed: int, m: int = 12000, dim: int = 16, sigma_f: float = 0.05, omega: float = 10.0,
                 noise: float = 0.002, feat_noise: float = 0.005, keep: float = 0.7, clutter: float = 0.3,
                 max_angle_deg: float = 180.0, max_trans: float = 0.3) -> Pair:
    """Global registration by descriptors (Eq. 8 with features only; Tab. 2 stand-in).

    Model: ``m`` points on an ellipsoid with semi-axes U[0.05, 0.15] m.  Each point carries the
    unit-norm descriptor f(p) = normalise(cos(W p + c)) of its model-frame position (W ~ N(0,
    omega^2) of shape (dim, 3), c ~ U[0, 2 pi)), so nearby points have nearby descriptors and the
    descriptor does not depend on the pose.  Observation: the ``keep`` fraction of model points
    facing a random view direction, moved by a random motion (rotation angle U[0, max_angle_deg],
    uniform axis; translation U[-max_trans, max_trans]^3), with position noise ``noise`` and
    descriptor noise ``feat_noise`` (renormalised), plus ``clutter`` * (kept points) background
    points uniform in the box around the object carrying random unit descriptors.
    ``extra``: model_feat (M, dim), obs_feat (N, dim) float32, dim, sigma_f.
    """
    rng = np.random.default_rng(seed)
    axes = rng.uniform(0.05, 0.15, size=3)
    x, xn = _ellipsoid_surface(rng, axes, m)
    W = rng.normal(scale=omega, size=(dim, 3))
    c = rng.uniform(0.0, 2.0 * math.pi, size=dim)

    def desc(p):
        f = np.cos(p @ W.T + c)
        return f / np.linalg.norm(f, axis=1, keepdims=True)

    fx = desc(x)
    view = rng.normal(size=3)
    view /= np.linalg.norm(view)
    order = np.argsort(-(xn @ view))
    vis = np.sort(order[: int(round(keep * m))])
    T = random_motion(rng, math.radians(max_angle_deg), max_trans)
    y = _apply(T, x[vis]) + rng.normal(scale=noise, size=(len(vis), 3))
    fy = fx[vis] + rng.normal(scale=feat_noise, size=(len(vis), dim))
    fy /= np.linalg.norm(fy, axis=1, keepdims=True)
    n_bg = int(round(clutter * len(vis)))
    lo, hi = y.min(0) - 0.1, y.max(0) + 0.1
    yb = rng.uniform(lo, hi, size=(n_bg, 3))
    fb = rng.normal(size=(n_bg, dim))
    fb /= np.linalg.norm(fb, axis=1, keepdims=True)
    return Pair(model=_f32(x), obs=_f32(np.concatenate([y, yb])), T_gt=T, sigma=(0.01, 0.01, 0.01), feat=dim,
                residual="pt2pt", iters=20, model_n=_f32(xn), w=clutter / (1.0 + clutter),
                name=f"feature-{dim}-{m}-seed{seed}",
                extra={"model_feat": _f32(fx), "obs_feat": _f32(np.concatenate([fy, fb])), "dim": dim,
                       "sigma_f": sigma_f})


# ---------------------------------------------------------------------------
# Articulated: a tree of capsule links with revolute joints
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class KinTree:
    """Kinematic tree: parent[b] < b (-1 = world); body b owns DOFs [dof_offset[b], dof_offset[b+1]);
    joint origin origin[b] in the parent frame; axis[k] in the frame left by the preceding rotations."""
    parent: np.ndarray
    dof_offset: np.ndarray
    origin: np.ndarray
    axis: np.ndarray


def _pose_bodies(tree: KinTree, theta):
    """Body frames for joint angles theta (independent posing code for generating observations)."""
    B = len(tree.parent)
    Rs, ts = [None] * B, [None] * B
    for b in range(B):
        if tree.parent[b] < 0:
            Rp, tp = np.eye(3), np.zeros(3)
        else:
            Rp, tp = Rs[tree.parent[b]], ts[tree.parent[b]]
        t = Rp @ tree.origin[b] + tp
        R = Rp
        for k in range(tree.dof_offset[b], tree.dof_offset[b + 1]):
            R = R @ Rotation.from_rotvec(tree.axis[k] * theta[k]).as_matrix()
        Rs[b], ts[b] = R, t
    return Rs, ts


def _capsule_points(rng, length, radius, n):
    """Uniform-by-area samples on a capsule along +x from the origin, with outward normals."""
    a_cyl = 2 * math.pi * radius * length
    a_cap = 4 * math.pi * radius ** 2
    n_cyl = rng.binomial(n, a_cyl / (a_cyl + a_cap))
    u = rng.uniform(0, length, n_cyl)
    phi = rng.uniform(0, 2 * math.pi, n_cyl)
    nc = np.column_stack([np.zeros(n_cyl), np.cos(phi), np.sin(phi)])
    pc = np.column_stack([u, np.zeros(n_cyl), np.zeros(n_cyl)]) + radius * nc
    m = n - n_cyl
    d = rng.normal(size=(m, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    centre = np.where(d[:, :1] >= 0, length, 0.0) * np.array([[1.0, 0.0, 0.0]])
    ps = centre + radius * d
    return np.concatenate([pc, ps]), np.concatenate([nc, d])


def articulated_pair(seed: int, n_bodies: int = 20, n_dof: int = 32, m: int = 60_000, noise: float = 0.003,
                     occlusion: float = 0.15, sigma: float = 0.01, sigma_n: float = 0.5, iters: int = 15,
                     max_angle: float = 0.5, start_perturb: float = 0.03) -> Pair:
    """Articulated workload: capsule links (length U[0.05, 0.15], radius U[0.015, 0.03], axis along
    the body's x) in a random tree, 1-3 revolute DOFs per joint summing to ``n_dof``, joint angles
    U[-0.5, 0.5]; observation = posed model + Gaussian noise, minus the ``occlusion`` fraction of
    points with the largest projection on a random direction.  ``extra`` holds the tree, the
    per-body point offsets, theta_gt and the start theta0 = theta_gt + U[-start_perturb, start_perturb].

    A capsule is symmetric about its own axis, so a spin about that axis is seen only through the
    bodies hanging from it.  Joint axes are chosen so that every DOF moves some surface: one or two
    DOFs turn about orthogonal axes across the link (in its y-z plane); a third DOF, the spin about
    the link axis, is given only to bodies with children, and children hang off-axis from the end
    of their parent."""
    rng = np.random.default_rng(seed)
    parent = np.array([-1] + [int(rng.integers(0, b)) for b in range(1, n_bodies)])
    has_child = np.zeros(n_bodies, bool)
    has_child[parent[parent >= 0]] = True
    dofs = np.ones(n_bodies, dtype=np.int64)
    if n_dof > int(np.where(has_child, 3, 2).sum()):
        raise ValueError("too many DOFs for this tree")
    while dofs.sum() < n_dof:
        b = int(rng.integers(0, n_bodies))
        if dofs[b] < (3 if has_child[b] else 2):
            dofs[b] += 1
    dof_offset = np.concatenate([[0], np.cumsum(dofs)])
    lengths = rng.uniform(0.05, 0.15, n_bodies)
    radii = rng.uniform(0.015, 0.03, n_bodies)
    origin = np.zeros((n_bodies, 3))
    for b in range(1, n_bodies):
        phi = rng.uniform(0, 2 * math.pi)
        r = 0.7 * radii[parent[b]]
        origin[b] = [lengths[parent[b]], r * math.cos(phi), r * math.sin(phi)]
    axis = np.zeros((n_dof, 3))
    for b in range(n_bodies):
        k0, nb = dof_offset[b], dofs[b]
        phi = rng.uniform(0, 2 * math.pi)
        across = [np.array([0.0, math.cos(phi), math.sin(phi)]), np.array([0.0, -math.sin(phi), math.cos(phi)])]
        seq = across[:nb] if nb <= 2 else [np.array([1.0, 0.0, 0.0])] + across
        for j, a in enumerate(seq):
            axis[k0 + j] = a
    tree = KinTree(parent, dof_offset, origin, axis)
    area = 2 * math.pi * radii * lengths + 4 * math.pi * radii ** 2
    counts = rng.multinomial(m, area / area.sum())
    pts, nrm = [], []
    for b in range(n_bodies):
        p, n = _capsule_points(rng, lengths[b], radii[b], int(counts[b]))
        pts.append(p)
        nrm.append(n)
    body_offsets = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    x_ref = np.concatenate(pts)
    n_ref = np.concatenate(nrm)
    theta_gt = rng.uniform(-max_angle, max_angle, n_dof)
    Rs, ts = _pose_bodies(tree, theta_gt)
    y = np.zeros_like(x_ref)
    yn = np.zeros_like(n_ref)
    for b in range(n_bodies):
        sl = slice(body_offsets[b], body_offsets[b + 1])
        y[sl] = x_ref[sl] @ Rs[b].T + ts[b]
        yn[sl] = n_ref[sl] @ Rs[b].T
    y = y + rng.normal(scale=noise, size=y.shape)
    direction = rng.normal(size=3)
    proj = y @ direction
    keep = proj <= np.quantile(proj, 1.0 - occlusion) if occlusion > 0 else np.ones(len(y), bool)
    theta0 = theta_gt + rng.uniform(-start_perturb, start_perturb, n_dof)
    return Pair(model=_f32(x_ref), obs=_f32(y[keep]), T_gt=np.eye(4), sigma=(sigma, sigma, sigma), feat=6,
                residual="pt2pl", iters=iters, model_n=_f32(n_ref), obs_n=_f32(yn[keep]), sigma_n=sigma_n, w=0.1,
                name=f"articulated-{m}-seed{seed}",
                extra={"tree": tree, "body_offsets": body_offsets, "theta_gt": theta_gt, "theta0": theta0})


# ---------------------------------------------------------------------------
# Node graph: a displaced-sphere blob skinned to farthest-point-sampled nodes
# ---------------------------------------------------------------------------

def _farthest_points(rng, pts, k):
    idx = np.zeros(k, dtype=np.int64)
    idx[0] = int(rng.integers(0, len(pts)))
    d = np.linalg.norm(pts - pts[idx[0]], axis=1)
    for i in range(1, k):
        idx[i] = int(np.argmax(d))
        d = np.minimum(d, np.linalg.norm(pts - pts[idx[i]], axis=1))
    return idx


def _dq_blend(node_R, node_t, skin_idx, skin_w):
    """Dual-quaternion blended rotation matrices and translations (generator's own implementation)."""
    q = Rotation.from_matrix(node_R).as_quat()             # (K, 4) x, y, z, w
    qr = np.concatenate([q[:, 3:], q[:, :3]], 1)            # w, x, y, z
    tq = np.concatenate([np.zeros((len(node_t), 1)), node_t], 1)

    def mul(a, b):
        return np.stack([a[..., 0] * b[..., 0] - np.sum(a[..., 1:] * b[..., 1:], -1),
                         *(a[..., :1] * b[..., 1:] + b[..., :1] * a[..., 1:] + np.cross(a[..., 1:], b[..., 1:])).T], -1) \
            if a.ndim == 1 else np.concatenate(
                [(a[..., 0] * b[..., 0] - np.sum(a[..., 1:] * b[..., 1:], -1))[..., None],
                 a[..., :1] * b[..., 1:] + b[..., :1] * a[..., 1:] + np.cross(a[..., 1:], b[..., 1:])], -1)

    qd = 0.5 * mul(tq, qr)
    ref = qr[skin_idx[:, 0]]
    sgn = np.where(np.einsum("ij,ikj->ik", ref, qr[skin_idx]) >= 0, 1.0, -1.0)
    ww = skin_w * sgn
    br = np.einsum("ik,ikj->ij", ww, qr[skin_idx])
    bd = np.einsum("ik,ikj->ij", ww, qd[skin_idx])
    nrm = np.linalg.norm(br, axis=1, keepdims=True)
    br, bd = br / nrm, bd / nrm
    R = Rotation.from_quat(np.concatenate([br[:, 1:], br[:, :1]], 1)).as_matrix()
    conj = br * np.array([1.0, -1.0, -1.0, -1.0])
    t = 2.0 * mul(bd, conj)[:, 1:]
    return R, t


def nodegraph_pair(seed: int, m: int = 100_000, n_nodes: int = 512, noise: float = 0.003, sigma: float = 0.02,
                   max_angle_deg: float = 5.0, max_trans: float = 0.02, iters: int = 20, n_edges: int = 8,
                   rigid: bool = False) -> Pair:
    """Node-graph workload: ``m`` points on a sphere displaced by low-frequency noise, ``n_nodes``
    nodes by farthest-point sampling, each point skinned to its 4 nearest nodes with weights
    exp(-d^2 / (2 r^2)) (r = mean nearest-node spacing), ground-truth node motions from a smooth
    random twist field (<= 5 deg, <= 0.02), observation = blended model + noise.
    ``extra``: nodes, skin_idx, skin_w, edges (8-NN, directed), node_R/node_t ground truth."""
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(seed)
    u = rng.normal(size=(m, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    freqs = rng.normal(size=(6, 3)) * 1.5
    phases = rng.uniform(0, 2 * math.pi, 6)
    amps = rng.uniform(0.03, 0.08, 6)
    radius = 1.0 + np.sum(amps[None] * np.sin(u @ freqs.T + phases[None]), 1)
    x = u * radius[:, None]
    # normals from the radial function by finite differences on the sphere
    eps = 1e-4
    def surf(v):
        v = v / np.linalg.norm(v, axis=1, keepdims=True)
        return v * (1.0 + np.sum(amps[None] * np.sin(v @ freqs.T + phases[None]), 1))[:, None]
    a = np.cross(u, np.where(np.abs(u[:, :1]) < 0.9, [[1.0, 0, 0]], [[0, 1.0, 0]]))
    a /= np.linalg.norm(a, axis=1, keepdims=True)
    bvec = np.cross(u, a)
    n = np.cross(surf(u + eps * a) - surf(u - eps * a), surf(u + eps * bvec) - surf(u - eps * bvec))
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    n *= np.sign(np.sum(n * u, 1, keepdims=True))
    nodes = x[_farthest_points(rng, x, n_nodes)]
    tree = cKDTree(nodes)
    dn, _ = tree.query(nodes, k=2)
    r = float(np.mean(dn[:, 1]))
    d4, i4 = tree.query(x, k=4)
    w4 = np.exp(-d4 ** 2 / (2 * r * r))
    w4 /= w4.sum(1, keepdims=True)
    _, ie = tree.query(nodes, k=n_edges + 1)
    edges = np.array([(j, k) for j in range(n_nodes) for k in ie[j, 1:]], dtype=np.int64)
    if rigid:
        T = random_motion(rng, math.radians(max_angle_deg), max_trans)
        node_R = np.repeat(T[:3, :3][None], n_nodes, 0)
        node_t = np.repeat(T[:3, 3][None], n_nodes, 0)
    else:
        fw = rng.normal(size=(3, 3)) * 1.2
        fv = rng.normal(size=(3, 3)) * 1.2
        pw = rng.uniform(0, 2 * math.pi, 3)
        pv = rng.uniform(0, 2 * math.pi, 3)
        wfield = np.sin(nodes @ fw.T + pw)
        vfield = np.sin(nodes @ fv.T + pv)
        wfield *= math.radians(max_angle_deg) / np.max(np.linalg.norm(wfield, axis=1))
        vfield *= max_trans / np.max(np.abs(vfield))
        node_R = Rotation.from_rotvec(wfield).as_matrix()
        node_t = vfield
    R, t = _dq_blend(node_R, node_t, i4, w4)
    y = np.einsum("ijk,ik->ij", R, x) + t + rng.normal(scale=noise, size=x.shape)
    yn = np.einsum("ijk,ik->ij", R, n)
    return Pair(model=_f32(x), obs=_f32(y), T_gt=np.eye(4), sigma=(sigma, sigma, sigma), feat=3, residual="pt2pt",
                iters=iters, model_n=_f32(n), obs_n=_f32(yn), w=0.1, name=f"nodegraph-{m}-seed{seed}",
                extra={"nodes": nodes, "skin_idx": i4.astype(np.int32), "skin_w": w4, "edges": edges,
                       "node_R": node_R, "node_t": node_t, "spacing": r})


# ---------------------------------------------------------------------------
# Request stream (served batch)
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Request:
    rid: int
    arrival_s: float
    size: int
    seed: int


def request_stream(seed: int, n_requests: int = 4096, lo: int = 1000, hi: int = 300_000,
                   rate_per_s: float = 100.0):
    """Poisson arrivals (exponential gaps, ``rate_per_s``) of log-uniform sizes in [lo, hi]."""
    rng = np.random.default_rng(seed)
    sizes = np.exp(rng.uniform(math.log(lo), math.log(hi), size=n_requests)).astype(np.int64)
    gaps = rng.exponential(1.0 / rate_per_s, size=n_requests)
    t = np.cumsum(gaps) - gaps[0]
    seeds = rng.integers(0, 2**31 - 1, size=n_requests)
    return [Request(i, float(t[i]), int(sizes[i]), int(seeds[i])) for i in range(n_requests)]
