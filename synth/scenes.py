"""Seeded synthetic scenes and cameras for the Gaussian-enhanced-surfel render.

This module only draws random numbers and places cameras.  It holds none of
the rendering arithmetic, so both the FP64 oracle and the HIP path can take
their inputs from it without sharing any of the method.

Representation (paper Sec. 3 and the pipeline figure): a surfel set
S = {p, r, s in R^2, SH} and a Gaussian set G = {p, sigma, r, s in R^3, SH}.
All arrays are structure-of-arrays float32, primitive index fastest:

  surfels:   mean [3][N], quat [4][N] (w,x,y,z), scale [2][N], sh [K][3][N]
  gaussians: mean [3][M], quat [4][M], scale [3][M], opacity [M], sh [K][3][M]

with K = (deg+1)^2 spherical-harmonic coefficients per colour channel.

Cameras are pinhole, world->camera (R, t) with OpenCV axes (x right, y down,
z forward); the pixel (i, j) centre is at (i + 0.5, j + 0.5).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

SH_DEGREE = 3
SH_K = (SH_DEGREE + 1) ** 2
BASE_SEED = 17545


@dataclasses.dataclass
class Surfels:
    mean: np.ndarray   # [3][N]
    quat: np.ndarray   # [4][N]
    scale: np.ndarray  # [2][N]
    sh: np.ndarray     # [K][3][N]

    @property
    def n(self) -> int:
        return int(self.mean.shape[1])


@dataclasses.dataclass
class Gaussians:
    mean: np.ndarray     # [3][M]
    quat: np.ndarray     # [4][M]
    scale: np.ndarray    # [3][M]
    opacity: np.ndarray  # [M]
    sh: np.ndarray       # [K][3][M]
    filter3d: Optional[np.ndarray] = None  # [M] variance of a 3D low-pass filter (Mip-GES), or None

    @property
    def m(self) -> int:
        return int(self.mean.shape[1])


@dataclasses.dataclass
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    R: np.ndarray  # [3,3] world -> camera rotation (row-major)
    t: np.ndarray  # [3]   world -> camera translation
    znear: float = 0.2
    bg: tuple = (0.0, 0.0, 0.0)

    @property
    def pixels(self) -> int:
        return self.width * self.height


@dataclasses.dataclass
class Scene:
    surfels: Surfels
    gaussians: Gaussians
    cameras: List[Camera]
    name: str = ""


# ----------------------------------------------------------------------------
# random draws


def _log_uniform(rng, lo, hi, size):
    return np.exp(rng.uniform(math.log(lo), math.log(hi), size=size))


def _random_quats(rng, n):
    q = rng.standard_normal((4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    return q


def _sh(rng, n, degree=SH_DEGREE):
    k = (degree + 1) ** 2
    sh = rng.normal(0.0, 0.2, size=(k, 3, n))
    sh[0] = rng.normal(0.5, 0.2, size=(3, n))
    return sh


def _frame_to_quat(t1, t2, n):
    """Unit quaternions (w,x,y,z) of the rotations whose columns are t1, t2, n.

    Inputs are [3][k] orthonormal right-handed frames.  Standard trace-branch
    conversion of a rotation matrix to a quaternion.
    """
    m = np.stack([t1, t2, n], axis=1)  # [3 rows][3 cols][k]
    k = t1.shape[1]
    q = np.empty((4, k))
    tr = m[0, 0] + m[1, 1] + m[2, 2]
    c0 = tr > 0
    c1 = (~c0) & (m[0, 0] >= m[1, 1]) & (m[0, 0] >= m[2, 2])
    c2 = (~c0) & (~c1) & (m[1, 1] >= m[2, 2])
    c3 = ~(c0 | c1 | c2)
    s = np.sqrt(np.maximum(tr + 1.0, 1e-30)) * 2
    q[0] = np.where(c0, 0.25 * s, 0)
    q[1] = np.where(c0, (m[2, 1] - m[1, 2]) / s, 0)
    q[2] = np.where(c0, (m[0, 2] - m[2, 0]) / s, 0)
    q[3] = np.where(c0, (m[1, 0] - m[0, 1]) / s, 0)
    s = np.sqrt(np.maximum(1.0 + m[0, 0] - m[1, 1] - m[2, 2], 1e-30)) * 2
    q[0] = np.where(c1, (m[2, 1] - m[1, 2]) / s, q[0])
    q[1] = np.where(c1, 0.25 * s, q[1])
    q[2] = np.where(c1, (m[0, 1] + m[1, 0]) / s, q[2])
    q[3] = np.where(c1, (m[0, 2] + m[2, 0]) / s, q[3])
    s = np.sqrt(np.maximum(1.0 + m[1, 1] - m[0, 0] - m[2, 2], 1e-30)) * 2
    q[0] = np.where(c2, (m[0, 2] - m[2, 0]) / s, q[0])
    q[1] = np.where(c2, (m[0, 1] + m[1, 0]) / s, q[1])
    q[2] = np.where(c2, 0.25 * s, q[2])
    q[3] = np.where(c2, (m[1, 2] + m[2, 1]) / s, q[3])
    s = np.sqrt(np.maximum(1.0 + m[2, 2] - m[0, 0] - m[1, 1], 1e-30)) * 2
    q[0] = np.where(c3, (m[1, 0] - m[0, 1]) / s, q[0])
    q[1] = np.where(c3, (m[0, 2] + m[2, 0]) / s, q[1])
    q[2] = np.where(c3, (m[1, 2] + m[2, 1]) / s, q[2])
    q[3] = np.where(c3, 0.25 * s, q[3])
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    return q


def _orthonormal_tangents(n, rng):
    """Random in-plane tangent frame (t1, t2) for unit normals n [3][k]."""
    k = n.shape[1]
    a = np.where(np.abs(n[0:1]) < 0.9, np.array([[1.0], [0.0], [0.0]]),
                 np.array([[0.0], [1.0], [0.0]]))
    a = np.broadcast_to(a, (3, k))
    u = np.cross(n.T, a.T).T
    u /= np.linalg.norm(u, axis=0, keepdims=True)
    v = np.cross(n.T, u.T).T
    th = rng.uniform(0, 2 * math.pi, size=k)
    t1 = np.cos(th) * u + np.sin(th) * v
    t2 = np.cross(n.T, t1.T).T
    return t1, t2


# ----------------------------------------------------------------------------
# scenes


def _surface_scene(rng, n_surf, n_surfels, n_gauss, box, scale_mult,
                   surfel_scale=(0.002, 0.03), gauss_scale=(0.002, 0.02),
                   offset_radius=0.02):
    """Surfels on seeded random spheres and square patches (half and half).

    Sphere: centre U[-0.8 box, 0.8 box]^3, radius U[0.3, 1.5]*mult.
    Patch:  centre U[-0.8 box, 0.8 box]^3, random normal, half-size
            U[0.5, 2.5]*mult.
    Surfels are sampled area-proportionally and uniformly on each surface,
    oriented to the surface normal with a random in-plane angle; points
    outside [-box, box]^3 are rejected.  Gaussians sit at a random surfel
    centre plus a uniform offset in a ball of radius `offset_radius`.
    """
    inner = 0.8 * box
    n_sph = n_surf // 2
    n_pln = n_surf - n_sph
    sph_c = rng.uniform(-inner, inner, size=(n_sph, 3))
    sph_r = rng.uniform(0.3, 1.5, size=n_sph) * scale_mult
    pln_c = rng.uniform(-inner, inner, size=(n_pln, 3))
    pln_n = rng.standard_normal((n_pln, 3))
    pln_n /= np.linalg.norm(pln_n, axis=1, keepdims=True)
    pln_h = rng.uniform(0.5, 2.5, size=n_pln) * scale_mult
    areas = np.concatenate([4 * math.pi * sph_r ** 2, (2 * pln_h) ** 2])
    prob = areas / areas.sum()

    pts = []
    nrm = []
    have = 0
    while have < n_surfels:
        want = int((n_surfels - have) * 1.3) + 1024
        which = rng.choice(n_surf, size=want, p=prob)
        p = np.empty((want, 3))
        nn = np.empty((want, 3))
        is_s = which < n_sph
        ks = which[is_s]
        d = rng.standard_normal((ks.size, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        p[is_s] = sph_c[ks] + sph_r[ks, None] * d
        nn[is_s] = d
        kp = which[~is_s] - n_sph
        nrm_p = pln_n[kp]
        t1, t2 = _orthonormal_tangents(nrm_p.T, rng)
        a = rng.uniform(-1, 1, size=kp.size) * pln_h[kp]
        b = rng.uniform(-1, 1, size=kp.size) * pln_h[kp]
        p[~is_s] = pln_c[kp] + (a * t1 + b * t2).T
        nn[~is_s] = nrm_p
        inside = np.all(np.abs(p) <= box, axis=1)
        pts.append(p[inside])
        nrm.append(nn[inside])
        have += int(inside.sum())
    pts = np.concatenate(pts)[:n_surfels]
    nrm = np.concatenate(nrm)[:n_surfels]

    t1, t2 = _orthonormal_tangents(nrm.T, rng)
    quat = _frame_to_quat(t1, t2, nrm.T)
    surfels = Surfels(
        mean=pts.T.astype(np.float32).copy(),
        quat=quat.astype(np.float32),
        scale=_log_uniform(rng, *surfel_scale, size=(2, n_surfels)).astype(np.float32),
        sh=_sh(rng, n_surfels).astype(np.float32),
    )
    pick = rng.integers(0, n_surfels, size=n_gauss)
    d = rng.standard_normal((n_gauss, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    rad = offset_radius * rng.uniform(0, 1, size=n_gauss) ** (1.0 / 3.0)
    gmean = pts[pick] + d * rad[:, None]
    gaussians = Gaussians(
        mean=gmean.T.astype(np.float32).copy(),
        quat=_random_quats(rng, n_gauss).astype(np.float32),
        scale=_log_uniform(rng, *gauss_scale, size=(3, n_gauss)).astype(np.float32),
        opacity=rng.uniform(0.05, 0.99, size=n_gauss).astype(np.float32),
        sh=_sh(rng, n_gauss).astype(np.float32),
    )
    return surfels, gaussians


def pinhole(width, height, eye, target=(0.0, 0.0, 0.0), fov_x_deg=60.0,
            up=(0.0, -1.0, 0.0), znear=0.2, bg=(0.0, 0.0, 0.0)) -> Camera:
    """Look-at pinhole camera, horizontal field of view `fov_x_deg`."""
    eye = np.asarray(eye, dtype=np.float64)
    f = np.asarray(target, dtype=np.float64) - eye
    f /= np.linalg.norm(f)
    r = np.cross(f, np.asarray(up, dtype=np.float64))
    r /= np.linalg.norm(r)
    d = np.cross(f, r)
    R = np.stack([r, d, f])
    t = -R @ eye
    fx = (width / 2.0) / math.tan(math.radians(fov_x_deg) / 2.0)
    return Camera(width, height, fx, fx, width / 2.0, height / 2.0,
                  R.astype(np.float64), t.astype(np.float64), znear, tuple(bg))


def ring_camera(width, height, radius, theta, **kw) -> Camera:
    eye = (radius * math.cos(theta), 0.0, radius * math.sin(theta))
    return pinhole(width, height, eye, **kw)


RING16_RESOLUTIONS = [(640, 360), (1280, 720), (1600, 1060), (1920, 1080)]

# workload name -> its seed offset (the scene is drawn from PCG64(17545 + offset))
WORKLOADS = {"tiny": 0, "surfaces_300k": 1, "surfaces_1m_1080p": 2, "ring16_1m": 3, "surfaces_3m_4k": 4}


def workload(name: str, seed: Optional[int] = None,
             n_surfels: Optional[int] = None,
             n_gaussians: Optional[int] = None) -> Scene:
    """The five synthetic workloads, each seeded with PCG64(17545 + offset)
    unless `seed` is set:

    tiny               128x128, 2k surfels in U[-1,1]^3, 1k Gaussians, camera at distance 3.
    surfaces_300k      300k surfels on 64 surfaces in [-5,5]^3, 150k Gaussians, 1600x1060.
    surfaces_1m_1080p  as surfaces_300k with 1M surfels, 500k Gaussians, 1920x1080.
    ring16_1m          the surfaces_1m_1080p scene, 16 ring cameras cycling four resolutions.
    surfaces_3m_4k     3M surfels + 1M Gaussians on 256 surfaces in [-20,20]^3, 8 x 3840x2160.

    `n_surfels` / `n_gaussians` shrink a workload (same recipe) for quick tests.
    """
    if name not in WORKLOADS:
        raise ValueError(f"unknown workload {name!r}")
    off = WORKLOADS[name]
    rng = np.random.Generator(np.random.PCG64(BASE_SEED + off if seed is None else seed))
    if name == "tiny":
        n = n_surfels or 2000
        m = n_gaussians or 1000
        mean = rng.uniform(-1, 1, size=(3, n))
        surfels = Surfels(
            mean=mean.astype(np.float32),
            quat=_random_quats(rng, n).astype(np.float32),
            scale=_log_uniform(rng, 0.005, 0.05, size=(2, n)).astype(np.float32),
            sh=_sh(rng, n).astype(np.float32),
        )
        pick = rng.integers(0, n, size=m)
        gmean = mean[:, pick] + rng.normal(0, 0.01, size=(3, m))
        gaussians = Gaussians(
            mean=gmean.astype(np.float32),
            quat=_random_quats(rng, m).astype(np.float32),
            scale=_log_uniform(rng, 0.002, 0.02, size=(3, m)).astype(np.float32),
            opacity=rng.uniform(0.05, 0.99, size=m).astype(np.float32),
            sh=_sh(rng, m).astype(np.float32),
        )
        fx = 64.0 / math.tan(math.radians(30.0))
        cam = Camera(128, 128, fx, fx, 64.0, 64.0, np.eye(3), np.array([0.0, 0.0, 3.0]))
        return Scene(surfels, gaussians, [cam], name)
    if name in ("surfaces_300k", "surfaces_1m_1080p", "ring16_1m"):
        small = name == "surfaces_300k"
        n = n_surfels or (300_000 if small else 1_000_000)
        m = n_gaussians or (150_000 if small else 500_000)
        if name == "ring16_1m":  # the same scene as surfaces_1m_1080p
            rng = np.random.Generator(np.random.PCG64(BASE_SEED + WORKLOADS["surfaces_1m_1080p"]
                                                      if seed is None else seed))
        surfels, gaussians = _surface_scene(rng, 64, n, m, 5.0, 1.0)
        if small:
            cams = [ring_camera(1600, 1060, 8.0, 0.0)]
        elif name == "surfaces_1m_1080p":
            cams = [ring_camera(1920, 1080, 8.0, 0.0)]
        else:
            cams = [ring_camera(*RING16_RESOLUTIONS[k % 4], 8.0, 2 * math.pi * k / 16)
                    for k in range(16)]
        return Scene(surfels, gaussians, cams, name)
    n = n_surfels or 3_000_000
    m = n_gaussians or 1_000_000
    surfels, gaussians = _surface_scene(rng, 256, n, m, 20.0, 4.0,
                                        surfel_scale=(0.008, 0.12),
                                        gauss_scale=(0.008, 0.08),
                                        offset_radius=0.08)
    cams = [ring_camera(3840, 2160, 32.0, 2 * math.pi * k / 8) for k in range(8)]
    return Scene(surfels, gaussians, cams, name)


def perturbed_copy(scene: Scene, seed: int) -> Scene:
    """Target scene for the differentiation workload: Gaussian means
    + N(0, 0.005^2), every Gaussian and surfel SH coefficient + N(0, 0.05^2)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    g = scene.gaussians
    s = scene.surfels
    g2 = Gaussians(
        mean=(g.mean + rng.normal(0, 0.005, size=g.mean.shape)).astype(np.float32),
        quat=g.quat.copy(), scale=g.scale.copy(), opacity=g.opacity.copy(),
        sh=(g.sh + rng.normal(0, 0.05, size=g.sh.shape)).astype(np.float32),
    )
    s2 = Surfels(mean=s.mean.copy(), quat=s.quat.copy(), scale=s.scale.copy(),
                 sh=(s.sh + rng.normal(0, 0.05, size=s.sh.shape)).astype(np.float32))
    return Scene(s2, g2, list(scene.cameras), scene.name + "-target")


def permute_gaussians(g: Gaussians, seed: int):
    """Random permutation of the Gaussian array (order-independence check).
    Returns (permuted set, perm) with permuted[k] = original[perm[k]]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    perm = rng.permutation(g.m)
    return Gaussians(mean=g.mean[:, perm].copy(), quat=g.quat[:, perm].copy(),
                     scale=g.scale[:, perm].copy(), opacity=g.opacity[perm].copy(),
                     sh=g.sh[:, :, perm].copy(),
                     filter3d=None if g.filter3d is None else g.filter3d[perm].copy()), perm


def permute_surfels(s: Surfels, seed: int):
    rng = np.random.Generator(np.random.PCG64(seed))
    perm = rng.permutation(s.n)
    return Surfels(mean=s.mean[:, perm].copy(), quat=s.quat[:, perm].copy(),
                   scale=s.scale[:, perm].copy(), sh=s.sh[:, :, perm].copy()), perm


def subset(scene: Scene, surfel_idx=None, gauss_idx=None) -> Scene:
    s, g = scene.surfels, scene.gaussians
    if surfel_idx is not None:
        s = Surfels(s.mean[:, surfel_idx].copy(), s.quat[:, surfel_idx].copy(),
                    s.scale[:, surfel_idx].copy(), s.sh[:, :, surfel_idx].copy())
    if gauss_idx is not None:
        g = Gaussians(g.mean[:, gauss_idx].copy(), g.quat[:, gauss_idx].copy(),
                      g.scale[:, gauss_idx].copy(), g.opacity[gauss_idx].copy(),
                      g.sh[:, :, gauss_idx].copy(),
                      None if g.filter3d is None else g.filter3d[gauss_idx].copy())
    return Scene(s, g, list(scene.cameras), scene.name)


def empty_surfels(k=SH_K) -> Surfels:
    return Surfels(np.zeros((3, 0), np.float32), np.zeros((4, 0), np.float32),
                   np.zeros((2, 0), np.float32), np.zeros((k, 3, 0), np.float32))


def empty_gaussians(k=SH_K) -> Gaussians:
    return Gaussians(np.zeros((3, 0), np.float32), np.zeros((4, 0), np.float32),
                     np.zeros((3, 0), np.float32), np.zeros((0,), np.float32),
                     np.zeros((k, 3, 0), np.float32))
