"""Seeded synthetic inputs: isotropic Gaussian scenes and pinhole cameras.

This module draws random numbers and builds camera poses. It contains none of the
rendering arithmetic (no projection, no kernel, no compositing): both the FP64 oracle
and the GPU path consume what it produces, and neither is imported here.

Every generator uses ``numpy.random.default_rng(seed)`` (PCG64) with the draws taken
in the order written below, computed in FP64 and stored as FP32, so a scene is a pure
function of its seed and sizes.

Scene layout (structure of arrays, FP32, the layout the renderer reads):
  pos      [3, N]   world-space centres mu (rows x, y, z)
  scale    [N]      isotropic scale sigma (linear world units, eq. 8 of the paper)
  opacity  [N]      activated opacity o in (0, 1)
  color    [3K, N]  colour coefficients, K = (deg+1)^2, row 3k+ch holds coefficient k of
                    channel ch; k = l*l + l + m. Row block k=0 is the base colour.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np

__all__ = [
    "Scene", "Camera", "look_at_camera", "orbit_camera", "uniform_cube_scene",
    "mixture_scene", "stress_scene", "jitter_scene", "subset_scene",
    "WORKLOADS", "workload_scene", "workload_cameras", "random_projected",
    "field2d_target", "field2d_init", "AnisoScene", "aniso_from_iso", "aniso_mixture_scene", "point_cloud",
]


@dataclass
class Scene:
    pos: np.ndarray
    scale: np.ndarray
    opacity: np.ndarray
    color: np.ndarray
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.scale.shape[0])

    def validate(self) -> None:
        n = self.n
        k = (self.sh_degree + 1) ** 2
        assert self.pos.shape == (3, n) and self.pos.dtype == np.float32
        assert self.scale.shape == (n,) and self.scale.dtype == np.float32
        assert self.opacity.shape == (n,) and self.opacity.dtype == np.float32
        assert self.color.shape == (3 * k, n) and self.color.dtype == np.float32


@dataclass
class Camera:
    """Pinhole camera. Camera frame: x right, y down, z forward (depth).

    A world point mu maps to p = R mu + t; eye is the camera centre in world space.
    f is the focal length in pixels (square pixels), (cx, cy) the principal point.
    """
    R: np.ndarray            # float32 [3, 3], rows = camera axes in world coordinates
    t: np.ndarray            # float32 [3]
    eye: np.ndarray          # float32 [3]
    f: float
    cx: float
    cy: float
    width: int
    height: int
    near: float = 0.2

    def shifted(self, dx: float, dy: float, width: int, height: int) -> "Camera":
        """A crop of this camera: the principal point moves by (-dx, -dy)."""
        return replace(self, cx=float(np.float32(self.cx - dx)), cy=float(np.float32(self.cy - dy)),
                       width=int(width), height=int(height))


def _f32(x) -> float:
    return float(np.float32(x))


def look_at_camera(eye, target=(0.0, 0.0, 0.0), up=(0.0, 1.0, 0.0), width=256, height=256,
                   fov_y_deg=60.0, near=0.2) -> Camera:
    """Camera at ``eye`` looking at ``target``; vertical field of view ``fov_y_deg``.

    Axes: forward = normalize(target - eye), x = normalize(forward x up), y = forward x x,
    so x points right and y points down in the image. Focal length
    f = (height / 2) / tan(fov_y / 2); principal point at the image centre.
    """
    eye = np.asarray(eye, dtype=np.float64)
    fwd = np.asarray(target, dtype=np.float64) - eye
    fwd /= np.linalg.norm(fwd)
    x = np.cross(fwd, np.asarray(up, dtype=np.float64))
    x /= np.linalg.norm(x)
    y = np.cross(fwd, x)
    R = np.stack([x, y, fwd]).astype(np.float64)
    t = -R @ eye
    f = (height / 2.0) / math.tan(math.radians(fov_y_deg) / 2.0)
    return Camera(R=R.astype(np.float32), t=t.astype(np.float32), eye=eye.astype(np.float32),
                  f=_f32(f), cx=_f32(width / 2.0), cy=_f32(height / 2.0),
                  width=int(width), height=int(height), near=_f32(near))


def orbit_camera(theta: float, radius: float = 4.0, width=1920, height=1080, fov_y_deg=60.0,
                 near=0.2) -> Camera:
    """Camera on the horizontal orbit eye = radius (sin theta, 0, cos theta), looking at 0."""
    eye = (radius * math.sin(theta), 0.0, radius * math.cos(theta))
    return look_at_camera(eye, width=width, height=height, fov_y_deg=fov_y_deg, near=near)


def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def _pack(pos64, log_scale, opacity, color64, deg) -> Scene:
    s = Scene(pos=np.ascontiguousarray(pos64.T.astype(np.float32)),
              scale=np.exp(log_scale).astype(np.float32),
              opacity=opacity.astype(np.float32),
              color=np.ascontiguousarray(color64.astype(np.float32)),
              sh_degree=int(deg))
    s.validate()
    return s


def uniform_cube_scene(n=10_000, seed=0, log_scale_mean=math.log(0.02), log_scale_std=0.3) -> Scene:
    """Positions U[-1,1]^3, ln sigma ~ N(mean, std), o = sigmoid(N(0,1)), RGB U[0,1] (degree 0)."""
    rng = np.random.default_rng(seed)
    pos = rng.uniform(-1.0, 1.0, size=(n, 3))
    log_scale = rng.normal(log_scale_mean, log_scale_std, size=n)
    opacity = _sigmoid(rng.normal(0.0, 1.0, size=n))
    rgb = rng.uniform(0.0, 1.0, size=(n, 3))
    return _pack(pos, log_scale, opacity, rgb.T, 0)


def _sh_coeffs(rng, n, deg):
    k = (deg + 1) ** 2
    color = np.empty((3 * k, n), dtype=np.float64)
    color[0:3] = rng.uniform(0.0, 1.0, size=(3, n))
    if k > 1:
        color[3:] = rng.normal(0.0, 0.05, size=(3 * k - 3, n))
    return color


def _mixture_points(rng, n):
    n_sphere = int(round(0.3 * n))
    n_cluster = n - n_sphere
    centres = rng.uniform(-1.0, 1.0, size=(64, 3))
    stds = rng.uniform(0.05, 0.3, size=64)
    assign = rng.integers(0, 64, size=n_cluster)
    pc = centres[assign] + rng.normal(size=(n_cluster, 3)) * stds[assign, None]
    s_centres = rng.uniform(-0.8, 0.8, size=(8, 3))
    s_radii = rng.uniform(0.1, 0.5, size=8)
    s_assign = rng.integers(0, 8, size=n_sphere)
    nrm = rng.normal(size=(n_sphere, 3))
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    ps = s_centres[s_assign] + s_radii[s_assign, None] * nrm
    pos = np.concatenate([pc, ps], axis=0)
    return pos[rng.permutation(n)]


def point_cloud(n=200_000, seed=30, extent=1.0, n_clusters=24):
    """A coloured point cloud (the stand-in for the points a 3D reconstruction starts
    from): clusters of isotropic normal points (centres U[-extent/2, extent/2]^3, std
    U[0.03, 0.25] extent) plus 25% uniform in the cube [-extent, extent]^3; every cluster
    has a base colour U[0,1]^3, its points that colour plus N(0, 0.04) clipped to [0, 1],
    the uniform points U[0,1]^3. Returns (points [3, n], colours [3, n]), FP32."""
    rng = np.random.default_rng(seed)
    n_u = n // 4
    n_c = n - n_u
    centres = rng.uniform(-0.5 * extent, 0.5 * extent, size=(n_clusters, 3))
    stds = rng.uniform(0.03, 0.25, size=n_clusters) * extent
    base = rng.uniform(0.0, 1.0, size=(n_clusters, 3))
    assign = rng.integers(0, n_clusters, size=n_c)
    pc = centres[assign] + rng.normal(size=(n_c, 3)) * stds[assign, None]
    cc = np.clip(base[assign] + rng.normal(0.0, 0.04, size=(n_c, 3)), 0.0, 1.0)
    pu = rng.uniform(-extent, extent, size=(n_u, 3))
    cu = rng.uniform(0.0, 1.0, size=(n_u, 3))
    order = rng.permutation(n)
    pos = np.concatenate([pc, pu])[order]
    col = np.concatenate([cc, cu])[order]
    return np.ascontiguousarray(pos.T.astype(np.float32)), np.ascontiguousarray(col.T.astype(np.float32))


def mixture_scene(n=1_000_000, seed=0, log_scale_mean=math.log(0.005), log_scale_std=0.5,
                  sh_degree=3) -> Scene:
    """70% of points from 64 isotropic clusters (std U[0.05,0.3]) and 30% on 8 sphere
    surfaces; ln sigma ~ N(mean, std); o = sigmoid(N(0,1)); colour coefficients with
    base colour U[0,1] and higher bands N(0, 0.05)."""
    rng = np.random.default_rng(seed)
    pos = _mixture_points(rng, n)
    log_scale = rng.normal(log_scale_mean, log_scale_std, size=n)
    opacity = _sigmoid(rng.normal(0.0, 1.0, size=n))
    color = _sh_coeffs(rng, n, sh_degree)
    return _pack(pos, log_scale, opacity, color, sh_degree)


def stress_scene(n=6_000_000, seed=5, sh_degree=3) -> Scene:
    """70% of points in 16 tight clusters (std 0.02), 30% from the mixture layout;
    ln sigma ~ N(ln 0.003, 0.7): skews per-tile list lengths by orders of magnitude."""
    rng = np.random.default_rng(seed)
    n_tight = int(round(0.7 * n))
    centres = rng.uniform(-1.0, 1.0, size=(16, 3))
    assign = rng.integers(0, 16, size=n_tight)
    pt = centres[assign] + rng.normal(size=(n_tight, 3)) * 0.02
    pm = _mixture_points(rng, n - n_tight)
    pos = np.concatenate([pt, pm], axis=0)[rng.permutation(n)]
    log_scale = rng.normal(math.log(0.003), 0.7, size=n)
    opacity = _sigmoid(rng.normal(0.0, 1.0, size=n))
    color = _sh_coeffs(rng, n, sh_degree)
    return _pack(pos, log_scale, opacity, color, sh_degree)


@dataclass
class AnisoScene:
    """Particles with a full covariance (the anisotropic variant): pos [3, N], rot [4, N]
    quaternions (w, x, y, z; not necessarily unit), scale [3, N] linear per-axis scales,
    opacity [N], color [3K, N] as in Scene. FP32."""
    pos: np.ndarray
    rot: np.ndarray
    scale: np.ndarray
    opacity: np.ndarray
    color: np.ndarray
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.opacity.shape[0])


def aniso_from_iso(scene: Scene) -> AnisoScene:
    """The same particles as anisotropic ones: identity rotation, the scale on all three
    axes (so the covariance is sigma^2 I)."""
    n = scene.n
    rot = np.zeros((4, n), dtype=np.float32)
    rot[0] = 1.0
    return AnisoScene(pos=scene.pos.copy(), rot=rot, scale=np.ascontiguousarray(np.repeat(scene.scale[None], 3, 0)),
                      opacity=scene.opacity.copy(), color=scene.color.copy(), sh_degree=scene.sh_degree)


def aniso_mixture_scene(n=1_000_000, seed=0, log_scale_mean=math.log(0.005), log_scale_std=0.5,
                        axis_log_std=0.5, sh_degree=3) -> AnisoScene:
    """The mixture layout of mixture_scene with a random orientation per particle
    (quaternion of four N(0, 1) draws) and per-axis scales exp(b + N(0, axis_log_std)) around
    a per-particle log-scale b ~ N(log_scale_mean, log_scale_std). Draw order: positions,
    b, opacity, colour, quaternions, per-axis offsets."""
    rng = np.random.default_rng(seed)
    pos = _mixture_points(rng, n)
    b = rng.normal(log_scale_mean, log_scale_std, size=n)
    opacity = _sigmoid(rng.normal(0.0, 1.0, size=n))
    color = _sh_coeffs(rng, n, sh_degree)
    q = rng.normal(0.0, 1.0, size=(4, n))
    axis = rng.normal(0.0, axis_log_std, size=(3, n))
    return AnisoScene(pos=np.ascontiguousarray(pos.T.astype(np.float32)), rot=q.astype(np.float32),
                      scale=np.exp(b[None, :] + axis).astype(np.float32), opacity=opacity.astype(np.float32),
                      color=np.ascontiguousarray(color.astype(np.float32)), sh_degree=int(sh_degree))


def jitter_scene(scene: Scene, seed=1, pos_std=0.01, log_scale_std=0.2) -> Scene:
    """Perturbed copy: mu += N(0, pos_std), sigma *= exp(N(0, log_scale_std))."""
    rng = np.random.default_rng(seed)
    pos = scene.pos.astype(np.float64) + rng.normal(0.0, pos_std, size=scene.pos.shape)
    scale = scene.scale.astype(np.float64) * np.exp(rng.normal(0.0, log_scale_std, size=scene.n))
    return Scene(pos=pos.astype(np.float32), scale=scale.astype(np.float32),
                 opacity=scene.opacity.copy(), color=scene.color.copy(), sh_degree=scene.sh_degree)


def subset_scene(scene: Scene, idx) -> Scene:
    idx = np.asarray(idx)
    return Scene(pos=np.ascontiguousarray(scene.pos[:, idx]), scale=scene.scale[idx].copy(),
                 opacity=scene.opacity[idx].copy(), color=np.ascontiguousarray(scene.color[:, idx]),
                 sh_degree=scene.sh_degree)


# Named workloads: the render sizes and scene recipes that tests and the benchmark use.
WORKLOADS = {
    # 10k Gaussians in a cube, degree-0 colour, one 256x256 view from distance 3.
    "cube10k_256": dict(scene=("cube", 10_000, 0), views=1, radius=3.0, width=256, height=256),
    # 1M Gaussians, clusters + spheres, degree-3 SH, orbit of 100 views at 1080p.
    "mix1m_1080p": dict(scene=("mix", 1_000_000, 0), views=100, radius=4.0, width=1920, height=1080),
    # 500k Gaussians, batch of 4 views at 720p (training step).
    "mix500k_720p_x4": dict(scene=("mix", 500_000, 0), views=4, radius=4.0, width=1280, height=720),
    # 6M Gaussians with tight clusters, 8 views at 4K (stress).
    "stress6m_4k_x8": dict(scene=("stress", 6_000_000, 5), views=8, radius=4.0, width=3840, height=2160),
}


def workload_scene(name: str, n: int | None = None) -> Scene:
    kind, n0, seed = WORKLOADS[name]["scene"]
    n = n0 if n is None else n
    if kind == "cube":
        return uniform_cube_scene(n, seed)
    if kind == "mix":
        return mixture_scene(n, seed)
    return stress_scene(n, seed)


def workload_cameras(name: str, view_ids=None, width=None, height=None):
    w = WORKLOADS[name]
    nv = w["views"]
    ids = range(nv) if view_ids is None else view_ids
    if name.startswith("cube"):
        return [look_at_camera((0.0, 0.0, w["radius"]), width=width or w["width"],
                               height=height or w["height"]) for _ in ids]
    if name.startswith("mix500k"):
        # the training batch uses views 0, 25, 50, 75 of a 100-view orbit
        ids = [0, 25, 50, 75] if view_ids is None else view_ids
        step = 100
    else:
        step = nv
    return [orbit_camera(2.0 * math.pi * i / step, w["radius"], width or w["width"],
                         height or w["height"]) for i in ids]


def crowded_projected(n, width, height, cx, cy, spread, seed=0, max_radius=6.0, depths=None):
    """Binning-only footprints crowded around (cx, cy) (uniform within +-spread), so that
    one tile holds many entries. `depths`: a set of values to draw from (exact ties), or
    None for uniform depths in [0.5, 80]."""
    rng = np.random.default_rng(seed)
    u = cx + rng.uniform(-spread, spread, size=n)
    v = cy + rng.uniform(-spread, spread, size=n)
    r = rng.uniform(0.0, max_radius, size=n)
    z = rng.uniform(0.5, 80.0, size=n) if depths is None else rng.choice(np.asarray(depths, np.float64), size=n)
    return u.astype(np.float32), v.astype(np.float32), z.astype(np.float32), r.astype(np.float32)


def random_projected(n, width, height, seed=0, max_radius=12.0, depth_ties=False):
    """Random per-Gaussian screen footprints (u, v, depth, radius) in FP32, for the
    binning stage alone: centres spread past the image borders, some radii zero-ish,
    and optionally many exactly equal depths to exercise the sort's tie order."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(-0.2 * width, 1.2 * width, size=n)
    v = rng.uniform(-0.2 * height, 1.2 * height, size=n)
    r = rng.exponential(max_radius / 4.0, size=n).clip(0.0, max_radius)
    z = rng.uniform(0.5, 8.0, size=n)
    if depth_ties:
        z = rng.choice(np.array([1.0, 1.5, 2.0, 2.0000002]), size=n)
    return u.astype(np.float32), v.astype(np.float32), z.astype(np.float32), r.astype(np.float32)


# --------------------------------------------------------------------------------------
# 2D image fitting (the paper's 2D experiment): a procedural target image and a random
# initial set of particles. Draws only; the kernel sum itself lives elsewhere.
# --------------------------------------------------------------------------------------

def field2d_target(width=512, height=512, seed=20) -> np.ndarray:
    """Procedural RGB target [3][H][W] in [0, 1] (a stand-in for the paper's images, which
    are not available): a linear colour ramp, 12 filled discs of random colour and radius
    16-80 px, and a band of sinusoidal stripes. Draws: ramp direction and end colours,
    then per disc centre, radius, colour, then the band's row range, period and phase."""
    rng = np.random.default_rng(seed)
    yy, xx = np.mgrid[0:height, 0:width].astype(np.float64) + 0.5
    ang = rng.uniform(0.0, 2.0 * math.pi)
    c0, c1 = rng.uniform(0.0, 1.0, 3), rng.uniform(0.0, 1.0, 3)
    t = ((xx - width / 2) * math.cos(ang) + (yy - height / 2) * math.sin(ang)) / max(width, height) + 0.5
    t = t.clip(0.0, 1.0)
    img = c0[:, None, None] * (1.0 - t) + c1[:, None, None] * t
    for _ in range(12):
        cx, cy = rng.uniform(0, width), rng.uniform(0, height)
        rad = rng.uniform(16.0, 80.0)
        col = rng.uniform(0.0, 1.0, 3)
        m = (xx - cx) ** 2 + (yy - cy) ** 2 < rad * rad
        img[:, m] = col[:, None]
    y0 = rng.uniform(0.6, 0.8) * height
    y1 = y0 + rng.uniform(0.08, 0.15) * height
    period, phase = rng.uniform(6.0, 20.0), rng.uniform(0.0, 2.0 * math.pi)
    band = (yy >= y0) & (yy < y1)
    stripes = 0.5 + 0.5 * np.sin(2.0 * math.pi * xx / period + phase)
    img[:, band] = stripes[band][None, :]
    return img.astype(np.float32)


def field2d_init(target: np.ndarray, K: int, seed=21):
    """Random initial particles for fitting `target` [3][H][W] (the paper's random
    initialisation): centres uniform over the image, scale half the width of one cell of
    a K-cell partition of the image, amplitude the target colour of the pixel under the
    centre. Returns (mu [2][K], sigma [K], amp [3][K]) in FP32."""
    rng = np.random.default_rng(seed)
    _, H, W = target.shape
    mu = np.stack([rng.uniform(0.0, W, K), rng.uniform(0.0, H, K)])
    sigma = np.full(K, 0.5 * math.sqrt(W * H / K))
    ix = np.clip(mu[0].astype(np.int64), 0, W - 1)
    iy = np.clip(mu[1].astype(np.int64), 0, H - 1)
    amp = target[:, iy, ix].astype(np.float64)
    return mu.astype(np.float32), sigma.astype(np.float32), amp.astype(np.float32)
