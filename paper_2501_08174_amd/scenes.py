"""Seeded synthetic scenes for the surfel rasterizer.

This module only draws inputs: surfel parameters, pinhole cameras, binary
object masks and target images.  It holds none of the renderer's arithmetic
and is the one module shared by the GPU path's tests/bench and the oracle's
tests.  Every array is drawn with ``numpy.random.default_rng(seed)`` in
float64 and stored as float32 (uint8 for masks).

Conventions of the produced data (inputs to both sides):
  * surfel parameters: ``means[N,3]``, ``scales[N,2]`` (already activated,
    i.e. positive), ``quats[N,4]`` raw quaternion in (w, x, y, z) order,
    ``opac[N]`` (already activated, in (0,1)), ``sh[N,K,3]`` real spherical
    harmonic coefficients, K = (degree+1)^2, coefficient-major then channel;
  * camera: ``viewmat`` is the 3x4 world->camera matrix [R|t] with OpenCV
    axes (x right, y down, z forward); pixel (i, j) is sampled at
    (i + 0.5, j + 0.5); ``campos`` is the camera centre in world space.

The workloads stand in for the paper's datasets (DTU frames at 800x600 with
~1-2e5 Gaussians and Mip-NeRF360 frames at ~1237x822 / 1559x1039 with up to
~2e6 Gaussians, Sections 5.1 and 5.3), which are not available here.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

# Real SH band-0 basis value 1/(2 sqrt(pi)); only used to store a plain RGB
# colour as a degree-0 coefficient (input recipe of the small scenes).
_Y00 = 0.5 / math.sqrt(math.pi)

ZNEAR_DEFAULT = 0.2


@dataclass
class Camera:
    viewmat: np.ndarray          # (3,4) float32 world->camera [R|t]
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    campos: np.ndarray           # (3,) float32
    znear: float = ZNEAR_DEFAULT
    bg: np.ndarray = field(default_factory=lambda: np.zeros(3, np.float32))

    @property
    def npix(self) -> int:
        return self.width * self.height


@dataclass
class Scene:
    means: np.ndarray            # (N,3) float32
    scales: np.ndarray           # (N,2) float32
    quats: np.ndarray            # (N,4) float32  (w,x,y,z), unnormalised
    opac: np.ndarray             # (N,)  float32
    sh: np.ndarray               # (N,K,3) float32
    sh_degree: int
    cams: List[Camera]
    masks: List[np.ndarray]      # per view (H,W) uint8 in {0,1}
    targets: Optional[List[np.ndarray]] = None   # per view (3,H,W) float32
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    @property
    def v(self) -> int:
        return len(self.cams)


# ----------------------------------------------------------------------------
# cameras
# ----------------------------------------------------------------------------

def fov60_focal(width: int) -> float:
    """Horizontal field of view of 60 degrees, square pixels."""
    return width / (2.0 * math.tan(math.radians(30.0)))


def make_camera(R: np.ndarray, pos: np.ndarray, width: int, height: int,
                fx: Optional[float] = None, fy: Optional[float] = None,
                cx: Optional[float] = None, cy: Optional[float] = None,
                znear: float = ZNEAR_DEFAULT, bg=None) -> Camera:
    """Camera from a world->camera rotation ``R`` (rows = camera axes in
    world coordinates) and a centre ``pos``; t = -R pos."""
    R = np.asarray(R, np.float64)
    pos = np.asarray(pos, np.float64)
    t = -R @ pos
    vm = np.concatenate([R, t[:, None]], axis=1).astype(np.float32)
    fx = fov60_focal(width) if fx is None else fx
    fy = fx if fy is None else fy
    cx = width / 2.0 if cx is None else cx
    cy = height / 2.0 if cy is None else cy
    return Camera(viewmat=vm, fx=float(np.float32(fx)), fy=float(np.float32(fy)),
                  cx=float(np.float32(cx)), cy=float(np.float32(cy)),
                  width=int(width), height=int(height),
                  campos=pos.astype(np.float32), znear=float(np.float32(znear)),
                  bg=np.zeros(3, np.float32) if bg is None else np.asarray(bg, np.float32))


def look_at_rotation(pos: np.ndarray, target=(0.0, 0.0, 0.0), up=(0.0, 1.0, 0.0)) -> np.ndarray:
    """World->camera rotation for OpenCV axes (z forward, y down).  ``up`` is
    swapped to +x when it is nearly parallel to the viewing direction."""
    pos = np.asarray(pos, np.float64)
    f = np.asarray(target, np.float64) - pos
    f /= np.linalg.norm(f)
    up = np.asarray(up, np.float64)
    if abs(float(f @ up)) > 0.99:
        up = np.array([1.0, 0.0, 0.0])
    down = -up
    xc = np.cross(down, f)
    xc /= np.linalg.norm(xc)
    yc = np.cross(f, xc)
    return np.stack([xc, yc, f], axis=0)


def fibonacci_sphere(n: int, radius: float) -> np.ndarray:
    i = np.arange(n, dtype=np.float64)
    z = 1.0 - 2.0 * (i + 0.5) / n
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = i * math.pi * (3.0 - math.sqrt(5.0))
    return radius * np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)


def pixel_rays(cam: Camera):
    """World-space ray origin and (unnormalised) directions through every
    pixel centre, (H*W,3) float64."""
    j, i = np.meshgrid(np.arange(cam.height), np.arange(cam.width), indexing="ij")
    d = np.stack([(i + 0.5 - cam.cx) / cam.fx, (j + 0.5 - cam.cy) / cam.fy,
                  np.ones_like(i, dtype=np.float64)], axis=-1).reshape(-1, 3)
    R = cam.viewmat[:, :3].astype(np.float64)
    return cam.campos.astype(np.float64), d @ R   # rows: R^T d


def ellipsoid_mask(cam: Camera, centre, axes, rot=None) -> np.ndarray:
    """uint8 (H,W): 1 where the pixel's ray hits the ellipsoid
    {x : |diag(1/axes) rot^T (x - centre)| <= 1}."""
    o, d = pixel_rays(cam)
    rot = np.eye(3) if rot is None else np.asarray(rot, np.float64)
    inv = 1.0 / np.asarray(axes, np.float64)
    oo = ((o - np.asarray(centre, np.float64)) @ rot) * inv
    dd = (d @ rot) * inv
    a = np.einsum("ij,ij->i", dd, dd)
    b = 2.0 * dd @ oo
    c = oo @ oo - 1.0
    disc = b * b - 4.0 * a * c
    hit = disc >= 0.0
    # the far root must be in front of the camera
    far = (-b + np.sqrt(np.maximum(disc, 0.0))) / (2.0 * a)
    hit &= far > 0.0
    return hit.reshape(cam.height, cam.width).astype(np.uint8)


def random_rotation(rng: np.random.Generator) -> np.ndarray:
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


# ----------------------------------------------------------------------------
# surfel attribute draws
# ----------------------------------------------------------------------------

def _draw_shape(rng: np.random.Generator, n: int):
    scales = np.exp(rng.uniform(math.log(0.01), math.log(0.1), size=(n, 2)))
    quats = rng.normal(size=(n, 4))
    quats /= np.linalg.norm(quats, axis=1, keepdims=True)
    opac = 1.0 / (1.0 + np.exp(-rng.normal(size=n)))
    return scales, quats, opac


def _rgb_as_sh0(rgb: np.ndarray) -> np.ndarray:
    return ((rgb - 0.5) / _Y00)[:, None, :]


def _uniform_in_ellipsoid(rng, n, axes):
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    r = rng.uniform(size=n) ** (1.0 / 3.0)
    return d * r[:, None] * np.asarray(axes, np.float64)


def _uniform_in_shell(rng, n, r0, r1):
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    r = (rng.uniform(size=n) * (r1 ** 3 - r0 ** 3) + r0 ** 3) ** (1.0 / 3.0)
    return d * r[:, None]


def _f32(*arrs):
    return [np.ascontiguousarray(a, dtype=np.float32) for a in arrs]


OBJECT_AXES = (1.0, 0.75, 0.5)


def _object_mixture(rng, n):
    n_obj = int(round(0.7 * n))
    inside = _uniform_in_ellipsoid(rng, n_obj, OBJECT_AXES)
    outside = rng.uniform(-3.0, 3.0, size=(n - n_obj, 3))
    return np.concatenate([inside, outside], axis=0)


def _random_views(rng, n_views, radius, sizes):
    cams = []
    for v in range(n_views):
        c = rng.normal(size=3)
        c = radius * c / np.linalg.norm(c)
        W, H = sizes[v]
        cams.append(make_camera(look_at_rotation(c), c, W, H))
    return cams


# ----------------------------------------------------------------------------
# the five workloads
# ----------------------------------------------------------------------------

def make_frame64_1k(seed: int = 1) -> Scene:
    """1 view 64x64, 1,000 surfels, SH degree 0, forward only."""
    rng = np.random.default_rng(seed)
    n = 1000
    means = rng.uniform(-1.0, 1.0, size=(n, 3))
    scales, quats, opac = _draw_shape(rng, n)
    rgb = rng.uniform(0.0, 1.0, size=(n, 3))
    sh = _rgb_as_sh0(rgb)
    cam = make_camera(np.eye(3), np.array([0.0, 0.0, -4.0]), 64, 64)
    mask = ellipsoid_mask(cam, (0, 0, 0), (0.6, 0.6, 0.6))
    means, scales, quats, opac, sh = _f32(means, scales, quats, opac, sh)
    return Scene(means, scales, quats, opac, sh, 0, [cam], [mask], None, "frame64-1k")


def make_frame800_100k(seed: int = 2, n: int = 100_000, width: int = 800, height: int = 800) -> Scene:
    """1 view 800x800, 100k surfels, SH degree 3, random target and a random
    ellipsoid mask; forward + backward."""
    rng = np.random.default_rng(seed)
    means = rng.uniform(-1.0, 1.0, size=(n, 3))
    scales, quats, opac = _draw_shape(rng, n)
    sh = rng.normal(0.0, 0.2, size=(n, 16, 3))
    cam = make_camera(np.eye(3), np.array([0.0, 0.0, -4.0]), width, height)
    centre = rng.uniform(-0.3, 0.3, size=3)
    axes = rng.uniform(0.4, 1.0, size=3)
    rot = random_rotation(rng)
    mask = ellipsoid_mask(cam, centre, axes, rot)
    target = rng.uniform(0.0, 1.0, size=(3, height, width)).astype(np.float32)
    means, scales, quats, opac, sh = _f32(means, scales, quats, opac, sh)
    return Scene(means, scales, quats, opac, sh, 3, [cam], [mask], [target], "frame800-100k")


def make_ragged16_1m(seed: int = 3, n: int = 1_000_000, n_views: int = 16) -> Scene:
    """16 views of uneven resolution (sides uniform in 400..1600), 1M surfels
    (70% in the object ellipsoid, 30% background in [-3,3]^3), SH degree 3."""
    rng = np.random.default_rng(seed)
    means = _object_mixture(rng, n)
    scales, quats, opac = _draw_shape(rng, n)
    sh = rng.normal(0.0, 0.2, size=(n, 16, 3))
    sizes = [(int(rng.integers(400, 1601)), int(rng.integers(400, 1601))) for _ in range(n_views)]
    cams = _random_views(rng, n_views, 4.0, sizes)
    masks = [ellipsoid_mask(c, (0, 0, 0), OBJECT_AXES) for c in cams]
    targets = [rng.uniform(0.0, 1.0, size=(3, c.height, c.width)).astype(np.float32) for c in cams]
    means, scales, quats, opac, sh = _f32(means, scales, quats, opac, sh)
    return Scene(means, scales, quats, opac, sh, 3, cams, masks, targets, "ragged16-1m")


def make_shell100_3d(seed: int = 4, **kw):
    """The 3D-Gaussian counterpart of the shell scene for the pruning pass of
    Appendix B: the same centres, rotations and opacities; each surfel's two
    tangent scales plus a third (normal) scale of 0.1 times the smaller one,
    so the shell is a closed layer of thin, opaque 3D Gaussians.  Returns
    (scene, scales3 [N,3] float32)."""
    sc = make_shell100(seed, **kw)
    s = sc.scales.astype(np.float64)
    s3 = np.concatenate([s, 0.1 * s.min(axis=1, keepdims=True)], axis=1).astype(np.float32)
    return sc, s3


def make_shell100(seed: int = 4, n_shell: int = 300_000, n_inner: int = 700_000,
                 n_outer: int = 100_000, n_views: int = 100, size: int = 800) -> Scene:
    """Occlusion pruning workload: an opaque shell on the unit sphere
    (normals radial, opacity 0.99) hiding an interior ball of radius 0.6,
    plus exterior surfels in 1.5 <= r <= 3; 100 views on a Fibonacci sphere
    of radius 4.  No colour is used."""
    from scipy.spatial.transform import Rotation
    rng = np.random.default_rng(seed)
    # shell
    d = rng.normal(size=(n_shell, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    helper = np.where(np.abs(d[:, 0:1]) < 0.9, np.array([[1.0, 0, 0]]), np.array([[0, 1.0, 0]]))
    e1 = np.cross(helper, d)
    e1 /= np.linalg.norm(e1, axis=1, keepdims=True)
    e2 = np.cross(d, e1)
    spin = rng.uniform(0.0, 2.0 * math.pi, size=n_shell)[:, None]
    tu = np.cos(spin) * e1 + np.sin(spin) * e2
    tv = np.cross(d, tu)
    mats = np.stack([tu, tv, d], axis=2)          # columns: tangent u, tangent v, normal
    xyzw = Rotation.from_matrix(mats).as_quat()
    shell_q = np.concatenate([xyzw[:, 3:4], xyzw[:, :3]], axis=1)
    shell_s = np.exp(rng.uniform(math.log(0.01), math.log(0.1), size=(n_shell, 2)))
    shell_o = np.full(n_shell, 0.99)
    # interior and exterior
    inner = _uniform_in_shell(rng, n_inner, 0.0, 0.6)
    outer = _uniform_in_shell(rng, n_outer, 1.5, 3.0)
    s2, q2, o2 = _draw_shape(rng, n_inner + n_outer)
    means = np.concatenate([d, inner, outer], axis=0)
    scales = np.concatenate([shell_s, s2], axis=0)
    quats = np.concatenate([shell_q, q2], axis=0)
    opac = np.concatenate([shell_o, o2], axis=0)
    n = means.shape[0]
    sh = np.zeros((n, 1, 3))
    cams = []
    for c in fibonacci_sphere(n_views, 4.0):
        cams.append(make_camera(look_at_rotation(c), c, size, size))
    masks = [np.ones((size, size), np.uint8) for _ in cams]
    means, scales, quats, opac, sh = _f32(means, scales, quats, opac, sh)
    return Scene(means, scales, quats, opac, sh, 0, cams, masks, None, "shell100")


def make_wide8_3m(seed: int = 5, n: int = 3_000_000, n_views: int = 8) -> Scene:
    """Training-step workload: 3M surfels with the object/background mixture,
    SH degree 3, 8 views at 1960x1090 (fx = fy = 1697.41, cx = 980,
    cy = 545) on the radius-4 sphere."""
    rng = np.random.default_rng(seed)
    means = _object_mixture(rng, n)
    scales, quats, opac = _draw_shape(rng, n)
    sh = rng.normal(0.0, 0.2, size=(n, 16, 3))
    cams = []
    for _ in range(n_views):
        c = rng.normal(size=3)
        c = 4.0 * c / np.linalg.norm(c)
        cams.append(make_camera(look_at_rotation(c), c, 1960, 1090, fx=1697.41, fy=1697.41,
                                cx=980.0, cy=545.0))
    masks = [ellipsoid_mask(c, (0, 0, 0), OBJECT_AXES) for c in cams]
    targets = [rng.uniform(0.0, 1.0, size=(3, c.height, c.width)).astype(np.float32) for c in cams]
    means, scales, quats, opac, sh = _f32(means, scales, quats, opac, sh)
    return Scene(means, scales, quats, opac, sh, 3, cams, masks, targets, "wide8-3m")


def make_random_scene(seed: int, n: int, n_views: int = 1, width: int = 32, height: int = 32,
                      sh_degree: int = 0, spread: float = 1.0, radius: float = 4.0,
                      scale_range=(0.01, 0.1), with_targets: bool = True) -> Scene:
    """Small scene with the config-1 distributions, for parity and
    finite-difference checks (uneven sizes allowed via width/height lists)."""
    rng = np.random.default_rng(seed)
    means = rng.uniform(-spread, spread, size=(n, 3))
    scales = np.exp(rng.uniform(math.log(scale_range[0]), math.log(scale_range[1]), size=(n, 2)))
    quats = rng.normal(size=(n, 4))
    opac = 1.0 / (1.0 + np.exp(-rng.normal(size=n)))
    K = (sh_degree + 1) ** 2
    sh = rng.normal(0.0, 0.2, size=(n, K, 3))
    sh[:, 0, :] += rng.uniform(-0.5, 0.5, size=(n, 3)) / _Y00
    ws = width if isinstance(width, (list, tuple)) else [width] * n_views
    hs = height if isinstance(height, (list, tuple)) else [height] * n_views
    cams = []
    for v in range(n_views):
        if v == 0:
            R, c = np.eye(3), np.array([0.0, 0.0, -radius])
        else:
            c = rng.normal(size=3)
            c = radius * c / np.linalg.norm(c)
            R = look_at_rotation(c)
        cams.append(make_camera(R, c, ws[v], hs[v]))
    masks = []
    targets = [] if with_targets else None
    for cam in cams:
        centre = rng.uniform(-0.3, 0.3, size=3)
        axes = rng.uniform(0.4, 1.0, size=3)
        masks.append(ellipsoid_mask(cam, centre, axes, random_rotation(rng)))
        if with_targets:
            targets.append(rng.uniform(0, 1, size=(3, cam.height, cam.width)).astype(np.float32))
    means, scales, quats, opac, sh = _f32(means, scales, quats, opac, sh)
    return Scene(means, scales, quats, opac, sh, sh_degree, cams, masks, targets, f"random{seed}")


WORKLOADS = {"frame64-1k": make_frame64_1k, "frame800-100k": make_frame800_100k, "ragged16-1m": make_ragged16_1m,
             "shell100": make_shell100, "wide8-3m": make_wide8_3m}


def scene_digest(scene: Scene) -> str:
    """Hash of every array of a scene (reproducibility check)."""
    import hashlib
    h = hashlib.sha256()
    for a in (scene.means, scene.scales, scene.quats, scene.opac, scene.sh):
        h.update(np.ascontiguousarray(a).tobytes())
    for c in scene.cams:
        h.update(c.viewmat.tobytes())
        h.update(np.array([c.fx, c.fy, c.cx, c.cy, c.width, c.height], np.float64).tobytes())
    for m in scene.masks:
        h.update(m.tobytes())
    return h.hexdigest()
