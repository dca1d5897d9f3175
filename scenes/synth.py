"""Synthetic street-like scenes and depth maps (inputs only).

Scenes are unions of axis-aligned boxes (a thin box stands in for a plane).
A camera looks along +z of its own frame (x right, y down, z forward); a
pixel (x, y) has its centre at integer coordinates, so its ray in the camera
frame is r = ((x - cx)/fx, (y - cy)/fy, 1) and the depth of a hit is the
camera-frame z of the hit point, i.e. the ray parameter.

Noise follows a stereo camera: the true depth Z is turned into a disparity
fx*B/Z, Gaussian noise of sigma pixels is added, and the noisy disparity is
turned back into depth.  Pixels with no hit, a non-positive noisy disparity,
a depth beyond max_depth, or drawn invalid at the given rate are 0.

The paper evaluates on KITTI-VO (Section V); that dataset is not available,
so these seeded scenes stand in for it with the same kind of geometry
(forward-facing car camera, road plane, facades, parked cars).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class Camera:
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int


@dataclass
class Frames:
    """A sequence of depth maps with their camera->world poses."""
    camera: Camera
    depths: list            # list of float32 [H][W]
    poses: list             # list of float64 [4][4], camera -> world
    voxel_size: float
    mu: float
    max_depth: float
    meta: dict = field(default_factory=dict)


def pose_translation(tx: float, ty: float, tz: float) -> np.ndarray:
    T = np.eye(4)
    T[:3, 3] = (tx, ty, tz)
    return T


def pose_yaw(yaw: float, tx: float, ty: float, tz: float, pitch: float = 0.0) -> np.ndarray:
    """Camera->world pose rotated by `yaw` about the camera y axis and
    `pitch` about its x axis (radians), then translated."""
    cy, sy = np.cos(yaw), np.sin(yaw)
    cp, sp = np.cos(pitch), np.sin(pitch)
    Ry = np.array([[cy, 0.0, sy], [0.0, 1.0, 0.0], [-sy, 0.0, cy]])
    Rx = np.array([[1.0, 0.0, 0.0], [0.0, cp, -sp], [0.0, sp, cp]])
    T = np.eye(4)
    T[:3, :3] = Ry @ Rx
    T[:3, 3] = (tx, ty, tz)
    return T


def _rays_world(cam: Camera, pose: np.ndarray):
    xs = (np.arange(cam.width, dtype=np.float64) - cam.cx) / cam.fx
    ys = (np.arange(cam.height, dtype=np.float64) - cam.cy) / cam.fy
    rx, ry = np.meshgrid(xs, ys)                      # [H][W]
    r = np.stack([rx, ry, np.ones_like(rx)], axis=-1)  # camera frame, z = 1
    d = r @ pose[:3, :3].T                             # world direction
    return pose[:3, 3].copy(), d


def _pixel_window(lo, hi, cam: Camera, pose: np.ndarray):
    """Pixel rectangle that can see the box, for an unrotated camera; None
    if the box is entirely behind the camera.  Conservative (1 px margin)."""
    o = pose[:3, 3]
    zlo = max(lo[2], o[2] + 1e-3)
    if zlo >= hi[2]:
        return None
    xs, ys = [], []
    for x in (lo[0], hi[0]):
        for y in (lo[1], hi[1]):
            for z in (zlo, hi[2]):
                xs.append(cam.fx * (x - o[0]) / (z - o[2]) + cam.cx)
                ys.append(cam.fy * (y - o[1]) / (z - o[2]) + cam.cy)
    x0 = max(0, int(np.floor(min(xs))) - 1)
    x1 = min(cam.width, int(np.ceil(max(xs))) + 2)
    y0 = max(0, int(np.floor(min(ys))) - 1)
    y1 = min(cam.height, int(np.ceil(max(ys))) + 2)
    if x0 >= x1 or y0 >= y1:
        return None
    return y0, y1, x0, x1


def true_depth(boxes: np.ndarray, cam: Camera, pose: np.ndarray) -> np.ndarray:
    """Nearest positive hit parameter of each pixel ray against the boxes
    (float64 [H][W], +inf where nothing is hit).  boxes: [n][2][3] (lo, hi)."""
    o, d = _rays_world(cam, pose)
    best = np.full(d.shape[:2], np.inf)
    unrotated = np.array_equal(pose[:3, :3], np.eye(3))
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / d
        for lo, hi in boxes:
            if unrotated:
                win = _pixel_window(lo, hi, cam, pose)
                if win is None:
                    continue
                y0, y1, x0, x1 = win
            else:
                y0, y1, x0, x1 = 0, cam.height, 0, cam.width
            iv = inv[y0:y1, x0:x1]
            t0 = (lo - o) * iv
            t1 = (hi - o) * iv
            tn = np.nanmax(np.minimum(t0, t1), axis=-1)
            tf = np.nanmin(np.maximum(t0, t1), axis=-1)
            bw = best[y0:y1, x0:x1]
            hit = (tn <= tf) & (tn > 1e-6) & (tn < bw)
            best[y0:y1, x0:x1] = np.where(hit, tn, bw)
    return best


def render_depth(boxes, cam: Camera, pose, rng: np.random.Generator,
                 sigma_px: float, baseline: float, max_depth: float,
                 invalid_frac: float = 0.0) -> np.ndarray:
    Z = true_depth(boxes, cam, pose)
    hit = np.isfinite(Z)
    disp = np.where(hit, cam.fx * baseline / np.where(hit, Z, 1.0), 0.0)
    noisy = disp + rng.normal(0.0, sigma_px, size=disp.shape) if sigma_px > 0 else disp
    with np.errstate(divide="ignore"):
        Zn = np.where(noisy > 0, cam.fx * baseline / np.where(noisy > 0, noisy, 1.0), 0.0)
    ok = hit & (noisy > 0) & (Zn <= max_depth) & (Zn > 0)
    if invalid_frac > 0:
        ok &= rng.random(size=Zn.shape) >= invalid_frac
    return np.where(ok, Zn, 0.0).astype(np.float32)


def laser_scan(boxes: np.ndarray, pose: np.ndarray, seed: int, n_rings: int = 16, n_azimuth: int = 360,
               elev_deg=(-15.0, 15.0), sigma_m: float = 0.01, max_range: float = 50.0) -> np.ndarray:
    """A spinning range scanner at `pose` (sensor -> world; the sensor looks
    along +z, rings spread in elevation about the sensor x axis, azimuth
    about its y axis): float32 [n_rings * n_azimuth][3] returns in the
    sensor frame, range noise N(0, sigma_m) along the ray; returns with no
    hit or beyond max_range are NaN."""
    rng = np.random.default_rng(np.random.SeedSequence([11, seed]))
    el = np.deg2rad(np.linspace(elev_deg[0], elev_deg[1], n_rings))
    az = np.linspace(-np.pi, np.pi, n_azimuth, endpoint=False)
    E, A = np.meshgrid(el, az, indexing="ij")
    ds = np.stack([np.cos(E) * np.sin(A), -np.sin(E), np.cos(E) * np.cos(A)], -1).reshape(-1, 3)
    dw = ds @ pose[:3, :3].T
    o = pose[:3, 3]
    best = np.full(len(ds), np.inf)
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / dw
        for lo, hi in boxes:
            t0 = (lo - o) * inv
            t1 = (hi - o) * inv
            tn = np.nanmax(np.minimum(t0, t1), axis=-1)
            tf = np.nanmin(np.maximum(t0, t1), axis=-1)
            hit = (tn <= tf) & (tn > 1e-6) & (tn < best)
            best = np.where(hit, tn, best)
    r = best + rng.normal(0.0, sigma_m, size=best.shape)
    ok = np.isfinite(best) & (r > 0) & (r <= max_range)
    pts = np.where(ok[:, None], ds * np.where(ok, r, 0.0)[:, None], np.nan)
    return pts.astype(np.float32)


def _box(lo, hi):
    return np.array([lo, hi], dtype=np.float64)


# ---------------------------------------------------------------- config 1
def scene_c1() -> np.ndarray:
    """Ground plane, two walls and three boxes (the small parity scene)."""
    b = [
        _box((-6.0, 1.2, -2.0), (6.0, 1.4, 24.0)),     # ground, y down => below camera
        _box((-4.2, -2.0, -2.0), (-4.0, 1.2, 24.0)),   # left wall x = -4
        _box((4.0, -2.0, -2.0), (4.2, 1.2, 24.0)),     # right wall x = +4
        _box((-2.1, 0.2, 7.4), (-0.9, 1.2, 8.6)),      # box A, centre (-1.5, 0.7, 8)
        _box((1.3, -0.3, 10.5), (2.3, 1.2, 11.5)),     # box B, centre (1.8, 0.45, 11)
        _box((-0.8, 0.0, 14.2), (0.8, 1.2, 15.8)),     # box C, centre (0, 0.6, 15)
    ]
    return np.stack(b)


C1_CAMERA = Camera(300.0, 300.0, 159.5, 47.5, 320, 96)


def frames_c1(seed: int = 0, n_frames: int = 4, sigma_px: float = 0.3) -> Frames:
    """Config 1: 4 depth maps of 320x96 along a 2 m straight path."""
    boxes = scene_c1()
    cam = C1_CAMERA
    depths, poses = [], []
    for k in range(n_frames):
        T = pose_translation(0.0, 0.0, 2.0 * k / max(1, n_frames - 1))
        rng = np.random.default_rng(np.random.SeedSequence([1, seed, k]))
        depths.append(render_depth(boxes, cam, T, rng, sigma_px, 0.54, 20.0))
        poses.append(T)
    return Frames(cam, depths, poses, voxel_size=0.1, mu=0.3, max_depth=20.0,
                  meta={"config": "c1", "seed": seed})


# ------------------------------------------------------------ street scenes
def scene_street(length: float, seed: int, config_id: int = 2) -> np.ndarray:
    """Procedural street along +z: road plane, facades with a seeded setback
    per 10 m segment, parked-car boxes with seeded gaps, and an end wall."""
    rng = np.random.default_rng(np.random.SeedSequence([config_id, seed, 1_000_003]))
    b = [_box((-25.0, 1.65, -10.0), (25.0, 1.85, length + 15.0))]          # road
    nseg = int(np.ceil((length + 10.0) / 10.0))
    for j in range(nseg):
        z0, z1 = 10.0 * j - 5.0, 10.0 * j + 5.0
        for side in (-1.0, 1.0):
            X = 7.0 + rng.uniform(0.0, 1.5)
            h = rng.uniform(8.0, 16.0)
            lo = (side * X, -h, z0) if side > 0 else (-X - 1.0, -h, z0)
            hi = (side * X + 1.0, 1.65, z1) if side > 0 else (-X, 1.65, z1)
            b.append(_box(lo, hi))
    for side in (-1.0, 1.0):
        z = -3.0 + rng.uniform(0.0, 4.0)
        while z < length + 5.0:
            cx = side * 5.5
            b.append(_box((cx - 0.9, 0.15, z), (cx + 0.9, 1.65, z + 4.2)))
            z += 4.2 + rng.uniform(1.0, 6.0)
    b.append(_box((-20.0, -20.0, length + 10.0), (20.0, 1.65, length + 11.0)))  # end wall
    return np.stack(b)


C2_CAMERA = Camera(700.0, 700.0, 620.5, 187.0, 1242, 375)


def frames_street(length: float = 100.0, n_frames: int = 100, seed: int = 0,
                  config_id: int = 2, camera: Camera = C2_CAMERA,
                  sigma_px: float = 0.5, invalid_frac: float = 0.05,
                  voxel_size: float = 0.2, mu: float = 0.6,
                  max_depth: float = 50.0) -> Frames:
    boxes = scene_street(length, seed, config_id)
    depths, poses = [], []
    step = length / max(1, n_frames)
    for k in range(n_frames):
        T = pose_translation(0.0, 0.0, k * step)
        rng = np.random.default_rng(np.random.SeedSequence([config_id, seed, k]))
        depths.append(render_depth(boxes, camera, T, rng, sigma_px, 0.54,
                                   max_depth, invalid_frac))
        poses.append(T)
    return Frames(camera, depths, poses, voxel_size, mu, max_depth,
                  meta={"config": f"street{config_id}", "seed": seed,
                        "length_m": length})


def frames_c2(seed: int = 0, n_frames: int = 100) -> Frames:
    """Config 2: 100 depth maps of 1242x375 along a 100 m street."""
    return frames_street(100.0, n_frames, seed, config_id=2)


# ------------------------------------------------------ direct block fields
def random_block_field(n_blocks: int, seed: int, extent: int = 6,
                       omega_frac: float = 0.8, max_w: int = 4):
    """A random set of distinct block keys inside a cube of `extent` blocks
    per axis, with random fused values f in [-1, 1] and integer weights
    w in {0..max_w} (w == 0 marks unobserved voxels).  Used to exercise the
    operators on arbitrary sparsity patterns without running fusion."""
    rng = np.random.default_rng(np.random.SeedSequence([7, seed, n_blocks]))
    cells = rng.choice(extent ** 3, size=n_blocks, replace=False)
    coords = np.stack([cells % extent, (cells // extent) % extent,
                       cells // (extent * extent)], axis=1).astype(np.int32)
    coords -= extent // 2
    f = rng.uniform(-1.0, 1.0, size=(n_blocks, 512))
    w = rng.integers(1, max_w + 1, size=(n_blocks, 512)).astype(np.float64)
    w[rng.random(size=w.shape) >= omega_frac] = 0.0
    f[w == 0] = 0.0
    return coords, f, w


def c4_block_counts(n: int = 64, seed: int = 0, lo: float = 1e3, hi: float = 5e4):
    """Sub-map sizes for the batched workload: log-uniform in [lo, hi]."""
    rng = np.random.default_rng(np.random.SeedSequence([4, seed]))
    return np.round(np.exp(rng.uniform(np.log(lo), np.log(hi), size=n))).astype(np.int64)


def inside_scene(points: np.ndarray, boxes: np.ndarray, chunk: int = 65536) -> np.ndarray:
    """True for each point (float [n][3], metres) strictly inside one of the
    scene's solid boxes."""
    out = np.zeros(len(points), bool)
    for s0 in range(0, len(points), chunk):
        P = np.asarray(points[s0:s0 + chunk], np.float64)
        hit = np.zeros(len(P), bool)
        for lo, hi in boxes:
            hit |= np.all((P > lo) & (P < hi), axis=1)
        out[s0:s0 + chunk] = hit
    return out


def distance_to_scene(points: np.ndarray, boxes: np.ndarray, chunk: int = 65536) -> np.ndarray:
    """Unsigned distance of each point (float [n][3], metres) to the nearest
    box surface of the scene (ground truth for accuracy statistics)."""
    out = np.empty(len(points))
    for s0 in range(0, len(points), chunk):
        P = np.asarray(points[s0:s0 + chunk], np.float64)
        best = np.full(len(P), np.inf)
        for lo, hi in boxes:
            d_out = np.linalg.norm(np.maximum(np.maximum(lo - P, P - hi), 0.0), axis=1)
            d_in = np.min(np.minimum(P - lo, hi - P), axis=1)
            d = np.where(d_out > 0, d_out, np.maximum(d_in, 0.0))
            best = np.minimum(best, d)
        out[s0:s0 + chunk] = best
    return out
