"""Pins of the oracle's laser fusion (Section III-A: the update along each
ray from the sensor to mu behind the return) against geometry computed
here: blocks and voxels met by a segment from an exact segment/box test,
the truncated distance of each voxel in closed form, the per-scan mean
over rays, invalid returns.  CPU only."""
import numpy as np
import pytest

import oracle
import scenes

S, MU, MAXD = 0.1, 0.3, 20.0


def _hits_box(A, B, lo, hi):
    d = B - A
    t0, t1 = 0.0, 1.0
    for i in range(3):
        if abs(d[i]) < 1e-300:
            if A[i] < lo[i] or A[i] > hi[i]:
                return False
            continue
        a, b = (lo[i] - A[i]) / d[i], (hi[i] - A[i]) / d[i]
        a, b = min(a, b), max(a, b)
        t0, t1 = max(t0, a), min(t1, b)
    return t0 <= t1


def _cells_on_segment(A, B, cell):
    lo = np.floor(np.minimum(A, B) / cell).astype(int) - 1
    hi = np.floor(np.maximum(A, B) / cell).astype(int) + 1
    out = set()
    for x in range(lo[0], hi[0] + 1):
        for y in range(lo[1], hi[1] + 1):
            for z in range(lo[2], hi[2] + 1):
                c = np.array([x, y, z], float)
                if _hits_box(A, B, c * cell, (c + 1) * cell):
                    out.add((x, y, z))
    return out


def _pose(seed):
    rng = np.random.default_rng(seed)
    return scenes.pose_yaw(rng.uniform(-0.6, 0.6), *rng.uniform(-0.35, 0.35, 3), rng.uniform(-0.3, 0.3))


def _ray(T, p, rho):
    r = np.linalg.norm(p)
    return T[:3, :3] @ (rho * p / r) + T[:3, 3]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_single_return_allocation_and_values(seed):
    rng = np.random.default_rng(100 + seed)
    T = _pose(seed)
    p = np.array([rng.uniform(-0.4, 0.4), rng.uniform(-0.4, 0.4), rng.uniform(0.8, 1.6)], np.float32)
    r = float(np.linalg.norm(p.astype(np.float64)))
    ov = oracle.OracleVolume(S, MU, MAXD, 4096, 12, 256)
    assert ov.alloc_laser(p[None], T) > 0
    # the allocated blocks are the blocks the band segment meets
    band = _cells_on_segment(_ray(T, p.astype(float), r - MU), _ray(T, p.astype(float), r + MU), 8 * S)
    assert set(map(tuple, ov.coords.tolist())) == band
    ov.fuse_laser(p[None], T)
    # every voxel of an allocated block that the ray [0, r + mu] meets, with
    # eta >= -mu, has w = 1 and f = min(1, eta / mu); no other voxel changed
    o = T[:3, 3]
    D = T[:3, :3] @ (p.astype(float) / r)
    cells = _cells_on_segment(_ray(T, p.astype(float), 0.0), _ray(T, p.astype(float), r + MU), S)
    expect_w = np.zeros_like(ov.w)
    expect_f = np.zeros_like(ov.f)
    index = {tuple(c): i for i, c in enumerate(ov.coords.tolist())}
    for g in cells:
        b = index.get(tuple(int(np.floor(x / 8)) for x in g))
        if b is None:
            continue
        eta = r - (((np.array(g) + 0.5) * S - o) @ D)
        if eta < -MU:
            continue
        v = (g[0] % 8) + 8 * (g[1] % 8) + 64 * (g[2] % 8)
        expect_w[b, v] = 1.0
        expect_f[b, v] = min(1.0, eta / MU)
    np.testing.assert_array_equal(ov.w, expect_w)
    assert np.abs(ov.f - expect_f).max() < 1e-12
    assert expect_w.sum() > 5


def test_scan_mean_over_rays_and_two_scans():
    """Rays of one scan meeting a voxel are averaged; a second scan gives
    the pooled mean (w counts observations)."""
    rng = np.random.default_rng(7)
    T = _pose(3)
    pts = np.stack([rng.uniform(-0.3, 0.3, 40), rng.uniform(-0.3, 0.3, 40), rng.uniform(1.0, 1.3, 40)], 1)
    pts = pts.astype(np.float32)
    ov = oracle.OracleVolume(S, MU, MAXD, 4096, 12, 256)
    ov.alloc_laser(pts, T)
    obs = {}
    o = T[:3, 3]
    index = {tuple(c): i for i, c in enumerate(ov.coords.tolist())}

    def observe(P):
        for p in P.astype(np.float64):
            r = np.linalg.norm(p)
            D = T[:3, :3] @ (p / r)
            for g in _cells_on_segment(_ray(T, p, 0.0), _ray(T, p, r + MU), S):
                b = index.get(tuple(int(np.floor(x / 8)) for x in g))
                if b is None:
                    continue
                eta = r - (((np.array(g) + 0.5) * S - o) @ D)
                if eta >= -MU:
                    obs.setdefault((b, (g[0] % 8) + 8 * (g[1] % 8) + 64 * (g[2] % 8)), []).append(min(1.0, eta / MU))

    ov.fuse_laser(pts[:25], T)
    ov.fuse_laser(pts[25:], T)
    observe(pts)
    assert len(obs) > 50
    for (b, v), ps in obs.items():
        assert ov.w[b, v] == len(ps)
        assert abs(ov.f[b, v] - np.mean(ps)) < 1e-12
    assert ov.w.sum() == sum(len(x) for x in obs.values())


def test_invalid_returns_change_nothing():
    T = _pose(5)
    good = np.array([[0.1, -0.2, 1.2]], np.float32)
    ov = oracle.OracleVolume(S, MU, MAXD, 4096, 12, 256)
    ov.alloc_laser(good, T)
    bad = np.array([[np.nan, 0.0, 1.0], [0.0, 0.0, 0.0], [0.0, 0.0, 25.0], [np.inf, 1.0, 1.0]], np.float32)
    nb = ov.nb
    assert ov.alloc_laser(bad, T) == 0 and ov.nb == nb
    f0, w0 = ov.f.copy(), ov.w.copy()
    ov.fuse_laser(bad, T)
    np.testing.assert_array_equal(ov.f, f0)
    np.testing.assert_array_equal(ov.w, w0)
