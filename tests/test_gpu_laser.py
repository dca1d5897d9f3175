"""Laser range fusion on the GPU against the oracle: allocation (block
keys, pool order, hash slots, neighbour table) and weights bit-exact,
f within 1e-5, over several scans, interleaved with depth maps into the
same block pool, and with invalid returns."""
import numpy as np
import pytest

import oracle
import scenes
from gpu_common import K4, dn, host, intr, to_dev

pytestmark = pytest.mark.gpu

# room for scans of up to 24 x 720 returns within 20 m (and 320 x 96 depth maps)
LASER = dict(max_points=1 << 15, max_observations=24 * 720 * (4 + int(np.sqrt(3.0) * 20.3 / 0.1)))


def _check(D, ov, gv):
    assert gv.num_blocks == ov.nb
    np.testing.assert_array_equal(host(gv.extract(D.DN_X_COORDS)), ov.coords)
    np.testing.assert_array_equal(host(gv.extract(D.DN_X_HASH)), ov.slots)
    np.testing.assert_array_equal(host(gv.extract(D.DN_X_NBR)), ov.nbr)
    np.testing.assert_array_equal(host(gv.extract(D.DN_X_W)), ov.w)
    err = np.abs(host(gv.extract(D.DN_X_F)) - ov.f).max() if ov.nb else 0.0
    assert err <= 1e-5, err
    return err


def _poses():
    return [scenes.pose_yaw(0.0, 0.0, 0.0, 0.0), scenes.pose_yaw(0.15, 0.3, -0.1, 0.7),
            scenes.pose_yaw(-0.2, -0.4, 0.1, 1.4, 0.05)]


def test_laser_scans_match_the_oracle():
    D = dn()
    boxes = scenes.scene_c1()
    ov = oracle.OracleVolume(0.1, 0.3, 20.0, 8192, 12, 256)
    gv = D.Volume(0.1, 0.3, 20.0, 8192, 12, 256, **LASER)
    for k, T in enumerate(_poses()):
        pts = scenes.laser_scan(boxes, T, k, n_rings=24, n_azimuth=720)
        n_o = ov.alloc_laser(pts, T)
        dp = to_dev(pts)
        n_g = gv.alloc_laser(dp, T)
        assert n_o == n_g
        np.testing.assert_array_equal(host(gv.extract(D.DN_X_CANDIDATES)), ov.last_candidates)
        ov.fuse_laser(pts, T)
        gv.fuse_laser(dp, T)
        err = _check(D, ov, gv)
        print(f"scan {k}: {n_g} new blocks, {gv.num_blocks} total, max |df| {err:.2e}")
    assert (ov.w > 1).sum() > 1000


def test_laser_and_depth_share_the_block_pool():
    D = dn()
    fr = scenes.frames_c1(0, n_frames=2)
    boxes = scenes.scene_c1()
    cam = fr.camera
    ov = oracle.OracleVolume(0.1, 0.3, 20.0, 8192, 12, 256)
    gv = D.Volume(0.1, 0.3, 20.0, 8192, 12, 256, **LASER)
    K = intr(D, cam)
    for k, (d, T) in enumerate(zip(fr.depths, fr.poses)):
        assert ov.alloc(d, K4(cam), T) == gv.alloc_blocks(to_dev(d), K, T)
        ov.fuse(d, K4(cam), T)
        gv.fuse_depth(to_dev(d), K, T)
        pts = scenes.laser_scan(boxes, T, 10 + k)
        assert ov.alloc_laser(pts, T) == gv.alloc_laser(to_dev(pts), T)
        ov.fuse_laser(pts, T)
        gv.fuse_laser(to_dev(pts), T)
        _check(D, ov, gv)


def test_invalid_and_empty_scans_change_nothing():
    D = dn()
    boxes = scenes.scene_c1()
    T = _poses()[1]
    gv = D.Volume(0.1, 0.3, 20.0, 4096, 12, 256, **LASER)
    pts = scenes.laser_scan(boxes, T, 3)
    gv.integrate_laser(to_dev(pts), T)
    nb = gv.num_blocks
    f0, w0 = host(gv.extract(D.DN_X_F)), host(gv.extract(D.DN_X_W))
    bad = np.array([[np.nan, 0, 1], [0, 0, 0], [0, 0, 25.0], [np.inf, 1, 1]], np.float32)
    assert gv.integrate_laser(to_dev(bad), T) == 0
    assert gv.integrate_laser(to_dev(np.zeros((0, 3), np.float32)), T) == 0
    assert gv.num_blocks == nb
    np.testing.assert_array_equal(host(gv.extract(D.DN_X_F)), f0)
    np.testing.assert_array_equal(host(gv.extract(D.DN_X_W)), w0)


def test_scans_of_one_and_three_returns():
    """The smallest scans: a handful of observations (the scan's scratch
    holds them, their sorted copies, the per-voxel counts and the count)."""
    D = dn()
    ov = oracle.OracleVolume(0.1, 0.3, 20.0, 1024, 10, 128)
    gv = D.Volume(0.1, 0.3, 20.0, 1024, 10, 128, **LASER)
    T = _poses()[0]
    for pts in (np.array([[2.0, 0.1, 0.05]], np.float32),
                np.array([[1.5, 0.0, 0.0], [0.3, 1.1, 0.2], [-0.7, 0.2, 2.5]], np.float32)):
        assert ov.alloc_laser(pts, T) == gv.alloc_laser(to_dev(pts), T)
        ov.fuse_laser(pts, T)
        gv.fuse_laser(to_dev(pts), T)
        _check(D, ov, gv)
    assert (ov.w > 0).sum() > 0
