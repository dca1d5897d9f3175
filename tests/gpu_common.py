"""Shared helpers of the GPU tests (device side through the C ABI)."""
import os

import numpy as np

import oracle
import scenes

LAM = 0.5
TAU = SIG = 1.0 / np.sqrt(12.0)


def dn():
    from paper_1604_03734_amd import build, denser
    if not os.path.exists(denser.LIB_PATH):
        build.build()
    denser.lib()
    return denser


def K4(cam):
    return [cam.fx, cam.fy, cam.cx, cam.cy]


def intr(D, cam):
    return D.intrinsics(cam.fx, cam.fy, cam.cx, cam.cy, cam.width, cam.height)


def to_dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    return t.detach().cpu().numpy()


def fuse_both(fr, max_blocks=8192, cap_log2=12, tail=256, check_each_frame=True):
    """Fuse a frame sequence with the oracle and with the GPU library and
    return both volumes, checking allocation bit-exactly per frame."""
    D = dn()
    cam = fr.camera
    ov = oracle.OracleVolume(fr.voxel_size, fr.mu, fr.max_depth, max_blocks, cap_log2, tail)
    gv = D.Volume(fr.voxel_size, fr.mu, fr.max_depth, max_blocks, cap_log2, tail,
                  max_points=cam.width * cam.height)
    K = intr(D, cam)
    for d, T in zip(fr.depths, fr.poses):
        n_o = ov.alloc(d, K4(cam), T)
        dd = to_dev(d)
        n_g = gv.alloc_blocks(dd, K, T)
        assert n_o == n_g
        if check_each_frame:
            np.testing.assert_array_equal(host(gv.extract(D.DN_X_CANDIDATES)), ov.last_candidates)
        ov.fuse(d, K4(cam), T)
        gv.fuse_depth(dd, K, T)
    return ov, gv


def state_of(D, gv):
    u = host(gv.extract(D.DN_X_U)).astype(np.float64)
    p = host(gv.extract(D.DN_X_P)).astype(np.float64)
    ub = host(gv.extract(D.DN_X_UBAR)).astype(np.float64)
    return u, ub, p
