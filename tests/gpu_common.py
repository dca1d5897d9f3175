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


# Network outputs are compared twice: with the oracle network evaluated on
# the same bfloat16 operands with float64 sums (gate 2), where only the
# order and precision of the sums differ (relative L2 <= NET_EMU_BAR), and
# with the float64 network (gate 0), where the difference is the bfloat16
# rounding itself: its L2 norm stays within NET_RMS_FACTOR of the norm the
# oracle's variance model of that rounding predicts (oracle.net_error_rms).
# A clip or a projection onto the unit ball after the network is
# 1-Lipschitz, so the same bars hold after it.
NET_EMU_BAR = 1e-3
NET_RMS_FACTOR = 2.0


def net_forward_checks(g, tiles, prm, label, region=None):
    """g: device outputs [B][10][10][10] (float64) for `tiles`; region: a
    function cropping/arranging a [B][10][10][10] field (default: all)."""
    region = region or (lambda a: a)
    r2 = region(oracle.net_forward(tiles, prm, gate=2))
    r0 = region(oracle.net_forward(tiles, prm, gate=0))
    sig = np.linalg.norm(region(oracle.net_error_rms(tiles, prm)))
    g = region(g)
    emu = np.linalg.norm(g - r2) / np.linalg.norm(r2)
    d0 = np.linalg.norm(g - r0)
    print(f"{label}: rel-L2 to bfloat16-operand network {emu:.3e}; to float64 network "
          f"{d0 / np.linalg.norm(r0):.3e}, {d0 / sig:.2f} x the modelled rounding")
    assert emu <= NET_EMU_BAR, label
    assert d0 <= NET_RMS_FACTOR * sig, label


def _dual_fields(nbr, f, w, blocks, em, field):
    """field(tiles) -> [B][10][10][10] for each axis a, cropped to the
    centre, put back in block voxel order and masked by m_a: [3][B][512]."""
    out = np.zeros((3, len(blocks), 512))
    for a in range(3):
        c = field(oracle.net_gather(nbr, f, w, blocks, a))[:, 1:9, 1:9, 1:9]
        if a == 1:
            c = c.transpose(0, 1, 3, 2)
        elif a == 2:
            c = c.transpose(0, 3, 2, 1)
        out[a] = np.where((em >> (a + 1)) & 1, c.reshape(len(blocks), 512), 0.0)
    return out


def dual_warm_start_checks(gp, nbr, f, w, blocks, em, prm, label):
    """gp: device p0 [3][B][512] (float64) of the dual warm start on
    `blocks`; em: their edge masks.  The network's output on the tile of
    each axis, masked, projected voxel by voxel onto the unit ball."""
    f = np.asarray(f, np.float64)
    w = np.asarray(w, np.float64)
    proj = lambda r: r / np.maximum(1.0, np.sqrt((r ** 2).sum(0)))  # noqa: E731
    r2 = proj(_dual_fields(nbr, f, w, blocks, em, lambda t: oracle.net_forward(t, prm, gate=2)))
    r0 = proj(_dual_fields(nbr, f, w, blocks, em, lambda t: oracle.net_forward(t, prm, gate=0)))
    sig = np.linalg.norm(_dual_fields(nbr, f, w, blocks, em, lambda t: oracle.net_error_rms(t, prm)))
    emu = np.linalg.norm(gp - r2) / np.linalg.norm(r2)
    d0 = np.linalg.norm(gp - r0)
    print(f"{label}: rel-L2 to bfloat16-operand network {emu:.3e}; to float64 network "
          f"{d0 / np.linalg.norm(r0):.3e}, {d0 / sig:.2f} x the modelled rounding")
    assert emu <= NET_EMU_BAR, label
    assert d0 <= NET_RMS_FACTOR * sig, label
