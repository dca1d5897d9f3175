"""Network kernels (BF16 MFMA, FP32 accumulation) against the FP64 oracle:
gather, forward, loss gradient (all three layers), Adam, warm start.

Forward output and warm-start fields: against the oracle network on the
same bfloat16 operands (relative L2 <= 1e-3) and against the float64
network (L2 within twice the oracle's model of the bfloat16 rounding); see
gpu_common.net_forward_checks.  Gradients: relative L2 <= 1e-2 against the
float64 oracle for every layer.  Whether a ReLU is open is a discrete
decision that floating point takes; for the gradients it is taken in the
network's own precision on both sides (the oracle's gate 1: the sign of a
pre-activation computed from bfloat16-rounded operands), the values are
compared in float64.  The errors against the oracle with float64 decisions
(gate 0) are printed beside them."""
import numpy as np
import pytest

import oracle
import scenes
from gpu_common import dn, dual_warm_start_checks, fuse_both, host, net_forward_checks, to_dev

pytestmark = pytest.mark.gpu


def _rel_l2(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)


def _cos(a, b):
    return float(np.dot(a.ravel(), b.ravel()) / (np.linalg.norm(a) * np.linalg.norm(b)))


BAR = 1e-2


def _params(seed, scale=0.15):
    rng = np.random.default_rng(seed)
    p = rng.normal(0, scale, oracle.NET_PARAMS)
    return p


def test_gather_matches_oracle():
    D = dn()
    import torch
    fr = scenes.frames_c1(0, n_frames=2)
    ov, gv = fuse_both(fr, check_each_frame=False)
    blocks = np.arange(0, gv.num_blocks, 3, dtype=np.int32)
    tiles = torch.empty((len(blocks), 2, 10, 10, 10), device="cuda")
    gv.net_gather(to_dev(blocks), tiles)
    ref = oracle.net_gather(ov.nbr, host(gv.extract(D.DN_X_F)).astype(np.float64), ov.w, blocks)
    assert np.abs(host(tiles) - ref).max() <= 1e-6


@pytest.mark.parametrize("seed,B", [(0, 1), (1, 7)])
def test_forward_matches_oracle(seed, B):
    D = dn()
    import torch
    rng = np.random.default_rng(10 + seed)
    tiles = rng.normal(0, 0.6, (B, 2, 10, 10, 10))
    prm = _params(seed)
    out = torch.empty((B, 10, 10, 10), device="cuda")
    D.net_forward(to_dev(tiles, torch.float32), to_dev(prm, torch.float32), out)
    torch.cuda.synchronize()
    net_forward_checks(host(out).astype(np.float64), tiles, prm, f"forward B={B}")


def test_loss_gradient_matches_oracle():
    D = dn()
    import torch
    rng = np.random.default_rng(3)
    B = 6
    tiles = rng.normal(0, 0.6, (B, 2, 10, 10, 10))
    targets = rng.normal(0, 0.5, (B, 512))
    mask = (rng.random((B, 512)) < 0.6).astype(np.float64)
    prm = _params(4)
    grad = torch.empty(oracle.NET_PARAMS, device="cuda")
    loss = D.net_loss_grad(to_dev(tiles, torch.float32), to_dev(prm, torch.float32),
                           to_dev(targets, torch.float32), to_dev(mask, torch.float32), grad)
    L, g_ref = oracle.net_loss_grad(tiles, prm, targets, mask, gate=1)
    _, g_ref0 = oracle.net_loss_grad(tiles, prm, targets, mask)
    g = host(grad).astype(np.float64)
    print(f"loss {loss:.6e} oracle {L:.6e}")
    assert abs(loss - L) <= BAR * abs(L)
    for lo, hi, name in [(0, 880, "layer1"), (880, 7808, "layer2"), (7808, 8241, "layer3")]:
        rel, cos = _rel_l2(g[lo:hi], g_ref[lo:hi]), _cos(g[lo:hi], g_ref[lo:hi])
        print(f"{name}: rel-L2 {rel:.3e} cos {cos:.6f} (float64 decisions: rel-L2 "
              f"{_rel_l2(g[lo:hi], g_ref0[lo:hi]):.3e})")
        assert rel <= BAR and cos >= 0.999, name


def test_adam_step():
    D = dn()
    import torch
    rng = np.random.default_rng(5)
    n = 1000
    p = rng.normal(size=n); g = rng.normal(size=n); m = rng.normal(size=n) * 0.1; v = rng.random(n) * 0.1
    tp, tg, tm, tv = (to_dev(a, torch.float32) for a in (p, g, m, v))
    D.net_adam(tp, tg, tm, tv, 1e-2, 3)
    torch.cuda.synchronize()
    b1, b2, eps = 0.9, 0.999, 1e-8
    m2 = b1 * m + (1 - b1) * g
    v2 = b2 * v + (1 - b2) * g * g
    p2 = p - 1e-2 * (m2 / (1 - b1 ** 3)) / (np.sqrt(v2 / (1 - b2 ** 3)) + eps)
    assert np.abs(host(tp) - p2).max() <= 1e-5


def test_warm_start_fields():
    D = dn()
    import torch
    fr = scenes.frames_c1(0, n_frames=2)
    ov, gv = fuse_both(fr, check_each_frame=False)
    prm = _params(7, 0.05)
    nb = gv.num_blocks
    u0 = torch.empty((nb, 512), device="cuda")
    p0 = torch.empty((3, nb, 512), device="cuda")
    gv.net_warm_start(to_dev(prm, torch.float32), u0, p0, mode=D.DN_WARM_PRIMAL, delta=0.1)
    torch.cuda.synchronize()
    f = host(gv.extract(D.DN_X_F)).astype(np.float64)
    w = ov.w
    tiles = oracle.net_gather(ov.nbr, f, w, np.arange(nb, dtype=np.int32))
    gu = host(u0).astype(np.float64)
    om = w > 0
    # u0 = clip(f + r) on Omega: compare the network part r = u0 - f where
    # the clip is inactive on both sides
    r_dev = np.zeros((nb, 10, 10, 10))
    r_dev[:, 1:9, 1:9, 1:9] = (gu - f).reshape(nb, 8, 8, 8)
    keep = np.zeros((nb, 10, 10, 10), bool)
    r64 = oracle.net_forward(tiles, prm, gate=0)[:, 1:9, 1:9, 1:9].reshape(nb, 512)
    inner = om & (np.abs(gu) < 1) & (np.abs(f + r64) < 1)
    keep[:, 1:9, 1:9, 1:9] = inner.reshape(nb, 8, 8, 8)
    net_forward_checks(r_dev, tiles, prm, "primal warm start", region=lambda a: a[keep])
    ref = np.where(om, np.clip(f + r64, -1, 1), 0.0)
    print(f"primal warm start: rel-L2 to the float64 fields {_rel_l2(gu[om], ref[om]):.3e}")
    assert (gu[w == 0] == 0).all()
    g = oracle.grad(ov.nbr, w, gu) / 0.1
    nrm = np.maximum(1.0, np.sqrt((g ** 2).sum(0)))
    assert np.abs(host(p0) - g / nrm).max() <= 1e-5


@pytest.mark.parametrize("perm", [1, 2])
def test_permuted_gather_matches_oracle(perm):
    D = dn()
    import torch
    fr = scenes.frames_c1(0, n_frames=2)
    ov, gv = fuse_both(fr, check_each_frame=False)
    blocks = np.arange(0, gv.num_blocks, 5, dtype=np.int32)
    tiles = torch.empty((len(blocks), 2, 10, 10, 10), device="cuda")
    gv.net_gather(to_dev(blocks), tiles, perm=perm)
    ref = oracle.net_gather(ov.nbr, host(gv.extract(D.DN_X_F)).astype(np.float64), ov.w, blocks, perm)
    assert np.abs(host(tiles) - ref).max() <= 1e-6


def test_dual_kind_loss_gradient_matches_oracle():
    D = dn()
    import torch
    rng = np.random.default_rng(8)
    B = 5
    tiles = rng.normal(0, 0.6, (B, 2, 10, 10, 10))
    targets = rng.uniform(-1, 1, (B, 512))
    mask = (rng.random((B, 512)) < 0.5).astype(np.float64)
    prm = _params(9)
    grad = torch.empty(oracle.NET_PARAMS, device="cuda")
    loss = D.net_loss_grad(to_dev(tiles, torch.float32), to_dev(prm, torch.float32),
                           to_dev(targets, torch.float32), to_dev(mask, torch.float32), grad, kind=1)
    L, g_ref = oracle.net_loss_grad(tiles, prm, targets, mask, kind=1, gate=1)
    _, g_ref0 = oracle.net_loss_grad(tiles, prm, targets, mask, kind=1)
    g = host(grad).astype(np.float64)
    print(f"dual kind loss {loss:.6e} oracle {L:.6e}")
    assert abs(loss - L) <= BAR * abs(L)
    for lo, hi, name in [(0, 880, "layer1"), (880, 7808, "layer2"), (7808, 8241, "layer3")]:
        rel = _rel_l2(g[lo:hi], g_ref[lo:hi])
        print(f"dual kind {name}: rel-L2 {rel:.3e} (float64 decisions: {_rel_l2(g[lo:hi], g_ref0[lo:hi]):.3e})")
        assert rel <= BAR and _cos(g[lo:hi], g_ref[lo:hi]) >= 0.999, name


def test_dual_warm_start_matches_oracle():
    """DN_WARM_DUAL: p_a = network output on the tile whose x axis is a,
    masked by m_a, projected onto the unit ball; u0 = f on Omega."""
    D = dn()
    import torch
    fr = scenes.frames_c1(0, n_frames=2)
    ov, gv = fuse_both(fr, check_each_frame=False)
    prm = _params(11, 0.1)
    nb = gv.num_blocks
    u0 = torch.empty((nb, 512), device="cuda")
    p0 = torch.empty((3, nb, 512), device="cuda")
    gv.net_warm_start(to_dev(prm, torch.float32), u0, p0, mode=D.DN_WARM_DUAL)
    torch.cuda.synchronize()
    f = host(gv.extract(D.DN_X_F)).astype(np.float64)
    em = host(gv.extract(D.DN_X_EMASK))
    dual_warm_start_checks(host(p0).astype(np.float64), ov.nbr, f, ov.w, np.arange(nb, dtype=np.int32), em, prm,
                           "dual warm start")
    assert np.array_equal(host(u0), np.where(ov.w > 0, f, 0.0).astype(np.float32))


def test_loss_gradient_over_more_tiles_than_workgroups():
    """The weight-gradient kernel keeps one partial per workgroup and loops
    over tiles: 260 tiles (more than its 256 workgroups) against the oracle."""
    D = dn()
    import torch
    rng = np.random.default_rng(13)
    B = 260
    tiles = rng.normal(0, 0.5, (B, 2, 10, 10, 10))
    targets = rng.normal(0, 0.5, (B, 512))
    mask = (rng.random((B, 512)) < 0.5).astype(np.float64)
    prm = _params(14, 0.12)
    grad = torch.empty(oracle.NET_PARAMS, device="cuda")
    loss = D.net_loss_grad(to_dev(tiles, torch.float32), to_dev(prm, torch.float32),
                           to_dev(targets, torch.float32), to_dev(mask, torch.float32), grad, kind=1)
    L, g_ref = oracle.net_loss_grad(tiles, prm, targets, mask, kind=1, gate=1)
    g = host(grad).astype(np.float64)
    print(f"260 tiles: loss {loss:.6e} oracle {L:.6e}")
    assert abs(loss - L) <= BAR * abs(L)
    for lo, hi, name in [(0, 880, "layer1"), (880, 7808, "layer2"), (7808, 8241, "layer3")]:
        rel = _rel_l2(g[lo:hi], g_ref[lo:hi])
        print(f"260 tiles {name}: rel-L2 {rel:.3e}")
        assert rel <= BAR, name
