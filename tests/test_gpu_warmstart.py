"""Learned warm start: trained on the GPU by the library's own kernels on
pairs the method generates, evaluated on a held-out street against the
plain solver, with the fallback to a cold start."""
import numpy as np
import pytest

import scenes
from gpu_common import dn

pytestmark = pytest.mark.gpu

TOL = 1e-3


@pytest.fixture(scope="module")
def trained():
    import torch
    from paper_1604_03734_amd import warmstart as W
    tiles, tgt, msk = W.make_pairs(seeds=(1001, 1002), n_pairs=3000, length=60.0, n_frames=60)
    p, hist = W.train(tiles, tgt, msk, epochs=12, batch=256, lr=2e-3)
    D = dn()
    g = torch.empty_like(p)
    zero = torch.zeros_like(p)
    l0 = D.net_loss_grad(tiles[:1024].contiguous(), zero, tgt[:1024].contiguous(), msk[:1024].contiguous(), g,
                         kind=1)
    l1 = D.net_loss_grad(tiles[:1024].contiguous(), p, tgt[:1024].contiguous(), msk[:1024].contiguous(), g,
                         kind=1)
    return p, hist, l0, l1


@pytest.fixture(scope="module")
def heldout():
    from paper_1604_03734_amd import warmstart as W
    fr = scenes.frames_street(60.0, 60, seed=2001, config_id=5)
    return W.fuse_frames(fr)


def test_training_reduces_the_loss(trained):
    p, hist, l0, l1 = trained
    print(f"training loss {hist[0]:.5f} -> {hist[-1]:.5f}; loss of p = 0: {l0:.5f}, trained: {l1:.5f}")
    assert hist[-1] < hist[0]
    assert l1 < l0


@pytest.mark.parametrize("gamma", [0.0, 0.5])
def test_warm_start_gain_on_a_held_out_street(trained, heldout, gamma):
    D = dn()
    import torch
    from paper_1604_03734_amd import warmstart as W
    p = trained[0]
    vol = heldout
    plain = vol.regularize(D.reg_params(0.5, iters=20000, gap_every=10, gap_tol=TOL, kernel=D.DN_K_FUSED,
                                        gamma=gamma))
    ref = vol.regularize(D.reg_params(0.5, iters=100, kernel=D.DN_K_FUSED, gamma=gamma))
    res = W.solve_warm(vol, p, tol=TOL, k=100, plain_rel_gap_at_k=ref.rel_gap, gamma=gamma)
    print(f"gamma {gamma}: plain {plain.iters_run} iterations, warm {res['iters']} iterations "
          f"(fallback {res['fallback']}, gap after 100: warm {res['rel_gap_at_k']:.2e} plain {ref.rel_gap:.2e})")
    assert plain.converged and res["converged"]
    assert res["rel_gap"] <= TOL
    # what the trained network gains over the method without it
    assert not res["fallback"]
    assert res["iters"] < plain.iters_run


@pytest.mark.parametrize("gamma", [0.0, 0.5])
def test_shipped_weights_gain_with_the_stored_calibration(heldout, gamma):
    """The shipped weights on the held-out street, the fallback judged by
    the calibration stored with them (no plain run on this volume): no
    fallback, fewer iterations than the plain solver."""
    D = dn()
    from paper_1604_03734_amd import warmstart as W
    p = W.load_default_weights()
    assert p is not None and W.load_calibration() is not None
    vol = heldout
    plain = vol.regularize(D.reg_params(0.5, iters=20000, gap_every=10, gap_tol=TOL, kernel=D.DN_K_FUSED,
                                        gamma=gamma))
    res = W.solve_warm(vol, p, tol=TOL, k=100, gamma=gamma, kernel=D.DN_K_FUSED)
    print(f"shipped weights, gamma {gamma}: plain {plain.iters_run}, warm {res['iters']} "
          f"(reference {res['reference']} {res['plain_rel_gap_at_k']:.2e}, warm gap after 100 "
          f"{res['rel_gap_at_k']:.2e})")
    assert res["reference"] == "calibration"
    assert res["converged"] and not res["fallback"]
    assert res["iters"] < plain.iters_run


def test_fallback_on_a_wrong_network_with_the_stored_calibration(trained, heldout):
    """The wrong network of the next test, judged by the stored calibration:
    the warm start is discarded and the solve still converges."""
    from paper_1604_03734_amd import warmstart as W
    bad = trained[0].clone()
    bad[7808:8241] *= -20.0
    res = W.solve_warm(heldout, bad, tol=TOL, k=100)
    print(f"wrong network, calibrated reference {res['plain_rel_gap_at_k']:.3e}: gap after 100 warm "
          f"{res['rel_gap_at_k']:.3e}, fallback {res['fallback']}")
    assert res["reference"] == "calibration"
    assert res["fallback"] and res["converged"] and res["rel_gap"] <= TOL


def test_fallback_on_a_wrong_network(trained, heldout):
    """A genuinely wrong network (the trained one with its output layer
    negated and scaled by 20, so every dual component points the wrong way
    at full length) makes the gap after K warm iterations more than twice
    the plain solver's: the warm start is discarded, the solve restarts from
    zero and still reaches the target in K plus the plain iterations."""
    D = dn()
    import torch
    from paper_1604_03734_amd import warmstart as W
    vol = heldout
    bad = trained[0].clone()
    bad[7808:8241] *= -20.0
    ref = vol.regularize(D.reg_params(0.5, iters=100, kernel=D.DN_K_FUSED))
    res = W.solve_warm(vol, bad, tol=TOL, k=100, plain_rel_gap_at_k=ref.rel_gap)
    print(f"wrong network: gap after 100 warm {res['rel_gap_at_k']:.3e}, plain {ref.rel_gap:.3e}, "
          f"fallback {res['fallback']}")
    assert res["fallback"] and res["converged"] and res["rel_gap"] <= TOL
    plain = vol.regularize(D.reg_params(0.5, iters=20000, gap_every=10, gap_tol=TOL, kernel=D.DN_K_FUSED))
    assert res["iters"] == 100 + plain.iters_run
    torch.cuda.synchronize()


def test_fallback_to_a_cold_start(trained, heldout):
    """The fallback rule, forced from the host: with a plain-run reference
    gap far below what K warm iterations reach, the warm start is discarded
    and the solve restarts from zero; it still reaches the target."""
    D = dn()
    from paper_1604_03734_amd import warmstart as W
    vol = heldout
    ref = vol.regularize(D.reg_params(0.5, iters=100, kernel=D.DN_K_FUSED))
    res = W.solve_warm(vol, trained[0], tol=TOL, k=100, plain_rel_gap_at_k=ref.rel_gap * 1e-6)
    assert res["fallback"] and res["converged"] and res["rel_gap"] <= TOL
    plain = vol.regularize(D.reg_params(0.5, iters=20000, gap_every=10, gap_tol=TOL, kernel=D.DN_K_FUSED))
    assert res["iters"] == 100 + plain.iters_run
