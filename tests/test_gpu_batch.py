"""Batched regularisation of uneven sub-maps (one HIP graph: the persistent
kernel with grid barriers, or one launch per iteration, or the tuner's
choice) against the single-volume kernel and the oracle."""
import numpy as np
import pytest

import oracle
import scenes
from gpu_common import LAM, SIG, TAU, dn, host, state_of, to_dev

pytestmark = pytest.mark.gpu


def _make(D, nb, seed, extent):
    import torch
    coords, f, w = scenes.random_block_field(nb, seed, extent=extent, omega_frac=0.75)
    gv = D.Volume(0.1, 0.3, 10.0, nb, 8, 64, max_points=0)
    gv.insert_blocks(to_dev(coords.astype(np.int32)))
    c = host(gv.extract(D.DN_X_COORDS))
    order = np.array([np.nonzero((coords == x).all(1))[0][0] for x in c])
    f, w = f[order].astype(np.float32), w[order].astype(np.float32)
    gv.load_fused(to_dev(f), to_dev(w))
    return gv, c, f.astype(np.float64), w.astype(np.float64)


SIZES = [(3, 0, 2), (40, 1, 4), (7, 2, 3), (120, 3, 6), (1, 4, 2)]
# tuner's choice / persistent kernel / one launch per iteration
KERNELS = ["auto", "persistent", "per_iteration"]


def _kernel(D, name):
    return {"auto": D.DN_K_AUTO, "persistent": D.DN_K_FUSED, "per_iteration": D.DN_K_FUSED256}[name]


@pytest.mark.parametrize("kname", KERNELS)
def test_batch_matches_single_volume_and_oracle(kname):
    D = dn()
    vols = [_make(D, *s) for s in SIZES]
    stats = D.regularize_batch([v[0] for v in vols], D.reg_params(LAM, iters=30, kernel=_kernel(D, kname)))
    want = {"persistent": 257, "per_iteration": 1}.get(kname)
    if want is not None:
        assert all(st.kernel_used // 100 == want for st in stats)
    for (gv, c, f, w), st in zip(vols, stats):
        gu, gub, gp = state_of(D, gv)
        nbr = host(gv.extract(D.DN_X_NBR))
        u = np.zeros_like(f); ub = np.zeros_like(u); p = np.zeros((3,) + u.shape)
        oracle.cp(nbr, f, w, u, ub, p, 30, LAM, TAU, SIG, 1.0)
        assert np.abs(gu - u).max() <= 1e-4
        E, Dd = oracle.energy(nbr, f, w, gu, gp, LAM)
        assert abs(st.energy - E) <= 1e-9 * abs(E) and abs(st.dual - Dd) <= 1e-9 * abs(E)
        single = gv.regularize(D.reg_params(LAM, iters=30, kernel=D.DN_K_FUSED))
        su, sub, sp = state_of(D, gv)
        np.testing.assert_array_equal(su, gu)
        np.testing.assert_array_equal(sp, gp)


@pytest.mark.parametrize("kname", KERNELS)
def test_batch_keep_resumes_and_graph_replays(kname):
    D = dn()
    k = _kernel(D, kname)
    vols = [_make(D, *s) for s in SIZES[:3]]
    handles = [v[0] for v in vols]
    D.regularize_batch(handles, D.reg_params(LAM, iters=24, kernel=k))
    whole = [state_of(D, h) for h in handles]
    for rep in range(3):  # the same configuration replays the cached graph
        D.regularize_batch(handles, D.reg_params(LAM, iters=11, kernel=k))
        D.regularize_batch(handles, D.reg_params(LAM, iters=13, kernel=k, init=D.DN_INIT_KEEP))
        for h, ref in zip(handles, whole):
            for a, b in zip(state_of(D, h), ref):
                np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("kname", KERNELS)
def test_batch_accelerated_matches_single(kname):
    D = dn()
    vols = [_make(D, *s) for s in SIZES[:4]]
    handles = [v[0] for v in vols]
    D.regularize_batch(handles, D.reg_params(LAM, iters=40, kernel=_kernel(D, kname), gamma=LAM))
    batched = [state_of(D, h) for h in handles]
    for h, ref in zip(handles, batched):
        h.regularize(D.reg_params(LAM, iters=40, kernel=D.DN_K_FUSED, gamma=LAM))
        for a, b in zip(state_of(D, h), ref):
            np.testing.assert_array_equal(a, b)


def test_batch_of_many_small_sub_maps():
    """70 sub-maps of one to three blocks, one launch per iteration: every
    sub-map equals the single-volume kernel."""
    D = dn()
    vols = [_make(D, 1 + i % 3, 100 + i, 2) for i in range(70)]
    handles = [v[0] for v in vols]
    stats = D.regularize_batch(handles, D.reg_params(LAM, iters=20, kernel=D.DN_K_FUSED256))
    assert all(st.kernel_used // 100 == 1 for st in stats)
    batched = [state_of(D, h) for h in handles]
    for h, ref in zip(handles, batched):
        h.regularize(D.reg_params(LAM, iters=20, kernel=D.DN_K_FUSED))
        for a, b in zip(state_of(D, h), ref):
            np.testing.assert_array_equal(a, b)
