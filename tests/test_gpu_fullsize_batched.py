"""Parity at the batched workload's full size, in the launch configuration
bench.py times: 64 street segments of 1e3..5e4 blocks (1.04e6 blocks,
5.3e8 voxels) regularised together for 300 iterations in one HIP graph
(autotuned: the persistent kernel or one launch per iteration).  Checked through properties that hold
at any size (|p| <= 1, unobserved voxels untouched), bit-exact equality of
sub-maps with the single-volume kernel run on them alone, and the smallest
sub-maps against the oracle."""
import numpy as np
import pytest

import oracle
from gpu_common import LAM, SIG, TAU, dn, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def batch():
    import os
    import sys
    import types
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import bench
    args = types.SimpleNamespace(frames=100, copies=35, iters=300, kernel="auto", storage="f32", submaps=64)
    wl = bench.BatchedWorkload(args)
    st, _ = wl.step()
    D = dn()
    stats = D.regularize_batch(wl.subs, D.reg_params(LAM, iters=300, kernel=D.DN_K_AUTO))
    return wl, stats


def test_batched_full_size_properties(batch):
    D = dn()
    wl, stats = batch
    assert sum(v.num_blocks for v in wl.subs) == sum(int(n) for n in wl.counts)
    for vol, st in zip(wl.subs, stats):
        u = host(vol.extract(D.DN_X_U))
        w = host(vol.extract(D.DN_X_W))
        p = host(vol.extract(D.DN_X_P)).astype(np.float64)
        assert np.sqrt((p ** 2).sum(0)).max() <= 1.0 + 1e-6
        assert (u[w == 0] == 0).all()
        assert st.gap >= 0 and st.iters_run == 300


def test_batched_sub_maps_equal_the_single_volume_kernel(batch):
    D = dn()
    wl, stats = batch
    order = np.argsort(wl.counts)
    for i in (order[0], order[len(order) // 2]):
        vol = wl.subs[i]
        bu = host(vol.extract(D.DN_X_U)).copy()
        bp = host(vol.extract(D.DN_X_P)).copy()
        vol.regularize(D.reg_params(LAM, iters=300, kernel=D.DN_K_FUSED256))
        np.testing.assert_array_equal(host(vol.extract(D.DN_X_U)), bu)
        np.testing.assert_array_equal(host(vol.extract(D.DN_X_P)), bp)


def test_batched_smallest_sub_maps_against_the_oracle(batch):
    D = dn()
    wl, stats = batch
    for i in np.argsort(wl.counts)[:2]:
        vol = wl.subs[i]
        # the batch left vol's state; the previous test may have rerun it
        # with the single-volume kernel, which gives the same bits
        gu = host(vol.extract(D.DN_X_U)).astype(np.float64)
        gp = host(vol.extract(D.DN_X_P)).astype(np.float64)
        f = host(vol.extract(D.DN_X_F)).astype(np.float64)
        w = host(vol.extract(D.DN_X_W)).astype(np.float64)
        nbr = host(vol.extract(D.DN_X_NBR))
        u = np.zeros_like(f); ub = np.zeros_like(f); p = np.zeros((3,) + f.shape)
        oracle.cp(nbr, f, w, u, ub, p, 300, LAM, TAU, SIG, 1.0)
        err = np.abs(gu - u).max()
        print(f"sub-map {i} ({vol.num_blocks} blocks): max |du| {err:.2e}")
        assert err <= 1e-4
        E, Dd = oracle.energy(nbr, f, w, gu, gp, LAM)
        assert abs(stats[i].energy - E) <= 1e-9 * abs(E) and abs(stats[i].dual - Dd) <= 1e-9 * abs(E)
