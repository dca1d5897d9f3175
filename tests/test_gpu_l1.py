"""TV-L1 variant (L1 data term, u in [-1, 1]) of the regulariser on the GPU
against the oracle's: single volume with every kernel, 16-bit storage,
the batched launch, gap stopping, and the error paths.  Bars as
for the quadratic data term: max-abs 1e-4 on u after the same iterations,
energies within 1e-9 relative of the oracle on the GPU state."""
import numpy as np
import pytest

import oracle
import scenes
from gpu_common import LAM, SIG, TAU, dn, fuse_both, host, state_of, to_dev

pytestmark = pytest.mark.gpu

LAM1 = 0.8


@pytest.fixture(scope="module")
def c1():
    fr = scenes.frames_c1(0)
    ov, gv = fuse_both(fr, check_each_frame=False)
    return fr, ov, gv


def _oracle_l1(ov, iters, lam=LAM1):
    u = np.zeros_like(ov.f); ub = np.zeros_like(u); p = np.zeros((3,) + u.shape)
    oracle.cp_l1(ov.nbr, ov.f, ov.w, u, ub, p, iters, lam, TAU, SIG, 1.0)
    return u, p


@pytest.mark.parametrize("kernel,lam", [("twopass", 0.8), ("fused", 0.8), ("fused256", 0.8), ("fused256", 0.5),
                                        ("twopass", 0.5)])
def test_l1_parity_every_kernel(c1, kernel, lam):
    """Config 1 (200 iterations; lambda 0.5 is the configuration's) with
    each kernel."""
    D = dn()
    fr, ov, gv = c1
    k = {"twopass": D.DN_K_TWOPASS, "fused": D.DN_K_FUSED, "fused256": D.DN_K_FUSED256}[kernel]
    st = gv.regularize(D.reg_params(lam, TAU, SIG, 1.0, iters=200, kernel=k, data_term=D.DN_DATA_L1))
    u, p = _oracle_l1(ov, 200, lam)
    gu, gub, gp = state_of(D, gv)
    print(f"{kernel}: max |du| {np.abs(gu - u).max():.2e}")
    assert np.abs(gu - u).max() <= 1e-4
    assert np.abs(gu).max() <= 1.0 and np.sqrt((gp ** 2).sum(0)).max() <= 1.0 + 1e-6
    assert (gu[ov.w == 0] == 0).all()
    # energies of the GPU state, with the fused field the library holds (the
    # L1 term is first-order sensitive to the 1e-4 fusion differences)
    gf = host(gv.extract(D.DN_X_F)).astype(np.float64)
    E, Dd = oracle.energy_l1(ov.nbr, gf, ov.w, gu, gp, lam)
    assert abs(st.energy - E) <= 1e-9 * abs(E) and abs(st.dual - Dd) <= 1e-9 * abs(E)
    assert st.gap >= 0
    # dn_energy with the L1 term gives the same pair; the L2 pair differs
    e1 = gv.energy(lam, D.DN_DATA_L1)
    assert abs(e1[0] - st.energy) <= 1e-12 * abs(E) and abs(e1[1] - st.dual) <= 1e-12 * abs(E)
    E2, D2 = oracle.energy(ov.nbr, gf, ov.w, gu, gp, lam)
    e2 = gv.energy(lam, D.DN_DATA_L2)
    assert abs(e2[0] - E2) <= 1e-9 * abs(E2) and abs(e2[1] - D2) <= 1e-9 * abs(E2)


def test_l1_gap_stop_and_split_resume(c1):
    D = dn()
    fr, ov, gv = c1
    st = gv.regularize(D.reg_params(LAM1, iters=5000, gap_every=10, gap_tol=1e-3, kernel=D.DN_K_FUSED,
                                    data_term=D.DN_DATA_L1))
    assert st.converged and st.rel_gap <= 1e-3 and st.iters_run % 10 == 0 and st.iters_run < 5000
    gv.regularize(D.reg_params(LAM1, iters=50, kernel=D.DN_K_FUSED, data_term=D.DN_DATA_L1))
    whole = state_of(D, gv)
    gv.regularize(D.reg_params(LAM1, iters=20, kernel=D.DN_K_FUSED, data_term=D.DN_DATA_L1))
    gv.regularize(D.reg_params(LAM1, iters=30, kernel=D.DN_K_FUSED, data_term=D.DN_DATA_L1, init=D.DN_INIT_KEEP))
    for a, b in zip(state_of(D, gv), whole):
        np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_l1_16bit_storage(c1, storage):
    D = dn()
    fr, ov, gv = c1
    s = D.DN_F16 if storage == "f16" else D.DN_BF16
    st = gv.regularize(D.reg_params(LAM1, iters=200, storage=s, refine_every=50, kernel=D.DN_K_AUTO,
                                    data_term=D.DN_DATA_L1))
    u, p = _oracle_l1(ov, 200)
    gu, _, gp = state_of(D, gv)
    err = np.abs(gu - u)[ov.w > 0]
    print(f"{storage}: max {err.max():.2e} median {np.median(err):.2e}")
    assert np.abs(gu).max() <= 1.0
    assert err.max() <= (1e-2 if storage == "f16" else 6e-2) and np.median(err) <= (2e-3 if storage == "f16" else 2e-2)
    gf = host(gv.extract(D.DN_X_F)).astype(np.float64)
    E, Dd = oracle.energy_l1(ov.nbr, gf, ov.w, gu, gp, LAM1)
    assert abs(st.energy - E) <= 1e-9 * abs(E)


def test_l1_batch_matches_single_and_oracle():
    D = dn()
    vols = []
    for nb, seed, ext in [(3, 0, 2), (40, 1, 4), (7, 2, 3)]:
        coords, f, w = scenes.random_block_field(nb, seed, extent=ext, omega_frac=0.75)
        gv = D.Volume(0.1, 0.3, 10.0, nb, 8, 64, max_points=0)
        gv.insert_blocks(to_dev(coords.astype(np.int32)))
        c = host(gv.extract(D.DN_X_COORDS))
        order = np.array([np.nonzero((coords == x).all(1))[0][0] for x in c])
        f, w = f[order].astype(np.float32), w[order].astype(np.float32)
        gv.load_fused(to_dev(f), to_dev(w))
        vols.append((gv, f.astype(np.float64), w.astype(np.float64)))
    stats = D.regularize_batch([v[0] for v in vols], D.reg_params(LAM1, iters=40, kernel=D.DN_K_AUTO,
                                                                  data_term=D.DN_DATA_L1))
    for (gv, f, w), st in zip(vols, stats):
        gu, _, gp = state_of(D, gv)
        nbr = host(gv.extract(D.DN_X_NBR))
        u = np.zeros_like(f); ub = np.zeros_like(u); p = np.zeros((3,) + u.shape)
        oracle.cp_l1(nbr, f, w, u, ub, p, 40, LAM1, TAU, SIG, 1.0)
        assert np.abs(gu - u).max() <= 1e-4
        E, Dd = oracle.energy_l1(nbr, f, w, gu, gp, LAM1)
        assert abs(st.energy - E) <= 1e-9 * abs(E) and abs(st.dual - Dd) <= 1e-9 * abs(E)
        gv.regularize(D.reg_params(LAM1, iters=40, kernel=D.DN_K_FUSED256, data_term=D.DN_DATA_L1))
        su, _, sp = state_of(D, gv)
        np.testing.assert_array_equal(su, gu)
        np.testing.assert_array_equal(sp, gp)


def test_l1_rejects_the_accelerated_schedule_and_bad_terms(c1):
    D = dn()
    fr, ov, gv = c1
    with pytest.raises(D.DenserError) as e:
        gv.regularize(D.reg_params(LAM1, iters=5, gamma=0.4, data_term=D.DN_DATA_L1))
    assert e.value.code == D.DN_E_INVALID
    with pytest.raises(D.DenserError):
        gv.regularize(D.reg_params(LAM1, iters=5, data_term=7))
    with pytest.raises(D.DenserError):
        gv.energy(LAM1, 3)
