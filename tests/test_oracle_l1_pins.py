"""Pins of the oracle's TV-L1 variant (L1 data term, u in [-1, 1]) against
facts that do not come from its code: the dual as a brute-force minimum,
closed forms, a linear program, weak duality.  CPU only."""
import numpy as np
import pytest

import oracle

TAU = SIG = 1.0 / np.sqrt(12.0)


def _volume_from_blocks(coords, cap_log2=10, tail=64):
    cap = 1 << cap_log2
    rc, slots = oracle.hash_build(coords, cap, tail)
    assert rc == oracle.OK
    return oracle.nbr_table(coords, slots, cap, tail)


def _random_field(seed, nb=6, frac=0.6):
    rng = np.random.default_rng(seed)
    coords = rng.choice(27, size=nb, replace=False)
    coords = np.stack([coords % 3, (coords // 3) % 3, coords // 9], 1).astype(np.int32)
    coords = coords[np.lexsort((coords[:, 2], coords[:, 1], coords[:, 0]))]
    nbr = _volume_from_blocks(coords)
    w = np.where(rng.random((nb, 512)) < frac, rng.integers(1, 5, (nb, 512)).astype(np.float64), 0.0)
    f = np.where(w > 0, rng.uniform(-1, 1, (nb, 512)), 0.0)
    return coords, nbr, f, w, rng


@pytest.mark.parametrize("seed,lam", [(0, 0.3), (1, 1.2)])
def test_l1_dual_is_the_minimum_over_the_box(seed, lam):
    """D(p) = sum_Omega min_{u in [-1,1]} (-u div p + lam w |u - f|), the
    inner minimum taken by brute force on a fine grid."""
    coords, nbr, f, w, rng = _random_field(seed)
    p = rng.normal(size=(3,) + f.shape)
    p /= np.maximum(1.0, np.sqrt((p ** 2).sum(0)))
    d = oracle.div(nbr, w, p)
    grid = np.linspace(-1.0, 1.0, 4001)
    om = w > 0
    dd, ff, ww = d[om], f[om], w[om]
    brute = 0.0
    for k in range(0, len(dd), 256):
        vals = -grid[None, :] * dd[k:k + 256, None] + lam * ww[k:k + 256, None] * np.abs(grid[None, :] - ff[k:k + 256, None])
        brute += vals.min(1).sum()
    E, D = oracle.energy_l1(nbr, f, w, np.zeros_like(f), p, lam)
    # the grid minimum is above the exact one by at most half a step times the slope
    slack = (0.5 * (grid[1] - grid[0]) * (np.abs(dd) + lam * ww)).sum()
    assert D <= brute + 1e-9 and D >= brute - slack - 1e-9


def test_l1_energy_of_a_shifted_field():
    """E(f + c) = TV(f) + lam |c| sum_Omega w, with TV(f) = E of the
    quadratic-data energy at u = f (its data term vanishes there)."""
    coords, nbr, f, w, rng = _random_field(3)
    lam, c = 0.7, 0.125
    u = np.where(w > 0, f + c, 0.0)
    tv, _ = oracle.energy(nbr, f, w, f, np.zeros((3,) + f.shape), lam)
    E, _ = oracle.energy_l1(nbr, f, w, u, np.zeros((3,) + f.shape), lam)
    assert abs(E - (tv + lam * c * w.sum())) <= 1e-9 * abs(E)


def _two_voxels(f1, f2, w1, w2, lam, iters):
    coords = np.array([[0, 0, 0], [1, 0, 0]], np.int32)
    nbr = _volume_from_blocks(coords)
    f = np.zeros((2, 512)); w = np.zeros((2, 512))
    f[0, 7], w[0, 7] = f1, w1
    f[1, 0], w[1, 0] = f2, w2
    u = np.zeros_like(f); ub = np.zeros_like(f); p = np.zeros((3, 2, 512))
    oracle.cp_l1(nbr, f, w, u, ub, p, iters, lam, TAU, SIG, 1.0, nthreads=1)
    E, D = oracle.energy_l1(nbr, f, w, u, p, lam)
    return u[0, 7], u[1, 0], u, E, D


@pytest.mark.parametrize("f1,f2,w1,w2", [(0.6, -0.7, 3, 4), (0.6, -0.7, 1, 4), (-0.3, 0.8, 0.5, 1.5)])
def test_l1_two_voxels_across_a_block_face_closed_form(f1, f2, w1, w2):
    """min |u1 - u2| + lam (w1 |u1 - f1| + w2 |u2 - f2|), lam = 0.5: with
    lam w_i > 1 for both the data are kept; otherwise the lighter voxel
    takes the heavier one's value (w1 < w2 here)."""
    lam = 0.5
    u1, u2, u, E, D = _two_voxels(f1, f2, w1, w2, lam, 20000)
    if lam * min(w1, w2) > 1.0:
        e1, e2 = f1, f2
    else:
        e1 = e2 = f2
    assert abs(u1 - e1) < 1e-6 and abs(u2 - e2) < 1e-6
    assert E - D >= -1e-12 and E - D < 1e-6
    observed = np.zeros((2, 512), bool)
    observed[0, 7] = observed[1, 0] = True
    assert not u[~observed].any()


def test_l1_large_lambda_keeps_the_data():
    """|div p| <= 6 for |p| <= 1, so lam w > 6 makes u = f the minimiser."""
    coords, nbr, f, w, rng = _random_field(4)
    u = np.zeros_like(f); ub = np.zeros_like(f); p = np.zeros((3,) + f.shape)
    oracle.cp_l1(nbr, f, w, u, ub, p, 300, 7.0, TAU, SIG, 1.0)
    assert np.abs(u - f)[w > 0].max() < 1e-12
    assert not u[w == 0].any()


@pytest.mark.parametrize("seed", [0, 1])
def test_l1_chain_matches_a_linear_program(seed):
    """A chain of 16 observed voxels along x across two blocks: TV is
    sum |u_{i+1} - u_i|, so the problem is a linear program (scipy HiGHS)."""
    from scipy.optimize import linprog
    rng = np.random.default_rng(10 + seed)
    coords = np.array([[0, 0, 0], [1, 0, 0]], np.int32)
    nbr = _volume_from_blocks(coords)
    n = 16
    fv = rng.uniform(-1, 1, n)
    wv = rng.integers(1, 5, n).astype(np.float64)
    lam = 0.3
    f = np.zeros((2, 512)); w = np.zeros((2, 512))
    for i in range(n):
        b, x = divmod(i, 8)
        f[b, x], w[b, x] = fv[i], wv[i]
    # variables [u (n), t (n-1), s (n)]: min sum t + lam sum w s
    nv = n + (n - 1) + n
    c = np.concatenate([np.zeros(n), np.ones(n - 1), lam * wv])
    A, bvec = [], []
    for i in range(n - 1):
        r = np.zeros(nv); r[i + 1], r[i], r[n + i] = 1, -1, -1; A.append(r); bvec.append(0)
        r = np.zeros(nv); r[i + 1], r[i], r[n + i] = -1, 1, -1; A.append(r); bvec.append(0)
    for i in range(n):
        r = np.zeros(nv); r[i], r[2 * n - 1 + i] = 1, -1; A.append(r); bvec.append(fv[i])
        r = np.zeros(nv); r[i], r[2 * n - 1 + i] = -1, -1; A.append(r); bvec.append(-fv[i])
    bounds = [(-1, 1)] * n + [(0, None)] * (2 * n - 1)
    lp = linprog(c, A_ub=np.array(A), b_ub=np.array(bvec), bounds=bounds, method="highs")
    assert lp.success
    u = np.zeros_like(f); ub = np.zeros_like(f); p = np.zeros((3, 2, 512))
    oracle.cp_l1(nbr, f, w, u, ub, p, 20000, lam, TAU, SIG, 1.0, nthreads=1)
    E, D = oracle.energy_l1(nbr, f, w, u, p, lam)
    assert abs(E - lp.fun) <= 1e-6 * max(1.0, abs(lp.fun))
    assert D <= lp.fun + 1e-9 and E - D < 1e-5


def test_l1_weak_duality_and_convergence_on_a_sparse_field():
    coords, nbr, f, w, rng = _random_field(5, nb=8)
    lam = 0.6
    u = np.zeros_like(f); ub = np.zeros_like(f); p = np.zeros((3,) + f.shape)
    gaps = []
    for _ in range(20):
        oracle.cp_l1(nbr, f, w, u, ub, p, 100, lam, TAU, SIG, 1.0)
        E, D = oracle.energy_l1(nbr, f, w, u, p, lam)
        assert E - D >= -1e-9
        assert np.abs(u).max() <= 1.0 and np.sqrt((p ** 2).sum(0)).max() <= 1.0 + 1e-12
        gaps.append((E - D) / E)
    assert gaps[-1] < 1e-3 and gaps[-1] < 0.05 * gaps[0]
