"""GPU (HIP library through the C ABI) against the FP64 oracle.

Bars: bit-exact for allocation (candidate keys, pool order, hash slots,
neighbour table) and for the fusion weights; max-abs 1e-4 on the fused
TSDF f and on u after the same number of iterations (FP32 arithmetic);
energies within 1e-9 relative of the oracle evaluated on the GPU state."""
import numpy as np
import pytest

import oracle
import scenes
from gpu_common import LAM, SIG, TAU, dn, fuse_both, host, intr, K4, state_of, to_dev

pytestmark = pytest.mark.gpu

TOL_F = 1e-4
TOL_U = 1e-4


@pytest.fixture(scope="module")
def c1():
    fr = scenes.frames_c1(0)
    ov, gv = fuse_both(fr)
    return fr, ov, gv


def test_c1_allocation_bit_exact(c1):
    D = dn()
    fr, ov, gv = c1
    assert gv.num_blocks == ov.nb
    np.testing.assert_array_equal(host(gv.extract(D.DN_X_COORDS)), ov.coords)
    np.testing.assert_array_equal(host(gv.extract(D.DN_X_HASH)), ov.slots)
    np.testing.assert_array_equal(host(gv.extract(D.DN_X_NBR)), ov.nbr)


def test_c1_fusion_parity(c1):
    D = dn()
    fr, ov, gv = c1
    w = host(gv.extract(D.DN_X_W))
    f = host(gv.extract(D.DN_X_F))
    np.testing.assert_array_equal(w, ov.w)
    assert np.abs(f - ov.f).max() <= TOL_F
    assert (w > 0).sum() > 50000


def test_fusion_culling_keeps_every_updatable_block():
    """Fusion skips blocks out of view; a dense cube of blocks around the
    camera (behind it, straddling its plane, beside the image, beyond
    max_depth + mu) fused from three poses (one rotated, one looking back
    through the cube) matches the oracle's fusion of every block: w
    bit-exact, f within 1e-4, and some blocks are out of view."""
    D = dn()
    fr = scenes.frames_c1(0)
    cam = fr.camera
    r = np.arange(-5, 6)
    coords = np.stack(np.meshgrid(r, r, r, indexing="ij"), -1).reshape(-1, 3).astype(np.int32)
    max_depth = 2.6
    gv = D.Volume(fr.voxel_size, fr.mu, max_depth, len(coords), 12, 256, max_points=0)
    gv.insert_blocks(to_dev(coords))
    pc = host(gv.extract(D.DN_X_COORDS))[:, :3]
    f = np.zeros((len(pc), 512))
    w = np.zeros((len(pc), 512))
    K = intr(D, cam)
    c, s_ = np.cos(0.7), np.sin(0.7)
    R = np.array([[c, 0, s_], [0, 1, 0], [-s_, 0, c]])
    poses = [fr.poses[0], fr.poses[1].copy(), np.eye(4)]
    poses[1][:3, :3] = R @ poses[1][:3, :3]
    poses[2][:3, :3] = np.diag([-1.0, 1.0, -1.0])   # at the origin, looking along -z through the cube
    H, W = cam.height, cam.width
    rng = np.random.default_rng(5)
    depths = []
    for k in range(3):   # slanted planes 1 to 2.8 m away, 5% invalid
        d = (1.0 + 1.8 * np.arange(W)[None, :] / W + 0.2 * k + 0.0 * np.arange(H)[:, None]).astype(np.float32)
        d[rng.random((H, W)) < 0.05] = np.nan
        depths.append(d)
    for d, T in zip(depths, poses):
        oracle.fuse(pc, f, w, d, K4(cam), T, fr.voxel_size, fr.mu, max_depth)
        gv.fuse_depth(to_dev(d), K, T)
    gw = host(gv.extract(D.DN_X_W))
    gf = host(gv.extract(D.DN_X_F))
    np.testing.assert_array_equal(gw, w)
    assert np.abs(gf - f).max() <= TOL_F
    touched = (w > 0).any(1)
    print(f"culling cube: {int(touched.sum())} of {len(pc)} blocks updated")
    assert 0 < touched.sum() < len(pc)


@pytest.mark.parametrize("kernel", ["twopass", "fused"])
def test_c1_regularize_parity(c1, kernel):
    D = dn()
    fr, ov, gv = c1
    k = D.DN_K_TWOPASS if kernel == "twopass" else D.DN_K_FUSED
    st = gv.regularize(D.reg_params(LAM, TAU, SIG, 1.0, iters=200, kernel=k))
    assert st.iters_run == 200
    u = np.zeros_like(ov.f); ub = np.zeros_like(u); p = np.zeros((3,) + u.shape)
    oracle.cp(ov.nbr, ov.f, ov.w, u, ub, p, 200, LAM, TAU, SIG, 1.0)
    gu, gub, gp = state_of(D, gv)
    assert np.abs(gu - u).max() <= TOL_U
    assert np.abs(gp - p).max() <= 10 * TOL_U
    assert np.sqrt((gp ** 2).sum(0)).max() <= 1.0 + 1e-6
    assert (gu[ov.w == 0] == 0).all()
    # the library's energies equal the oracle's on the same (GPU) state
    E, Dd = oracle.energy(ov.nbr, ov.f, ov.w, gu, gp, LAM)
    assert abs(st.energy - E) <= 1e-9 * abs(E)
    assert abs(st.dual - Dd) <= 1e-9 * abs(E)
    assert st.gap >= 0


def test_fused_equals_twopass_and_is_deterministic(c1):
    D = dn()
    fr, ov, gv = c1
    gv.regularize(D.reg_params(LAM, iters=60, kernel=D.DN_K_FUSED))
    a = state_of(D, gv)
    gv.regularize(D.reg_params(LAM, iters=60, kernel=D.DN_K_FUSED))
    b = state_of(D, gv)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)
    gv.regularize(D.reg_params(LAM, iters=60, kernel=D.DN_K_TWOPASS))
    c = state_of(D, gv)
    assert np.abs(a[0] - c[0]).max() <= 1e-5
    # 256 threads x 2 voxels computes each voxel with the same arithmetic
    gv.regularize(D.reg_params(LAM, iters=60, kernel=D.DN_K_FUSED256))
    for x, y in zip(a, state_of(D, gv)):
        np.testing.assert_array_equal(x, y)


def test_split_run_resumes_exactly(c1):
    D = dn()
    fr, ov, gv = c1
    gv.regularize(D.reg_params(LAM, iters=80, kernel=D.DN_K_FUSED))
    whole = state_of(D, gv)
    gv.regularize(D.reg_params(LAM, iters=30, kernel=D.DN_K_FUSED))
    gv.regularize(D.reg_params(LAM, iters=50, kernel=D.DN_K_FUSED, init=D.DN_INIT_KEEP))
    split = state_of(D, gv)
    for x, y in zip(whole, split):
        np.testing.assert_array_equal(x, y)


def test_gap_checks_and_early_stop(c1):
    D = dn()
    fr, ov, gv = c1
    st = gv.regularize(D.reg_params(LAM, iters=2000, gap_every=10, gap_tol=1e-2, kernel=D.DN_K_FUSED))
    assert st.converged == 1 and st.iters_run < 2000 and st.iters_run % 10 == 0
    assert st.rel_gap <= 1e-2
    st2 = gv.regularize(D.reg_params(LAM, iters=st.iters_run - 10, kernel=D.DN_K_FUSED))
    assert st2.rel_gap > 1e-2


def test_c1_surface_parity(c1):
    D = dn()
    fr, ov, gv = c1
    gv.regularize(D.reg_params(LAM, iters=100, kernel=D.DN_K_FUSED))
    gu = host(gv.extract(D.DN_X_U)).astype(np.float64)
    pts = host(gv.extract(D.DN_X_SURFACE)).astype(np.float64)
    ref = oracle.extract(ov.coords, ov.nbr, ov.w, gu, fr.voxel_size)
    assert len(pts) == len(ref) and len(ref) > 1000
    assert np.abs(pts - ref).max() <= 1e-5


@pytest.mark.parametrize("seed,nb,extent", [(0, 1, 2), (1, 13, 3), (2, 37, 4), (3, 90, 5)])
def test_random_sparse_fields_regularize_parity(seed, nb, extent):
    """Arbitrary block sets with unobserved voxels and unallocated
    neighbours (every boundary case of Eqs. 3-4)."""
    D = dn()
    import torch
    coords, f, w = scenes.random_block_field(nb, seed, extent=extent, omega_frac=0.7)
    cap, tail = 64, 64
    ov = oracle.OracleVolume(0.1, 0.3, 10.0, 1024, 6, tail)
    assert ov.insert(coords) == nb
    order = np.array([np.nonzero((coords == c).all(1))[0][0] for c in ov.coords])
    ov.f[:] = f[order]; ov.w[:] = w[order]
    gv = D.Volume(0.1, 0.3, 10.0, 1024, 6, tail)
    assert gv.insert_blocks(to_dev(coords.astype(np.int32))) == nb
    np.testing.assert_array_equal(host(gv.extract(D.DN_X_COORDS)), ov.coords)
    np.testing.assert_array_equal(host(gv.extract(D.DN_X_HASH)), ov.slots)
    np.testing.assert_array_equal(host(gv.extract(D.DN_X_NBR)), ov.nbr)
    gv.load_fused(to_dev(ov.f, torch.float32), to_dev(ov.w, torch.float32))
    fo = ov.f.astype(np.float32).astype(np.float64)
    for kernel in (D.DN_K_FUSED, D.DN_K_TWOPASS):
        st = gv.regularize(D.reg_params(LAM, iters=50, kernel=kernel))
        u = np.zeros_like(fo); ub = np.zeros_like(u); p = np.zeros((3,) + u.shape)
        oracle.cp(ov.nbr, fo, ov.w, u, ub, p, 50, LAM, TAU, SIG, 1.0)
        gu, gub, gp = state_of(D, gv)
        assert np.abs(gu - u).max() <= TOL_U
        assert np.abs(gub - ub).max() <= 3 * TOL_U
        em = host(gv.extract(D.DN_X_EMASK))
        assert ((em & 1) == (ov.w > 0)).all()
        E, Dd = oracle.energy(ov.nbr, fo, ov.w, gu, gp, LAM)
        assert abs(st.energy - E) <= 1e-9 * abs(E) and abs(st.dual - Dd) <= 1e-9 * abs(E)


def test_given_initial_state_and_ragged_capacity():
    D = dn()
    import torch
    coords, f, w = scenes.random_block_field(20, 5, extent=3, omega_frac=0.8)
    gv = D.Volume(0.1, 0.3, 10.0, 20, 5, 32)
    gv.insert_blocks(to_dev(coords.astype(np.int32)))
    c = host(gv.extract(D.DN_X_COORDS))
    order = np.array([np.nonzero((coords == x).all(1))[0][0] for x in c])
    f, w = f[order], w[order]
    gv.load_fused(to_dev(f, torch.float32), to_dev(w, torch.float32))
    rng = np.random.default_rng(0)
    u0 = rng.uniform(-1, 1, f.shape)
    p0 = rng.uniform(-0.5, 0.5, (3,) + f.shape)
    st = gv.regularize(D.reg_params(LAM, iters=25, init=D.DN_INIT_GIVEN, kernel=D.DN_K_FUSED),
                       u0=to_dev(u0, torch.float32), p0=to_dev(p0, torch.float32))
    _, nbr = oracle.OracleVolume, host(gv.extract(D.DN_X_NBR))
    fo = f.astype(np.float32).astype(np.float64)
    u = u0.astype(np.float32).astype(np.float64); ub = u.copy()
    p = p0.astype(np.float32).astype(np.float64)
    oracle.cp(nbr, fo, w, u, ub, p, 25, LAM, TAU, SIG, 1.0)
    gu = host(gv.extract(D.DN_X_U))
    assert np.abs(gu - u).max() <= TOL_U
    # the pool is full: one more block is a capacity error, volume unchanged
    with pytest.raises(D.DenserError) as e:
        gv.insert_blocks(to_dev(np.array([[50, 50, 50]], np.int32)))
    assert e.value.code == D.DN_E_CAPACITY
    assert gv.num_blocks == 20


def test_candidates_survive_other_work_and_known_frames():
    """The distinct candidate keys of the last frame are built when they are
    extracted, from the frame's raw candidate list: a regularisation in
    between (which reuses the sort scratch) must not change them, and a
    frame whose blocks all exist allocates nothing but still reports its
    candidates."""
    D = dn()
    fr = scenes.frames_c1(0)
    cam = fr.camera
    ov = oracle.OracleVolume(fr.voxel_size, fr.mu, fr.max_depth, 8192, 12, 256)
    gv = D.Volume(fr.voxel_size, fr.mu, fr.max_depth, 8192, 12, 256)
    K = intr(D, cam)
    d0, T0 = fr.depths[0], fr.poses[0]
    n_o = ov.alloc(d0, K4(cam), T0)
    dd = to_dev(d0)
    assert gv.alloc_blocks(dd, K, T0) == n_o > 0
    gv.fuse_depth(dd, K, T0)
    gv.regularize(D.reg_params(LAM, iters=5, kernel=D.DN_K_FUSED))
    np.testing.assert_array_equal(host(gv.extract(D.DN_X_CANDIDATES)), ov.last_candidates)
    # the same frame again: every candidate is known
    assert ov.alloc(d0, K4(cam), T0) == 0
    assert gv.alloc_blocks(dd, K, T0) == 0
    np.testing.assert_array_equal(host(gv.extract(D.DN_X_CANDIDATES)), ov.last_candidates)
    # a second extraction returns the same list
    np.testing.assert_array_equal(host(gv.extract(D.DN_X_CANDIDATES)), ov.last_candidates)
    np.testing.assert_array_equal(host(gv.extract(D.DN_X_COORDS)), ov.coords)
    np.testing.assert_array_equal(host(gv.extract(D.DN_X_HASH)), ov.slots)
    # a frame with new and known blocks, then a clear
    d1, T1 = fr.depths[1], fr.poses[1]
    assert gv.alloc_blocks(to_dev(d1), K, T1) == ov.alloc(d1, K4(cam), T1)
    np.testing.assert_array_equal(host(gv.extract(D.DN_X_CANDIDATES)), ov.last_candidates)
    np.testing.assert_array_equal(host(gv.extract(D.DN_X_NBR)), ov.nbr)
    gv.clear()
    assert host(gv.extract(D.DN_X_CANDIDATES)).shape == (0, 3)


def test_error_paths_and_degenerate_inputs():
    D = dn()
    import torch
    gv = D.Volume(0.1, 0.3, 10.0, 64, 6, 8)
    # empty volume: regularize and extract are no-ops
    st = gv.regularize(D.reg_params(LAM, iters=10))
    assert st.iters_run == 0 and st.energy == 0.0
    assert gv.extract(D.DN_X_SURFACE).shape[0] == 0
    # an all-invalid frame allocates nothing
    cam = scenes.Camera(50, 50, 15.5, 11.5, 32, 24)
    bad = np.full((24, 32), np.nan, np.float32)
    bad[::2] = 0.0
    assert gv.alloc_blocks(to_dev(bad), intr(D, cam), np.eye(4)) == 0
    # invalid parameters
    with pytest.raises(D.DenserError) as e:
        gv.regularize(D.reg_params(LAM, tau=1.0, sigma=1.0, iters=1))
    assert e.value.code == D.DN_E_INVALID
    with pytest.raises(D.DenserError):
        D.Volume(0.1, 0.3, 10.0, 64, 2, 8)
    # hash overflow leaves the volume unchanged
    tiny = D.Volume(0.1, 0.3, 10.0, 1000, 4, 2)
    keys = np.stack([np.arange(40), np.zeros(40), np.zeros(40)], 1).astype(np.int32)
    with pytest.raises(D.DenserError) as e:
        tiny.insert_blocks(to_dev(keys))
    assert e.value.code == D.DN_E_CAPACITY and tiny.num_blocks == 0
    assert tiny.insert_blocks(to_dev(keys[:5])) == 5


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_mixed_precision_error_is_reported_and_bounded(c1, storage):
    D = dn()
    fr, ov, gv = c1
    s = D.DN_F16 if storage == "f16" else D.DN_BF16
    st = gv.regularize(D.reg_params(LAM, iters=200, storage=s, refine_every=50))
    u = np.zeros_like(ov.f); ub = np.zeros_like(u); p = np.zeros((3,) + u.shape)
    oracle.cp(ov.nbr, ov.f, ov.w, u, ub, p, 200, LAM, TAU, SIG, 1.0)
    gu = host(gv.extract(D.DN_X_U)).astype(np.float64)
    om = ov.w > 0
    err = np.abs(gu - u)[om]
    print(f"{storage}: max {err.max():.3e} median {np.median(err):.3e} rel_gap {st.rel_gap:.3e}")
    # stochastic rounding of the stored state: no stagnation, errors near
    # the rounding noise (FP16 step 2^-11 at |u| ~ 0.5, BF16 2^-8)
    bound, med = (5e-3, 4e-4) if storage == "f16" else (3e-2, 3e-3)
    assert err.max() <= bound and np.median(err) <= med
    assert st.gap >= 0
    gp = host(gv.extract(D.DN_X_P))
    assert np.sqrt((gp.astype(np.float64) ** 2).sum(0)).max() <= 1.0 + 1e-6
    # the rounding bits are a function of (voxel, iteration): equal calls agree
    gv.regularize(D.reg_params(LAM, iters=200, storage=s, refine_every=50))
    np.testing.assert_array_equal(host(gv.extract(D.DN_X_U)).astype(np.float64), gu)


def test_accelerated_variant_parity_and_resume(c1):
    D = dn()
    fr, ov, gv = c1
    gam = LAM * 1.0  # lambda * min w over Omega (w counts frames, >= 1)
    st = gv.regularize(D.reg_params(LAM, iters=200, kernel=D.DN_K_FUSED, gamma=gam))
    u = np.zeros_like(ov.f); ub = np.zeros_like(u); p = np.zeros((3,) + u.shape)
    state = np.array([TAU, SIG])
    oracle.cp_accel(ov.nbr, ov.f, ov.w, u, ub, p, 200, LAM, gam, state)
    gu, gub, gp = state_of(D, gv)
    assert np.abs(gu - u).max() <= TOL_U
    assert np.sqrt((gp ** 2).sum(0)).max() <= 1.0 + 1e-6
    E, Dd = oracle.energy(ov.nbr, ov.f, ov.w, u, p, LAM)
    assert abs(st.rel_gap - (E - Dd) / E) <= 1e-3 * (E - Dd) / E + 1e-7
    # split run continues the schedule exactly
    gv.regularize(D.reg_params(LAM, iters=120, kernel=D.DN_K_FUSED, gamma=gam))
    gv.regularize(D.reg_params(LAM, iters=80, kernel=D.DN_K_FUSED, gamma=gam, init=D.DN_INIT_KEEP))
    for x, y in zip(state_of(D, gv), (gu, gub, gp)):
        np.testing.assert_array_equal(x, y)
    # it reaches the gap target in far fewer iterations than fixed steps
    a = gv.regularize(D.reg_params(LAM, iters=3000, gap_every=10, gap_tol=1e-3, kernel=D.DN_K_FUSED, gamma=gam))
    b = gv.regularize(D.reg_params(LAM, iters=3000, gap_every=10, gap_tol=1e-3, kernel=D.DN_K_FUSED))
    print(f"iterations to rel gap 1e-3: accelerated {a.iters_run}, fixed steps {b.iters_run}")
    assert a.converged and b.converged and 3 * a.iters_run < b.iters_run


def test_continuous_regularisation_interleaved_with_fusion():
    """Fuse a frame, iterate, fuse the next, continue: old blocks keep their
    state, new blocks start at u = f.  Checked step by step against the
    oracle running the same sequence."""
    D = dn()
    fr = scenes.frames_c1(1)
    cam = fr.camera
    K = intr(D, cam)
    ov = oracle.OracleVolume(fr.voxel_size, fr.mu, fr.max_depth, 4096, 12, 256)
    gv = D.Volume(fr.voxel_size, fr.mu, fr.max_depth, 4096, 12, 256)
    u = np.zeros((0, 512)); ub = np.zeros((0, 512)); p = np.zeros((3, 0, 512))
    for d, T in zip(fr.depths, fr.poses):
        ov.integrate(d, K4(cam), T)
        gv.integrate(to_dev(d), K, T)
        nnew = ov.nb - u.shape[0]
        f32 = host(gv.extract(D.DN_X_F)).astype(np.float64)
        u = np.concatenate([u, f32[u.shape[0]:]])
        ub = np.concatenate([ub, f32[ub.shape[0]:]])
        p = np.concatenate([p, np.zeros((3, nnew, 512))], axis=1)
        u = np.ascontiguousarray(u); ub = np.ascontiguousarray(ub); p = np.ascontiguousarray(p)
        oracle.cp(ov.nbr, f32, ov.w, u, ub, p, 30, LAM, TAU, SIG, 1.0)
        gv.regularize(D.reg_params(LAM, iters=30, kernel=D.DN_K_FUSED, init=D.DN_INIT_CONTINUE))
        gu = host(gv.extract(D.DN_X_U))
        assert np.abs(gu - u).max() <= TOL_U


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_mixed_precision_early_stop_leaves_the_current_state(c1, storage):
    """A 16-bit run that reaches gap_tol between refinement sweeps leaves its
    current state in the FP32 buffers: DN_X_U, the reported energies and an
    FP32 continuation all see the state after iters_run iterations."""
    D = dn()
    fr, ov, gv = c1
    s = D.DN_F16 if storage == "f16" else D.DN_BF16
    st = gv.regularize(D.reg_params(LAM, iters=200, storage=s, refine_every=50, gap_every=10, gap_tol=0.2))
    k = st.iters_run
    assert st.converged and 0 < k < 50 and k % 10 == 0
    u = np.zeros_like(ov.f); ub = np.zeros_like(u); p = np.zeros((3,) + u.shape)
    oracle.cp(ov.nbr, ov.f, ov.w, u, ub, p, k, LAM, TAU, SIG, 1.0)
    gu = host(gv.extract(D.DN_X_U)).astype(np.float64)
    om = ov.w > 0
    err = np.abs(gu - u)[om]
    print(f"{storage} stopped at {k}: max {err.max():.3e} median {np.median(err):.3e}")
    assert err.max() <= (2e-2 if storage == "f16" else 1.5e-1)
    E, Dd = gv.energy(LAM)
    assert abs(E - st.energy) <= 1e-12 * abs(E) and abs(Dd - st.dual) <= 1e-12 * abs(E)
    # an FP32 continuation starts from that state: its first iteration equals
    # the oracle's iteration from the extracted FP32 state
    gu0, gub0, gp0 = state_of(D, gv)
    gv.regularize(D.reg_params(LAM, iters=1, init=D.DN_INIT_KEEP, kernel=D.DN_K_FUSED))
    u1, ub1, p1 = gu0.copy(), gub0.copy(), gp0.copy()
    oracle.cp(ov.nbr, ov.f, ov.w, u1, ub1, p1, 1, LAM, TAU, SIG, 1.0)
    assert np.abs(host(gv.extract(D.DN_X_U)) - u1).max() <= 1e-5


def test_non_finite_data_is_a_numeric_error():
    """A NaN in the fused TSDF of an observed voxel makes the energy
    non-finite: dn_regularize returns DN_E_NUMERIC at its gap check."""
    D = dn()
    import torch
    coords, f, w = scenes.random_block_field(6, 3, extent=2, omega_frac=0.8)
    gv = D.Volume(0.1, 0.3, 10.0, 64, 8, 64)
    assert gv.insert_blocks(to_dev(coords.astype(np.int32))) == len(coords)
    f = f.copy()
    i = np.argwhere(w > 0)[0]
    f[i[0], i[1]] = np.nan
    gv.load_fused(to_dev(f, torch.float32), to_dev(w, torch.float32))
    with pytest.raises(D.DenserError) as e:
        gv.regularize(D.reg_params(LAM, iters=20, gap_every=10, kernel=D.DN_K_FUSED))
    assert e.value.code == D.DN_E_NUMERIC
    # without gap checks the final energy is the one that fails
    with pytest.raises(D.DenserError) as e:
        gv.regularize(D.reg_params(LAM, iters=5, kernel=D.DN_K_FUSED))
    assert e.value.code == D.DN_E_NUMERIC


def test_ordered_insertion_keeps_first_occurrence_order():
    """dn_insert_blocks_ordered appends the new keys in the order of their
    first occurrence (repeats and keys already present ignored); the block
    set, the hash lookups and the neighbour table are those of the
    ascending insertion of the same keys, up to the permutation."""
    D = dn()
    rng = np.random.default_rng(5)
    keys = rng.integers(-6, 6, size=(900, 3)).astype(np.int32)   # 12^3 cells: repeats certain
    pre = keys[::7][:40].copy()
    vols = []
    for keep in (True, False):
        v = D.Volume(0.1, 0.3, 10.0, 4096, 13, 1024, max_points=0)
        n0 = v.insert_blocks(to_dev(pre))
        n1 = v.insert_blocks(to_dev(keys), keep_order=keep)
        vols.append((v, n0, n1))
    (va, a0, a1), (vb, b0, b1) = vols
    seen = set(map(tuple, pre.tolist()))
    expect = []
    for k in map(tuple, keys.tolist()):
        if k not in seen:
            seen.add(k)
            expect.append(k)
    assert a0 == b0 == len(set(map(tuple, pre.tolist())))
    assert a1 == b1 == len(expect)
    ca = host(va.extract(D.DN_X_COORDS))
    cb = host(vb.extract(D.DN_X_COORDS))
    np.testing.assert_array_equal(ca[:a0], cb[:b0])                     # the earlier blocks stay put
    np.testing.assert_array_equal(ca[a0:], np.array(expect, np.int32))  # new ones in first-occurrence order
    assert sorted(map(tuple, ca.tolist())) == sorted(map(tuple, cb.tolist()))
    # neighbour tables: the same neighbour coordinates (or none) per block
    na = host(va.extract(D.DN_X_NBR))
    nb = host(vb.extract(D.DN_X_NBR))
    ib = {tuple(c): i for i, c in enumerate(cb.tolist())}
    for i, c in enumerate(ca.tolist()):
        j = ib[tuple(c)]
        for o in range(27):
            x, y = na[i, o], nb[j, o]
            assert (x < 0) == (y < 0)
            if x >= 0:
                assert tuple(ca[x]) == tuple(cb[y])
    # a second ordered call with only known keys adds nothing
    assert va.insert_blocks(to_dev(keys[::-1].copy()), keep_order=True) == 0
    # a full pool leaves the volume unchanged; an empty list adds nothing
    small = D.Volume(0.1, 0.3, 10.0, 16, 8, 64, max_points=0, max_candidates=256)
    with pytest.raises(D.DenserError) as e:
        small.insert_blocks(to_dev(keys[:200].copy()), keep_order=True)
    assert e.value.code == D.DN_E_CAPACITY and small.num_blocks == 0
    assert small.insert_blocks(to_dev(np.zeros((0, 3), np.int32)), keep_order=True) == 0
    first = []
    for k in map(tuple, keys[:12].tolist()):
        if k not in first:
            first.append(k)
    assert small.insert_blocks(to_dev(keys[:12].copy()), keep_order=True) == len(first)
    np.testing.assert_array_equal(host(small.extract(D.DN_X_COORDS)), np.array(first, np.int32))
