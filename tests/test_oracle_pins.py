"""Pins of the FP64 oracle against facts that do not come from the oracle
itself: closed forms, invariants, textbook special cases, brute force on
tiny inputs and library routines.  CPU only."""
import itertools
import os

import numpy as np
import pytest

import oracle
import scenes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

LAM, TAU, SIG = 0.5, 1.0 / np.sqrt(12.0), 1.0 / np.sqrt(12.0)


def _volume_from_blocks(coords, cap_log2=10, tail=64):
    cap = 1 << cap_log2
    rc, slots = oracle.hash_build(coords, cap, tail)
    assert rc == oracle.OK
    return slots, oracle.nbr_table(coords, slots, cap, tail)


# ------------------------------------------------------------------ fusion
def _plane_setup(yaw, pitch):
    cam = scenes.Camera(40.0, 40.0, 15.5, 11.5, 32, 24)
    K4 = [cam.fx, cam.fy, cam.cx, cam.cy]
    poses, depths = [], []
    base = scenes.pose_yaw(yaw, 0.3, -0.2, 0.1, pitch)
    axis = base[:3, 2]
    Z0 = 3.0  # plane at distance Z0 along the optical axis from the first pose
    for k, shift in enumerate([0.0, 0.25, 0.55]):
        T = base.copy()
        T[:3, 3] = base[:3, 3] + shift * axis
        poses.append(T)
        depths.append(np.full((cam.height, cam.width), Z0 - shift, np.float32))
    return cam, K4, poses, depths, Z0, base


@pytest.mark.parametrize("yaw,pitch", [(0.0, 0.0), (0.37, -0.21)])
def test_fusion_fronto_parallel_plane_closed_form(yaw, pitch):
    """A plane seen fronto-parallel from poses moving along the optical axis
    has constant depth, so for every voxel f is the mean over frames of
    min(1, (d_k - z_k)/mu) where (d_k - z_k) >= -mu and w counts those frames
    (Eq. 1).  The expectation below uses the pose's columns as camera axes,
    which pins the use of T^-1 (a transposed rotation fails it)."""
    cam, K4, poses, depths, Z0, base = _plane_setup(yaw, pitch)
    s, mu = 0.1, 0.3
    # blocks covering the region in front of and behind the plane
    c0 = np.floor((base[:3, 3] + Z0 * base[:3, 2]) / (8 * s)).astype(int)
    coords = np.array([c0 + np.array(o) for o in itertools.product(range(-2, 3), repeat=3)],
                      np.int32)
    nb = len(coords)
    f = np.zeros((nb, 512))
    w = np.zeros((nb, 512))
    for d, T in zip(depths, poses):
        oracle.fuse(coords, f, w, d, K4, T, s, mu, 100.0)
    l = np.arange(512)
    loc = np.stack([l % 8, (l // 8) % 8, l // 64], 1)
    g = coords[:, None, :] * 8 + loc[None]
    pg = (g + 0.5) * s
    num = np.zeros((nb, 512))
    cnt = np.zeros((nb, 512))
    ambiguous = np.zeros((nb, 512), bool)
    for d, T in zip(depths, poses):
        R, t = T[:3, :3], T[:3, 3]
        rel = pg - t
        xc, yc, zc = (rel @ R[:, 0]), (rel @ R[:, 1]), (rel @ R[:, 2])
        with np.errstate(divide="ignore", invalid="ignore"):
            vx = cam.fx * xc / zc + cam.cx + 0.5
            vy = cam.fy * yc / zc + cam.cy + 0.5
        eta = float(d[0, 0]) - zc
        inside = (zc > 0) & (vx >= 0) & (vx < cam.width) & (vy >= 0) & (vy < cam.height)
        upd = inside & (eta >= -mu)
        num += np.where(upd, np.minimum(1.0, eta / mu), 0.0)
        cnt += upd
        tol = 1e-9
        near = (np.abs(vx) < tol) | (np.abs(vx - cam.width) < tol) | (np.abs(vy) < tol) | \
               (np.abs(vy - cam.height) < tol) | (np.abs(eta + mu) < tol)
        ambiguous |= near
    ok = ~ambiguous
    assert ok.mean() > 0.95
    np.testing.assert_array_equal(w[ok], cnt[ok])
    exp_f = np.where(cnt > 0, num / np.maximum(cnt, 1), 0.0)
    np.testing.assert_allclose(f[ok], exp_f[ok], atol=1e-12)
    # the plane itself: voxels observed in all frames exist and straddle 0
    assert (cnt == 3).sum() > 1000
    assert f[cnt == 3].min() < -0.5 and f[cnt == 3].max() > 0.99


def test_fusion_invalid_pixels_and_behind_camera_are_ignored():
    cam, K4, poses, depths, Z0, base = _plane_setup(0.2, 0.1)
    s, mu = 0.1, 0.3
    c0 = np.floor((base[:3, 3] + Z0 * base[:3, 2]) / (8 * s)).astype(int)
    coords = np.array([c0 + np.array(o) for o in itertools.product(range(-2, 3), repeat=3)],
                      np.int32)
    bad = np.full_like(depths[0], np.nan)
    bad[::2, ::2] = 0.0
    bad[1::2, ::2] = -1.0
    bad[::2, 1::2] = np.inf
    bad[1::2, 1::2] = 150.0  # beyond max_depth
    f = np.zeros((len(coords), 512)); w = np.zeros_like(f)
    oracle.fuse(coords, f, w, bad, K4, poses[0], s, mu, 100.0)
    assert not w.any() and not f.any()
    # camera turned around: every voxel is behind it
    T = poses[0].copy()
    T[:3, :3] = T[:3, :3] @ np.diag([-1.0, 1.0, -1.0])
    oracle.fuse(coords, f, w, depths[0], K4, T, s, mu, 100.0)
    assert not w.any()


# -------------------------------------------------------------- allocation
def _segment_blocks_bruteforce(A, B, bs, n=4001):
    t = np.linspace(0.0, 1.0, n)[:, None]
    P = A[None] + t * (B - A)[None]
    return set(map(tuple, np.floor(P / bs).astype(int)))


def _segment_hits_box(A, B, lo, hi, eps=1e-9):
    d = B - A
    t0, t1 = 0.0, 1.0
    for i in range(3):
        if abs(d[i]) < 1e-300:
            if A[i] < lo[i] - eps or A[i] > hi[i] + eps:
                return False
            continue
        a, b = (lo[i] - eps - A[i]) / d[i], (hi[i] + eps - A[i]) / d[i]
        a, b = min(a, b), max(a, b)
        t0, t1 = max(t0, a), min(t1, b)
    return t0 <= t1


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_allocation_band_equals_segment_block_set(seed):
    """Every block the band segment [d-mu, d+mu] of a pixel passes through is
    emitted, and nothing else (brute-force sampling of the segment plus an
    exact segment/box test)."""
    rng = np.random.default_rng(seed)
    cam = scenes.Camera(20.0, 20.0, 3.5, 2.5, 8, 6)
    K4 = [cam.fx, cam.fy, cam.cx, cam.cy]
    T = scenes.pose_yaw(rng.uniform(-1, 1), *rng.uniform(-3, 3, 3), pitch=rng.uniform(-0.5, 0.5))
    depth = rng.uniform(0.5, 6.0, (cam.height, cam.width)).astype(np.float32)
    depth[0, 0] = 0.0
    s, mu = 0.07, 0.45
    bs = 8 * s
    got = oracle.candidates(depth, K4, T, s, mu, 10.0)
    R, t = T[:3, :3], T[:3, 3]
    ofs = 0
    for y in range(cam.height):
        for x in range(cam.width):
            d = float(depth[y, x])
            if not (d > 0):
                continue
            r = np.array([(x - cam.cx) / cam.fx, (y - cam.cy) / cam.fy, 1.0])
            z0, z1 = max(d - mu, 1e-3), d + mu
            A, B = R @ (z0 * r) + t, R @ (z1 * r) + t
            sampled = _segment_blocks_bruteforce(A, B, bs)
            # count of this pixel's keys: DDA visits 1 + sum |e - k| blocks
            n = 1 + int(np.abs(np.floor(B / bs) - np.floor(A / bs)).sum())
            mine = got[ofs:ofs + n]
            ofs += n
            mine_set = set(map(tuple, mine.tolist()))
            assert len(mine_set) == n  # a traversal never revisits a block
            assert sampled <= mine_set
            for k in mine_set:
                lo = np.array(k) * bs
                assert _segment_hits_box(A, B, lo, lo + bs)
            # consecutive blocks are face neighbours
            assert (np.abs(np.diff(mine, axis=0)).sum(1) == 1).all()
    assert ofs == len(got)


def test_volume_alloc_appends_sorted_and_never_renumbers():
    fr = scenes.frames_c1(0)
    cam = fr.camera
    K4 = [cam.fx, cam.fy, cam.cx, cam.cy]
    vol = oracle.OracleVolume(fr.voxel_size, fr.mu, fr.max_depth, 4096, 11, 64)
    prev = np.zeros((0, 3), np.int32)
    for d, T in zip(fr.depths, fr.poses):
        n = vol.alloc(d, K4, T)
        assert n >= 0
        np.testing.assert_array_equal(vol.coords[:len(prev)], prev)
        new = vol.coords[len(prev):]
        assert len(np.unique(vol.coords, axis=0)) == vol.nb
        if len(new) > 1:
            order = np.lexsort((new[:, 2], new[:, 1], new[:, 0]))
            np.testing.assert_array_equal(order, np.arange(len(new)))
        prev = vol.coords.copy()
    # capacity: a volume too small for the first frame is left unchanged
    small = oracle.OracleVolume(fr.voxel_size, fr.mu, fr.max_depth, 10, 11, 64)
    assert small.alloc(fr.depths[0], K4, fr.poses[0]) == oracle.E_CAPACITY
    assert small.nb == 0
    tiny_hash = oracle.OracleVolume(fr.voxel_size, fr.mu, fr.max_depth, 4096, 4, 2)
    assert tiny_hash.alloc(fr.depths[0], K4, fr.poses[0]) == oracle.E_CAPACITY
    assert tiny_hash.nb == 0


def test_allocation_covers_every_band_voxel_c1():
    """Every voxel whose centre fuses with |eta| <= mu lies in an allocated
    block (fusion never needs a block that allocation did not create)."""
    fr = scenes.frames_c1(0)
    cam = fr.camera
    K4 = [cam.fx, cam.fy, cam.cx, cam.cy]
    vol = oracle.OracleVolume(fr.voxel_size, fr.mu, fr.max_depth, 4096, 11, 64)
    for d, T in zip(fr.depths, fr.poses):
        assert vol.integrate(d, K4, T) >= 0
    # grow a shell of blocks around the allocated set and fuse into it:
    # no voxel there may receive a band observation (|eta| < mu - 1e-9)
    shell = set()
    have = set(map(tuple, vol.coords.tolist()))
    for c in vol.coords:
        for o in itertools.product((-1, 0, 1), repeat=3):
            k = tuple(c + np.array(o))
            if k not in have:
                shell.add(k)
    shell = np.array(sorted(shell), np.int32)
    for d, T in zip(fr.depths, fr.poses):
        f = np.zeros((len(shell), 512)); w = np.zeros_like(f)
        oracle.fuse(shell, f, w, d, K4, T, fr.voxel_size, fr.mu, fr.max_depth)
        band = (w > 0) & (np.abs(f) < 1.0 - 1e-6)
        assert band.sum() == 0


# -------------------------------------------------------------------- hash
@pytest.mark.parametrize("seed,cap_log2,tail", [(0, 6, 40), (1, 4, 64), (2, 10, 8)])
def test_hash_linear_probing_invariants(seed, cap_log2, tail):
    rng = np.random.default_rng(seed)
    n = min(50, (1 << cap_log2) + tail // 2)
    keys = np.unique(rng.integers(-300, 300, (n, 3)), axis=0).astype(np.int32)
    rng.shuffle(keys)
    cap = 1 << cap_log2
    rc, slots = oracle.hash_build(keys, cap, tail)
    assert rc == oracle.OK
    occ = slots[:, 3] >= 0
    assert occ.sum() == len(keys)
    assert sorted(slots[occ, 3].tolist()) == list(range(len(keys)))
    pos_of = {}
    for pos in np.nonzero(occ)[0]:
        x, y, z, i = slots[pos]
        np.testing.assert_array_equal(keys[i], (x, y, z))
        home = oracle.hash_home(x, y, z, cap)
        assert home <= pos
        assert occ[home:pos + 1].all()      # probing path is unbroken
        pos_of[(x, y, z)] = pos
    # canonical order: along the table, (home, key) never decreases
    seq = [(oracle.hash_home(*slots[p][:3], cap), tuple(slots[p][:3])) for p in np.nonzero(occ)[0]]
    for a, b in zip(seq, seq[1:]):
        if a[0] <= b[0]:
            continue
        pytest.fail("keys out of canonical order")
    for k in keys:
        assert oracle.hash_find(slots, cap, tail, *k) >= 0
    for k in rng.integers(400, 600, (20, 3)):
        assert oracle.hash_find(slots, cap, tail, *k) == -1


def test_hash_capacity_error():
    keys = np.stack([np.arange(40), np.zeros(40), np.zeros(40)], 1).astype(np.int32)
    rc, _ = oracle.hash_build(keys, 16, 4)
    assert rc == oracle.E_CAPACITY


def test_neighbour_table_matches_dictionary():
    coords, f, w = scenes.random_block_field(60, 3, extent=5)
    slots, nbr = _volume_from_blocks(coords, cap_log2=5, tail=64)
    ids = {tuple(c): i for i, c in enumerate(coords.tolist())}
    for b, c in enumerate(coords.tolist()):
        for dz, dy, dx in itertools.product((-1, 0, 1), repeat=3):
            k = (c[0] + dx, c[1] + dy, c[2] + dz)
            assert nbr[b, (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)] == ids.get(k, -1)


# ---------------------------------------------------------------- operators
@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_gradient_divergence_adjoint(seed):
    """div is the negative adjoint of the masked gradient (Eq. 4 is defined
    as the dual of Eq. 3): <grad u, p> = -<u, div p> for any u, p."""
    coords, f, w = scenes.random_block_field(40, seed, extent=4, omega_frac=0.7)
    _, nbr = _volume_from_blocks(coords)
    rng = np.random.default_rng(100 + seed)
    u = rng.normal(size=(len(coords), 512))
    p = rng.normal(size=(3, len(coords), 512))
    g = oracle.grad(nbr, w, u)
    d = oracle.div(nbr, w, p)
    lhs, rhs = (g * p).sum(), -(u * d).sum()
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + abs(rhs) + 1.0)
    # sum of a divergence over the whole domain is zero (grad of a constant is 0)
    assert abs(d.sum()) < 1e-10 * np.abs(d).sum()
    # masking: no gradient touches a voxel outside Omega
    assert not g[:, w == 0].any() and not d[w == 0].any()


def test_gradient_masks_match_independent_dictionary():
    """Eq. (3) component by component from a dictionary of global voxels."""
    coords, f, w = scenes.random_block_field(20, 5, extent=3, omega_frac=0.6)
    _, nbr = _volume_from_blocks(coords)
    rng = np.random.default_rng(5)
    u = rng.normal(size=(len(coords), 512))
    g = oracle.grad(nbr, w, u)
    vox = {}
    for b, c in enumerate(coords.tolist()):
        for v in range(512):
            gg = (8 * c[0] + v % 8, 8 * c[1] + (v // 8) % 8, 8 * c[2] + v // 64)
            vox[gg] = (u[b, v], w[b, v] > 0)
    for b, c in enumerate(coords.tolist()):
        for v in range(0, 512, 7):
            gg = (8 * c[0] + v % 8, 8 * c[1] + (v // 8) % 8, 8 * c[2] + v // 64)
            for a in range(3):
                nb_ = list(gg); nb_[a] += 1
                u0, o0 = vox[gg]
                u1, o1 = vox.get(tuple(nb_), (0.0, False))
                exp = (u1 - u0) if (o0 and o1) else 0.0
                assert g[a, b, v] == exp


def _dense_rof_cp(f, w, iters, lam, tau, sigma, theta):
    """Textbook Chambolle-Pock for weighted ROF on a dense grid with Neumann
    boundaries (forward differences, zero at the last index; divergence the
    negative adjoint).  Arrays indexed [z][y][x]."""
    def grad(u):
        g = np.zeros((3,) + u.shape)
        g[0, :, :, :-1] = u[:, :, 1:] - u[:, :, :-1]
        g[1, :, :-1, :] = u[:, 1:, :] - u[:, :-1, :]
        g[2, :-1, :, :] = u[1:, :, :] - u[:-1, :, :]
        return g

    def div(p):
        d = np.zeros(p.shape[1:])
        for a, ax in ((0, 2), (1, 1), (2, 0)):
            q = np.moveaxis(p[a], ax, 0)
            dd = np.zeros_like(q)
            dd[:-1] += q[:-1]
            dd[1:] -= q[:-1]
            d += np.moveaxis(dd, 0, ax)
        return d

    u = np.zeros_like(f); ub = u.copy(); p = np.zeros((3,) + f.shape)
    for _ in range(iters):
        pt = p + sigma * grad(ub)
        p = pt / np.maximum(1.0, np.sqrt((pt ** 2).sum(0)))
        un = (u + tau * div(p) + tau * lam * w * f) / (1.0 + tau * lam * w)
        ub = un + theta * (un - u)
        u = un
    return u, p


def _blocks_to_dense(coords, a, nbx, nby, nbz):
    out = np.zeros((8 * nbz, 8 * nby, 8 * nbx))
    for b, c in enumerate(coords.tolist()):
        out[8 * c[2]:8 * c[2] + 8, 8 * c[1]:8 * c[1] + 8, 8 * c[0]:8 * c[0] + 8] = \
            a[b].reshape(8, 8, 8)
    return out


def test_fully_observed_box_equals_dense_grid_rof():
    """A box of allocated blocks with every voxel observed is a legacy dense
    grid: the masked operators reduce to Neumann forward differences and the
    iteration must equal textbook dense CP."""
    nbx, nby, nbz = 3, 2, 2
    coords = np.array([(x, y, z) for z in range(nbz) for y in range(nby) for x in range(nbx)],
                      np.int32)
    rng = np.random.default_rng(11)
    f = rng.uniform(-1, 1, (len(coords), 512))
    w = rng.integers(1, 5, (len(coords), 512)).astype(float)
    _, nbr = _volume_from_blocks(coords)
    u = np.zeros_like(f); ub = np.zeros_like(f); p = np.zeros((3,) + f.shape)
    oracle.cp(nbr, f, w, u, ub, p, 60, LAM, TAU, SIG, 1.0)
    ud, pd = _dense_rof_cp(_blocks_to_dense(coords, f, nbx, nby, nbz),
                           _blocks_to_dense(coords, w, nbx, nby, nbz), 60, LAM, TAU, SIG, 1.0)
    np.testing.assert_allclose(_blocks_to_dense(coords, u, nbx, nby, nbz), ud, atol=1e-12)
    for a in range(3):
        np.testing.assert_allclose(_blocks_to_dense(coords, p[a], nbx, nby, nbz), pd[a], atol=1e-12)


def _two_voxel_case(f1, f2, w1, w2, iters=4000):
    # voxel 1 at local x = 7 of block (0,0,0), voxel 2 at local x = 0 of (1,0,0)
    coords = np.array([[0, 0, 0], [1, 0, 0]], np.int32)
    _, nbr = _volume_from_blocks(coords)
    f = np.zeros((2, 512)); w = np.zeros((2, 512))
    f[0, 7], w[0, 7] = f1, w1
    f[1, 0], w[1, 0] = f2, w2
    u = np.zeros_like(f); ub = np.zeros_like(f); p = np.zeros((3, 2, 512))
    oracle.cp(nbr, f, w, u, ub, p, iters, LAM, TAU, SIG, 1.0, nthreads=1)
    return u[0, 7], u[1, 0], u, w


@pytest.mark.parametrize("f1,f2,w1,w2", [(0.9, -0.8, 3, 2), (0.2, 0.1, 1, 4), (-0.9, 0.95, 2, 2)])
def test_two_voxels_across_a_block_face_closed_form(f1, f2, w1, w2):
    """min |u1 - u2| + lam/2 (w1 (u1-f1)^2 + w2 (u2-f2)^2): the two values
    move towards each other by 1/(lam w_i) or meet at the weighted mean."""
    u1, u2, u, w = _two_voxel_case(f1, f2, w1, w2)
    a, b = 1.0 / (LAM * w1), 1.0 / (LAM * w2)
    if f1 - f2 >= a + b:
        e1, e2 = f1 - a, f2 + b
    elif f2 - f1 >= a + b:
        e1, e2 = f1 + a, f2 - b
    else:
        e1 = e2 = (w1 * f1 + w2 * f2) / (w1 + w2)
    assert abs(u1 - e1) < 1e-6 and abs(u2 - e2) < 1e-6
    # every other voxel is outside Omega and keeps its initial value 0
    mask = w > 0
    assert not u[~mask].any()


def test_constant_field_is_a_fixed_point():
    coords = np.array([[0, 0, 0], [0, 0, 1], [1, 0, 0]], np.int32)
    _, nbr = _volume_from_blocks(coords)
    w = np.full((3, 512), 2.0)
    f = np.full((3, 512), 0.375)
    u = f.copy(); ub = f.copy(); p = np.zeros((3, 3, 512))
    oracle.cp(nbr, f, w, u, ub, p, 50, LAM, TAU, SIG, 1.0)
    assert np.abs(u - 0.375).max() <= 1e-15 and not p.any()
    u = np.zeros_like(f); ub = np.zeros_like(f)
    oracle.cp(nbr, f, w, u, ub, p, 400, LAM, TAU, SIG, 1.0)
    assert np.abs(u - 0.375).max() < 1e-9


def _independent_dual_solver(coords, f, w, lam, iters=30000):
    """FISTA on the smooth dual max_{|p|<=1} D(p) with a gradient matrix
    built from a dictionary of global voxel coordinates (no oracle code).
    Returns the primal minimiser u = f + div p / (lam w) on Omega."""
    import scipy.sparse as sp
    idx = {}
    for b, c in enumerate(coords.tolist()):
        for v in range(512):
            if w[b, v] > 0:
                g = (8 * c[0] + v % 8, 8 * c[1] + (v // 8) % 8, 8 * c[2] + v // 64)
                idx[g] = len(idx)
    N = len(idx)
    rows, cols, vals = [], [], []
    for g, i in idx.items():
        for a in range(3):
            h = list(g); h[a] += 1
            j = idx.get(tuple(h))
            if j is not None:
                r = a * N + i
                rows += [r, r]; cols += [j, i]; vals += [1.0, -1.0]
    G = sp.csr_matrix((vals, (rows, cols)), shape=(3 * N, N))
    fv = np.zeros(N); wv = np.zeros(N)
    for b, c in enumerate(coords.tolist()):
        for v in range(512):
            if w[b, v] > 0:
                g = (8 * c[0] + v % 8, 8 * c[1] + (v // 8) % 8, 8 * c[2] + v // 64)
                fv[idx[g]] = f[b, v]; wv[idx[g]] = w[b, v]
    L = 12.0 / (lam * wv.min())
    p = np.zeros(3 * N); y = p.copy(); tk = 1.0

    def proj(q):
        q3 = q.reshape(3, N)
        return (q3 / np.maximum(1.0, np.sqrt((q3 ** 2).sum(0)))).reshape(-1)

    def u_of(q):
        return fv - (G.T @ q) / (lam * wv)

    for _ in range(iters):
        pn = proj(y + (G @ u_of(y)) / L)
        tn = 0.5 * (1 + np.sqrt(1 + 4 * tk * tk))
        y = pn + ((tk - 1) / tn) * (pn - p)
        p, tk = pn, tn
    u = u_of(p)
    out = np.zeros_like(f)
    for b, c in enumerate(coords.tolist()):
        for v in range(512):
            if w[b, v] > 0:
                g = (8 * c[0] + v % 8, 8 * c[1] + (v // 8) % 8, 8 * c[2] + v // 64)
                out[b, v] = u[idx[g]]
    return out


@pytest.mark.parametrize("seed,lam,iters,tol", [(0, 4.0, 6000, 1e-9), (1, 4.0, 6000, 1e-9),
                                                (0, LAM, 6000, None)])
def test_converges_to_independent_brute_force_minimiser(seed, lam, iters, tol):
    """CP reaches the minimiser found by an independent dual solver.  With a
    strongly convex data term (lam * min w) the primal error is also bounded
    by the gap: |u - u*|^2 <= 2 gap / (lam min w)."""
    coords = np.array([[0, 0, 0], [1, 0, 0]], np.int32)
    rng = np.random.default_rng(seed)
    w = rng.integers(1, 4, (2, 512)).astype(float)
    w[rng.random((2, 512)) < 0.35] = 0.0
    f = np.where(w > 0, rng.uniform(-1, 1, (2, 512)), 0.0)
    _, nbr = _volume_from_blocks(coords)
    u = np.zeros_like(f); ub = np.zeros_like(f); p = np.zeros((3, 2, 512))
    oracle.cp(nbr, f, w, u, ub, p, iters, lam, TAU, SIG, 1.0)
    ref = _independent_dual_solver(coords, f, w, lam)
    E, D = oracle.energy(nbr, f, w, u, p, lam)
    gap = E - D
    assert gap >= 0.0
    err2 = ((u - ref)[w > 0] ** 2).sum()
    assert err2 <= 2.0 * gap / (lam * w[w > 0].min()) + 1e-12
    Eref, _ = oracle.energy(nbr, f, w, ref, p, lam)
    assert Eref <= E + 1e-12 and E - Eref <= gap + 1e-12
    if tol is not None:
        assert np.abs(u - ref)[w > 0].max() < tol
        assert gap < 1e-9 * E


def test_invariants_on_c1_like_sparse_field():
    coords, f, w = scenes.random_block_field(24, 9, extent=4, omega_frac=0.75)
    _, nbr = _volume_from_blocks(coords)
    u = np.zeros_like(f); ub = np.zeros_like(f); p = np.zeros((3,) + f.shape)
    gaps = []
    for k in range(20):
        oracle.cp(nbr, f, w, u, ub, p, 10, LAM, TAU, SIG, 1.0)
        assert np.sqrt((p ** 2).sum(0)).max() <= 1.0 + 1e-15
        assert not u[w == 0].any()
        E, D = oracle.energy(nbr, f, w, u, p, LAM)
        assert E - D >= 0.0
        gaps.append(E - D)
    gaps = np.array(gaps)
    assert (np.diff(gaps) <= 1e-6 * gaps[:-1]).all()
    assert gaps[-1] < 0.05 * gaps[0]


def test_unobserved_data_does_not_leak_and_translation_is_exact():
    coords, f, w = scenes.random_block_field(16, 4, extent=3, omega_frac=0.7)
    _, nbr = _volume_from_blocks(coords)

    def run(c, ff, ww):
        _, nb_ = _volume_from_blocks(c)
        u = np.zeros_like(ff); ub = np.zeros_like(ff); p = np.zeros((3,) + ff.shape)
        oracle.cp(nb_, ff, ww, u, ub, p, 40, LAM, TAU, SIG, 1.0)
        return u
    u0 = run(coords, f, w)
    f2 = f.copy(); f2[w == 0] = 123.0
    np.testing.assert_array_equal(run(coords, f2, w)[w > 0], u0[w > 0])
    shifted = coords + np.array([5, -7, 3], np.int32)
    np.testing.assert_array_equal(run(shifted, f, w), u0)


def test_axis_permutation_equivariance():
    coords, f, w = scenes.random_block_field(12, 6, extent=3, omega_frac=0.8)

    def perm_blocks(c, a, perm):
        # permute global axes: key and voxel layout
        c2 = c[:, perm]
        a4 = a.reshape(-1, 8, 8, 8)  # [b][z][y][x]
        axes_zyx = [2 - perm[2 - i] for i in range(3)]
        return c2, np.ascontiguousarray(a4.transpose([0] + [1 + ax for ax in axes_zyx])).reshape(-1, 512)
    perm = [2, 0, 1]

    def run(c, ff, ww):
        _, nb_ = _volume_from_blocks(c)
        u = np.zeros_like(ff); ub = np.zeros_like(ff); p = np.zeros((3,) + ff.shape)
        oracle.cp(nb_, ff, ww, u, ub, p, 30, LAM, TAU, SIG, 1.0)
        return u
    u0 = run(coords, f, w)
    c2, f2 = perm_blocks(coords, f, perm)
    _, w2 = perm_blocks(coords, w, perm)
    _, u0p = perm_blocks(coords, u0, perm)
    np.testing.assert_allclose(run(c2, f2, w2), u0p, atol=1e-14)


def test_energy_closed_form_on_a_ramp():
    """u = a x on a fully observed box: |grad u| = a except on the last x
    layer, and D(0) = 0."""
    coords = np.array([[0, 0, 0], [1, 0, 0]], np.int32)
    _, nbr = _volume_from_blocks(coords)
    a = 0.125
    gx = np.concatenate([np.arange(512) % 8, 8 + np.arange(512) % 8]).reshape(2, 512)
    u = a * gx
    w = np.full((2, 512), 2.0)
    f = u + 0.5
    E, D = oracle.energy(nbr, f, w, u, np.zeros((3, 2, 512)), LAM)
    n_tv = 15 * 64  # voxels with an x neighbour
    assert abs(E - (a * n_tv + 0.5 * LAM * 2.0 * 0.25 * 1024)) < 1e-10
    assert D == 0.0


# ------------------------------------------------------------------ extract
def test_extract_plane_crossings():
    coords = np.array([(x, y, z) for z in range(2) for y in range(1) for x in range(2)], np.int32)
    _, nbr = _volume_from_blocks(coords)
    s, z0 = 0.1, 0.537
    l = np.arange(512)
    g = coords[:, None, :] * 8 + np.stack([l % 8, (l // 8) % 8, l // 64], 1)[None]
    u = (g[..., 2] + 0.5) * s - z0
    w = np.ones_like(u)
    pts = oracle.extract(coords, nbr, w, u, s)
    assert len(pts) == 16 * 8  # one crossing per (x, y) column
    np.testing.assert_allclose(pts[:, 2], z0, atol=1e-12)
    w[0, :] = 0.0
    assert len(oracle.extract(coords, nbr, w, u, s)) == 16 * 8 - 64


# -------------------------------------------------------------- network
def _rand_params(rng, scale=0.2):
    return rng.normal(0, scale, oracle.NET_PARAMS)


def test_net_forward_matches_torch_conv3d():
    torch = pytest.importorskip("torch")
    import torch.nn.functional as F
    rng = np.random.default_rng(0)
    prm = _rand_params(rng)
    tiles = rng.normal(size=(3, 2, 10, 10, 10))
    out = oracle.net_forward(tiles, prm)
    W1 = prm[:864].reshape(16, 2, 3, 3, 3); b1 = prm[864:880]
    W2 = prm[880:7792].reshape(16, 16, 3, 3, 3); b2 = prm[7792:7808]
    W3 = prm[7808:8240].reshape(1, 16, 3, 3, 3); b3 = prm[8240:8241]
    x = torch.from_numpy(tiles)
    h = F.relu(F.conv3d(x, torch.from_numpy(W1), torch.from_numpy(b1), padding=1))
    h = F.relu(F.conv3d(h, torch.from_numpy(W2), torch.from_numpy(b2), padding=1))
    y = F.conv3d(h, torch.from_numpy(W3), torch.from_numpy(b3), padding=1)
    np.testing.assert_allclose(out, y[:, 0].numpy(), atol=1e-12)


def test_net_gradient_matches_finite_differences():
    rng = np.random.default_rng(1)
    prm = _rand_params(rng, 0.3)
    tiles = rng.normal(size=(2, 2, 10, 10, 10))
    targets = rng.normal(size=(2, 512))
    mask = (rng.random((2, 512)) < 0.7).astype(float)
    L, g = oracle.net_loss_grad(tiles, prm, targets, mask)
    h = 1e-6
    idx = np.concatenate([rng.choice(864, 6, replace=False), 864 + rng.choice(16, 2, replace=False),
                          880 + rng.choice(6912, 8, replace=False), 7792 + rng.choice(16, 2),
                          7808 + rng.choice(432, 6, replace=False), [8240]])
    for i in idx:
        pp = prm.copy(); pp[i] += h
        pm = prm.copy(); pm[i] -= h
        num = (oracle.net_loss_grad(tiles, pp, targets, mask)[0] -
               oracle.net_loss_grad(tiles, pm, targets, mask)[0]) / (2 * h)
        assert abs(num - g[i]) <= 1e-6 * max(1.0, abs(num)), (i, num, g[i])


def _torch_gated_net(torch, tiles, prm, gate):
    """Reference of the oracle network written with torch: float64 values,
    each ReLU opened by the sign of a pre-activation computed either in
    float64 (gate 0) or with operands rounded float64 -> float32 ->
    bfloat16 by torch's own conversions (gate 1; layer-1 weights as the
    pair bf16(W) + bf16(W - bf16(W)))."""
    import torch.nn.functional as F
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a))
    bf = lambda x: x.float().bfloat16().double()
    W1 = t(prm[:864].reshape(16, 2, 3, 3, 3)); b1 = t(prm[864:880])
    W2 = t(prm[880:7792].reshape(16, 16, 3, 3, 3)); b2 = t(prm[7792:7808])
    W3 = t(prm[7808:8240].reshape(1, 16, 3, 3, 3)); b3 = t(prm[8240:8241])
    Ws = [W.clone().requires_grad_(True) for W in (W1, b1, W2, b2, W3, b3)]
    x = t(tiles)
    a1 = F.conv3d(x, Ws[0], Ws[1], padding=1)
    if gate:
        W1p = bf(W1) + bf(W1 - bf(W1))          # layer 1 runs on a weight pair
        g1 = F.conv3d(bf(x), W1p, b1, padding=1)
        m1 = g1 > 0
        g2 = F.conv3d(torch.where(m1, bf(g1), torch.zeros_like(g1)), bf(W2), b2, padding=1)
    else:
        m1 = a1 > 0
    h1 = torch.where(m1, a1, torch.zeros_like(a1))
    a2 = F.conv3d(h1, Ws[2], Ws[3], padding=1)
    m2 = (g2 > 0) if gate else (a2 > 0)
    h2 = torch.where(m2, a2, torch.zeros_like(a2))
    return F.conv3d(h2, Ws[4], Ws[5], padding=1)[:, 0], Ws, (m1, m2)


@pytest.mark.parametrize("gate", [0, 1])
def test_net_gated_forward_and_gradient_match_torch(gate):
    """The ReLU decision in bfloat16 operand precision (gate 1) against a
    torch reference (torch's float -> bfloat16 rounding, conv3d, autograd
    through the fixed activation pattern); gate 0 is the plain network."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(21 + gate)
    prm = _rand_params(rng, 0.25)
    tiles = rng.normal(0, 0.6, size=(2, 2, 10, 10, 10))
    targets = rng.normal(size=(2, 512))
    mask = (rng.random((2, 512)) < 0.7).astype(float)
    out, Ws, (m1, m2) = _torch_gated_net(torch, tiles, prm, gate)
    np.testing.assert_allclose(oracle.net_forward(tiles, prm, gate=gate), out.detach().numpy(), atol=1e-12)
    pred = out[:, 1:9, 1:9, 1:9].reshape(2, 512)
    for kind in (0, 1):
        if kind == 0:
            p_ = pred + torch.from_numpy(tiles[:, 0, 1:9, 1:9, 1:9].reshape(2, 512))
        else:
            p_ = pred
        m = torch.from_numpy(mask)
        loss = (((p_ - torch.from_numpy(targets)) ** 2) * m).sum() / m.sum()
        grads = torch.autograd.grad(loss, Ws, retain_graph=True)
        ref = torch.cat([g_.flatten() for g_ in grads]).numpy()
        L, g = oracle.net_loss_grad(tiles, prm, targets, mask, kind=kind, gate=gate)
        assert abs(L - float(loss.detach())) <= 1e-12 * max(1.0, abs(L))
        np.testing.assert_allclose(g, ref, rtol=1e-10, atol=1e-12)
    if gate:
        # the two decisions differ somewhere (else this pin would not pin the gate)
        _, _, (f1, f2) = _torch_gated_net(torch, tiles, prm, 0)
        assert int((m1 != f1).sum()) + int((m2 != f2).sum()) > 0


def _torch_bf16_net(torch, tiles, prm, acc):
    """The network with every operand rounded float64 -> float32 ->
    bfloat16 by torch's conversions (layer-1 weights as a bfloat16 pair,
    biases unrounded) and the sums in `acc` (torch.float64 or
    torch.float32)."""
    import torch.nn.functional as F
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(acc)
    bf = lambda x: x.float().bfloat16().to(acc)
    W1 = t(prm[:864].reshape(16, 2, 3, 3, 3)); b1 = t(prm[864:880])
    W2 = t(prm[880:7792].reshape(16, 16, 3, 3, 3)); b2 = t(prm[7792:7808])
    W3 = t(prm[7808:8240].reshape(1, 16, 3, 3, 3)); b3 = t(prm[8240:8241])
    W1p = torch.cat([bf(W1), bf(W1 - bf(W1))], 1)          # the pair as two input channels each
    x = bf(t(tiles))
    g1 = F.conv3d(torch.cat([x, x], 1), W1p, b1, padding=1)
    g2 = F.conv3d(bf(torch.relu(g1)), bf(W2), b2, padding=1)
    return F.conv3d(bf(torch.relu(g2)), bf(W3), b3, padding=1)[:, 0]


def test_net_bf16_operand_forward_matches_torch():
    """gate 2 (every operand bfloat16, float64 sums) against the same
    network written with torch's own rounding and conv3d in float64."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(41)
    prm = _rand_params(rng, 0.25)
    tiles = rng.normal(0, 0.6, size=(3, 2, 10, 10, 10))
    ref = _torch_bf16_net(torch, tiles, prm, torch.float64).numpy()
    out = oracle.net_forward(tiles, prm, gate=2)
    np.testing.assert_allclose(out, ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    # it is not the float64 network (the rounding is really there)
    assert np.abs(out - oracle.net_forward(tiles, prm, gate=0)).max() > 1e-3 * np.abs(ref).max()


@pytest.mark.parametrize("seed,scale,weights", [(42, 0.25, None), (43, 0.12, None), (44, 0.3, "trained")])
def test_net_error_rms_predicts_bf16_error(seed, scale, weights):
    """The variance model of bfloat16 operand rounding against two
    evaluations that really round (float64 sums: gate 2; float32 sums:
    torch conv3d in float32): the L2 norm of their difference from the
    float64 network is within a factor 2 of the model's, for random weights
    and for the trained network's (whose cancellation is larger)."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(seed)
    if weights == "trained":
        prm = np.load(os.path.join(ROOT, "paper_1604_03734_amd", "weights", "warmstart.npy")).astype(np.float64)
        tiles = np.stack([rng.normal(0, 0.3, size=(4, 10, 10, 10)), rng.random((4, 10, 10, 10))], 1)
    else:
        prm = _rand_params(rng, scale)
        tiles = rng.normal(0, 0.6, size=(4, 2, 10, 10, 10))
    r64 = oracle.net_forward(tiles, prm, gate=0)
    sig = np.linalg.norm(oracle.net_error_rms(tiles, prm))
    e2 = np.linalg.norm(oracle.net_forward(tiles, prm, gate=2) - r64)
    e32 = np.linalg.norm(_torch_bf16_net(torch, tiles, prm, torch.float32).double().numpy() - r64)
    print(f"model {sig:.3e}, gate 2 {e2:.3e}, float32 sums {e32:.3e}, |r| {np.linalg.norm(r64):.3e}")
    assert 0.5 * sig <= e2 <= 2 * sig and 0.5 * sig <= e32 <= 2 * sig


def test_net_gather_halo_comes_from_neighbours():
    coords, f, w = scenes.random_block_field(20, 8, extent=3, omega_frac=0.9)
    _, nbr = _volume_from_blocks(coords)
    tiles = oracle.net_gather(nbr, f, w, np.arange(len(coords)))
    ids = {tuple(c): i for i, c in enumerate(coords.tolist())}
    for b, c in enumerate(coords.tolist()):
        for (x, y, z) in [(0, 4, 4), (9, 1, 2), (3, 0, 9), (0, 0, 0), (9, 9, 9), (5, 5, 5)]:
            g = (8 * c[0] + x - 1, 8 * c[1] + y - 1, 8 * c[2] + z - 1)
            k = (g[0] // 8, g[1] // 8, g[2] // 8)
            j = ids.get(k)
            v = (g[0] % 8) + 8 * (g[1] % 8) + 64 * (g[2] % 8)
            ef = f[j, v] if j is not None else 0.0
            ew = np.log1p(w[j, v]) / np.log(101.0) if j is not None else 0.0
            assert tiles[b, 0, z, y, x] == ef
            assert abs(tiles[b, 1, z, y, x] - ew) < 1e-15


# ------------------------------------------------- accelerated variant
def test_accelerated_variant_reaches_the_same_minimiser_faster():
    """The uniformly convex variant (gamma = lambda min w) converges to the
    minimiser of the independent dual solver, and its gap after N
    iterations is far below the fixed-step method's."""
    coords = np.array([[0, 0, 0], [1, 0, 0]], np.int32)
    rng = np.random.default_rng(0)
    w = rng.integers(1, 4, (2, 512)).astype(float)
    w[rng.random((2, 512)) < 0.35] = 0.0
    f = np.where(w > 0, rng.uniform(-1, 1, (2, 512)), 0.0)
    _, nbr = _volume_from_blocks(coords)
    ref = _independent_dual_solver(coords, f, w, LAM)
    u = np.zeros_like(f); ub = np.zeros_like(f); p = np.zeros((3, 2, 512))
    state = np.array([TAU, SIG])
    oracle.cp_accel(nbr, f, w, u, ub, p, 150, LAM, LAM * w[w > 0].min(), state)
    # split run resumes exactly
    u2 = np.zeros_like(f); ub2 = np.zeros_like(f); p2 = np.zeros((3, 2, 512))
    st2 = np.array([TAU, SIG])
    oracle.cp_accel(nbr, f, w, u2, ub2, p2, 70, LAM, LAM * w[w > 0].min(), st2)
    oracle.cp_accel(nbr, f, w, u2, ub2, p2, 80, LAM, LAM * w[w > 0].min(), st2)
    np.testing.assert_array_equal(u, u2)
    np.testing.assert_array_equal(state, st2)
    Ea, Da = oracle.energy(nbr, f, w, u, p, LAM)
    uf = np.zeros_like(f); ubf = np.zeros_like(f); pf = np.zeros((3, 2, 512))
    oracle.cp(nbr, f, w, uf, ubf, pf, 150, LAM, TAU, SIG, 1.0)
    Ef, Df = oracle.energy(nbr, f, w, uf, pf, LAM)
    assert 0.0 <= Ea - Da < 0.25 * (Ef - Df)
    err2 = ((u - ref)[w > 0] ** 2).sum()
    assert err2 <= 2.0 * (Ea - Da) / (LAM * w[w > 0].min()) + 1e-12
    # theta, tau, sigma schedule: tau * sigma stays 1/12
    assert abs(state[0] * state[1] - TAU * SIG) < 1e-15


def test_net_gather_axis_exchange_and_dual_loss_kind():
    """perm 1 / 2 exchange the tile's x axis with y / z (a transpose of the
    unpermuted tile); loss kind 1 predicts r alone (its gradient still
    matches finite differences)."""
    coords, f, w = scenes.random_block_field(20, 8, extent=3, omega_frac=0.9)
    _, nbr = _volume_from_blocks(coords)
    blocks = np.arange(len(coords))
    t0 = oracle.net_gather(nbr, f, w, blocks, 0)           # [B][c][z][y][x]
    np.testing.assert_array_equal(oracle.net_gather(nbr, f, w, blocks, 1), t0.transpose(0, 1, 2, 4, 3))
    np.testing.assert_array_equal(oracle.net_gather(nbr, f, w, blocks, 2), t0.transpose(0, 1, 4, 3, 2))
    rng = np.random.default_rng(2)
    prm = _rand_params(rng, 0.3)
    tiles = rng.normal(size=(2, 2, 10, 10, 10))
    targets = rng.normal(size=(2, 512))
    mask = (rng.random((2, 512)) < 0.7).astype(float)
    L, g = oracle.net_loss_grad(tiles, prm, targets, mask, kind=1)
    out = oracle.net_forward(tiles, prm)[:, 1:9, 1:9, 1:9].reshape(2, 512)
    assert abs(L - (((out - targets) ** 2) * mask).sum() / mask.sum()) < 1e-12
    h = 1e-6
    for i in (3, 900, 5000, 7810, 8240):
        pp = prm.copy(); pp[i] += h
        pm = prm.copy(); pm[i] -= h
        num = (oracle.net_loss_grad(tiles, pp, targets, mask, 1)[0] -
               oracle.net_loss_grad(tiles, pm, targets, mask, 1)[0]) / (2 * h)
        assert abs(num - g[i]) <= 1e-6 * max(1.0, abs(num))
