"""Zero-level-set mesh and its area on the GPU against the oracle's,
evaluated on the same float field (the library's u): same triangles in the
same order, area within 1e-9 relative; the regulariser lowers the area."""
import numpy as np
import pytest

import oracle
import scenes
from gpu_common import LAM, dn, fuse_both, host, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c1():
    fr = scenes.frames_c1(0)
    ov, gv = fuse_both(fr, check_each_frame=False)
    return fr, ov, gv


def _compare(D, gv, coords, w, s):
    tris = host(gv.extract(D.DN_X_MESH))
    u = host(gv.extract(D.DN_X_U)).astype(np.float64)
    ref, area = oracle.mesh(coords, host(gv.extract(D.DN_X_NBR)), w, u, s)
    assert tris.shape == ref.shape
    err = np.abs(tris.astype(np.float64) - ref).max() if len(ref) else 0.0
    print(f"{len(ref)} triangles, max |dvertex| {err:.2e} m, area {area:.4f} m^2")
    assert err <= 1e-6
    a, n = gv.mesh_area()
    assert n == len(ref) and abs(a - area) <= 1e-9 * max(area, 1e-30)
    return area


def test_mesh_of_the_fused_and_regularised_c1(c1):
    D = dn()
    fr, ov, gv = c1
    f = gv.extract(D.DN_X_F)
    gv.regularize(D.reg_params(LAM, iters=0, init=D.DN_INIT_GIVEN), u0=f)
    raw = _compare(D, gv, ov.coords, ov.w, fr.voxel_size)
    gv.regularize(D.reg_params(LAM, iters=200, kernel=D.DN_K_FUSED))
    reg = _compare(D, gv, ov.coords, ov.w, fr.voxel_size)
    print(f"area raw {raw:.3f} m^2 -> regularised {reg:.3f} m^2 ({reg / raw - 1:+.1%})")
    assert reg < raw


@pytest.mark.parametrize("nb,seed,extent", [(1, 0, 1), (17, 1, 3), (60, 2, 5)])
def test_mesh_of_random_fields(nb, seed, extent):
    D = dn()
    coords, f, w = scenes.random_block_field(nb, seed, extent=extent, omega_frac=0.9)
    gv = D.Volume(0.05, 0.3, 10.0, nb, 8, 64, max_points=0)
    gv.insert_blocks(to_dev(coords.astype(np.int32)))
    c = host(gv.extract(D.DN_X_COORDS))
    order = np.array([np.nonzero((coords == x).all(1))[0][0] for x in c])
    f, w = f[order].astype(np.float32), w[order].astype(np.float32)
    gv.load_fused(to_dev(f), to_dev(w))
    gv.regularize(D.reg_params(LAM, iters=0, init=D.DN_INIT_GIVEN), u0=to_dev(f))
    _compare(D, gv, c, w.astype(np.float64), 0.05)


def test_mesh_of_an_empty_volume():
    D = dn()
    gv = D.Volume(0.1, 0.3, 10.0, 16, 6, 16, max_points=0)
    assert gv.extract(D.DN_X_MESH).shape == (0, 3, 3)
    assert gv.mesh_area() == (0.0, 0)
