"""Pins of the oracle's zero-level-set mesh (marching tetrahedra over fully
observed cubes) against closed forms and invariants: planes are
reproduced exactly with the exact area, a sphere's area approaches
4 pi R^2, the mesh of a closed surface is watertight with outward normals,
and cubes with an unobserved corner emit nothing.  CPU only."""
import numpy as np
import pytest

import oracle


def _region(nbx, nby, nbz, s, field, origin=(0, 0, 0)):
    """Fully observed blocks [origin, origin + n) with u = field(x, y, z) at
    the voxel centres (world coordinates)."""
    coords = np.array([[origin[0] + x, origin[1] + y, origin[2] + z]
                       for x in range(nbx) for y in range(nby) for z in range(nbz)], np.int32)
    cap = 1 << 10
    rc, slots = oracle.hash_build(coords, cap, 64)
    assert rc == oracle.OK
    nbr = oracle.nbr_table(coords, slots, cap, 64)
    v = np.arange(512)
    loc = np.stack([v % 8, (v // 8) % 8, v // 64], 1)
    g = (8 * coords[:, None, :] + loc[None]).astype(np.float64)
    P = (g + 0.5) * s
    u = field(P[..., 0], P[..., 1], P[..., 2])
    w = np.ones((len(coords), 512))
    return coords, nbr, w, u, g


@pytest.mark.parametrize("a,b", [(0.0, 0.0), (0.2, -0.1)])
def test_plane_is_exact(a, b):
    s = 0.1
    z0 = 0.83
    coords, nbr, w, u, g = _region(2, 2, 2, s, lambda x, y, z: z - z0 - a * (x - 0.8) - b * (y - 0.8))
    tris, area = oracle.mesh(coords, nbr, w, u, s)
    assert len(tris) > 0
    x, y, z = tris[..., 0], tris[..., 1], tris[..., 2]
    assert np.abs(z - z0 - a * (x - 0.8) - b * (y - 0.8)).max() < 1e-12
    # the cubes span voxel centres 0.5 s .. 15.5 s in x and y
    side = 15 * s
    assert abs(area - side * side * np.sqrt(1 + a * a + b * b)) < 1e-9
    # normals point to u > 0 (+z side)
    n = np.cross(tris[:, 1] - tris[:, 0], tris[:, 2] - tris[:, 0])
    assert (n[:, 2] > 0).all()


def _sphere(R, s=1.0):
    c = 12.0 * s
    return _region(3, 3, 3, s, lambda x, y, z: np.sqrt((x - c) ** 2 + (y - c) ** 2 + (z - c) ** 2) - R), c


def test_sphere_area_watertight_and_outward():
    R = 7.3
    (coords, nbr, w, u, g), c = _sphere(R)
    tris, area = oracle.mesh(coords, nbr, w, u, 1.0)
    assert abs(area / (4 * np.pi * R * R) - 1.0) < 0.02
    # every edge (as a pair of bit-identical points) is shared by two triangles
    edges = {}
    for t in tris:
        pts = [tuple(p) for p in t]
        for i in range(3):
            e = tuple(sorted((pts[i], pts[(i + 1) % 3])))
            edges[e] = edges.get(e, 0) + 1
    counts = np.array(list(edges.values()))
    assert (counts == 2).all()
    n = np.cross(tris[:, 1] - tris[:, 0], tris[:, 2] - tris[:, 0])
    out = tris.mean(1) - c
    assert ((n * out).sum(1) > 0).all()
    # vertices lie on the sphere up to the interpolation error of a voxel
    r = np.sqrt(((tris - c) ** 2).sum(-1))
    assert np.abs(r - R).max() < 0.1


def test_unobserved_corner_removes_its_cubes():
    R = 7.3
    (coords, nbr, w, u, g), c = _sphere(R)
    tris0, _ = oracle.mesh(coords, nbr, w, u, 1.0)
    # a voxel next to the surface: the eight cubes that contain it vanish
    b, v = 13, None
    d = np.abs(np.sqrt(((g[b] + 0.5 - c) ** 2).sum(1)) - R)
    v = int(np.argmin(d))
    q = g[b, v] + 0.5
    w2 = w.copy(); w2[b, v] = 0.0
    tris1, _ = oracle.mesh(coords, nbr, w2, u, 1.0)
    assert 0 < len(tris1) < len(tris0)
    inside = np.all(np.abs(tris1 - q) < 1.0 - 1e-12, axis=-1)
    assert not inside.any()
    # a voxel far from the surface changes nothing
    far = int(np.argmax(d))
    w3 = w.copy(); w3[b, far] = 0.0
    if d[far] > 3.0:
        tris2, _ = oracle.mesh(coords, nbr, w3, u, 1.0)
        np.testing.assert_array_equal(tris2, tris0)
