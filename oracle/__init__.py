"""FP64 CPU oracle (TEST INFRASTRUCTURE ONLY).

A plain, slow, obviously correct implementation of what the GPU path
computes, used by the tests, the smoke check and the CPU-baseline leg of the
benchmark.  The product path never imports it.  The arithmetic lives in
`denser_oracle.c` (double precision, gcc -O2 -ffp-contract=off); this module
only marshals numpy arrays and keeps the pool/hash bookkeeping of a volume
with numpy library primitives (unique, sort, isin).

Parity status: every function is pinned by tests/test_oracle_pins.py
against closed forms, invariants, brute force or library routines.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "denser_oracle.c")
# DN_ORACLE_SANITIZE=1: an AddressSanitizer + UndefinedBehaviorSanitizer
# build of the same source (the process must preload libasan; see
# tests/test_oracle_sanitized.py)
_SANITIZE = os.environ.get("DN_ORACLE_SANITIZE") == "1"
_LIB = os.path.join(_HERE, "liboracle_san.so" if _SANITIZE else "liboracle.so")
SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g"]

OK = 0
E_CAPACITY = -2


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (CPU only)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                               "-fPIC", "-shared", "-std=c11"] + (SAN_FLAGS if _SANITIZE else []) +
                              [_SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i32, i64, f64, u32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_uint32
        sig = {
            "or_candidates": (i64, [P, i32, i32, P, P, f64, f64, f64, P, i64]),
            "or_hash_home": (u32, [i32, i32, i32, u32]),
            "or_hash_build": (i32, [P, i64, i32, i32, P]),
            "or_hash_find": (i32, [P, i32, i32, i32, i32, i32]),
            "or_nbr": (None, [P, i64, P, i32, i32, P]),
            "or_fuse": (None, [P, i64, P, P, P, i32, i32, P, P, f64, f64, f64, i32]),
            "or_grad": (None, [P, i64, P, P, P]),
            "or_div": (None, [P, i64, P, P, P]),
            "or_cp": (None, [P, i64, P, P, P, P, P, i32, f64, f64, f64, f64, i32]),
            "or_energy": (None, [P, i64, P, P, P, P, f64, P, i32]),
            "or_cp_accel": (None, [P, i64, P, P, P, P, P, i32, f64, f64, P, i32]),
            "or_cp_l1": (None, [P, i64, P, P, P, P, P, i32, f64, f64, f64, f64, i32]),
            "or_energy_l1": (None, [P, i64, P, P, P, P, f64, P, i32]),
            "or_extract": (i64, [P, P, i64, P, P, f64, P, i64]),
            "or_mesh": (i64, [P, P, i64, P, P, f64, P, i64, P]),
            "or_candidates_laser": (i64, [P, i64, P, f64, f64, f64, P, i64]),
            "or_fuse_laser": (None, [P, i32, i32, i64, P, P, P, i64, P, f64, f64, f64]),
            "or_net_forward": (None, [P, i64, P, P, P, P, i32]),
            "or_net_error_rms": (None, [P, i64, P, P]),
            "or_net_loss_grad": (f64, [P, i64, P, P, P, P, i32, i32]),
            "or_net_gather": (None, [P, P, P, P, i64, P, i32]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def nthreads_default() -> int:
    return int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))


# --------------------------------------------------------------- raw calls
def candidates(depth, K4, T, s, mu, max_depth) -> np.ndarray:
    """Every block key visited by every valid pixel's band (with repeats)."""
    depth = _c(depth, np.float32)
    K4 = _c(K4, np.float64)
    T = _c(T, np.float64)
    H, W = depth.shape
    cap = max(1024, W * H * 8)
    while True:
        out = np.empty((cap, 3), np.int32)
        n = lib().or_candidates(_p(depth), W, H, _p(K4), _p(T), s, mu, max_depth, _p(out), cap)
        if n <= cap:
            return out[:n]
        cap = int(n)


def candidates_laser(pts, T, s, mu, max_depth) -> np.ndarray:
    """Every block key visited by every valid return's band (with repeats)."""
    pts = _c(pts, np.float32).reshape(-1, 3)
    T = _c(T, np.float64)
    cap = max(1024, len(pts) * 16)
    while True:
        out = np.empty((cap, 3), np.int32)
        n = lib().or_candidates_laser(_p(pts), len(pts), _p(T), s, mu, max_depth, _p(out), cap)
        if n <= cap:
            return out[:n]
        cap = int(n)


def hash_home(x, y, z, cap) -> int:
    return int(lib().or_hash_home(int(x), int(y), int(z), int(cap)))


def hash_build(coords, cap, tail):
    coords = _c(coords, np.int32).reshape(-1, 3)
    slots = np.empty((cap + tail, 4), np.int32)
    rc = lib().or_hash_build(_p(coords), len(coords), cap, tail, _p(slots))
    return rc, slots


def hash_find(slots, cap, tail, x, y, z) -> int:
    return int(lib().or_hash_find(_p(slots), cap, tail, int(x), int(y), int(z)))


def nbr_table(coords, slots, cap, tail) -> np.ndarray:
    coords = _c(coords, np.int32).reshape(-1, 3)
    nbr = np.empty((len(coords), 27), np.int32)
    lib().or_nbr(_p(coords), len(coords), _p(slots), cap, tail, _p(nbr))
    return nbr


def fuse(coords, f, w, depth, K4, T, s, mu, max_depth, nthreads=None):
    """In-place Eq. (1) update of f, w (float64 [nb][512])."""
    assert f.dtype == np.float64 and w.dtype == np.float64
    coords = _c(coords, np.int32).reshape(-1, 3)
    depth = _c(depth, np.float32)
    H, W = depth.shape
    lib().or_fuse(_p(coords), len(coords), _p(f), _p(w), _p(depth), W, H,
                  _p(_c(K4, np.float64)), _p(_c(T, np.float64)), s, mu, max_depth,
                  nthreads or nthreads_default())


def grad(nbr, w, u):
    nb = len(nbr)
    g = np.empty((3, nb, 512))
    lib().or_grad(_p(_c(nbr, np.int32)), nb, _p(_c(w, np.float64)), _p(_c(u, np.float64)), _p(g))
    return g


def div(nbr, w, p):
    nb = len(nbr)
    d = np.empty((nb, 512))
    lib().or_div(_p(_c(nbr, np.int32)), nb, _p(_c(w, np.float64)), _p(_c(p, np.float64)), _p(d))
    return d


def cp(nbr, f, w, u, ubar, p, iters, lam, tau, sigma, theta=1.0, nthreads=None):
    """In-place Chambolle-Pock iterations on (u, ubar, p)."""
    for a in (u, ubar, p):
        assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    nb = len(nbr)
    lib().or_cp(_p(_c(nbr, np.int32)), nb, _p(_c(f, np.float64)), _p(_c(w, np.float64)),
                _p(u), _p(ubar), _p(p), int(iters), lam, tau, sigma, theta,
                nthreads or nthreads_default())


def cp_accel(nbr, f, w, u, ubar, p, iters, lam, gamma, state, nthreads=None):
    """Accelerated iterations; state = float64 [tau_n, sigma_n], updated."""
    for a in (u, ubar, p, state):
        assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    nb = len(nbr)
    lib().or_cp_accel(_p(_c(nbr, np.int32)), nb, _p(_c(f, np.float64)), _p(_c(w, np.float64)),
                      _p(u), _p(ubar), _p(p), int(iters), lam, gamma, _p(state),
                      nthreads or nthreads_default())


def energy(nbr, f, w, u, p, lam, nthreads=None):
    """(E(u), D(p)) of Eq. (2) / Eq. (6)."""
    out = np.zeros(2)
    nb = len(nbr)
    lib().or_energy(_p(_c(nbr, np.int32)), nb, _p(_c(f, np.float64)), _p(_c(w, np.float64)),
                    _p(_c(u, np.float64)), _p(_c(p, np.float64)), lam, _p(out),
                    nthreads or nthreads_default())
    return float(out[0]), float(out[1])


def cp_l1(nbr, f, w, u, ubar, p, iters, lam, tau, sigma, theta=1.0, nthreads=None):
    """In-place iterations of the TV-L1 variant on (u, ubar, p)."""
    for a in (u, ubar, p):
        assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    nb = len(nbr)
    lib().or_cp_l1(_p(_c(nbr, np.int32)), nb, _p(_c(f, np.float64)), _p(_c(w, np.float64)),
                   _p(u), _p(ubar), _p(p), int(iters), lam, tau, sigma, theta,
                   nthreads or nthreads_default())


def energy_l1(nbr, f, w, u, p, lam, nthreads=None):
    """(E(u), D(p)) of the TV-L1 variant."""
    out = np.zeros(2)
    nb = len(nbr)
    lib().or_energy_l1(_p(_c(nbr, np.int32)), nb, _p(_c(f, np.float64)), _p(_c(w, np.float64)),
                       _p(_c(u, np.float64)), _p(_c(p, np.float64)), lam, _p(out),
                       nthreads or nthreads_default())
    return float(out[0]), float(out[1])


def mesh(coords, nbr, w, u, s):
    """Triangles [n][3][3] of the zero level set over fully observed cubes,
    and their total area."""
    coords = _c(coords, np.int32).reshape(-1, 3)
    nb = len(coords)
    area = np.zeros(1)
    cap = 1024
    while True:
        out = np.zeros((cap, 9))
        n = lib().or_mesh(_p(coords), _p(_c(nbr, np.int32)), nb, _p(_c(w, np.float64)), _p(_c(u, np.float64)),
                          float(s), _p(out), cap, _p(area))
        if n <= cap:
            return out[:n].reshape(n, 3, 3), float(area[0])
        cap = n


def extract(coords, nbr, w, u, s) -> np.ndarray:
    coords = _c(coords, np.int32).reshape(-1, 3)
    nb = len(coords)
    cap = 1024
    while True:
        pts = np.empty((cap, 3))
        n = lib().or_extract(_p(coords), _p(_c(nbr, np.int32)), nb, _p(_c(w, np.float64)),
                             _p(_c(u, np.float64)), s, _p(pts), cap)
        if n <= cap:
            return pts[:n]
        cap = int(n)


NET_PARAMS = 8241


def net_forward(tiles, params, gate=0):
    """gate 0: ReLUs open where the float64 pre-activation is > 0; gate 1:
    the open/closed decision is taken with bfloat16 operands (the network's
    own precision), the values stay float64; gate 2: the whole network with
    bfloat16 operands and float64 sums."""
    tiles = _c(tiles, np.float64)
    B = tiles.shape[0]
    out = np.empty((B, 10, 10, 10))
    lib().or_net_forward(_p(tiles), B, _p(_c(params, np.float64)), _p(out), None, None, int(gate))
    return out


def net_error_rms(tiles, params):
    """Element-wise standard deviation [B][10][10][10] of the difference
    between net_forward(tiles, params, gate=0) and an evaluation with
    bfloat16 operands, from propagating the variances of the roundings
    through the layers (the model is stated in the C source)."""
    tiles = _c(tiles, np.float64)
    B = tiles.shape[0]
    out = np.empty((B, 10, 10, 10))
    lib().or_net_error_rms(_p(tiles), B, _p(_c(params, np.float64)), _p(out))
    return out


def net_loss_grad(tiles, params, targets, mask, kind=0, gate=0):
    """kind 0: prediction f + r (primal residual); kind 1: prediction r.
    gate: as in net_forward."""
    tiles = _c(tiles, np.float64)
    B = tiles.shape[0]
    g = np.empty(NET_PARAMS)
    L = lib().or_net_loss_grad(_p(tiles), B, _p(_c(params, np.float64)),
                               _p(_c(targets, np.float64)), _p(_c(mask, np.float64)), _p(g), int(kind),
                               int(gate))
    return float(L), g


def net_gather(nbr, f, w, blocks, perm=0):
    blocks = _c(blocks, np.int32)
    tiles = np.empty((len(blocks), 2, 10, 10, 10))
    lib().or_net_gather(_p(_c(nbr, np.int32)), _p(_c(f, np.float64)), _p(_c(w, np.float64)),
                        _p(blocks), len(blocks), _p(tiles), int(perm))
    return tiles


# ------------------------------------------------------------ the volume
def _pack(c: np.ndarray) -> np.ndarray:
    c = c.astype(np.int64) + (1 << 20)
    return (c[:, 0] << 42) | (c[:, 1] << 21) | c[:, 2]


def _unique_rows(c) -> np.ndarray:
    """Distinct (x, y, z) rows in ascending lexicographic order."""
    c = np.asarray(c, np.int32).reshape(-1, 3)
    if len(c) == 0:
        return c
    k = np.unique(_pack(c))
    m = (1 << 21) - 1
    return np.stack([(k >> 42) & m, (k >> 21) & m, k & m], 1).astype(np.int64).__sub__(1 << 20).astype(np.int32)


@dataclass
class OracleVolume:
    """Block pool + hash + fused fields, bookkept exactly as the boundary
    specifies: new blocks of a frame are appended in ascending (x, y, z)
    order, pool ids are never renumbered, the hash is rebuilt after every
    allocation, and a frame that does not fit leaves the volume unchanged."""
    voxel_size: float
    mu: float
    max_depth: float
    max_blocks: int
    hash_cap_log2: int
    hash_tail: int

    def __post_init__(self):
        self.cap = 1 << self.hash_cap_log2
        self.coords = np.zeros((0, 3), np.int32)
        self.f = np.zeros((0, 512))
        self.w = np.zeros((0, 512))
        rc, self.slots = hash_build(self.coords, self.cap, self.hash_tail)
        self.nbr = np.zeros((0, 27), np.int32)
        self.last_candidates = np.zeros((0, 3), np.int32)

    @property
    def nb(self):
        return len(self.coords)

    def insert(self, keys: np.ndarray) -> int:
        """Append the keys not yet present, in ascending order."""
        keys = _unique_rows(keys)
        if len(self.coords):
            new = keys[~np.isin(_pack(keys), _pack(self.coords))]
        else:
            new = keys
        if self.nb + len(new) > self.max_blocks:
            return E_CAPACITY
        coords = np.concatenate([self.coords, new]).astype(np.int32)
        rc, slots = hash_build(coords, self.cap, self.hash_tail)
        if rc != OK:
            return E_CAPACITY
        self.coords, self.slots = coords, slots
        self.f = np.concatenate([self.f, np.zeros((len(new), 512))])
        self.w = np.concatenate([self.w, np.zeros((len(new), 512))])
        self.nbr = nbr_table(self.coords, self.slots, self.cap, self.hash_tail)
        return len(new)

    def alloc(self, depth, K4, T) -> int:
        c = candidates(depth, K4, T, self.voxel_size, self.mu, self.max_depth)
        self.last_candidates = _unique_rows(c)
        return self.insert(self.last_candidates)

    def fuse(self, depth, K4, T, nthreads=None):
        fuse(self.coords, self.f, self.w, depth, K4, T, self.voxel_size, self.mu,
             self.max_depth, nthreads)

    def alloc_laser(self, pts, T) -> int:
        c = candidates_laser(pts, T, self.voxel_size, self.mu, self.max_depth)
        self.last_candidates = _unique_rows(c)
        return self.insert(self.last_candidates)

    def fuse_laser(self, pts, T):
        assert self.f.flags["C_CONTIGUOUS"] and self.w.flags["C_CONTIGUOUS"]
        pts = _c(pts, np.float32).reshape(-1, 3)
        lib().or_fuse_laser(_p(_c(self.slots, np.int32)), self.cap, self.hash_tail, self.nb, _p(self.f),
                            _p(self.w), _p(pts), len(pts), _p(_c(T, np.float64)), self.voxel_size, self.mu,
                            self.max_depth)

    def integrate(self, depth, K4, T):
        n = self.alloc(depth, K4, T)
        if n < 0:
            return n
        self.fuse(depth, K4, T)
        return n
