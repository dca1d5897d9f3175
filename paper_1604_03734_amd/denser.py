"""Thin ctypes binding of libdenser.so (include/denser.h).

Argument marshalling only: every computation runs in the library's HIP
kernels.  Device buffers are torch tensors on the HIP device; the library
orders its work on the stream the volume was created with (by default
torch's current stream).  If the shared library is missing this module
raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdenser.so")

DN_OK, DN_E_INVALID, DN_E_CAPACITY, DN_E_NUMERIC, DN_E_DEVICE = 0, -1, -2, -3, -4
DN_F32, DN_F16, DN_BF16 = 0, 1, 2
DN_INIT_ZERO, DN_INIT_KEEP, DN_INIT_GIVEN, DN_INIT_CONTINUE = 0, 1, 2, 3
DN_K_AUTO, DN_K_TWOPASS, DN_K_FUSED, DN_K_FUSED256 = 0, 1, 2, 3
(DN_X_COORDS, DN_X_HASH, DN_X_NBR, DN_X_F, DN_X_W, DN_X_U, DN_X_UBAR, DN_X_P, DN_X_SURFACE,
 DN_X_CANDIDATES, DN_X_EMASK, DN_X_MESH) = range(1, 13)
NET_PARAMS = 8241
DN_WARM_PRIMAL, DN_WARM_DUAL = 0, 1
DN_DATA_L2, DN_DATA_L1 = 0, 1


class DenserError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"denser error {code}: {msg}")
        self.code = code


class Intrinsics(ctypes.Structure):
    _fields_ = [("fx", ctypes.c_double), ("fy", ctypes.c_double), ("cx", ctypes.c_double),
                ("cy", ctypes.c_double), ("width", ctypes.c_int32), ("height", ctypes.c_int32)]


class VolumeParams(ctypes.Structure):
    _fields_ = [("voxel_size", ctypes.c_double), ("mu", ctypes.c_double), ("max_depth", ctypes.c_double),
                ("max_blocks", ctypes.c_int32), ("hash_cap_log2", ctypes.c_int32),
                ("hash_tail", ctypes.c_int32), ("state16", ctypes.c_int32),
                ("max_points", ctypes.c_int64), ("max_candidates", ctypes.c_int64),
                ("max_observations", ctypes.c_int64)]


class RegParams(ctypes.Structure):
    _fields_ = [("lam", ctypes.c_double), ("tau", ctypes.c_double), ("sigma", ctypes.c_double),
                ("theta", ctypes.c_double), ("iters", ctypes.c_int32), ("gap_every", ctypes.c_int32),
                ("gap_tol", ctypes.c_double), ("storage", ctypes.c_int32),
                ("refine_every", ctypes.c_int32), ("init", ctypes.c_int32), ("kernel", ctypes.c_int32),
                ("gamma", ctypes.c_double), ("data_term", ctypes.c_int32)]


class RegStats(ctypes.Structure):
    _fields_ = [("energy", ctypes.c_double), ("dual", ctypes.c_double), ("gap", ctypes.c_double),
                ("rel_gap", ctypes.c_double), ("iters_run", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("ms_loop", ctypes.c_double), ("kernel_used", ctypes.c_int32), ("layout_used", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def reg_params(lam=0.5, tau=None, sigma=None, theta=1.0, iters=200, gap_every=0, gap_tol=0.0,
               storage=DN_F32, refine_every=50, init=DN_INIT_ZERO, kernel=DN_K_AUTO, gamma=0.0,
               data_term=0) -> RegParams:
    tau = 1.0 / np.sqrt(12.0) if tau is None else tau
    sigma = 1.0 / np.sqrt(12.0) if sigma is None else sigma
    return RegParams(lam, tau, sigma, theta, iters, gap_every, gap_tol, storage, refine_every, init, kernel,
                     gamma, data_term)


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1604_03734_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    P, i32, i64, f64, f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_float
    sz = ctypes.c_size_t
    sig = {
        "dn_volume_bytes": (sz, [P]),
        "dn_volume_create": (i32, [P, P, sz, P, P]),
        "dn_regularize_batch_bytes": (sz, [i32, i64]),
        "dn_net_bytes": (sz, [i64, i32]),
        "dn_warm_start_bytes": (sz, [i64]),
        "dn_volume_destroy": (None, [P]),
        "dn_set_stream": (i32, [P, P]),
        "dn_volume_clear": (i32, [P]),
        "dn_num_blocks": (i64, [P]),
        "dn_sync": (i32, [P]),
        "dn_last_error": (ctypes.c_char_p, []),
        "dn_alloc_blocks": (i32, [P, P, P, P, P]),
        "dn_insert_blocks": (i32, [P, P, i64, P]),
        "dn_insert_blocks_ordered": (i32, [P, P, i64, P]),
        "dn_fuse_depth": (i32, [P, P, P, P]),
        "dn_alloc_laser": (i32, [P, P, i64, P, P]),
        "dn_fuse_laser": (i32, [P, P, i64, P]),
        "dn_load_fused": (i32, [P, P, P]),
        "dn_regularize": (i32, [P, P, P, P, P]),
        "dn_regularize_batch": (i32, [P, i32, P, P, sz, P]),
        "dn_energy": (i32, [P, f64, i32, P]),
        "dn_mesh_area": (i32, [P, P, P]),
        "dn_extract": (i32, [P, i32, P, ctypes.c_size_t, P]),
        "dn_net_gather": (i32, [P, P, i64, i32, P]),
        "dn_net_forward": (i32, [P, i64, P, P, P, sz, P]),
        "dn_net_forward_static": (i32, [P, i64, P, P, P]),
        "dn_net_loss_grad": (i32, [P, i64, P, P, P, i32, P, P, sz, P, P]),
        "dn_net_adam": (i32, [P, P, P, P, i64, f32, f32, f32, f32, i32, P]),
        "dn_net_warm_start": (i32, [P, P, i32, f64, P, P, P, sz]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name, None)
        if fn is None:
            continue
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def check(rc):
    if rc != DN_OK:
        msg = lib().dn_last_error().decode(errors="replace")
        raise DenserError(rc, msg)
    return rc


def _ptr(t):
    if t is None:
        return None
    import torch
    assert isinstance(t, torch.Tensor) and t.is_cuda and t.is_contiguous(), "need a contiguous device tensor"
    return ctypes.c_void_p(t.data_ptr())


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def device_bytes(nbytes, device=None):
    """A device buffer of at least nbytes whose address is 256-byte
    aligned: (owning tensor, aligned address)."""
    import torch
    if device is None:
        device = torch.device("cuda", torch.cuda.current_device())
    t = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=device)
    addr = t.data_ptr()
    return t, addr + (-addr) % 256


_workspaces = {}


def workspace(purpose, nbytes):
    """A cached workspace (grown on demand) per (device, purpose): the
    library never allocates device memory; the binding keeps one buffer per
    use so that repeated calls (and the batched solver's captured graph)
    see the same address."""
    import torch
    key = (torch.cuda.current_device(), purpose)
    cur = _workspaces.get(key)
    if cur is None or cur[2] < nbytes:
        t, addr = device_bytes(max(int(nbytes), 256))
        cur = (t, addr, int(nbytes))
        _workspaces[key] = cur
    return ctypes.c_void_p(cur[1]), ctypes.c_size_t(cur[2])


def band_cells_per_point(voxel_size, mu, ray_norm=2.0):
    """Most blocks one pixel's band [d - mu, d + mu] can cross: 4 plus the
    band's L1 length in block units, for rays r = ((x - cx)/fx, (y - cy)/fy,
    1) with |r| <= ray_norm."""
    return 4 + int(np.floor(np.sqrt(3.0) * 2.0 * mu * ray_norm / (8.0 * voxel_size)))


def laser_observations_bound(n_returns, voxel_size, mu, max_depth):
    """Most voxel observations n_returns laser returns can make: each ray is
    walked from the sensor to range + mu <= max_depth + mu, at most 4 plus
    its L1 length in voxels."""
    return int(n_returns) * (4 + int(np.floor(np.sqrt(3.0) * (max_depth + mu) / voxel_size)))


def intrinsics(fx, fy, cx, cy, width, height) -> Intrinsics:
    return Intrinsics(fx, fy, cx, cy, width, height)


def _pose(T):
    T = np.ascontiguousarray(T, dtype=np.float64).reshape(16)
    return T, T.ctypes.data_as(ctypes.c_void_p)


class Volume:
    """A hashed-block TSDF volume living on the GPU, in one arena that this
    object allocates with torch and hands to the library.

    max_points: most pixels of a depth map (or returns of a laser scan) one
    call takes; max_candidates: most band cells one allocation call lists
    (default: max_points times the band bound of band_cells_per_point, at
    least max_blocks); max_observations: most voxel observations of one
    laser fusion call (0: no laser fusion); state16: room for FP16/BF16
    solver state."""

    def __init__(self, voxel_size, mu, max_depth, max_blocks, hash_cap_log2=20, hash_tail=1024,
                 stream=None, *, max_points=1 << 19, max_candidates=None, max_observations=0, state16=True):
        import torch
        if max_candidates is None:
            max_candidates = max(int(max_blocks), int(max_points) * band_cells_per_point(voxel_size, mu))
        self.params = VolumeParams(voxel_size, mu, max_depth, max_blocks, hash_cap_log2, hash_tail,
                                   1 if state16 else 0, int(max_points), int(max_candidates),
                                   int(max_observations))
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.arena_bytes = int(lib().dn_volume_bytes(ctypes.byref(self.params)))
        if self.arena_bytes == 0:
            raise DenserError(DN_E_INVALID, "invalid volume parameters")
        self._arena, addr = device_bytes(self.arena_bytes)
        h = ctypes.c_void_p()
        check(lib().dn_volume_create(ctypes.byref(self.params), ctypes.c_void_p(addr), self.arena_bytes,
                                     _stream_handle(self.stream), ctypes.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            lib().dn_volume_destroy(self.handle)
            self.handle = None
        self._arena = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def clear(self):
        check(lib().dn_volume_clear(self.handle))

    @property
    def num_blocks(self) -> int:
        return int(lib().dn_num_blocks(self.handle))

    def sync(self):
        check(lib().dn_sync(self.handle))

    def alloc_blocks(self, depth, K: Intrinsics, T) -> int:
        n = ctypes.c_int32(0)
        _, tp = _pose(T)
        check(lib().dn_alloc_blocks(self.handle, _ptr(depth), ctypes.byref(K), tp, ctypes.byref(n)))
        return n.value

    def insert_blocks(self, coords, keep_order=False) -> int:
        """Append the new keys of coords (int32 [n][3], device): in ascending
        order, or with keep_order in the order of their first occurrence."""
        n = ctypes.c_int32(0)
        fn = lib().dn_insert_blocks_ordered if keep_order else lib().dn_insert_blocks
        check(fn(self.handle, _ptr(coords), coords.shape[0], ctypes.byref(n)))
        return n.value

    def fuse_depth(self, depth, K: Intrinsics, T):
        _, tp = _pose(T)
        check(lib().dn_fuse_depth(self.handle, _ptr(depth), ctypes.byref(K), tp))

    def integrate(self, depth, K: Intrinsics, T) -> int:
        n = self.alloc_blocks(depth, K, T)
        self.fuse_depth(depth, K, T)
        return n

    def alloc_laser(self, pts, T) -> int:
        """pts: device float [n][3] returns in the sensor frame; T: sensor -> world."""
        n = ctypes.c_int32(0)
        _, tp = _pose(T)
        check(lib().dn_alloc_laser(self.handle, _ptr(pts), pts.shape[0], tp, ctypes.byref(n)))
        return n.value

    def fuse_laser(self, pts, T):
        _, tp = _pose(T)
        check(lib().dn_fuse_laser(self.handle, _ptr(pts), pts.shape[0], tp))

    def integrate_laser(self, pts, T) -> int:
        n = self.alloc_laser(pts, T)
        self.fuse_laser(pts, T)
        return n

    def load_fused(self, f, w):
        check(lib().dn_load_fused(self.handle, _ptr(f), _ptr(w)))

    def regularize(self, params: RegParams, u0=None, p0=None) -> RegStats:
        st = RegStats()
        check(lib().dn_regularize(self.handle, ctypes.byref(params), _ptr(u0), _ptr(p0), ctypes.byref(st)))
        return st

    def energy(self, lam, data_term=DN_DATA_L2):
        out = (ctypes.c_double * 2)()
        check(lib().dn_energy(self.handle, lam, int(data_term), out))
        return out[0], out[1]

    _SHAPES = {DN_X_COORDS: ("int32", (3,)), DN_X_HASH: ("int32", (4,)), DN_X_NBR: ("int32", (27,)),
               DN_X_F: ("float32", (512,)), DN_X_W: ("float32", (512,)), DN_X_U: ("float32", (512,)),
               DN_X_UBAR: ("float32", (512,)), DN_X_SURFACE: ("float32", (3,)),
               DN_X_CANDIDATES: ("int32", (3,)), DN_X_EMASK: ("uint8", (512,)),
               DN_X_MESH: ("float32", (3, 3))}

    def extract(self, what):
        """Return the requested part as a device tensor."""
        import torch
        n = ctypes.c_int64(0)
        rc = lib().dn_extract(self.handle, what, None, 0, ctypes.byref(n))
        if rc not in (DN_OK, DN_E_CAPACITY):
            check(rc)
        dev = torch.device("cuda", torch.cuda.current_device())
        if what == DN_X_P:
            out = torch.empty((3, n.value, 512), dtype=torch.float32, device=dev)
        else:
            dt, tail = self._SHAPES[what]
            out = torch.empty((n.value,) + tail, dtype=getattr(torch, dt), device=dev)
        if out.numel() == 0:
            return out
        check(lib().dn_extract(self.handle, what, _ptr(out), out.numel() * out.element_size(), ctypes.byref(n)))
        return out

    def mesh_area(self):
        """(area in square metres, number of triangles) of the DN_X_MESH surface."""
        a = ctypes.c_double(0)
        n = ctypes.c_int64(0)
        check(lib().dn_mesh_area(self.handle, ctypes.byref(a), ctypes.byref(n)))
        return a.value, n.value

    # ------------------------------------------------------- warm start
    def net_gather(self, blocks, tiles, perm=0):
        check(lib().dn_net_gather(self.handle, _ptr(blocks), blocks.shape[0], int(perm), _ptr(tiles)))

    def net_warm_start(self, params, u0, p0=None, mode=DN_WARM_DUAL, delta=0.1):
        ws, nbytes = workspace("warm_start", lib().dn_warm_start_bytes(self.num_blocks))
        check(lib().dn_net_warm_start(self.handle, _ptr(params), int(mode), float(delta), _ptr(u0), _ptr(p0),
                                      ws, nbytes))


def regularize_batch(volumes, params: RegParams):
    arr = (ctypes.c_void_p * len(volumes))(*[v.handle.value for v in volumes])
    stats = (RegStats * len(volumes))()
    total = sum(v.num_blocks for v in volumes)
    ws, nbytes = workspace("batch", lib().dn_regularize_batch_bytes(len(volumes), total))
    check(lib().dn_regularize_batch(arr, len(volumes), ctypes.byref(params), ws, nbytes, stats))
    return list(stats)


def net_forward(tiles, params, out, stream=None):
    ws, nbytes = workspace("net", lib().dn_net_bytes(tiles.shape[0], 0))
    check(lib().dn_net_forward(_ptr(tiles), tiles.shape[0], _ptr(params), _ptr(out), ws, nbytes,
                               _stream_handle(stream)))


NET_STATIC_TILES = 32


def net_forward_static(tiles, params, out, stream=None):
    """dn_net_forward_static: the forward pass with the library's static
    scratch (no workspace; at most NET_STATIC_TILES tiles per call)."""
    check(lib().dn_net_forward_static(_ptr(tiles), tiles.shape[0], _ptr(params), _ptr(out),
                                      _stream_handle(stream)))


def net_loss_grad(tiles, params, targets, mask, grad, kind=0, stream=None, sync=True):
    """Loss (returned when sync, which waits for it) and gradient into grad."""
    loss = ctypes.c_double(0)
    ws, nbytes = workspace("net_train", lib().dn_net_bytes(tiles.shape[0], 1))
    check(lib().dn_net_loss_grad(_ptr(tiles), tiles.shape[0], _ptr(params), _ptr(targets), _ptr(mask),
                                 int(kind), _ptr(grad), ws, nbytes, ctypes.byref(loss) if sync else None,
                                 _stream_handle(stream)))
    return loss.value if sync else None


def net_adam(params, grad, m, v, lr, step, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    check(lib().dn_net_adam(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), params.numel(), lr, beta1, beta2,
                            eps, int(step), _stream_handle(stream)))
