"""The C-ABI library loads without a GPU and exports every function that
include/denser.h declares; the binding marshals no computation of its own."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "denser.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dn_[a-z0-9_]+)\s*\(", text)))


def _lib():
    from paper_1604_03734_amd import build, denser
    if not os.path.exists(denser.LIB_PATH):
        build.build()
    return ctypes.CDLL(denser.LIB_PATH)


def test_header_declares_the_boundary():
    names = _declared()
    for core in ("dn_alloc_blocks", "dn_fuse_depth", "dn_regularize", "dn_extract",
                 "dn_regularize_batch", "dn_net_forward", "dn_net_loss_grad", "dn_net_warm_start"):
        assert core in names
    assert len(names) >= 20


def test_library_exports_every_declared_symbol():
    L = _lib()
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing


def test_binding_declares_only_exported_symbols():
    from paper_1604_03734_amd import denser
    L = denser.lib()
    names = set(_declared())
    for n in ("dn_volume_create", "dn_regularize", "dn_extract", "dn_net_adam"):
        assert n in names and getattr(L, n).restype is not None


def test_error_text_without_a_device():
    L = _lib()
    L.dn_last_error.restype = ctypes.c_char_p
    L.dn_volume_create.restype = ctypes.c_int
    rc = L.dn_volume_create(None, None, ctypes.c_size_t(0), None, None)
    assert rc == -1  # DN_E_INVALID: checked before any device call
    assert b"null" in L.dn_last_error()


def _params(D, **kw):
    base = dict(voxel_size=0.2, mu=0.6, max_depth=50.0, max_blocks=4096, hash_cap_log2=14, hash_tail=256,
                state16=1, max_points=1242 * 375, max_candidates=2_000_000, max_observations=0)
    base.update(kw)
    return D.VolumeParams(*[base[k] for k, _ in D.VolumeParams._fields_])


def test_arena_size_is_pure_arithmetic_and_covers_every_part():
    """dn_volume_bytes needs no device; it grows with every limit, and the
    per-voxel part is at least the fields (f, w, u, two ubar, two p of three
    components: 44 B, edge mask 1 B) plus 18 B of 16-bit state."""
    from paper_1604_03734_amd import denser as D
    L = D.lib()
    size = lambda **kw: L.dn_volume_bytes(ctypes.byref(_params(D, **kw)))  # noqa: E731
    b0 = size()
    assert b0 > 0
    assert size(max_blocks=8192) - b0 >= 4096 * 512 * (45 + 18)
    assert size(state16=0) <= b0 - 4096 * 512 * 18
    assert size(max_candidates=4_000_000) - b0 >= 2_000_000 * 8 * 5
    # scratch is shared by the calls (the largest need counts): observation
    # lists larger than every other need add their 36 B per observation
    assert size(max_observations=20_000_000) >= 20_000_000 * 36 + size(max_points=0, max_candidates=0)
    assert size(max_points=0, max_candidates=0) < b0
    for bad in (dict(max_blocks=0), dict(hash_cap_log2=3), dict(mu=0.0), dict(max_points=-1),
                dict(state16=2), dict(hash_tail=-1)):
        assert size(**bad) == 0, bad


def test_short_or_misaligned_arena_is_refused_before_any_device_call():
    from paper_1604_03734_amd import denser as D
    L = D.lib()
    prm = _params(D)
    need = L.dn_volume_bytes(ctypes.byref(prm))
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(1 << 40)            # never dereferenced: the checks come first
    assert L.dn_volume_create(ctypes.byref(prm), fake, need - 1, None, ctypes.byref(h)) == D.DN_E_CAPACITY
    assert b"short" in L.dn_last_error()
    assert L.dn_volume_create(ctypes.byref(prm), ctypes.c_void_p((1 << 40) + 64), need, None,
                              ctypes.byref(h)) == D.DN_E_INVALID
    assert L.dn_volume_create(ctypes.byref(prm), None, need, None, ctypes.byref(h)) == D.DN_E_INVALID
    assert h.value is None


def test_workspace_sizes_without_a_device():
    from paper_1604_03734_amd import denser as D
    L = D.lib()
    assert L.dn_regularize_batch_bytes(64, 1_000_000) >= 1_000_000 * 8
    assert L.dn_regularize_batch_bytes(0, 10) == 0
    assert L.dn_net_bytes(256, 1) > L.dn_net_bytes(256, 0) >= 256 * 1000 * 16 * 2 * 3
    assert L.dn_net_bytes(-1, 0) == 0
    assert L.dn_warm_start_bytes(1000) >= 1000 * 512 * 4
    assert L.dn_warm_start_bytes(-5) == 0


def test_library_source_never_allocates_device_memory():
    csrc = os.path.join(ROOT, "paper_1604_03734_amd", "csrc")
    for fn in os.listdir(csrc):
        src = open(os.path.join(csrc, fn)).read()
        for call in ("hipMalloc", "hipFree", "hipHostMalloc", "hipMallocAsync", "hipExtMalloc"):
            assert call + "(" not in src, (fn, call)


def test_product_path_never_imports_the_oracle():
    pkg = os.path.join(ROOT, "paper_1604_03734_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, fn)).read()
                assert "import oracle" not in src and "from oracle" not in src, fn
                assert "liboracle" not in src, fn
