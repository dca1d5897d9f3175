"""dn_net_forward_static (the entry point that allocates nothing: its
scratch is a static device array) against dn_net_forward (caller
workspace): identical outputs on two calls in a row, the second smaller,
and a capacity error beyond its maximum."""
import numpy as np
import pytest

from gpu_common import dn, to_dev

pytestmark = pytest.mark.gpu


def test_static_forward_matches_workspace_forward():
    D = dn()
    import torch
    rng = np.random.default_rng(3)
    prm = to_dev(rng.normal(0, 0.15, D.NET_PARAMS), torch.float32)
    for n in (D.NET_STATIC_TILES, 7):
        print(f"static forward: {n} tiles", flush=True)
        tiles = to_dev(rng.normal(0, 0.6, (n, 2, 10, 10, 10)), torch.float32)
        a = torch.empty((n, 10, 10, 10), device="cuda")
        b = torch.full_like(a, float("nan"))
        D.net_forward(tiles, prm, a)
        D.net_forward_static(tiles, prm, b)
        torch.cuda.synchronize()
        assert torch.equal(a, b)
    n = D.NET_STATIC_TILES + 1
    with pytest.raises(D.DenserError) as e:
        D.net_forward_static(torch.zeros((n, 2, 10, 10, 10), device="cuda"), prm,
                             torch.empty((n, 10, 10, 10), device="cuda"))
    assert e.value.code == D.DN_E_CAPACITY
