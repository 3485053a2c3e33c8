"""The entry point that allocates nothing (ibm_create_grid_noalloc: the workspace is
the library's fixed device array) against ibm_create_grid on a caller's workspace,
through the C ABI: two contexts in a row, the second on a smaller grid, each stepped
and compared bitwise with a workspace context stepped alike."""
import numpy as np
import pytest
import torch

from paper_2301_09349_amd import _lib, inputs
from helpers import make_gpu, to_np

pytestmark = pytest.mark.gpu


def _same(a, b):
    ra, ma, Ea, Fa = a.get_state()
    rb, mb, Eb, Fb = b.get_state()
    assert torch.equal(ra, rb) and torch.equal(ma, mb) and torch.equal(Ea, Eb)
    for x, y in zip(Fa, Fb):
        assert torch.equal(x, y)


def test_noalloc_context_matches_workspace_context(cuda):
    for shape, ns, precision in (((128, 128), 100, "fp64"), ((96, 80), 60, "fp32")):
        c = inputs.scaled("cfg1", shape, ns=ns)
        ref = make_gpu(c, precision)
        g = make_gpu(c, precision, noalloc=True)
        assert g.ws is None
        ids_a, eps_a = ref.markers_in_use()
        ids_b, eps_b = g.markers_in_use()
        assert torch.equal(ids_a, ids_b) and torch.equal(eps_a, eps_b)
        ha, ia = ref.step(6)
        hb, ib = g.step(6)
        assert torch.equal(ha, hb)
        assert ia["cg_iters_total"] == ib["cg_iters_total"] and ia["mass"] == ib["mass"]
        _same(ref, g)
        f_a, h_a, t_a = ref.wall_fluxes()
        f_b, h_b, t_b = g.wall_fluxes()
        assert torch.equal(f_a, f_b) and torch.equal(h_a, h_b) and np.array_equal(t_a, t_b)
        g.close()
        ref.close()


def test_noalloc_one_live_context_per_device_and_size_limit(cuda):
    c = inputs.scaled("cfg1", (64, 48), ns=40)
    a = make_gpu(c, noalloc=True)
    with pytest.raises(_lib.IBMError) as e:
        make_gpu(c, noalloc=True)
    assert e.value.status == _lib.IBM_E_STATE
    a.step(2)
    a.close()
    # released: a new one may be created, and it starts from its own state
    b = make_gpu(c, noalloc=True)
    ref = make_gpu(c)
    b.step(2)
    ref.step(2)
    _same(ref, b)
    b.close()
    # a workspace above the fixed array's 64 MiB is refused
    big = inputs.case("cfg2a")
    with pytest.raises(_lib.IBMError) as e:
        make_gpu(big, noalloc=True)
    assert e.value.status == _lib.IBM_E_SIZE
