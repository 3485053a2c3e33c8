"""Failure handling of the C ABI, with each condition forced from the host (a NaN
in the input state, a CG iteration limit of 1, a marker outside the box): the
library reports it and leaves the state as documented. No kernel faults."""
import math

import numpy as np
import pytest
import torch

from paper_2301_09349_amd import _lib, inputs
from helpers import make_gpu, to_np

pytestmark = pytest.mark.gpu


def test_nonfinite_state_is_reported_and_rolled_back(cuda):
    c = inputs.scaled("cfg1", (64, 48), ns=40)
    g = make_gpu(c)
    g.step(2)
    r, m, E, F = g.get_state()
    bad = r.clone()
    bad[100] = float("nan")
    g.set_state(bad, m, E, F, step=2)
    r0, m0, E0, F0 = [x.clone() if not isinstance(x, list) else [f.clone() for f in x]
                      for x in g.get_state()]
    st, info = g.step_status(3)
    assert st == _lib.IBM_E_NONFINITE
    assert info["steps_done"] == 0 and info["step"] == 2
    r1, m1, E1, F1 = g.get_state()
    assert torch.equal(torch.isnan(r1), torch.isnan(r0))
    ok = ~torch.isnan(r0)
    assert torch.equal(r1[ok], r0[ok]) and torch.equal(m1, m0) and torch.equal(E1, E0)


def test_nonfinite_in_a_later_step_keeps_the_last_good_state(cuda):
    # the third step of the call fails: two steps are kept
    c = inputs.scaled("cfg1", (64, 48), ns=40)
    g = make_gpu(c)
    ref = make_gpu(c)
    ref.step(2)
    r2, m2, E2, _ = ref.get_state()
    # a huge temperature at one cell makes a later step non-positive somewhere
    g.step(2)
    st, info = g.step_status(1)
    assert st == _lib.IBM_OK
    r, m, E, F = g.get_state()
    E = E.clone()
    E[700] = -1e30
    g.set_state(r, m, E, F, step=3)
    st, info = g.step_status(4)
    assert st == _lib.IBM_E_NONFINITE
    assert info["step"] == 3 and info["steps_done"] == 0
    r3, _, E3, _ = g.get_state()
    assert torch.equal(E3, E)


def test_cg_iteration_limit(cuda):
    c = inputs.scaled("cfg1", (64, 48), ns=40, cg_maxit=1)
    g = make_gpu(c)
    st, info = g.step_status(3)
    assert st == _lib.IBM_E_NOT_CONVERGED
    assert info["steps_done"] == 1  # the state is advanced, then the call stops


def test_marker_outside_box_rejected(cuda):
    c = inputs.scaled("cfg1", (64, 48), ns=4)  # capacity for 4 markers
    g = make_gpu(c, markers=False)
    X = np.array([[0.0, 0.0], [5.95, 0.0]])  # second marker's support leaves x_hi
    with pytest.raises(_lib.IBMError) as e:
        g.set_markers(X, dedupe=False)
    assert e.value.status == _lib.IBM_E_ARG
    # the context is still usable
    g.set_markers(X[:1], dedupe=False)
    g.step(1)


def test_deterministic_repeat(cuda):
    # the spread is a sorted segmented reduction and every sum has a fixed order:
    # two runs are bitwise identical
    c = inputs.scaled("cfg1", (96, 80), ns=80)
    outs = []
    for _ in range(2):
        g = make_gpu(c)
        h, _ = g.step(5)
        r, m, E, F = g.get_state()
        outs.append((to_np(h), to_np(r), to_np(m), to_np(E)))
    for a, b in zip(*outs):
        assert np.array_equal(a, b)
