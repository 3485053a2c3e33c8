"""Pins of the oracle's outer passes (App. A step 3 repeated "until convergence":
each pass after the first re-evaluates the predictor's fluxes and cell terms at
the latest iterate, keeps the step's start for the time derivative and the
marker sources of the first pass, and solves the pressure equation again).

- One pass is the default step, bit for bit.
- The passes are a fixed-point iteration that contracts at these step sizes.
- The converged step is a consistent time integrator: its difference to the
  one-pass step, relative to the change the step makes, shrinks in proportion
  to dt. The start state must not carry anything made with a longer step: its
  face flux is the interpolated momentum, and its forcing history was built
  with steps of 1e-6 (after a step of length dt0 the face flux and the
  near-wall field differ from their forced values by O(dt0), which a shorter
  step then removes at once, and the ratio would stall).
- The marker sources are formed once: the first step's force and heat are the
  same with any number of passes.
- Mass conservation and free-stream preservation hold with several passes."""
import numpy as np
import pytest

from paper_2301_09349_amd import inputs
from helpers import make_oracle


def _state(o):
    r, m, e, F = o.get_state()
    return np.concatenate([r, m.ravel(), e] + list(F))


def test_one_pass_is_the_default_step():
    c = inputs.scaled("cfg1", (40, 32), ns=40, Re=20.0)
    outs = []
    for over in ({}, {"n_outer": 0}, {"n_outer": 1}):
        o = make_oracle(dict(c, **over), amplitude=5e-2)
        h = o.step(3)
        outs.append((_state(o), h))
    for x, h in outs[1:]:
        assert np.array_equal(x, outs[0][0]) and np.array_equal(h, outs[0][1])


@pytest.mark.parametrize("name,shape", [("cfg1", (40, 32)), ("cfg3", (14, 12, 12))])
def test_outer_passes_contract(name, shape):
    xs = []
    for K in range(1, 8):
        c = inputs.scaled(name, shape, ns=40, Re=20.0, dt=2e-3, n_outer=K)
        o = make_oracle(c, amplitude=5e-2)
        o.step(1)
        xs.append(_state(o))
    d = [np.linalg.norm(xs[k + 1] - xs[k]) / np.linalg.norm(xs[k]) for k in range(len(xs) - 1)]
    assert d[0] > 1e-6, d  # the second pass does change the step
    for a, b in zip(d[:4], d[1:5]):
        assert b < 0.2 * a, d
    assert d[-1] < 1e-9, d


@pytest.mark.parametrize("name,shape", [("cfg1", (40, 32)), ("cfg3", (14, 12, 12))])
def test_converged_passes_are_consistent(name, shape):
    c0 = inputs.scaled(name, shape, ns=40, Re=20.0, dt=1e-6)
    o0 = make_oracle(c0, amplitude=5e-2)
    o0.step(30)
    S = o0.get_state()
    ratios = []
    for dt in (2.5e-4, 1.25e-4):
        out = []
        for K in (1, 6):
            c = inputs.scaled(name, shape, ns=40, Re=20.0, dt=dt, n_outer=K)
            o = make_oracle(c, amplitude=5e-2)
            o.set_state(S[0], S[1], S[2], None, step=30)  # face flux from the momentum
            o.step(1)
            out.append(o.get_state())
        r = []
        for i in (1, 2):  # momentum, energy
            step = np.linalg.norm(out[0][i] - S[i])
            r.append(np.linalg.norm(out[1][i] - out[0][i]) / step)
        ratios.append(r)
    for a, b in zip(ratios[0], ratios[1]):
        assert 1.7 < a / b < 2.3, ratios


def test_marker_sources_are_formed_once():
    hs = []
    for K in (1, 3):
        c = inputs.scaled("cfg1", (40, 32), ns=40, Re=20.0, dt=2e-3, n_outer=K)
        o = make_oracle(c, amplitude=5e-2)
        hs.append(o.step(2))
    # the first step's force and heat come from its first pass alone; the second
    # step starts from a different state
    assert np.array_equal(hs[0][0, :4], hs[1][0, :4])
    assert not np.array_equal(hs[0][1, :4], hs[1][1, :4])


def test_outer_passes_conserve_mass_and_keep_the_free_stream():
    per = [[inputs.PERIODIC] * 2, [inputs.PERIODIC] * 2]
    c = inputs.scaled("cfg1", (36, 28), ns=0, Re=10.0, bc=per, n_outer=4)
    o = make_oracle(c, amplitude=5e-2)
    m0 = float(np.sum(o.get_state()[0]))
    o.step(5)
    m1 = float(np.sum(o.get_state()[0]))
    assert abs(m1 - m0) <= 1e-13 * abs(m0)
    # uniform stream through inflow/outflow/slip boundaries stays uniform
    c = inputs.scaled("cfg1", (36, 28), ns=0, n_outer=3)
    o = make_oracle(c, amplitude=0.0)
    x0 = _state(o)
    o.step(4)
    assert np.max(np.abs(_state(o) - x0)) <= 1e-12 * np.max(np.abs(x0))
