"""Pins of the oracle's tangent-linear runs (dual numbers through the whole step):
the directional derivatives along the wall temperatures and along the state agree
with central differences of the oracle's own FP64 step.

Linear convection is smooth, so there the agreement is limited only by the
difference quotient. With van Leer convection the dual numbers follow the branch
the step takes (upwind side, limiter on or off); central differences agree with
that derivative where no branch changes within the step, which noisy states, a
step small enough (here 1e-6) and no flux perturbation on faces with zero flux
(slip walls) give."""
import numpy as np
import pytest

from paper_2301_09349_amd import inputs
from helpers import make_oracle

LIN = inputs.CONV_LINEAR
VL = inputs.CONV_VANLEER


def _state(o):
    r, m, e, F = o.get_state()
    return np.concatenate([r, m.ravel(), e] + list(F))


def _set(o, x, step):
    N, dim = o.N, o.dim
    F, off = [], (2 + dim) * N
    for d in range(dim):
        F.append(x[off: off + o.NF[d]])
        off += o.NF[d]
    o.set_state(x[:N], x[N:(1 + dim) * N].reshape(dim, N), x[(1 + dim) * N:(2 + dim) * N], F,
                step=step)


def _blocks(o):
    N, dim = o.N, o.dim
    b = {"rho": (0, N)}
    for q in range(dim):
        b[f"mom{q}"] = ((1 + q) * N, (2 + q) * N)
    b["E"] = ((1 + dim) * N, (2 + dim) * N)
    off = (2 + dim) * N
    for d in range(dim):
        b[f"F{d}"] = (off, off + o.NF[d])
        off += o.NF[d]
    return b


def _noisy(o, gen, thermal):
    x = _state(o)
    N, dim = o.N, o.dim
    for a, b in ((0, N), ((1 + dim) * N, (2 + dim) * N)):
        x[a:b] *= 1.0 + thermal * gen.uniform(-1.0, 1.0, b - a)
    return x


def _state_case(c, nsteps, h, seed, thermal, skip_zero_flux):
    o = make_oracle(c, amplitude=5e-2)
    o.step(2)
    gen = np.random.default_rng(seed)
    x0 = _noisy(o, gen, thermal)
    w = gen.standard_normal(x0.size)
    ob = gen.standard_normal((nsteps, 4)) * 1e-2
    out = {}
    for name, (a, b) in _blocks(o).items():
        v = np.zeros_like(x0)
        # scaled to the block's size, so that every block is perturbed alike
        v[a:b] = gen.standard_normal(b - a) * np.sqrt(np.mean(x0[a:b] ** 2))
        if skip_zero_flux and name.startswith("F"):
            v[a:b][x0[a:b] == 0.0] = 0.0
        _set(o, x0, 2)
        _, hd, dout = o.tangent_linear_state(nsteps, v)
        tl = float(w @ dout) + float(np.sum(ob * hd))
        J = []
        for sgn in (1.0, -1.0):
            _set(o, x0 + sgn * h * v, 2)
            hist = o.step(nsteps)
            J.append(float(w @ _state(o)) + float(np.sum(ob * hist[:, :4])))
        out[name] = (tl, (J[0] - J[1]) / (2 * h))
    return out


def _check(out, tol):
    bad = {k: (tl, fd, abs(tl - fd) / abs(tl)) for k, (tl, fd) in out.items()
           if not abs(tl - fd) <= tol * abs(tl)}
    assert not bad, bad


def test_tl_state_linear_channel_with_body():
    c = inputs.scaled("cfg1", (28, 20), ns=24, convection=LIN, Re=20.0)
    _check(_state_case(c, 2, 1e-5, 41, 2e-2, False), 1e-6)


def test_tl_state_vanleer_channel_with_body():
    c = inputs.scaled("cfg1", (28, 20), ns=24, convection=VL, Re=20.0)
    _check(_state_case(c, 1, 1e-6, 42, 2e-2, True), 1e-5)


def test_tl_state_vanleer_sphere_3d():
    # a seed whose +-h states take the limiter's branches of the unperturbed one on
    # every face (its difference quotients at h = 1e-6 and 1e-7 agree); with about
    # 15000 face values a seed can also put one within 1e-6 of a branch point
    c = inputs.scaled("cfg3", (12, 10, 10), ns=40, convection=VL, Re=50.0)
    _check(_state_case(c, 1, 1e-6, 45, 2e-2, True), 1e-5)


@pytest.mark.parametrize("conv", [LIN, VL])
def test_tl_wall_temperature_matches_central_differences(conv):
    c = inputs.scaled("cfg5", (32, 32), ns=24, convection=conv)
    nsteps = 4
    o = make_oracle(c)
    x0 = _state(o)
    gen = np.random.default_rng(44)
    ob = gen.standard_normal((nsteps, 4))
    d = gen.standard_normal(c["ns"])
    _, hd = o.tangent_linear(nsteps, d)
    tl = float(np.sum(ob * hd))
    # the state form with a zero state direction is the same derivative
    _, hd2, _ = o.tangent_linear_state(nsteps, np.zeros_like(x0), d)
    assert np.array_equal(hd, hd2)
    Tw0 = np.full(c["ns"], float(c["Tw"]))
    h = 1e-6
    J = []
    for sgn in (1.0, -1.0):
        _set(o, x0, 0)
        o.set_wall_temperature(Tw0 + sgn * h * d)
        J.append(float(np.sum(ob * o.step(nsteps)[:, :4])))
    fd = (J[0] - J[1]) / (2 * h)
    assert abs(fd - tl) <= 1e-6 * abs(tl), (tl, fd)


@pytest.mark.parametrize("conv", [LIN, VL])
def test_tl_marker_positions_matches_central_differences(conv):
    # derivative along the candidate positions: kernel weights, the quadrature
    # weights (A eps = 1) and everything downstream. The ring is turned by 0.1 rad:
    # no candidate then lies on a grid line and no two are mirror images across a
    # symmetry line of a cell (an exact tie of the check routine, which any
    # perturbation breaks one way or the other), so within the step the check
    # routine keeps the same markers and every support the same cells
    c = inputs.scaled("cfg5", (32, 32), ns=24, convection=conv)
    nsteps = 3
    o = make_oracle(c)
    X, Ud, Tw, dA = inputs.markers(c)
    cs, sn = np.cos(0.1), np.sin(0.1)
    X = np.stack([cs * X[:, 0] - sn * X[:, 1], sn * X[:, 0] + cs * X[:, 1]], axis=1)
    o.set_markers(X, Ud, Tw, dA, dedupe=c.get("dedupe", True))
    x0 = _state(o)
    gen = np.random.default_rng(46)
    ob = gen.standard_normal((nsteps, 4))
    dX = gen.standard_normal(X.shape)
    _, hd = o.tangent_linear_shape(nsteps, dX)
    tl = float(np.sum(ob * hd))
    h = 1e-6
    J = []
    for sgn in (1.0, -1.0):
        o.set_markers(X + sgn * h * dX, Ud, Tw, dA, dedupe=c.get("dedupe", True))
        _set(o, x0, 0)
        J.append(float(np.sum(ob * o.step(nsteps)[:, :4])))
    fd = (J[0] - J[1]) / (2 * h)
    assert abs(fd - tl) <= 1e-6 * abs(tl), (tl, fd)
