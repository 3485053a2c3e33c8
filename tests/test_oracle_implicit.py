"""Pins of the oracle's implicit (backward-Euler) treatment of the compact
face-normal viscous and conductive fluxes.

- It differs from the explicit step only at second order in the time step: one
  step from the same state with dt and dt/2 gives differences in the ratio 4.
- Couette flow and linear conduction between immersed walls reach linear
  profiles and the analytic wall fluxes (to O(h)) with a time step five and ten
  times the explicit diffusion limit. Their steady states depend on the step at
  first order (the forcing is formed from the field the implicit predictor
  diffused without it), and tend to the explicit scheme's as dt -> 0: the wall
  flux's departure from the explicit value halves with dt.
- Free stream preservation and mass conservation hold as for the explicit step."""
import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2301_09349_amd import inputs
from helpers import make_oracle


def _state(o):
    r, m, e, F = o.get_state()
    return np.concatenate([r, m.ravel(), e] + list(F))


@pytest.mark.parametrize("name,shape", [("cfg1", (40, 32)), ("cfg3", (14, 12, 12))])
def test_implicit_differs_from_explicit_at_second_order(name, shape):
    diffs = []
    for dt in (4e-3, 2e-3):
        out = []
        for diffusion in (0, 1):
            c = inputs.scaled(name, shape, ns=40, Re=20.0, dt=dt, diffusion=diffusion)
            o = make_oracle(c, amplitude=5e-2)
            o.step(1)
            out.append(_state(o))
        diffs.append(np.linalg.norm(out[1] - out[0]) / np.linalg.norm(out[0]))
    ratio = diffs[0] / diffs[1]
    assert 3.3 < ratio < 4.7, (diffs, ratio)


def _walls(Uw, Ttop, Tbot, ny, dt, steps, diffusion, nx=8):
    h = 2.0 / ny
    c = dict(dim=2, n=(nx, ny), lo=(0.0, -1.0), hi=(nx * h, 1.0), bc=[[0, 0], [0, 0]], Re=10.0,
             Ma=0.1, Pr=0.71, gamma=1.4, sutherland_S=0.3831, U_inf=(0.0, 0.0, 0.0), dt=dt,
             cfl=0.5, dt_theta_max=max(1.0, Ttop, Tbot), dt_u_max=Uw, convection=1,
             viscosity_law=1, cg_rtol=1e-12, cg_maxit=5000, diffusion=diffusion)
    o = Oracle(c)
    xs = (np.arange(nx) + 0.5) * h
    X = np.concatenate([np.stack([xs, np.full(nx, 0.5)], 1), np.stack([xs, np.full(nx, -0.5)], 1)])
    Ud = np.zeros_like(X)
    Ud[:nx, 0] = Uw
    Ud[nx:, 0] = -Uw
    Tw = np.concatenate([np.full(nx, Ttop), np.full(nx, Tbot)])
    o.init_primitive(np.ones(nx * ny), np.zeros((2, nx * ny)), np.ones(nx * ny))
    o.set_markers(X, Ud, Tw, dedupe=True)
    o.step(steps)
    r, m, E, _ = o.get_state()
    cv = 1.0 / (1.4 * 0.01) / 0.4
    u = (m[0] / r).reshape(ny, nx).mean(1)
    th = (E / r / cv).reshape(ny, nx).mean(1)
    yc = -1 + (np.arange(ny) + 0.5) * h
    mf = o.marker_fields()
    eps = o.eps()
    top = o.keep() < nx
    dV = h * h
    F_top = -dV * (eps[top] * mf[top, 4]).sum()
    H_top = dV * (eps[top] * mf[top, 6]).sum()
    inner = np.abs(yc) < 0.5 - 2 * h
    return dict(yc=yc, u=u, th=th, inner=inner, F_top=F_top, H_top=H_top, Lx=nx * h)


def _explicit_dt(ny):
    # the explicit step's limit for these walls: 0.5 / (2 alpha sum h^-2), alpha =
    # gamma mu / Pr at theta = 1 (the convective part is negligible)
    h = 2.0 / ny
    alpha = 1.4 * 0.1 / 0.71
    return 0.5 / (2.0 * alpha * 2.0 / h ** 2)


def _runs(Uw, Ttop, Tbot, ny=32, t_end=7.5):
    out = {}
    for mult in (10, 5):
        dt = mult * _explicit_dt(ny)
        out[mult] = _walls(Uw, Ttop, Tbot, ny, dt, int(round(t_end / dt)), 1)
    out[0] = _walls(Uw, Ttop, Tbot, ny, _explicit_dt(ny), 3000, 0)
    return out


def test_implicit_couette_with_large_steps():
    Uw, mu = 0.1, 0.1
    r = _runs(Uw, 1.0, 1.0)
    F_exact = -4.0 * mu * Uw * r[0]["Lx"]
    for mult in (10, 5):
        yi, ui = r[mult]["yc"][r[mult]["inner"]], r[mult]["u"][r[mult]["inner"]]
        slope, icpt = np.polyfit(yi, ui, 1)
        assert np.abs(ui - (slope * yi + icpt)).max() < 1e-6 * Uw
        assert abs(slope - 2 * Uw) < 0.1 * 2 * Uw
        assert abs(r[mult]["F_top"] - F_exact) < 0.1 * abs(F_exact)
    d10 = abs(r[10]["F_top"] - r[0]["F_top"])
    d5 = abs(r[5]["F_top"] - r[0]["F_top"])
    assert 1.6 < d10 / d5 < 2.4, (d10, d5)


def test_implicit_conduction_with_large_steps():
    Ttop, Tbot = 0.9, 1.1
    r = _runs(0.0, Ttop, Tbot)
    cp = 1.0 / (1.4 * 0.01) / 0.4 * 1.4
    lam = cp * 0.1 / 0.71
    H_exact = 2.0 * lam * (Ttop - Tbot) / 1.0 * r[0]["Lx"]
    for mult in (10, 5):
        yi, ti = r[mult]["yc"][r[mult]["inner"]], r[mult]["th"][r[mult]["inner"]]
        slope, icpt = np.polyfit(yi, ti, 1)
        assert np.abs(ti - (slope * yi + icpt)).max() < 1e-6
        assert abs(slope - (Ttop - Tbot)) < 0.1 * abs(Ttop - Tbot)
        assert abs(r[mult]["H_top"] - H_exact) < 0.1 * abs(H_exact)
    d10 = abs(r[10]["H_top"] - r[0]["H_top"])
    d5 = abs(r[5]["H_top"] - r[0]["H_top"])
    assert 1.6 < d10 / d5 < 2.4, (d10, d5)


def test_implicit_free_stream_and_mass():
    c = inputs.scaled("cfg1", (32, 24), ns=0, diffusion=1)
    o = make_oracle(c, markers=False, amplitude=0.0)
    x0 = _state(o)
    o.step(5)
    assert np.abs(_state(o) - x0).max() < 1e-12 * np.abs(x0).max()
    cp = inputs.scaled("cfg1", (32, 24), ns=30, diffusion=1,
                       bc=[[inputs.PERIODIC] * 2, [inputs.PERIODIC] * 2])
    o = make_oracle(cp)
    m0 = o.get_state()[0].sum()
    o.step(5)
    assert abs(o.get_state()[0].sum() - m0) < 1e-12 * m0
