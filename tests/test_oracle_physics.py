"""Physics pins of the oracle's whole step: steady Couette flow and linear conduction
between two immersed walls (lines of markers) in a periodic box. The analytic
solutions are linear profiles; the wall shear and the wall heat flux follow from
mu dU/dy and lambda dT/dy. The immersed walls are diffuse over O(h), so the
discrete solution reaches the analytic wall fluxes to O(h)."""
import numpy as np
import pytest

from oracle.oracle import Oracle


def _walls(Uw, Ttop, Tbot, ny, steps, nx=8):
    h = 2.0 / ny
    c = dict(dim=2, n=(nx, ny), lo=(0.0, -1.0), hi=(nx * h, 1.0), bc=[[0, 0], [0, 0]], Re=10.0,
             Ma=0.1, Pr=0.71, gamma=1.4, sutherland_S=0.3831, U_inf=(0.0, 0.0, 0.0), dt=0.0,
             cfl=0.5, dt_theta_max=max(1.0, Ttop, Tbot), dt_u_max=Uw, convection=1,
             viscosity_law=1, cg_rtol=1e-12, cg_maxit=5000)
    o = Oracle(c)
    xs = (np.arange(nx) + 0.5) * h
    X = np.concatenate([np.stack([xs, np.full(nx, 0.5)], 1), np.stack([xs, np.full(nx, -0.5)], 1)])
    Ud = np.zeros_like(X)
    Ud[:nx, 0] = Uw
    Ud[nx:, 0] = -Uw
    Tw = np.concatenate([np.full(nx, Ttop), np.full(nx, Tbot)])
    o.init_primitive(np.ones(nx * ny), np.zeros((2, nx * ny)), np.ones(nx * ny))
    # each marker stands for a segment h of its wall (per unit span)
    o.set_markers(X, Ud, Tw, dA=np.full(2 * nx, h), dedupe=True)
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
    F_top = -dV * (eps[top] * mf[top, 4]).sum()  # force of the fluid on the upper wall
    H_top = dV * (eps[top] * mf[top, 6]).sum()  # heat given by the upper wall to the fluid
    inner = np.abs(yc) < 0.5 - 2 * h
    _, heat, qloc = o.wall_fluxes()
    return dict(yc=yc, u=u, th=th, inner=inner, F_top=F_top, H_top=H_top, Lx=nx * h, h=h,
                v=(m[1] / r), heat=heat, qloc=qloc, top=top)


def test_couette_between_immersed_walls():
    Uw, mu = 0.1, 0.1
    errs = []
    for ny, steps in ((32, 3000), (64, 11000)):
        r = _walls(Uw, 1.0, 1.0, ny, steps)
        yi, ui = r["yc"][r["inner"]], r["u"][r["inner"]]
        slope, icpt = np.polyfit(yi, ui, 1)
        assert np.abs(ui - (slope * yi + icpt)).max() < 1e-6 * Uw  # linear profile
        assert abs(icpt) < 1e-9 and np.abs(r["v"]).max() < 1e-9
        assert abs(slope - 2 * Uw) < 0.1 * 2 * Uw  # U_w / half-gap, to O(h)
        # both faces of the wall resist its motion: F = -mu (2Uw/1) * 2 * Lx
        F_exact = -4.0 * mu * Uw * r["Lx"]
        assert abs(r["F_top"] - F_exact) < 0.1 * abs(F_exact)
        errs.append(abs(r["F_top"] - F_exact) / abs(F_exact))
    # first order in h, as a diffuse interface should be
    assert 1.6 < errs[0] / errs[1] < 2.4


def test_linear_conduction_between_immersed_walls():
    Ttop, Tbot = 0.9, 1.1
    r = _walls(0.0, Ttop, Tbot, 32, 3000)
    yi, ti = r["yc"][r["inner"]], r["th"][r["inner"]]
    slope, icpt = np.polyfit(yi, ti, 1)
    assert np.abs(ti - (slope * yi + icpt)).max() < 1e-6
    assert abs(icpt - 1.0) < 1e-6
    assert abs(slope - (Ttop - Tbot)) < 0.1 * abs(Ttop - Tbot)
    cp = 1.0 / (1.4 * 0.01) / 0.4 * 1.4
    lam = cp * 0.1 / 0.71
    # heat given to the fluid by the cold upper wall: both sides conduct into it
    H_exact = 2.0 * lam * (Ttop - Tbot) / 1.0 * r["Lx"]
    assert abs(r["H_top"] - H_exact) < 0.1 * abs(H_exact)
    # the local heat flux per unit wall area: the same at every marker of a wall (the
    # problem does not depend on x) and lambda dT/dy on each of the wall's two faces
    q_top = r["qloc"][r["top"]]
    assert np.abs(q_top - q_top.mean()).max() < 1e-10 * abs(q_top.mean())
    q_exact = 2.0 * lam * (Ttop - Tbot) / 1.0
    assert abs(q_top.mean() - q_exact) < 0.1 * abs(q_exact)
    assert abs((r["qloc"] * r["h"]).sum() - r["heat"].sum()) < 1e-12 * np.abs(r["heat"]).sum()
