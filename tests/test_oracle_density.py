"""Pins of the oracle's density-based step (App. B: central-upwind fluxes of
Kurganov, Noelle and Petrova for the inviscid part, explicit viscous and
conductive part at the intermediate state, then the marker sources).

- Sod's shock tube against the exact solution of the Riemann problem (the
  standard iterative solution for the star pressure and the wave pattern, as
  in Toro's textbook, written out below): L1 errors fall with the mesh and the
  star state is reached.
- The first step of a shear wave u = A sin(k y) (uniform rho, p) is exactly the
  explicit viscous step: the inviscid part is zero for it, the velocity drops
  by the factor 1 - dt (mu/rho) (4/h^2) sin^2(k h/2) and the internal energy
  gains dt mu (du/dy)^2 from the centred gradient.
- A uniform stream through inflow, outflow and slip sides stays uniform; in a
  periodic box mass, momentum and (inviscid) total energy are conserved.
- With one isolated marker the new state interpolates exactly to the targets
  rho_L U^d and c_v rho_L Theta^d (the sources are added to the final state)."""
import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2301_09349_amd import inputs

G = 1.4


def exact_riemann(x, t, left, right, x0=0.5):
    """rho, u, p of the exact solution of the 1D Riemann problem for an ideal gas
    (gamma = 1.4) at time t; left/right = (rho, u, p)."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl, cr = np.sqrt(G * pl / rl), np.sqrt(G * pr / rr)

    def f(p, rk, pk, ck):  # velocity jump across the wave of side k, and its derivative
        if p > pk:  # shock
            A, B = 2.0 / ((G + 1) * rk), (G - 1) / (G + 1) * pk
            s = np.sqrt(A / (p + B))
            return (p - pk) * s, s * (1.0 - (p - pk) / (2.0 * (B + p)))
        e = (G - 1) / (2 * G)  # rarefaction
        return 2 * ck / (G - 1) * ((p / pk) ** e - 1.0), (p / pk) ** (-(G + 1) / (2 * G)) / (rk * ck)

    p = 0.5 * (pl + pr)
    for _ in range(100):
        f1, d1 = f(p, rl, pl, cl)
        f2, d2 = f(p, rr, pr, cr)
        dp = (f1 + f2 + ur - ul) / (d1 + d2)
        p -= dp
        if abs(dp) < 1e-15:
            break
    f1, _ = f(p, rl, pl, cl)
    f2, _ = f(p, rr, pr, cr)
    us = 0.5 * (ul + ur) + 0.5 * (f2 - f1)
    g1, g2 = (G - 1) / (G + 1), (G - 1) / (2 * G)
    out = np.zeros((3, x.size))
    for i, xi in enumerate(x):
        s = (xi - x0) / t
        if s <= us:  # left of the contact
            if p > pl:
                sl = ul - cl * np.sqrt((G + 1) / (2 * G) * p / pl + g2)
                w = (rl, ul, pl) if s <= sl else (rl * (p / pl + g1) / (g1 * p / pl + 1), us, p)
            else:
                head, tail = ul - cl, us - cl * (p / pl) ** g2
                if s <= head:
                    w = (rl, ul, pl)
                elif s >= tail:
                    w = (rl * (p / pl) ** (1 / G), us, p)
                else:
                    u = 2 / (G + 1) * (cl + (G - 1) / 2 * ul + s)
                    c = 2 / (G + 1) * (cl + (G - 1) / 2 * (ul - s))
                    w = (rl * (c / cl) ** (2 / (G - 1)), u, pl * (c / cl) ** (2 * G / (G - 1)))
        else:
            if p > pr:
                sr = ur + cr * np.sqrt((G + 1) / (2 * G) * p / pr + g2)
                w = (rr, ur, pr) if s >= sr else (rr * (p / pr + g1) / (g1 * p / pr + 1), us, p)
            else:
                head, tail = ur + cr, us + cr * (p / pr) ** g2
                if s >= head:
                    w = (rr, ur, pr)
                elif s <= tail:
                    w = (rr * (p / pr) ** (1 / G), us, p)
                else:
                    u = 2 / (G + 1) * (-cr + (G - 1) / 2 * ur + s)
                    c = 2 / (G + 1) * (cr - (G - 1) / 2 * (ur - s))
                    w = (rr * (c / cr) ** (2 / (G - 1)), u, pr * (c / cr) ** (2 * G / (G - 1)))
        out[:, i] = w
    return out, p, us


def _box(n, bc, **over):
    h = 1.0 / n[0]
    c = dict(dim=2, n=n, lo=(0.0, 0.0), hi=(1.0, n[1] * h), bc=bc, Re=1e12, Ma=1 / np.sqrt(G),
             Pr=0.71, gamma=G, sutherland_S=0.3831, U_inf=(0.0, 0.0, 0.0), dt=0.0, cfl=0.5,
             dt_theta_max=1.0, dt_u_max=0.0, convection=inputs.CONV_VANLEER,
             viscosity_law=inputs.MU_CONSTANT, cg_rtol=1e-12, cg_maxit=100, scheme=1)
    c.update(over)
    return c


def _sod(N):
    # Ma = 1/sqrt(gamma): R = 1, theta = p / rho; reflecting (slip) ends, periodic in y
    c = _box((N, 3), [[inputs.SLIP] * 2, [inputs.PERIODIC] * 2], dt=0.1 / N)
    o = Oracle(c)
    xc = (np.arange(N) + 0.5) / N
    rho = np.tile(np.where(xc < 0.5, 1.0, 0.125), 3)
    th = np.tile(np.where(xc < 0.5, 1.0, 0.8), 3)
    o.init_primitive(rho, np.zeros((2, 3 * N)), th)
    o.step(2 * N)  # t = 0.2, before any wave reaches an end
    r, m, E, _ = o.get_state()
    r = r[:N]
    return xc, r, m[0][:N] / r, (G - 1) * E[:N]


def test_exact_riemann_solution_is_the_textbook_one():
    _, p, u = exact_riemann(np.array([0.5]), 0.2, (1.0, 0.0, 1.0), (0.125, 0.0, 0.1))
    assert p == pytest.approx(0.30313, abs=1e-5) and u == pytest.approx(0.92745, abs=1e-5)


def test_sod_shock_tube_against_the_exact_solution():
    errs = []
    for N in (200, 400):
        xc, r, u, p = _sod(N)
        ex, ps, us = exact_riemann(xc, 0.2, (1.0, 0.0, 1.0), (0.125, 0.0, 0.1))
        errs.append([np.mean(np.abs(r - ex[0])), np.mean(np.abs(u - ex[1])),
                     np.mean(np.abs(p - ex[2]))])
        star = (xc > 0.55) & (xc < 0.65)  # between the contact and the shock
        assert np.median(p[star]) == pytest.approx(ps, rel=2e-3)
        assert np.median(u[star]) == pytest.approx(us, rel=2e-3)
    assert errs[0][0] < 3.5e-3 and errs[0][1] < 6e-3 and errs[0][2] < 2.5e-3, errs
    for a, b in zip(errs[0], errs[1]):
        assert 1.4 < a / b < 2.2, errs


def test_first_step_of_a_shear_wave_is_the_viscous_step():
    n, A, Re = 32, 0.01, 50.0
    # linear face values: both sides of a face agree, so the central-upwind
    # dissipation (on jumps between the two sides) is zero for this flow
    c = _box((4, n), [[inputs.PERIODIC] * 2, [inputs.PERIODIC] * 2], Re=Re, dt=1e-3,
             hi=(4.0 / n, 1.0), convection=inputs.CONV_LINEAR)
    o = Oracle(c)
    h = 1.0 / n
    yc = (np.arange(n) + 0.5) * h
    k = 2 * np.pi
    u0 = A * np.sin(k * yc)
    u = np.zeros((2, 4 * n))
    u[0] = np.repeat(u0, 4)
    o.init_primitive(np.ones(4 * n), u, np.ones(4 * n))
    E0 = o.get_state()[2].copy()
    o.step(1)
    r, m, E, _ = o.get_state()
    mu, dt = 1.0 / Re, 1e-3
    factor = 1.0 - dt * mu * (4.0 / h ** 2) * np.sin(k * h / 2) ** 2
    assert np.allclose(m[0].reshape(n, 4)[:, 0], factor * u0, rtol=0, atol=1e-15)
    assert np.abs(m[1]).max() < 1e-15 and np.abs(r - 1.0).max() < 1e-15
    du = (np.roll(u0, -1) - np.roll(u0, 1)) / (2 * h)
    # E is about 2.5: its change of ~1e-7 is known to a few 1e-16 absolutely
    assert np.allclose((E - E0).reshape(n, 4)[:, 0], dt * mu * du ** 2, rtol=0, atol=2e-15)


def test_free_stream_is_kept():
    c = inputs.scaled("cfg1", (40, 32), ns=0, scheme=1, Ma=0.8)
    o = Oracle(c)
    rho, u, th = inputs.initial_fields(c, amplitude=0.0)
    o.init_primitive(rho, u, th)
    x0 = np.concatenate([np.ravel(v) for v in o.get_state()[:3]])
    o.step(10)
    x1 = np.concatenate([np.ravel(v) for v in o.get_state()[:3]])
    assert np.max(np.abs(x1 - x0)) <= 1e-13 * np.max(np.abs(x0))


def test_conservation_in_a_periodic_box():
    per = [[inputs.PERIODIC] * 2, [inputs.PERIODIC] * 2]
    c = inputs.scaled("cfg1", (36, 28), ns=0, bc=per, scheme=1, Ma=0.8, Re=1e12,
                      viscosity_law=inputs.MU_CONSTANT, U_inf=(0.5, 0.2, 0.0))
    o = Oracle(c)
    rho, u, th = inputs.initial_fields(c, amplitude=0.1)
    o.init_primitive(rho, u, th)

    def totals():
        r, m, E, _ = o.get_state()
        return np.array([r.sum(), m[0].sum(), m[1].sum(), (E + 0.5 * (m ** 2).sum(0) / r).sum()])

    t0 = totals()
    o.step(20)
    t1 = totals()
    assert np.all(np.abs(t1 - t0) <= 1e-13 * np.abs(t0).max()), (t0, t1)


def test_isolated_marker_reaches_its_targets():
    per = [[inputs.PERIODIC] * 2, [inputs.PERIODIC] * 2]
    c = inputs.scaled("cfg1", (32, 32), ns=0, bc=per, scheme=1, Ma=0.8, Re=100.0)
    o = Oracle(c)
    rho, u, th = inputs.initial_fields(dict(c, seed=3), amplitude=0.05)
    o.init_primitive(rho, u, th)
    Ud, Tw = np.array([[0.2, -0.1]]), np.array([1.25])
    o.set_markers(np.array([[0.3, 0.2]]), Ud=Ud, Tw=Tw)
    o.step(1)
    r, m, E, _ = o.get_state()
    rho_L = o.interp(r)[0]
    R = 1.0 / (G * 0.8 ** 2)
    cv = R / (G - 1)
    for q in range(2):
        assert o.interp(m[q])[0] == pytest.approx(rho_L * Ud[0, q], abs=1e-13)
    assert o.interp(E)[0] == pytest.approx(cv * rho_L * Tw[0], rel=1e-14)


def test_supersonic_sides_keep_a_uniform_stream():
    # Ma 2.5 through supersonic inflow and outflow sides stays uniform
    c = inputs.scaled("sup10", (48, 40), ns=0)
    o = Oracle(c)
    rho, u, th = inputs.initial_fields(c, amplitude=0.0)
    o.init_primitive(rho, u, th)
    x0 = np.concatenate([np.ravel(v) for v in o.get_state()[:3]])
    o.step(20)
    x1 = np.concatenate([np.ravel(v) for v in o.get_state()[:3]])
    assert np.max(np.abs(x1 - x0)) <= 1e-13 * np.max(np.abs(x0))


def test_supersonic_sides_need_the_density_based_step():
    c = inputs.scaled("sup10", (48, 40), ns=0, scheme=inputs.SCHEME_PRESSURE)
    with pytest.raises(ValueError):
        Oracle(c)


def test_markers_without_heat_exchange():
    # the energy source is zero: E** = E* and the heat total is zero, while the
    # momentum forcing acts as usual
    c = inputs.scaled("sup10", (64, 64), ns=28)
    from helpers import make_oracle

    o = make_oracle(c)
    h = o.step(3)
    assert np.all(h[:, 3] == 0.0)
    assert np.array_equal(o.intermediate("E_ss"), o.intermediate("E_s"))
    assert np.abs(h[:, 0]).min() > 0.0
    assert not np.array_equal(o.intermediate("mom_ss"), o.intermediate("mom_s"))
