"""Pins of the FP64 oracle against what the paper and the mathematics fix, independent
of the oracle's own code paths: closed forms of the Pinelli kernel (Sec. 2.2, Eq. (6)),
moment identities that make interpolation exact on linear fields, the partition of
unity that defines eps (Eqs. (8)-(9)), the discrete adjointness of interpolation
(Eq. (5)) and spreading (Eq. (7)), the forcing identities (Eqs. (10), (17)) on an
isolated marker, free-stream preservation, mass conservation, second-order
consistency of the step with the continuous balance laws (Sec. 2.1, Eqs. (1)-(4))
on a manufactured field, and the Fourier symbol of the pressure operator."""
import math

import numpy as np
import pytest

from oracle.oracle import Oracle, kernel
from paper_2301_09349_amd import inputs

pytestmark = pytest.mark.filterwarnings("ignore")


# ------------------------------------------------------------------ kernel
def test_kernel_closed_form_values():
    assert kernel(0.0) == pytest.approx(2.0 / 3.0, abs=1e-16)
    assert kernel(0.5) == pytest.approx(0.5, abs=1e-16)
    assert kernel(1.0) == pytest.approx(1.0 / 6.0, abs=1e-16)
    assert kernel(1.5) == 0.0
    assert kernel(1.6) == 0.0 and kernel(-2.0) == 0.0
    # even, continuous at 0.5 from both branches
    for r in (0.1, 0.37, 0.9, 1.3):
        assert kernel(r) == kernel(-r)
    assert abs(kernel(0.5 - 1e-12) - kernel(0.5 + 1e-12)) < 1e-11


def test_kernel_moments():
    # for every shift: sum phi = 1, sum r phi = 0, sum phi^2 = 1/2 (the three
    # conditions the 3-point kernel is built on)
    rng = np.random.default_rng(0)
    for xi in rng.uniform(0.0, 1.0, 2000):
        r = np.array([(-1.0 + 0.5) - xi, 0.5 - xi, 1.5 - xi])
        w = np.array([kernel(v) for v in r])
        assert abs(w.sum() - 1.0) < 3e-16
        assert abs((r * w).sum()) < 3e-16
        assert abs((w * w).sum() - 0.5) < 3e-16


# ------------------------------------------------------------ markers / IBM
def _periodic_case(dim, n, Re=50.0, Ma=0.2, **over):
    L = 2.0 * math.pi
    c = dict(dim=dim, n=tuple(n), lo=tuple([0.0] * dim), hi=tuple([L] * dim),
             bc=[[inputs.PERIODIC] * 2 for _ in range(dim)], Re=Re, Ma=Ma, Pr=0.71, gamma=1.4,
             sutherland_S=inputs.SUTHERLAND_AIR, U_inf=(1.0, 0.0, 0.0), dt=1e-3,
             convection=inputs.CONV_LINEAR, viscosity_law=inputs.MU_SUTHERLAND, cg_rtol=1e-13,
             cg_maxit=5000, dt_theta_max=1.0, dt_u_max=0.0, Tw=1.0, ns=0, seed=7)
    c.update(over)
    return c


def _cell_centres(o):
    c = o.case
    h = [(c["hi"][a] - c["lo"][a]) / c["n"][a] for a in range(o.dim)]
    axes = [c["lo"][a] + (np.arange(c["n"][a]) + 0.5) * h[a] for a in range(o.dim)]
    grids = np.meshgrid(*axes, indexing="ij")
    # x-fastest flattening
    return [g.transpose(*range(o.dim)[::-1]).ravel() for g in grids], h


@pytest.mark.parametrize("dim", [2, 3])
def test_support_weights_reproduce_linear_fields(dim):
    n = (24, 20, 18)[:dim]
    c = _periodic_case(dim, n)
    o = Oracle(c)
    rng = np.random.default_rng(1)
    X = rng.uniform(1.0, 5.0, (25, dim))
    o.set_markers(X)
    cells, w = o.support()
    assert np.allclose(w.sum(axis=1), 1.0, atol=1e-15)  # partition of unity per marker
    xc, h = _cell_centres(o)
    for a in range(dim):
        # first moment: sum_c w_ck x_c = X_k  (interpolation exact on linear fields)
        mom1 = (w * xc[a][cells]).sum(axis=1)
        assert np.abs(mom1 - X[:, a]).max() < 1e-13
        lin = 0.3 + 0.7 * xc[a]
        assert np.abs(o.interp(lin) - (0.3 + 0.7 * X[:, a])).max() < 1e-13


@pytest.mark.parametrize("dim", [2, 3])
def test_isolated_marker_quadrature(dim):
    # A_kk = prod_d sum phi^2 = 2^-d, so an isolated marker has eps = 2^d
    c = _periodic_case(dim, (20, 20, 20)[:dim])
    o = Oracle(c)
    o.set_markers(np.array([[2.1, 3.3, 2.9][:dim]]))
    assert o.eps()[0] == pytest.approx(2.0 ** dim, rel=1e-14)


def test_partition_of_unity_and_adjointness():
    c = _periodic_case(2, (64, 64))
    o = Oracle(c)
    X, _ = inputs.ring(60, diameter=2.0, center=(math.pi, math.pi))
    o.set_markers(X)
    eps = o.eps()
    # I S 1 = 1 at every marker (Eq. (8))
    assert np.abs(o.interp(o.spread(np.ones(o.ns))) - 1.0).max() < 1e-11
    # <I u, F>_eps = <u, S F> for random u, F
    rng = np.random.default_rng(2)
    for _ in range(3):
        u = rng.standard_normal(o.N)
        F = rng.standard_normal(o.ns)
        lhs = np.sum(eps * F * o.interp(u))
        rhs = np.sum(u * o.spread(F))
        assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + np.abs(eps * F).sum())
    # spreading conserves the total: sum_c (S F)_c = sum_k eps_k F_k
    F = rng.standard_normal(o.ns)
    assert abs(o.spread(F).sum() - (eps * F).sum()) < 1e-10


def test_eps_against_brute_force_gram():
    # tiny set: build A from the support weights by brute force over all cells and
    # solve with LAPACK; compare with the oracle's quadrature
    c = _periodic_case(2, (16, 16))
    o = Oracle(c)
    X = np.array([[2.0, 2.0], [2.25, 2.1], [2.6, 2.3], [3.9, 1.7]])
    o.set_markers(X)
    cells, w = o.support()
    W = np.zeros((o.N, o.ns))
    for k in range(o.ns):
        for s in range(cells.shape[1]):
            W[cells[k, s], k] += w[k, s]
    A = W.T @ W
    assert np.allclose(np.diag(A)[3], 0.25, atol=1e-15)  # isolated marker: 2^-d
    eps = np.linalg.solve(A, np.ones(o.ns))
    assert np.abs(o.eps() - eps).max() < 1e-12 * np.abs(eps).max()


def test_check_routine_keeps_nearest_marker_per_cell():
    c = _periodic_case(2, (16, 16))
    o = Oracle(c)
    h = 2.0 * math.pi / 16
    # three candidates in cell (3, 4), one alone in cell (8, 8)
    ctr = np.array([3.5 * h, 4.5 * h])
    X = np.array([ctr + [0.3 * h, 0.1 * h], ctr + [-0.05 * h, 0.02 * h], ctr + [0.2 * h, -0.3 * h],
                  [8.5 * h, 8.4 * h]])
    o.set_markers(X, dedupe=True)
    assert list(o.keep()) == [1, 3]
    o2 = Oracle(c)
    o2.set_markers(X, dedupe=False)
    assert list(o2.keep()) == [0, 1, 2, 3]


def _isolated_step_case():
    c = _periodic_case(2, (32, 32), Re=100.0, Ma=0.3, dt=2e-3)
    o = Oracle(c)
    rho, u, th = inputs.initial_fields(dict(c, seed=3), amplitude=0.05)
    o.init_primitive(rho, u, th)
    Ud = np.array([[0.2, -0.1]])
    Tw = np.array([1.25])
    o.set_markers(np.array([[3.0, 3.2]]), Ud=Ud, Tw=Tw)
    return o, Ud, Tw


def test_forcing_reaches_target_at_isolated_marker():
    # one marker: eps = 4 and I S F = F, so after spreading the interpolated momentum is
    # exactly rho_L U^d (Eq. (10)) and the interpolated internal energy is exactly
    # c_v rho_L Theta^d (Eq. (17))
    o, Ud, Tw = _isolated_step_case()
    o.step(1)
    mf = o.marker_fields()
    rho_L = mf[0, 0]
    R = 1.0 / (1.4 * 0.3 ** 2)
    cv = R / 0.4
    mss = o.intermediate("mom_ss")
    Ess = o.intermediate("E_ss")
    for q in range(2):
        assert o.interp(mss[q])[0] == pytest.approx(rho_L * Ud[0, q], abs=1e-13)
    assert o.interp(Ess)[0] == pytest.approx(cv * rho_L * Tw[0], rel=1e-14)
    # forces and heat: F = (rho_L U^d - M)/dt, Q = (c_v rho_L Theta^d - E_L)/dt
    dt = o.dt
    M = mf[0, 1:3]
    EL = mf[0, 3]
    assert np.allclose(mf[0, 4:6], (rho_L * Ud[0] - M) / dt, rtol=0, atol=1e-12 * abs(M).max() / dt)
    assert mf[0, 6] == pytest.approx((cv * rho_L * Tw[0] - EL) / dt, rel=1e-12)


def test_free_stream_preserved_without_body():
    c = inputs.scaled("cfg1", (40, 32), ns=0)
    o = Oracle(c)
    rho, u, th = inputs.initial_fields(c, amplitude=0.0)
    o.init_primitive(rho, u, th)
    h = o.step(10)
    r, m, E, F = o.get_state()
    R = 1.0 / (1.4 * 0.1 ** 2)
    cv = R / 0.4
    assert np.abs(r - 1.0).max() < 1e-13
    assert np.abs(m[0] - 1.0).max() < 1e-13 and np.abs(m[1]).max() < 1e-13
    assert np.abs(E / cv - 1.0).max() < 1e-13
    assert h[:, 5].max() <= 1  # the pressure equation is satisfied by the start value


def test_mass_conserved_in_periodic_box_with_body():
    c = _periodic_case(2, (48, 40), Re=100.0, Ma=0.2, dt=4e-3)
    o = Oracle(c)
    rho, u, th = inputs.initial_fields(dict(c, seed=4), amplitude=0.02)
    o.init_primitive(rho, u, th)
    X, dA = inputs.ring(40, center=(math.pi, math.pi))
    o.set_markers(X, Tw=np.full(40, 1.3), dA=dA, dedupe=True)
    h = o.step(15)
    m0 = (2 * math.pi) ** 2 / (48 * 40) * rho.sum()
    assert np.abs(h[:, 4] - m0).max() < 1e-13 * m0


def test_mirror_symmetry_without_perturbation():
    c = inputs.scaled("cfg1", (64, 64), ns=60)
    o = Oracle(c)
    rho, u, th = inputs.initial_fields(c, amplitude=0.0)
    o.init_primitive(rho, u, th)
    X, Ud, Tw, dA = inputs.markers(c)
    o.set_markers(X, Ud, Tw, dA, dedupe=True)
    h = o.step(8)
    r, m, E, F = o.get_state()
    r2 = r.reshape(64, 64)
    mx = m[0].reshape(64, 64)
    my = m[1].reshape(64, 64)
    assert np.abs(r2 - r2[::-1, :]).max() < 1e-12
    assert np.abs(mx - mx[::-1, :]).max() < 1e-11
    assert np.abs(my + my[::-1, :]).max() < 1e-11
    assert np.abs(h[:, 1]).max() < 1e-9 * np.abs(h[:, 0]).max()  # no lift


# --------------------------------------------- pressure operator (CG system)
def test_pressure_operator_fourier_symbol_and_cg():
    n = (32, 24)
    c = _periodic_case(2, n, dt=0.05)
    o = Oracle(c)
    L = 2 * math.pi
    h = [L / n[0], L / n[1]]
    xc, _ = _cell_centres(o)
    psi = np.full(o.N, 0.7)
    dt = 0.05
    for kx, ky in ((1, 0), (3, 2), (7, 5)):
        mode = np.cos(kx * xc[0] + ky * xc[1])
        lam = 0.7 + dt * dt * (4 / h[0] ** 2 * math.sin(kx * h[0] / 2) ** 2 +
                               4 / h[1] ** 2 * math.sin(ky * h[1] / 2) ** 2)
        assert np.abs(o.helmholtz(psi, mode) - lam * mode).max() < 1e-12
    # CG against an FFT solve of the same periodic problem
    rng = np.random.default_rng(5)
    b = rng.standard_normal(o.N)
    x, it = o.cg(psi, b, np.zeros(o.N))
    kx = 2 * math.pi * np.fft.fftfreq(n[0], d=h[0])
    ky = 2 * math.pi * np.fft.fftfreq(n[1], d=h[1])
    KX, KY = np.meshgrid(kx, ky, indexing="xy")
    sym = 0.7 + dt * dt * (4 / h[0] ** 2 * np.sin(KX * h[0] / 2) ** 2 +
                           4 / h[1] ** 2 * np.sin(KY * h[1] / 2) ** 2)
    xf = np.real(np.fft.ifft2(np.fft.fft2(b.reshape(n[1], n[0])) / sym)).ravel()
    assert it > 0
    assert np.abs(x - xf).max() < 1e-11 * np.abs(xf).max()


def test_pressure_operator_symmetric_positive_with_walls():
    c = inputs.scaled("cfg1", (20, 14), ns=0)
    o = Oracle(c)
    rng = np.random.default_rng(6)
    psi = rng.uniform(0.5, 1.5, o.N)
    A = np.stack([o.helmholtz(psi, e) for e in np.eye(o.N)], axis=1)
    assert np.abs(A - A.T).max() < 1e-14 * np.abs(A).max()
    assert np.linalg.eigvalsh(0.5 * (A + A.T)).min() > 0


# --------------------------------------------- consistency with the PDE (MMS)
def _mms_rhs(dim, Re, Ma, Pr=0.71, gamma=1.4, S=inputs.SUTHERLAND_AIR):
    """Continuous right-hand sides of Eqs. (1)-(3) (internal-energy form, q = f = 0)
    for a smooth periodic field, by symbolic differentiation."""
    import sympy as sp

    X = sp.symbols("x0:%d" % dim, real=True)
    x, y = X[0], X[1]
    z = X[2] if dim == 3 else 0
    rho = 1 + sp.Rational(1, 10) * sp.sin(x) * sp.cos(y) + sp.Rational(1, 20) * sp.sin(z)
    u = [1 + sp.Rational(1, 10) * sp.cos(x + y) + sp.Rational(1, 20) * sp.cos(z),
         sp.Rational(1, 10) * sp.sin(x - 2 * y) + sp.Rational(1, 20) * sp.sin(z)]
    if dim == 3:
        u.append(sp.Rational(1, 10) * sp.cos(x) * sp.sin(z) + sp.Rational(1, 20) * sp.sin(y))
    th = 1 + sp.Rational(1, 10) * sp.cos(x) * sp.sin(y) + sp.Rational(1, 20) * sp.cos(z)
    R = 1 / (gamma * Ma ** 2)
    cv = R / (gamma - 1)
    cp = gamma * cv
    mu = (1 / Re) * th * sp.sqrt(th) * (1 + S) / (th + S)
    lam = cp * mu / Pr
    p = rho * R * th
    e = cv * th
    div = sum(sp.diff(u[a], X[a]) for a in range(dim))
    tau = [[mu * (sp.diff(u[a], X[b]) + sp.diff(u[b], X[a])) - (2 * mu * div / 3 if a == b else 0)
            for b in range(dim)] for a in range(dim)]
    r_rho = -sum(sp.diff(rho * u[a], X[a]) for a in range(dim))
    r_m = [-sum(sp.diff(rho * u[a] * u[b], X[b]) for b in range(dim)) - sp.diff(p, X[a]) +
           sum(sp.diff(tau[a][b], X[b]) for b in range(dim)) for a in range(dim)]
    phi = sum(tau[a][b] * sp.diff(u[a], X[b]) for a in range(dim) for b in range(dim))
    r_E = (-sum(sp.diff(rho * e * u[a], X[a]) for a in range(dim)) - p * div + phi +
           sum(sp.diff(lam * sp.diff(th, X[a]), X[a]) for a in range(dim)))
    f = lambda ex: sp.lambdify(X, ex, "numpy")  # noqa: E731
    return f(rho), [f(v) for v in u], f(th), f(r_rho), [f(v) for v in r_m], f(r_E)


def _mms_errors(dim, n, full_step):
    Re, Ma = 20.0, 0.5
    c = _periodic_case(dim, n, Re=Re, Ma=Ma)
    frho, fu, fth, rr, rm, rE = _mms_rhs(dim, Re, Ma)
    o = Oracle(c)
    xc, h = _cell_centres(o)
    ones = np.ones(o.N)
    rho = frho(*xc) * ones
    u = np.stack([fu[a](*xc) * ones for a in range(dim)])
    th = fth(*xc) * ones
    o.init_primitive(rho, u, th)
    R = 1.0 / (1.4 * Ma ** 2)
    cv = R / 0.4
    if full_step:
        # dt ~ h^2 so that the O(dt) splitting error converges with the O(h^2) one
        dt = 0.05 * min(h) ** 2
        c2 = dict(c, dt=dt)
        o = Oracle(c2)
        o.init_primitive(rho, u, th)
        r0, m0, E0, _ = o.get_state()
        o.step(1)
        r1, m1, E1, _ = o.get_state()
        d_rho, d_m, d_E = (r1 - r0) / dt, (m1 - m0) / dt, (E1 - E0) / dt
    else:
        dt = o.dt
        r0, m0, E0, _ = o.get_state()
        o.predictor_only()
        d_rho = (o.intermediate("rho_s") - r0) / dt
        d_m = (o.intermediate("mom_s") - m0) / dt
        d_E = (o.intermediate("E_s") - E0) / dt
    e_rho = np.abs(d_rho - rr(*xc) * ones).max()
    e_m = max(np.abs(d_m[a] - rm[a](*xc) * ones).max() for a in range(dim))
    e_E = np.abs(d_E - rE(*xc) * ones).max() / cv
    return np.array([e_rho, e_m, e_E])


@pytest.mark.parametrize("full_step", [False, True])
def test_second_order_consistency_2d(full_step):
    e1 = _mms_errors(2, (24, 24), full_step)
    e2 = _mms_errors(2, (48, 48), full_step)
    order = np.log2(e1 / e2)
    assert (order > 1.75).all(), (e1, e2, order)


def test_second_order_consistency_3d_predictor():
    e1 = _mms_errors(3, (12, 12, 12), False)
    e2 = _mms_errors(3, (24, 24, 24), False)
    order = np.log2(e1 / e2)
    assert (order > 1.75).all(), (e1, e2, order)
