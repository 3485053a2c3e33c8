"""GPU parity of the density-based step (App. B: central-upwind inviscid part,
explicit viscous and conductive part, marker sources) against the oracle's,
on the same seeded inputs; FP64 states are held to 1e-11."""
import numpy as np
import pytest
import torch

from paper_2301_09349_amd import _lib, inputs
from helpers import make_gpu, make_oracle, rel_l2, state_errors, to_np
from test_oracle_density import G, _box, exact_riemann

pytestmark = pytest.mark.gpu

DENS = inputs.SCHEME_DENSITY


def _sod_pair(N, precision="fp64"):
    from oracle.oracle import Oracle
    from paper_2301_09349_amd.solver import IBMSolver

    c = _box((N, 3), [[inputs.SLIP] * 2, [inputs.PERIODIC] * 2], dt=0.1 / N)
    xc = (np.arange(N) + 0.5) / N
    rho = np.tile(np.where(xc < 0.5, 1.0, 0.125), 3)
    th = np.tile(np.where(xc < 0.5, 1.0, 0.8), 3)
    u = np.zeros((2, 3 * N))
    g = IBMSolver(c, precision, max_markers=1)
    g.init_primitive(rho, u, th)
    o = Oracle(c)
    o.init_primitive(rho, u, th)
    return c, xc, g, o


def test_sod_shock_tube_parity_and_exact_solution(cuda):
    N = 200
    c, xc, g, o = _sod_pair(N)
    g.step(2 * N)
    o.step(2 * N)
    for k, v in state_errors(g, o).items():
        assert v < 1e-11, (k, v)
    r, m, E, _ = g.get_state()
    r = to_np(r)[:N]
    p = (G - 1) * to_np(E)[:N]
    ex, ps, _ = exact_riemann(xc, 0.2, (1.0, 0.0, 1.0), (0.125, 0.0, 0.1))
    assert np.mean(np.abs(r - ex[0])) < 3.5e-3
    assert np.median(p[(xc > 0.55) & (xc < 0.65)]) == pytest.approx(ps, rel=2e-3)


@pytest.mark.parametrize("conv", [inputs.CONV_VANLEER, inputs.CONV_LINEAR])
def test_density_cylinder_parity(cuda, conv):
    # ragged grid, body, Ma 0.8, inflow/outflow/slip sides
    c = inputs.scaled("cfg1", (97, 78), ns=60, Ma=0.8, Re=50.0, convection=conv, scheme=DENS)
    g, o = make_gpu(c, amplitude=2e-2), make_oracle(c, amplitude=2e-2)
    assert g.dt == o.dt
    hg, _ = g.step(20)
    ho = o.step(20)
    for k, v in state_errors(g, o).items():
        assert v < 1e-11, (k, v)
    assert rel_l2(to_np(hg), ho[:, :4]) < 1e-9
    # the momentum after the sources (the new state's)
    assert rel_l2(to_np(g.field("mom_ss")), o.intermediate("mom_ss")) < 1e-11


def test_density_sphere_3d_parity(cuda):
    c = inputs.scaled("cfg3", (36, 30, 28), ns=300, Ma=0.8, Re=100.0, scheme=DENS)
    g, o = make_gpu(c, amplitude=2e-2), make_oracle(c, amplitude=2e-2)
    hg, _ = g.step(5)
    ho = o.step(5)
    for k, v in state_errors(g, o).items():
        assert v < 1e-11, (k, v)
    assert rel_l2(to_np(hg), ho[:, :4]) < 1e-9


def test_density_moving_body_parity(cuda):
    c = inputs.scaled("osc2", (96, 96), ns=80, Ma=0.8, scheme=DENS)
    g, o = make_gpu(c), make_oracle(c)
    hg, _ = g.step(6)
    ho = o.step(6)
    for k, v in state_errors(g, o).items():
        assert v < 1e-11, (k, v)
    assert rel_l2(to_np(hg), ho[:, :4]) < 1e-8


def test_density_periodic_box_conserves(cuda):
    per = [[inputs.PERIODIC] * 2, [inputs.PERIODIC] * 2]
    c = inputs.scaled("cfg1", (70, 37), ns=0, bc=per, scheme=DENS, Ma=0.8, Re=1e12,
                      viscosity_law=inputs.MU_CONSTANT, U_inf=(0.5, 0.2, 0.0))
    g, o = make_gpu(c, amplitude=0.1), make_oracle(c, amplitude=0.1)

    def totals(s):
        r, m, E, _ = [to_np(x) if not isinstance(x, list) else x for x in s.get_state()]
        m = m.reshape(2, -1)
        return np.array([r.sum(), m[0].sum(), m[1].sum(), (E + 0.5 * (m ** 2).sum(0) / r).sum()])

    t0 = totals(g)
    g.step(20)
    o.step(20)
    t1 = totals(g)
    assert np.all(np.abs(t1 - t0) <= 1e-13 * np.abs(t0).max()), (t0, t1)
    for k, v in state_errors(g, o).items():
        assert v < 1e-11, (k, v)


def test_density_free_stream_is_kept(cuda):
    c = inputs.scaled("cfg1", (70, 37), ns=0, scheme=DENS, Ma=0.8)
    g = make_gpu(c, amplitude=0.0)
    x0 = [to_np(x).copy() for x in g.get_state()[:3]]
    g.step(10)
    for a, b in zip(x0, g.get_state()[:3]):
        assert np.max(np.abs(to_np(b) - a)) <= 1e-13 * np.max(np.abs(a))


def test_density_fp32_form_close_to_the_oracle(cuda):
    c = inputs.scaled("cfg1", (97, 78), ns=60, Ma=0.8, Re=50.0, scheme=DENS)
    g32, o = make_gpu(c, precision="fp32", amplitude=2e-2), make_oracle(c, amplitude=2e-2)
    h32, _ = g32.step(20)
    ho = o.step(20)
    r, m, E, _ = g32.get_state()
    ro, mo, Eo, _ = o.get_state()
    assert rel_l2(to_np(m).reshape(2, -1) / to_np(r), mo / ro) < 1e-5
    assert rel_l2(to_np(E), Eo) < 1e-6
    assert rel_l2(to_np(h32)[:, [0, 3]], ho[:, [0, 3]]) < 1e-4


def test_density_failure_rolls_back(cuda):
    c = inputs.scaled("cfg1", (64, 48), ns=40, scheme=DENS, Ma=0.8)
    g = make_gpu(c)
    g.step(2)
    r, m, E, F = g.get_state()
    E = E.clone()
    E[700] = -1e30
    g.set_state(r, m, E, F, step=2)
    st, info = g.step_status(3)
    assert st == _lib.IBM_E_NONFINITE
    assert info["step"] == 2 and info["steps_done"] == 0
    _, _, E2, _ = g.get_state()
    assert torch.equal(E2, E)


def test_density_rejections(cuda):
    from paper_2301_09349_amd.solver import IBMSolver

    c = inputs.scaled("cfg1", (40, 32), ns=20, scheme=DENS, Ma=0.8)
    with pytest.raises(_lib.IBMError):
        IBMSolver(dict(c, diffusion=inputs.DIFF_IMPLICIT), "fp64", max_markers=20)
    with pytest.raises(_lib.IBMError):
        IBMSolver(dict(c, n_outer=2), "fp64", max_markers=20)
    s = make_gpu(c, tape_steps=2)
    with pytest.raises(_lib.IBMError):
        s.step(1, record=True)
    s.step(1)


def test_full_size_density_cylinder_1024_parity(cuda):
    # the bench's density-based 1024^2 workload at its full size
    c = inputs.case("cfg2a", Ma=0.8, scheme=DENS)
    g, o = make_gpu(c), make_oracle(c)
    hg, _ = g.step(3)
    ho = o.step(3)
    for k, v in state_errors(g, o).items():
        assert v < 1e-12, (k, v)
    assert rel_l2(to_np(hg), ho[:, :4]) < 1e-9


@pytest.mark.slow
def test_full_size_density_sphere_256_parity(cuda):
    # 256^3 cells, 3200 candidate markers, Ma 0.8: one step
    c = inputs.case("cfg3", Ma=0.8, scheme=DENS)
    g, o = make_gpu(c), make_oracle(c)
    hg, _ = g.step(1)
    ho = o.step(1)
    for k, v in state_errors(g, o).items():
        assert v < 1e-12, (k, v)
    assert rel_l2(to_np(hg), ho[:, :4]) < 1e-9


def test_supersonic_cylinder_parity(cuda):
    # the grid-convergence case of App. C on its coarsest grid: Ma 2.5, Re 250,
    # markers without heat exchange, supersonic inflow and outflow sides
    c = inputs.case("sup10")
    g, o = make_gpu(c), make_oracle(c)
    assert g.dt == o.dt
    hg, _ = g.step(60)
    ho = o.step(60)
    for k, v in state_errors(g, o).items():
        assert v < 1e-11, (k, v)
    hg = to_np(hg)
    assert rel_l2(hg[:, :3], ho[:, :3]) < 1e-9
    assert np.all(hg[:, 3] == 0.0)


def test_supersonic_sides_rejected_with_the_pressure_based_step(cuda):
    from paper_2301_09349_amd.solver import IBMSolver

    c = inputs.scaled("sup10", (48, 40), ns=0, scheme=inputs.SCHEME_PRESSURE)
    with pytest.raises(_lib.IBMError):
        IBMSolver(c, "fp64", max_markers=1)
