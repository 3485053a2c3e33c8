"""GPU parity of the implicit (backward-Euler) compact viscous and conductive
fluxes against the oracle's implicit step on the same seeded inputs: the face
viscosities, the dim + 1 diffusion solves (to cg_rtol, from u^n and theta^n),
and everything downstream. The solves are well conditioned (rho* plus a
diffusion term), so both sides' solutions agree to about cg_rtol; FP64 states
are held to 1e-11 per step and 1e-10 over tens of steps."""
import numpy as np
import pytest
import torch

from paper_2301_09349_amd import inputs
from helpers import make_gpu, make_oracle, rel_l2, state_errors, to_np

pytestmark = pytest.mark.gpu

IMP = inputs.DIFF_IMPLICIT
VL, LIN = inputs.CONV_VANLEER, inputs.CONV_LINEAR


@pytest.mark.parametrize("conv", [VL, LIN])
def test_implicit_one_step_substeps_parity(cuda, conv):
    # ragged grid with a body; Re = 20, so that the solves do real work
    c = inputs.scaled("cfg1", (97, 78), ns=60, Re=20.0, convection=conv, diffusion=IMP)
    g, o = make_gpu(c, amplitude=5e-2), make_oracle(c, amplitude=5e-2)
    assert g.dt == o.dt  # the step follows convection alone, on both sides
    hg, _ = g.step(1)
    ho = o.step(1)
    assert rel_l2(to_np(g.field("rho_s")), o.intermediate("rho_s")) < 1e-14
    assert rel_l2(to_np(g.field("mom_ss")), o.intermediate("mom_ss")) < 1e-11
    assert rel_l2(to_np(g.field("E_ss")), o.intermediate("E_ss")) < 1e-12
    assert rel_l2(to_np(g.field("psi")), o.intermediate("psi")) < 1e-12
    assert rel_l2(to_np(g.field("pres")), o.intermediate("pres")) < 1e-10
    assert rel_l2(to_np(hg), ho[:, :4]) < 1e-9
    for k, v in state_errors(g, o).items():
        assert v < 1e-11, (k, v)


def test_implicit_cylinder_128_parity(cuda):
    c = inputs.case("cfg1", diffusion=IMP)
    g, o = make_gpu(c), make_oracle(c)
    hg, info = g.step(40)
    ho = o.step(40)
    for k, v in state_errors(g, o).items():
        assert v < 1e-10, (k, v)
    assert rel_l2(to_np(hg), ho[:, :4]) < 1e-8
    assert abs(info["mass"] - ho[-1, 4]) < 1e-12 * ho[-1, 4]


def test_implicit_sphere_3d_parity(cuda):
    c = inputs.scaled("cfg3", (40, 34, 30), ns=300, Re=30.0, diffusion=IMP)
    g, o = make_gpu(c, amplitude=2e-2), make_oracle(c, amplitude=2e-2)
    hg, _ = g.step(3)
    ho = o.step(3)
    for k, v in state_errors(g, o).items():
        assert v < 1e-11, (k, v)
    assert rel_l2(to_np(hg), ho[:, :4]) < 1e-9


def test_implicit_periodic_box_sutherland_parity(cuda):
    # every direction periodic (no boundary rule in the operator), Sutherland's law
    c = inputs.scaled("cfg1", (70, 37), ns=0, Re=10.0,
                      bc=[[inputs.PERIODIC] * 2, [inputs.PERIODIC] * 2], diffusion=IMP,
                      U_inf=(0.3, 0.1, 0.0))
    g, o = make_gpu(c, amplitude=5e-2), make_oracle(c, amplitude=5e-2)
    g.step(5)
    o.step(5)
    # the slow stream gives a long step (an acoustic CFL number near 10): the
    # pressure operator's condition number grows with its square, and both sides
    # stop their CG at rtol
    for k, v in state_errors(g, o).items():
        assert v < 1e-10, (k, v)


def test_implicit_moving_body_parity(cuda):
    c = inputs.scaled("osc2", (96, 96), ns=80, diffusion=IMP, scheme=inputs.SCHEME_PRESSURE)
    g, o = make_gpu(c), make_oracle(c)
    hg, _ = g.step(6)
    ho = o.step(6)
    for k, v in state_errors(g, o).items():
        assert v < 1e-11, (k, v)
    assert rel_l2(to_np(hg), ho[:, :4]) < 1e-8


def test_implicit_step_beyond_the_explicit_limit(cuda):
    # Re = 2: the explicit step is limited by diffusion; the implicit one follows
    # convection alone, several times longer, and matches the oracle over 20 steps
    c_exp = inputs.scaled("cfg1", (64, 48), ns=40, Re=2.0)
    c_imp = dict(c_exp, diffusion=IMP)
    dt_exp = make_gpu(c_exp).dt
    g, o = make_gpu(c_imp), make_oracle(c_imp)
    assert g.dt > 4.0 * dt_exp, (g.dt, dt_exp)
    hg, _ = g.step(20)
    ho = o.step(20)
    assert np.all(np.isfinite(to_np(hg)))
    for k, v in state_errors(g, o).items():
        assert v < 1e-10, (k, v)
    assert rel_l2(to_np(hg), ho[:, :4]) < 1e-8


def test_implicit_fp32_form_close_to_fp64_oracle(cuda):
    c = inputs.case("cfg1", diffusion=IMP)
    g32, o = make_gpu(c, precision="fp32"), make_oracle(c)
    h32, _ = g32.step(40)
    ho = o.step(40)
    R = 1.0 / (1.4 * c["Ma"] ** 2)
    cv = R / 0.4
    r, m, E, _ = g32.get_state()
    ro, mo, Eo, _ = o.get_state()
    u32 = to_np(m) / to_np(r)
    u64 = mo / ro
    t32 = to_np(E) / (to_np(r) * cv)
    t64 = Eo / (ro * cv)
    assert rel_l2(u32, u64) < 1e-4
    assert rel_l2(t32 - 1.0, t64 - 1.0) < 1e-3
    h32 = to_np(h32)
    assert abs(h32[:, 0].mean() - ho[:, 0].mean()) < 1e-4 * abs(ho[:, 0].mean())
    assert abs(h32[:, 3].mean() - ho[:, 3].mean()) < 1e-4 * abs(ho[:, 3].mean())


def test_implicit_profile_class_and_no_adjoint(cuda):
    from paper_2301_09349_amd._lib import IBMError

    c = inputs.scaled("cfg1", (40, 32), ns=20, convection=LIN, diffusion=IMP)
    s = make_gpu(c, tape_steps=2)
    s.profile(True)
    s.step(2, record=True)
    prof = s.profile_read()
    assert prof["diffusion"][1] == 2 and prof["diffusion"][0] > 0.0
    s.profile(False)
    sb = torch.zeros(s.state_size, dtype=torch.float64, device=s.device)
    sb2 = torch.zeros_like(sb)
    Twb = torch.zeros(s.nc, dtype=torch.float64, device=s.device)
    with pytest.raises(IBMError):
        s.adjoint_step(1, sb, sb2, np.zeros(4), Twb)


@pytest.mark.parametrize("variant", ["plain", "lds"])
@pytest.mark.parametrize("shape", [(133, 75), (36, 30, 26)])
def test_implicit_predictor_variants_parity(cuda, monkeypatch, variant, shape):
    # both predictor kernels leave out the compact diffusive fluxes alike
    monkeypatch.setenv("IBM_PREDICTOR", variant)
    name = "cfg1" if len(shape) == 2 else "cfg3"
    c = inputs.scaled(name, shape, ns=80 if len(shape) == 2 else 200, Re=20.0, diffusion=IMP)
    g, o = make_gpu(c, amplitude=2e-2), make_oracle(c, amplitude=2e-2)
    g.step(2)
    o.step(2)
    assert rel_l2(to_np(g.field("mom_ss")), o.intermediate("mom_ss")) < 1e-11
    assert rel_l2(to_np(g.field("E_ss")), o.intermediate("E_ss")) < 1e-12
    for k, v in state_errors(g, o).items():
        assert v < 1e-11, (k, v)


def test_implicit_start_does_not_change_the_solution(cuda, monkeypatch):
    # the diffusion solves start from the state at step n (IBM_CG_START=plain) or
    # from the extrapolation of the two previous steps' solutions: same states to
    # about rtol, and the extrapolated start needs fewer iterations
    c = inputs.case("cfg1", diffusion=IMP)
    runs = {}
    for mode in ("plain", None):
        if mode:
            monkeypatch.setenv("IBM_CG_START", mode)
        else:
            monkeypatch.delenv("IBM_CG_START", raising=False)
        g = make_gpu(c)
        g.step(5)
        _, info = g.step(20)
        runs[mode] = (g.get_state(), info["diff_iters_total"])
    (a, ia), (b, ib) = runs["plain"], runs[None]
    print(f"diffusion iterations over 20 steps: start from u^n {ia}, extrapolated {ib}")
    for x, y in zip(a[:3], b[:3]):
        assert rel_l2(to_np(y), to_np(x)) < 1e-11
    assert ib < ia


def test_full_size_implicit_cylinder_1024_parity(cuda):
    # the benchmark workload at its full size with the implicit terms
    c = inputs.case("cfg2a", diffusion=IMP)
    g, o = make_gpu(c), make_oracle(c)
    hg, _ = g.step(2)
    ho = o.step(2)
    for k, v in state_errors(g, o).items():
        assert v < 1e-11, (k, v)
    assert rel_l2(to_np(hg), ho[:, :4]) < 1e-9
