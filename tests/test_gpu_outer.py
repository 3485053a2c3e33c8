"""GPU parity of the outer passes (App. A step 3 repeated: the predictor at the
latest iterate with the step's start as old values, the first pass's marker
sources re-spread, the pressure solved again) against the oracle's, on the same
seeded inputs. FP64 states are held to 1e-11 over a few steps."""
import numpy as np
import pytest
import torch

from paper_2301_09349_amd import _lib, inputs
from helpers import make_gpu, make_oracle, rel_l2, state_errors, to_np

pytestmark = pytest.mark.gpu

IMP = inputs.DIFF_IMPLICIT
VL, LIN = inputs.CONV_VANLEER, inputs.CONV_LINEAR


@pytest.mark.parametrize("conv", [VL, LIN])
def test_outer_passes_parity_2d(cuda, conv):
    c = inputs.scaled("cfg1", (97, 78), ns=60, Re=20.0, convection=conv, n_outer=3)
    g, o = make_gpu(c, amplitude=5e-2), make_oracle(c, amplitude=5e-2)
    hg, info = g.step(4)
    ho = o.step(4)
    assert rel_l2(to_np(g.field("mom_ss")), o.intermediate("mom_ss")) < 1e-11
    assert rel_l2(to_np(g.field("pres")), o.intermediate("pres")) < 1e-10
    for k, v in state_errors(g, o).items():
        assert v < 1e-11, (k, v)
    assert rel_l2(to_np(hg), ho[:, :4]) < 1e-9
    assert info["cg_iters_total"] > info["cg_iters_last"] * 4  # every pass is counted


def test_one_pass_is_the_default_step(cuda):
    c = inputs.scaled("cfg1", (64, 48), ns=40)
    outs = []
    for over in ({}, {"n_outer": 1}):
        g = make_gpu(dict(c, **over))
        h, _ = g.step(3)
        outs.append([to_np(h)] + [to_np(x) for x in g.get_state()[:3]])
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


def test_outer_passes_sphere_3d_parity(cuda):
    c = inputs.scaled("cfg3", (36, 30, 28), ns=300, Re=30.0, n_outer=3)
    g, o = make_gpu(c, amplitude=2e-2), make_oracle(c, amplitude=2e-2)
    hg, _ = g.step(2)
    ho = o.step(2)
    for k, v in state_errors(g, o).items():
        assert v < 1e-11, (k, v)
    assert rel_l2(to_np(hg), ho[:, :4]) < 1e-9


def test_outer_passes_moving_body_parity(cuda):
    c = inputs.scaled("osc2", (96, 96), ns=80, n_outer=2, scheme=inputs.SCHEME_PRESSURE)
    g, o = make_gpu(c), make_oracle(c)
    hg, _ = g.step(4)
    ho = o.step(4)
    for k, v in state_errors(g, o).items():
        assert v < 1e-11, (k, v)
    assert rel_l2(to_np(hg), ho[:, :4]) < 1e-8


def test_outer_passes_with_implicit_diffusion_parity(cuda):
    c = inputs.scaled("cfg1", (97, 78), ns=60, Re=20.0, diffusion=IMP, n_outer=3)
    g, o = make_gpu(c, amplitude=2e-2), make_oracle(c, amplitude=2e-2)
    hg, _ = g.step(4)
    ho = o.step(4)
    for k, v in state_errors(g, o).items():
        assert v < 1e-11, (k, v)
    assert rel_l2(to_np(hg), ho[:, :4]) < 1e-9


@pytest.mark.parametrize("variant", ["plain", "lds"])
def test_outer_passes_predictor_variants_parity(cuda, monkeypatch, variant):
    monkeypatch.setenv("IBM_PREDICTOR", variant)
    c = inputs.scaled("cfg1", (133, 75), ns=80, Re=20.0, n_outer=2)
    g, o = make_gpu(c, amplitude=2e-2), make_oracle(c, amplitude=2e-2)
    g.step(2)
    o.step(2)
    for k, v in state_errors(g, o).items():
        assert v < 1e-11, (k, v)


@pytest.mark.parametrize("solve", ["fp64_cg", "refine"])
def test_outer_passes_fp32_form(cuda, monkeypatch, solve):
    c = inputs.scaled("cfg1", (97, 78), ns=60, Re=20.0, n_outer=3)
    monkeypatch.setenv("IBM_FP32_SOLVE", "refine" if solve == "refine" else "fp64")
    g32 = make_gpu(c, precision="fp32", amplitude=2e-2)
    monkeypatch.delenv("IBM_FP32_SOLVE", raising=False)
    o = make_oracle(c, amplitude=2e-2)
    h32, _ = g32.step(10)
    ho = o.step(10)
    r, m, E, _ = g32.get_state()
    ro, mo, Eo, _ = o.get_state()
    assert rel_l2(to_np(m) / to_np(r), mo / ro) < 1e-5
    assert rel_l2(to_np(E), Eo) < 1e-6
    assert rel_l2(to_np(h32)[:, [0, 3]], ho[:, [0, 3]]) < 1e-4


def test_outer_passes_failure_rolls_back_to_the_step_start(cuda):
    c = inputs.scaled("cfg1", (64, 48), ns=40, n_outer=3)
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


def test_outer_passes_have_no_adjoint(cuda):
    c = inputs.scaled("cfg1", (40, 32), ns=20, convection=LIN, n_outer=2)
    s = make_gpu(c, tape_steps=2)
    s.step(2, record=True)
    sb = torch.zeros(s.state_size, dtype=torch.float64, device=s.device)
    sb2 = torch.zeros_like(sb)
    Twb = torch.zeros(s.nc, dtype=torch.float64, device=s.device)
    with pytest.raises(_lib.IBMError):
        s.adjoint_step(1, sb, sb2, np.zeros(4), Twb)


def test_full_size_outer_passes_cylinder_1024_parity(cuda):
    # the benchmark workload at its full size, three passes at CFL 0.25 (as the bench)
    c = inputs.case("cfg2a", n_outer=3, cfl=0.25)
    g, o = make_gpu(c), make_oracle(c)
    hg, _ = g.step(2)
    ho = o.step(2)
    for k, v in state_errors(g, o).items():
        assert v < 1e-11, (k, v)
    assert rel_l2(to_np(hg), ho[:, :4]) < 1e-9
