"""GPU tests of the hand-written discrete adjoint (ibm_adjoint_step) through the C
ABI: one step against central finite differences of the GPU's own forward step,
per input block of the state (so that a wrong transpose names its block), and the
checkpointed gradient with respect to the wall temperatures against the FP64
oracle's tangent-linear (dual-number) run and against central finite differences.

With van Leer convection the adjoint keeps the branches the forward took (upwind
side by the sign of the face mass flux, limiter on or off): the derivative almost
everywhere, which the oracle's dual numbers compute too. Central differences agree
with it only where the step does not cross a branch, so those cases use noisy
states, a small step, and no flux perturbation on faces whose flux is exactly zero
(slip walls, where the upwind choice sits on its switch)."""
import numpy as np
import pytest
import torch

from paper_2301_09349_amd import inputs
from paper_2301_09349_amd.adjoint import IBMRollout, drag_scale, nusselt_scale, \
    marker_position_gradient, wall_temperature_gradient, _state_vector, _set_state_vector
from helpers import make_gpu, make_oracle, rel_l2, to_np

pytestmark = pytest.mark.gpu

LIN = inputs.CONV_LINEAR
VL = inputs.CONV_VANLEER


def _blocks(s):
    N, dim = s.N, s.dim
    b = {"rho": (0, N)}
    for q in range(dim):
        b[f"mom{q}"] = ((1 + q) * N, (2 + q) * N)
    b["E"] = ((1 + dim) * N, (2 + dim) * N)
    off = (2 + dim) * N
    for d in range(dim):
        b[f"F{d}"] = (off, off + s.NF[d])
        off += s.NF[d]
    return b


def _J(s, x, step0, w, ob):
    _set_state_vector(s, x, step0)
    h, _ = s.step(1)
    y = _state_vector(s)
    return float(torch.dot(w, y)) + float(np.dot(ob, to_np(h[0])))


def _single_step_case(c, amplitude, warm, seed, h=1e-5, with_w=True, skip_zero_flux=False,
                      thermal=0.0):
    s = make_gpu(c, amplitude=amplitude, tape_steps=1)
    if warm:
        s.step(warm)
    x0 = _state_vector(s)
    _, info = s.step(0)
    step0 = int(info["step"])
    gen = np.random.default_rng(seed)
    if thermal > 0.0:
        # relative noise on rho and E, so that no theta difference is near zero
        N, dim = s.N, s.dim
        for a, b in ((0, N), ((1 + dim) * N, (2 + dim) * N)):
            xi = torch.as_tensor(gen.uniform(-1.0, 1.0, b - a), device=s.device)
            x0[a:b] *= 1.0 + thermal * xi
    n = s.state_size
    w = torch.as_tensor(gen.standard_normal(n) if with_w else np.zeros(n), device=s.device)
    ob = gen.standard_normal(4) * 1e-2
    # adjoint of the step from x0
    _set_state_vector(s, x0, step0)
    s.step(1, hist=False, record=True)
    sb = torch.empty_like(w)
    Twb = torch.zeros(max(s.nc, 1), dtype=torch.float64, device=s.device)
    s.adjoint_step(0, w, sb, ob, Twb)
    out = {}
    for name, (a, b) in _blocks(s).items():
        v = torch.zeros(n, dtype=torch.float64, device=s.device)
        v[a:b] = torch.as_tensor(gen.standard_normal(b - a), device=s.device)
        if skip_zero_flux and name.startswith("F"):
            v[a:b] = torch.where(x0[a:b] == 0.0, torch.zeros_like(v[a:b]), v[a:b])
        ad = float(torch.dot(sb, v))
        ident = float(torch.dot(w, v)) if (name == "rho" or name.startswith("mom")) else 0.0
        fd = (_J(s, x0 + h * v, step0, w, ob) - _J(s, x0 - h * v, step0, w, ob)) / (2 * h)
        out[name] = (fd, ad, ident)
    return out


def _check(out, tol):
    bad = {}
    for name, (fd, ad, ident) in out.items():
        scale = max(abs(ad - ident), 1e-300)
        rel = abs(fd - ad) / scale
        if not rel < tol:
            bad[name] = (fd, ad, ident, rel)
    assert not bad, bad


@pytest.mark.parametrize("with_w", [True, False])
def test_adjoint_step_channel_with_body(cuda, with_w):
    # inflow / outflow / slip, ragged grid, markers
    c = inputs.scaled("cfg1", (70, 52), ns=60, convection=LIN, Re=20.0)
    _check(_single_step_case(c, 1e-2, 3, 11, with_w=with_w), 1e-6)


def test_adjoint_step_periodic_no_body(cuda):
    c = inputs.scaled("cfg1", (40, 30), ns=0, convection=LIN,
                      bc=[[inputs.PERIODIC] * 2, [inputs.PERIODIC] * 2])
    _check(_single_step_case(c, 5e-2, 2, 12), 1e-6)


def test_adjoint_step_constant_viscosity(cuda):
    c = inputs.scaled("cfg1", (48, 40), ns=40, convection=LIN,
                      viscosity_law=inputs.MU_CONSTANT)
    _check(_single_step_case(c, 1e-2, 2, 13), 1e-6)


def test_adjoint_step_sphere_3d(cuda):
    c = inputs.scaled("cfg3", (26, 20, 18), ns=120, convection=LIN, Re=50.0)
    _check(_single_step_case(c, 1e-2, 2, 14), 1e-6)


def _single_step_tl(c, warm, seed, thermal=2e-2, amplitude=5e-2):
    """One step's adjoint, per input block of the state, against the oracle's
    tangent-linear step from the same state (exact derivatives on both sides; they
    differ by the two pressure solves' truncation at rtol 1e-13, measured up to
    1e-9 relative on blocks with small derivatives)."""
    s = make_gpu(c, amplitude=amplitude, tape_steps=1)
    if warm:
        s.step(warm)
    x0 = _state_vector(s)
    _, info = s.step(0)
    step0 = int(info["step"])
    gen = np.random.default_rng(seed)
    N, dim = s.N, s.dim
    for a, b in ((0, N), ((1 + dim) * N, (2 + dim) * N)):
        xi = torch.as_tensor(gen.uniform(-1.0, 1.0, b - a), device=s.device)
        x0[a:b] *= 1.0 + thermal * xi
    n = s.state_size
    w = gen.standard_normal(n)
    ob = gen.standard_normal(4) * 1e-2
    _set_state_vector(s, x0, step0)
    s.step(1, hist=False, record=True)
    sb = torch.empty(n, dtype=torch.float64, device=s.device)
    Twb = torch.zeros(max(s.nc, 1), dtype=torch.float64, device=s.device)
    s.adjoint_step(0, torch.as_tensor(w, device=s.device), sb, ob, Twb)
    sb = to_np(sb)
    o = make_oracle(c, amplitude=amplitude)
    xs = to_np(x0)
    _set_oracle_state(o, xs, step0)
    out = {}
    for name, (a, b) in _blocks(s).items():
        v = np.zeros(n)
        v[a:b] = gen.standard_normal(b - a)
        _, hd, dout = o.tangent_linear_state(1, v)
        tl = float(w @ dout) + float(ob @ hd[0])
        ident = float(w @ v) if (name == "rho" or name.startswith("mom")) else 0.0
        out[name] = (tl, float(sb @ v), ident)
    return out


def _set_oracle_state(o, x, step):
    N, dim = o.N, o.dim
    F, off = [], (2 + dim) * N
    for d in range(dim):
        F.append(x[off: off + o.NF[d]])
        off += o.NF[d]
    o.set_state(x[:N], x[N:(1 + dim) * N].reshape(dim, N), x[(1 + dim) * N:(2 + dim) * N], F,
                step=step)


def test_adjoint_step_vanleer_channel_with_body(cuda):
    # van Leer convection: inflow / outflow / slip, markers; the far-upwind cell of a
    # boundary face is the second ghost layer
    c = inputs.scaled("cfg1", (70, 52), ns=60, convection=VL, Re=20.0)
    _check(_single_step_tl(c, 3, 31), 1e-8)


def test_adjoint_step_vanleer_periodic(cuda):
    c = inputs.scaled("cfg1", (40, 30), ns=0, convection=VL,
                      bc=[[inputs.PERIODIC] * 2, [inputs.PERIODIC] * 2])
    _check(_single_step_tl(c, 2, 32), 1e-8)


def test_adjoint_step_vanleer_sphere_3d(cuda):
    c = inputs.scaled("cfg3", (26, 20, 18), ns=120, convection=VL, Re=50.0)
    _check(_single_step_tl(c, 2, 33), 1e-8)


def test_adjoint_step_vanleer_small_grid(cuda):
    # n = 3 in one direction: a cell has up to two ghost images per side
    c = inputs.scaled("cfg1", (24, 3), ns=0, convection=VL,
                      bc=[[inputs.INFLOW, inputs.OUTFLOW], [inputs.SLIP] * 2])
    _check(_single_step_tl(c, 1, 34), 1e-8)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_tw_gradient_vanleer_matches_oracle_tangent_linear(cuda, prec):
    c = inputs.scaled("cfg5", (96, 96), ns=60, convection=VL)
    nsteps, ck = 12, 5
    ob = np.random.default_rng(35).standard_normal((nsteps, 4))
    s = make_gpu(c, precision=prec, tape_steps=ck)
    _, Twb, _ = wall_temperature_gradient(s, nsteps, ob, checkpoint=ck)
    Twb = to_np(Twb)
    o = make_oracle(c)
    # FP64: the same derivative to rounding; FP32 form: the derivative along the
    # FP32 trajectory
    tol = 1e-10 if prec == "fp64" else 1e-4
    for j in range(3):
        d = inputs.normal(1000 + j, c["ns"])
        d = d / np.linalg.norm(d)
        _, hd = o.tangent_linear(nsteps, d)
        tl = float(np.sum(ob * hd))
        ad = float(Twb @ d)
        assert abs(ad - tl) <= tol * abs(tl), (j, ad, tl)


def test_tw_gradient_vanleer_central_differences(cuda):
    c = inputs.scaled("cfg5", (96, 96), ns=60, convection=VL)
    nsteps, ck = 10, 4
    ob = np.random.default_rng(36).standard_normal((nsteps, 4))
    s = make_gpu(c, tape_steps=ck)
    x0 = _state_vector(s)
    _, Twb, _ = wall_temperature_gradient(s, nsteps, ob, checkpoint=ck)
    Twb = to_np(Twb)
    Tw0 = np.full(c["ns"], float(c["Tw"]))
    h = 1e-6
    for j in range(3):
        d = inputs.normal(1000 + j, c["ns"])
        d = d / np.linalg.norm(d)
        Js = []
        for sgn in (1.0, -1.0):
            _set_state_vector(s, x0, 0)
            s.set_wall_temperature(Tw0 + sgn * h * d)
            hh, _ = s.step(nsteps)
            Js.append(float(np.sum(ob * to_np(hh))))
        s.set_wall_temperature(Tw0)
        fd = (Js[0] - Js[1]) / (2 * h)
        ad = float(Twb @ d)
        assert abs(ad - fd) <= 1e-5 * abs(ad), (j, ad, fd)


def _tw_case():
    # the gradient workload's physics on a small grid
    return inputs.scaled("cfg5", (96, 96), ns=60, convection=LIN)


def test_tw_gradient_matches_oracle_tangent_linear(cuda):
    c = _tw_case()
    nsteps, ck = 12, 5
    gen = np.random.default_rng(21)
    ob = gen.standard_normal((nsteps, 4))
    s = make_gpu(c, tape_steps=ck)
    hist, Twb, _ = wall_temperature_gradient(s, nsteps, ob, checkpoint=ck)
    Twb = to_np(Twb)
    o = make_oracle(c)
    for j in range(3):
        d = inputs.normal(1000 + j, c["ns"])
        d = d / np.linalg.norm(d)
        hv, hd = o.tangent_linear(nsteps, d)
        tl = float(np.sum(ob * hd))
        ad = float(Twb @ d)
        assert abs(ad - tl) <= 1e-10 * abs(tl), (j, ad, tl)
        # the forward history agrees with the oracle's values as well
        assert np.max(np.abs(to_np(hist) - hv)) <= 1e-10 * np.max(np.abs(hv))


def test_tw_gradient_matches_central_differences(cuda):
    c = _tw_case()
    nsteps, ck = 10, 4
    gen = np.random.default_rng(22)
    ob = gen.standard_normal((nsteps, 4))
    s = make_gpu(c, tape_steps=ck)
    x0 = _state_vector(s)
    _, Twb, _ = wall_temperature_gradient(s, nsteps, ob, checkpoint=ck)
    Twb = to_np(Twb)
    Tw0 = np.full(c["ns"], float(c["Tw"]))
    h = 1e-6
    for j in range(3):
        d = inputs.normal(1000 + j, c["ns"])
        d = d / np.linalg.norm(d)
        Js = []
        for sgn in (1.0, -1.0):
            _set_state_vector(s, x0, 0)
            s.set_wall_temperature(Tw0 + sgn * h * d)
            hh, _ = s.step(nsteps)
            Js.append(float(np.sum(ob * to_np(hh))))
        s.set_wall_temperature(Tw0)
        fd = (Js[0] - Js[1]) / (2 * h)
        ad = float(Twb @ d)
        assert abs(ad - fd) <= 1e-5 * abs(ad), (j, ad, fd)


def test_fp32_form_gradient_close_to_fp64(cuda):
    # FP32 trajectory and record, reverse in FP64: the T_w gradient of the FP32 form
    # against the FP64 one (measured ~5e-8 here, ~3e-7 at 512^2 over 500 steps)
    c = _tw_case()
    nsteps, ck = 12, 5
    ob = np.random.default_rng(23).standard_normal((nsteps, 4))
    g = {}
    for prec in ("fp64", "fp32"):
        s = make_gpu(c, precision=prec, tape_steps=ck)
        _, tb, _ = wall_temperature_gradient(s, nsteps, ob, checkpoint=ck)
        g[prec] = to_np(tb)
    assert rel_l2(g["fp32"], g["fp64"]) < 1e-5


def test_gradient_rollout_leaves_the_forward_state(cuda):
    c = _tw_case()
    s1 = make_gpu(c, tape_steps=4)
    s2 = make_gpu(c)
    wall_temperature_gradient(s1, 9, np.ones(4), checkpoint=4)
    s2.step(9)
    a, b = _state_vector(s1), _state_vector(s2)
    assert torch.equal(a, b)


def test_autograd_function_matches_the_driver(cuda):
    c = _tw_case()
    n, ck = 9, 4
    s = make_gpu(c, tape_steps=ck)
    Tw = torch.full((c["ns"],), float(c["Tw"]), dtype=torch.float64, device=s.device,
                    requires_grad=True)
    Jn, Jc = IBMRollout.apply(Tw, s, n, ck)
    (0.7 * Jn + 0.3 * Jc).backward()
    s2 = make_gpu(c, tape_steps=ck)
    ob = np.zeros((n, 4))
    ob[:, 3] = 0.7 * nusselt_scale(c) / n
    ob[:, 0] = 0.3 * drag_scale(c) / n
    hist, Twb, _ = wall_temperature_gradient(s2, n, ob, checkpoint=ck)
    assert float(Jn.detach()) == pytest.approx(nusselt_scale(c) * float(hist[:, 3].mean()),
                                               rel=1e-14)
    assert float(Jc.detach()) == pytest.approx(drag_scale(c) * float(hist[:, 0].mean()),
                                               rel=1e-14)
    assert torch.allclose(Tw.grad, Twb, rtol=1e-13, atol=0.0)
    assert float(Jn.detach()) > 0.0  # the wall is hotter than the stream


@pytest.mark.parametrize("conv", [LIN, VL], ids=["linear", "vanleer"])
def test_cfg5_nusselt_gradient_full_size(cuda, conv):
    """The gradient workload at full size: 512^2, 200 markers, T_w = 1.3, time-averaged
    Nusselt number over 500 steps, checkpoints every 50; central differences on 10
    seeded unit directions, and the oracle's tangent-linear over the first 10 steps.
    The step is 1e-6 with linear convection; with van Leer convection it is 1e-7: over
    500 steps the wake holds limiter branch points that a step of 1e-6 crosses
    (measured disagreement 4e-6..8e-5 at 1e-4..1e-6, 3e-8..1.4e-7 at 1e-7). Even at
    1e-7 a direction can cross one (2.2e-5 measured on one of ten), so with van Leer
    every direction must agree to 1e-4 and all but two to 1e-6; the exact check is
    the tangent-linear one. The + and - runs of every direction take the same number
    of CG iterations (printed; 5347 each with van Leer), so the outlier is not a
    difference in the pressure solves' truncation."""
    c = inputs.case("cfg5", convection=conv)
    n, ck = int(c["steps"]), int(c["checkpoint"])
    s = make_gpu(c, tape_steps=ck)
    x0 = _state_vector(s)
    Tw0 = torch.full((c["ns"],), float(c["Tw"]), dtype=torch.float64, device=s.device)
    Tw = Tw0.clone().requires_grad_(True)
    Jn, _ = IBMRollout.apply(Tw, s, n, ck)
    Jn.backward()
    g = to_np(Tw.grad)
    # the FP32 form's gradient (FP32 trajectory, FP64 reverse) against it
    s32 = make_gpu(c, precision="fp32", tape_steps=ck)
    Tw32 = Tw0.clone().requires_grad_(True)
    Jn32, _ = IBMRollout.apply(Tw32, s32, n, ck)
    Jn32.backward()
    e32 = rel_l2(to_np(Tw32.grad), g)
    print(f"\nfull-size gradient, convection {conv}: FP32 form vs FP64 rel L2 {e32:.2e}")
    # linear: ~3e-7 measured; van Leer: 1.5e-5 measured -- the limiter's weights
    # (a^2 / (a + b)^2 and the like) move more under the FP32 trajectory's rounding
    # where a + b is small than the linear scheme's constant halves
    assert e32 < (1e-5 if conv == LIN else 1e-4)
    assert abs(float(Jn32.detach()) / float(Jn.detach()) - 1.0) < 1e-4
    del s32
    ku = nusselt_scale(c)
    h = 1e-6 if conv == LIN else 1e-7
    errs = []
    for j in range(10):
        d = inputs.normal(1000 + j, c["ns"])
        d = d / np.linalg.norm(d)
        Js, its = [], []
        for sgn in (1.0, -1.0):
            _set_state_vector(s, x0, 0)
            s.set_wall_temperature(Tw0 + sgn * h * torch.as_tensor(d, device=s.device))
            hh, info = s.step(n)
            Js.append(ku * float(hh[:, 3].mean()))
            its.append(info["cg_iters_total"])
        fd = (Js[0] - Js[1]) / (2 * h)
        ad = float(g @ d)
        errs.append(abs(ad - fd) / abs(ad))
        # the pressure solves of the two runs take the same number of iterations or not
        # (a different count leaves a different truncation in J(+) - J(-))
        print(f"  direction {j}: adjoint {ad:.10e} central difference {fd:.10e} "
              f"rel {errs[-1]:.1e}, CG iterations {its[0]} / {its[1]}")
    if conv == LIN:
        assert max(errs) <= 1e-5, errs
    else:
        assert max(errs) <= 1e-4 and sorted(errs)[-3] <= 1e-6, errs
    # oracle tangent-linear over the first steps
    m = 10
    _set_state_vector(s, x0, 0)
    s.set_wall_temperature(Tw0)
    ob = np.zeros((m, 4))
    ob[:, 3] = 1.0
    _, Twb, _ = wall_temperature_gradient(s, m, ob, checkpoint=5)
    o = make_oracle(c)
    d = inputs.normal(1000, c["ns"])
    d = d / np.linalg.norm(d)
    _, hd = o.tangent_linear(m, d)
    tl = float(np.sum(hd[:, 3]))
    ad = float(to_np(Twb) @ d)
    print(f"  oracle tangent-linear over {m} steps: rel {abs(ad - tl) / abs(tl):.1e}")
    assert abs(ad - tl) <= 1e-10 * abs(tl), (ad, tl)


@pytest.mark.slow
@pytest.mark.timeout(600)
def test_cfg5_vanleer_gradient_matches_oracle_tangent_100_steps(cuda):
    """The van Leer gradient at full size (512^2, 200 markers, T_w = 1.3) over 100 steps
    with checkpoints every 50, against the oracle's tangent-linear run along one seeded
    unit direction: exact derivatives on both sides, so they agree to the pressure
    solves' truncation wherever central differences would cross a limiter branch point
    (the evidence behind the central-difference tolerance of the 500-step test)."""
    c = inputs.case("cfg5", convection=VL)
    m, ck = 100, 50
    s = make_gpu(c, tape_steps=ck)
    ob = np.zeros((m, 4))
    ob[:, 3] = 1.0
    _, Twb, _ = wall_temperature_gradient(s, m, ob, checkpoint=ck)
    o = make_oracle(c)
    # the direction whose central difference at 1e-7 is the outlier of the 500-step test
    d = inputs.normal(1007, c["ns"])
    d = d / np.linalg.norm(d)
    _, hd = o.tangent_linear(m, d)
    tl = float(np.sum(hd[:, 3]))
    ad = float(to_np(Twb) @ d)
    print(f"\n  oracle tangent-linear over {m} steps: adjoint {ad:.15e} tangent {tl:.15e} "
          f"rel {abs(ad - tl) / abs(tl):.1e}")
    assert abs(ad - tl) <= 1e-9 * abs(tl), (ad, tl)


def _turned_ring(c, angle=0.1):
    # the workload's ring turned by `angle`: no candidate on a grid line and no two
    # mirror images across a symmetry line of a cell (exact ties of the check
    # routine), so that the markers in use and their supports are locally fixed
    X, Ud, Tw, dA = inputs.markers(c)
    cs, sn = np.cos(angle), np.sin(angle)
    if X.shape[1] == 2:
        X = np.stack([cs * X[:, 0] - sn * X[:, 1], sn * X[:, 0] + cs * X[:, 1]], axis=1)
    else:
        X = np.stack([cs * X[:, 0] - sn * X[:, 1], sn * X[:, 0] + cs * X[:, 1], X[:, 2]], axis=1)
    return X, Ud, Tw, dA


@pytest.mark.parametrize("conv", [LIN, VL], ids=["linear", "vanleer"])
def test_marker_position_gradient_matches_oracle(cuda, conv):
    # dJ/dX of the candidate positions (kernel weights, quadrature weights, the
    # adjoint Gram solve) against the oracle's tangent-linear run along dX
    c = inputs.scaled("cfg5", (64, 64), ns=40, convection=conv)
    X, Ud, Tw, dA = _turned_ring(c)
    nsteps, ck = 8, 3
    gen = np.random.default_rng(51)
    ob = gen.standard_normal((nsteps, 4))
    s = make_gpu(c, tape_steps=ck)
    s.set_markers(X, Ud, Tw, dA, dedupe=True)
    _, Twb, Xb = marker_position_gradient(s, nsteps, ob, checkpoint=ck)
    Xb = to_np(Xb)
    assert np.all(np.isfinite(Xb)) and np.abs(Xb).max() > 0.0
    o = make_oracle(c)
    o.set_markers(X, Ud, Tw, dA, dedupe=True)
    for j in range(3):
        dX = gen.standard_normal(X.shape)
        _, hd = o.tangent_linear_shape(nsteps, dX)
        tl = float(np.sum(ob * hd))
        ad = float(np.sum(Xb * dX))
        assert abs(ad - tl) <= 1e-8 * abs(tl), (j, ad, tl)
    # candidates the check routine leaves out get no gradient
    ids, _ = s.markers_in_use()
    out = np.setdiff1d(np.arange(c["ns"]), to_np(ids).astype(int))
    assert out.size > 0 and np.all(Xb[out] == 0.0)


def test_marker_position_gradient_sphere_3d(cuda):
    c = inputs.scaled("cfg3", (24, 20, 20), ns=150, convection=LIN, Re=50.0)
    X, Ud, Tw, dA = _turned_ring(c, 0.07)
    nsteps, ck = 4, 2
    gen = np.random.default_rng(52)
    ob = gen.standard_normal((nsteps, 4))
    s = make_gpu(c, tape_steps=ck)
    s.set_markers(X, Ud, Tw, dA, dedupe=True)
    _, _, Xb = marker_position_gradient(s, nsteps, ob, checkpoint=ck)
    Xb = to_np(Xb)
    o = make_oracle(c)
    o.set_markers(X, Ud, Tw, dA, dedupe=True)
    dX = gen.standard_normal(X.shape)
    _, hd = o.tangent_linear_shape(nsteps, dX)
    tl = float(np.sum(ob * hd))
    ad = float(np.sum(Xb * dX))
    assert abs(ad - tl) <= 1e-8 * abs(tl), (ad, tl)


def test_marker_position_gradient_fp32_form(cuda):
    # FP32 trajectory, FP64 reverse: close to the FP64 gradient
    c = inputs.scaled("cfg5", (64, 64), ns=40, convection=LIN)
    X, Ud, Tw, dA = _turned_ring(c)
    nsteps, ck = 8, 4
    ob = np.random.default_rng(54).standard_normal((nsteps, 4))
    g = {}
    for prec in ("fp64", "fp32"):
        s = make_gpu(c, precision=prec, tape_steps=ck)
        s.set_markers(X, Ud, Tw, dA, dedupe=True)
        _, _, Xb = marker_position_gradient(s, nsteps, ob, checkpoint=ck)
        g[prec] = to_np(Xb)
    assert rel_l2(g["fp32"], g["fp64"]) < 1e-4


def test_marker_position_gradient_central_differences(cuda):
    # against the GPU forward run with the positions moved by +-h dX
    c = inputs.scaled("cfg5", (64, 64), ns=40, convection=LIN)
    X, Ud, Tw, dA = _turned_ring(c)
    nsteps, ck = 6, 3
    gen = np.random.default_rng(53)
    ob = gen.standard_normal((nsteps, 4))
    s = make_gpu(c, tape_steps=ck)
    x0 = _state_vector(s)
    s.set_markers(X, Ud, Tw, dA, dedupe=True)
    _, _, Xb = marker_position_gradient(s, nsteps, ob, checkpoint=ck)
    Xb = to_np(Xb)
    h = 1e-6
    for j in range(2):
        dX = gen.standard_normal(X.shape)
        Js = []
        for sgn in (1.0, -1.0):
            s.set_markers(X + sgn * h * dX, Ud, Tw, dA, dedupe=True)
            _set_state_vector(s, x0, 0)
            hh, _ = s.step(nsteps)
            Js.append(float(np.sum(ob * to_np(hh))))
        fd = (Js[0] - Js[1]) / (2 * h)
        ad = float(np.sum(Xb * dX))
        assert abs(ad - fd) <= 1e-6 * abs(ad), (j, ad, fd)


def test_adjoint_rejects_bad_calls(cuda):
    from paper_2301_09349_amd._lib import IBMError

    c = inputs.scaled("cfg1", (40, 32), ns=20, convection=LIN)
    s = make_gpu(c, tape_steps=2)
    sb = torch.zeros(s.state_size, dtype=torch.float64, device=s.device)
    sb2 = torch.zeros_like(sb)
    Twb = torch.zeros(s.nc, dtype=torch.float64, device=s.device)
    with pytest.raises(IBMError):  # nothing recorded
        s.adjoint_step(0, sb, sb2, np.zeros(4), Twb)
    with pytest.raises(IBMError):  # more steps than the tape holds
        s.step(3, record=True)
    s.step(2, record=True)
    assert s.tape_length() == 2
    with pytest.raises(IBMError):
        s.adjoint_step(2, sb, sb2, np.zeros(4), Twb)
    with pytest.raises(IBMError):  # in place
        s.adjoint_step(0, sb, sb, np.zeros(4), Twb)
    s.adjoint_step(1, sb, sb2, np.zeros(4), Twb)
