"""Gradients of wall-flux objectives with respect to the wall temperatures, by
the library's hand-written discrete adjoint (``ibm_adjoint_step``) and
checkpointing.

The objective is linear in the per-step wall totals of the forcing
(Sec. 2.2, Eq. (10) for the force and Eqs. (16)-(17) for the heat):
``J = sum_n out_bar[n] . (Fx, Fy, Fz, H)_n`` over ``n_steps`` steps from the
current state. Time-averaged drag and Nusselt number are such objectives: their
normalisations (``drag_scale``, ``nusselt_scale``) only scale ``out_bar``.
The forward pass stores the state every ``checkpoint`` steps and records its last
segment on the tape as it runs; the reverse pass walks that segment backwards at
once, then re-runs each earlier segment with the tape on and walks it backwards, so
device memory grows with ``checkpoint``, not with ``n_steps``. With a tape of all
the steps (``checkpoint >= n_steps`` and the solver's ``tape_steps`` as large: about
8 MB per step on a 512^2 FP32 grid, well within one GPU's HBM) nothing is re-run.
"""

from __future__ import annotations

import math

import numpy as np
import torch

from .solver import IBMSolver


def _state_vector(s: IBMSolver) -> torch.Tensor:
    r, m, e, F = s.get_state()
    return torch.cat([r, m.reshape(-1), e] + list(F)).clone()


def _set_state_vector(s: IBMSolver, v: torch.Tensor, step: int):
    N, dim = s.N, s.dim
    s.set_state(v[:N], v[N: (1 + dim) * N], v[(1 + dim) * N: (2 + dim) * N],
                v[(2 + dim) * N:], step=step)


def drag_scale(case, diameter: float = 1.0) -> float:
    """C_d = scale * F_x: 2 / (rho_inf U_inf^2 L) with L = D in 2D (per unit span)
    and the frontal area pi D^2 / 4 in 3D (rho_inf = |U_inf| = 1)."""
    L = diameter if int(case["dim"]) == 2 else math.pi * diameter ** 2 / 4.0
    return 2.0 / L


def nusselt_scale(case, diameter: float = 1.0, dT_ref=None) -> float:
    """Nu = scale * H: D / (A_body lambda_inf dT_ref), A_body = pi D (2D) or pi D^2
    (3D), lambda_inf = c_p mu_inf / Pr, dT_ref = T_w(base) - T_inf (a constant)."""
    gamma, Ma, Re, Pr = (float(case[k]) for k in ("gamma", "Ma", "Re", "Pr"))
    R = 1.0 / (gamma * Ma * Ma)
    cp = gamma * R / (gamma - 1.0)
    lam_inf = cp / (Re * Pr)
    area = math.pi * diameter if int(case["dim"]) == 2 else math.pi * diameter ** 2
    dT = float(case["Tw"]) - 1.0 if dT_ref is None else float(dT_ref)
    if dT == 0.0:
        raise ValueError("nusselt_scale: the reference temperature difference is zero")
    return diameter / (area * lam_inf * dT)


class Rollout:
    """``n_steps`` steps from the solver's current state, with checkpoints every
    ``checkpoint`` steps (the solver needs ``tape_steps >= checkpoint`` and
    markers at rest)."""

    def __init__(self, s: IBMSolver, n_steps: int, checkpoint: int = 50):
        if s.nc == 0:
            raise ValueError("Rollout: the solver has no markers")
        if n_steps < 1 or checkpoint < 1:
            raise ValueError("n_steps and checkpoint must be >= 1")
        self.s, self.n_steps, self.checkpoint = s, int(n_steps), int(checkpoint)
        self.segs = []
        self.final = None
        self.final_step = 0
        self.taped = None  # the segment the forward pass left on the tape

    def forward(self) -> torch.Tensor:
        """Runs the steps; returns the history [n_steps, 4] (Fx, Fy, Fz, H)."""
        s = self.s
        hist = torch.zeros((self.n_steps, 4), dtype=torch.float64, device=s.device)
        self.segs = []
        done = 0
        self.taped = None
        while done < self.n_steps:
            k = min(self.checkpoint, self.n_steps - done)
            ck = _state_vector(s)
            last = done + k == self.n_steps
            h, info = s.step(k, record=last)
            self.segs.append((done, k, ck, int(info["step"]) - k))
            if last:
                self.taped = len(self.segs) - 1
            hist[done: done + k] = h
            done += k
        self.final = _state_vector(s)
        self.final_step = int(info["step"])
        return hist

    def reverse(self, out_bar, state_bar_final=None, positions=False):
        """Returns (dJ/dT_w [n candidates], dJ/d(initial state)) for the per-step seeds
        ``out_bar`` ([n_steps, 4] or [4]), and dJ/dX [n candidates, dim] of the
        candidate marker positions as a third item with ``positions``; leaves the
        solver in the final state."""
        if self.final is None:
            raise RuntimeError("Rollout.reverse before forward")
        s = self.s
        ob = np.asarray(out_bar, dtype=np.float64)
        if ob.ndim == 1:
            ob = np.broadcast_to(ob, (self.n_steps, 4))
        if ob.shape != (self.n_steps, 4):
            raise ValueError("out_bar must be [4] or [n_steps, 4]")
        sb = torch.zeros(s.state_size, dtype=torch.float64, device=s.device)
        if state_bar_final is not None:
            sb.copy_(state_bar_final)
        sb2 = torch.empty_like(sb)
        Tw_bar = torch.zeros(s.nc, dtype=torch.float64, device=s.device)
        if positions:
            s.shape_gradient(None)  # the adjoint steps below accumulate from zero
        for idx in reversed(range(len(self.segs))):
            start, k, ck, st_step = self.segs[idx]
            # the last segment is still on the tape from the forward pass
            if idx != self.taped or s.tape_length() != k:
                _set_state_vector(s, ck, st_step)
                s.step(k, hist=False, record=True)
            self.taped = None
            for i in reversed(range(k)):
                s.adjoint_step(i, sb, sb2, ob[start + i], Tw_bar)
                sb, sb2 = sb2, sb
        _set_state_vector(s, self.final, self.final_step)
        if positions:
            X_bar = torch.zeros((s.nc, s.dim), dtype=torch.float64, device=s.device)
            s.shape_gradient(X_bar)
            return Tw_bar, sb, X_bar
        return Tw_bar, sb


def wall_temperature_gradient(s: IBMSolver, n_steps: int, out_bar, checkpoint: int = 50,
                              state_bar_final=None):
    """Returns (hist [n_steps, 4] float64 device tensor, dJ/dT_w [n candidates],
    dJ/d(initial state) [state_size]); the solver ends in the state after
    ``n_steps`` steps, as after ``s.step(n_steps)``."""
    r = Rollout(s, n_steps, checkpoint)
    hist = r.forward()
    Tw_bar, sb = r.reverse(out_bar, state_bar_final)
    return hist, Tw_bar, sb


def marker_position_gradient(s: IBMSolver, n_steps: int, out_bar, checkpoint: int = 50):
    """Returns (hist [n_steps, 4], dJ/dT_w [n candidates], dJ/dX [n candidates, dim])
    for J = sum_n out_bar[n] . (Fx, Fy, Fz, H)_n over ``n_steps`` steps: the
    sensitivity of the wall totals to the positions of the (resting) markers, with
    the check routine's choice and the support cells held fixed. The solver ends in
    the state after ``n_steps`` steps."""
    r = Rollout(s, n_steps, checkpoint)
    hist = r.forward()
    Tw_bar, _, X_bar = r.reverse(out_bar, positions=True)
    return hist, Tw_bar, X_bar


class IBMRollout(torch.autograd.Function):
    """(J_Nu, J_Cd) = time averages of the Nusselt number and the drag coefficient
    over ``n_steps`` steps from the solver's current state, as a function of the
    per-marker wall temperatures ``Tw`` [n candidates]; ``backward`` runs the
    checkpointed discrete adjoint. The solver ends in the final state of the
    rollout (also after backward)."""

    @staticmethod
    def forward(ctx, Tw, solver: IBMSolver, n_steps: int, checkpoint: int = 50):
        solver.set_wall_temperature(Tw.detach().to(torch.float64))
        roll = Rollout(solver, n_steps, checkpoint)
        hist = roll.forward()
        ku, kd = nusselt_scale(solver.case), drag_scale(solver.case)
        J_nu = ku * hist[:, 3].mean()
        J_cd = kd * hist[:, 0].mean()
        ctx.roll, ctx.ku, ctx.kd, ctx.dtype = roll, ku, kd, Tw.dtype
        return J_nu.to(Tw.dtype), J_cd.to(Tw.dtype)

    @staticmethod
    def backward(ctx, g_nu, g_cd):
        roll = ctx.roll
        n = roll.n_steps
        ob = np.zeros((n, 4))
        gn = 0.0 if g_nu is None else float(g_nu)
        gc = 0.0 if g_cd is None else float(g_cd)
        ob[:, 3] = gn * ctx.ku / n
        ob[:, 0] = gc * ctx.kd / n
        Tw_bar, _ = roll.reverse(ob)
        return Tw_bar.to(ctx.dtype), None, None, None
