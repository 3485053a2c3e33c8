"""Gradients of wall-flux objectives with respect to the wall temperatures, by
the library's hand-written discrete adjoint (``ibm_adjoint_step``) and
checkpointing.

The objective is linear in the per-step wall totals of the forcing
(Sec. 2.2, Eq. (10) for the force and Eqs. (16)-(17) for the heat):
``J = sum_n out_bar[n] . (Fx, Fy, Fz, H)_n`` over ``n_steps`` steps from the
current state; time-averaged drag and Nusselt number are such objectives (their
normalisations only scale ``out_bar``). The forward pass stores the state every
``checkpoint`` steps; the reverse pass re-runs each segment with the tape on and
walks it backwards, so device memory grows with ``checkpoint``, not with
``n_steps``.
"""

from __future__ import annotations

import numpy as np
import torch

from .solver import IBMSolver


def _state_vector(s: IBMSolver) -> torch.Tensor:
    r, m, e, F = s.get_state()
    return torch.cat([r, m.reshape(-1), e] + list(F)).clone()


def _set_state_vector(s: IBMSolver, v: torch.Tensor, step: int):
    N, dim = s.N, s.dim
    r = v[:N]
    m = v[N: (1 + dim) * N]
    e = v[(1 + dim) * N: (2 + dim) * N]
    F = v[(2 + dim) * N:]
    s.set_state(r, m, e, F, step=step)


def wall_temperature_gradient(s: IBMSolver, n_steps: int, out_bar, checkpoint: int = 50,
                              state_bar_final=None):
    """Returns (hist [n_steps, 4] float64 device tensor, dJ/dT_w [n candidates],
    dJ/d(initial state) [state_size]); the solver ends in the state after
    ``n_steps`` steps, as after ``s.step(n_steps)``.

    ``out_bar`` is [n_steps, 4] (or [4], the same every step); ``s`` must have been
    created with ``tape_steps >= checkpoint`` (FP64, linear convection, markers at
    rest). ``state_bar_final`` optionally seeds the final state."""
    if s.nc == 0:
        raise ValueError("wall_temperature_gradient: the solver has no markers")
    if n_steps < 1 or checkpoint < 1:
        raise ValueError("n_steps and checkpoint must be >= 1")
    ob = np.asarray(out_bar, dtype=np.float64)
    if ob.ndim == 1:
        ob = np.broadcast_to(ob, (n_steps, 4))
    if ob.shape != (n_steps, 4):
        raise ValueError("out_bar must be [4] or [n_steps, 4]")
    dev = s.device
    # forward: checkpoints at the segment starts
    segs = []
    hist = torch.zeros((n_steps, 4), dtype=torch.float64, device=dev)
    done = 0
    while done < n_steps:
        k = min(checkpoint, n_steps - done)
        ck = _state_vector(s)
        h, info = s.step(k)
        segs.append((done, k, ck, int(info["step"]) - k))
        hist[done: done + k] = h
        done += k
    final = _state_vector(s)
    final_step = int(info["step"])
    # reverse
    sb = torch.zeros(s.state_size, dtype=torch.float64, device=dev)
    if state_bar_final is not None:
        sb.copy_(state_bar_final)
    sb2 = torch.empty_like(sb)
    Tw_bar = torch.zeros(s.nc, dtype=torch.float64, device=dev)
    for start, k, ck, st_step in reversed(segs):
        _set_state_vector(s, ck, st_step)
        s.step(k, hist=False, record=True)
        for i in reversed(range(k)):
            s.adjoint_step(i, sb, sb2, ob[start + i], Tw_bar)
            sb, sb2 = sb2, sb
    _set_state_vector(s, final, final_step)
    return hist, Tw_bar, sb
