"""Python face of the HIP library: one ``IBMSolver`` per grid, holding the device
workspace (a torch tensor) and the library context. Marshalling only."""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib as L


def make_desc(case, precision: str = "fp64", max_markers=None) -> L.ibm_grid_desc:
    d = L.ibm_grid_desc()
    dim = int(case["dim"])
    d.dim = dim
    n = list(case["n"]) + [1] * (3 - len(case["n"]))
    lo = list(case["lo"]) + [0.0] * (3 - len(case["lo"]))
    hi = list(case["hi"]) + [1.0] * (3 - len(case["hi"]))
    for a in range(3):
        d.n[a] = int(n[a]) if a < dim else 1
        d.lo[a] = float(lo[a])
        d.hi[a] = float(hi[a])
    for a in range(3):
        for s in range(2):
            d.bc[a][s] = int(case["bc"][a][s]) if a < dim else L.IBM_PERIODIC
    d.precision = L.IBM_FP32 if precision == "fp32" else L.IBM_FP64
    d.convection = int(case.get("convection", L.IBM_CONV_VANLEER))
    d.viscosity_law = int(case.get("viscosity_law", L.IBM_MU_SUTHERLAND))
    d.diffusion = int(case.get("diffusion", 0))
    d.n_outer = int(case.get("n_outer", 1))
    d.scheme = int(case.get("scheme", 0))
    d.Re = float(case["Re"])
    d.Ma = float(case["Ma"])
    d.Pr = float(case.get("Pr", 0.71))
    d.gamma = float(case.get("gamma", 1.4))
    d.sutherland_S = float(case.get("sutherland_S", 110.4 / 288.15))
    U = list(case.get("U_inf", (1.0, 0.0, 0.0))) + [0.0] * 3
    for a in range(3):
        d.U_inf[a] = float(U[a])
    d.dt = float(case.get("dt", 0.0))
    d.cfl = float(case.get("cfl", 0.5))
    d.dt_theta_max = float(case.get("dt_theta_max", 1.0))
    d.dt_u_max = float(case.get("dt_u_max", 0.0))
    d.cg_rtol = float(case.get("cg_rtol", 1e-13))
    d.cg_maxit = int(case.get("cg_maxit", 2000))
    d.max_markers = int(case.get("ns", 0) if max_markers is None else max_markers)
    return d


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(None)


class IBMSolver:
    """A grid, its state and its body on one GPU."""

    def __init__(self, case, precision: str = "fp64", max_markers=None, tape_steps: int = 0,
                 device="cuda", noalloc: bool = False):
        """``noalloc``: create the context with ibm_create_grid_noalloc (the library's
        fixed device array as workspace; no workspace tensor)."""
        self.lib = L.load()
        self.case = dict(case)
        self.precision = precision
        self.dtype = torch.float32 if precision == "fp32" else torch.float64
        self.device = torch.device(device)
        self.desc = make_desc(case, precision, max_markers)
        self.dim = int(case["dim"])
        self.n = [int(v) for v in case["n"]][: self.dim]
        self.N = int(np.prod(self.n))
        self.NF = []
        for d in range(self.dim):
            m = list(self.n)
            m[d] += 1
            self.NF.append(int(np.prod(m)))
        nbytes = self.lib.ibm_workspace_bytes(ctypes.byref(self.desc), self.desc.max_markers,
                                              int(tape_steps))
        if nbytes == 0:
            raise L.IBMError(L.IBM_E_ARG, "invalid grid description")
        self.ws_bytes = int(nbytes)
        self.stream = torch.cuda.current_stream(self.device)
        ctx = ctypes.c_void_p()
        if noalloc:
            self.ws = None
            st = L.load().ibm_create_grid_noalloc(ctypes.byref(self.desc), int(tape_steps),
                                                  ctypes.c_void_p(self.stream.cuda_stream),
                                                  ctypes.byref(ctx))
            L.check(st, None, "ibm_create_grid_noalloc")
        else:
            self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
            base = self.ws.data_ptr()
            self._ws_ptr = (base + 255) // 256 * 256
            st = L.load().ibm_create_grid(ctypes.byref(self.desc), ctypes.c_void_p(self._ws_ptr),
                                          self.ws_bytes, int(tape_steps),
                                          ctypes.c_void_p(self.stream.cuda_stream),
                                          ctypes.byref(ctx))
            L.check(st, None, "ibm_create_grid")
        self.ctx = ctx
        self.nc = 0

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.ibm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ state
    @property
    def dt(self) -> float:
        return self.lib.ibm_dt(self.ctx)

    def _dev(self, a, dtype=None):
        dtype = self.dtype if dtype is None else dtype
        if isinstance(a, torch.Tensor):
            return a.to(device=self.device, dtype=dtype).contiguous()
        return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=self.device)

    def init_primitive(self, rho, u, theta):
        r, uu, t = self._dev(rho).reshape(-1), self._dev(u).reshape(-1), self._dev(theta).reshape(-1)
        L.check(self.lib.ibm_init_primitive(self.ctx, _ptr(r), _ptr(uu), _ptr(t)), self.ctx,
                "ibm_init_primitive")

    def set_state(self, rho, mom, E, F=None, step: int = 0):
        r, m, e = self._dev(rho).reshape(-1), self._dev(mom).reshape(-1), self._dev(E).reshape(-1)
        f = None
        if F is not None:
            f = torch.cat([self._dev(x).reshape(-1) for x in F]) if isinstance(F, (list, tuple)) \
                else self._dev(F).reshape(-1)
        L.check(self.lib.ibm_set_state(self.ctx, _ptr(r), _ptr(m), _ptr(e), _ptr(f), int(step)),
                self.ctx, "ibm_set_state")

    def get_state(self):
        """Returns device tensors rho [N], mom [dim, N], E [N], F list of [NF_d]."""
        r = torch.empty(self.N, dtype=self.dtype, device=self.device)
        m = torch.empty(self.dim * self.N, dtype=self.dtype, device=self.device)
        e = torch.empty(self.N, dtype=self.dtype, device=self.device)
        f = torch.empty(sum(self.NF), dtype=self.dtype, device=self.device)
        L.check(self.lib.ibm_get_state(self.ctx, _ptr(r), _ptr(m), _ptr(e), _ptr(f)), self.ctx,
                "ibm_get_state")
        self.stream.synchronize()
        Fs, off = [], 0
        for d in range(self.dim):
            Fs.append(f[off: off + self.NF[d]])
            off += self.NF[d]
        return r, m.reshape(self.dim, self.N), e, Fs

    # ---------------------------------------------------------------- markers
    def set_markers(self, X, Ud=None, Tw=None, dA=None, dedupe: bool = True,
                    no_heat: bool = False):
        X = self._dev(X, torch.float64).reshape(-1, self.dim)
        n = X.shape[0]
        Ud = None if Ud is None else self._dev(Ud, torch.float64).reshape(n, self.dim)
        Tw = None if Tw is None else self._dev(Tw, torch.float64).reshape(n)
        dA = None if dA is None else self._dev(dA, torch.float64).reshape(n)
        flags = (L.IBM_DEDUPE if dedupe else 0) | (L.IBM_NO_HEAT if no_heat else 0)
        st = self.lib.ibm_set_markers(self.ctx, n, _ptr(X), _ptr(Ud), _ptr(Tw), _ptr(dA), flags)
        L.check(st, self.ctx, "ibm_set_markers")
        self.nc = n

    def set_motion(self, axis: int, amplitude: float, frequency: float):
        L.check(self.lib.ibm_set_motion(self.ctx, int(axis), float(amplitude), float(frequency)),
                self.ctx, "ibm_set_motion")

    def set_wall_temperature(self, Tw):
        Tw = self._dev(Tw, torch.float64).reshape(-1)
        L.check(self.lib.ibm_set_wall_temperature(self.ctx, _ptr(Tw)), self.ctx,
                "ibm_set_wall_temperature")

    def markers_in_use(self):
        """(candidate ids [n_used] int32, eps [n_used] float64) as device tensors."""
        nu = ctypes.c_int32(0)
        L.check(self.lib.ibm_markers_in_use(self.ctx, ctypes.byref(nu), None, None), self.ctx,
                "ibm_markers_in_use")
        ids = torch.empty(max(nu.value, 1), dtype=torch.int32, device=self.device)
        eps = torch.empty(max(nu.value, 1), dtype=torch.float64, device=self.device)
        L.check(self.lib.ibm_markers_in_use(self.ctx, ctypes.byref(nu), _ptr(ids), _ptr(eps)),
                self.ctx, "ibm_markers_in_use")
        return ids[: nu.value], eps[: nu.value]

    # ------------------------------------------------------------------ steps
    def step(self, n_steps: int = 1, hist: bool = True, record: bool = False,
             hist_out=None):
        """Advances n_steps; returns (history [n_steps, 4] device tensor or None, info dict)."""
        h = None
        if hist_out is not None:
            h = hist_out
        elif hist:
            h = torch.zeros((max(n_steps, 1), 4), dtype=torch.float64, device=self.device)
        info = L.ibm_step_info()
        flags = L.IBM_RECORD if record else 0
        st = self.lib.ibm_step(self.ctx, int(n_steps), flags, _ptr(h), ctypes.byref(info))
        L.check(st, self.ctx, "ibm_step")
        out = {k: getattr(info, k) for k, _ in L.ibm_step_info._fields_}
        return (h[:n_steps] if h is not None else None), out

    def step_status(self, n_steps: int = 1):
        """Like step() but returns the status code instead of raising."""
        info = L.ibm_step_info()
        st = self.lib.ibm_step(self.ctx, int(n_steps), 0, None, ctypes.byref(info))
        return st, {k: getattr(info, k) for k, _ in L.ibm_step_info._fields_}

    def wall_fluxes(self):
        """(force [n_used, dim], heat [n_used], totals (Fx, Fy, Fz, H))."""
        ids, _ = self.markers_in_use()
        nu = ids.shape[0]
        force = torch.zeros((max(nu, 1), self.dim), dtype=torch.float64, device=self.device)
        heat = torch.zeros(max(nu, 1), dtype=torch.float64, device=self.device)
        tot = (ctypes.c_double * 4)()
        L.check(self.lib.ibm_wall_fluxes(self.ctx, _ptr(force), _ptr(heat), tot), self.ctx,
                "ibm_wall_fluxes")
        self.stream.synchronize()
        return force[:nu], heat[:nu], np.array(tot[:])

    def wall_heat_flux(self):
        """Local wall heat flux H_k / dA'_k of the markers in use [n_used] (device)."""
        ids, _ = self.markers_in_use()
        nu = ids.shape[0]
        q = torch.zeros(max(nu, 1), dtype=torch.float64, device=self.device)
        L.check(self.lib.ibm_wall_heat_flux(self.ctx, _ptr(q)), self.ctx, "ibm_wall_heat_flux")
        return q[:nu]

    # ---------------------------------------------------------------- adjoint
    @property
    def state_size(self) -> int:
        """Entries of a state (or state cotangent) in the ibm_set_state layout."""
        return (2 + self.dim) * self.N + sum(self.NF)

    def tape_length(self) -> int:
        return int(self.lib.ibm_tape_length(self.ctx))

    def adjoint_step(self, tape_index: int, state_bar_in, state_bar_out, out_bar=None,
                     Tw_bar=None):
        """Reverse of recorded step ``tape_index``: writes the cotangent of the state
        before the step into ``state_bar_out`` (device float64 [state_size]) from that
        after it (``state_bar_in``) and the cotangents ``out_bar`` of the step's
        (Fx, Fy, Fz, H); adds the step's part of dJ/dT_w to ``Tw_bar``."""
        ob = (ctypes.c_double * 4)(*([0.0] * 4 if out_bar is None else [float(v) for v in out_bar]))
        st = self.lib.ibm_adjoint_step(self.ctx, int(tape_index), _ptr(state_bar_in),
                                       _ptr(state_bar_out), ob, _ptr(Tw_bar))
        L.check(st, self.ctx, "ibm_adjoint_step")

    def shape_gradient(self, X_bar=None):
        """Adds dJ/dX of the candidate marker positions, accumulated by the adjoint
        steps since the last call, to ``X_bar`` (device float64 [n candidates, dim])
        and clears the accumulation; ``None`` only clears it."""
        st = self.lib.ibm_shape_gradient(self.ctx, None if X_bar is None else _ptr(X_bar))
        L.check(st, self.ctx, "ibm_shape_gradient")

    def profile(self, enable: bool):
        L.check(self.lib.ibm_profile(self.ctx, 1 if enable else 0), self.ctx, "ibm_profile")

    def profile_read(self):
        """{class: (total ms, launches)} of the kernel classes timed since enabling."""
        ms = (ctypes.c_double * 8)()
        n = (ctypes.c_int64 * 8)()
        L.check(self.lib.ibm_profile_read(self.ctx, ms, n), self.ctx, "ibm_profile_read")
        return {name: (ms[i], n[i]) for i, name in enumerate(L.PROF_CLASSES)}

    def field(self, name: str):
        idx = {"rho_s": 0, "mom_ss": 1, "E_ss": 2, "psi": 3, "rhs": 4, "pres": 5, "markers": 6}[name]
        if name == "markers":
            ids, _ = self.markers_in_use()
            out = torch.zeros((max(ids.shape[0], 1), 2 * self.dim + 3), dtype=torch.float64,
                              device=self.device)
            L.check(self.lib.ibm_get_field(self.ctx, idx, _ptr(out)), self.ctx, "ibm_get_field")
            return out[: ids.shape[0]]
        dt = torch.float64 if name in ("rhs", "pres") else self.dtype
        size = self.N * (self.dim if name == "mom_ss" else 1)
        out = torch.empty(size, dtype=dt, device=self.device)
        L.check(self.lib.ibm_get_field(self.ctx, idx, _ptr(out)), self.ctx, "ibm_get_field")
        return out.reshape(self.dim, self.N) if name == "mom_ss" else out
