"""ctypes wrapper of the FP64 oracle (oracle/ibm_oracle.cpp).

TEST INFRASTRUCTURE: only tests/, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` may import this module. It imports nothing from the product
package; both sides are handed the same seeded inputs by the caller.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ibm_oracle.cpp")
LIB = os.path.join(HERE, "libibm_oracle.so")

PERIODIC, INFLOW, OUTFLOW, SLIP = 0, 1, 2, 3
SUP_INFLOW, SUP_OUTFLOW = 4, 5
CONV_VANLEER, CONV_LINEAR = 0, 1
MU_SUTHERLAND, MU_CONSTANT = 0, 1


class Desc(ctypes.Structure):
    """Mirror of the oracle's own problem description struct."""

    _fields_ = [
        ("dim", ctypes.c_int32),
        ("n", ctypes.c_int32 * 3),
        ("lo", ctypes.c_double * 3),
        ("hi", ctypes.c_double * 3),
        ("bc", (ctypes.c_int32 * 2) * 3),
        ("convection", ctypes.c_int32),
        ("viscosity_law", ctypes.c_int32),
        ("Re", ctypes.c_double),
        ("Ma", ctypes.c_double),
        ("Pr", ctypes.c_double),
        ("gamma", ctypes.c_double),
        ("sutherland_S", ctypes.c_double),
        ("U_inf", ctypes.c_double * 3),
        ("dt", ctypes.c_double),
        ("cfl", ctypes.c_double),
        ("dt_theta_max", ctypes.c_double),
        ("dt_u_max", ctypes.c_double),
        ("cg_rtol", ctypes.c_double),
        ("cg_maxit", ctypes.c_int32),
        ("diffusion", ctypes.c_int32),
        ("n_outer", ctypes.c_int32),
        ("scheme", ctypes.c_int32),
    ]


# the same source built for the host it runs on (-O3 -march=native; still no FMA
# contraction, so the arithmetic is unchanged), for timing the oracle as it stands
NATIVE_LIB = os.path.join(HERE, "libibm_oracle_native.so")
_use_native = False


def build(force: bool = False, native: bool = False) -> str:
    """Compile the oracle with g++ (plain IEEE arithmetic: no FMA contraction)."""
    out = NATIVE_LIB if native else LIB
    opt = ["-O3", "-march=native"] if native else ["-O2"]
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(SRC):
        cmd = ["g++", *opt, "-std=c++17", "-ffp-contract=off", "-fno-fast-math",
               "-shared", "-fPIC", SRC, "-o", out + ".tmp"]
        subprocess.check_call(cmd)
        os.replace(out + ".tmp", out)
    return out


def use_native():
    """Load the -O3 -march=native build (compiled here, for this host) instead of the
    default one; must be called before the first oracle call of the process."""
    global _use_native
    if _lib is not None:
        raise RuntimeError("oracle library already loaded")
    _use_native = True


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = build(native=_use_native)
        L = ctypes.CDLL(path)
        P = ctypes.c_void_p
        D = ctypes.POINTER(ctypes.c_double)
        L.orc_create.restype = P
        L.orc_create.argtypes = [ctypes.POINTER(Desc)]
        L.orc_destroy.argtypes = [P]
        L.orc_dt.restype = ctypes.c_double
        L.orc_dt.argtypes = [P]
        L.orc_num_cells.restype = ctypes.c_long
        L.orc_num_cells.argtypes = [P]
        L.orc_num_faces.restype = ctypes.c_long
        L.orc_num_faces.argtypes = [P, ctypes.c_int]
        L.orc_mu.restype = ctypes.c_double
        L.orc_mu.argtypes = [P, ctypes.c_double]
        L.orc_kernel.restype = ctypes.c_double
        L.orc_kernel.argtypes = [ctypes.c_double]
        L.orc_set_markers.restype = ctypes.c_int
        L.orc_set_markers.argtypes = [P, ctypes.c_int, D, D, D, D, ctypes.c_int]
        L.orc_get_keep.restype = ctypes.c_int
        L.orc_get_keep.argtypes = [P, ctypes.POINTER(ctypes.c_int)]
        L.orc_set_motion.argtypes = [P, ctypes.c_int, ctypes.c_double, ctypes.c_double]
        L.orc_set_wall_temperature.argtypes = [P, D]
        L.orc_get_eps.restype = ctypes.c_int
        L.orc_get_eps.argtypes = [P, D]
        L.orc_get_support.argtypes = [P, ctypes.POINTER(ctypes.c_long), D]
        L.orc_init_primitive.argtypes = [P, D, D, D]
        L.orc_set_state.argtypes = [P, D, D, D, D, ctypes.c_long]
        L.orc_get_state.argtypes = [P, D, D, D, D]
        L.orc_step.restype = ctypes.c_int
        L.orc_step.argtypes = [P, ctypes.c_int, D]
        L.orc_get_intermediate.argtypes = [P, ctypes.c_int, D]
        L.orc_get_marker_fields.argtypes = [P, D]
        L.orc_predictor_only.restype = ctypes.c_int
        L.orc_predictor_only.argtypes = [P]
        L.orc_helmholtz.argtypes = [P, D, D, D]
        L.orc_cg.restype = ctypes.c_int
        L.orc_cg.argtypes = [P, D, D, D]
        L.orc_interp.argtypes = [P, D, D]
        L.orc_spread.argtypes = [P, D, D]
        L.orc_tl_run.restype = ctypes.c_int
        L.orc_tl_run.argtypes = [P, ctypes.c_int, D, D, D]
        L.orc_tl_shape.restype = ctypes.c_int
        L.orc_tl_shape.argtypes = [P, ctypes.c_int, D, D, D]
        L.orc_tl_state.restype = ctypes.c_int
        L.orc_tl_state.argtypes = [P, ctypes.c_int, D, D, D, D, D]
        L.orc_wall_fluxes.restype = ctypes.c_int
        L.orc_wall_fluxes.argtypes = [P, D, D, D]
        L.orc_get_markers.restype = ctypes.c_int
        L.orc_get_markers.argtypes = [P, D, D]
        L.orc_face_value.restype = ctypes.c_double
        L.orc_face_value.argtypes = [P, D, ctypes.c_int, ctypes.c_int, ctypes.c_long,
                                     ctypes.c_long, ctypes.c_long, ctypes.c_double]
        _lib = L
    return _lib


def _p(a):
    if a is None:
        return ctypes.cast(None, ctypes.POINTER(ctypes.c_double))
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def kernel(r: float) -> float:
    return lib().orc_kernel(float(r))


class Oracle:
    """One oracle solver instance: grid, markers and state, all FP64 on the host."""

    def __init__(self, case):
        """``case`` is a dict with the keys of the problem description (see
        ``make_desc``)."""
        self.case = case
        self.desc = make_desc(case)
        self.h = lib().orc_create(ctypes.byref(self.desc))
        if not self.h:
            raise ValueError("oracle: invalid problem description")
        self.dim = int(case["dim"])
        self.n = [int(v) for v in case["n"]][: self.dim]
        self.N = int(lib().orc_num_cells(self.h))
        self.NF = [int(lib().orc_num_faces(self.h, d)) for d in range(self.dim)]
        self.ns = 0

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().orc_destroy(self.h)
                self.h = None
        except Exception:
            pass

    @property
    def dt(self) -> float:
        return lib().orc_dt(self.h)

    def mu(self, theta: float) -> float:
        return lib().orc_mu(self.h, float(theta))

    def set_markers(self, X, Ud=None, Tw=None, dA=None, dedupe=False, no_heat=False):
        """Candidate markers; with ``dedupe`` only the one nearest to the centre of
        each cell is used (the check routine of Sec. 3.1); with ``no_heat`` the
        markers exchange no heat (their energy source is zero)."""
        X = np.ascontiguousarray(X, dtype=np.float64)
        ns = X.shape[0]
        Ud = np.zeros_like(X) if Ud is None else np.ascontiguousarray(Ud, dtype=np.float64)
        Tw = np.ones(ns) if Tw is None else np.ascontiguousarray(Tw, dtype=np.float64)
        dA = np.zeros(ns) if dA is None else np.ascontiguousarray(dA, dtype=np.float64)
        rc = lib().orc_set_markers(self.h, ns, _p(X), _p(Ud), _p(Tw), _p(dA),
                                   (1 if dedupe else 0) | (2 if no_heat else 0))
        if rc:
            raise ValueError(f"oracle: set_markers failed ({rc})")
        self.nc = ns
        self.ns = int(lib().orc_get_keep(self.h, (ctypes.c_int * ns)()))

    def keep(self):
        """Candidate ids of the markers in use."""
        ids = (ctypes.c_int * max(self.nc, 1))()
        k = lib().orc_get_keep(self.h, ids)
        self.ns = k
        return np.array(ids[:k], dtype=np.int64)

    def set_motion(self, axis: int, amp: float, freq: float):
        lib().orc_set_motion(self.h, int(axis), float(amp), float(freq))

    def set_wall_temperature(self, Tw):
        Tw = np.ascontiguousarray(Tw, dtype=np.float64)
        lib().orc_set_wall_temperature(self.h, _p(Tw))

    def eps(self):
        self.keep()
        out = np.zeros(self.ns)
        lib().orc_get_eps(self.h, _p(out))
        return out

    def support(self):
        self.keep()
        cells = np.zeros(self.ns * 27, dtype=np.int64)
        w = np.zeros(self.ns * 27)
        lib().orc_get_support(self.h, cells.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), _p(w))
        k = 9 if self.dim == 2 else 27
        return cells.reshape(self.ns, 27)[:, :k], w.reshape(self.ns, 27)[:, :k]

    def init_primitive(self, rho, u, theta):
        rho = np.ascontiguousarray(rho, dtype=np.float64).ravel()
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(self.dim, -1)
        theta = np.ascontiguousarray(theta, dtype=np.float64).ravel()
        lib().orc_init_primitive(self.h, _p(rho), _p(np.ascontiguousarray(u)), _p(theta))

    def set_state(self, rho, mom, E, F=None, step=0):
        rho = np.ascontiguousarray(rho, dtype=np.float64).ravel()
        mom = np.ascontiguousarray(mom, dtype=np.float64).reshape(self.dim, -1)
        E = np.ascontiguousarray(E, dtype=np.float64).ravel()
        Fc = None
        if F is not None:
            Fc = np.ascontiguousarray(np.concatenate([np.ravel(f) for f in F]), dtype=np.float64)
        lib().orc_set_state(self.h, _p(rho), _p(mom), _p(E), _p(Fc), int(step))

    def get_state(self):
        rho = np.zeros(self.N)
        mom = np.zeros((self.dim, self.N))
        E = np.zeros(self.N)
        F = np.zeros(sum(self.NF))
        lib().orc_get_state(self.h, _p(rho), _p(mom), _p(E), _p(F))
        Fs, off = [], 0
        for d in range(self.dim):
            Fs.append(F[off: off + self.NF[d]].copy())
            off += self.NF[d]
        return rho, mom, E, Fs

    def step(self, nsteps: int = 1):
        """Runs ``nsteps`` steps; returns the per-step history as an array of rows
        (Fx, Fy, Fz, H, mass, cg_iters, cg_rel_residual, t)."""
        hist = np.zeros((nsteps, 8))
        rc = lib().orc_step(self.h, int(nsteps), _p(hist))
        if rc:
            raise RuntimeError(f"oracle: step failed ({rc})")
        return hist

    def intermediate(self, which: str):
        idx = {"rho_s": 0, "mom_s": 1, "E_s": 2, "mom_ss": 3, "E_ss": 4, "psi": 5,
               "rhs": 6, "pres": 7}[which]
        size = self.N * (self.dim if which in ("mom_s", "mom_ss") else 1)
        out = np.zeros(size)
        lib().orc_get_intermediate(self.h, idx, _p(out))
        return out.reshape(self.dim, -1) if which in ("mom_s", "mom_ss") else out

    def marker_fields(self):
        """Per marker: rho_L, M (dim), E_L, F (dim), Q of the last step."""
        self.keep()
        w = 2 * self.dim + 3
        out = np.zeros(self.ns * w)
        lib().orc_get_marker_fields(self.h, _p(out))
        return out.reshape(self.ns, w)

    def wall_fluxes(self):
        """Per marker in use after the last step: force on the body -dV eps_k F_k
        [ns, dim], heat given to the fluid H_k = dV eps_k Q_k [ns], and the local heat
        flux H_k / dA'_k [ns] (the surface elements of the markers in use scaled to
        the whole given surface; None when the markers carry no surface)."""
        self.keep()
        f = np.zeros(self.ns * self.dim)
        hq = np.zeros(self.ns)
        q = np.zeros(self.ns)
        rc = lib().orc_wall_fluxes(self.h, _p(f), _p(hq), _p(q))
        return f.reshape(self.ns, self.dim), hq, (None if rc else q)

    def markers(self):
        """Positions [ns, dim] and desired velocities [ns, dim] of the markers in use."""
        self.keep()
        X = np.zeros(self.ns * self.dim)
        U = np.zeros(self.ns * self.dim)
        lib().orc_get_markers(self.h, _p(X), _p(U))
        return X.reshape(self.ns, self.dim), U.reshape(self.ns, self.dim)

    def face_value(self, field, var: int, d: int, idx, F: float) -> float:
        """Convected face value (Sec. 2.2.2) of the cell field ``field`` [N] (variable
        kind ``var``: 0 rho, 1..3 velocity components, 4 theta, 5 p, 6 E) on the face
        of direction ``d`` between cell ``idx`` - e_d and cell ``idx``, for face mass
        flux ``F``."""
        a = np.ascontiguousarray(field, dtype=np.float64).ravel()
        i = list(idx) + [0] * (3 - len(idx))
        return lib().orc_face_value(self.h, _p(a), int(var), int(d), int(i[0]), int(i[1]),
                                    int(i[2]), float(F))

    def predictor_only(self):
        rc = lib().orc_predictor_only(self.h)
        if rc:
            raise RuntimeError(f"oracle: predictor failed ({rc})")

    def helmholtz(self, psi, x):
        psi = np.ascontiguousarray(psi, dtype=np.float64).ravel()
        x = np.ascontiguousarray(x, dtype=np.float64).ravel()
        y = np.zeros(self.N)
        lib().orc_helmholtz(self.h, _p(psi), _p(x), _p(y))
        return y

    def cg(self, psi, b, x0):
        psi = np.ascontiguousarray(psi, dtype=np.float64).ravel()
        b = np.ascontiguousarray(b, dtype=np.float64).ravel()
        x = np.ascontiguousarray(x0, dtype=np.float64).ravel().copy()
        it = lib().orc_cg(self.h, _p(psi), _p(b), _p(x))
        return x, it

    def interp(self, field):
        field = np.ascontiguousarray(field, dtype=np.float64).ravel()
        out = np.zeros(self.ns)
        lib().orc_interp(self.h, _p(field), _p(out))
        return out

    def spread(self, Rk):
        Rk = np.ascontiguousarray(Rk, dtype=np.float64).ravel()
        out = np.zeros(self.N)
        lib().orc_spread(self.h, _p(Rk), _p(out))
        return out

    def tangent_linear(self, nsteps: int, dTw):
        """Directional derivative along ``dTw`` of the per-step (Fx, Fy, Fz, H) from
        the current state (which is left unchanged)."""
        dTw = np.ascontiguousarray(dTw, dtype=np.float64)
        hv = np.zeros((nsteps, 4))
        hd = np.zeros((nsteps, 4))
        rc = lib().orc_tl_run(self.h, int(nsteps), _p(dTw), _p(hv), _p(hd))
        if rc:
            raise RuntimeError(f"oracle: tangent-linear run failed ({rc})")
        return hv, hd

    def tangent_linear_shape(self, nsteps: int, dX):
        """Directional derivative along ``dX`` ([n candidates, dim]: the candidate
        marker positions) of the per-step (Fx, Fy, Fz, H) from the current state
        (left unchanged); returns (values, derivatives), each [nsteps, 4]."""
        dX = np.ascontiguousarray(dX, dtype=np.float64).reshape(-1)
        hv = np.zeros((nsteps, 4))
        hd = np.zeros((nsteps, 4))
        rc = lib().orc_tl_shape(self.h, int(nsteps), _p(dX), _p(hv), _p(hd))
        if rc:
            raise RuntimeError(f"oracle: tangent-linear run failed ({rc})")
        return hv, hd

    @property
    def state_size(self) -> int:
        return (2 + self.dim) * self.N + sum(self.NF)

    def tangent_linear_state(self, nsteps: int, dstate, dTw=None):
        """Directional derivative from the current state (left unchanged) along
        ``dstate`` (rho [N], mom [dim][N], E [N], F [sum NF]) and, optionally, ``dTw``:
        returns (history values [nsteps, 4], their derivatives [nsteps, 4], the
        derivative of the state after the steps [state_size])."""
        ds = np.ascontiguousarray(dstate, dtype=np.float64).ravel()
        if ds.size != self.state_size:
            raise ValueError("dstate has the wrong size")
        dT = None if dTw is None else np.ascontiguousarray(dTw, dtype=np.float64)
        hv = np.zeros((nsteps, 4))
        hd = np.zeros((nsteps, 4))
        dout = np.zeros(self.state_size)
        rc = lib().orc_tl_state(self.h, int(nsteps), _p(ds), _p(dT), _p(hv), _p(hd),
                                _p(dout))
        if rc:
            raise RuntimeError(f"oracle: tangent-linear run failed ({rc})")
        return hv, hd, dout


def make_desc(case) -> Desc:
    d = Desc()
    d.dim = int(case["dim"])
    n = list(case["n"]) + [1] * (3 - len(case["n"]))
    lo = list(case["lo"]) + [0.0] * (3 - len(case["lo"]))
    hi = list(case["hi"]) + [1.0] * (3 - len(case["hi"]))
    for a in range(3):
        d.n[a] = int(n[a])
        d.lo[a] = float(lo[a])
        d.hi[a] = float(hi[a])
    bc = case["bc"]
    for a in range(3):
        for s in range(2):
            d.bc[a][s] = int(bc[a][s]) if a < len(bc) else PERIODIC
    d.convection = int(case.get("convection", CONV_VANLEER))
    d.viscosity_law = int(case.get("viscosity_law", MU_SUTHERLAND))
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
    d.diffusion = int(case.get("diffusion", 0))
    d.n_outer = int(case.get("n_outer", 1))
    d.scheme = int(case.get("scheme", 0))
    return d
