"""CPU oracle of the moment-based multi-resolution HWENO scheme.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark may import this package; the GPU library
never does.  The arithmetic lives in ``mrhweno_oracle.c`` (plain C, FP64,
no FMA contraction); this module only marshals numpy arrays through ctypes.

Parity status of each function is listed in ``ORACLE_PINS`` below; every
function there is pinned by a ``-m "not gpu"`` test against what the paper
or the mathematics fixes.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mrhweno_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

ORACLE_PINS = {
    "step1_1d": "exactness of q2/q3/q4 on polynomial data; closed forms; eq. (pq); Remark 1; Table 1/3 orders",
    "step1_2d": "exactness of the least-squares q2/q3/q4 on P2/P3/P5 data; eq. (2D-pq); D4 symmetry; Table 2/4 orders; "
                "beta_1 worked example (eqs. (2D-q1-1234)-(2D-beta1)); 2D Remark 1 expansion of beta on exp data; "
                "reduction of y-invariant data to the 1D algorithm",
    "modification": "eq. (vi) printed coefficients",
    "kxrcf": "smooth/discontinuous scaling (Remark 2); inflow side of a moving step; Lax problem flags; "
             "2D: denominator on uniform flows, face-length scaling on non-square cells, two inflow faces, "
             "x and y faces of a raised cell, norm over all sixteen points",
    "hllc": "consistency, supersonic branches, stationary contact",
    "wall_flux": "gas at rest keeps its pressure; star pressure of the reflected shock against the Rankine-Hugoniot "
                 "relations and the shock speed; isentropic rarefaction and vacuum; mirror-direction symmetry",
    "step": "gas at rest in a tunnel with a step stays at rest; mirror images of the step cells (depth rule, "
            "corner); uniform flow along the step top is preserved; step faces are walls in the KXRCF test",
    "residual": "conservation; free-stream preservation; convergence orders; Lax problem vs exact Riemann solution",
    "rk3": "third-order temporal convergence",
}


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (FP64, -ffp-contract=off, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Prob(C.Structure):
    _fields_ = [("dim", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("system", C.c_int),
                ("bc_x", C.c_int), ("bc_y", C.c_int), ("tc_mode", C.c_int), ("beta_on", C.c_int),
                ("dx", C.c_double), ("dy", C.c_double), ("gamma", C.c_double),
                ("gbar", C.c_double * 4), ("eps", C.c_double), ("tvb_m", C.c_double),
                ("charwise", C.c_int),
                ("x0", C.c_double), ("y0", C.c_double), ("t", C.c_double),
                ("side_kind", C.c_int * 4), ("side_state", C.c_double * 16),
                ("side_pre", C.c_double * 16), ("side_split", C.c_double * 12),
                ("step_i", C.c_int), ("step_j", C.c_int), ("wall_flux", C.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        D = C.POINTER(C.c_double)
        B = C.POINTER(C.c_ubyte)
        P = C.POINTER(_Prob)
        L.orc_step1_1d.argtypes = [P, D, D, D, D, D]
        L.orc_step1_2d.argtypes = [P, D, D, D, D, D, D]
        L.orc_qmap_1d.argtypes = [C.c_int, D]
        L.orc_modmap_1d.argtypes = [D]
        L.orc_qmap_2d.argtypes = [C.c_int, D]
        L.orc_qcoef_2d.argtypes = [C.c_int, D, D, D, D]
        L.orc_monomials_2d.argtypes = [C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.orc_hllc.argtypes = [D, D, C.c_int, C.c_int, C.c_double, D]
        L.orc_wall_flux.argtypes = [D, C.c_int, C.c_int, C.c_int, C.c_double, D]
        L.orc_residual.argtypes = [P, D, D, B]
        L.orc_residual_given.argtypes = [P, D, B, D]
        L.orc_reconstruct.argtypes = [P, D, D, B, D, D]
        L.orc_wave_speeds.argtypes = [P, D, D]
        L.orc_dt.argtypes = [P, D, C.c_double]
        L.orc_dt.restype = C.c_double
        L.orc_rk3_step.argtypes = [P, D, C.c_double, B]
        L.orc_moment.argtypes = [P, D, C.c_int, C.c_int, C.c_int, C.c_int]
        L.orc_moment.restype = C.c_double
        L.orc_rk3_step_p.argtypes = [P, D, C.c_double, B, C.c_int]
        L.orc_modify.argtypes = [P, D, B, D]
        L.orc_residual_cell_2d.argtypes = [P, D, C.c_double, C.c_int, C.c_int, D]
        L.orc_gl.argtypes = [D, D]
        L.orc_euler2_eigen.argtypes = [D, C.c_double, C.c_int, D, D]
        L.orc_step1_2d_sys.argtypes = [P, D, D, D, C.c_int, D]
        L.orc_max_threads.restype = C.c_int
        L.orc_set_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _bp(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.uint8 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_ubyte))


def cprob(prob, t: float = 0.0) -> _Prob:
    """The oracle's problem struct; t is the time of the boundary data."""
    p = _Prob()
    p.dim, p.nx, p.ny = prob.dim, prob.nx, (prob.ny if prob.dim == 2 else 1)
    p.system, p.bc_x, p.bc_y = prob.system, prob.bc_x, prob.bc_y
    p.tc_mode = 1 if prob.tc_mode == 3 else prob.tc_mode
    p.beta_on = prob.beta_on
    p.dx, p.dy, p.gamma, p.eps = prob.dx, prob.dy, prob.gamma, prob.eps
    for k in range(4):
        p.gbar[k] = prob.gbar[k]
    p.tvb_m = getattr(prob, "tvb_m", 0.0)
    p.charwise = getattr(prob, "charwise", 0)
    p.x0, p.y0, p.t = prob.x0, prob.y0, float(t)
    p.step_i, p.step_j = getattr(prob, "step_i", 0), getattr(prob, "step_j", 0)
    p.wall_flux = getattr(prob, "wall_flux", 0)
    for k in range(4):
        p.side_split[3 * k] = -math.inf
    sides = getattr(prob, "sides", None)
    if sides is not None:
        for k, sd in enumerate(sides):
            if sd is None:
                continue
            if k < 2 and sd.split[0] != -math.inf:
                raise ValueError("a split is defined on the bottom and top sides only")
            p.side_kind[k] = sd.kind
            for c in range(len(sd.state)):
                p.side_state[4 * k + c] = sd.state[c]
            for c in range(len(sd.pre)):
                p.side_pre[4 * k + c] = sd.pre[c]
            for q in range(3):
                p.side_split[3 * k + q] = sd.split[q]
    return p


def _arr(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64))


# ---------------------------------------------------------------- per stencil
def step1_1d(prob, ub, vb) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Step 1 (1D) for one component: returns (gl[4], weights[4], betas[4])."""
    ub, vb = _arr(ub), _arr(vb)
    gl, w, b = np.zeros(4), np.zeros(4), np.zeros(4)
    lib().orc_step1_1d(C.byref(cprob(prob)), _dp(ub), _dp(vb), _dp(gl), _dp(w), _dp(b))
    return gl, w, b


def step1_2d(prob, ub, vb, wb) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Step 1 (2D) for one component; ub/vb/wb indexed by stencil label-1.
    Returns (gl[16] with gl[k + 4 l] at (xi_k, eta_l), weights[4], betas[4])."""
    ub, vb, wb = _arr(ub), _arr(vb), _arr(wb)
    gl, w, b = np.zeros(16), np.zeros(4), np.zeros(4)
    lib().orc_step1_2d(C.byref(cprob(prob)), _dp(ub), _dp(vb), _dp(wb), _dp(gl), _dp(w), _dp(b))
    return gl, w, b


def step1_2d_sys(prob, ub, vb, wb, direction: int = 0) -> np.ndarray:
    """Step 1 (2D) for all components of one cell; ub/vb/wb [ncomp][9]
    indexed by stencil label-1.  With prob.charwise on 2D Euler: the set of
    values of the given direction (0: x, 1: y).  Returns [ncomp][16]."""
    ub, vb, wb = _arr(ub), _arr(vb), _arr(wb)
    out = np.zeros((ub.shape[0], 16))
    lib().orc_step1_2d_sys(C.byref(cprob(prob)), _dp(ub), _dp(vb), _dp(wb), int(direction), _dp(out))
    return out


def qmap_1d(level: int) -> np.ndarray:
    deg = {2: 2, 3: 3, 4: 5}[level]
    out = np.zeros((deg + 1, 6))
    lib().orc_qmap_1d(level, _dp(out))
    return out


def modmap_1d() -> np.ndarray:
    out = np.zeros(6)
    lib().orc_modmap_1d(_dp(out))
    return out


def euler1_eigen(u, gamma: float) -> Tuple[np.ndarray, np.ndarray]:
    """Left and right eigenvector matrices of the 1D Euler flux Jacobian at
    the conserved state u (rows of L, columns of R)."""
    L, R = np.zeros(9), np.zeros(9)
    lib().orc_euler1_eigen(_dp(np.ascontiguousarray(u, dtype=np.float64)), C.c_double(gamma), _dp(L), _dp(R))
    return L.reshape(3, 3), R.reshape(3, 3)


def euler2_eigen(u, gamma: float, direction: int) -> Tuple[np.ndarray, np.ndarray]:
    """Left and right eigenvector matrices of the 2D Euler flux Jacobian in
    direction 0 (x) or 1 (y) at the conserved state u (rows of L, columns
    of R)."""
    L, R = np.zeros(16), np.zeros(16)
    lib().orc_euler2_eigen(_dp(np.ascontiguousarray(u, dtype=np.float64)), C.c_double(gamma), int(direction),
                           _dp(L), _dp(R))
    return L.reshape(4, 4), R.reshape(4, 4)


def monomials_2d() -> Tuple[np.ndarray, np.ndarray]:
    a = (C.c_int * 21)()
    b = (C.c_int * 21)()
    lib().orc_monomials_2d(a, b)
    return np.array(a[:]), np.array(b[:])


def qmap_2d(level: int) -> np.ndarray:
    nco = {2: 6, 3: 10, 4: 21}[level]
    out = np.zeros((nco, 27))
    lib().orc_qmap_2d(level, _dp(out))
    return out


def qcoef_2d(level: int, ub, vb, wb) -> np.ndarray:
    nco = {2: 6, 3: 10, 4: 21}[level]
    out = np.zeros(nco)
    lib().orc_qcoef_2d(level, _dp(_arr(ub)), _dp(_arr(vb)), _dp(_arr(wb)), _dp(out))
    return out


def hllc(uL, uR, gamma: float, direction: int = 0) -> np.ndarray:
    uL, uR = _arr(uL), _arr(uR)
    f = np.zeros(len(uL))
    lib().orc_hllc(_dp(uL), _dp(uR), len(uL), direction, gamma, _dp(f))
    return f


def wall_flux(u, gamma: float, direction: int = 0, sgn: int = 1) -> np.ndarray:
    """Flux through a wall face normal to `direction` of the fluid trace u,
    the wall on the side sgn (+1: towards +direction) (reading R20)."""
    u = _arr(u)
    f = np.zeros(len(u))
    lib().orc_wall_flux(_dp(u), len(u), direction, sgn, gamma, _dp(f))
    return f


# ---------------------------------------------------------------- whole grid
def residual(prob, U, t: float = 0.0) -> Tuple[np.ndarray, np.ndarray]:
    """L(U) and the troubled-cell flags of the interior (boundary data at
    time t)."""
    U = _arr(U).reshape(prob.shape())
    L = np.zeros_like(U)
    flags = np.zeros(prob.ncell, dtype=np.uint8)
    lib().orc_residual(C.byref(cprob(prob, t)), _dp(U), _dp(L), _bp(flags))
    return L, flags.reshape(prob.shape()[2:])


def residual_given(prob, U, flags_ext, t: float = 0.0) -> np.ndarray:
    """2D L(U) with the troubled-cell map of cells [-2, n+2)^2 supplied as a
    (ny+4, nx+4) uint8 array instead of Step 2.1."""
    U = _arr(U).reshape(prob.shape())
    fe = np.ascontiguousarray(flags_ext, dtype=np.uint8)
    if prob.dim != 2 or fe.shape != (prob.ny + 4, prob.nx + 4):
        raise ValueError("2D problem and a (ny+4, nx+4) flag map required")
    L = np.zeros_like(U)
    if lib().orc_residual_given(C.byref(cprob(prob, t)), _dp(U), _bp(fe), _dp(L)) != 0:
        raise RuntimeError("orc_residual_given failed")
    return L


def reconstruct(prob, U, t: float = 0.0):
    """Final Gauss-Lobatto values (1D [comp][4][nx], 2D [comp][16][ny][nx]),
    flags, and the KXRCF numerator and denominator."""
    U = _arr(U).reshape(prob.shape())
    npt = 4 if prob.dim == 1 else 16
    gl = np.zeros((prob.ncomp, npt) + prob.shape()[2:])
    flags = np.zeros(prob.ncell, dtype=np.uint8)
    num = np.zeros(prob.ncell)
    den = np.zeros(prob.ncell)
    lib().orc_reconstruct(C.byref(cprob(prob, t)), _dp(U), _dp(gl), _bp(flags), _dp(num), _dp(den))
    sh = prob.shape()[2:]
    return gl, flags.reshape(sh), num.reshape(sh), den.reshape(sh)


def moment(prob, U, c: int, m: int, i: int, j: int = 0, t: float = 0.0) -> float:
    """Moment m of component c at cell (i, j), ghost cells included, with
    the boundary data at time t."""
    U = _arr(U).reshape(prob.shape())
    return float(lib().orc_moment(C.byref(cprob(prob, t)), _dp(U), c, m, i, j))


def wave_speeds(prob, U) -> Tuple[float, float]:
    U = _arr(U).reshape(prob.shape())
    out = np.zeros(2)
    lib().orc_wave_speeds(C.byref(cprob(prob)), _dp(U), _dp(out))
    return float(out[0]), float(out[1])


def dt(prob, U, cfl: Optional[float] = None) -> float:
    U = _arr(U).reshape(prob.shape())
    return float(lib().orc_dt(C.byref(cprob(prob)), _dp(U), prob.cfl if cfl is None else cfl))


# placement of the modified first moments (problem field `modification`:
# 0 every stage input and U^n, 1 nowhere, 2 stage inputs only) -> the C
# oracle's persist argument (1, 0, 2)
_PERSIST = {0: 1, 1: 0, 2: 2}


def rk3_step(prob, U, dt_: float, want_flags: bool = False, persist: Optional[int] = None,
             t: float = 0.0):
    """One SSP-RK3 step from time t; returns U^{n+1} (and the flags of the
    3 stages).  persist defaults to the problem's modification placement."""
    if persist is None:
        persist = _PERSIST[getattr(prob, "modification", 0)]
    U = _arr(U).reshape(prob.shape()).copy()
    flags = np.zeros(3 * prob.ncell, dtype=np.uint8) if want_flags else None
    lib().orc_rk3_step_p(C.byref(cprob(prob, t)), _dp(U), dt_, _bp(flags), persist)
    if want_flags:
        return U, flags.reshape((3,) + prob.shape()[2:])
    return U


def residual_cell_2d(prob, U, i: int, j: int, alpha: float = 0.0, t: float = 0.0) -> np.ndarray:
    """L(U) at one cell of a 2D grid, recomputed from scratch (for sampling)."""
    out = np.zeros((prob.ncomp, 3))
    lib().orc_residual_cell_2d(C.byref(cprob(prob, t)), _dp(U), alpha, i, j, _dp(out))
    return out


def modify(prob, U, flags, t: float = 0.0) -> np.ndarray:
    """Stage input with troubled cells' first moments replaced (Step 2.2)."""
    U = _arr(U).reshape(prob.shape())
    fl = np.ascontiguousarray(np.asarray(flags, dtype=np.uint8).ravel())
    out = np.zeros_like(U)
    lib().orc_modify(C.byref(cprob(prob, t)), _dp(U), _bp(fl), _dp(out))
    return out


def run(prob, U, t_final: Optional[float] = None, max_steps: int = 10 ** 9, dt_fn=None,
        persist: Optional[int] = None, t0: float = 0.0):
    """March from t0 to t_final with the CFL time step (clipped at t_final)."""
    T = prob.t_final if t_final is None else t_final
    U = _arr(U).reshape(prob.shape()).copy()
    t, steps = t0, 0
    while t < T and steps < max_steps:
        d = dt(prob, U) if dt_fn is None else dt_fn(prob, U)
        d = min(d, T - t)
        U = rk3_step(prob, U, d, persist=persist, t=t)
        t += d
        steps += 1
    return U, t, steps


def gl_rule():
    x, w = np.zeros(4), np.zeros(4)
    lib().orc_gl(_dp(x), _dp(w))
    return x, w


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def max_threads() -> int:
    return int(lib().orc_max_threads())
