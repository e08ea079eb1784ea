"""Python binding of libmrhweno.so (argument marshalling only).

Every step of the scheme runs in the library's HIP kernels; PyTorch only
provides device memory (tensors) and the HIP stream.  The names follow the
C ABI in include/mrhweno.h.  There is no fallback: if the shared library is
missing or no GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from typing import List, Optional, Sequence, Tuple

from .inputs import TC_KXRCF, Problem

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmrhweno.so")

OK = 0
ERR_INVALID_ARG = -1
ERR_UNSUPPORTED = -2
ERR_DEVICE = -3
ERR_NONPHYSICAL = -4
ERR_NOT_READY = -5
MLP_FEATURES = 320
MLP_PARAMS = 24776

EXPORTS = ["mrhweno_workspace_bytes", "mrhweno_create", "mrhweno_step", "mrhweno_sync",
           "mrhweno_set_time", "mrhweno_last_dt", "mrhweno_reconstruct", "mrhweno_flag",
           "mrhweno_residual", "mrhweno_residual_noalloc", "mrhweno_set_launch", "mrhweno_autotune",
           "mrhweno_set_indicator_launch", "mrhweno_autotune_indicator", "mrhweno_profile",
           "mrhweno_set_indicator", "mrhweno_indicator", "mrhweno_features",
           "mrhweno_mlp_param_count", "mrhweno_mlp_feature_count", "mrhweno_mlp_cache_bytes",
           "mrhweno_mlp_gemm", "mrhweno_mlp_forward", "mrhweno_mlp_backward", "mrhweno_mlp_adam",
           "mrhweno_last_error", "mrhweno_destroy"]


class MrSide(C.Structure):
    _fields_ = [("kind", C.c_int), ("front", C.c_int), ("state", C.c_double * 4),
                ("pre", C.c_double * 4), ("split", C.c_double * 3)]


class MrProblem(C.Structure):
    _fields_ = [("dim", C.c_int), ("nx", C.c_int), ("ny", C.c_int),
                ("x0", C.c_double), ("x1", C.c_double), ("y0", C.c_double), ("y1", C.c_double),
                ("bc_x", C.c_int), ("bc_y", C.c_int), ("flux", C.c_int),
                ("gamma_gas", C.c_double), ("cfl", C.c_double), ("t_final", C.c_double),
                ("gamma_bar", C.c_double * 4), ("eps", C.c_double),
                ("tc_mode", C.c_int), ("beta_on", C.c_int), ("modification", C.c_int),
                ("tvb_m", C.c_double), ("charwise", C.c_int), ("side", MrSide * 4),
                ("step_i", C.c_int), ("step_j", C.c_int), ("wall_flux", C.c_int)]


def to_c(p: Problem) -> MrProblem:
    c = MrProblem()
    c.dim, c.nx, c.ny = p.dim, p.nx, (p.ny if p.dim == 2 else 1)
    c.x0, c.x1, c.y0, c.y1 = p.x0, p.x1, p.y0, p.y1
    c.bc_x, c.bc_y, c.flux = p.bc_x, p.bc_y, p.system
    c.gamma_gas, c.cfl = p.gamma, p.cfl
    c.t_final = p.t_final if math.isfinite(p.t_final) else float("inf")
    for k in range(4):
        c.gamma_bar[k] = p.gbar[k]
    c.eps, c.tc_mode, c.beta_on, c.modification = p.eps, p.tc_mode, p.beta_on, p.modification
    c.tvb_m = p.tvb_m
    c.charwise = p.charwise
    c.step_i, c.step_j, c.wall_flux = p.step_i, p.step_j, p.wall_flux
    if p.sides is not None:
        for k, sd in enumerate(p.sides):
            if sd is None:
                continue
            c.side[k].kind = sd.kind
            c.side[k].front = 1 if sd.split[0] != -math.inf else 0
            for q, v in enumerate(sd.state):
                c.side[k].state[q] = v
            for q, v in enumerate(sd.pre):
                c.side[k].pre[q] = v
            for q in range(3):
                c.side[k].split[q] = sd.split[q] if c.side[k].front else 0.0
    return c


_lib = None


class MrError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"mrhweno status {status}: {msg}")
        self.status = status


def lib():
    """Load libmrhweno.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
        L = C.CDLL(LIB_PATH)
        vp, PP = C.c_void_p, C.POINTER(MrProblem)
        L.mrhweno_workspace_bytes.argtypes = [PP, C.c_int]
        L.mrhweno_workspace_bytes.restype = C.c_size_t
        L.mrhweno_create.argtypes = [PP, C.c_int, C.POINTER(vp), vp, vp, C.POINTER(vp)]
        L.mrhweno_step.argtypes = [vp, C.c_int]
        L.mrhweno_sync.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_long)]
        L.mrhweno_set_time.argtypes = [vp, C.c_int, C.c_double, C.c_long]
        L.mrhweno_last_dt.argtypes = [vp, C.POINTER(C.c_double)]
        L.mrhweno_reconstruct.argtypes = [vp, C.c_int, vp, vp, vp]
        L.mrhweno_flag.argtypes = [vp, C.c_int, vp, vp, vp]
        L.mrhweno_residual.argtypes = [vp, C.c_int, vp, vp, vp]
        L.mrhweno_residual_noalloc.argtypes = [PP, vp, vp, vp, vp]
        L.mrhweno_set_launch.argtypes = [vp, C.c_int, C.c_int]
        L.mrhweno_profile.argtypes = [vp, C.c_int, C.POINTER(C.c_float), C.POINTER(C.c_int)]
        IP = C.POINTER(C.c_int)
        L.mrhweno_autotune.argtypes = [vp, IP, C.c_int, IP, C.c_int, C.c_int, IP, IP, C.POINTER(C.c_float)]
        L.mrhweno_set_indicator_launch.argtypes = [vp, C.c_int]
        L.mrhweno_autotune_indicator.argtypes = [vp, IP, C.c_int, C.c_int, IP, C.POINTER(C.c_float)]
        L.mrhweno_set_indicator.argtypes = [vp, vp, C.c_double, C.c_double]
        L.mrhweno_indicator.argtypes = [vp, C.c_int, vp, vp, vp]
        L.mrhweno_features.argtypes = [vp, C.c_int, vp, vp, C.c_int, vp]
        L.mrhweno_mlp_param_count.argtypes = []
        L.mrhweno_mlp_feature_count.argtypes = []
        L.mrhweno_mlp_cache_bytes.argtypes = [C.c_int]
        L.mrhweno_mlp_cache_bytes.restype = C.c_size_t
        LL = C.c_longlong
        L.mrhweno_mlp_gemm.argtypes = [vp, C.c_int, C.c_int, C.c_int, vp, LL, LL, vp, LL, LL, vp, LL, LL]
        L.mrhweno_mlp_forward.argtypes = [vp, vp, vp, vp, vp, C.c_int]
        L.mrhweno_mlp_backward.argtypes = [vp, vp, vp, vp, vp, vp, vp, C.c_int]
        L.mrhweno_mlp_adam.argtypes = [vp, vp, vp, vp, vp, vp, C.c_int, C.c_float, C.c_float, C.c_float,
                                       C.c_float]
        L.mrhweno_last_error.argtypes = [vp]
        L.mrhweno_last_error.restype = C.c_char_p
        L.mrhweno_destroy.argtypes = [vp]
        L.mrhweno_destroy.restype = None
        _lib = L
    return _lib


def _check(ctx, status: int) -> None:
    if status != OK:
        msg = lib().mrhweno_last_error(ctx)
        raise MrError(status, msg.decode() if msg else "")


def workspace_bytes(problems: Sequence[Problem]) -> int:
    arr = (MrProblem * len(problems))(*[to_c(p) for p in problems])
    return int(lib().mrhweno_workspace_bytes(arr, len(problems)))


def residual_noalloc(problem: Problem, U, R=None, flags=None, stream=None):
    """L(U) of one problem without a context or any allocation inside the
    library (mrhweno_residual_noalloc).  U, R: contiguous float64 CUDA
    tensors of shape problem.shape() (R allocated here if not given);
    flags: uint8 CUDA tensor of the grid's shape, or None.  Returns
    (R, flags)."""
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU: the MR-HWENO library runs on the device only")
    if U.dtype != torch.float64 or not U.is_cuda or not U.is_contiguous() or tuple(U.shape) != problem.shape():
        raise ValueError("U must be a contiguous float64 CUDA tensor of shape Problem.shape()")
    if R is None:
        R = torch.empty_like(U)
    st = stream if stream is not None else torch.cuda.current_stream()
    cp = to_c(problem)
    _check(None, lib().mrhweno_residual_noalloc(C.byref(cp), C.c_void_p(U.data_ptr()), C.c_void_p(R.data_ptr()),
                                                C.c_void_p(flags.data_ptr() if flags is not None else None),
                                                C.c_void_p(st.cuda_stream)))
    return R, flags


class Solver:
    """A batch of instances advanced together (mrhweno_create .. destroy).

    moments: list of float64 CUDA tensors, one per problem, with the layout
    Problem.shape(); they are read and written in place (the current state
    is handed back by sync())."""

    def __init__(self, problems: Sequence[Problem], moments, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the MR-HWENO library runs on the device only")
        self.problems = list(problems)
        self.moments = list(moments)
        for p, m in zip(self.problems, self.moments):
            if m.dtype != torch.float64 or not m.is_cuda or not m.is_contiguous() or tuple(m.shape) != p.shape():
                raise ValueError("moments must be contiguous float64 CUDA tensors of shape Problem.shape()")
        self.stream = stream if stream is not None else torch.cuda.Stream()
        n = len(self.problems)
        self._cp = (MrProblem * n)(*[to_c(p) for p in self.problems])
        nbytes = int(lib().mrhweno_workspace_bytes(self._cp, n))
        if nbytes == 0:
            raise MrError(ERR_INVALID_ARG, lib().mrhweno_last_error(None).decode())
        # 256-byte aligned device workspace owned by torch
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.moments[0].device)
        base = self._ws.data_ptr()
        self._ws_ptr = (base + 255) & ~255
        ptrs = (C.c_void_p * n)(*[m.data_ptr() for m in self.moments])
        ctx = C.c_void_p()
        torch.cuda.synchronize()
        _check(None, lib().mrhweno_create(self._cp, n, ptrs, C.c_void_p(self._ws_ptr),
                                          C.c_void_p(self.stream.cuda_stream), C.byref(ctx)))
        self.ctx = ctx

    def step(self, nsteps: int = 1) -> None:
        _check(self.ctx, lib().mrhweno_step(self.ctx, int(nsteps)))

    def sync(self, raise_on_error: bool = True) -> Tuple[List[float], List[int], int]:
        n = len(self.problems)
        t = (C.c_double * n)()
        s = (C.c_long * n)()
        st = lib().mrhweno_sync(self.ctx, t, s)
        if st != OK and (raise_on_error or st != ERR_NONPHYSICAL):
            _check(self.ctx, st)
        return list(t), list(s), st

    def set_time(self, instance: int, t: float, steps: int) -> None:
        _check(self.ctx, lib().mrhweno_set_time(self.ctx, instance, float(t), int(steps)))

    def last_dt(self) -> List[float]:
        n = len(self.problems)
        d = (C.c_double * n)()
        _check(self.ctx, lib().mrhweno_last_dt(self.ctx, d))
        return list(d)

    def set_launch(self, rows_2d: int, grid_2d: int = 0) -> None:
        _check(self.ctx, lib().mrhweno_set_launch(self.ctx, int(rows_2d), int(grid_2d)))

    def autotune(self, rows=(8, 16, 32, 64, 128), grids=(0,), reps: int = 3):
        """Time the candidate 2D launch shapes (state untouched) and apply the
        fastest; returns (rows, grid, ms)."""
        r = (C.c_int * len(rows))(*rows)
        g = (C.c_int * len(grids))(*grids)
        br, bg, bm = C.c_int(), C.c_int(), C.c_float()
        _check(self.ctx, lib().mrhweno_autotune(self.ctx, r, len(rows), g, len(grids), int(reps),
                                                C.byref(br), C.byref(bg), C.byref(bm)))
        return br.value, bg.value, bm.value

    def set_indicator_launch(self, rows: int) -> None:
        """Flag rows per work item of the 2D KXRCF pass (0: chosen per problem)."""
        _check(self.ctx, lib().mrhweno_set_indicator_launch(self.ctx, int(rows)))

    def autotune_indicator(self, rows=(0, 8, 16, 24, 32, 46, 64, 96, 140), reps: int = 3):
        """Time the candidate KXRCF strip heights (0: the height chosen per
        problem; state untouched) and apply the fastest; returns (rows, ms)."""
        r = (C.c_int * len(rows))(*rows)
        br, bm = C.c_int(), C.c_float()
        _check(self.ctx, lib().mrhweno_autotune_indicator(self.ctx, r, len(rows), int(reps), C.byref(br), C.byref(bm)))
        return br.value, bm.value

    def profile(self, nsteps: int):
        """Advance nsteps with per-kernel-class HIP event timing.  Returns
        (ms[4], launches[4]) for [reduce/dt, summary, flags, stage]."""
        ms = (C.c_float * 4)()
        nl = (C.c_int * 4)()
        _check(self.ctx, lib().mrhweno_profile(self.ctx, int(nsteps), ms, nl))
        return list(ms), list(nl)

    # -------------------------------------------------------------- probes
    def reconstruct(self, instance: int, U):
        import torch
        torch.cuda.synchronize()
        p = self.problems[instance]
        npt = 4 if p.dim == 1 else 16
        gl = torch.empty((p.ncomp, npt) + p.shape()[2:], dtype=torch.float64, device=U.device)
        fl = torch.empty(p.shape()[2:], dtype=torch.uint8, device=U.device)
        _check(self.ctx, lib().mrhweno_reconstruct(self.ctx, instance, C.c_void_p(U.data_ptr()),
                                                   C.c_void_p(gl.data_ptr()), C.c_void_p(fl.data_ptr())))
        return gl, fl

    def flag(self, instance: int, U):
        import torch
        torch.cuda.synchronize()
        p = self.problems[instance]
        fl = torch.empty(p.shape()[2:], dtype=torch.uint8, device=U.device)
        # the KXRCF ratio (numerator, denominator) exists for KXRCF instances only
        al = (torch.empty(p.shape()[2:] + (2,), dtype=torch.float64, device=U.device)
              if p.tc_mode == TC_KXRCF else None)
        _check(self.ctx, lib().mrhweno_flag(self.ctx, instance, C.c_void_p(U.data_ptr()),
                                            C.c_void_p(fl.data_ptr()),
                                            C.c_void_p(al.data_ptr() if al is not None else None)))
        return fl, al

    def residual(self, instance: int, U):
        import torch
        torch.cuda.synchronize()
        p = self.problems[instance]
        R = torch.empty(p.shape(), dtype=torch.float64, device=U.device)
        fl = torch.empty(p.shape()[2:], dtype=torch.uint8, device=U.device)
        _check(self.ctx, lib().mrhweno_residual(self.ctx, instance, C.c_void_p(U.data_ptr()),
                                                C.c_void_p(R.data_ptr()), C.c_void_p(fl.data_ptr())))
        return R, fl

    # ---------------------------------------------------- learned indicator
    def set_indicator(self, params, band_lo: float = 0.2, band_hi: float = 0.8) -> None:
        """params: BF16 CUDA tensor of MLP_PARAMS entries."""
        import torch
        if params.dtype != torch.bfloat16 or not params.is_cuda or params.numel() != MLP_PARAMS:
            raise ValueError("params must be a bfloat16 CUDA tensor of MLP_PARAMS entries")
        params = params.contiguous()
        torch.cuda.synchronize()
        _check(self.ctx, lib().mrhweno_set_indicator(self.ctx, C.c_void_p(params.data_ptr()),
                                                     float(band_lo), float(band_hi)))

    def indicator(self, instance: int, U):
        """(decision, flags): network decision 0/1/2 (2 = left to KXRCF) and
        the final troubled-cell map, both uint8 [ny][nx]."""
        import torch
        torch.cuda.synchronize()
        p = self.problems[instance]
        dec = torch.empty(p.shape()[2:], dtype=torch.uint8, device=U.device)
        fl = torch.empty(p.shape()[2:], dtype=torch.uint8, device=U.device)
        _check(self.ctx, lib().mrhweno_indicator(self.ctx, instance, C.c_void_p(U.data_ptr()),
                                                 C.c_void_p(dec.data_ptr()), C.c_void_p(fl.data_ptr())))
        return dec, fl

    def features(self, instance: int, U, cells):
        """BF16 [n][MLP_FEATURES] features of the interior cells `cells`
        (int32 CUDA tensor of indices j*nx + i)."""
        import torch
        torch.cuda.synchronize()
        cells = cells.to(torch.int32).contiguous()
        out = torch.empty((cells.numel(), MLP_FEATURES), dtype=torch.bfloat16, device=U.device)
        _check(self.ctx, lib().mrhweno_features(self.ctx, instance, C.c_void_p(U.data_ptr()),
                                                C.c_void_p(cells.data_ptr()), int(cells.numel()),
                                                C.c_void_p(out.data_ptr())))
        return out

    def close(self) -> None:
        if getattr(self, "ctx", None):
            lib().mrhweno_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ training
def _stream_ptr(stream) -> C.c_void_p:
    import torch
    st = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(st.cuda_stream)


def mlp_cache_bytes(batch: int) -> int:
    return int(lib().mrhweno_mlp_cache_bytes(int(batch)))


def mlp_gemm(A, B, stream=None):
    """C = A @ B for 2D bfloat16 CUDA tensors (any strides) on the library's
    MFMA GEMM; returns a float32 tensor."""
    import torch
    M, K = A.shape
    K2, N = B.shape
    if K != K2 or A.dtype != torch.bfloat16 or B.dtype != torch.bfloat16:
        raise ValueError("bf16 operands with matching inner dimension required")
    Cm = torch.empty((M, N), dtype=torch.float32, device=A.device)
    _check(None, lib().mrhweno_mlp_gemm(_stream_ptr(stream), M, N, K,
                                        C.c_void_p(A.data_ptr()), A.stride(0), A.stride(1),
                                        C.c_void_p(B.data_ptr()), B.stride(0), B.stride(1),
                                        C.c_void_p(Cm.data_ptr()), Cm.stride(0), Cm.stride(1)))
    return Cm


def mlp_forward(x, params, cache, z, stream=None) -> None:
    _check(None, lib().mrhweno_mlp_forward(_stream_ptr(stream), C.c_void_p(x.data_ptr()),
                                           C.c_void_p(params.data_ptr()), C.c_void_p(cache.data_ptr()),
                                           C.c_void_p(z.data_ptr()), int(x.shape[0])))


def mlp_backward(x, params, cache, labels, grads, loss, stream=None) -> None:
    _check(None, lib().mrhweno_mlp_backward(_stream_ptr(stream), C.c_void_p(x.data_ptr()),
                                            C.c_void_p(params.data_ptr()), C.c_void_p(cache.data_ptr()),
                                            C.c_void_p(labels.data_ptr()), C.c_void_p(grads.data_ptr()),
                                            C.c_void_p(loss.data_ptr()), int(x.shape[0])))


def mlp_adam(master, params, grads, m, v, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
             eps: float = 1e-8, stream=None) -> None:
    _check(None, lib().mrhweno_mlp_adam(_stream_ptr(stream), C.c_void_p(master.data_ptr()),
                                        C.c_void_p(params.data_ptr()), C.c_void_p(grads.data_ptr()),
                                        C.c_void_p(m.data_ptr()), C.c_void_p(v.data_ptr()), int(step),
                                        float(lr), float(beta1), float(beta2), float(eps)))
