"""The C-ABI library loads and exports every entry point include/mrhweno.h
declares; host-side argument validation works without a GPU."""
import ctypes as C
import math
import os
import re

import pytest

from paper_2201_12193_amd import inputs as I
from paper_2201_12193_amd import mrhweno as M

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "mrhweno.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mrhweno_[a-z_]+)\s*\(", src)))


def test_header_declares_the_binding_names():
    assert _declared() == sorted(M.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = M.lib()
    for name in _declared():
        assert hasattr(lib, name), name


def test_workspace_bytes_validates_problems():
    good = I.Problem(dim=2, nx=64, ny=64)
    assert M.workspace_bytes([good]) > 0
    dmr, _ = I.double_mach_2d(ny=16)
    W = dmr.sides[0].state
    bad = [I.Problem(dim=3, nx=64), I.Problem(dim=2, nx=4, ny=64), I.Problem(dim=2, nx=64, ny=32),
           good.replace(cfl=0.0), good.replace(gbar=(1, -1, 1, 1)), good.replace(eps=0.0),
           good.replace(tc_mode=7), I.Problem(dim=1, nx=64, gamma=1.0),
           good.replace(modification=3), good.replace(tvb_m=-1.0), good.replace(tvb_m=float("nan")),
           good.replace(charwise=1, tc_mode=I.TC_TVB),                 # 2D characteristic-wise: KXRCF/all/none
           good.replace(charwise=1, tc_mode=I.TC_LEARNED),
           I.Problem(dim=1, nx=64, system=I.BURGERS, charwise=1), I.Problem(dim=1, nx=64, charwise=2),
           I.Problem(dim=1, nx=64, system=I.BURGERS, bc_x=I.REFLECTIVE), good.replace(bc_y=4),
           good.replace(bc_y=I.SIDES),                                  # side kinds left unset
           dmr.replace(sides=(I.Side(kind=I.INFLOW, state=W, split=(0.1, 0.0, 0.0)),) + dmr.sides[1:]),
           dmr.replace(sides=dmr.sides[:3] + (I.Side(kind=I.INFLOW, state=(1.0, 0.0, 0.0, -1.0)),)),
           dmr.replace(sides=dmr.sides[:2] + (I.Side(kind=I.REFLECTIVE, pre=W, split=(0.1, math.inf, 0.0)),)
                       + dmr.sides[3:]),
           dmr.replace(tc_mode=I.TC_LEARNED),                           # no per-side data with it
           I.Problem(dim=1, nx=64, system=I.BURGERS, bc_x=I.SIDES,
                     sides=(I.Side(kind=I.REFLECTIVE), I.Side(), None, None)),
           I.Problem(dim=1, nx=64, step_i=8, step_j=4),                    # a step is 2D Euler
           good.replace(system=I.BURGERS, step_i=20, step_j=8),
           good.replace(step_i=20, step_j=24),                             # step_j > step_i
           good.replace(step_i=40, step_j=33),                             # mirror rows leave the grid
           good.replace(step_i=64, step_j=8),                              # step_i < nx
           good.replace(step_i=0, step_j=8), good.replace(step_i=20, step_j=-2),
           good.replace(step_i=20, step_j=8, tc_mode=I.TC_TVB),
           good.replace(step_i=20, step_j=8, tc_mode=I.TC_LEARNED),
           good.replace(wall_flux=2), I.Problem(dim=1, nx=64, wall_flux=1),
           good.replace(system=I.BURGERS, wall_flux=1)]
    assert M.workspace_bytes([dmr]) > 0
    assert M.workspace_bytes([good.replace(charwise=1)]) > 0                  # 2D Euler, KXRCF
    step, _ = I.forward_step(ny=20)
    assert M.workspace_bytes([step]) > 0 and M.workspace_bytes([step.replace(charwise=1, tc_mode=I.TC_ALL)]) > 0
    assert M.workspace_bytes([good.replace(step_i=32, step_j=32)]) > 0       # step_j = step_i, 2 step_j = ny
    for b in bad:
        assert M.workspace_bytes([b]) == 0, b
    assert M.workspace_bytes([good, bad[0]]) == 0
    # the workspace grows with the batch
    assert M.workspace_bytes([good, good]) > M.workspace_bytes([good])


def test_create_rejects_bad_arguments_on_the_host():
    lib = M.lib()
    ctx = C.c_void_p()
    p = (M.MrProblem * 1)(M.to_c(I.Problem(dim=1, nx=64)))
    st = lib.mrhweno_create(p, 1, None, None, None, C.byref(ctx))
    assert st == M.ERR_INVALID_ARG and not ctx.value
    assert b"NULL" in lib.mrhweno_last_error(None)
    ptrs = (C.c_void_p * 1)(C.c_void_p(0x1000))
    st = lib.mrhweno_create(p, 1, ptrs, C.c_void_p(0x1001), None, C.byref(ctx))   # misaligned workspace
    assert st == M.ERR_INVALID_ARG
    assert lib.mrhweno_step(None, 1) == M.ERR_INVALID_ARG
