"""Comparison helpers for the GPU-vs-oracle parity tests."""
import json
import os

import numpy as np


def comp_scale(prob, U):
    """Per-component scale max_i |ubar_c,i| (the zeroth-moment magnitude)."""
    U = np.asarray(U)
    return np.abs(U[:, 0]).reshape(prob.ncomp, -1).max(axis=1)


def rel_state_err(prob, got, ref, scale):
    d = np.abs(np.asarray(got) - np.asarray(ref)).reshape(prob.ncomp, -1).max(axis=1)
    return float((d / scale).max())


# per-step bar of the FP64 values: within TOL of the component's scale
TOL = 1e-12

# Parity cases whose troubled-cell maps were measured to differ from the
# oracle's (every such cell inside the rounding band); every other case must
# match bit for bit.
MISMATCHES_ALLOWED = {}


def kxrcf_band(prob, scale0):
    """Width of the rounding band of the KXRCF test |J| > h^2 |dI^-| ||u||
    implied by Gauss-Lobatto values that agree to TOL * scale0 (the value bar
    of the indicator variable): J is a sum over the inflow faces of the face
    length times GL-weighted jumps (weights sum to 1), so each face moves J
    by at most 2 delta times its length and the denominator moves by at most
    h^2 |dI^-| delta.  A flag can differ between two evaluations only where
    |num - den| is within (2 + h^2) delta |dI^-|, |dI^-| <= 2 (dx + dy) in 2D
    (1D: no length, two faces: (4 + h^2) delta)."""
    h = prob.dx
    delta = TOL * scale0
    if prob.dim == 1:
        return (4.0 + h * h) * delta
    return (2.0 + h * h) * delta * 2.0 * (prob.dx + prob.dy)


def flag_report(tag, fl_gpu, fl_orc, in_band):
    """Count the cells whose troubled-cell flags differ, print the counts as
    one `FLAGS {json}` line (appended to the file named by MRHWENO_FLAG_LOG
    when set) and return (mismatches, mismatches outside the rounding
    band)."""
    a = np.asarray(fl_gpu).astype(bool)
    b = np.asarray(fl_orc).astype(bool)
    diff = a != b
    rec = {"case": tag, "cells": int(diff.size), "gpu_flagged": int(a.sum()), "oracle_flagged": int(b.sum()),
           "mismatches": int(diff.sum()), "outside_band": int((diff & ~in_band).sum()),
           "cells_in_band": int(np.asarray(in_band).sum())}
    line = "FLAGS " + json.dumps(rec)
    print(line, flush=True)
    path = os.environ.get("MRHWENO_FLAG_LOG")
    if path:
        with open(path, "a") as f:
            f.write(line + "\n")
    return rec["mismatches"], rec["outside_band"]


def kxrcf_flags(tag, prob, fl_gpu, fl_orc, num, den, scale0):
    """flag_report for the KXRCF test, band from kxrcf_band."""
    band = np.abs(np.asarray(num) - np.asarray(den)) <= kxrcf_band(prob, scale0)
    return flag_report(tag, fl_gpu, fl_orc, band)


def tvb_tie_map(prob, U, gl, margin=TOL):
    """Cells whose TVB minmod verdict sits within rounding of a threshold:
    a face deviation within `margin` (relative to the average's scale, the
    value bar) of
    M h^2, of a neighbouring difference, or of zero, or a difference within
    it of zero.  Recomputed here from the oracle's Gauss-Lobatto values of
    the indicator variable (component 0) and the cell averages."""
    U = np.asarray(U)
    ub = U[0, 0]
    scale = np.abs(ub).max()
    eps = margin * scale
    mh2 = prob.tvb_m * prob.dx * prob.dx
    g = np.asarray(gl)[0]
    w = np.array([1.0, 5.0, 5.0, 1.0]) / 12.0
    wrap = prob.bc_x == 0

    def nb(a, shift, axis):
        # neighbour averages with the boundary rule (periodic wrap or copy)
        if wrap:
            return np.roll(a, -shift, axis=axis)
        idx = np.clip(np.arange(a.shape[axis]) + shift, 0, a.shape[axis] - 1)
        return np.take(a, idx, axis=axis)

    pairs = []
    if prob.dim == 1:
        dp, dm = nb(ub, 1, 0) - ub, ub - nb(ub, -1, 0)
        pairs += [(g[3] - ub, dp, dm), (ub - g[0], dp, dm)]
    else:
        fl = sum(w[m] * g[4 * m] for m in range(4))
        fr = sum(w[m] * g[3 + 4 * m] for m in range(4))
        fb = sum(w[m] * g[m] for m in range(4))
        ft = sum(w[m] * g[12 + m] for m in range(4))
        dpx, dmx = nb(ub, 1, 1) - ub, ub - nb(ub, -1, 1)
        dpy, dmy = nb(ub, 1, 0) - ub, ub - nb(ub, -1, 0)
        pairs += [(fr - ub, dpx, dmx), (ub - fl, dpx, dmx), (ft - ub, dpy, dmy), (ub - fb, dpy, dmy)]
    tie = np.zeros(ub.shape, dtype=bool)
    for a, dp, dm in pairs:
        tie |= np.abs(np.abs(a) - mh2) <= eps
        tie |= (np.abs(np.abs(a) - np.abs(dp)) <= eps) | (np.abs(np.abs(a) - np.abs(dm)) <= eps)
        tie |= (np.abs(a) <= eps) | (np.abs(dp) <= eps) | (np.abs(dm) <= eps)
    return tie
