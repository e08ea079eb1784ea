"""Comparison helpers for the GPU-vs-oracle parity tests."""
import numpy as np


def comp_scale(prob, U):
    """Per-component scale max_i |ubar_c,i| (the zeroth-moment magnitude)."""
    U = np.asarray(U)
    return np.abs(U[:, 0]).reshape(prob.ncomp, -1).max(axis=1)


def rel_state_err(prob, got, ref, scale):
    d = np.abs(np.asarray(got) - np.asarray(ref)).reshape(prob.ncomp, -1).max(axis=1)
    return float((d / scale).max())


def flag_mismatch(fl_gpu, fl_orc, num, den, margin=1e-9):
    """Cells where the flags differ, split into genuine mismatches and
    near-ties (|J| within `margin` of the threshold, where rounding decides)."""
    fl_gpu = np.asarray(fl_gpu).astype(bool)
    fl_orc = np.asarray(fl_orc).astype(bool)
    diff = fl_gpu != fl_orc
    tie = np.abs(num - den) <= margin * np.maximum(den, 1e-300)
    return int((diff & ~tie).sum()), int((diff & tie).sum())


def tvb_tie_map(prob, U, gl, margin=1e-9):
    """Cells whose TVB minmod verdict sits within rounding of a threshold:
    a face deviation within `margin` (relative to the average's scale) of
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
