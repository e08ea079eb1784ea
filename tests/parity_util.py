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
