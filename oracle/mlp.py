"""TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT PATH.

Plain FP64 numpy reference of the learned troubled-cell indicator (an
addition to the paper's method, which flags troubled cells with KXRCF,
eq. (KXRCF_)): the feature vector of a cell, the network's forward pass, the
gradient of the mean binary cross-entropy, and one Adam step.  Written from
the definition of the indicator, independently of the GPU kernels; only the
tests may import it.

Feature definition.  For cell (i, j) of a 2D Euler state, moment m in
{0, 1, 2} (cell average, x and y first moments) of component c in
{rho, rho u, rho v, E} at cell (i + wx, j + wy), |wx|, |wy| <= 2, becomes

    (raw - [m == 0] * centre_c) / norm_c,

with centre_c the cell's own average of component c and norm_rho = rho,
norm_(rho u) = norm_(rho v) = rho * c (c the sound speed of the cell
average), norm_E = E.  One more feature is log2(h)/16.  Each feature has a
fixed position in a vector of 320 (the rest zero): window rows wy = -2..1
belong to lane group g = wy + 2 and slot s = 15 c + 5 m + (wx + 2); window
row wy = 2 belongs to lane group g = c and slot s = 60 + 5 m + (wx + 2);
log2(h)/16 is lane group 0, slot 75; the position is
f = 32 (s // 8) + 8 g + (s % 8).  Ghost cells follow the solver's boundary
conditions: periodic wrap, or (transmissive) the nearest interior cell's
average with zero first moments, or (reflective) the mirror image with the
wall-normal momentum and the first moment along the normal flipped.

Network: z = W3 . relu(W2 relu(W1 x + b1) + b2) + b3, score sigmoid(z);
parameter vector W1 [64][320], b1 [64], W2 [64][64], b2 [64], W3 [64], b3,
7 padding zeros (24776 entries).  Loss: mean over the batch of
log(1 + exp(-|z|)) + max(z, 0) - y z.

Parity pinned by tests/test_oracle_mlp.py: closed-form features of
hand-built states, invariance of the features under scaling of the state,
mirror symmetry, a forward pass computed by hand, central finite
differences of the loss for the gradient, and Adam's first step.
"""
from __future__ import annotations

import math
from typing import Dict, Tuple

import numpy as np

NF = 301
KP = 320
NH = 64
OFF = {"W1": 0, "b1": NH * KP}
OFF["W2"] = OFF["b1"] + NH
OFF["b2"] = OFF["W2"] + NH * NH
OFF["W3"] = OFF["b2"] + NH
OFF["b3"] = OFF["W3"] + NH
NPARAM = OFF["b3"] + 8


def feature_index(c: int, m: int, wx: int, wy: int) -> int:
    """Position of the (component, moment, offset) feature in the vector."""
    if wy < 2:
        g, s = wy + 2, 15 * c + 5 * m + (wx + 2)
    else:
        g, s = c, 60 + 5 * m + (wx + 2)
    return 32 * (s // 8) + 8 * g + (s % 8)


LOGH_INDEX = 32 * (75 // 8) + 8 * 0 + 75 % 8


def _moment(prob, U, c: int, m: int, i: int, j: int) -> float:
    """Moment m of component c at cell (i, j), ghosts by the boundary rule
    (periodic wrap; transmissive: nearest average, first moments zero;
    reflective: mirror image, the wall-normal momentum and the first moment
    along the normal flip)."""
    ii, jj, ghost, flip = i, j, False, False
    if not 0 <= ii < prob.nx:
        if prob.bc_x == 0:
            ii %= prob.nx
        elif prob.bc_x == 1:
            ii, ghost = min(max(ii, 0), prob.nx - 1), True
        else:
            ii = -1 - ii if ii < 0 else 2 * prob.nx - 1 - ii
            flip ^= (c == 1) != (m == 1)
    if not 0 <= jj < prob.ny:
        if prob.bc_y == 0:
            jj %= prob.ny
        elif prob.bc_y == 1:
            jj, ghost = min(max(jj, 0), prob.ny - 1), True
        else:
            jj = -1 - jj if jj < 0 else 2 * prob.ny - 1 - jj
            flip ^= (c == 2) != (m == 2)
    if ghost and m > 0:
        return 0.0
    v = float(U[c, m, jj, ii])
    return -v if flip else v


def features(prob, U, cells) -> np.ndarray:
    """FP64 features [n][320] of interior cells (indices j*nx + i)."""
    U = np.asarray(U, dtype=np.float64).reshape(prob.shape())
    cells = np.asarray(cells).ravel()
    out = np.zeros((cells.size, KP))
    for n, cell in enumerate(cells):
        i, j = int(cell) % prob.nx, int(cell) // prob.nx
        rho, mx, my, E = (float(U[c, 0, j, i]) for c in range(4))
        p = (prob.gamma - 1.0) * (E - 0.5 * (mx * mx + my * my) / rho)
        snd = math.sqrt(prob.gamma * p / rho)
        centre = (rho, mx, my, E)
        norm = (rho, rho * snd, rho * snd, E)
        for c in range(4):
            for m in range(3):
                for wy in range(-2, 3):
                    for wx in range(-2, 3):
                        raw = _moment(prob, U, c, m, i + wx, j + wy)
                        if m == 0:
                            raw -= centre[c]
                        out[n, feature_index(c, m, wx, wy)] = raw / norm[c]
        out[n, LOGH_INDEX] = math.log2(prob.dx) / 16.0
    return out


def unpack(P) -> Dict[str, np.ndarray]:
    P = np.asarray(P, dtype=np.float64)
    return {"W1": P[OFF["W1"]:OFF["b1"]].reshape(NH, KP), "b1": P[OFF["b1"]:OFF["W2"]],
            "W2": P[OFF["W2"]:OFF["b2"]].reshape(NH, NH), "b2": P[OFF["b2"]:OFF["W3"]],
            "W3": P[OFF["W3"]:OFF["b3"]], "b3": P[OFF["b3"]]}


def forward(X, P, bf16_hidden: bool = False) -> Tuple[np.ndarray, Dict[str, np.ndarray]]:
    """Logits z [B] and the intermediate activations.  bf16_hidden rounds
    the first hidden layer's output to BF16, the precision in which the
    network hands it to the second layer."""
    X = np.asarray(X, dtype=np.float64)
    w = unpack(P)
    a1 = X @ w["W1"].T + w["b1"]
    h1 = np.maximum(a1, 0.0)
    if bf16_hidden:
        h1 = bf16_round(h1)
    a2 = h1 @ w["W2"].T + w["b2"]
    h2 = np.maximum(a2, 0.0)
    z = h2 @ w["W3"] + w["b3"]
    return z, {"a1": a1, "h1": h1, "a2": a2, "h2": h2}


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-np.asarray(z, dtype=np.float64)))


def bce(z, y) -> np.ndarray:
    """Per-sample binary cross-entropy of logits z against labels y."""
    z = np.asarray(z, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    return np.log1p(np.exp(-np.abs(z))) + np.maximum(z, 0.0) - y * z


def loss(X, P, y, bf16_hidden: bool = False) -> float:
    z, _ = forward(X, P, bf16_hidden)
    return float(np.mean(bce(z, y)))


def gradient(X, P, y, bf16_hidden: bool = False) -> np.ndarray:
    """Gradient of the mean binary cross-entropy w.r.t. the parameter vector
    (chain rule through the three layers; with bf16_hidden the rounding of
    the first hidden layer counts as the identity)."""
    X = np.asarray(X, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    w = unpack(P)
    z, a = forward(X, P, bf16_hidden)
    B = X.shape[0]
    dz = (sigmoid(z) - y) / B                    # d loss / d z
    g = np.zeros(NPARAM)
    g[OFF["W3"]:OFF["b3"]] = a["h2"].T @ dz
    g[OFF["b3"]] = dz.sum()
    da2 = np.outer(dz, w["W3"]) * (a["a2"] > 0)  # through relu
    g[OFF["W2"]:OFF["b2"]] = (da2.T @ a["h1"]).ravel()
    g[OFF["b2"]:OFF["W3"]] = da2.sum(axis=0)
    da1 = (da2 @ w["W2"]) * (a["a1"] > 0)
    g[OFF["W1"]:OFF["b1"]] = (da1.T @ X).ravel()
    g[OFF["b1"]:OFF["W2"]] = da1.sum(axis=0)
    return g


def adam(w, g, m, v, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """One Adam step (Kingma and Ba, Algorithm 1); returns (w, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return w - lr * mhat / (np.sqrt(vhat) + eps), m, v


def bf16_round(x) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) >> 16 << 16
    return b.astype(np.uint32).view(np.float32).astype(np.float64)
