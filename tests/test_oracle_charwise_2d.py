"""Pins of the oracle's characteristic-wise Step 1 in 2D (Euler; the
paper reconstructs component by component, Sec. 2.2 Step 1; this is the
common alternative for systems): eigenvectors of the flux Jacobians checked
against a finite-difference Jacobian of the flux written here, exactness on
linear data, the x <-> y symmetry that exchanges the two sets of values,
free-stream preservation and the convergence order on the smooth 2D Euler
test of Example 3.4."""
import math

import numpy as np
import pytest

import oracle
from oracle import exact as X
from paper_2201_12193_amd import inputs as I

G = 1.4


def _cons(r, u, v, p, g=G):
    return np.array([r, r * u, r * v, p / (g - 1) + 0.5 * r * (u * u + v * v)])


def _flux(U, d, g=G):
    """2D Euler flux in direction d (0: x, 1: y) from conserved variables"""
    r, mu, mv, E = U
    u, v = mu / r, mv / r
    p = (g - 1) * (E - 0.5 * r * (u * u + v * v))
    vn = u if d == 0 else v
    f = np.array([r * vn, mu * vn, mv * vn, vn * (E + p)])
    f[1 + d] += p
    return f


def _jacobian(U, d, h=1e-6):
    J = np.zeros((4, 4))
    for k in range(4):
        e = np.zeros(4)
        e[k] = h * max(1.0, abs(U[k]))
        J[:, k] = (_flux(U + e, d) - _flux(U - e, d)) / (2 * e[k])
    return J


def test_charwise2d_eigenvectors_against_a_finite_difference_jacobian():
    """For random physical states and both directions: L R = I, and the
    columns of R (rows of L) are right (left) eigenvectors of the flux
    Jacobian with eigenvalues vn - c, vn, vn, vn + c."""
    rng = np.random.default_rng(8)
    for _ in range(8):
        r, u, v, p = rng.uniform(0.2, 2.0), rng.uniform(-1.5, 1.5), rng.uniform(-1.5, 1.5), rng.uniform(0.2, 2.0)
        U = _cons(r, u, v, p)
        c = math.sqrt(G * p / r)
        for d in (0, 1):
            L, R = oracle.euler2_eigen(U, G, d)
            assert np.abs(L @ R - np.eye(4)).max() < 1e-12
            A = _jacobian(U, d)
            vn = u if d == 0 else v
            lam = np.array([vn - c, vn, vn, vn + c])
            scale = np.abs(A).max()
            assert np.abs(A @ R - R * lam[None, :]).max() < 1e-7 * scale, d
            assert np.abs(L @ A - lam[:, None] * L).max() < 1e-7 * scale * np.abs(L).max(), d


def _linear_stencil(base, sx, sy):
    """moments of the linear conserved field base + sx xi + sy eta (reference
    coordinates of the centre cell) on the 3x3 stencil"""
    ub, vb, wb = np.zeros((4, 9)), np.zeros((4, 9)), np.zeros((4, 9))
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            k = (dx + 1) + 3 * (dy + 1)
            ub[:, k] = base + sx * dx + sy * dy
            vb[:, k] = sx / 12.0
            wb[:, k] = sy / 12.0
    return ub, vb, wb


def test_charwise2d_exact_on_linear_data():
    """The projections are linear and Step 1 reproduces linear data, so both
    sets of values of a linear conserved field are its exact point values."""
    prob = I.Problem(dim=2, nx=8, ny=8, charwise=1)
    base = _cons(1.0, 0.3, -0.2, 1.5)
    sx = np.array([0.05, 0.02, -0.01, 0.07])
    sy = np.array([-0.03, 0.01, 0.04, -0.02])
    ub, vb, wb = _linear_stencil(base, sx, sy)
    xn, _ = oracle.gl_rule()
    want = np.array([[base[c] + sx[c] * xn[k] + sy[c] * xn[l] for l in range(4) for k in range(4)] for c in range(4)])
    for d in (0, 1):
        got = oracle.step1_2d_sys(prob, ub, vb, wb, d)
        assert np.allclose(got, want, rtol=0, atol=1e-13), d


def test_charwise2d_sets_exchange_under_transposition():
    """Exchanging x and y (stencil transposed, momenta and first moments
    swapped) maps the y set of the transposed data onto the x set of the
    original, transposed: a slip in one direction's eigenvectors or in the
    assignment of the sets breaks it."""
    prob = I.Problem(dim=2, nx=8, ny=8, charwise=1)
    rng = np.random.default_rng(12)
    ub, vb, wb = np.zeros((4, 9)), np.zeros((4, 9)), np.zeros((4, 9))
    for k in range(9):
        ub[:, k] = _cons(rng.uniform(0.5, 1.5), rng.uniform(-0.5, 0.5), rng.uniform(-0.5, 0.5), rng.uniform(0.5, 1.5))
    vb = rng.uniform(-0.05, 0.05, (4, 9))
    wb = rng.uniform(-0.05, 0.05, (4, 9))
    gx = oracle.step1_2d_sys(prob, ub, vb, wb, 0)
    perm = [0, 2, 1, 3]
    T = lambda a: a.reshape(-1, 3, 3).transpose(0, 2, 1).reshape(-1, 9)
    gyt = oracle.step1_2d_sys(prob, T(ub)[perm], T(wb)[perm], T(vb)[perm], 1)
    want = gx.reshape(4, 4, 4).transpose(0, 2, 1).reshape(4, 16)[perm]
    assert np.allclose(gyt, want, rtol=0, atol=1e-13)
    # and the sets differ for such data (the characteristic fields depend on the direction)
    assert np.abs(oracle.step1_2d_sys(prob, ub, vb, wb, 1) - gx).max() > 1e-6


def test_charwise2d_free_stream():
    """A uniform state has zero residual with the characteristic-wise
    reconstruction too."""
    prob = I.Problem(dim=2, nx=12, ny=12, charwise=1)
    U = np.zeros(prob.shape())
    U[:, 0] = _cons(0.9, 0.4, -0.3, 1.2)[:, None, None]
    L, fl = oracle.residual(prob, U)
    assert np.abs(L).max() < 1e-13 and fl.sum() == 0


def test_charwise2d_smooth_order():
    """Example 3.4 (gamma = 3) with the characteristic-wise Step 1: high-order
    convergence on the simple-wave exact solution (short final time), like
    the component-wise reconstruction."""
    errs = []
    for n in (16, 32):
        prob, U = I.example_euler_2d(n)
        prob = prob.replace(t_final=0.5, charwise=1)
        V, _, _ = oracle.run(prob, U, dt_fn=lambda p, W: min(oracle.dt(p, W), 0.6 * (4 * math.pi / p.nx) ** 2 / 10))
        ex = I.cell_averages_2d(prob, lambda x, y: X.euler2d_gamma3(x, y, 0.5)[0])
        errs.append(np.abs(V[0, 0] - ex).mean())
    assert math.log2(errs[0] / errs[1]) > 4.5, errs
