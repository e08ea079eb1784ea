"""Pins of the per-side boundary data (inflow sides, moving fronts) and of
the double Mach reflection set-up (Example 3.9), checked against the
Rankine-Hugoniot relations, brute-force integration and exact solutions."""
import math

import numpy as np
import pytest

import oracle
from paper_2201_12193_amd import inputs as I

GAMMA = 1.4


def _prim(u):
    rho = u[0]
    vel = np.asarray(u[1:-1]) / rho
    p = (GAMMA - 1.0) * (u[-1] - 0.5 * rho * float(np.dot(vel, vel)))
    return rho, vel, p


def test_mach_shock_states_satisfy_rankine_hugoniot():
    """Mass, momentum and energy fluxes agree on both sides of the shock in
    its own frame, and it moves at 10 times the sound speed of the gas
    ahead (which is 1)."""
    (r1, u1, p1), (r2, u2, p2), s = I.mach_shock_states(10.0, GAMMA)
    assert abs(math.sqrt(GAMMA * p1 / r1) - 1.0) < 1e-15 and s == 10.0
    w1, w2 = u1 - s, u2 - s
    assert abs(r1 * w1 - r2 * w2) <= 1e-13 * abs(r1 * w1)
    assert abs((r1 * w1 * w1 + p1) - (r2 * w2 * w2 + p2)) <= 1e-13 * (r1 * w1 * w1 + p1)
    h1 = GAMMA * p1 / ((GAMMA - 1.0) * r1) + 0.5 * w1 * w1
    h2 = GAMMA * p2 / ((GAMMA - 1.0) * r2) + 0.5 * w2 * w2
    assert abs(h1 - h2) <= 1e-13 * h1
    assert r2 > r1 and p2 > p1 and u2 > 0.0   # compressive, gas set moving behind it


@pytest.mark.parametrize("a,b,c", [(1.0, -0.577, 0.1), (0.025, -0.0144, 0.003), (1.0, 0.0, 0.2),
                                   (0.0, 1.0, -0.3), (1.0, 1.0, 0.0), (0.3, -0.9, 0.45),
                                   (-0.7, 0.2, 0.6), (1.0, -0.577, -0.9)])
def test_clipped_cell_moments_brute_force(a, b, c):
    """Area and first moments of the part of the reference cell below a line
    against a fine midpoint rule; the two parts add up to the whole cell."""
    n = 1200
    g = (np.arange(n) + 0.5) / n - 0.5
    X, Y = np.meshgrid(g, g)
    m = a * X + b * Y < c
    area, mx, my = I._clip_moments(a, b, c)
    assert abs(area - m.mean()) < 3e-3 and abs(mx - (X * m).mean()) < 1e-3 and abs(my - (Y * m).mean()) < 1e-3
    ca, cx, cy = I._clip_moments(-a, -b, -c)
    assert abs(area + ca - 1.0) < 1e-14 and abs(mx + cx) < 1e-14 and abs(my + cy) < 1e-14


def _exact_dmr(x, y, t):
    """Conserved state of the plane Mach 10 shock of the double Mach
    reflection at (x, y, t), from its geometry: through (1/6, 0) at t = 0,
    at 60 degrees to the x axis, moving along its normal (cos 30, -sin 30)
    at speed 10."""
    (r1, _, p1), (r2, un, p2), s = I.mach_shock_states(10.0, GAMMA)
    nxv, nyv = math.cos(math.pi / 6), -math.sin(math.pi / 6)
    # signed distance ahead of the shock along its normal
    d = (x - 1.0 / 6.0) * nxv + y * nyv - s * t
    post = I.euler2d_cons(np.array(r2), np.array(un * nxv), np.array(un * nyv), np.array(p2), GAMMA)
    pre = I.euler2d_cons(np.array(r1), np.array(0.0), np.array(0.0), np.array(p1), GAMMA)
    d = np.asarray(d, dtype=float)
    sh = (4,) + (1,) * d.ndim
    return np.where(d < 0.0, np.asarray(post, dtype=float).reshape(sh), np.asarray(pre, dtype=float).reshape(sh))


def test_double_mach_initial_moments_exact():
    """Cells cut by the initial shock hold the moments of the exact
    piecewise-constant data (fine midpoint rule per cell)."""
    prob, U = I.double_mach_2d(ny=8)
    n = 400
    g = (np.arange(n) + 0.5) / n - 0.5
    Xi, Eta = np.meshgrid(g, g)
    checked = 0
    for j in range(prob.ny):
        for i in range(prob.nx):
            xc, yc = (i + 0.5) * prob.dx, (j + 0.5) * prob.dy
            rho = np.where((xc + Xi * prob.dx - 1 / 6) * math.cos(math.pi / 6)
                           - (yc + Eta * prob.dy) * math.sin(math.pi / 6) < 0, 1.0, 0.0)
            if 0.0 < rho.mean() < 1.0:
                post = _exact_dmr(0.0, 0.0, 0.0)
                pre = _exact_dmr(3.9, 0.0, 0.0)
                for c in range(4):
                    f = pre[c] + (post[c] - pre[c]) * rho
                    sc = abs(post[c] - pre[c]) + 1.0
                    assert abs(U[c, 0, j, i] - f.mean()) < 5e-3 * sc
                    assert abs(U[c, 1, j, i] - (f * Xi).mean()) < 2e-3 * sc
                    assert abs(U[c, 2, j, i] - (f * Eta).mean()) < 2e-3 * sc
                checked += 1
            else:
                ref = _exact_dmr(xc, yc, 0.0)
                assert np.all(U[:, 0, j, i] == ref) and np.all(U[:, 1:, j, i] == 0.0)
    assert checked >= 8


@pytest.mark.parametrize("t", [0.0, 0.0137, 0.05])
def test_double_mach_ghosts_follow_the_exact_shock(t):
    """Ghost cells of Example 3.9 at time t: along the top the moments of
    the exact moving shock over each ghost cell (a fine midpoint rule; cells
    the shock does not cut hold a constant state exactly); along the bottom
    the post-shock state left of x = 1/6 and the mirror image beyond;
    post-shock inflow on the left; zero-gradient on the right."""
    prob, U = I.double_mach_2d(ny=10)
    rng = np.random.default_rng(5)
    V = U * (1.0 + 0.01 * rng.standard_normal(U.shape))   # interior values distinguishable
    nx, ny, h = prob.nx, prob.ny, prob.dx
    nq = 200
    g = (np.arange(nq) + 0.5) / nq - 0.5
    Xi, Eta = np.meshgrid(g, g)
    cut = 0
    for j in range(ny, ny + 4):                       # top
        for i in range(-4, nx + 4):
            xc, yc = (i + 0.5) * h, (j + 0.5) * h
            W = _exact_dmr(xc + Xi * h, yc + Eta * h, t)
            for c in range(4):
                got = [oracle.moment(prob, V, c, m, i, j, t) for m in range(3)]
                ref = [W[c].mean(), (W[c] * Xi).mean(), (W[c] * Eta).mean()]
                if W[c].min() == W[c].max():
                    assert got == [W[c, 0, 0], 0.0, 0.0]
                else:
                    sc = W[c].max() - W[c].min()
                    assert all(abs(a - b) < 1e-2 * sc / nq * 4 for a, b in zip(got, ref)), (i, j, c, got, ref)
                    cut += c == 0
    assert cut >= 4
    post = _exact_dmr(0.0, 0.0, 0.0)
    for j in range(-4, 0):                            # bottom
        for i in range(-4, nx + 4):
            xc = (i + 0.5) * h
            if xc < 1.0 / 6.0:
                for c in range(4):
                    assert oracle.moment(prob, V, c, 0, i, j, t) == post[c]
                    assert oracle.moment(prob, V, c, 2, i, j, t) == 0.0
            elif 0 <= i < nx:
                jj = -1 - j
                for c in range(4):
                    for m in range(3):
                        flip = (c == 2) != (m == 2)
                        ref = V[c, m, jj, i] * (-1.0 if flip else 1.0)
                        assert oracle.moment(prob, V, c, m, i, j, t) == ref
    for j in range(0, ny):                            # left and right
        for k in range(1, 5):
            for c in range(4):
                assert oracle.moment(prob, V, c, 0, -k, j, t) == post[c]
                assert oracle.moment(prob, V, c, 1, -k, j, t) == 0.0
                assert oracle.moment(prob, V, c, 0, nx - 1 + k, j, t) == V[c, 0, j, nx - 1]
                assert oracle.moment(prob, V, c, 1, nx - 1 + k, j, t) == 0.0


def test_inflow_sides_preserve_free_stream():
    """A uniform flow along a wall, fed through inflow sides that prescribe
    that same state (with a moving front between two equal states), is an
    exact steady solution: L(U) vanishes at any time."""
    W = I.euler2d_cons(np.array(1.3), np.array(0.7), np.array(0.0), np.array(2.0), GAMMA)
    W = tuple(float(z) for z in W)
    sides = (I.Side(kind=I.INFLOW, state=W), I.Side(kind=I.TRANSMISSIVE),
             I.Side(kind=I.REFLECTIVE, pre=W, split=(0.3, 0.5, 0.2)),
             I.Side(kind=I.INFLOW, state=W, pre=W, split=(0.2, 2.0, -0.1)))
    prob = I.Problem(dim=2, nx=24, ny=16, x0=0.0, x1=1.5, y0=0.0, y1=1.0, bc_x=I.SIDES, bc_y=I.SIDES,
                     sides=sides)
    U = np.zeros(prob.shape())
    U[:, 0] = np.array(W)[:, None, None]
    for t in (0.0, 0.1, 0.37):
        L, fl = oracle.residual(prob, U, t)
        assert np.abs(L).max() < 1e-12 and fl.sum() == 0
    W1 = tuple(float(z) for z in I.euler1d_cons(np.array(0.9), np.array(-0.4), np.array(1.1), GAMMA))
    p1 = I.Problem(dim=1, nx=40, bc_x=I.SIDES, sides=(I.Side(kind=I.INFLOW, state=W1),
                                                      I.Side(kind=I.INFLOW, state=W1), None, None))
    U1 = np.zeros(p1.shape())
    U1[:, 0] = np.array(W1)[:, None]
    L1, _ = oracle.residual(p1, U1)
    assert np.abs(L1).max() < 1e-12


def test_fronts_only_on_bottom_and_top():
    prob = I.Problem(dim=2, nx=16, ny=16, bc_x=I.SIDES, bc_y=I.PERIODIC,
                     sides=(I.Side(kind=I.INFLOW, state=(1, 0, 0, 2.5), split=(0.1, 0.0, 0.0)),
                            I.Side(), None, None))
    with pytest.raises(ValueError):
        oracle.residual(prob, np.zeros(prob.shape()))


def _plane_shock_box(n: int = 32, speed_scale: float = 1.0):
    """The Mach 10 plane shock of Example 3.9 crossing the unit square, all
    four sides prescribed by the exact solution: post-shock inflow on the
    left, pre-shock on the right, the exact front on bottom and top."""
    pd, Ud = I.double_mach_2d(ny=n)
    post, pre = pd.sides[0].state, pd.sides[3].state
    s3 = math.sqrt(3.0)
    front = (1.0 / 6.0, speed_scale * 20.0 / s3, 1.0 / s3)
    sides = (I.Side(kind=I.INFLOW, state=post), I.Side(kind=I.INFLOW, state=pre),
             I.Side(kind=I.INFLOW, state=pre, pre=post, split=front),
             I.Side(kind=I.INFLOW, state=pre, pre=post, split=front))
    prob = I.Problem(dim=2, nx=n, ny=n, x0=0.0, x1=1.0, y0=0.0, y1=1.0, bc_x=I.SIDES, bc_y=I.SIDES,
                     sides=sides, gamma=GAMMA)
    return prob, np.ascontiguousarray(Ud[:, :, :, :n])


def test_moving_front_mass_balance():
    """With exact data on every side the mass in the box follows the exact
    solution: rho_1 + (rho_2 - rho_1) * (area behind the shock), the shock
    being x = 1/6 + (y + 20 t)/sqrt(3).  A front that does not move is far
    off."""
    (r1, _, _), (r2, _, _), _ = I.mach_shock_states(10.0, GAMMA)
    errs = []
    for scale in (1.0, 0.0):
        prob, U = _plane_shock_box(32, scale)
        t = 0.0
        for _ in range(12):
            d = oracle.dt(prob, U)
            U = oracle.rk3_step(prob, U, d, t=t)
            t += d
        a = 1.0 / 6.0 + 20.0 * t / math.sqrt(3.0)
        assert a + 1.0 / math.sqrt(3.0) < 1.0          # the shock stays inside the box
        exact = r1 + (r2 - r1) * (a + 0.5 / math.sqrt(3.0))
        errs.append(abs(U[0, 0].mean() - exact) / exact)
    assert errs[0] < 5e-4 and errs[1] > 5 * errs[0]


def test_stage_times_of_the_rk3_step():
    """One SSP-RK3 step evaluates the boundary data at the stage times of
    its tableau (c = 0, 1, 1/2): it equals the step composed from single
    residual evaluations at t, t + dt and t + dt/2 (persisted
    modification), and differs from one with every stage at t."""
    prob, U = _plane_shock_box(16)
    d = oracle.dt(prob, U)
    # start a quarter step before the front passes the centre of a top
    # ghost cell, so that the stages see different ghost states
    h, s3 = prob.dx, math.sqrt(3.0)
    y = 1.0 + 0.5 * h
    xf = 1.0 / 6.0 + (y + 20.0 * 0.004) / s3
    xc = (math.floor(xf / h - 0.5) + 1.5) * h
    t0 = (s3 * (xc - 1.0 / 6.0) - y) / 20.0 - 0.25 * d

    def stage(V, t):
        L, fl = oracle.residual(prob, V, t)
        return L, oracle.modify(prob, V, fl, t)

    def composed(times):
        L, Ut = stage(U, times[0])
        Un = Ut
        U1 = Ut + d * L
        L, Ut = stage(U1, times[1])
        U2 = 3.0 / 4.0 * Un + 1.0 / 4.0 * Ut + 1.0 / 4.0 * d * L
        L, Ut = stage(U2, times[2])
        return 1.0 / 3.0 * Un + 2.0 / 3.0 * Ut + 2.0 / 3.0 * d * L

    got = oracle.rk3_step(prob, U, d, t=t0)
    scale = np.abs(U).max()
    assert np.abs(got - composed((t0, t0 + d, t0 + 0.5 * d))).max() <= 1e-14 * scale
    assert np.abs(got - composed((t0, t0, t0))).max() > 1e-6 * scale
