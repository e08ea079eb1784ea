"""Pins of the oracle's forward step (Example 3.10) and of its wall flux
(readings R19 and R20 of the oracle header).

The wall flux -- the Godunov flux of the mirror-image Riemann problem --
is checked against what fixes it independently of its closed form: the
Rankine-Hugoniot relations of the reflected shock (mass and momentum across
a shock whose speed follows from mass conservation), the Riemann invariant
of the reflected rarefaction, vacuum, and gas at rest.  The step's mirror
images are checked against tunnels without a step whose data are mirrored
by hand across the step's face: away from the corner, the residual of every
cell whose dependency cone sees only one face of the step must be that of
the mirrored tunnel."""
import math

import numpy as np
import pytest

import oracle
from paper_2201_12193_amd import inputs as I

G = 1.4


def _cons(r, u, v, p, g=G):
    return np.array([r, r * u, r * v, p / (g - 1) + 0.5 * r * (u * u + v * v)])


def _p(U, g=G):
    return (g - 1) * (U[3] - 0.5 * (U[1] ** 2 + U[2] ** 2) / U[0])


@pytest.mark.parametrize("d", [0, 1])
@pytest.mark.parametrize("sgn", [1, -1])
def test_wall_flux_of_gas_at_rest_is_its_pressure(d, sgn):
    f = oracle.wall_flux(_cons(1.3, 0.0, 0.0, 0.7), G, d, sgn)
    want = np.zeros(4)
    want[1 + d] = 0.7
    assert np.array_equal(f, want)


@pytest.mark.parametrize("mach", [0.01, 0.5, 2.0, 3.0, 10.0])
def test_wall_flux_reflected_shock_satisfies_rankine_hugoniot(mach):
    """Gas of Mach number `mach` into a wall: the star pressure p* is that
    behind a reflected shock with the gas at rest.  Post-shock density from
    the Hugoniot, shock speed from mass conservation; momentum must then
    balance across the shock."""
    r, p = 1.4, 1.0
    c = math.sqrt(G * p / r)
    u = mach * c
    f = oracle.wall_flux(_cons(r, u, 0.0, p), G, 0, 1)
    ps = f[1]
    assert f[0] == 0.0 and f[2] == 0.0 and f[3] == 0.0
    rs = r * ((G + 1) * ps + (G - 1) * p) / ((G - 1) * ps + (G + 1) * p)
    S = -r * u / (rs - r)                       # shock speed: rho (u - S) = rho* (0 - S)
    assert S < 0.0                              # it moves away from the wall
    mom = p + r * u * (u - S)                   # p + rho u (u - S) = p* + rho* 0 (0 - S)
    assert abs(ps - mom) <= 1e-13 * ps
    # energy across the shock: rho (u - S) (e + (u - S)^2 / 2) + p (u - S) = ...
    e, es = p / ((G - 1) * r), ps / ((G - 1) * rs)
    lhs = r * (u - S) * (e + 0.5 * (u - S) ** 2) + p * (u - S)
    rhs = rs * (0 - S) * (es + 0.5 * S * S) + ps * (0 - S)
    assert abs(lhs - rhs) <= 1e-12 * abs(rhs)


@pytest.mark.parametrize("mach", [0.1, 1.0, 4.0])
def test_wall_flux_reflected_rarefaction_keeps_the_riemann_invariant(mach):
    """Gas leaving the wall: p* behind the rarefaction, isentropic, with the
    Riemann invariant u + 2c/(g-1) carried to the gas at rest."""
    r, p = 1.0, 2.0
    c = math.sqrt(G * p / r)
    u = -mach * c                               # velocity into the wall: negative
    ps = oracle.wall_flux(_cons(r, u, 0.0, p), G, 0, 1)[1]
    cs = c * (ps / p) ** ((G - 1) / (2 * G))
    assert abs((u + 2 * c / (G - 1)) - 2 * cs / (G - 1)) <= 1e-12 * c


def test_wall_flux_vacuum_and_mirror_direction():
    r, p = 1.0, 1.0
    c = math.sqrt(G * p / r)
    assert oracle.wall_flux(_cons(r, -5.1 * c, 0.0, p), G, 0, 1)[1] == 0.0   # beyond 2c/(g-1) = 5c
    U = _cons(1.2, 0.7, -0.4, 1.5)
    # the wall below (sgn -1, y faces) sees v = -0.4 as velocity into it, as
    # the wall to the right (x faces) sees u = 0.4 with the roles exchanged
    fy = oracle.wall_flux(U, G, 1, -1)
    fx = oracle.wall_flux(_cons(1.2, 0.4, 0.7, 1.5), G, 0, 1)
    assert fy[2] == fx[1] and fy[0] == fy[1] == fy[3] == 0.0


def _tunnel(nx, ny, si, sj, wall_flux=0, tc=I.TC_KXRCF, **kw):
    return I.Problem(dim=2, nx=nx, ny=ny, x0=0.0, x1=nx / ny, y0=0.0, y1=1.0, system=I.EULER,
                     bc_x=I.TRANSMISSIVE, bc_y=I.REFLECTIVE, tc_mode=tc, step_i=si, step_j=sj,
                     wall_flux=wall_flux, **kw)


def _random_state(prob, seed):
    rng = np.random.default_rng(seed)
    sh = (prob.ny, prob.nx)
    r = 1.0 + 0.3 * rng.random(sh)
    u, v = rng.uniform(-0.6, 0.6, sh), rng.uniform(-0.6, 0.6, sh)
    p = 1.0 + 0.3 * rng.random(sh)
    U = np.zeros(prob.shape())
    U[:, 0] = _cons(r, u, v, p)
    U[:, 1:] = rng.uniform(-0.05, 0.05, U[:, 1:].shape)
    U[:, :, :prob.step_j, prob.step_i:] = 0.0
    return U


def test_gas_at_rest_in_a_tunnel_with_a_step_stays_at_rest():
    for wf in (0, 1):
        prob = _tunnel(40, 20, 12, 6, wall_flux=wf)
        U = np.zeros(prob.shape())
        U[:, 0] = _cons(1.3, 0.0, 0.0, 0.9)[:, None, None]
        U[:, :, :6, 12:] = 0.0
        L, fl = oracle.residual(prob, U)
        assert np.abs(L).max() <= 1e-13
        assert fl.sum() == 0


def test_step_cells_read_as_mirror_images():
    """Step cells as ghosts: across the vertical face when fewer columns
    into the step than rows below its top, across the top in the opposite
    case, through the corner when equal; first moments along the mirror's
    normal and the normal momentum flip; their residual is zero."""
    prob = _tunnel(40, 24, 14, 12)
    U = _random_state(prob, 3)
    si, sj = 14, 12
    for (i, j, src, fx, fy) in [(14, 11, (13, 12), 1, 1), (14, 5, (13, 5), 1, 0), (20, 11, (20, 12), 0, 1),
                                (16, 9, (11, 14), 1, 1), (15, 3, (12, 3), 1, 0), (25, 8, (25, 15), 0, 1)]:
        for c in range(4):
            for m in range(3):
                flip = (fx and ((c == 1) != (m == 1))) != (fy and ((c == 2) != (m == 2)))
                want = U[c, m, src[1], src[0]] * (-1.0 if flip else 1.0)
                assert oracle.moment(prob, U, c, m, i, j) == want, (i, j, c, m)
    L, fl = oracle.residual(prob, U)
    assert np.all(L[:, :, :sj, si:] == 0.0)


def test_step_faces_match_tunnels_mirrored_by_hand():
    """Residuals next to the step's vertical face (rows far below its top)
    and above its top (columns far right of its face) equal those of tunnels
    without a step whose data are mirrored across that face (printed HLLC on
    both sides of the face, KXRCF, modification)."""
    si, sj = 14, 12
    prob = _tunnel(40, 24, si, sj)
    U = _random_state(prob, 7)
    L, fl = oracle.residual(prob, U)
    flip_x = np.array([[(c == 1) != (m == 1) for m in range(3)] for c in range(4)])
    flip_y = np.array([[(c == 2) != (m == 2) for m in range(3)] for c in range(4)])
    # vertical face: columns 0 .. si-1 and their mirror images si .. 2 si - 1
    px = _tunnel(2 * si, 24, 0, 0)
    Ux = np.zeros(px.shape())
    Ux[:, :, :, :si] = U[:, :, :, :si]
    Ux[:, :, :, si:] = np.where(flip_x[:, :, None, None], -1.0, 1.0) * U[:, :, :, si - 1::-1]
    Lx, flx = oracle.residual(px, Ux)
    a, b = L[:, :, :4, si - 3:si], Lx[:, :, :4, si - 3:si]
    assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()
    assert np.array_equal(fl[:4, si - 3:si], flx[:4, si - 3:si])
    # top face: rows sj .. ny-1 and their mirror images below
    ny = 24
    h = ny - sj
    py = I.Problem(dim=2, nx=40, ny=2 * h, x0=0.0, x1=40 / 24, y0=0.0, y1=2 * h / 24, system=I.EULER,
                   bc_x=I.TRANSMISSIVE, bc_y=I.REFLECTIVE, tc_mode=I.TC_KXRCF)
    Uy = np.zeros(py.shape())
    Uy[:, :, h:, :] = U[:, :, sj:, :]
    Uy[:, :, :h, :] = np.where(flip_y[:, :, None, None], -1.0, 1.0) * U[:, :, ny - 1:sj - 1:-1, :]
    Ly, fly = oracle.residual(py, Uy)
    a, b = L[:, :, sj:sj + 3, si + 8:35], Ly[:, :, h:h + 3, si + 8:35]
    assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()
    assert np.array_equal(fl[sj:sj + 3, si + 8:35], fly[h:h + 3, si + 8:35])


def test_forward_step_setup():
    prob, U = I.forward_step(ny=20)
    assert (prob.nx, prob.ny, prob.step_i, prob.step_j) == (60, 20, 12, 4)
    assert prob.dx == prob.dy == 0.05
    r, u, p = U[0, 0, 10, 5], U[1, 0, 10, 5] / U[0, 0, 10, 5], _p(U[:, 0, 10, 5])
    assert r == 1.4 and abs(u - 3.0) < 1e-15 and abs(p - 1.0) < 1e-15 and abs(math.sqrt(G * p / r) - 1.0) < 1e-15
    assert np.all(U[:, :, :4, 12:] == 0.0)
