"""Seeded synthetic inputs: problem descriptions and initial moments.

This module is the only code shared by the GPU library's tests/benchmark and
the CPU oracle.  It holds no arithmetic of the scheme itself: it describes
problems (grid, flux, boundary conditions, linear weights, CFL, final time)
and projects initial data onto the zeroth and first moments of eq.
(1D-moment) / (2D-moment) by Gauss-Legendre quadrature, splitting cells at
known jump locations so that piecewise-smooth data are projected exactly up
to quadrature error.

Moment layout (structure of arrays, x fastest):
  1D: U[comp][m][nx],      m = 0 (ubar), 1 (vbar)
  2D: U[comp][m][ny][nx],  m = 0 (ubar), 1 (vtilde, x), 2 (wtilde, y)
Components: Burgers (u); 1D Euler (rho, rho*mu, E); 2D Euler
(rho, rho*mu, rho*nu, E).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, List, Optional, Sequence, Tuple

import numpy as np

BURGERS = 0
EULER = 1
PERIODIC = 0
TRANSMISSIVE = 1
REFLECTIVE = 2   # Euler: mirror-image ghosts (wall-normal momentum and normal first moment flip)
SIDES = 3        # per-side boundary data in Problem.sides (bc_x / bc_y)
INFLOW = 3       # side kind: ghosts hold a prescribed constant state
TC_NONE = 0     # HWENO6: no first-moment modification
TC_KXRCF = 1    # HWENO6-M5-I
TC_ALL = 2      # HWENO6-M5-NI
TC_LEARNED = 3  # learned indicator with KXRCF fallback
TC_TVB = 4      # TVB minmod indicator (one of Remark 2's alternatives)
BETA_ON_Q = 0
BETA_ON_P = 1
MOD_PERSIST = 0   # modified first moments replace those of every stage input, U^n included
MOD_INTERNAL = 1  # modification internal to L(U)
MOD_STAGE = 2     # replace those of the stage input only


@dataclasses.dataclass(frozen=True)
class Side:
    """Boundary data of one side (used where bc_x or bc_y is SIDES).

    kind: TRANSMISSIVE, REFLECTIVE or INFLOW (ghosts hold `state`, first
    moments zero).  On the bottom and top sides a front x < s0 + st t + sn y
    (split = (s0, st, sn); a straight front moving at a constant speed) puts
    `pre` before it: on an INFLOW side ghosts hold the exact moments of the
    two-state field, before a folded side a ghost whose centre lies before
    the front holds `pre`."""
    kind: int = TRANSMISSIVE
    state: Tuple[float, ...] = (0.0, 0.0, 0.0, 0.0)
    pre: Tuple[float, ...] = (0.0, 0.0, 0.0, 0.0)
    split: Tuple[float, float, float] = (-math.inf, 0.0, 0.0)


@dataclasses.dataclass
class Problem:
    """A conservation-law problem posed as the paper poses it (Sec. 2, 3)."""
    dim: int
    nx: int
    ny: int = 1
    x0: float = 0.0
    x1: float = 1.0
    y0: float = 0.0
    y1: float = 1.0
    system: int = EULER
    bc_x: int = PERIODIC
    bc_y: int = PERIODIC
    gamma: float = 1.4
    cfl: float = 0.6
    t_final: float = math.inf
    gbar: Tuple[float, float, float, float] = (1.0, 10.0, 100.0, 1000.0)
    eps: float = 1e-10
    tc_mode: int = TC_KXRCF
    beta_on: int = BETA_ON_Q
    modification: int = MOD_PERSIST
    tvb_m: float = 0.0   # TVB constant M of the minmod indicator (TC_TVB)
    charwise: int = 0    # 1D Euler: Step 1 on characteristic fields (0: component-wise)
    sides: Optional[Tuple[Side, Side, Side, Side]] = None   # left, right, bottom, top (SIDES)
    step_i: int = 0      # 2D Euler: a solid step of the cells i >= step_i, j < step_j
    step_j: int = 0      # (Example 3.10's forward step); step_j = 0: none
    wall_flux: int = 0   # 1: exact mirror-problem flux on wall faces (0: HLLC on the mirror state)

    @property
    def dx(self) -> float:
        return (self.x1 - self.x0) / self.nx

    @property
    def dy(self) -> float:
        return (self.y1 - self.y0) / self.ny if self.dim == 2 else 1.0

    @property
    def ncomp(self) -> int:
        if self.system == BURGERS:
            return 1
        return 3 if self.dim == 1 else 4

    @property
    def nmom(self) -> int:
        return self.dim + 1

    @property
    def ncell(self) -> int:
        return self.nx * (self.ny if self.dim == 2 else 1)

    def shape(self) -> Tuple[int, ...]:
        if self.dim == 1:
            return (self.ncomp, 2, self.nx)
        return (self.ncomp, 3, self.ny, self.nx)

    def replace(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)


# --------------------------------------------------------------------------
# Projection onto moments
# --------------------------------------------------------------------------
def _gauss(nq: int):
    x, w = np.polynomial.legendre.leggauss(nq)
    return 0.5 * x, 0.5 * w  # on [-1/2, 1/2], weights sum to 1


def project_1d(prob: Problem, cons: Callable[[np.ndarray], np.ndarray],
               jumps: Sequence[float] = (), nq: int = 8) -> np.ndarray:
    """Moments of conserved data cons(x) -> array (ncomp, len(x)).

    Cells containing a jump location are split there and each part is
    integrated with its own Gauss rule."""
    n, dx = prob.nx, prob.dx
    xc = prob.x0 + (np.arange(n) + 0.5) * dx
    xs, ws = _gauss(nq)
    U = np.zeros((prob.ncomp, 2, n))
    # sub-intervals in reference coordinates per cell
    cuts = [[] for _ in range(n)]
    for xj in jumps:
        s = (xj - prob.x0) / dx
        i = int(math.floor(s))
        frac = s - i - 0.5
        if 0 <= i < n and -0.5 < frac < 0.5:
            cuts[i].append(frac)
    plain = [i for i in range(n) if not cuts[i]]
    if plain:
        idx = np.array(plain)
        pts = xc[idx][:, None] + xs[None, :] * dx          # (m, nq)
        vals = cons(pts.ravel()).reshape(prob.ncomp, len(idx), nq)
        U[:, 0, idx] = (vals * ws).sum(-1)
        U[:, 1, idx] = (vals * ws * xs).sum(-1)
    for i in range(n):
        if not cuts[i]:
            continue
        edges = [-0.5] + sorted(cuts[i]) + [0.5]
        for a, b in zip(edges[:-1], edges[1:]):
            s = 0.5 * (a + b) + xs * (b - a)
            w = ws * (b - a)
            vals = cons(xc[i] + s * dx).reshape(prob.ncomp, nq)
            U[:, 0, i] += (vals * w).sum(-1)
            U[:, 1, i] += (vals * w * s).sum(-1)
    return U


def project_2d(prob: Problem, cons: Callable[[np.ndarray, np.ndarray], np.ndarray],
               nq: int = 8, rows_per_block: int = 64) -> np.ndarray:
    """Moments of conserved data cons(x, y) -> (ncomp, ...); discontinuities
    must lie on cell faces (the configurations here put them there)."""
    nx, ny, dx, dy = prob.nx, prob.ny, prob.dx, prob.dy
    xs, ws = _gauss(nq)
    xc = prob.x0 + (np.arange(nx) + 0.5) * dx
    U = np.zeros((prob.ncomp, 3, ny, nx))
    wxy = ws[:, None] * ws[None, :]       # (qy, qx)
    for j0 in range(0, ny, rows_per_block):
        j1 = min(ny, j0 + rows_per_block)
        yc = prob.y0 + (np.arange(j0, j1) + 0.5) * dy
        X = xc[None, None, :, None] + xs[None, None, None, :] * dx   # (1,1,nx,qx)
        Y = yc[:, None, None, None] + xs[None, :, None, None] * dy   # (nyb,qy,1,1)
        X, Y = np.broadcast_arrays(X, Y)
        vals = cons(X, Y)                                            # (nc, nyb, qy, nx, qx)
        w = wxy[None, None, :, None, :]
        U[:, 0, j0:j1] = (vals * w).sum(axis=(2, 4))
        U[:, 1, j0:j1] = (vals * w * xs[None, None, None, None, :]).sum(axis=(2, 4))
        U[:, 2, j0:j1] = (vals * w * xs[None, None, :, None, None]).sum(axis=(2, 4))
    return U


def cell_averages_1d(prob: Problem, f: Callable[[np.ndarray], np.ndarray], nq: int = 8) -> np.ndarray:
    xs, ws = _gauss(nq)
    xc = prob.x0 + (np.arange(prob.nx) + 0.5) * prob.dx
    pts = xc[:, None] + xs[None, :] * prob.dx
    return (f(pts) * ws).sum(-1)


def cell_averages_2d(prob: Problem, f: Callable[[np.ndarray, np.ndarray], np.ndarray], nq: int = 8) -> np.ndarray:
    xs, ws = _gauss(nq)
    xc = prob.x0 + (np.arange(prob.nx) + 0.5) * prob.dx
    yc = prob.y0 + (np.arange(prob.ny) + 0.5) * prob.dy
    X = xc[None, None, :, None] + xs[None, None, None, :] * prob.dx
    Y = yc[:, None, None, None] + xs[None, :, None, None] * prob.dy
    X, Y = np.broadcast_arrays(X, Y)
    return (f(X, Y) * (ws[:, None] * ws[None, :])[None, :, None, :]).sum(axis=(1, 3))


# --------------------------------------------------------------------------
# Primitive -> conserved conversions for initial data only
# --------------------------------------------------------------------------
def euler1d_cons(rho, u, p, gamma):
    return np.stack([rho, rho * u, p / (gamma - 1.0) + 0.5 * rho * u * u])


def euler2d_cons(rho, u, v, p, gamma):
    return np.stack([rho, rho * u, rho * v, p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)])


# --------------------------------------------------------------------------
# The paper's smooth and Riemann test problems (Sec. 3)
# --------------------------------------------------------------------------
def example_burgers_1d(n: int, tc_mode: int = TC_KXRCF, **kw):
    """Example 3.1: u0 = 0.5 + sin(pi x) on [0, 2], periodic, T = 0.5/pi."""
    prob = Problem(dim=1, nx=n, x0=0.0, x1=2.0, system=BURGERS, bc_x=PERIODIC,
                   t_final=0.5 / math.pi, tc_mode=tc_mode, **kw)
    U = project_1d(prob, lambda x: (0.5 + np.sin(np.pi * x))[None])
    return prob, U


def example_burgers_2d(n: int, tc_mode: int = TC_KXRCF, **kw):
    """Example 3.2: u0 = 0.5 + sin(pi (x+y)/2) on [0, 4]^2, T = 0.5/pi."""
    prob = Problem(dim=2, nx=n, ny=n, x0=0.0, x1=4.0, y0=0.0, y1=4.0, system=BURGERS,
                   t_final=0.5 / math.pi, tc_mode=tc_mode, **kw)
    U = project_2d(prob, lambda x, y: (0.5 + np.sin(np.pi * (x + y) / 2.0))[None])
    return prob, U


def example_euler_1d(n: int, gamma: float = 3.0, tc_mode: int = TC_KXRCF, **kw):
    """Example 3.3 (gamma = 3 reading): rho = (1 + 0.2 sin x)/(2 sqrt 3),
    mu = sqrt(gamma) rho, p = rho^gamma, periodic on [0, 2 pi], T = 3."""
    prob = Problem(dim=1, nx=n, x0=0.0, x1=2.0 * math.pi, system=EULER, gamma=gamma,
                   t_final=3.0, tc_mode=tc_mode, **kw)

    def cons(x):
        rho = (1.0 + 0.2 * np.sin(x)) / (2.0 * math.sqrt(3.0))
        return euler1d_cons(rho, math.sqrt(gamma) * rho, rho ** gamma, gamma)
    return prob, project_1d(prob, cons)


def example_euler_2d(n: int, gamma: float = 3.0, tc_mode: int = TC_KXRCF, **kw):
    """Example 3.4 (gamma = 3 reading) on [0, 4 pi]^2, T = 3."""
    L = 4.0 * math.pi
    prob = Problem(dim=2, nx=n, ny=n, x0=0.0, x1=L, y0=0.0, y1=L, system=EULER, gamma=gamma,
                   t_final=3.0, tc_mode=tc_mode, **kw)

    def cons(x, y):
        rho = (1.0 + 0.2 * np.sin((x + y) / 2.0)) / math.sqrt(6.0)
        vel = math.sqrt(gamma / 2.0) * rho
        return euler2d_cons(rho, vel, vel, rho ** gamma, gamma)
    return prob, project_2d(prob, cons)


def example_lax(n: int = 200, tc_mode: int = TC_KXRCF, **kw):
    """Example 3.5, the Lax problem on [-0.5, 0.5], T = 0.16, gamma = 1.4."""
    prob = Problem(dim=1, nx=n, x0=-0.5, x1=0.5, system=EULER, gamma=1.4, bc_x=TRANSMISSIVE,
                   t_final=0.16, tc_mode=tc_mode, **kw)
    left, right = (0.445, 0.698, 3.528), (0.5, 0.0, 0.571)

    def cons(x):
        l = x < 0.0
        rho = np.where(l, left[0], right[0])
        u = np.where(l, left[1], right[1])
        p = np.where(l, left[2], right[2])
        return euler1d_cons(rho, u, p, 1.4)
    return prob, project_1d(prob, cons, jumps=[0.0]), (left, right)


def example_shock_density(n: int = 400, tc_mode: int = TC_KXRCF, **kw):
    """Example 3.6, a Mach 3 shock running into sine waves in the density on
    [-5, 5], T = 1.8, gamma = 1.4; transmissive ends (the paper does not
    state them)."""
    prob = Problem(dim=1, nx=n, x0=-5.0, x1=5.0, system=EULER, gamma=1.4, bc_x=TRANSMISSIVE,
                   t_final=1.8, tc_mode=tc_mode, **kw)
    left = (3.857143, 2.629369, 10.333333)

    def cons(x):
        l = x < -4.0
        rho = np.where(l, left[0], 1.0 + 0.2 * np.sin(5.0 * x))
        u = np.where(l, left[1], 0.0)
        p = np.where(l, left[2], 1.0)
        return euler1d_cons(rho, u, p, 1.4)
    return prob, project_1d(prob, cons, jumps=[-4.0]), left


def example_sedov(n: int = 401, tc_mode: int = TC_KXRCF, **kw):
    """Example 3.8, the Sedov blast wave on [-2, 2], T = 0.001, gamma = 1.4:
    rho = 1, u = 0, E = 1e-12 except the centre cell, E = 3200000/dx there
    (an odd cell count, so that there is a centre cell); transmissive ends."""
    if n % 2 == 0:
        raise ValueError("the Sedov problem needs an odd number of cells")
    prob = Problem(dim=1, nx=n, x0=-2.0, x1=2.0, system=EULER, gamma=1.4, bc_x=TRANSMISSIVE,
                   t_final=0.001, tc_mode=tc_mode, **kw)
    U = np.zeros(prob.shape())
    U[0, 0] = 1.0
    U[2, 0] = 1e-12
    U[2, 0, n // 2] = 3200000.0 / prob.dx
    return prob, U


# --------------------------------------------------------------------------
# Seeded synthetic workloads
# --------------------------------------------------------------------------
def _riemann_ok(rl, ul, pl, rr, ur, pr, gamma) -> bool:
    """Reject draws within a factor 2 of vacuum generation."""
    cl, cr = math.sqrt(gamma * pl / rl), math.sqrt(gamma * pr / rr)
    return (ur - ul) < (cl + cr) / (gamma - 1.0)


def burgers_smooth_1d(seed: int, n: int = 200, **kw):
    """Periodic Burgers on [0, 2 pi], u0 = 0.5 + sin(x + phi), phi ~ U(0, 2 pi),
    Lax-Friedrichs flux, KXRCF, CFL 0.6, T = 0.5 (smooth up to t = 1)."""
    rng = np.random.default_rng(seed)
    phi = rng.uniform(0.0, 2.0 * math.pi)
    prob = Problem(dim=1, nx=n, x0=0.0, x1=2.0 * math.pi, system=BURGERS, bc_x=PERIODIC,
                   t_final=0.5, tc_mode=kw.pop("tc_mode", TC_KXRCF), **kw)
    U = project_1d(prob, lambda x: (0.5 + np.sin(x + phi))[None])
    return prob, U, {"phi": phi}


def euler_riemann_1d(seed: int, n: int = 4096, t_final: float = 0.2, **kw):
    """1D Euler (gamma 1.4) on [0, 1], transmissive; left/right rho ~ U(0.1, 1),
    u ~ U(-1, 1), p ~ U(0.1, 1), jump at x_d ~ U(0.3, 0.7); density multiplied
    by (1 + 0.2 sin(2 pi k x)), k ~ U{5..20}; HLLC."""
    rng = np.random.default_rng(seed)
    gamma = 1.4
    while True:
        rl, rr = rng.uniform(0.1, 1.0, 2)
        ul, ur = rng.uniform(-1.0, 1.0, 2)
        pl, pr = rng.uniform(0.1, 1.0, 2)
        # the density perturbation can raise rho by 20 %, lowering c
        if _riemann_ok(rl * 1.2, ul, pl, rr * 1.2, ur, pr, gamma):
            break
    xd = rng.uniform(0.3, 0.7)
    k = int(rng.integers(5, 21))
    prob = Problem(dim=1, nx=n, x0=0.0, x1=1.0, system=EULER, gamma=gamma, bc_x=TRANSMISSIVE,
                   t_final=t_final, tc_mode=kw.pop("tc_mode", TC_KXRCF), **kw)

    def cons(x):
        l = x < xd
        rho = np.where(l, rl, rr) * (1.0 + 0.2 * np.sin(2.0 * math.pi * k * x))
        return euler1d_cons(rho, np.where(l, ul, ur), np.where(l, pl, pr), gamma)
    U = project_1d(prob, cons, jumps=[xd])
    return prob, U, {"states": ((rl, ul, pl), (rr, ur, pr)), "xd": xd, "k": k}


def euler_quadrants_2d(seed: int, n: int = 2048, nq: int = 4, **kw):
    """2D Euler (gamma 1.4), periodic [0, 1]^2: four constant quadrant states
    (rho, p ~ U(0.1, 1.5), u, v ~ U(-0.8, 0.8)) split at x = y = 1/2, overlaid
    with a smooth 8-mode Fourier field F (wave vectors in {-4..4}^2 \\ 0,
    sum |a_m| = 1): rho (1 + 0.05 F), p (1 + 0.05 F), u + 0.05 F, v + 0.05 F.
    HLLC flux.  The split lies on cell faces for even n."""
    rng = np.random.default_rng(seed)
    gamma = 1.4
    while True:
        rho = rng.uniform(0.1, 1.5, 4)
        p = rng.uniform(0.1, 1.5, 4)
        u = rng.uniform(-0.8, 0.8, 4)
        v = rng.uniform(-0.8, 0.8, 4)
        # quadrants: 0 = (x<.5,y<.5), 1 = (x>.5,y<.5), 2 = (x<.5,y>.5), 3 = (x>.5,y>.5);
        # worst case of the 5 % overlay: rho up, p down, velocity jump widened
        ok = True
        for a, b in ((0, 1), (2, 3), (1, 0), (3, 2)):   # x neighbours, periodic images
            ok &= _riemann_ok(rho[a] * 1.05, u[a] - 0.05, p[a] * 0.95,
                              rho[b] * 1.05, u[b] + 0.05, p[b] * 0.95, gamma)
        for a, b in ((0, 2), (1, 3), (2, 0), (3, 1)):   # y neighbours
            ok &= _riemann_ok(rho[a] * 1.05, v[a] - 0.05, p[a] * 0.95,
                              rho[b] * 1.05, v[b] + 0.05, p[b] * 0.95, gamma)
        if ok:
            break
    modes = []
    allk = [(kx, ky) for kx in range(-4, 5) for ky in range(-4, 5) if (kx, ky) != (0, 0)]
    pick = rng.choice(len(allk), size=8, replace=False)
    amp = rng.uniform(-1.0, 1.0, 8)
    amp = amp / np.abs(amp).sum()
    phase = rng.uniform(0.0, 2.0 * math.pi, 8)
    for m in range(8):
        modes.append((allk[pick[m]][0], allk[pick[m]][1], amp[m], phase[m]))
    prob = Problem(dim=2, nx=n, ny=n, x0=0.0, x1=1.0, y0=0.0, y1=1.0, system=EULER, gamma=gamma,
                   tc_mode=kw.pop("tc_mode", TC_KXRCF), **kw)

    def cons(x, y):
        F = np.zeros_like(x)
        for kx, ky, a, ph in modes:
            F += a * np.sin(2.0 * math.pi * (kx * x + ky * y) + ph)
        q = (x > 0.5).astype(np.int64) + 2 * (y > 0.5).astype(np.int64)
        r = rho[q] * (1.0 + 0.05 * F)
        pp = p[q] * (1.0 + 0.05 * F)
        return euler2d_cons(r, u[q] + 0.05 * F, v[q] + 0.05 * F, pp, gamma)
    U = project_2d(prob, cons, nq=nq)
    return prob, U, {"rho": rho, "p": p, "u": u, "v": v, "modes": modes}


def contact_wave_2d(seed: int, nx: int, ny: int, amp: float = 0.2, jump: float = 0.5, **kw):
    """2D Euler (gamma 1.4), periodic [0, nx/ny] x [0, 1]: a density field
    rho = 1 + amp sin(2 pi (x + phx)) sin(2 pi (y + phy)) + jump [x > X/2]
    carried by a constant velocity (u, v) ~ U(-0.5, 0.5)^2 at constant
    pressure p ~ U(0.8, 1.2), phases from the seed (a contact discontinuity
    on a cell face for even nx, smooth elsewhere).  Its moments are separable
    products of 1D cell moments (Gauss quadrature per column and row), so a
    grid of tens of millions of cells takes seconds: the generator of the
    largest grids."""
    rng = np.random.default_rng(seed)
    gamma = 1.4
    phx, phy = rng.uniform(0.0, 1.0, 2)
    u0, v0 = rng.uniform(-0.5, 0.5, 2)
    p0 = rng.uniform(0.8, 1.2)
    prob = Problem(dim=2, nx=nx, ny=ny, x0=0.0, x1=nx / ny, y0=0.0, y1=1.0, system=EULER, gamma=gamma,
                   tc_mode=kw.pop("tc_mode", TC_KXRCF), **kw)
    xs, ws = _gauss(8)

    def moments_1d(n, d, ph):
        c = (np.arange(n) + 0.5) * d
        s = np.sin(2.0 * math.pi * (c[:, None] + xs[None, :] * d + ph))
        return (s * ws).sum(-1), (s * ws * xs).sum(-1)   # average, first moment
    ax, mx = moments_1d(nx, prob.dx, phx)
    ay, my = moments_1d(ny, prob.dy, phy)
    hx = ((np.arange(nx) + 0.5) * prob.dx > 0.5 * (nx / ny)).astype(np.float64)
    # moments of rho: average, x moment, y moment
    r = [1.0 + amp * np.multiply.outer(ay, ax) + jump * hx[None, :],
         amp * np.multiply.outer(ay, mx), amp * np.multiply.outer(my, ax)]
    U = np.empty(prob.shape())
    ke = 0.5 * (u0 * u0 + v0 * v0)
    for m in range(3):
        U[0, m] = r[m]
        np.multiply(r[m], u0, out=U[1, m])
        np.multiply(r[m], v0, out=U[2, m])
        np.multiply(r[m], ke, out=U[3, m])
    U[3, 0] += p0 / (gamma - 1.0)
    return prob, U, {"u": u0, "v": v0, "p": p0}


def batched_instances(seed: int, n1d: int = 192, n2d: int = 64,
                      n1_range=(128, 16384), n2_range=(64, 1024)):
    """Batched workload: n1d 1D Euler Riemann instances with N log-uniform in
    n1_range and n2d 2D Euler quadrant instances with side log-uniform in
    n2_range (rounded to an even side so the quadrant split is a cell face).
    Returns a list of (Problem, U) with per-instance seeds."""
    rng = np.random.default_rng(seed)
    out = []
    lo, hi = n1_range
    for k in range(n1d):
        n = int(round(lo * (hi / lo) ** rng.uniform()))
        prob, U, _ = euler_riemann_1d(int(rng.integers(1 << 31)), n=n)
        out.append((prob, U))
    lo, hi = n2_range
    for k in range(n2d):
        n = int(round(lo * (hi / lo) ** rng.uniform()))
        n += n % 2
        prob, U, _ = euler_quadrants_2d(int(rng.integers(1 << 31)), n=n, nq=2)
        out.append((prob, U))
    return out


# --------------------------------------------------------------------------
# Double Mach reflection (Example 3.9)
# --------------------------------------------------------------------------
def _clip_moments(a: float, b: float, c: float) -> Tuple[float, float, float]:
    """Area and first moments (of xi and eta) of the part of the reference
    cell [-1/2, 1/2]^2 where a*xi + b*eta < c: the square clipped by the
    half-plane (Sutherland-Hodgman) and integrated with the polygon
    (shoelace) formulas, which are exact for polygons."""
    sq = [(-0.5, -0.5), (0.5, -0.5), (0.5, 0.5), (-0.5, 0.5)]
    out = []
    for k in range(4):
        p, q = sq[k], sq[(k + 1) % 4]
        fp, fq = a * p[0] + b * p[1] - c, a * q[0] + b * q[1] - c
        if fp < 0.0:
            out.append(p)
        if (fp < 0.0) != (fq < 0.0):
            s = fp / (fp - fq)
            out.append((p[0] + s * (q[0] - p[0]), p[1] + s * (q[1] - p[1])))
    area = mx = my = 0.0
    for k in range(len(out)):
        (x0, y0), (x1, y1) = out[k], out[(k + 1) % len(out)]
        cr = x0 * y1 - x1 * y0
        area += cr
        mx += (x0 + x1) * cr
        my += (y0 + y1) * cr
    return area / 2.0, mx / 6.0, my / 6.0


def mach_shock_states(mach: float = 10.0, gamma: float = 1.4):
    """Primitive states (rho, u_n, p) on both sides of a normal shock of
    Mach number `mach` running into gas at rest with rho = gamma, p = 1
    (sound speed 1), from the Rankine-Hugoniot relations; and the shock
    speed."""
    m2 = mach * mach
    rho2 = gamma * (gamma + 1.0) * m2 / ((gamma - 1.0) * m2 + 2.0)
    p2 = 1.0 + 2.0 * gamma / (gamma + 1.0) * (m2 - 1.0)
    un = mach * (1.0 - gamma / rho2)
    return (gamma, 0.0, 1.0), (rho2, un, p2), mach


def double_mach_2d(ny: int = 400, tc_mode: int = TC_KXRCF, t_final: float = 0.2,
                   modification: int = MOD_INTERNAL, **kw):
    """Example 3.9: [0, 4] x [0, 1], 4*ny x ny cells, a Mach 10 shock
    (gamma 1.4) through (1/6, 0) at 60 degrees to the x axis moving right
    into gas at rest (rho = 1.4, p = 1).  Bottom: the post-shock state for
    x < 1/6 (ghost centres), a reflective wall beyond; top: the exact motion
    of the shock x = 1/6 + (y + 20 t)/sqrt(3) (ghosts hold the exact moments
    of the two states); left: post-shock inflow; right: transmissive.  The
    modified first moments stay internal to L by default: with them
    persisted the run breaks down at the post-shock/wall junction of the
    bottom after a fixed number of steps at any resolution.  Initial moments are exact: cells cut by the front
    are clipped by it.  Returns (problem, U)."""
    gamma = 1.4
    (r1, _, p1), (r2, un, p2), ms = mach_shock_states(10.0, gamma)
    th = math.pi / 6.0                          # the shock normal is 30 degrees below the x axis
    u2, v2 = un * math.cos(th), -un * math.sin(th)
    pre = tuple(float(z) for z in euler2d_cons(np.array(r1), np.array(0.0), np.array(0.0), np.array(p1), gamma))
    post = tuple(float(z) for z in euler2d_cons(np.array(r2), np.array(u2), np.array(v2), np.array(p2), gamma))
    s3 = math.sqrt(3.0)
    speed = ms / math.sin(math.pi / 3.0)       # horizontal speed of the front: 20/sqrt(3)
    sides = (Side(kind=INFLOW, state=post),
             Side(kind=TRANSMISSIVE),
             Side(kind=REFLECTIVE, pre=post, split=(1.0 / 6.0, 0.0, 0.0)),
             Side(kind=INFLOW, state=pre, pre=post, split=(1.0 / 6.0, speed, 1.0 / s3)))
    prob = Problem(dim=2, nx=4 * ny, ny=ny, x0=0.0, x1=4.0, y0=0.0, y1=1.0, system=EULER,
                   bc_x=SIDES, bc_y=SIDES, gamma=gamma, t_final=t_final, tc_mode=tc_mode,
                   modification=modification, sides=sides, **kw)
    dx, dy = prob.dx, prob.dy
    # post-shock where x - y/sqrt(3) < 1/6; in reference coordinates of cell
    # (i, j): dx xi - dy eta / sqrt(3) < 1/6 - xc + yc / sqrt(3)
    U = np.zeros(prob.shape())
    xc = prob.x0 + (np.arange(prob.nx) + 0.5) * dx
    yc = prob.y0 + (np.arange(prob.ny) + 0.5) * dy
    reach = 0.5 * dx + 0.5 * dy / s3
    pre_a, post_a = np.array(pre), np.array(post)
    for j in range(prob.ny):
        g = 1.0 / 6.0 - xc + yc[j] / s3           # > 0: centre on the post-shock side
        full = g >= reach
        none = g <= -reach
        U[:, 0, j, full] = post_a[:, None]
        U[:, 0, j, none] = pre_a[:, None]
        for i in np.nonzero(~full & ~none)[0]:
            a, mx, my = _clip_moments(dx, -dy / s3, g[i])
            U[:, 0, j, i] = post_a * a + pre_a * (1.0 - a)
            U[:, 1, j, i] = (post_a - pre_a) * mx
            U[:, 2, j, i] = (post_a - pre_a) * my
    return prob, U


def forward_step(ny: int = 200, tc_mode: int = TC_KXRCF, t_final: float = 4.0,
                 modification: int = MOD_INTERNAL, wall_flux: int = 1, **kw):
    """Example 3.10: a tunnel [0, 3] x [0, 1] of 3*ny x ny cells with a step
    of height 0.2 from x = 0.6 to the exit (the cells i >= 0.6 ny,
    j < 0.2 ny), filled at t = 0 with a right-going Mach 3 flow (gamma 1.4,
    rho = 1.4, u = 3, p = 1, so c = 1).  Left: inflow of that state; right:
    transmissive; the tunnel's top and bottom and the step are reflective
    walls, with the exact mirror-problem flux on the wall faces by default
    (wall_flux = 1: the printed HLLC on the mirror state lets a stream of
    normal Mach 3 through the step's face).  The step's cells hold zeros.
    Returns (problem, U)."""
    if ny % 5:
        raise ValueError("ny must be a multiple of 5 (step at 0.6, height 0.2)")
    gamma = 1.4
    state = tuple(float(z) for z in euler2d_cons(np.array(1.4), np.array(3.0), np.array(0.0), np.array(1.0), gamma))
    sides = (Side(kind=INFLOW, state=state), Side(kind=TRANSMISSIVE), Side(kind=REFLECTIVE), Side(kind=REFLECTIVE))
    prob = Problem(dim=2, nx=3 * ny, ny=ny, x0=0.0, x1=3.0, y0=0.0, y1=1.0, system=EULER,
                   bc_x=SIDES, bc_y=REFLECTIVE, gamma=gamma, t_final=t_final, tc_mode=tc_mode,
                   modification=modification, sides=sides, step_i=3 * ny // 5, step_j=ny // 5,
                   wall_flux=wall_flux, **kw)
    U = np.zeros(prob.shape())
    U[:, 0] = np.array(state)[:, None, None]
    U[:, :, :prob.step_j, prob.step_i:] = 0.0
    return prob, U
