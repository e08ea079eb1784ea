"""GPU vs oracle with a solid step in the tunnel (the forward step of
Example 3.10) and the wall flux of the mirror-image Riemann problem:
Gauss-Lobatto values, troubled-cell flags, residuals and SSP-RK3 steps,
component-wise and characteristic-wise, at the oracle's bar (FP64 values
within 1e-12 of the component's scale, flags bit-exact with the counts
printed).  The full-size run (600 x 200 to T = 4, characteristic-wise, as
the component-wise scheme breaks down at the step's corner) is checked on
sampled cells of its final state."""
import numpy as np
import pytest

import oracle
from paper_2201_12193_amd import inputs as I
from tests.parity_util import comp_scale, rel_state_err, kxrcf_flags, MISMATCHES_ALLOWED

pytestmark = pytest.mark.gpu
TOL = 1e-12
G = 1.4


def _dev():
    import torch
    return torch.device("cuda:0")


def _cons(r, u, v, p):
    return np.array([r, r * u, r * v, p / (G - 1) + 0.5 * r * (u * u + v * v)])


def _tunnel(seed, wall_flux, charwise, nx=40, ny=24, si=14, sj=12, noise=False):
    """A tunnel with a step (transmissive ends, reflective top and bottom)
    holding the seeded quadrant states plus Fourier modes of the quadrant
    workload (noise=False; troubled cells along its waves, the KXRCF test
    clear of its threshold) or white noise (density and pressure in
    [1, 1.3], velocities in [-0.6, 0.6], first moments in [-0.05, 0.05]:
    nearly every cell troubled, many of them within rounding of the
    threshold); zeros in the step."""
    prob = I.Problem(dim=2, nx=nx, ny=ny, x0=0.0, x1=nx / ny, y0=0.0, y1=1.0, system=I.EULER,
                     bc_x=I.TRANSMISSIVE, bc_y=I.REFLECTIVE, tc_mode=I.TC_KXRCF, step_i=si, step_j=sj,
                     wall_flux=wall_flux, charwise=charwise)
    if noise:
        rng = np.random.default_rng(seed)
        sh = (ny, nx)
        U = np.zeros(prob.shape())
        U[:, 0] = _cons(1.0 + 0.3 * rng.random(sh), rng.uniform(-0.6, 0.6, sh), rng.uniform(-0.6, 0.6, sh),
                        1.0 + 0.3 * rng.random(sh))
        U[:, 1:] = rng.uniform(-0.05, 0.05, U[:, 1:].shape)
    else:
        _, Uq, _ = I.euler_quadrants_2d(seed=seed, n=nx, nq=2)
        U = np.ascontiguousarray(Uq[:, :, :ny, :nx])
    U[:, :, :sj, si:] = 0.0
    return prob, U


def _advance(prob, U, k):
    t = 0.0
    for _ in range(k):
        d = oracle.dt(prob, U)
        U = oracle.rk3_step(prob, U, d, t=t)
        t += d
    return U, t


def _check(tag, prob, U, t, k, nsteps):
    import torch
    from paper_2201_12193_amd.mrhweno import Solver
    Ut = torch.from_numpy(np.ascontiguousarray(U)).to(_dev())
    s = Solver([prob], [Ut])
    s.set_time(0, t, k)
    Uin = torch.from_numpy(np.ascontiguousarray(U)).to(_dev())
    R, fl = s.residual(0, Uin)
    gl, _ = s.reconstruct(0, Uin)
    R, fl, gl = R.cpu().numpy(), fl.cpu().numpy(), gl.cpu().numpy()
    Lref, flref = oracle.residual(prob, U, t)
    glref, _, num, den = oracle.reconstruct(prob, U, t)
    sc = comp_scale(prob, U)
    dt = oracle.dt(prob, U)
    if prob.tc_mode == I.TC_KXRCF:
        n, out = kxrcf_flags(tag, prob, fl, flref, num, den, sc[0])
        assert out == 0 and n <= MISMATCHES_ALLOWED.get(tag, 0), (n, out)
    else:
        assert np.array_equal(fl, flref)
    assert (np.abs(gl - glref).reshape(prob.ncomp, -1).max(axis=1) / sc).max() <= TOL
    assert (np.abs(R - Lref).reshape(prob.ncomp, -1).max(axis=1) / (sc / dt)).max() <= TOL
    assert np.all(R[:, :, :prob.step_j, prob.step_i:] == 0.0)
    prev, tp = U.copy(), t
    for j in range(nsteps):
        s.step(1)
        d = s.last_dt()[0]
        times, _, st = s.sync()
        got = Ut.cpu().numpy()
        e = rel_state_err(prob, got, oracle.rk3_step(prob, prev, d, t=tp), sc)
        assert e <= TOL, (j, e)
        assert np.all(got[:, :, :prob.step_j, prob.step_i:] == 0.0)
        prev, tp = got, times[0]
    s.close()
    return flref


@pytest.mark.parametrize("wall_flux", [0, 1])
@pytest.mark.parametrize("charwise", [0, 1])
def test_step_tunnel_quadrants(wall_flux, charwise):
    prob, U = _tunnel(5 + wall_flux + 2 * charwise, wall_flux, charwise)
    fl = _check(f"step/tunnel_wf{wall_flux}_cw{charwise}", prob, U, 0.0, 0, 3)
    assert fl.sum() > 0


@pytest.mark.parametrize("charwise", [0, 1])
def test_step_tunnel_white_noise_probe(charwise):
    """Values, flags and residual on white noise (no steps: with nearly
    every cell troubled and many within rounding of the KXRCF threshold, a
    step compares two independent sets of near-tie decisions)."""
    prob, U = _tunnel(11 + charwise, 1, charwise, noise=True)
    fl = _check(f"step/tunnel_noise_cw{charwise}", prob, U, 0.0, 0, 0)
    assert fl.sum() > 0


@pytest.mark.parametrize("tc", [I.TC_KXRCF, I.TC_ALL, I.TC_NONE])
def test_forward_step_characteristic_wise(tc):
    """Example 3.10 at 60 x 20 after 12 steps (the reflected shock off the
    step's face, the flow around its corner)."""
    prob, U = I.forward_step(ny=20, tc_mode=tc)
    prob = prob.replace(charwise=1)
    U, t = _advance(prob, U, 12)
    _check(f"step/fstep_60x20_cw1_k12_tc{tc}", prob, U, t, 12, 3)


def test_forward_step_component_wise_early():
    """Component by component, as the paper's scheme, before its breakdown
    at the step's corner (about 26 steps at any resolution)."""
    prob, U = I.forward_step(ny=20)
    U, t = _advance(prob, U, 10)
    _check("step/fstep_60x20_cw0_k10", prob, U, t, 10, 3)


def test_step_launch_shape_invariance():
    """Strip heights and grids leave every bit of the forward step's steps
    unchanged (the step's rows fall in different work items)."""
    import torch
    from paper_2201_12193_amd.mrhweno import Solver
    prob, U = I.forward_step(ny=40)
    prob = prob.replace(charwise=1)
    outs = []
    for rows, grid in ((8, 0), (24, 64), (56, 0)):
        Ut = torch.from_numpy(U.copy()).to(_dev())
        s = Solver([prob], [Ut])
        s.set_launch(rows, grid)
        s.step(6)
        s.sync()
        outs.append(Ut.cpu().numpy())
        s.close()
    assert all(np.array_equal(outs[0], o) for o in outs[1:])


@pytest.mark.slow
def test_forward_step_fullsize_reaches_final_time():
    """600 x 200 (the paper's grid) to T = 4, characteristic-wise KXRCF
    (HWENO6-M5-I): stays physical; densities within the range of the
    paper's contours (0.32 .. 6.15) up to a margin; the residual of the
    final state at cells along the step's faces and corner, the walls, the
    inflow and the exit and at random cells against the oracle's per-cell
    evaluation."""
    import torch
    from paper_2201_12193_amd.mrhweno import Solver
    prob, U0 = I.forward_step(ny=200)
    prob = prob.replace(charwise=1)
    Ut = torch.from_numpy(U0).to(_dev())
    s = Solver([prob], [Ut])
    st = 0
    while st == 0:
        s.step(1000)
        t, steps, st = s.sync(raise_on_error=False)
        if t[0] >= prob.t_final:
            break
    print(f"forward step 600x200: t = {t[0]}, steps = {steps[0]}, status = {st}", flush=True)
    assert st == 0 and t[0] == prob.t_final and steps[0] > 3000
    U = Ut.cpu().numpy()
    fluid = np.ones((prob.ny, prob.nx), bool)
    fluid[:prob.step_j, prob.step_i:] = False
    rho = U[0, 0][fluid]
    p = (G - 1) * (U[3, 0] - 0.5 * (U[1, 0] ** 2 + U[2, 0] ** 2) / np.where(fluid, U[0, 0], 1.0))[fluid]
    print(f"rho in [{rho.min()}, {rho.max()}], p min {p.min()}", flush=True)
    assert rho.min() > 0.0 and p.min() > 0.0
    assert 0.1 < rho.min() < 0.6 and 5.5 < rho.max() < 7.5
    R, fl = s.residual(0, Ut)
    R = R.cpu().numpy()
    s.close()
    si, sj, nx, ny = prob.step_i, prob.step_j, prob.nx, prob.ny
    rng = np.random.default_rng(31)
    cells = {(int(i), int(j)) for i, j in zip(rng.integers(0, nx, 30), rng.integers(sj, ny, 30))}
    cells |= {(si - 1, j) for j in (0, 1, sj // 2, sj - 2, sj - 1)}        # before the vertical face
    cells |= {(i, sj) for i in (si - 1, si, si + 1, si + 2, nx // 2, nx - 1)}   # above the top, corner
    cells |= {(si - 2, sj + 1), (si + 1, sj + 1), (0, 0), (0, ny - 1), (nx - 1, ny - 1), (nx - 1, sj)}
    cells |= {(i, ny - 1) for i in (100, 300, 500)} | {(i, 0) for i in (10, 60, 110)}
    sc = comp_scale(prob, U)
    dt = oracle.dt(prob, U)
    worst = 0.0
    for (i, j) in sorted(cells):
        ref = oracle.residual_cell_2d(prob, U, i, j, t=t[0])
        worst = max(worst, float((np.abs(R[:, :, j, i] - ref).max(axis=1) / (sc / dt)).max()))
    assert worst <= TOL, worst
