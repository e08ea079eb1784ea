"""1D steps across the tile edges of the step's 1D kernel (k1_fused: tiles
of 250 cells, each recomputing the face data and flags of three ring cells
on either side): jumps placed on the faces between tiles, a ragged last
tile (N = 777), every troubled-cell mode and both component- and
characteristic-wise Step 1; each GPU step against the oracle's step with
the GPU's time step (bit-equal to the oracle's), within 1e-12 of each
component's scale."""
import numpy as np
import pytest

import oracle
from paper_2201_12193_amd import inputs as I
from tests.parity_util import comp_scale, rel_state_err

pytestmark = pytest.mark.gpu
TOL = 1e-12
N = 777
EDGES = (250, 500)        # first cells of the second and third tile


def _euler_jumps():
    """Four constant states (rho, u, p) with jumps on the faces x = 250/N,
    500/N (tile edges) and 640/N, transmissive ends."""
    prob = I.Problem(dim=1, nx=N, x0=0.0, x1=1.0, system=I.EULER, bc_x=I.TRANSMISSIVE, t_final=1.0)
    xs = [e / N for e in EDGES] + [640 / N]
    st = [(1.0, 0.0, 1.0), (0.3, 0.2, 0.4), (0.7, -0.1, 0.8), (0.5, 0.3, 0.6)]

    def cons(x):
        k = (x > xs[0]).astype(int) + (x > xs[1]).astype(int) + (x > xs[2]).astype(int)
        r = np.array([s[0] for s in st])[k]
        u = np.array([s[1] for s in st])[k]
        p = np.array([s[2] for s in st])[k]
        return I.euler1d_cons(r, u, p, 1.4)
    return prob, I.project_1d(prob, cons, jumps=xs)


def _burgers_shock():
    """Burgers, periodic: u0 = 0.5 + sin(2 pi x) with a jump of 0.8 on the
    face x = 250/N, Lax-Friedrichs."""
    prob = I.Problem(dim=1, nx=N, x0=0.0, x1=1.0, system=I.BURGERS, bc_x=I.PERIODIC, t_final=1.0)
    xj = EDGES[0] / N
    U = I.project_1d(prob, lambda x: (0.5 + np.sin(2 * np.pi * x) + 0.8 * (x > xj))[None], jumps=[xj])
    return prob, U


def _steps(prob, U, n):
    import torch
    from paper_2201_12193_amd.mrhweno import Solver
    Ut = torch.from_numpy(np.ascontiguousarray(U)).cuda()
    s = Solver([prob], [Ut])
    sc = comp_scale(prob, U)
    prev = U.copy()
    worst = 0.0
    for k in range(n):
        s.step(1)
        dt = s.last_dt()[0]
        s.sync()
        got = Ut.cpu().numpy()
        assert dt == oracle.dt(prob, prev), (k, dt, oracle.dt(prob, prev))
        e = rel_state_err(prob, got, oracle.rk3_step(prob, prev, dt), sc)
        worst = max(worst, e)
        assert e <= TOL, (k, e)
        prev = got
    s.close()
    return worst


@pytest.mark.parametrize("charwise", [0, 1])
@pytest.mark.parametrize("tc", [I.TC_KXRCF, I.TC_TVB, I.TC_ALL, I.TC_NONE])
def test_euler_jumps_on_tile_edges(tc, charwise):
    prob, U = _euler_jumps()
    prob = prob.replace(tc_mode=tc, charwise=charwise, tvb_m=1.0)
    if tc == I.TC_KXRCF:
        _, fl = oracle.residual(prob, U)
        hit = np.flatnonzero(fl)
        print(f"troubled cells at t = 0: {hit.tolist()}", flush=True)
        for e in EDGES:   # the jumps on the tile edges are troubled on one side or both
            assert np.isin([e - 1, e], hit).any(), e
    w = _steps(prob, U, 8)
    print(f"tc {tc} charwise {charwise}: worst step difference {w:.2e}", flush=True)


@pytest.mark.parametrize("tc", [I.TC_KXRCF, I.TC_TVB])
@pytest.mark.parametrize("mod", [I.MOD_PERSIST, I.MOD_INTERNAL, I.MOD_STAGE])
def test_burgers_shock_on_a_tile_edge(tc, mod):
    prob, U = _burgers_shock()
    prob = prob.replace(tc_mode=tc, modification=mod, tvb_m=1.0)
    w = _steps(prob, U, 8)
    print(f"burgers tc {tc} mod {mod}: worst step difference {w:.2e}", flush=True)
