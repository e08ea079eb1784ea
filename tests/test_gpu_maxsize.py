"""The largest 2D grid the library takes: 13 nx ny < 2^30, 9088 x 9088
(82.6 million cells, 7.9 GB per state), where the stage kernel's 30-bit
staging offsets come closest to their limit.  2D Euler contact wave
(a smooth density wave and a contact discontinuity on a cell face,
periodic), through the C ABI at the shapes the autotuned step uses:
sampled residuals against the oracle's per-cell evaluation (the last rows
and columns, where the offsets are largest, the contact's troubled cells,
random cells), the troubled cells found exactly along the contact, the
time step bit-equal to the oracle's, and one SSP-RK3 step that conserves
every component's total."""
import numpy as np
import pytest

import oracle
from paper_2201_12193_amd import inputs as I
from tests.parity_util import comp_scale

pytestmark = [pytest.mark.gpu, pytest.mark.slow]
N = 9088
TOL = 1e-12


def test_largest_grid_residual_flags_and_step():
    import torch
    from paper_2201_12193_amd.mrhweno import Solver
    prob, U, _ = I.contact_wave_2d(N, N, N)
    assert 13 * prob.ncell < 2 ** 30 <= 13 * (N + 1) ** 2
    print(f"largest grid {N} x {N}: {prob.ncell} cells, {U.nbytes / 1e9:.1f} GB per state", flush=True)
    Ut = torch.from_numpy(U).cuda()
    s = Solver([prob], [Ut])
    s.set_launch(56, 512)
    R, fl = s.residual(0, Ut)
    fl = fl.cpu().numpy()
    # troubled cells: only next to the two contacts (x = X/2 and the periodic
    # seam), on every row
    cols = np.flatnonzero(fl.any(axis=0))
    near = np.minimum(np.abs(cols - (N // 2 - 0.5)), np.minimum(cols + 0.5, N - 0.5 - cols))
    print(f"troubled cells {int(fl.sum())} in columns {cols.tolist()}", flush=True)
    assert cols.size > 0 and near.max() <= 3.0
    assert fl[:, N // 2 - 2:N // 2 + 2].any(axis=1).all()
    rng = np.random.default_rng(9088)
    cells = {(int(i), int(j)) for i, j in zip(rng.integers(0, N, 24), rng.integers(0, N, 24))}
    for j in (0, 1, 777, N // 2, N - 3, N - 2, N - 1):
        for i in (0, 1, 61, 62, N // 2 - 2, N // 2 - 1, N // 2, N // 2 + 1, N - 2, N - 1):
            cells.add((i, j))
    sc = comp_scale(prob, U)
    dt = oracle.dt(prob, U)
    idx_i = torch.tensor([c[0] for c in sorted(cells)], device=Ut.device)
    idx_j = torch.tensor([c[1] for c in sorted(cells)], device=Ut.device)
    got = R[:, :, idx_j, idx_i].cpu().numpy()
    del R
    worst = 0.0
    for n, (i, j) in enumerate(sorted(cells)):
        ref = oracle.residual_cell_2d(prob, U, i, j)
        worst = max(worst, float((np.abs(got[:, :, n] - ref).max(axis=1) / (sc / dt)).max()))
    print(f"sampled residuals: {len(cells)} cells, worst relative difference {worst:.3e}", flush=True)
    assert worst <= TOL, worst
    # one step: the oracle's time step bit for bit, totals conserved
    before = Ut[:, 0].sum(dim=(1, 2)).cpu().numpy()
    mag = Ut[:, 0].abs().sum(dim=(1, 2)).cpu().numpy()
    s.step(1)
    s.sync()
    assert s.last_dt()[0] == dt
    after = Ut[:, 0].sum(dim=(1, 2)).cpu().numpy()
    s.close()
    drift = np.abs(after - before) / mag
    print(f"step: dt {dt:.6e}, relative drift of the totals {drift.tolist()}", flush=True)
    assert drift.max() <= 1e-13
    assert torch.isfinite(Ut).all()
