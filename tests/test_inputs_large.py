"""The separable generator of the largest grids, and the grid-size limits
of the C-ABI (host-side validation, no GPU)."""
import numpy as np

from paper_2201_12193_amd import inputs as I
from paper_2201_12193_amd import mrhweno as M


def test_contact_wave_moments_equal_the_quadrature_projection():
    """Separable products of 1D cell moments = the 2D Gauss projection of
    the same field (the contact lies on a cell face: exact on both sides)."""
    prob, U, st = I.contact_wave_2d(7, 24, 12)
    rng = np.random.default_rng(7)
    phx, phy = rng.uniform(0.0, 1.0, 2)
    X = prob.nx / prob.ny

    def cons(x, y):
        rho = 1.0 + 0.2 * np.sin(2 * np.pi * (x + phx)) * np.sin(2 * np.pi * (y + phy)) + 0.5 * (x > X / 2)
        return I.euler2d_cons(rho, st["u"] + 0 * x, st["v"] + 0 * x, st["p"] + 0 * x, 1.4)
    ref = I.project_2d(prob, cons)
    assert np.abs(U - ref).max() <= 1e-14
    assert prob.dx == prob.dy


def test_grid_size_limits():
    """2D: 13 nx ny < 2^30 (the stage kernel's 30-bit staging offsets);
    1D: nx < 2^30."""
    top = I.Problem(dim=2, nx=9088, ny=9088)                   # 82,591,744 cells
    assert 13 * top.ncell < 2 ** 30 <= 13 * 9089 * 9089
    assert M.workspace_bytes([top]) > 0
    assert M.workspace_bytes([I.Problem(dim=2, nx=9089, ny=9089)]) == 0
    assert M.workspace_bytes([I.Problem(dim=2, nx=18176, ny=4544, x1=4.0)]) > 0           # same cells
    assert M.workspace_bytes([I.Problem(dim=2, nx=18178, ny=4545, x1=18178 / 4545)]) == 0
    assert M.workspace_bytes([I.Problem(dim=1, nx=2 ** 30 - 1)]) > 0
    assert M.workspace_bytes([I.Problem(dim=1, nx=2 ** 30)]) == 0
