"""Pins of the set-ups of the paper's 1D shock examples (inputs only)."""
import math

import numpy as np

from paper_2201_12193_amd import inputs as I


def test_shock_density_left_state_is_a_mach3_post_shock_state():
    """Example 3.6's printed left state is the gas behind a Mach 3 shock
    running into rho = 1, u = 0, p = 1 (Rankine-Hugoniot, gamma = 1.4), to
    the printed digits."""
    g, M = 1.4, 3.0
    rho2 = (g + 1) * M * M / ((g - 1) * M * M + 2)
    p2 = 1 + 2 * g / (g + 1) * (M * M - 1)
    s = M * math.sqrt(g)
    u2 = s * (1 - 1 / rho2)
    _, U, left = I.example_shock_density()
    assert abs(left[0] - rho2) < 1e-6 and abs(left[1] - u2) < 1e-6 and abs(left[2] - p2) < 1e-6
    # the cells left of x = -4 hold that state exactly (first moments zero)
    prob, _, _ = I.example_shock_density()
    x = prob.x0 + (np.arange(prob.nx) + 0.5) * prob.dx
    inside = x < -4.0 - prob.dx
    assert np.allclose(U[0, 0, inside], left[0], rtol=1e-15) and np.all(U[:, 1, inside] == 0.0)


def test_sedov_energy_deposit():
    prob, U = I.example_sedov()
    c = prob.nx // 2
    assert abs(prob.x0 + (c + 0.5) * prob.dx) < 1e-15          # the centre cell straddles x = 0
    assert U[2, 0, c] * prob.dx == 3200000.0
    assert np.all(U[0, 0] == 1.0) and np.all(U[1] == 0.0) and np.all(U[2, 1] == 0.0)
    assert np.all(np.delete(U[2, 0], c) == 1e-12)
