"""Host-side statistics helpers: bins and the potential core length."""
import numpy as np

from paper_2003_09926_amd import inputs as I
from paper_2003_09926_amd import stats as ST


def test_potential_core_length_closed_form():
    x = np.linspace(0.0, 10.0, 101)
    u = 1.4 * (1.0 - 0.02 * x)                      # 0.95 U_j at x = 2.5
    assert abs(ST.potential_core_length(x, u, 1.4) - 2.5) < 1e-12
    assert ST.potential_core_length(x, np.full_like(x, 1.4), 1.4) == 10.0
    assert ST.potential_core_length(x, np.full_like(x, 0.5), 1.4) == 0.0


def test_radial_bins_on_the_cylindrical_mesh_follow_the_rings():
    g = I.cylindrical_grid(6, 9, 16, radius=1.6)
    b = ST.radial_bins(g.y, g.z, g.dims, 3, nbins=10, rmax=1.7).reshape(16, 9)
    # ring j sits at r = 0.2 j (no ring on a bin edge of width 0.17)
    for j in range(9):
        assert np.all(b[:, j] == int(np.floor(0.2 * j / 0.17)))
    b2 = ST.radial_bins(g.y, g.z, g.dims, 3, nbins=10, rmax=1.5).reshape(16, 9)
    assert np.all(b2[:, 8] == -1)                    # r = 1.6 beyond rmax
