"""The domain split of the paper (Sec. 4.1 partitioning, Sec. 4.3 two-layer
ghost fringe) mirrored on the CPU: parts advanced from the oracle's own
residual with ghost exchanges between stages must reproduce the unsplit
oracle bitwise; dropping the corner ghosts must not."""
import numpy as np
import pytest

import oracle
from oracle import domain as OD
from paper_2003_09926_amd import inputs as I


def test_part_sizes_balanced():
    # the quotient in every part, the remainder spread one node each over the first parts
    assert OD.part_sizes(10, 3) == [4, 3, 3]
    assert OD.part_sizes(12, 4) == [3, 3, 3, 3]
    assert OD.part_sizes(37, 4) == [10, 9, 9, 9]
    for n in range(4, 60):
        for p in range(1, n // 2 + 1):
            s = OD.part_sizes(n, p)
            assert sum(s) == n and max(s) - min(s) <= 1 and s == sorted(s, reverse=True)
    with pytest.raises(ValueError):
        OD.part_sizes(5, 3)


def _case():
    g = I.wavy_grid(23, 10, 19)
    m = oracle.metrics_tl(*g.dims, g.x, g.y, g.z, g.period)
    q = I.jet_state(g, 1.4, seed=7, noise=0.03)
    return g, m, q


@pytest.mark.parametrize("parts", [(2, 1), (1, 2), (3, 1), (1, 4), (2, 3)])
def test_split_matches_unsplit_bitwise(parts):
    g, m, q = _case()
    P = oracle.default_params(re_d=2.0e3)
    q1, t1, rms1, linf1 = oracle.advance(g.dims, P, m, q, 2)
    q2, t2, rms2, linf2 = OD.advance(g.dims, P, m, q, 2, parts=parts)
    assert np.array_equal(q1, q2)
    assert t1 == t2
    # norms: the maxima exactly, the sums up to their order
    assert np.array_equal(linf1, linf2)
    np.testing.assert_allclose(rms2, rms1, rtol=1e-13, atol=0)


def test_corner_ghosts_matter():
    """The viscous fluxes at a part's edge take cross differences through the
    ghost nodes that are ghosts along both xi and zeta; leaving those stale
    changes the result (so the bitwise test above sees the corners)."""
    g, m, q = _case()
    P = oracle.default_params(re_d=2.0e3)
    q1, _, _, _ = oracle.advance(g.dims, P, m, q, 2)
    q2, _, _, _ = OD.advance(g.dims, P, m, q, 2, parts=(2, 2), corners=False)
    assert not np.array_equal(q1, q2)
    q3, _, _, _ = OD.advance(g.dims, P, m, q, 2, parts=(2, 2))
    assert np.array_equal(q1, q3)
