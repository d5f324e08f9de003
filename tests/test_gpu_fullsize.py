"""Parity at the full production size, 512 x 256 x 256 (33.5M nodes, the
separable tanh-stretched jet grid with analytic metrics), in the launch
configuration the benchmark times.

The oracle cannot step 33.5M nodes in seconds, but one step at a node depends
only on the nodes within 5 stages x 2 = 10 of it.  So for each sampled node
the oracle steps a 21^3 periodic patch around it (its wrong periodic closure
reaches at most 9 nodes in from the patch faces) with the full-field dt, and
the centre is compared with the GPU's value.
"""
import numpy as np
import pytest

import oracle
from paper_2003_09926_amd import inputs as I

from _parity import flat, patch

pytestmark = pytest.mark.gpu

DIMS = (512, 256, 256)
R = 10


def _samples(dims, rng, n=24):
    ni, nj, nk = dims
    pts = [(0, 0, 0), (ni - 1, nj - 1, nk - 1), (27, 11, 31), (28, 12, 32), (255, 127, 128),
           (1, nj - 2, 1), (ni - 2, 1, nk - 2), (ni // 2, nj // 2, 0)]
    while len(pts) < n:
        pts.append(tuple(int(rng.integers(0, d)) for d in dims))
    return pts


def test_fullsize_one_step_sampled_parity():
    import torch
    from paper_2003_09926_amd import binding as B
    assert torch.cuda.is_available()
    print("[gpu-case] full size 512x256x256 one step", flush=True)
    g, q = I.stretched_jet_case(DIMS, seed=2)
    P = oracle.default_params(re_d=1.0e6)
    dt, _ = oracle.cfl_dt(g.dims, P, g.metrics, q)
    with B.Solver(g.dims, B.params_default(re_d=1.0e6)) as s:
        s.set_grid_metrics(g.metrics)
        s.set_state(q)
        dtg, _ = s.eval_dt()
        s.advance(1)
        qg = s.get_state()
        t, _, _ = s.clock()
    assert abs(dtg - dt) <= 1e-13 * dt and abs(t - dt) <= 1e-13 * dt
    rng = np.random.default_rng(12)
    worst = 0.0
    for c in _samples(DIMS, rng):
        qp = patch(q, DIMS, c, R)
        mp = patch(g.metrics, DIMS, c, R)
        q1, _, _, _ = oracle.step((2 * R + 1,) * 3, P, mp, qp, dt=dt)
        centre = R + (2 * R + 1) * (R + (2 * R + 1) * R)
        n = flat(DIMS, *c)
        for v in range(5):
            inc_o = q1[v, centre] - qp[v, centre]
            inc_g = qg[v, n] - q[v, n]
            err = abs(inc_g - inc_o)
            worst = max(worst, err)
            # increment within 1e-9 of its own size (or of the state's roundoff)
            assert err <= 1e-9 * abs(inc_o) + 1e-15 * (1 + abs(q[v, n])), (c, v, inc_g, inc_o)
    print(f"[gpu-case] worst abs increment error {worst:.3e}", flush=True)


def test_fullsize_bounded_jet_domain_one_step():
    """The bounded jet domain of the benchmark (512 x 256 x 256, inflow at the
    jet exit, far field elsewhere), one step in the benchmark's launch
    configuration: inflow layers held bitwise; every boundary layer equals the
    oracle's boundary rule applied to the GPU's own interior; interior nodes at
    least 12 nodes from every face match the oracle stepping a periodic patch
    around them (the patch closure cannot reach the centre) with the
    full-field dt."""
    import torch
    from paper_2003_09926_amd import binding as B
    assert torch.cuda.is_available()
    print("[gpu-case] full size bounded jet domain 512x256x256 one step", flush=True)
    g, q, bc = I.jet_domain_case(DIMS, mach=1.4, seed=2)
    P = oracle.default_params(re_d=1.0e6, bc=bc)
    dt, _ = oracle.cfl_dt(g.dims, P, g.metrics, q)
    with B.Solver(g.dims, B.params_default(re_d=1.0e6, bc=bc)) as s:
        s.set_grid_metrics(g.metrics)
        s.set_state(q)
        dtg, _ = s.eval_dt()
        s.advance(1)
        qg = s.get_state()
    assert abs(dtg - dt) <= 1e-13 * dt
    ni, nj, nk = DIMS
    a = q.reshape(5, nk, nj, ni)
    b = qg.reshape(5, nk, nj, ni)
    np.testing.assert_array_equal(b[:, :, :, :2], a[:, :, :, :2])
    qb = oracle.apply_bc(DIMS, P, g.metrics, qg, q)
    scale = np.abs(qg).max(axis=1, keepdims=True)
    assert np.max(np.abs(qb - qg) / scale) <= 1e-13
    rng = np.random.default_rng(13)
    Pp = oracle.default_params(re_d=1.0e6)           # the patch is periodic
    for _ in range(8):
        c = (int(rng.integers(12, ni - 12)), int(rng.integers(12, nj - 12)), int(rng.integers(12, nk - 12)))
        qp = patch(q, DIMS, c, R)
        mp = patch(g.metrics, DIMS, c, R)
        q1, _, _, _ = oracle.step((2 * R + 1,) * 3, Pp, mp, qp, dt=dt)
        centre = R + (2 * R + 1) * (R + (2 * R + 1) * R)
        n = flat(DIMS, *c)
        for v in range(5):
            inc_o = q1[v, centre] - qp[v, centre]
            inc_g = qg[v, n] - q[v, n]
            assert abs(inc_g - inc_o) <= 1e-9 * abs(inc_o) + 1e-15 * (1 + abs(q[v, n])), (c, v, inc_g, inc_o)
