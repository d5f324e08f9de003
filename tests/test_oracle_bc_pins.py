"""Pins of the oracle's physical boundaries (Sec. 3, boundary conditions:
supersonic inflow at the jet exit, far field from Riemann invariants) against
what the mathematics fixes: metric identities on bounded blocks, the
characteristic invariants the far-field rule must carry, fixed points,
exact conservation while the boundaries see undisturbed ambient fluid, and
transparency of the far field to an outgoing acoustic pulse.  None of them
retypes the oracle's boundary formulas."""
import numpy as np
import pytest

import oracle
from paper_2003_09926_amd import inputs as I

G = 1.4
FF, IN = I.BC_FARFIELD, I.BC_INFLOW
ALL_FF = (FF,) * 6


def _prims(q):
    rho = q[0]
    u = q[1:4] / rho
    p = (G - 1.0) * (q[4] - 0.5 * rho * (u * u).sum(0))
    return rho, u, p


def _idx(dims, i, j, k):
    return i + dims[0] * (j + dims[1] * k)


# --------------------------------------------------------------------------
# metrics on bounded blocks
# --------------------------------------------------------------------------
def test_tl_metrics_of_bounded_uniform_box_are_exact_everywhere():
    """On a Cartesian block the one-sided end differences are exact, so the
    Thomas-Lombard set equals the analytic one at every node, ends included."""
    g = I.bounded_box(9, 8, 7)
    m = oracle.metrics_tl(*g.dims, g.x, g.y, g.z, g.period, bc=ALL_FF)
    np.testing.assert_allclose(m, g.metrics, rtol=1e-13, atol=1e-15)


def test_tl_metrics_of_bounded_wavy_block_keep_the_gcl_inside():
    """sum_d delta_d S^d_a = 0 at every node whose stencil stays off the
    one-sided end nodes, and the metrics converge to the exact mapping."""
    errs = []
    for n in (12, 24):
        g = I.bounded_wavy_grid(n, n - 2, n - 4)
        ni, nj, nk = g.dims
        m = oracle.metrics_tl(ni, nj, nk, g.x, g.y, g.z, g.period, bc=ALL_FF)
        S = m[:9].reshape(3, 3, nk, nj, ni)  # [d][a][k][j][i]
        gcl = (0.5 * (S[0][:, 1:-1, 1:-1, 2:] - S[0][:, 1:-1, 1:-1, :-2])
               + 0.5 * (S[1][:, 1:-1, 2:, 1:-1] - S[1][:, 1:-1, :-2, 1:-1])
               + 0.5 * (S[2][:, 2:, 1:-1, 1:-1] - S[2][:, :-2, 1:-1, 1:-1]))
        assert np.abs(gcl).max() < 1e-15 * 50
        # J^-1 = det of the exact mapping at interior nodes (second order)
        det = np.linalg.det(np.moveaxis(g.jacobian, -1, 0))
        inner = np.zeros((nk, nj, ni), bool)
        inner[1:-1, 1:-1, 1:-1] = True
        errs.append(np.abs(1.0 / m[9] - det)[inner.ravel()].max())
    assert errs[1] < errs[0] / 3.0


# --------------------------------------------------------------------------
# far field: fixed point and Riemann invariants
# --------------------------------------------------------------------------
def test_free_stream_is_a_fixed_point_of_the_far_field():
    g = I.bounded_wavy_grid(10, 9, 8)
    m = oracle.metrics_tl(*g.dims, g.x, g.y, g.z, g.period, bc=ALL_FF)
    n = g.n
    q = I.conserved(np.ones(n), np.full(n, 0.3), np.zeros(n), np.zeros(n), np.full(n, 1 / G))
    P = oracle.default_params(bc=ALL_FF, mach_inf=0.3)
    qb = oracle.apply_bc(g.dims, P, m, q, q)
    np.testing.assert_allclose(qb, q, rtol=1e-14, atol=1e-15)


def _face_nodes(dims, d, lo):
    """boundary-layer nodes of face (d, lo) away from the other directions'
    layers, with their reference node (index 2 or n-3 along d)"""
    out = []
    rng = [range(2, dims[e] - 2) for e in range(3)]
    layers = (0, 1) if lo else (dims[d] - 2, dims[d] - 1)
    refi = 2 if lo else dims[d] - 3
    for li in layers:
        rng_d = list(rng)
        rng_d[d] = [li]
        for k in rng_d[2]:
            for j in rng_d[1]:
                for i in rng_d[0]:
                    c = [i, j, k]
                    r = list(c)
                    r[d] = refi
                    out.append((_idx(dims, *c), _idx(dims, *r)))
    return out


@pytest.mark.parametrize("mach_inf", [0.0, 0.2])
def test_subsonic_far_field_carries_the_riemann_invariants(mach_inf):
    dims = (9, 8, 7)
    g = I.bounded_box(*dims)
    rng = np.random.default_rng(7)
    n = g.n
    rho = 1.0 + 0.05 * rng.standard_normal(n)
    u = np.stack([mach_inf + 0.1 * rng.standard_normal(n), 0.1 * rng.standard_normal(n),
                  0.1 * rng.standard_normal(n)])
    p = 1 / G * (1.0 + 0.05 * rng.standard_normal(n))
    q = I.conserved(rho, u[0], u[1], u[2], p)
    P = oracle.default_params(bc=ALL_FF, mach_inf=mach_inf)
    qb = oracle.apply_bc(dims, P, g.metrics, q, q)
    rb, ub, pb = _prims(qb)
    ri, ui, pi = _prims(q)
    ue = np.array([mach_inf, 0.0, 0.0])
    seen = {True: 0, False: 0}
    for d in range(3):
        for lo in (True, False):
            nh = np.zeros(3)
            nh[d] = -1.0 if lo else 1.0
            for nb, nr in _face_nodes(dims, d, lo):
                ab, ai = np.sqrt(G * pb[nb] / rb[nb]), np.sqrt(G * pi[nr] / ri[nr])
                unb, uni, une = ub[:, nb] @ nh, ui[:, nr] @ nh, ue @ nh
                # outgoing invariant from the interior, incoming from the free stream
                assert unb + 2 * ab / (G - 1) == pytest.approx(uni + 2 * ai / (G - 1), rel=1e-13, abs=1e-13)
                assert unb - 2 * ab / (G - 1) == pytest.approx(une - 2 * 1.0 / (G - 1), rel=1e-13, abs=1e-13)
                out = unb > 0
                seen[out] += 1
                ent_b = pb[nb] / rb[nb] ** G
                src_u = ui[:, nr] if out else ue
                src_ent = pi[nr] / ri[nr] ** G if out else (1 / G)
                assert ent_b == pytest.approx(src_ent, rel=1e-12)
                tb, ts = ub[:, nb] - unb * nh, src_u - (src_u @ nh) * nh
                np.testing.assert_allclose(tb, ts, rtol=0, atol=1e-13)
    assert seen[True] > 0 and seen[False] > 0   # both branches exercised


def test_supersonic_far_field_takes_the_upwind_state():
    dims = (9, 8, 7)
    g = I.bounded_box(*dims)
    n = g.n
    q = I.conserved(np.full(n, 1.1), np.full(n, 1.6), np.full(n, 0.05), np.zeros(n), np.full(n, 0.8 / G))
    P = oracle.default_params(bc=ALL_FF, mach_inf=0.0)
    qb = oracle.apply_bc(dims, P, g.metrics, q, q)
    fs = I.conserved(np.ones(1), np.zeros(1), np.zeros(1), np.zeros(1), np.full(1, 1 / G))[:, 0]
    for nb, nr in _face_nodes(dims, 0, False):      # u_n = 1.6 > a: supersonic outflow
        np.testing.assert_array_equal(qb[:, nb], q[:, nr])
    for nb, nr in _face_nodes(dims, 0, True):       # u_n = -1.6 < -a: supersonic inflow
        np.testing.assert_allclose(qb[:, nb], fs, rtol=0, atol=1e-15)


# --------------------------------------------------------------------------
# whole steps on bounded blocks
# --------------------------------------------------------------------------
def test_inflow_layers_are_held_and_residual_is_zero_on_boundary_layers():
    dims = (16, 12, 10)
    g, q, bc = I.jet_domain_case(dims, seed=3)
    P = oracle.default_params(bc=bc, re_d=2000.0)
    r = oracle.residual(dims, P, g.metrics, q).reshape(5, dims[2], dims[1], dims[0])
    inner = np.zeros((dims[2], dims[1], dims[0]), bool)
    inner[2:-2, 2:-2, 2:-2] = True
    assert np.all(r[:, ~inner] == 0.0) and np.abs(r[:, inner]).max() > 0
    q3, _, _, _ = oracle.advance(dims, P, g.metrics, q, 3)
    a = q.reshape(5, dims[2], dims[1], dims[0])
    b = q3.reshape(5, dims[2], dims[1], dims[0])
    np.testing.assert_array_equal(b[:, :, :, :2], a[:, :, :, :2])
    assert np.abs(b[:, 2:-2, 2:-2, 2:-2] - a[:, 2:-2, 2:-2, 2:-2]).max() > 1e-6


def test_uniform_stream_is_preserved_on_a_bounded_curvilinear_block():
    g = I.bounded_wavy_grid(14, 12, 10)
    bc = I.JET_DOMAIN_BC
    m = oracle.metrics_tl(*g.dims, g.x, g.y, g.z, g.period, bc=bc)
    n = g.n
    q = I.conserved(np.ones(n), np.full(n, 0.5), np.zeros(n), np.zeros(n), np.full(n, 1 / G))
    P = oracle.default_params(bc=bc, mach_inf=0.5, re_d=500.0)
    q3, _, _, _ = oracle.advance(g.dims, P, m, q, 3)
    np.testing.assert_allclose(q3, q, rtol=0, atol=1e-12)


def test_mass_momentum_energy_conserved_while_boundaries_see_ambient():
    """A compact pulse far from every face: the interior sums of the
    conserved variables (J is constant) change only by the telescoped fluxes
    through the faces next to the boundary layers, which carry none while the
    far field hands back the ambient state.  Two stages, so that the second
    one reads boundary layers the far-field rule has set.  (More stages let
    rounding noise of the ambient region, present in a periodic block too,
    dominate the bound.)"""
    dims = (24, 20, 18)
    g = I.bounded_box(*dims)
    r2 = (g.x - 2.0) ** 2 + g.y ** 2 + g.z ** 2
    bump = np.exp(-r2 / 0.15 ** 2)
    q = I.conserved(1.0 + 0.1 * bump, 0.05 * bump, -0.03 * bump, 0.02 * bump, (1.0 + 0.2 * bump) / G)
    P = oracle.default_params(bc=ALL_FF, re_d=300.0, dt_fixed=2e-3, n_stages=2, rk_alpha=[0.5, 1.0])
    q1, _, _, _ = oracle.step(dims, P, g.metrics, q)
    a = q.reshape(5, dims[2], dims[1], dims[0])[:, 2:-2, 2:-2, 2:-2]
    b = q1.reshape(5, dims[2], dims[1], dims[0])[:, 2:-2, 2:-2, 2:-2]
    nint = a[0].size
    for v in range(5):
        change = np.abs(b[v] - a[v]).sum()
        assert change > 1e-4
        # rounding of the per-node updates bounds what is left
        assert abs(b[v].sum() - a[v].sum()) <= 1e-12 * change + nint * 4e-16 * np.abs(a[v]).max()
    # a far field that handed back a wrong ambient state would not conserve
    Pw = oracle.default_params(bc=ALL_FF, re_d=300.0, dt_fixed=2e-3, n_stages=2, rk_alpha=[0.5, 1.0],
                               mach_inf=0.01)
    qw, _, _, _ = oracle.step(dims, Pw, g.metrics, q)
    bw = qw.reshape(5, dims[2], dims[1], dims[0])[:, 2:-2, 2:-2, 2:-2]
    assert abs(bw[1].sum() - a[1].sum()) > 1e3 * (1e-12 * change + nint * 4e-16 * np.abs(a[1]).max())


def test_far_field_lets_an_acoustic_pulse_leave():
    """A right-running plane acoustic pulse (p' = rho a u', rho' = p'/a^2)
    leaves through the far-field face at x = 4 and nothing comes back; in a
    periodic block of the same size it stays.  Inviscid, no subgrid model."""
    dims = (161, 5, 5)
    bc = (FF, FF, I.BC_PERIODIC, I.BC_PERIODIC, I.BC_PERIODIC, I.BC_PERIODIC)
    g = I.bounded_box(*dims, bounded=(True, False, False))
    amp = 1e-3
    pp = amp * np.exp(-((g.x - 2.0) / 0.2) ** 2) / G
    q = I.conserved(1.0 + pp, pp, np.zeros(g.n), np.zeros(g.n), 1 / G + pp)
    P = oracle.default_params(bc=bc, re_d=float("inf"), cs=0.0)
    _, p0 = _prims(q)[0], _prims(q)[2]
    e0 = ((p0 - 1 / G) ** 2).sum()
    qt, t, _, _ = oracle.advance(dims, P, g.metrics, q, 1)
    steps = int(np.ceil(3.0 / t))
    qt, t, _, _ = oracle.advance(dims, P, g.metrics, q, steps)
    assert t > 2.9
    e_left = ((_prims(qt)[2] - 1 / G) ** 2).sum()
    Pp = oracle.default_params(re_d=float("inf"), cs=0.0)
    gp = I.bounded_box(*dims, bounded=(False, False, False))
    qp, _, _, _ = oracle.advance(dims, Pp, gp.metrics, q, steps)
    e_periodic = ((_prims(qp)[2] - 1 / G) ** 2).sum()
    assert e_periodic > 0.5 * e0
    assert e_left < 1e-6 * e0


# --------------------------------------------------------------------------
# centreline of a cylindrical mesh
# --------------------------------------------------------------------------
CYL = I.JET_CYLINDER_BC


def _cyl(dims=(14, 9, 16), seed=5, noise=0.01):
    g, q, bc = I.jet_cylinder_case(dims, seed=seed, noise=noise)
    m = oracle.metrics_tl(*g.dims, g.x, g.y, g.z, g.period, bc=bc)
    return g, q, bc, m


def test_centreline_takes_the_ordered_azimuthal_mean_of_the_adjacent_ring():
    import math
    g, q, bc, m = _cyl()
    ni, nj, nk = g.dims
    rng = np.random.default_rng(3)
    qr = q * (1.0 + 0.01 * rng.standard_normal(q.shape))
    P = oracle.default_params(bc=bc)
    qb = oracle.apply_bc(g.dims, P, m, qr, q).reshape(5, nk, nj, ni)
    a = qr.reshape(5, nk, nj, ni)
    for i in range(2, ni - 2):                     # inflow layers i < 2 are held
        np.testing.assert_array_equal(qb[:, :, 1, i], a[:, :, 2, i])
        axis = qb[:, :, 0, i]
        assert np.all(axis == axis[:, :1])         # one value for every azimuth
        for v in range(5):
            assert axis[v, 0] == pytest.approx(math.fsum(a[v, :, 2, i]) / nk, rel=1e-15)
    np.testing.assert_array_equal(qb[:, :, :, :2], q.reshape(5, nk, nj, ni)[:, :, :, :2])


def test_uniform_stream_is_preserved_on_the_cylindrical_mesh():
    g, _, bc, m = _cyl()
    n = g.n
    assert np.isinf(m[9].reshape(g.dims[2], g.dims[1], g.dims[0])[:, 0, :]).all()  # no metrics on the axis
    q = I.conserved(np.ones(n), np.full(n, 0.5), np.zeros(n), np.zeros(n), np.full(n, 1 / G))
    P = oracle.default_params(bc=bc, mach_inf=0.5, re_d=500.0)
    q3, _, _, _ = oracle.advance(g.dims, P, m, q, 3)
    np.testing.assert_allclose(q3, q, rtol=0, atol=1e-12)


def _rotate_quarter(q, dims):
    """the field turned by +90 degrees about the x axis on an nk = 4 m mesh:
    node k takes the state of node k - nk/4 with (rho v, rho w) -> (-rho w, rho v)"""
    ni, nj, nk = dims
    a = q.reshape(5, nk, nj, ni)
    b = np.roll(a, nk // 4, axis=1).copy()
    v, w = b[2].copy(), b[3].copy()
    b[2], b[3] = -w, v
    return b.reshape(5, -1)


def test_exact_cylindrical_metrics_match_thomas_lombard_off_the_axis():
    """The metric set of the mapping and the discrete Thomas-Lombard set agree
    to second order away from the axis and the one-sided end layers."""
    errs = []
    for n in (8, 16):
        g = I.cylindrical_grid(4 * n, n + 1, 4 * n)
        m = oracle.metrics_tl(*g.dims, g.x, g.y, g.z, g.period, bc=CYL)
        ni, nj, nk = g.dims
        sel = np.zeros((nk, nj, ni), bool)
        sel[:, 2:-1, 1:-1] = True
        sel = sel.ravel()
        errs.append(np.abs(m[:9, sel] - g.metrics[:9, sel]).max() / np.abs(g.metrics[:9, sel]).max())
    assert errs[1] < errs[0] / 3.0 and errs[1] < 1e-2


def test_a_quarter_turn_commutes_with_the_step():
    """With the exact metrics of the cylindrical mesh, the mesh and every
    rule (far field, centreline average, inflow) are invariant under a turn
    by a quarter of the azimuth, so stepping a turned state gives the turned
    result (to the rounding of cos/sin).  (The Thomas-Lombard set is not
    exactly invariant: its cyclic form treats the coordinates unequally.)"""
    dims = (14, 9, 16)
    g, q, bc, _ = _cyl(dims, seed=6)
    m = g.metrics
    P = oracle.default_params(bc=bc, re_d=3000.0)
    qa, _, _, _ = oracle.advance(dims, P, m, q, 2)
    qr = _rotate_quarter(q, dims)
    qb, _, _, _ = oracle.advance(dims, P, m, qr, 2)
    scale = np.abs(qa).max(axis=1, keepdims=True)
    assert np.max(np.abs(qb - _rotate_quarter(qa, dims)) / scale) < 1e-12
    assert np.max(np.abs(qa - q) / scale) > 1e-4          # the state did change
