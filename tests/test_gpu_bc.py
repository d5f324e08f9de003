"""Physical boundaries (supersonic inflow at the jet exit, Riemann-invariant
far field) on the GPU against the CPU oracle, through the C ABI.

Same bars as the periodic parity tests: state after a step <= 1e-12,
increment <= 1e-9, residual <= 1e-10 (relative L2 per variable); metrics
1e-13; boundary-layer values and inflow layers compared to the same bars,
the held inflow layers and the zero residual on boundary layers bitwise.
FP32-flux form: the bounds of its periodic tests.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2003_09926_amd import inputs as I

from _parity import per_var_rel

pytestmark = pytest.mark.gpu

TOL_STATE = 1e-12
TOL_INC = 1e-9
TOL_RES = 1e-10
FF, IN, PER = I.BC_FARFIELD, I.BC_INFLOW, I.BC_PERIODIC


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU test without a GPU"
    from paper_2003_09926_amd import binding
    binding.library()
    return binding


def _log(msg):
    print(f"[gpu-case] {msg}", flush=True)


CASES = {
    # every direction bounded; interior 36 x 26 x 22 spans several 28 x 12
    # tiles with ragged tails
    "jetdomain_40x30x26": dict(dims=(40, 30, 26), bc=I.JET_DOMAIN_BC, mach_inf=0.0),
    # xi bounded (inflow / far field), eta far field, zeta periodic, coflow
    "mixed_33x21x17": dict(dims=(33, 21, 17), bc=(IN, FF, FF, FF, PER, PER), mach_inf=0.1),
    # far field on every face, the smallest bounded block
    "farfield_5x7x6": dict(dims=(5, 7, 6), bc=(FF,) * 6, mach_inf=0.0),
}


def _case(name, seed=1):
    c = CASES[name]
    g, q, bc = I.jet_domain_case(c["dims"], seed=seed, bc=c["bc"])
    return g, q, bc, c["mach_inf"]


@pytest.mark.parametrize("name", list(CASES))
def test_bounded_residual_matches_oracle(B, name):
    _log(f"bounded residual {name}")
    g, q, bc, mi = _case(name)
    with B.Solver(g.dims, B.params_default(bc=bc, mach_inf=mi)) as s:
        s.set_grid_metrics(g.metrics)
        s.set_state(q)
        r = s.eval_residual()
        dt, lm = s.eval_dt()
    P = oracle.default_params(bc=bc, mach_inf=mi)
    ro = oracle.residual(g.dims, P, g.metrics, q)
    ni, nj, nk = g.dims
    inner = np.ones((nk, nj, ni), bool)
    for d, n in enumerate(g.dims):
        if bc[2 * d] != PER:
            sl = [slice(None)] * 3
            sl[2 - d] = np.r_[0, 1, n - 2, n - 1]
            inner[tuple(sl)] = False
    inner = inner.ravel()
    assert np.all(r[:, ~inner] == 0.0) and np.all(ro[:, ~inner] == 0.0)
    assert max(per_var_rel(r, ro)) <= TOL_RES
    dto, lmo = oracle.cfl_dt(g.dims, P, g.metrics, q)
    assert abs(dt - dto) <= 1e-13 * dto and abs(lm - lmo) <= 1e-13 * lmo


@pytest.mark.parametrize("name", list(CASES))
def test_bounded_steps_per_step_parity(B, name):
    """three steps, each from the oracle's state: state, increment, norms,
    clock; inflow layers held bitwise"""
    _log(f"bounded three steps {name}")
    g, q, bc, mi = _case(name, seed=2)
    P = oracle.default_params(bc=bc, mach_inf=mi, re_d=2.0e4)
    qo = q.copy()
    t_o = 0.0
    with B.Solver(g.dims, B.params_default(bc=bc, mach_inf=mi, re_d=2.0e4)) as s:
        s.set_grid_metrics(g.metrics)
        s.set_state(q)
        for step in range(3):
            q_prev = qo
            qo, dto, rms_o, linf_o = oracle.step(g.dims, P, g.metrics, qo)
            t_o += dto
            s.advance(1)
            qg = s.get_state()
            rms, linf = s.residual_norms()
            t, _, n = s.clock()
            assert max(per_var_rel(qg, qo)) <= TOL_STATE, step
            assert max(per_var_rel(qg - q_prev, qo - q_prev)) <= TOL_INC, step
            assert np.allclose(rms, rms_o, rtol=1e-9, atol=0) and np.allclose(linf, linf_o, rtol=1e-9, atol=0)
            assert n == step + 1 and math.isclose(t, t_o, rel_tol=1e-13)
            s.set_state(qo)
    if bc[0] == IN:
        nk, nj, ni = g.dims[2], g.dims[1], g.dims[0]
        a = q.reshape(5, nk, nj, ni)[:, :, :, :2]
        b = qg.reshape(5, nk, nj, ni)[:, :, :, :2]
        np.testing.assert_array_equal(b, a)


def test_bounded_free_running_and_tile_shapes_agree(B):
    """ten free-running steps match the oracle; two launch shapes give
    bitwise identical states"""
    _log("bounded jet domain 40x30x26 ten steps, two tile shapes")
    g, q, bc, mi = _case("jetdomain_40x30x26", seed=3)
    P = oracle.default_params(bc=bc)
    qo, _, _, _ = oracle.advance(g.dims, P, g.metrics, q, 10)
    out = []
    for tile, kc in (((28, 12), 0), ((12, 12), 5)):
        with B.Solver(g.dims, B.params_default(bc=bc, tile_i=tile[0], tile_j=tile[1], kchunk=kc)) as s:
            s.set_grid_metrics(g.metrics)
            s.set_state(q)
            s.advance(10)
            out.append(s.get_state())
    assert np.array_equal(out[0], out[1])
    assert max(per_var_rel(out[0], qo)) <= TOL_STATE
    assert max(per_var_rel(out[0] - q, qo - q)) <= TOL_INC


def test_bounded_tl_metrics_and_uniform_stream(B):
    """Thomas-Lombard metrics with one-sided ends on a bounded curvilinear
    block match the oracle; a uniform stream with matching inflow and far
    field stays uniform"""
    _log("bounded wavy 18x14x12 metrics and uniform stream")
    g = I.bounded_wavy_grid(18, 14, 12)
    bc = I.JET_DOMAIN_BC
    mo = oracle.metrics_tl(*g.dims, g.x, g.y, g.z, g.period, bc=bc)
    n = g.n
    q = I.conserved(np.ones(n), np.full(n, 0.5), np.zeros(n), np.zeros(n), np.full(n, 1 / 1.4))
    with B.Solver(g.dims, B.params_default(bc=bc, mach_inf=0.5, re_d=500.0)) as s:
        s.set_grid_coords(g.x, g.y, g.z, g.period)
        mg = s.get_grid_metrics()
        s.set_state(q)
        s.advance(3)
        q3 = s.get_state()
    scale = np.max(np.abs(mo[:9]))
    assert np.max(np.abs(mg[:9] - mo[:9])) <= 1e-13 * scale
    assert np.max(np.abs(mg[9] - mo[9]) / mo[9]) <= 1e-13
    np.testing.assert_allclose(q3, q, rtol=0, atol=1e-12)


def _farfield_branches(q, m, dims, bc, gamma=1.4):
    """Per far-field boundary node, the side the far-field rule takes entropy
    and tangential velocity from, computed from the state of its reference
    node (index 2 or n-3 along the face normal) as the rule defines it:
    +-2 supersonic out/in, +1 subsonic outflow (interior), -1 subsonic inflow
    (free stream).  Test-side restatement of the decision only."""
    ni, nj, nk = dims
    Q = q.reshape(5, nk, nj, ni)
    M = m.reshape(10, nk, nj, ni)
    out = []
    for d in range(3):
        for side in (0, 1):
            if bc[2 * d + side] != I.BC_FARFIELD:
                continue
            n = dims[d]
            ref = 2 if side == 0 else n - 3
            for layer in ((0, 1) if side == 0 else (n - 2, n - 1)):
                sl = [slice(None)] * 3
                sl[2 - d] = ref
                qi = Q[(slice(None),) + tuple(sl)]
                sl[2 - d] = layer
                mm = M[(slice(None),) + tuple(sl)]
                r = qi[0]
                u = qi[1:4] / r
                p = (gamma - 1) * (qi[4] - 0.5 * r * (u ** 2).sum(0))
                a = np.sqrt(gamma * p / r)
                nh = np.stack([mm[9] * mm[3 * d + k] for k in range(3)])
                nh = nh / np.sqrt((nh ** 2).sum(0))
                if side == 0:
                    nh = -nh
                un = (u * nh).sum(0)
                unb = 0.5 * (un + 2 * a / (gamma - 1) - 2 / (gamma - 1))   # free stream at rest, a = 1
                out.append(np.where(un >= a, 2, np.where(un <= -a, -2, np.where(unb > 0, 1, -1))).ravel())
    return np.concatenate(out)


def test_bounded_fp32_flux_form_close_to_oracle(B):
    """The FP32-flux form on the bounded jet domain with the bench's own state
    (noise on every node, up to the far-field faces, where the ambient fluid
    is at rest and u_n is pure noise), against the FP64 oracle after 1, 20 and
    100 steps, per conserved variable.  The far-field rule takes entropy and
    tangential velocity from the interior or the free stream depending on the
    sign of u_n, a jump of the size of the noise; it decides from the double
    update of its reference node, which the FP32-flux stages keep for the
    reference planes, so that it flips against the oracle only where u_n is
    within the flux error (about 1e-8 relative) of 0.  The errors then stay
    at the level of the same state on a periodic block (below 3 times it, or
    1e-6 above it), the branches agree with the oracle's at the checked
    steps, and the 100-step error meets the form's 1e-5 target.  (Deciding
    from the float stage state instead flipped at a few nodes per step and
    gave 1e-4 in rho v after one step.)"""
    _log("bounded jet domain 40x30x26 FP32-flux vs periodic, 1, 20, 100 steps")
    c = CASES["jetdomain_40x30x26"]
    g, q, bc = I.jet_domain_case(c["dims"], seed=4, bc=c["bc"])
    errs = {}
    for name, bcs in (("bounded", bc), ("periodic", (PER,) * 6)):
        P = oracle.default_params(bc=bcs)
        ref, got = [], []
        qo = q.copy()
        with B.Solver(g.dims, B.params_default(bc=bcs, precision=B.JZ_FP32_FLUX)) as s:
            s.set_grid_metrics(g.metrics)
            s.set_state(q)
            done = 0
            for n in (1, 20, 100):
                qo, _, _, _ = oracle.advance(g.dims, P, g.metrics, qo, n - done)
                s.advance(n - done)
                done = n
                ref.append(qo)
                got.append(s.get_state())
        errs[name] = [per_var_rel(a, b) for a, b in zip(got, ref)]
        if name == "bounded":
            for a, b in zip(got, ref):
                assert np.array_equal(_farfield_branches(a, g.metrics, g.dims, bc),
                                      _farfield_branches(b, g.metrics, g.dims, bc))
    print("[gpu-case] fp32 bounded / periodic errors per variable", errs, flush=True)
    for eb, ep in zip(errs["bounded"], errs["periodic"]):
        for v in range(5):
            assert eb[v] <= 3.0 * ep[v] + 1e-6, (v, eb, ep)
    assert max(errs["bounded"][2]) <= 1e-5


def test_batch_rejects_bounded_members(B):
    _log("batch rejects a bounded member")
    g, q, bc, mi = _case("farfield_5x7x6")
    with B.Solver(g.dims, B.params_default(bc=bc)) as s:
        s.set_grid_metrics(g.metrics)
        s.set_state(q)
        with pytest.raises(B.JzError) as ei:
            B.Batch([s])
        assert ei.value.code == B.JZ_EINVAL


def test_cylinder_centreline_parity(B):
    """Cylindrical jet mesh (jet exit, far field, centreline, periodic
    azimuth) with Thomas-Lombard metrics computed on both sides: metrics
    (none on the axis), three steps per-step parity, axis nodes of one i
    bitwise equal over the azimuth; one step with the exact metric set."""
    _log("cylinder 40x16x24: metrics, three steps, exact-metric step")
    dims = (40, 16, 24)
    g, q, bc = I.jet_cylinder_case(dims, seed=7)
    mo = oracle.metrics_tl(*dims, g.x, g.y, g.z, g.period, bc=bc)
    P = oracle.default_params(bc=bc, re_d=2.0e4)
    ni, nj, nk = dims
    with B.Solver(dims, B.params_default(bc=bc, re_d=2.0e4)) as s:
        s.set_grid_coords(g.x, g.y, g.z, g.period)
        mg = s.get_grid_metrics()
        fin = np.isfinite(mo[9])
        assert np.array_equal(fin, np.isfinite(mg[9]))
        assert not fin.reshape(nk, nj, ni)[:, 0, :].any() and fin.reshape(nk, nj, ni)[:, 1:, :].all()
        scale = np.max(np.abs(mo[:9, fin]))
        assert np.max(np.abs(mg[:9, fin] - mo[:9, fin])) <= 1e-13 * scale
        assert np.max(np.abs(mg[9, fin] - mo[9, fin]) / mo[9, fin]) <= 1e-13
        s.set_state(q)
        qo = q.copy()
        for step in range(3):
            q_prev = qo
            qo, _, rms_o, linf_o = oracle.step(dims, P, mo, qo)
            s.advance(1)
            qg = s.get_state()
            rms, linf = s.residual_norms()
            assert max(per_var_rel(qg, qo)) <= TOL_STATE, step
            assert max(per_var_rel(qg - q_prev, qo - q_prev)) <= TOL_INC, step
            assert np.allclose(rms, rms_o, rtol=1e-9, atol=0) and np.allclose(linf, linf_o, rtol=1e-9, atol=0)
            axis = qg.reshape(5, nk, nj, ni)[:, :, 0, 2:]
            assert np.all(axis == axis[:, :1, :])
            s.set_state(qo)
    qe, _, _, _ = oracle.step(dims, P, g.metrics, q)
    with B.Solver(dims, B.params_default(bc=bc, re_d=2.0e4)) as s:
        s.set_grid_metrics(g.metrics)
        s.set_state(q)
        s.advance(1)
        qg = s.get_state()
    assert max(per_var_rel(qg, qe)) <= TOL_STATE
    assert max(per_var_rel(qg - q, qe - q)) <= TOL_INC


def test_cylinder_axis_many_azimuths(B):
    """Centreline means over more azimuths than one LDS pass holds (264 =
    256 + 8) and an axial length that leaves the last workgroup of stations
    partly empty (18 = 4 * 4 + 2): one step against the oracle, axis nodes of
    one i bitwise equal over the azimuth, in both forms' state types."""
    _log("cylinder 18x8x264: axis mean over two LDS passes")
    dims = (18, 8, 264)
    g, q, bc = I.jet_cylinder_case(dims, seed=9)
    P = oracle.default_params(bc=bc, re_d=2.0e4)
    ni, nj, nk = dims
    qe, _, _, _ = oracle.step(dims, P, g.metrics, q)
    with B.Solver(dims, B.params_default(bc=bc, re_d=2.0e4)) as s:
        s.set_grid_metrics(g.metrics)
        s.set_state(q)
        s.advance(1)
        qg = s.get_state()
    assert max(per_var_rel(qg, qe)) <= TOL_STATE
    assert max(per_var_rel(qg - q, qe - q)) <= TOL_INC
    axis = qg.reshape(5, nk, nj, ni)[:, :, 0, 2:]
    assert np.all(axis == axis[:, :1, :])
    with B.Solver(dims, B.params_default(bc=bc, re_d=2.0e4, precision=B.JZ_FP32_FLUX)) as s:
        s.set_grid_metrics(g.metrics)
        s.set_state(q)
        s.advance(1)
        q32 = s.get_state()
    axis = q32.reshape(5, nk, nj, ni)[:, :, 0, 2:]
    assert np.all(axis == axis[:, :1, :])
    assert max(per_var_rel(q32, qe)) <= 1e-5


def test_cylinder_fp32_flux_form_close_to_oracle(B):
    """FP32-flux form on the cylindrical mesh with the bench's own state (noise
    on every node), per conserved variable, after 1, 20 and 100 steps: within
    the form's 1e-5 target at every checkpoint, and the far-field branches of
    the outflow and lateral faces agree with the oracle's."""
    _log("cylinder 40x16x24 FP32-flux, 1, 20, 100 steps")
    dims = (40, 16, 24)
    g, q, bc = I.jet_cylinder_case(dims, seed=8)
    P = oracle.default_params(bc=bc)
    qo = q.copy()
    errs = []
    with B.Solver(dims, B.params_default(bc=bc, precision=B.JZ_FP32_FLUX)) as s:
        s.set_grid_metrics(g.metrics)
        s.set_state(q)
        done = 0
        for n in (1, 20, 100):
            qo, _, _, _ = oracle.advance(dims, P, g.metrics, qo, n - done)
            s.advance(n - done)
            done = n
            qg = s.get_state()
            errs.append(per_var_rel(qg, qo))
            fin = np.isfinite(g.metrics[9])
            m = np.where(fin, g.metrics, 1.0)
            assert np.array_equal(_farfield_branches(qg, m, dims, bc), _farfield_branches(qo, m, dims, bc))
    print("[gpu-case] fp32 cylinder errors per variable", errs, flush=True)
    assert max(max(e) for e in errs) <= 1e-5


def test_axis_face_rules_are_validated(B):
    _log("axis face validation")
    for bad in ((FF, FF, FF, I.BC_AXIS, PER, PER), (I.BC_AXIS, FF, FF, FF, PER, PER),
                (IN, FF, I.BC_AXIS, FF, FF, FF)):
        with pytest.raises(B.JzError) as ei:
            B.Solver((10, 8, 8), B.params_default(bc=bad))
        assert ei.value.code == B.JZ_EINVAL
