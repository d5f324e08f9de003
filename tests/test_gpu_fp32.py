"""FP32-flux precision form against the FP64 oracle.

The form computes fluxes, dissipation and subgrid viscosity in float from
float stencil reads and float metrics; J, the update Q(k) = Q(0) - a dt R,
the norms and dt stay double.  Bounds (measured margins in the design notes):
  * residual R(Q):                 relative L2 per variable <= 3e-5;
  * one step (128 x 64 x 64):      state <= 2e-6, increment <= 3e-5;
  * 100 steps (128 x 64 x 64):     state <= 1e-5 (the stated target).
"""
import numpy as np
import pytest

import oracle
from paper_2003_09926_amd import inputs as I

from _parity import per_var_rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU test without a GPU"
    from paper_2003_09926_amd import binding
    binding.library()
    return binding


def _solver(B, g, q, **kw):
    s = B.Solver(g.dims, B.params_default(precision=B.JZ_FP32_FLUX, **kw))
    s.set_grid_metrics(g.metrics)
    s.set_state(q)
    return s


@pytest.mark.parametrize("case", ["jetbox_37x23x19", "stretched_32x16x16"])
def test_fp32_residual_close_to_oracle(B, case):
    print(f"[gpu-case] fp32 residual {case}", flush=True)
    if case.startswith("jetbox"):
        g, q = I.jet_box_case((37, 23, 19), seed=2)
    else:
        g, q = I.stretched_jet_case((128, 64, 64), seed=2, stride=4)
    with _solver(B, g, q) as s:
        r = s.eval_residual()
    ro = oracle.residual(g.dims, oracle.default_params(), g.metrics, q)
    assert max(per_var_rel(r, ro)) <= 3e-5


def test_fp32_error_after_1_and_100_steps(B):
    print("[gpu-case] fp32 128x64x64 subsample, 1 and 100 steps", flush=True)
    g, q = I.stretched_jet_case((512, 256, 256), seed=2, stride=4)
    P = oracle.default_params(re_d=1.0e6)
    q1, _, _, _ = oracle.step(g.dims, P, g.metrics, q)
    with _solver(B, g, q, re_d=1.0e6) as s:
        s.advance(1)
        g1 = s.get_state()
        s.advance(99)
        g100 = s.get_state()
    assert max(per_var_rel(g1, q1)) <= 2e-6
    assert max(per_var_rel(g1 - q, q1 - q)) <= 3e-5
    q100, _, _, _ = oracle.advance(g.dims, P, g.metrics, q, 100)
    err = per_var_rel(g100, q100)
    print(f"[gpu-case] fp32 100-step relative L2 per variable {err}", flush=True)
    assert max(err) <= 1e-5


def test_fp32_single_stage_against_oracle(B):
    """n_stages = 1 in the FP32-flux form: double in, double out, written to a
    stage buffer and copied into the state (the one-step bars)."""
    print("[gpu-case] fp32 single stage 37x23x19", flush=True)
    g, q = I.jet_box_case((37, 23, 19), seed=4)
    P = oracle.default_params(n_stages=1, rk_alpha=[1.0], cfl=0.1)
    qo = q.copy()
    with _solver(B, g, q, n_stages=1, rk_alpha=[1.0], cfl=0.1) as s:
        for step in range(3):
            q_prev = qo
            qo, _, _, _ = oracle.step(g.dims, P, g.metrics, qo)
            s.advance(1)
            qg = s.get_state()
            assert max(per_var_rel(qg, qo)) <= 2e-6, step
            assert max(per_var_rel(qg - q_prev, qo - q_prev)) <= 3e-5, step
            s.set_state(qo)


def test_fp32_tl_metrics_and_reproducibility(B):
    print("[gpu-case] fp32 metrics from coordinates, bitwise repeat", flush=True)
    g = I.wavy_grid(16, 12, 10)
    mo = oracle.metrics_tl(*g.dims, g.x, g.y, g.z, g.period)
    q = I.jet_state(g, 1.4, 4, r0=0.6, theta=0.1)
    outs = []
    for _ in range(2):
        with B.Solver(g.dims, B.params_default(precision=B.JZ_FP32_FLUX)) as s:
            s.set_grid_coords(g.x, g.y, g.z, g.period)
            mg = s.get_grid_metrics()
            s.set_state(q)
            s.advance(3)
            outs.append(s.get_state())
    assert np.array_equal(outs[0], outs[1])
    assert np.max(np.abs(mg[:9] - mo[:9])) <= 1e-7 * np.max(np.abs(mo[:9]))
    assert np.array_equal(mg[9], mo[9]) or np.max(np.abs(mg[9] - mo[9]) / mo[9]) <= 1e-13


@pytest.mark.parametrize("prec", [0, 1])
def test_result_independent_of_launch_shape(B, prec):
    """Each node's arithmetic does not depend on the tiling, so every launch
    shape gives a bitwise identical state (norms may differ in the last bit
    through the partial-sum order)."""
    print(f"[gpu-case] launch-shape independence precision={prec}", flush=True)
    g, q = I.jet_box_case((37, 23, 19), seed=11)
    shapes = [(28, 12, 0), (12, 12, 5)] + ([(28, 20, 3), (32, 16, 0), (32, 16, 4)] if prec == 1 else
                                           [(60, 4, 3), (12, 28, 1), (32, 8, 0), (16, 16, 3)])
    ref = None
    for ti, tj, kc in shapes:
        s = B.Solver(g.dims, B.params_default(precision=prec, tile_i=ti, tile_j=tj, kchunk=kc))
        s.set_grid_metrics(g.metrics)
        s.set_state(q)
        s.advance(2)
        out = s.get_state()
        s.close()
        if ref is None:
            ref = out
        else:
            assert np.array_equal(out, ref), (ti, tj, kc)
