"""Served form: continuous batching of arriving jet runs.  Every result must
be bitwise the run computed alone and within the oracle's bars (FP64 1e-12,
FP32-flux 1e-5 relative L2 per variable), the HBM budget must hold, and runs
must actually overlap on the device."""
import numpy as np
import pytest

import oracle
from paper_2003_09926_amd import inputs as I

from _parity import per_var_rel

pytestmark = pytest.mark.gpu


def _stream(n=10, steps=12):
    rng = np.random.default_rng(31)
    t = np.cumsum(rng.exponential(0.004, size=n))
    return [dict(arrival=float(t[r]), dims=tuple(int(v) for v in rng.integers(12, 33, size=3)),
                 mach=float(rng.uniform(1.2, 2.0)), re_d=float(10 ** rng.uniform(5, 6)),
                 steps=steps + 3 * (r % 3), seed=900 + r) for r in range(n)]


@pytest.mark.parametrize("mode", ["streams", "batch"])
@pytest.mark.parametrize("prec", [0, 1])
def test_served_results_equal_alone_and_budget_holds(prec, mode):
    import torch
    assert torch.cuda.is_available()
    from paper_2003_09926_amd import binding as B, serve as S
    print(f"[gpu-case] serve precision={prec} mode={mode}", flush=True)
    tile = (28, 12)
    runs = S.make_runs(_stream())
    big = max(S.footprint(r, prec, tile) for r in runs)
    budget = 3 * big
    srv = S.JetServer(precision=prec, budget_bytes=budget, max_resident=4, chunk_steps=5, tile=tile,
                      keep_results=True, mode=mode)
    st = srv.serve(runs)
    assert st.failed == 0 and st.runs == len(runs)
    assert st.max_resident > 1, "runs never overlapped"
    assert st.max_resident_bytes <= budget
    assert st.chunks > len(runs) // 4
    for r in runs:
        assert r.latency > 0 and r.admitted >= r.arrival
        _, alone = S.run_alone(S.Run(r.rid, r.arrival, r.dims, r.mach, r.re_d, r.steps, r.seed), prec, tile,
                               keep_result=True)
        assert np.array_equal(alone, r.result), r.rid
        # and the oracle, advanced alone from the same jet box
        g, q = I.jet_box_case(r.dims, mach=r.mach, seed=r.seed)
        qo, _, _, _ = oracle.advance(r.dims, oracle.default_params(mach_j=r.mach, re_d=r.re_d), g.metrics, q,
                                     r.steps)
        assert max(per_var_rel(r.result, qo)) <= (1e-12 if prec == 0 else 1e-5), r.rid
    s = st.summary()
    assert s["p99_latency_s"] >= s["p50_latency_s"] > 0


def test_oversized_run_is_rejected():
    from paper_2003_09926_amd import serve as S
    runs = S.make_runs(_stream(n=2))
    srv = S.JetServer(budget_bytes=1 << 10, max_resident=2)
    st = srv.serve(runs)
    assert st.failed == 2 and st.runs == 0
