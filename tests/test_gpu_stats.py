"""Time-averaged statistics accumulated on the GPU (Sec. 6: <U>, the RMS of
the axial velocity fluctuation, azimuthal averages over a cross-section),
against NumPy's mean and standard deviation of the oracle's states sampled at
the same steps, and against the closed form of two samples."""
import numpy as np
import pytest

import oracle
from paper_2003_09926_amd import inputs as I
from paper_2003_09926_amd import stats as ST

pytestmark = pytest.mark.gpu
G = 1.4


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU test without a GPU"
    from paper_2003_09926_amd import binding
    binding.library()
    return binding


def _log(msg):
    print(f"[gpu-case] {msg}", flush=True)


def _up(q):
    rho = q[0]
    u = q[1] / rho
    p = (G - 1.0) * (q[4] - 0.5 * (q[1] ** 2 + q[2] ** 2 + q[3] ** 2) / rho)
    return u, p


def test_two_samples_give_the_closed_form(B):
    _log("stats: two explicit samples")
    g, q, bc = I.jet_cylinder_case((20, 10, 16), seed=3)
    q2 = q.copy()
    q2[1] *= 1.1                                     # u -> 1.1 u
    with B.Solver(g.dims, B.params_default(bc=bc, stats_interval=5)) as s:
        s.set_grid_metrics(g.metrics)
        s.set_state(q)
        s.stats_sample()
        s.set_state(q2)
        s.stats_sample()
        st = s.stats()
    ua, pa = _up(q)
    ub, pb = _up(q2)
    assert st["samples"] == 2
    np.testing.assert_allclose(st["mean_u"], 0.5 * (ua + ub), rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(st["mean_p"], 0.5 * (pa + pb), rtol=1e-14)
    # variances against (a - b)^2 / 4, to the rounding of the sums of squares
    np.testing.assert_allclose(st["rms_u"] ** 2, 0.25 * (ua - ub) ** 2, rtol=0,
                               atol=1e-14 * (ua ** 2 + ub ** 2).max())
    np.testing.assert_allclose(st["rms_p"] ** 2, 0.25 * (pa - pb) ** 2, rtol=0,
                               atol=1e-14 * (pa ** 2 + pb ** 2).max())


def test_sampled_run_matches_numpy_statistics_of_the_oracle(B):
    _log("stats: cylinder 24x12x16, interval 2, 8 steps")
    dims = (24, 12, 16)
    g, q, bc = I.jet_cylinder_case(dims, seed=4)
    P = oracle.default_params(bc=bc, re_d=2.0e4)
    samples, qo = [], q.copy()
    for _ in range(4):
        qo, _, _, _ = oracle.advance(dims, P, g.metrics, qo, 2)
        samples.append(_up(qo))
    U = np.stack([s[0] for s in samples])
    Pp = np.stack([s[1] for s in samples])
    with B.Solver(dims, B.params_default(bc=bc, re_d=2.0e4, stats_interval=2)) as s:
        s.set_grid_metrics(g.metrics)
        s.set_state(q)
        s.advance(3)
        s.advance(5)                                  # sampling follows the step count across calls
        st = s.stats()
        bins = ST.radial_bins(g.y, g.z, dims, 12, nbins=6, rmax=1.5)
        prof = s.stats_profile(12, bins, 6)
        s.stats_reset()
        with pytest.raises(B.JzError) as ei:
            s.stats()
        assert ei.value.code == B.JZ_ESTATE
    assert st["samples"] == 4
    np.testing.assert_allclose(st["mean_u"], U.mean(0), rtol=0, atol=1e-12 * np.abs(U).max())
    np.testing.assert_allclose(st["mean_p"], Pp.mean(0), rtol=0, atol=1e-12 * np.abs(Pp).max())
    # variances: the sums carry a cancellation of order eps <x^2>
    np.testing.assert_allclose(st["rms_u"] ** 2, U.var(0), rtol=0, atol=1e-12 * (U ** 2).mean(0).max())
    np.testing.assert_allclose(st["rms_p"] ** 2, Pp.var(0), rtol=0, atol=1e-12 * (Pp ** 2).mean(0).max())
    assert st["rms_u"].max() > 1e-4
    # bin averages of the node statistics over the section i = 12
    ni, nj, nk = dims
    mu = st["mean_u"].reshape(nk, nj, ni)[:, :, 12].reshape(-1)
    for b in range(6):
        sel = bins == b
        assert prof["count"][b] == sel.sum()
        if sel.any():
            assert prof["mean_u"][b] == pytest.approx(mu[sel].mean(), rel=1e-13)


def test_statistics_off_and_batches(B):
    _log("stats: disabled / batch")
    g, q = I.jet_box_case((12, 10, 8), seed=5)
    with B.Solver(g.dims, B.params_default()) as s:
        s.set_grid_metrics(g.metrics)
        s.set_state(q)
        with pytest.raises(B.JzError) as ei:
            s.stats_sample()
        assert ei.value.code == B.JZ_ESTATE
    off = B.workspace_bytes(g.dims, B.params_default())
    on = B.workspace_bytes(g.dims, B.params_default(stats_interval=1))
    assert on - off >= 4 * 8 * g.n
    with B.Solver(g.dims, B.params_default(stats_interval=1)) as s:
        s.set_grid_metrics(g.metrics)
        s.set_state(q)
        with pytest.raises(B.JzError) as ei:
            B.Batch([s])
        assert ei.value.code == B.JZ_EINVAL
