"""The no-allocation entry point jz_advance_static against jz_advance.

jz_advance_static runs the same kernels with the same launch shape as a
solver created for the block, with its buffers in the library's static
device array instead of an allocated workspace, so its states must equal the
solver's bitwise (and a fortiori within the 1e-12 state bar).  Two calls in
a row, the second on a smaller block, show that nothing of the first call's
contents leaks into the second (the clock and flag are cleared per call)."""
import numpy as np
import pytest

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


def _via_solver(B, g, q, nsteps, **kw):
    with B.Solver(g.dims, B.params_default(**kw)) as s:
        s.set_grid_metrics(g.metrics)
        s.set_state(q)
        s.advance(nsteps)
        qs = s.get_state()
        rms, linf = s.residual_norms()
        t, dt, n = s.clock()
    return qs, rms, linf, t, dt, n


def _via_static(B, g, q, nsteps, **kw):
    import torch
    met = torch.from_numpy(np.ascontiguousarray(g.metrics)).cuda()
    qd = torch.from_numpy(np.ascontiguousarray(q)).cuda()
    info = torch.full((14,), -1.0, dtype=torch.float64, device="cuda")
    B.advance_static(g.dims, B.params_default(**kw), met, qd, nsteps, info=info)
    torch.cuda.synchronize()
    return qd.cpu().numpy(), info.cpu().numpy()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_static_entry_matches_solver_on_two_calls(B, prec):
    kw = {} if prec == "fp64" else {"precision": B.JZ_FP32_FLUX}
    for dims, seed, nsteps in (((64, 48, 48), 1, 3), ((37, 23, 19), 2, 2)):
        print(f"[gpu-case] static entry {prec} {dims} {nsteps} steps", flush=True)
        g, q = I.jet_box_case(dims, seed=seed)
        qs, rms, linf, t, dt, n = _via_solver(B, g, q, nsteps, **kw)
        qz, info = _via_static(B, g, q, nsteps, **kw)
        assert max(per_var_rel(qz, qs)) <= 1e-12
        assert np.array_equal(qz, qs)
        assert info[13] == 0.0 and info[12] == nsteps
        assert info[0] == t and info[1] == dt
        assert np.array_equal(info[2:7], rms) and np.array_equal(info[7:12], linf)


def test_static_entry_bounded_domain(B):
    print("[gpu-case] static entry bounded jet domain 40x30x26", flush=True)
    g, q, bc = I.jet_domain_case((40, 30, 26), seed=3)
    qs, _, _, t, _, _ = _via_solver(B, g, q, 2, bc=bc)
    qz, info = _via_static(B, g, q, 2, bc=bc)
    assert np.array_equal(qz, qs) and info[0] == t and info[13] == 0.0


def test_static_entry_rejects_oversize_and_statistics(B):
    import torch
    g, q = I.jet_box_case((8, 8, 8), seed=1)
    met = torch.zeros((10, 8 * 8 * 8), dtype=torch.float64, device="cuda")
    qd = torch.zeros((5, 8 * 8 * 8), dtype=torch.float64, device="cuda")
    with pytest.raises(B.JzError) as ei:
        B.advance_static(g.dims, B.params_default(stats_interval=1), met, qd, 1)
    assert ei.value.code == B.JZ_EINVAL
    big = (128, 128, 128)                          # 2.1 M nodes: beyond the scratch array
    assert B.workspace_bytes(big) > 64 << 20
    metb = torch.zeros((1,), dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        B.advance_static(big, B.params_default(), metb, qd, 1)
    lib = B.library()
    import ctypes
    P = B.params_default()
    rc = lib.jz_advance_static(128, 128, 128, ctypes.byref(P), met.data_ptr(), qd.data_ptr(), None, 1, None)
    assert rc == B.JZ_EINVAL and b"scratch" in lib.jz_last_error()
