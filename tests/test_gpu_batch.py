"""Batched form: many uneven blocks advanced by one persistent launch per
stage, the step replayed from a hipGraph.  Every member must come out bitwise
identical to the same block advanced alone (same tile shape), in both
precision forms; a member that fails is frozen without disturbing the rest."""
import numpy as np
import pytest

import oracle
from paper_2003_09926_amd import inputs as I

from _parity import per_var_rel

pytestmark = pytest.mark.gpu

DIMS = [(37, 23, 19), (20, 33, 12), (48, 16, 30), (9, 11, 13), (64, 40, 24), (31, 31, 31)]


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU test without a GPU"
    from paper_2003_09926_amd import binding
    binding.library()
    return binding


def _cases():
    out = []
    for b, d in enumerate(DIMS):
        g = I.uniform_box(*d)
        q = I.jet_state(g, 1.2 + 0.1 * b, seed=100 + b)
        out.append((g, q, dict(mach_j=1.2 + 0.1 * b, re_d=10 ** (5 + 0.2 * b))))
    return out


def _members(B, cases, prec, tile, **extra):
    ms = []
    for g, q, kw in cases:
        s = B.Solver(g.dims, B.params_default(precision=prec, tile_i=tile[0], tile_j=tile[1], **kw, **extra))
        s.set_grid_metrics(g.metrics)
        s.set_state(q)
        ms.append(s)
    return ms


@pytest.mark.parametrize("prec,tile", [(0, (16, 12)), (0, (28, 12)), (0, (12, 12)), (0, (32, 8)), (0, (16, 16)),
                                       (1, (28, 20)), (1, (12, 12)), (1, (32, 16))])
def test_batch_members_bitwise_equal_alone(B, prec, tile):
    print(f"[gpu-case] batch vs alone precision={prec} tile={tile}", flush=True)
    cases = _cases()
    alone = []
    for s in _members(B, cases, prec, tile):
        s.advance(3)
        alone.append((s.get_state(), s.residual_norms(), s.clock()))
        s.close()
    ms = _members(B, cases, prec, tile)
    with B.Batch(ms) as b:
        b.advance(3)
        b.synchronize()
    for s, (q, (rms, linf), clk) in zip(ms, alone):
        assert np.array_equal(s.get_state(), q)
        r2, l2 = s.residual_norms()
        assert np.array_equal(r2, rms) and np.array_equal(l2, linf)
        assert s.clock() == clk
        s.close()


@pytest.mark.parametrize("prec,tile", [(0, (0, 0)), (0, (16, 16)), (1, (0, 0))])
def test_batch_members_match_oracle(B, prec, tile):
    """Every member of a batch (own size, Mach and Re) against the oracle
    advanced alone from the same state: FP64 within the 1e-12 state and 1e-9
    increment bars after three steps, FP32-flux within its 1e-5 target.  The
    default tile shapes (compact 16 x 12 in FP64) and the 16 x 16 shape."""
    print(f"[gpu-case] batch vs oracle precision={prec} tile={tile}", flush=True)
    cases = _cases()
    ms = _members(B, cases, prec, tile)
    with B.Batch(ms) as b:
        b.advance(3)
        b.synchronize()
    for s, (g, q, kw) in zip(ms, cases):
        qo, _, _, _ = oracle.advance(g.dims, oracle.default_params(**kw), g.metrics, q, 3)
        qg = s.get_state()
        if prec == 0:
            assert max(per_var_rel(qg, qo)) <= 1e-12, g.dims
            assert max(per_var_rel(qg - q, qo - q)) <= 1e-9, g.dims
        else:
            assert max(per_var_rel(qg, qo)) <= 1e-5, g.dims
        s.close()


def test_graph_and_direct_launches_agree(B):
    print("[gpu-case] batch graph vs direct", flush=True)
    cases = _cases()
    res = []
    for graph in (True, False):
        ms = _members(B, cases, 0, (28, 12))
        with B.Batch(ms) as b:
            b.set_graph(graph)
            b.advance(2)
            b.advance(1)
            b.synchronize()
        res.append([s.get_state() for s in ms])
        for s in ms:
            s.close()
    for a, c in zip(*res):
        assert np.array_equal(a, c)


def test_autotune_keeps_results(B, tmp_path):
    print("[gpu-case] batch autotune", flush=True)
    cases = _cases()[:4]
    ref = []
    for s in _members(B, cases, 0, (28, 12)):
        s.advance(2)
        ref.append(s.get_state())
        s.close()
    ms = _members(B, cases, 0, (28, 12))
    cache = str(tmp_path / "tune.txt")
    with B.Batch(ms) as b:
        choice, best_ms = b.autotune(trial_steps=1, cache_path=cache)
        assert tuple(choice[:2]) in {(16, 12), (32, 8), (16, 16), (28, 12), (12, 12)} and best_ms > 0
        b.advance(2)
        b.synchronize()
        choice2, _ = b.autotune(trial_steps=1, cache_path=cache)   # from the cache
        assert choice2 == choice
    for s, q in zip(ms, ref):
        assert np.array_equal(s.get_state(), q)
        s.close()
    assert open(cache).read().count("\n") == 1


def _tune_key(prec, ns, dims):
    """The batch signature the autotuner files its choices under."""
    h = 1469598103934665603
    for v in sorted((ni << 40) | (nj << 20) | nk for ni, nj, nk in dims):
        h = ((h ^ v) * 1099511628211) % (1 << 64)
    return f"p{prec}-s{ns}-n{len(dims)}-{h:016x}"


def test_autotune_rejects_unusable_cached_choice(B, tmp_path):
    """A cache line whose tile shape has no stage kernel is refused: the call
    fails, every member keeps its launch shape, and the batch still steps to
    the same states as the members alone."""
    print("[gpu-case] batch autotune, unusable cached choice", flush=True)
    cases = _cases()[:3]
    ref = []
    for s in _members(B, cases, 0, (16, 12)):
        s.advance(2)
        ref.append(s.get_state())
        s.close()
    cache = tmp_path / "tune.txt"
    cache.write_text(f"{_tune_key(0, 5, [g.dims for g, _, _ in cases])} 15 7 32 1.0\n")
    ms = _members(B, cases, 0, (16, 12))
    before = [s.tiling() for s in ms]
    with B.Batch(ms) as b:
        with pytest.raises(B.JzError) as ei:
            b.autotune(trial_steps=1, cache_path=str(cache))
        assert ei.value.code == B.JZ_EINVAL
        assert [s.tiling() for s in ms] == before
        b.advance(2)
        b.synchronize()
    for s, q in zip(ms, ref):
        assert np.array_equal(s.get_state(), q)
        s.close()


def test_failing_member_is_isolated(B):
    """One member with a fixed dt far beyond stability blows up; it is
    flagged and frozen, the others match their solo runs bitwise."""
    print("[gpu-case] batch failing member", flush=True)
    cases = _cases()[:3]
    solo = []
    for s in _members(B, cases, 0, (28, 12)):
        s.advance(4)
        solo.append(s.get_state())
        s.close()
    ms = _members(B, cases[:2], 0, (28, 12))
    g, q, kw = cases[2]
    bad = B.Solver(g.dims, B.params_default(tile_i=28, tile_j=12, dt_fixed=5.0, **kw))
    bad.set_grid_metrics(g.metrics)
    bad.set_state(q)
    with B.Batch(ms + [bad]) as b:
        b.advance(4)
        b.synchronize()
    for s, qs in zip(ms, solo[:2]):
        assert np.array_equal(s.get_state(), qs)
    with pytest.raises(B.JzError) as ei:
        bad.get_state()
    assert ei.value.code == B.JZ_ENONFINITE
    for s in ms + [bad]:
        s.close()


def test_batch_rejects_mixed_members(B):
    cases = _cases()[:2]
    a = _members(B, cases[:1], 0, (28, 12))[0]
    c = _members(B, cases[1:], 1, (28, 12))[0]
    with pytest.raises(B.JzError) as ei:
        B.Batch([a, c])
    assert ei.value.code == B.JZ_EINVAL
    with pytest.raises(B.JzError):
        B.Batch([a, a])
    a.close()
    c.close()


def test_tiny_batch_with_fewer_tiles_than_xcds(B):
    """A batch of two small blocks has fewer tiles than there are XCD slots;
    every tile must still be processed exactly once."""
    print("[gpu-case] tiny batch", flush=True)
    cases = [(I.uniform_box(5, 5, 5), 1.3, 51), (I.uniform_box(9, 11, 13), 1.7, 52)]
    solo, members = [], []
    for g, mach, seed in cases:
        q = I.jet_state(g, mach, seed)
        for store in (solo, members):
            s = B.Solver(g.dims, B.params_default(tile_i=28, tile_j=12, mach_j=mach))
            s.set_grid_metrics(g.metrics)
            s.set_state(q)
            store.append(s)
    for s in solo:
        s.advance(3)
    with B.Batch(members) as b:
        b.advance(3)
        b.synchronize()
    for a, c in zip(solo, members):
        assert np.array_equal(a.get_state(), c.get_state())
        a.close()
        c.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_add_remove_bitwise_equal_alone(B, prec):
    """Continuous batching: members join and leave between steps (the step
    graph is not captured again) and each still comes out bitwise equal to
    the block advanced alone for the same number of steps; the batch may run
    empty; growing past the table slots (16) keeps the results too."""
    print(f"[gpu-case] batch add/remove precision={prec}", flush=True)
    cases = _cases()
    tile = (0, 0)
    alone = []
    # steps each member takes in the batch below
    for (g, q, kw), n in zip(cases, [4, 3, 3, 3, 1, 1]):
        with B.Solver(g.dims, B.params_default(precision=prec, **kw)) as s:
            s.set_grid_metrics(g.metrics)
            s.set_state(q)
            s.advance(n)
            alone.append((s.get_state(), s.clock()))
    ms = _members(B, cases, prec, tile)
    b = B.Batch(ms[:2])
    b.advance(1)                 # members 0, 1
    b.add(ms[2])
    b.add(ms[3])
    b.advance(1)                 # 0, 1, 2, 3
    b.remove(ms[1])
    b.add(ms[4])
    b.advance(1)                 # 0, 2, 3, 4
    b.remove(ms[3])
    b.remove(ms[4])
    b.add(ms[5])
    b.add(ms[1])
    b.advance(1)                 # 0, 2, 5, 1
    b.remove(ms[0])
    b.remove(ms[2])
    b.remove(ms[5])
    b.remove(ms[1])
    assert len(b) == 0
    b.advance(1)                 # empty
    b.add(ms[3])
    b.advance(1)                 # 3
    b.synchronize()
    b.close()
    for s, (q, clk) in zip(ms, alone):
        assert np.array_equal(s.get_state(), q)
        assert s.clock() == clk
        s.close()


def test_batch_grows_past_its_table_slots(B):
    print("[gpu-case] batch growth past 16 members", flush=True)
    small = [(I.uniform_box(9 + (i % 5), 11 + (i % 3), 13 + (i % 4)), 1.2 + 0.03 * i, 200 + i) for i in range(21)]
    solo, members = [], []
    for g, mach, seed in small:
        q = I.jet_state(g, mach, seed)
        for store in (solo, members):
            s = B.Solver(g.dims, B.params_default(mach_j=mach))
            s.set_grid_metrics(g.metrics)
            s.set_state(q)
            store.append(s)
    b = B.Batch(members[:1])
    b.advance(1)
    for s in members[1:]:
        b.add(s)
    b.advance(2)
    b.synchronize()
    b.close()
    solo[0].advance(3)
    for s in solo[1:]:
        s.advance(2)
    for a, c in zip(solo, members):
        assert np.array_equal(a.get_state(), c.get_state())
        a.close()
        c.close()


def test_batch_add_remove_rejections(B):
    cases = _cases()[:3]
    a, c = _members(B, cases[:2], 0, (0, 0))
    f32 = _members(B, cases[2:], 1, (0, 0))[0]
    other_tile = _members(B, cases[2:], 0, (16, 16))[0]
    with B.Batch([a]) as b:
        for bad in (a, f32, other_tile):
            with pytest.raises(B.JzError) as ei:
                b.add(bad)
            assert ei.value.code == B.JZ_EINVAL
        with pytest.raises(B.JzError):
            b.remove(c)           # not a member
        b.add(c)
        assert len(b) == 2
    for s in (a, c, f32, other_tile):
        s.close()
