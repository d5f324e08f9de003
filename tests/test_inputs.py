"""Input generators: counter-based noise, subsampling and the workload mixes."""
import numpy as np

from paper_2003_09926_amd import inputs as I


def test_splitmix64_reference_values():
    # published splitmix64 outputs for the state sequence starting at 0
    # (the generator's first outputs with seed 0: x = 0x9E37..., 2*0x9E37..., ...)
    x = np.array([0, 1, 2], dtype=np.uint64) * np.uint64(0x9E3779B97F4A7C15)
    got = I.splitmix64(x)
    assert int(got[0]) == 0xE220A8397B1DCDAF
    assert int(got[1]) == 0x6E789E6AA1B965F4
    assert int(got[2]) == 0x06C45D188009454F


def test_subsample_noise_is_the_subsample_of_the_full_field():
    full = I.stretched_jet_grid(32, 16, 16)
    qf = I.jet_state(full, 1.4, 5)
    _, qs = I.stretched_jet_case((32, 16, 16), seed=5, stride=4)
    sub = qf.reshape(5, 16, 16, 32)[:, ::4, ::4, ::4].reshape(5, -1)
    assert np.array_equal(qs[2], sub[2]) and np.array_equal(qs[3], sub[3])


def test_workload_mixes_are_seeded_and_in_range():
    a = I.batch_mix(seed=4)
    b = I.batch_mix(seed=4)
    assert a == b and len(a) == 64
    assert all(32 <= d <= 160 for blk in a for d in blk["dims"])
    s = I.arrival_stream(seed=5, nruns=50)
    t = [r["arrival"] for r in s]
    assert t == sorted(t) and all(48 <= r["dims"][0] <= 192 for r in s)
