"""The library's latency ABR controller against the ABR oracle (CPU; host
logic, no GPU): the same levels and the same throughput average, step by
step, on seeded random traces and configurations, through the C ABI."""
import numpy as np
import pytest

from oracle.abr import LatencyABR
from paper_2605_08699_amd import tigas


@pytest.mark.parametrize("seed", range(12))
def test_levels_and_average_equal_the_oracle(seed):
    rng = np.random.default_rng(seed)
    kw = dict(history=int(rng.integers(1, 8)), hold=int(rng.integers(1, 5)), alpha=float(rng.uniform(0.1, 1.0)),
              level=int(rng.integers(0, 4)))
    lib_abr = tigas.ABR(**kw)
    ref = LatencyABR(**kw)
    # throughput: a log-normal random walk around 20..2000 KB/s, payloads of
    # the level's expected size with spread, panning now and then
    log_rate = rng.uniform(np.log(20), np.log(2000))
    for i in range(400):
        log_rate = float(np.clip(log_rate + rng.normal(0, 0.3), np.log(5), np.log(20000)))
        nbytes = float(ref.expected[ref.level] * rng.uniform(0.6, 1.4))
        secs = nbytes / (np.exp(log_rate) * 1024.0)
        pan = bool(rng.random() < 0.1)
        a = lib_abr.observe(nbytes, secs, pan)
        b = ref.observe(nbytes, secs, pan)
        assert a == b, f"step {i}"
        assert lib_abr.rate_kbps == ref.rate_kbps, f"step {i}"
    lib_abr.close()


def test_invalid_configuration_and_observations():
    with pytest.raises(tigas.TigasError):
        tigas.ABR(t_target=0.2, t_margin=0.1)
    with pytest.raises(tigas.TigasError):
        tigas.ABR(expected_bytes=[10, 5])
    a = tigas.ABR()
    with pytest.raises(tigas.TigasError):
        a.observe(1000, 0.0)
    assert a.observe(1000, 0.01) == 0
