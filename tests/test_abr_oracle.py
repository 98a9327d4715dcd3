"""Pins of the latency-ABR oracle (CPU): the ladder against the paper's
Table 1, the moving average against hand-computed values, and the decision
rules (thresholds, deadband, hold counter, panning bypass) on traces whose
outcome follows from the rules by hand."""
import math
import os

import pytest

from oracle.abr import EXPECTED_BYTES, LatencyABR


def _table1():
    path = os.path.join(os.path.dirname(__file__), "golden", "ladder_table1_jpeg.txt")
    rows = [list(map(float, l.split())) for l in open(path) if l.strip() and not l.startswith("#")]
    return sorted(rows, key=lambda r: r[3])  # by rising quality


def test_expected_sizes_are_the_middles_of_table1():
    for (_, _, _, _, lo, hi), s in zip(_table1(), EXPECTED_BYTES):
        assert s == (lo + hi) / 2 * 1024


def test_moving_average_over_the_last_five_samples():
    a = LatencyABR()
    for kb in (100, 100, 100, 100):
        a.observe(kb * 1024, 1.0)
    assert a.rate_kbps == pytest.approx(100.0, rel=1e-12)
    a.observe(1000 * 1024, 1.0)  # window 100,100,100,100,1000: 0.3*1000 + 0.7*100
    assert a.rate_kbps == pytest.approx(370.0, rel=1e-12)
    for _ in range(5):
        a.observe(100 * 1024, 1.0)  # the 1000 has left the window
    assert a.rate_kbps == pytest.approx(100.0, rel=1e-12)
    b = LatencyABR()
    for kb in (10, 20, 40):
        b.observe(kb * 1024, 1.0)
    assert b.rate_kbps == pytest.approx(0.3 * 40 + 0.7 * (0.3 * 20 + 0.7 * 10), rel=1e-12)


def test_expected_time_formula():
    a = LatencyABR()
    a.observe(512 * 1024, 2.0)  # 256 KB/s
    assert a.expected_time(3) == pytest.approx(240 * 1024 / (256 * 1024), rel=1e-12)


@pytest.mark.parametrize("rate_kbps", [50, 150, 400, 1000, 5000])
def test_steady_level_is_the_highest_meeting_the_target(rate_kbps):
    a = LatencyABR()
    for _ in range(40):
        a.observe(rate_kbps * 1024 * 0.05, 0.05)
    want = max([0] + [l for l, s in enumerate(EXPECTED_BYTES) if s / (rate_kbps * 1024) <= 0.100])
    # a level may also stay put inside the deadband, but never above the target
    assert a.level == want


def test_hold_counter_three_consecutive_requests():
    a = LatencyABR()
    levels = [a.observe(10_000 * 1024, 1.0) for _ in range(9)]
    assert levels == [0, 0, 1, 1, 1, 2, 2, 2, 3]


def test_deadband_keeps_the_level():
    a = LatencyABR(level=2)
    # T_2 = 55 KB / r in (0.100, 0.150]: neither up (T_3 far above) nor down
    r = 55 / 0.12
    for _ in range(20):
        assert a.observe(r * 1024, 1.0) == 2


def test_downgrade_after_hold_or_at_once_when_panning():
    slow = 100  # KB/s: T_3 = 2.4 s, T_2 = 0.55 s, T_1 = 0.2 s, all above T_margin
    a = LatencyABR(level=3)
    assert [a.observe(slow * 1024, 1.0) for _ in range(3)] == [3, 3, 2]
    b = LatencyABR(level=3)
    assert [b.observe(slow * 1024, 1.0, rapid_pan=True) for _ in range(4)] == [2, 1, 0, 0]


def test_interrupted_streak_restarts():
    # a one-sample window makes the average the last sample: 300 KB/s qualifies
    # for 0 -> 1 (T_1 = 0.067 s) but not for 1 -> 2 (T_2 = 0.18 s); 150 KB/s
    # does not qualify (T_1 = 0.13 s) and breaks the count
    a = LatencyABR(history=1)
    out = [a.observe(x * 1024, 1.0) for x in (300, 300, 150, 300, 300, 300, 300)]
    assert out == [0, 0, 0, 0, 0, 1, 1]
