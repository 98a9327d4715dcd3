"""Latency ABR controller of the paper's adaptive client, written from its
rules (Section 5.3, "Throughput Monitoring" and "ABR Controller"): test
infrastructure only; the product's controller is the library's tigas_abr_*.

Per completed request i the client measures the payload size S_i and its
download time dt_i, i.e. the throughput S_i / dt_i, and keeps an exponential
moving average over the last `history` samples with factor `alpha`.  The
expected completion time of level l is T_l = S~_l / (r * 1024) with S~_l the
level's expected size in bytes and r the average in KB/s.  An upgrade to
l + 1 needs T_{l+1} <= T_target, a downgrade to l - 1 needs T_l > T_margin
(T_target < T_margin leaves a deadband), and a change is made only when its
condition held on `hold` consecutive requests, except that a downgrade during
rapid panning is made at once.

Readings where the paper is silent: levels are numbered by rising quality
(0 = Table 1's profile 3, 320x180 at quality 10; 3 = profile 0, 1280x720 at
90); S~_l is the middle of Table 1's size range; T_margin = 1.5 T_target; the
average restarts from the oldest sample of the window (the window's first
sample is taken as is, then the newer ones are folded in oldest first).
"""
from __future__ import annotations

# Table 1 size ranges (KB): middles, levels by rising quality
EXPECTED_BYTES = (7 * 1024.0, 20 * 1024.0, 55 * 1024.0, 240 * 1024.0)


class LatencyABR:
    def __init__(self, expected_bytes=EXPECTED_BYTES, t_target=0.100, t_margin=0.150, alpha=0.3, history=5,
                 hold=3, level=0):
        self.expected = list(expected_bytes)
        self.t_target, self.t_margin = t_target, t_margin
        self.alpha, self.history, self.hold = alpha, history, hold
        self.level = level
        self.samples = []
        self.rate_kbps = 0.0
        self.direction = 0  # +1 / -1: the condition seen on the last requests
        self.streak = 0

    def expected_time(self, level):
        return self.expected[level] / (self.rate_kbps * 1024.0)

    def observe(self, nbytes, seconds, rapid_pan=False):
        """One completed request; returns the level of the next one."""
        self.samples.append(nbytes / seconds / 1024.0)
        self.samples = self.samples[-self.history:]
        e = self.samples[0]
        for x in self.samples[1:]:
            e = self.alpha * x + (1.0 - self.alpha) * e
        self.rate_kbps = e
        want = 0
        if self.level + 1 < len(self.expected) and self.expected_time(self.level + 1) <= self.t_target:
            want = 1
        elif self.level > 0 and self.expected_time(self.level) > self.t_margin:
            want = -1
        if want == -1 and rapid_pan:
            self.level -= 1
            self.direction, self.streak = 0, 0
            return self.level
        if want != 0 and want == self.direction:
            self.streak += 1
        else:
            self.direction = want
            self.streak = 1 if want else 0
        if want != 0 and self.streak >= self.hold:
            self.level += want
            self.direction, self.streak = 0, 0
        return self.level
