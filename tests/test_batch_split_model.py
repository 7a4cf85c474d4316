"""The batch kernels' work split, modelled on the CPU: a list of messages
with costs (blocks x (Nr + 2)) is cut into S = rounds x W equal shares of
cost units; a share's ends become block indices of each message it touches,
rounded up to the split step and clamped to the message.  Whatever the
lengths, steps, waves and rounds, every block of every message must fall in
exactly one share, and the item search must find the message holding a
share's start.  (The GPU tests check the kernels' outputs; this checks the
rule they implement, including cases too large or too odd to run there.)"""
import numpy as np


def ceil_div(a, b):
    return -(-a // b)


def split_point(x, start, unit, step, nblk):
    if x <= start:
        return 0
    b = ceil_div(x - start, unit)
    b = ceil_div(b, step) * step
    return min(b, nblk)


def find_item(starts, n, x):
    """The kernels' 64-way search: the last item whose start is <= x."""
    lo, hi = 0, n
    while hi - lo > 1:
        span = hi - lo
        p = [lo + (lane * span >> 6) for lane in range(64)]
        passed = [starts[q] <= x for q in p]
        last = max(lane for lane in range(64) if passed[lane])
        assert all(passed[:last + 1])               # the starts never decrease
        lo, hi = p[last], (hi if last == 63 else p[last + 1])
    return lo


def test_shares_partition_every_message():
    rng = np.random.default_rng(7)
    for trial in range(60):
        n = int(rng.integers(1, 120))
        waves = int(rng.choice([1, 3, 16, 64, 256]))
        share = int(rng.choice([50, 1000, 65536]))
        nblk = [int(b) for b in np.where(rng.random(n) < 0.2, 0, rng.integers(0, 3000, n))]
        unit = [int(u) for u in rng.choice([12, 14, 16], n)]
        xts = rng.random(n) < 0.3
        step = [int(rng.choice([1, 2, 16, 256])) if xts[m] else int(rng.choice([1, 128, 512, 777])) for m in range(n)]
        starts = [0]
        for b, u in zip(nblk, unit):
            starts.append(starts[-1] + b * u)
        total = starts[-1]
        if total == 0:
            continue
        rounds = max(1, ceil_div(total, waves * share))
        S = rounds * waves
        cover = [np.zeros(b, np.int32) for b in nblk]
        for s in range(S):
            lo, hi = s * total // S, (s + 1) * total // S
            if lo >= hi:
                continue
            i = find_item(starts, n, lo)
            assert starts[i] <= lo and (i == n - 1 or starts[i + 1] > lo)
            while i < n and starts[i] < hi:
                first = split_point(lo, starts[i], unit[i], step[i], nblk[i])
                end = split_point(hi, starts[i], unit[i], step[i], nblk[i])
                if first < end:
                    assert first % step[i] == 0 and (end % step[i] == 0 or end == nblk[i])
                    cover[i][first:end] += 1
                i += 1
        for m in range(n):
            assert (cover[m] == 1).all(), (trial, m)
