"""Host-side checks of two arithmetic facts the kernels rely on.

1. The collision step's histogram from the counting atomics: every increment
   of a point's byte score from o to o+1 is one of the #{score >= o+1} points,
   so the number of increments whose old value was t-1 is #{score >= t}.
2. The integer re-rank of byte rows: for integer coordinates in 0..255 and
   d <= 256, every partial sum of (x - q)^2 stays below 2^24, so the FP32 sum
   is exact in any order and equals x.x - 2 x.q + q.q computed in integers
   with 4-byte dot products; past d = 258 an FP32 sum can round.
"""
import numpy as np


def test_histogram_from_old_values_of_increments():
    rng = np.random.default_rng(5)
    for trial in range(200):
        ns = int(rng.integers(1, 17))
        n = int(rng.integers(1, 500))
        # each subspace activates a random subset of points (a point at most once per subspace)
        incs = np.concatenate([rng.choice(n, int(rng.integers(0, n + 1)), replace=False) for _ in range(ns)])
        rng.shuffle(incs)                               # any order of the atomics
        score = np.zeros(n, np.int64)
        crossing = np.zeros(ns + 2, np.int64)
        for pid in incs:
            old = score[pid]
            crossing[old + 1] += 1                      # G[o+1] gains this point
            score[pid] = old + 1
        for t in range(1, ns + 1):
            assert crossing[t] == int((score >= t).sum())


def fp32_sequential(x, q):
    acc = np.float32(0.0)
    for a, b in zip(x.astype(np.float32), q.astype(np.float32)):
        t = np.float32(a - b)
        acc = np.float32(acc + np.float32(t * t))
    return acc


def dot4_form(x, q):
    """x.x - 2 x.q + q.q over 16-byte slices, in unsigned 32-bit (wrapping) arithmetic."""
    x = x.astype(np.int64)
    q = q.astype(np.int64)
    s = 0
    for j in range(0, x.size, 16):
        xs, qs = x[j:j + 16], q[j:j + 16]
        s = (s + int((xs * xs).sum()) - 2 * int((xs * qs).sum()) + int((qs * qs).sum())) % 2 ** 32
    return s


def test_byte_distances_exact_in_fp32_up_to_d256():
    rng = np.random.default_rng(11)
    for d in (16, 32, 128, 240, 256):
        for trial in range(50):
            x = rng.integers(0, 256, d)
            q = rng.integers(0, 256, d)
            exact = int(((x - q) ** 2).sum())
            assert exact < 2 ** 24
            assert int(fp32_sequential(x, q)) == exact
            assert dot4_form(x, q) == exact
        # the largest distance at this d: all 255 against all 0
        x, q = np.full(d, 255), np.zeros(d, np.int64)
        assert int(fp32_sequential(x, q)) == d * 255 * 255 == dot4_form(x, q)


def test_byte_distances_can_round_past_d258():
    # 259 * 255^2 = 16,841,475 > 2^24: the FP32 running sum loses its last bit
    d = 272
    x, q = np.full(d, 255), np.zeros(d, np.int64)
    x[-1] = 254                                         # make the exact sum odd
    exact = int(((x - q) ** 2).sum())
    assert exact > 2 ** 24 and exact % 2 == 1
    assert int(fp32_sequential(x, q)) != exact
