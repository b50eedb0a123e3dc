"""Host-side checks of the per-tile sort's network design (no GPU).

The per-tile sort (S3R_SORT_TILES) orders every tile list by (depth bits,
position) -- the blending order of Eq. (2) with ties in Gaussian order --
with a bitonic network written so that every merge first compares mirror
images and then elements j apart, every comparator keeping the smaller key
at the lower index.  Padding with the largest key then never moves, so any
length sorts.  The kernels run it (a) on LDS arrays, (b) on registers, lane l
of a wave holding positions l E .. l E + E - 1 (steps below E inside a lane,
longer ones between lanes, a mirror step also mirroring the register), with
steps between waves through LDS, and (c) merge sorted 2048-entry chunks by
rank.  These tests run the same index arithmetic in Python on random keys
with many ties and compare with Python's sort."""

import random

import pytest

WAVE = 64


def lower(q, j):
    return ((q & ~(j - 1)) << 1) | (q & (j - 1))


def next_pow2(n):
    m = 1
    while m < n:
        m <<= 1
    return m


def network_flat(keys, skip_padding=False):
    """(a): the network on one array; padded to a power of two with the
    largest key, or (skip_padding) comparators reaching past the end skipped."""
    n = len(keys)
    m = next_pow2(n)
    s = list(keys) + ([] if skip_padding else [float("inf")] * (m - n))
    k = 2
    while k <= m:
        j = k >> 1
        while j > 0:
            for q in range(m >> 1):
                i = lower(q, j)
                p = (i ^ (k - 1)) if j == (k >> 1) else (i + j)
                assert i < p < m
                if skip_padding and p >= n:
                    continue
                if s[p] < s[i]:
                    s[i], s[p] = s[p], s[i]
            j >>= 1
        k <<= 1
    return s[:n]


def wave_step(x, E, K, J):
    """(b): one step (K, J) on x[lane][e]."""
    flip = J == K // 2
    if J < E:
        for lane in range(WAVE):
            for e in range(E):
                f = (e ^ (K - 1)) if flip else (e ^ J)
                if f > e and x[lane][f] < x[lane][e]:
                    x[lane][e], x[lane][f] = x[lane][f], x[lane][e]
    else:
        lmask = (K // E - 1) if flip else (J // E)
        hb = (K // (2 * E)) if flip else (J // E)
        y = [[x[lane ^ lmask][(E - 1 - e) if flip else e] for e in range(E)] for lane in range(WAVE)]
        for lane in range(WAVE):
            low = (lane & hb) == 0
            for e in range(E):
                # lower lane keeps the smaller key, upper the larger (equal
                # keys, the padding, give the same value either way)
                if (y[lane][e] < x[lane][e]) == low:
                    x[lane][e] = y[lane][e]


def wave_merge(x, E, K, J):
    while J > 0:
        wave_step(x, E, K, J)
        J //= 2


def wave_sort(x, E, K):
    if K > 1:
        wave_sort(x, E, K // 2)
        wave_merge(x, E, K, K // 2)


def keys_with_ties(rng, n, distinct):
    # composite keys (depth << 32 | position) with repeated depths
    return [(rng.randrange(distinct) << 32) | i for i in range(n)]


@pytest.mark.parametrize("skip", [False, True])
def test_flat_network_sorts_any_length(skip):
    rng = random.Random(1)
    for n in list(range(0, 70)) + [127, 128, 129, 300, 513, 1000, 2047]:
        keys = keys_with_ties(rng, n, 7)
        rng.shuffle(keys)
        assert network_flat(keys, skip_padding=skip) == sorted(keys), n


@pytest.mark.parametrize("E", [1, 2, 4, 8])
def test_register_wave_network(E):
    rng = random.Random(2 + E)
    for n in (2, 3, 17, 40 * E + 3, WAVE * E - 1, WAVE * E):
        keys = keys_with_ties(rng, n, 11)
        rng.shuffle(keys)
        x = [[keys[lane * E + e] if lane * E + e < n else float("inf") for e in range(E)]
             for lane in range(WAVE)]
        wave_sort(x, E, WAVE * E)
        assert [x[lane][e] for lane in range(WAVE) for e in range(E)][:n] == sorted(keys), (E, n)


def test_four_waves_with_steps_between_waves():
    """Lists of 512..2048 entries: four waves of 512 register keys, merges of
    1024 and 2048 keys taking their steps of 512 and more through LDS."""
    rng = random.Random(3)
    E, WK = 8, WAVE * 8
    for n in (512, 513, 777, 1024, 1025, 1500, 2047, 2048):
        keys = keys_with_ties(rng, n, 13)
        rng.shuffle(keys)
        waves = []
        for w in range(4):
            x = [[keys[w * WK + lane * E + e] if w * WK + lane * E + e < n else float("inf")
                  for e in range(E)] for lane in range(WAVE)]
            wave_sort(x, E, WK)
            waves.append(x)
        k = 2 * WK
        while k <= next_pow2(n):
            j = k >> 1
            while j >= WK:
                flat = [waves[w][lane][e] for w in range(4) for lane in range(WAVE) for e in range(E)]
                for w in range(4):
                    for lane in range(WAVE):
                        for e in range(E):
                            p = w * WK + lane * E + e
                            q = (p ^ (k - 1)) if j == (k >> 1) else (p ^ j)
                            y = flat[q]
                            if (y < waves[w][lane][e]) == (p < q):
                                waves[w][lane][e] = y
                j >>= 1
            for w in range(4):
                wave_merge(waves[w], E, 4 * 2048, WK // 2)
            k <<= 1
        out = [waves[w][lane][e] for w in range(4) for lane in range(WAVE) for e in range(E)][:n]
        assert out == sorted(keys), n


def test_chunk_rank_merge():
    """Lists of 2048..16383 entries: sorted 2048-entry chunks merged by rank
    (place in own chunk + entries below it in every other chunk)."""
    import bisect
    rng = random.Random(4)
    CH = 2048
    for n in (2048, 2049, 4096, 5000, 8444, 16383):
        keys = keys_with_ties(rng, n, 300)
        rng.shuffle(keys)
        s = []
        for c0 in range(0, n, CH):
            s += sorted(keys[c0:c0 + CH])
        out = [None] * n
        nc = (n + CH - 1) // CH
        for q in range(n):
            c = q // CH
            pos = q - c * CH
            for d in range(nc):
                if d != c:
                    lo, hi = d * CH, min(n, d * CH + CH)
                    # fixed-step lower bound, as in the kernel
                    cnt, step = 0, CH
                    while step > 0:
                        t = cnt + step
                        if t <= hi - lo and s[lo + t - 1] < s[q]:
                            cnt = t
                        step >>= 1
                    assert cnt == bisect.bisect_left(s, s[q], lo, hi) - lo
                    pos += cnt
            assert out[pos] is None
            out[pos] = s[q]
        assert out == sorted(keys), n
