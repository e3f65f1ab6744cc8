"""Host checks of the index bookkeeping the 512-point column kernels rely on
(pure integer arithmetic, no GPU): the 2/3-band rows a thread owns in the
register-staged transforms, their band indices, the slot maps of the three
radix-8 stages and the LDS row swizzle.

n = 512, K = 170 (band rows 0..170 and 342..511, band index row or row - 171).
"""

import itertools

N, K = 512, 170
NB = 2 * K + 1


def in_band(row):
    return row <= K or row >= N - K


def band_index(row):
    return row if row <= K else row - (N - NB)


def swz(row):
    return row ^ ((row >> 3) & 1)


def test_one_column_slots_cover_the_band_once():
    # thread rows r0 + 32 m (r0 = 0..31, m = 0..15); the kernel's claim: m <= 4 and
    # m >= 11 always in the band, m = 5 iff r0 <= 10, m = 10 iff r0 >= 22, never 6..9
    seen = []
    for r0, m in itertools.product(range(32), range(16)):
        row = r0 + 32 * m
        claim = (m <= 4 or m >= 11) or (m == 5 and r0 <= 10) or (m == 10 and r0 >= 22)
        assert claim == in_band(row), (r0, m)
        # band index formula of the kernel, a valid compact row for every slot it loads
        if m <= 5 or m >= 10:
            i = r0 + 32 * m if m <= 5 else r0 + 32 * m - 171
            assert 0 <= i < NB
            if claim:
                assert i == band_index(row)
                seen.append(i)
    assert sorted(seen) == list(range(NB))


def test_paired_slots_cover_the_band_once():
    # lane rows rp + 64 m (rp = 0..63, m = 0..7): m = 0, 1, 6, 7 always, m = 2 iff
    # rp <= 42, m = 5 iff rp >= 22, never 3, 4
    seen = []
    for rp, m in itertools.product(range(64), range(8)):
        row = rp + 64 * m
        claim = m in (0, 1, 6, 7) or (m == 2 and rp <= 42) or (m == 5 and rp >= 22)
        assert claim == in_band(row), (rp, m)
        if claim:
            i = rp + 64 * m if m <= 2 else rp + 64 * m - 171
            assert i == band_index(row)
            seen.append(i)
    assert sorted(seen) == list(range(NB))


def stages(cols_of_thread):
    """(column, index) pairs handled by every thread in the three stages."""
    out = []
    for t in range(512):
        out.extend(cols_of_thread(t))
    return out


def test_slot_maps_cover_every_butterfly_once():
    W = 16
    onecol = stages(lambda t: [(t % W, t // W), (t % W, t // W + 32)])
    paired = stages(lambda t: [(2 * (t % (W // 2)), t // (W // 2)), (2 * (t % (W // 2)) + 1, t // (W // 2))])
    full = sorted(itertools.product(range(W), range(64)))
    assert sorted(onecol) == full
    assert sorted(paired) == full
    # one-column slot s of thread t holds rows t / W + 32 (s + 2 r): the thread's rows
    for t in range(512):
        rows = sorted(t // W + 32 * s + 64 * r for s in range(2) for r in range(8))
        assert rows == [t // W + 32 * m for m in range(16)]


def test_stage_rows_are_a_permutation_and_swizzle_bases_hold():
    # Stockham stages of 512 = 8 * 8 * 8: stage 1 writes rows 8 j + r, stage 2
    # reads j + 64 r and writes d0 + 8 r (d0 = 64 (j >> 3) + (j & 7)), stage 3
    # reads j + 64 r; each is a permutation of the 512 rows over j = 0..63, r = 0..7
    for rows in ([8 * j + r for j in range(64) for r in range(8)],
                 [j + 64 * r for j in range(64) for r in range(8)],
                 [64 * (j >> 3) + (j & 7) + 8 * r for j in range(64) for r in range(8)]):
        assert sorted(rows) == list(range(N))
    assert sorted(swz(r) for r in range(N)) == list(range(N))
    for j, r in itertools.product(range(64), range(8)):
        b = j & 1
        # stage-1 writes from the two parity bases
        want = swz(8 * j + r)
        got = (8 * j + b + r) if r % 2 == 0 else (8 * j + 1 - b + r - 1)
        assert got == want
        # reads: js ^ (bit 3 of js), plus 64 r
        assert swz(j + 64 * r) == (j ^ ((j >> 3) & 1)) + 64 * r
        # stage-2 writes: bit 3 of d0 is clear, so bit 3 of the row is r & 1
        d0 = 64 * (j >> 3) + (j & 7)
        assert (d0 >> 3) & 1 == 0
        assert swz(d0 + 8 * r) == ((d0 ^ 1) if r & 1 else d0) + 8 * r


def test_first_stage_rows_of_a_wave_fill_both_bank_halves():
    # a row of 16 complex FP32 values is 32 banks: rows of one parity share a half.
    # The eight (paired) or four (one-column) rows a wave writes per r in stage 1
    # split evenly over both halves after the swizzle.
    for r in range(8):
        paired = [swz(8 * j + r) % 2 for j in range(8)]
        onecol = [swz(8 * j + r) % 2 for j in range(4)]
        assert sorted(paired) == [0] * 4 + [1] * 4
        assert sorted(onecol) == [0, 0, 1, 1]
