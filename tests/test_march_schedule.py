"""The row schedule of the row-marching K-step kernel (stepm_kernel), checked
on the CPU for every supported (K, B) and a spread of sizes and chunk
lengths.  The kernel's index formulas are restated here: group j (1..K)
of B wavefronts computes marching row v = a_j + B i + r at iteration i
(r = 0..B-1), a_1 = y0 - (K - 1), a_j = a_1 - (j - 1)(B + 1); the row is
active when v lies in [y0 - (K - j), y1 + (K - j)) and the cavity row it
stands for (v, or y0 + y1 - 1 - v on odd chunks, which march down) lies in
[0, n); group j < K writes its rows to ring slot (v - a_K) mod (B + 2),
group j + 1 reads rows v - 1, v, v + 1 from it; T = (y1 - 1 - a_K) // B + 1
iterations; each iteration reads (before a barrier) and then writes.

Checked: every ring read finds the row it needs (written in an earlier
iteration, not yet overwritten), every cavity row is stored exactly once
by group K, slots are in range."""
import pytest

PAIRS = [(2, 8), (3, 2), (3, 4), (4, 1), (4, 2), (4, 3), (4, 4), (6, 2)]

def run_schedule(n, K, B, chunk):
    RS = B + 2
    stored = {}
    for c in range((n + chunk - 1) // chunk):
        y0, y1 = c * chunk, min(c * chunk + chunk, n)
        down = c % 2 == 1
        a1 = y0 - (K - 1)
        aK = a1 - (K - 1) * (B + 1)
        T = (y1 - 1 - aK) // B + 1
        ring = [[None] * RS for _ in range(K - 1)]
        for i in range(T):
            writes = []
            for j in range(1, K + 1):
                aj = a1 - (j - 1) * (B + 1)
                for r in range(B):
                    v = aj + B * i + r
                    y = y0 + y1 - 1 - v if down else v
                    assert v >= aK
                    s0 = (v - aK) % RS
                    assert 0 <= s0 < RS
                    if not (y0 - (K - j) <= v < y1 + (K - j) and 0 <= y < n):
                        continue
                    if j >= 2:
                        for dv in (-1, 0, 1):
                            yy = y0 + y1 - 1 - (v + dv) if down else v + dv
                            if 0 <= yy < n:          # rows outside are wall links
                                assert ring[j - 2][(s0 + dv) % RS] == v + dv, (n, K, B, chunk, c, i, j, v, dv)
                    if j < K:
                        writes.append((j - 1, s0, v))
                    else:
                        stored[y] = stored.get(y, 0) + 1
            for g, s, v in writes:
                ring[g][s] = v
    assert sorted(stored) == list(range(n)) and all(k == 1 for k in stored.values())

@pytest.mark.parametrize("K,B", PAIRS)
def test_every_read_finds_its_row_and_every_row_is_stored_once(K, B):
    for n in list(range(1, 40)) + [63, 64, 65, 130, 257, 1024]:
        for chunk in sorted({1, 2, 3, 5, 7, 13, 37, n, max(1, n // 3)}):
            run_schedule(n, K, B, chunk)

def test_a_shorter_ring_or_lag_fails():
    """The check has teeth: a ring of B + 1 rows, or groups only B rows
    apart, breaks it."""

    def broken(n, K, B, chunk, ring_extra, lag):
        RS = B + ring_extra
        for c in range((n + chunk - 1) // chunk):
            y0, y1 = c * chunk, min(c * chunk + chunk, n)
            a1 = y0 - (K - 1)
            aK = a1 - (K - 1) * lag
            T = (y1 - 1 - aK) // B + 1
            ring = [[None] * RS for _ in range(K - 1)]
            for i in range(T):
                writes = []
                for j in range(1, K + 1):
                    aj = a1 - (j - 1) * lag
                    for r in range(B):
                        v = aj + B * i + r
                        s0 = (v - aK) % RS
                        if not (y0 - (K - j) <= v < y1 + (K - j) and 0 <= v < n):
                            continue
                        if j >= 2:
                            for dv in (-1, 0, 1):
                                if 0 <= v + dv < n and ring[j - 2][(s0 + dv) % RS] != v + dv:
                                    return True
                        if j < K:
                            writes.append((j - 1, s0, v))
                for g, s, v in writes:
                    ring[g][s] = v
        return False

    assert not broken(100, 4, 3, 37, 2, 4)     # the kernel's choice passes
    assert broken(100, 4, 3, 37, 1, 4)         # ring one row short
    assert broken(100, 4, 3, 37, 2, 3)         # groups one row too close
