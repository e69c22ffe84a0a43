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


# The launch's tiles (stepm_body): the bands without a side wall first,
# chunk rows each, chunk row by chunk row, then the one or two bands that
# hold the side walls, chunk_w rows each, left and right in turn.
def tile_rows(n, K, chunk, chunk_w):
    W = 64 - 2 * (K - 1)
    nb = (n + W - 1) // W
    nw = min(nb, 2)
    nch = (n + chunk - 1) // chunk
    tiles = (nb - nw) * nch + nw * ((n + chunk_w - 1) // chunk_w)
    ni = (nb - 2) * nch if nb > 2 else 0
    out = []
    for tile in range(tiles):
        if tile < ni:
            tyt = tile // (nb - 2)
            txt = 1 + (tile - tyt * (nb - 2))
            ch = chunk
        else:
            t = tile - ni
            tyt = t if nb == 1 else t >> 1
            txt = 0 if nb == 1 else (nb - 1 if t & 1 else 0)
            ch = chunk_w
        out.append((txt, tyt * ch, min(tyt * ch + ch, n)))
    return nb, out


# The automatic chunks (march_chunk_auto): the shortest chunk that keeps
# every workgroup resident, and for the side-wall bands the chunk whose
# sweep, at 1.08 times the cost per row, takes about as long, lengthened
# until the launch fits the slots again.
def auto_chunks(n, K, B, slots, wall_cost=1.08):
    W = 64 - 2 * (K - 1)
    nb = (n + W - 1) // W
    chunks = max(1, slots // nb)
    chunk = max(1, (n + chunks - 1) // chunks)
    cw = chunk
    if nb >= 3:
        L = 2 * (K - 1) + (K - 1) * (B + 1)
        cw = max(1, min(chunk, int((chunk + L) / wall_cost - L + 0.5)))
        ni = (nb - 2) * ((n + chunk - 1) // chunk)
        while cw < chunk and ni + 2 * ((n + cw - 1) // cw) > slots:
            cw += 1
    return chunk, cw


@pytest.mark.parametrize("K", [2, 3, 4, 6])
def test_tiles_cover_every_band_and_row_once(K):
    for n in [4, 5, 7, 16, 54, 55, 60, 108, 109, 257, 1024, 2048]:
        for chunk in sorted({1, 3, 7, 37, 40, n}):
            for cw in sorted({1, 5, 35, chunk}):
                if cw > chunk or chunk > n:
                    continue
                nb, rows = tile_rows(n, K, chunk, cw)
                seen = {}
                for txt, y0, y1 in rows:
                    assert 0 <= txt < nb and 0 <= y0 < y1 <= n
                    for y in range(y0, y1):
                        seen[(txt, y)] = seen.get((txt, y), 0) + 1
                assert len(seen) == nb * n and set(seen.values()) == {1}, (n, K, chunk, cw)


def test_wall_band_chunks_keep_every_workgroup_resident():
    assert auto_chunks(1024, 6, 2, 512) == (40, 35)     # 17 x 26 + 2 x 30 = 502 workgroups
    for K, B in PAIRS:
        for n in [64, 100, 257, 512, 1024, 1536, 2048, 4096]:
            for slots in [256, 512, 768]:
                chunk, cw = auto_chunks(n, K, B, slots)
                assert 1 <= cw <= chunk
                nb, rows = tile_rows(n, K, chunk, cw)
                base = len(tile_rows(n, K, chunk, chunk)[1])
                assert len(rows) <= max(slots, base), (n, K, B, slots)
