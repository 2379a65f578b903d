"""Index maps of the HIP kernels, checked exhaustively on the CPU (no GPU).

Each map below is written out from the kernel's formulas (csrc/step_kernels.hip,
csrc/gmres_coop.hip, csrc/ifmm.hip) and checked for what the kernel relies on:
every element is visited exactly once and every index stays inside its buffer.
"""
import numpy as np
import pytest

# ------------------------------------------------------------------ near field
NEAR_LMAX = 512


def near_visits(lens, NU, NC):
    """(pair, lag) visits of k_near_jds1 for one row whose pairs have strip
    lengths `lens` (sorted longest first), with the lane layout 16 pairs x 4
    lags, chunks of 64 NC pairs and rounds of NU steps of 4 lags."""
    np_ = len(lens)
    CH, NG = 64 * NC, 4 * NC
    seen = []
    for c0 in range(0, np_, CH):
        cnt = min(CH, np_ - c0)
        lmax = lens[c0]
        for lane in range(64):
            sub, pg = lane & 3, lane >> 2
            for g in range(NG):
                q = 16 * g + pg
                ln = lens[c0 + q] if q < cnt else 0
                for lb in range(0, lmax, 4 * NU):
                    for t in range(NU):
                        l = lb + 4 * t + sub
                        if l < ln:
                            seen.append((c0 + q, l))
    return seen


@pytest.mark.parametrize("NU,NC", [(2, 1), (1, 1), (1, 2), (2, 2), (3, 1)])
@pytest.mark.parametrize("seed", range(4))
def test_near_round_visits_each_coefficient_once(NU, NC, seed):
    rng = np.random.default_rng(seed)
    np_ = int(rng.integers(1, 300))
    lens = sorted(rng.integers(1, 20, size=np_).tolist(), reverse=True)
    seen = near_visits(lens, NU, NC)
    want = [(p, l) for p in range(np_) for l in range(lens[p])]
    assert sorted(seen) == sorted(want)
    assert len(set(seen)) == len(seen)
    assert max(l for _, l in seen) < min(max(lens), NEAR_LMAX)


def test_near_jds_offsets_address_the_pair_and_lag():
    """v[off[l] + p] with off the exclusive prefix sum of nl[l] (pairs with a
    strip longer than l): distinct, inside the row's block, lag-major."""
    rng = np.random.default_rng(7)
    lens = np.sort(rng.integers(1, 15, size=111))[::-1]
    L = int(lens.max())
    nl = np.array([(lens > l).sum() for l in range(L)])
    off = np.concatenate([[0], np.cumsum(nl)[:-1]])
    addr = [off[l] + p for p in range(len(lens)) for l in range(lens[p])]
    assert len(set(addr)) == len(addr) == lens.sum()
    assert min(addr) == 0 and max(addr) == lens.sum() - 1


def near_leaf_visits(lens, NU, NC):
    """(pair, lag, coefficient address) visits of k_near_leaf for one row:
    lanes 16 pairs x 4 lags with the pairs fastest (pg = lane & 15, sub =
    lane >> 4), chunks of 64 NC pairs, rounds of NU steps of 4 lags."""
    np_ = len(lens)
    CH, NG = 64 * NC, 4 * NC
    L = max(lens)
    nl = [sum(1 for x in lens if x > l) for l in range(L)]
    off = np.concatenate([[0], np.cumsum(nl)[:-1]]).astype(int)
    seen, quarters = [], {}
    for c0 in range(0, np_, CH):
        cnt = min(CH, np_ - c0)
        lmax = lens[c0]
        for lane in range(64):
            pg, sub = lane & 15, lane >> 4
            for g in range(NG):
                q = 16 * g + pg
                ln = lens[c0 + q] if q < cnt else 0
                for lb in range(0, lmax, 4 * NU):
                    for t in range(NU):
                        l = lb + 4 * t + sub
                        if l < ln:
                            a = off[l] + c0 + 16 * g + pg
                            seen.append((c0 + q, l, a))
                            quarters.setdefault((c0, g, lb, t, sub), []).append((pg, a))
    return seen, quarters, off


@pytest.mark.parametrize("NU,NC", [(2, 2), (1, 2)])
@pytest.mark.parametrize("seed", range(4))
def test_near_leaf_rounds_visit_each_coefficient_once_in_whole_lines(NU, NC, seed):
    """Every (pair, lag) once, at its jagged-diagonal address; the lanes of one
    quarter-wave read consecutive values (consecutive pairs at one lag)."""
    rng = np.random.default_rng(100 + seed)
    np_ = int(rng.integers(1, 400))
    lens = sorted(rng.integers(1, 24, size=np_).tolist(), reverse=True)
    seen, quarters, off = near_leaf_visits(lens, NU, NC)
    want = [(p, l) for p in range(np_) for l in range(lens[p])]
    assert sorted((p, l) for p, l, _ in seen) == sorted(want)
    assert all(a == off[l] + p for p, l, a in seen)
    for lanes in quarters.values():
        lanes.sort()
        pgs = [pg for pg, _ in lanes]
        addr = [a for _, a in lanes]
        assert pgs == list(range(pgs[0], pgs[0] + len(pgs)))        # the active lanes are a prefix run
        assert addr == list(range(addr[0], addr[0] + len(addr)))    # consecutive values


def leaf_window(pairs):
    """The compressed window of a leaf as the set-up builds it: per source the
    lags its strips reach, laid end to end; per pair its window word."""
    srcs = sorted({j for j, _, _ in pairs})
    lo = {j: min(g0 for jj, g0, n in pairs if jj == j) for j in srcs}
    hi = {j: max(g0 + n - 1 for jj, g0, n in pairs if jj == j) for j in srcs}
    woff, w = {}, 0
    for j in srcs:
        woff[j] = w
        w += hi[j] - lo[j] + 1
    words = [(woff[j] + g0 - lo[j]) | (n << 16) for j, g0, n in pairs]
    recs = [(j, lo[j], woff[j], hi[j] - lo[j] + 1) for j in srcs]
    return words, recs, w


@pytest.mark.parametrize("seed", range(6))
def test_near_leaf_window_words_address_the_staged_current(seed):
    """W[o_s + w] holds J at lag a_s + w of source s (staging); the pair word
    (offset | length << 16) plus lag l addresses source j's lag g0 + l, inside
    j's part of the window; every window slot is staged once."""
    rng = np.random.default_rng(200 + seed)
    nsrc = int(rng.integers(1, 60))
    pairs = []
    for _ in range(int(rng.integers(1, 300))):
        j = int(rng.integers(0, nsrc))
        pairs.append((j, int(rng.integers(2, 40)), int(rng.integers(1, 12))))
    words, recs, w = leaf_window(pairs)
    staged = {}
    for j, a, o, n in recs:
        for k in range(n):
            assert o + k not in staged
            staged[o + k] = (j, a + k)
    assert sorted(staged) == list(range(w))
    for (j, g0, n), word in zip(pairs, words):
        assert word >> 16 == n and (word & 0xFFFF) + n <= w < 65536
        for l in range(n):
            assert staged[(word & 0xFFFF) + l] == (j, g0 + l)


@pytest.mark.parametrize("nrest,chunks,WPB", [(0, [(0, 0, 64), (1, 64, 100)], 16), (37, [(0, 0, 5)], 16),
                                               (16, [], 16), (5, [(2, 7, 71), (0, 0, 7)], 8)])
def test_near_leaf_blocks_cover_every_row_once(nrest, chunks, WPB):
    """The first ceil(nrest / WPB) blocks take the listed rows, a wavefront
    each; every other block one chunk, its wavefronts rows ra + wv, + WPB, ..."""
    rest = list(range(1000, 1000 + nrest))
    nrb = -(-nrest // WPB)
    rows = []
    for b in range(nrb + len(chunks)):
        for wv in range(WPB):
            if b < nrb:
                idx = b * WPB + wv
                if idx < nrest:
                    rows.append(rest[idx])
                continue
            _, ra, rb = chunks[b - nrb]
            rows.extend(range(ra + wv, rb, WPB))
    want = rest + [r for _, ra, rb in chunks for r in range(ra, rb)]
    assert sorted(rows) == sorted(want) and len(set(rows)) == len(rows)


# ------------------------------------------------------------------ batched near field, matrix cores
def test_leaf_mm_staging_covers_each_chunk_element_once():
    """KC = 32 columns of A (64 rows) and 32 window rows (64 rhs) per chunk,
    256 threads, 8 consecutive values each."""
    a, b = [], []
    for tid in range(256):
        ar, ac = tid >> 2, 8 * (tid & 3)
        bk, bc = tid >> 3, 8 * (tid & 7)
        a += [(ar, ac + e) for e in range(8)]
        b += [(bk, bc + e) for e in range(8)]
    assert sorted(a) == [(r, c) for r in range(64) for c in range(32)]
    assert sorted(b) == [(k, c) for k in range(32) for c in range(64)]


@pytest.mark.parametrize("kpad", [4, 2048, 2052, 9000])
def test_leaf_mm_segments_partition_the_columns(kpad):
    """Column segments of at most 2048 per leaf: a partition of [0, kpad), and
    the chunks of 32 inside a segment stop at its end."""
    seg = [(k, min(kpad, k + 2048)) for k in range(0, kpad, 2048)]
    cols = [c for kb, ke in seg for k0 in range(kb, ke, 32) for c in range(k0, min(k0 + 32, ke))]
    assert cols == list(range(kpad))


# ------------------------------------------------------------------ GMRES
GM_THREADS, GM_RU, GM_RC = 1024, 12, 4


@pytest.mark.parametrize("ne,nb", [(30720, 80), (480, 64), (480, 3), (7, 5), (384 * 9 + 1, 10)])
def test_gmres_lds_rows_cover_each_row_once(ne, nb):
    rows = []
    for bx in range(nb):
        r0, r1 = ne * bx // nb, ne * (bx + 1) // nb
        if r1 - r0 > 32 * GM_RU:
            rows.extend(range(r0, r1))                   # general path, row loop
            continue
        nu = (r1 - r0 + 31) // 32
        assert nu <= GM_RU
        assert -(-nu // GM_RC) * GM_RC <= GM_RU            # chunks of GM_RC slots stay in the table
        for t in range(GM_THREADS):
            hl, hw = t & 31, t >> 5
            for u in range(nu):
                i = r0 + hw + 32 * u
                if hl == 0 and i < r1:
                    rows.append(i)
    assert sorted(rows) == list(range(ne))


@pytest.mark.parametrize("rows,cols", [(30720, 64), (480, 5), (33, 1), (1, 65), (65, 33)])
def test_transpose_tiles_cover_each_element_once(rows, cols):
    tiles_r = (rows + 31) // 32
    ntiles = tiles_r * ((cols + 31) // 32)
    hit = np.zeros((rows, cols), int)
    for b in range(ntiles):
        r0, c0 = (b % tiles_r) * 32, (b // tiles_r) * 32
        rr = r0 + np.arange(32)[:, None] + 0 * np.arange(32)[None, :]
        cc = c0 + np.arange(32)[None, :] + 0 * np.arange(32)[:, None]
        ok = (rr < rows) & (cc < cols)
        np.add.at(hit, (rr[ok], cc[ok]), 1)
    assert (hit == 1).all()


# ------------------------------------------------------------------ M2L
NN, M2L_NT, KTAB, KTAB_MID = 256, 64, 2401, 1197


def test_m2l_row_pair_staging_covers_the_tile_once():
    hit = np.zeros((NN, M2L_NT), int)
    for tid in range(512):
        xr, xg = tid & (NN // 2 - 1), tid >> 7
        for i in range(M2L_NT // 4):
            col = xg + 4 * i
            hit[2 * xr, col] += 1
            hit[2 * xr + 1, col] += 1
    assert (hit == 1).all()


def test_m2l_row_quad_staging_of_the_fp32_form_covers_the_tile_once():
    """FP32 form: thread (row quad xq, first column xh) stages rows 4 xq..4 xq + 3
    of columns xh + 8 i with one 16-byte load and store each; the column stride
    of 260 floats keeps the stores 16-byte aligned."""
    XS = NN + 4
    hit = np.zeros((NN, M2L_NT), int)
    for tid in range(512):
        xq, xh = tid & 63, tid >> 6
        for i in range(M2L_NT // 8):
            col = xh + 8 * i
            assert ((col * XS + 4 * xq) * 4) % 16 == 0
            hit[4 * xq:4 * xq + 4, col] += 1
    assert (hit == 1).all()


def test_m2l_table_reads_are_in_range_and_index_the_lattice_difference():
    """A operand of row (a, m) at k-step (b, n): base + KTAB_MID - 7 (49 b1 +
    7 b2 + b3) must be the table entry of a - b per axis and m - n."""
    lane = np.arange(64)
    n = lane >> 4
    for wr in range(4):
        for rb in range(4):
            row = 64 * wr + 16 * rb + (lane & 15)
            a, m = row >> 2, row & 3
            a1, a2, a3 = a >> 4, (a >> 2) & 3, a & 3
            base = ((((a1 + 3) * 7 + a2 + 3) * 7 + a3 + 3) * 7 + m - n + 3) - KTAB_MID
            for ks in range(64):
                b1, b2, b3 = ks >> 4, (ks >> 2) & 3, ks & 3
                idx = base + KTAB_MID - 7 * ((b1 * 7 + b2) * 7 + b3)
                assert idx.min() >= 0 and idx.max() < KTAB
                want = (((a1 - b1 + 3) * 7 + (a2 - b2 + 3)) * 7 + (a3 - b3 + 3)) * 7 + (m - n + 3)
                assert (idx == want).all()
    # the table build decodes the same index
    e = np.arange(KTAB)
    w, d = e % 7 - 3, e // 7
    assert ((((d // 49) * 7 + (d // 7) % 7) * 7 + d % 7) * 7 + w + 3 == e).all()
