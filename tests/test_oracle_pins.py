"""Pins of the CPU oracle against what the paper and mathematics fix.

Every check here is independent of the oracle's own code: exhaustive
identities, the real-valued Le Gall 5/3 filters, textbook Huffman cost,
brute-force searches, hand-derived golden bitstreams and an independent
Python reader of the format.
"""
import glob
import heapq
import itertools
import os

import numpy as np
import pytest

import oracle
from paper_2005_08713_amd import synth
from tests import format_reader as fr
from tests import lift_literal as lit

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- colour transform
def test_rct_exhaustive_rgb8_roundtrip():
    # Sec. 3 (optional colour transform), reversible component transform reading.
    assert oracle.rct_selftest_u8() == 0


def test_rct_gray_and_hand_values():
    for v in (0, 1, 127, 255, 4095, 65535):
        assert oracle.rct_forward(v, v, v) == (v, 0, 0)
    with open(os.path.join(GOLDEN, "rct_examples.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            r, g, b, y, cb, cr = map(int, line.split())
            assert oracle.rct_forward(r, g, b) == (y, cb, cr)
            assert oracle.rct_inverse(y, cb, cr) == (r, g, b)


def test_rct_random_16bit_roundtrip():
    rng = np.random.default_rng(5)
    for r, g, b in rng.integers(0, 65536, size=(2000, 3)):
        assert oracle.rct_inverse(*oracle.rct_forward(r, g, b)) == (r, g, b)


def test_ycocg_exhaustive_rgb8_roundtrip_and_real_transform():
    """YCoCg-R (the alternative reversible colour transform): exact round trip
    over all RGB8 triples; against the real YCoCg matrix, Co is exactly R - B,
    Y lies in (R + 2G + B)/4 - 3/4 .. (R + 2G + B)/4 and Cg in
    G - (R + B)/2 .. G - (R + B)/2 + 1/2 (the two floors of the lifting
    steps); a gray pixel maps to (v, 0, 0)."""
    assert oracle.ycocg_selftest_u8() == 0
    rng = np.random.default_rng(6)
    for r, g, b in rng.integers(0, 1 << 24, size=(3000, 3)):
        y, co, cg = oracle.ycocg_forward(r, g, b)
        assert co == r - b
        exact_y = (int(r) + 2 * int(g) + int(b)) / 4
        assert exact_y - 0.75 <= y <= exact_y
        exact_cg = int(g) - (int(r) + int(b)) / 2
        assert exact_cg <= cg <= exact_cg + 0.5
        assert oracle.ycocg_inverse(y, co, cg) == (r, g, b)
    for v in (0, 1, 255, 65535, (1 << 24) - 1):
        assert oracle.ycocg_forward(v, v, v) == (v, 0, 0)


# ---------------------------------------------------------------- 5/3 lifting
LEGALL_LO = np.array([-1, 2, 6, 2, -1]) / 8.0
LEGALL_HI = np.array([-1, 2, -1]) / 2.0


def _legall_real(x):
    """Real-valued 5/3 Le Gall analysis on the whole-sample symmetric extension."""
    n = len(x)
    xe = np.pad(np.asarray(x, dtype=np.float64), 2, mode="reflect")
    lo = np.array([np.dot(LEGALL_LO, xe[2 * k:2 * k + 5]) for k in range((n + 1) // 2)])
    hi = np.array([np.dot(LEGALL_HI, xe[2 * k + 2:2 * k + 5]) for k in range(n // 2)])
    return lo, hi


@pytest.mark.parametrize("n", list(range(2, 65)))
def test_lifting_matches_legall_filters_within_rounding(n):
    rng = np.random.default_rng(n)
    for trial in range(20):
        lim = [2, 256, 1 << 17][trial % 3]
        x = rng.integers(-lim, lim, size=n)
        lo, hi = oracle.lift_forward_1d(x)
        rlo, rhi = _legall_real(x)
        # predict rounding: floor of a half-integer -> |err| <= 1/2;
        # update adds floor((d1+d2+2)/4) of rounded d's -> |err| <= 1
        assert np.all(np.abs(hi - rhi) <= 0.5 + 1e-9)
        assert np.all(np.abs(lo - rlo) <= 1.0 + 1e-9)
        assert np.array_equal(oracle.lift_inverse_1d(lo, hi, n), x)


def test_lifting_special_cases():
    assert oracle.lift_forward_1d([7])[0].tolist() == [7]
    assert oracle.lift_inverse_1d([7], [], 1).tolist() == [7]
    for n in range(2, 40):
        lo, hi = oracle.lift_forward_1d([9] * n)
        assert (hi == 0).all() and (lo == 9).all()
        ramp = np.arange(n) * 3 + 1
        lo, hi = oracle.lift_forward_1d(ramp)
        assert (hi[:max(0, (n - 1) // 2)] == 0).all()  # linear signals predicted exactly


def test_lifting_golden():
    with open(os.path.join(GOLDEN, "lift53_examples.txt")) as f:
        lines = [l for l in f if l.strip() and not l.startswith("#")]
    for i in range(0, len(lines), 3):
        x = list(map(int, lines[i].split()[1:]))
        s = list(map(int, lines[i + 1].split()[1:]))
        d = list(map(int, lines[i + 2].split()[1:]))
        lo, hi = oracle.lift_forward_1d(x)
        assert lo.tolist() == s and hi.tolist() == d


# ---------------------------------------------------------------- 2-D pyramid
def _legall_2d_real(a):
    rows = [_legall_real(r) for r in a]
    lo = np.array([r[0] for r in rows])
    hi = np.array([r[1] for r in rows]) if a.shape[1] > 1 else np.zeros((a.shape[0], 0))
    def cols(m):
        if m.shape[1] == 0:
            return np.zeros(((m.shape[0] + 1) // 2, 0)), np.zeros((m.shape[0] // 2, 0))
        c = [_legall_real(m[:, j]) for j in range(m.shape[1])]
        return np.array([x[0] for x in c]).T, np.array([x[1] for x in c]).T.reshape(m.shape[0] // 2, -1)
    ll, lh = cols(lo)
    hl, hh = cols(hi)
    return ll, hl, lh, hh


@pytest.mark.parametrize("w,h", [(8, 8), (9, 7), (16, 5), (33, 30), (2, 3)])
def test_one_level_2d_rows_then_columns_near_real_filters(w, h):
    rng = np.random.default_rng(w * 100 + h)
    img = rng.integers(0, 256, size=(h, w)).astype(np.uint8)
    c = oracle.forward_dump(img, 1, bits=8, ct=0)[0]
    ll, hl, lh, hh = _legall_2d_real(img.astype(np.float64))
    # rounding of the row pass propagates through the column filters
    # (L1 gain 1.5 low / 2 high) plus the column pass's own rounding.
    assert np.abs(c["LL"] - ll).max() <= 1.5 * 1 + 1 + 1e-9
    assert np.abs(c["HL"][1] - hl).max() <= 1.5 * 0.5 + 1 + 1e-9
    assert np.abs(c["LH"][1] - lh).max() <= 2 * 1 + 0.5 + 1e-9
    assert np.abs(c["HH"][1] - hh).max() <= 2 * 0.5 + 0.5 + 1e-9


def _read_dwt2_golden():
    cases, cur = [], None
    with open(os.path.join(GOLDEN, "dwt2_one_level.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            key, rest = line.split(None, 1)
            if key == "case":
                cur = {"img": [], "bands": {}}
                cases.append(cur)
            elif key == "row":
                cur["img"].append([int(v) for v in rest.split()])
            else:
                cur["bands"][key] = [[int(v) for v in r.split()] for r in rest.split("|")]
    return cases


def test_one_level_2d_golden_rows_then_columns():
    """Hand-worked bands of one level on images where the column-first order
    differs: pins the row-then-column order of the oracle exactly."""
    for case in _read_dwt2_golden():
        img = np.array(case["img"], dtype=np.uint8)
        got = oracle.forward_dump(img, 1, bits=8, ct=0)[0]
        for nm, rows in case["bands"].items():
            band = got[nm] if nm == "LL" else got[nm][1]
            assert band.tolist() == rows, nm
        assert lit.forward_2d_level(case["img"]) == case["bands"]
        assert lit.forward_2d_level(case["img"], rows_first=False) != case["bands"]


def _band_eq(band, rows):
    """An oracle band (2-D array) equals a literal band (list of rows);
    empty bands of either shape compare equal."""
    if band.size == 0:
        return sum(len(r) for r in rows) == 0
    return band.tolist() == rows


def test_literal_lifting_checker_equals_oracle_1d():
    """The literal checker (explicit symmetric extension, predict at every odd
    position of the extended range) equals the oracle's band-array lifting
    with ==, for every length 1..64 on random and extreme integers."""
    rng = np.random.default_rng(41)
    for n in range(1, 65):
        for lim in (2, 256, 1 << 20):
            for _ in range(4):
                x = rng.integers(-lim, lim, size=n)
                lo, hi = oracle.lift_forward_1d(x)
                llo, lhi = lit.forward_1d(x.tolist())
                assert lo.tolist() == llo and hi.tolist() == lhi, (n, x.tolist())
                assert oracle.lift_inverse_1d(lo, hi, n).tolist() == lit.inverse_1d(llo, lhi)


@pytest.mark.parametrize("w,h", [(1, 1), (1, 6), (5, 1), (2, 2), (3, 3), (2, 5), (7, 4),
                                 (8, 8), (9, 7), (16, 5), (13, 17), (33, 30)])
def test_one_level_2d_equals_literal_rows_then_columns(w, h):
    """One 2-D level of the oracle equals the literal checker composed rows
    first, then columns, with ==; the column-first composition differs on
    every size with both sides at least 2 (so this test tells the orders
    apart), and the literal inverse restores the image."""
    rng = np.random.default_rng(w * 131 + h)
    differs = 0
    for trial in range(6):
        img = rng.integers(0, 256, size=(h, w)).astype(np.uint8)
        got = oracle.forward_dump(img, 1, bits=8, ct=0)[0]
        ref = lit.forward_2d_level(img.tolist())
        assert got["LL"].tolist() == ref["LL"]
        for nm in ("HL", "LH", "HH"):
            assert _band_eq(got[nm][1], ref[nm]), nm
        differs += lit.forward_2d_level(img.tolist(), rows_first=False) != ref
        assert lit.inverse_2d_level(ref, w, h) == img.tolist()
    if w >= 2 and h >= 2:
        assert differs > 0


@pytest.mark.parametrize("w,h,levels", [(37, 29, 4), (64, 64, 3), (19, 50, 6), (5, 3, 5)])
def test_pyramid_equals_literal_recursion(w, h, levels):
    """Every band of an L-level oracle pyramid equals the literal checker's
    recursion on LL (Sec. 3: the decomposition is recursive)."""
    rng = np.random.default_rng(w + h + levels)
    img = rng.integers(0, 4096, size=(h, w)).astype(np.uint16)
    got = oracle.forward_dump(img, levels, bits=12, ct=0)[0]
    ref = lit.forward_pyramid(img.tolist(), levels)
    assert got["LL"].tolist() == ref["LL"]
    for lv in range(1, levels + 1):
        for nm in ("HL", "LH", "HH"):
            assert _band_eq(got[nm][lv], ref[nm][lv]), (nm, lv)


def test_pyramid_is_recursive_and_constant_image_has_zero_highpass():
    img = np.full((77, 50, 3), 200, dtype=np.uint8)
    c5 = oracle.forward_dump(img, 5)
    for ch in c5:
        for l in range(1, 6):
            for nm in ("HL", "LH", "HH"):
                assert not ch[nm][l].any()
    rng = np.random.default_rng(3)
    img = rng.integers(0, 256, size=(45, 61, 1)).astype(np.uint8)
    full = oracle.forward_dump(img, 4, ct=0)[0]
    for z in range(1, 4):
        part = oracle.forward_dump(img, z, ct=0)[0]
        for l in range(1, z + 1):
            for nm in ("HL", "LH", "HH"):
                assert np.array_equal(part[nm][l], full[nm][l])
        # LL_z of a z-level transform, transformed further, gives the L-level bands
        llz = part["LL"].astype(np.uint8) if part["LL"].min() >= 0 and part["LL"].max() < 256 else None
        if llz is not None:
            more = oracle.forward_dump(llz[:, :, None], 4 - z, ct=0)[0]
            assert np.array_equal(more["LL"], full["LL"])


# ---------------------------------------------------------------- area order (Eq. 1)
@pytest.mark.parametrize("wb", list(range(4, 132, 4)))
def test_area_order_is_bijection_and_snake(wb):
    for hb in (4, 8, 12, 64, 128):
        d = 3
        n = wb * hb // 8
        seen = set()
        prev = None
        for k in range(n * d):
            i, j, b = oracle.area_coord(k, wb, hb, d)
            assert 0 <= i < hb and i % 2 == 0 and 0 <= j < wb and j % 4 == 0 and 0 <= b < d
            seen.add((i, j, b))
            # plane-major from the sign plane down (Sec. 4)
            assert b == d - 1 - k // n
            # consecutive k alternate upper/lower area of one 4x4 cell (Eq. 1: k % 2)
            if k % 2 == 1:
                assert (i, j) == (prev[0] + 2, prev[1])
            prev = (i, j, b)
        assert len(seen) == n * d


# ---------------------------------------------------------------- Huffman
def _heap_huffman_cost(freq):
    h = [f for f in freq if f > 0]
    if len(h) <= 1:
        return 0
    heapq.heapify(h)
    cost = 0
    while len(h) > 1:
        a, b = heapq.heappop(h), heapq.heappop(h)
        cost += a + b
        heapq.heappush(h, a + b)
    return cost


def test_huffman_cost_is_optimal_and_kraft_complete():
    rng = np.random.default_rng(11)
    for trial in range(300):
        m = int(rng.integers(1, 257))
        f = np.zeros(256, dtype=np.uint64)
        idx = rng.choice(256, size=m, replace=False)
        f[idx] = rng.integers(1, [2, 10, 1000, 10 ** 6][trial % 4], size=m)
        ln = oracle.huffman_lengths(f)
        assert int((f * ln.astype(np.uint64)).sum()) == _heap_huffman_cost(f.tolist())
        if m >= 2:
            assert sum(2.0 ** -int(l) for l in ln[f > 0]) == 1.0
            assert (ln[f > 0] > 0).all() and (ln[f == 0] == 0).all()


def test_canonical_codes_prefix_free_and_ordered():
    rng = np.random.default_rng(12)
    for _ in range(50):
        f = rng.integers(0, 50, size=256).astype(np.uint64)
        ln = oracle.huffman_lengths(f)
        code = oracle.canonical_codes(ln)
        words = sorted((int(ln[s]), s) for s in range(256) if ln[s])
        strs = [format(int(code[s]), "0%db" % l) for l, s in words]
        for a, b in itertools.combinations(strs, 2):
            assert not b.startswith(a) and not a.startswith(b)
        # canonical: numeric order of the left-aligned codes follows (length, symbol)
        vals = [int(s.ljust(40, "0"), 2) for s in strs]
        assert vals == sorted(vals)


def _best_limited_cost(freq, limit):
    """Exhaustive optimum over length vectors with Kraft sum <= 1, lengths <= limit."""
    fs = [f for f in freq if f > 0]
    best = None
    for lens in itertools.product(range(1, limit + 1), repeat=len(fs)):
        if sum(2.0 ** -l for l in lens) <= 1.0 + 1e-12:
            c = sum(f * l for f, l in zip(fs, lens))
            best = c if best is None or c < best else best
    return best


def test_package_merge_is_optimal_length_limited():
    rng = np.random.default_rng(13)
    for trial in range(60):
        m = int(rng.integers(2, 6))
        limit = int(rng.integers(max(2, (m - 1).bit_length()), 5))
        f = np.zeros(256, dtype=np.uint64)
        idx = rng.choice(256, size=m, replace=False)
        f[idx] = rng.integers(1, 200, size=m)
        ln = oracle.huffman_lengths(f, limit=limit)
        assert ln.max() <= limit
        assert int((f * ln.astype(np.uint64)).sum()) == _best_limited_cost(f.tolist(), limit)
        assert sum(2.0 ** -int(l) for l in ln[f > 0]) == 1.0
    # Fibonacci weights: unlimited depth 20+, limited to 14 must still be optimal-ish and valid
    f = np.zeros(256, dtype=np.uint64)
    a, b = 1, 1
    for s in range(25):
        f[s] = a
        a, b = b, a + b
    assert oracle.huffman_lengths(f).max() > 14
    ln = oracle.huffman_lengths(f, limit=14)
    assert ln.max() == 14 and sum(2.0 ** -int(l) for l in ln[f > 0]) == 1.0


# ---------------------------------------------------------------- golden bitstreams
def _golden_tiles():
    return sorted(glob.glob(os.path.join(GOLDEN, "tile_*.txt")))


@pytest.mark.parametrize("path", _golden_tiles(), ids=os.path.basename)
def test_golden_bitstream(path):
    img = None
    blocks = {}
    with open(path) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            key, val = line.split(":", 1)
            if key == "image":
                parts = val.split()
                w, h, c, bits = map(int, parts[:4])
                kw = dict(p.split("=") for p in parts[4:])
                img = np.zeros((h, w, c), dtype=np.uint8 if bits <= 8 else np.uint16)
            elif key == "pixel":
                r, col, ch, v = map(int, val.split())
                img[r, col, ch] = v
            elif key.startswith("block"):
                bitstr = "".join(val.split())
                bitstr += "0" * (-len(bitstr) % 8)
                blocks[int(key.split()[1])] = bytes(int(bitstr[i:i + 8], 2)
                                                    for i in range(0, len(bitstr), 8))
    blob = oracle.encode_tile(img, int(kw["levels"]), bits=bits, ct=int(kw["ct"]),
                              qstep=int(kw["qstep"]))
    hdr, got = fr.parse_tile(blob)
    assert hdr["width"] == w and hdr["height"] == h and hdr["nblocks"] == len(blocks)
    for i, exp in blocks.items():
        assert got[i][1] == exp, f"block {i}: {got[i][1].hex()} != {exp.hex()}"
    assert np.array_equal(oracle.decode_tile(blob), img)


# ---------------------------------------------------------------- independent reader
CASES = [
    (1, 1, 1, 8, 0, 1, "uniform"), (5, 3, 1, 8, 2, 1, "uniform"), (37, 23, 3, 8, 3, 1, "uniform"),
    (64, 64, 1, 12, 2, 1, "uniform"), (130, 257, 3, 8, 5, 1, "ramp"), (33, 17, 1, 16, 6, 1, "uniform"),
    (50, 50, 3, 8, 3, 4, "uniform"), (40, 9, 3, 8, 4, 3, "checker"), (16, 16, 1, 1, 2, 1, "sparse"),
    (129, 3, 1, 10, 3, 1, "max"), (200, 150, 3, 8, 4, 1, "sparse"), (1, 40, 3, 8, 6, 2, "uniform"),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "x".join(map(str, c)))
def test_independent_reader_recovers_oracle_coefficients(case):
    w, h, c, bits, lv, q, kind = case
    img = synth.random_image(w, h, c, bits, seed=w * 7 + h, kind=kind)
    ct = 1 if c == 3 else 0
    blob = oracle.encode_tile(img, lv, bits=bits, ct=ct, qstep=q)
    hdr, coefs = fr.tile_coefficients(blob)
    ref = oracle.forward_dump(img, lv, bits=bits, ct=ct, qstep=q)
    for ch in range(c):
        assert np.array_equal(coefs[ch]["LL"], ref[ch]["LL"])
        for l in range(1, lv + 1):
            for nm in ("HL", "LH", "HH"):
                assert np.array_equal(coefs[ch][(nm, l)], ref[ch][nm][l])


def _runs(seq):
    out, k = [], 0
    while k < len(seq):
        if seq[k]:
            k += 1
            continue
        e = k
        while e < len(seq) and seq[e] == 0:
            e += 1
        out.append(e - k)
        k = e
    return out


def test_block_statistics_brute_force():
    """C_zr (least frequent, smallest on ties), the run histogram F_i, masks
    and Eq. 3's choice, recomputed in Python from independently scattered
    symbols."""
    rng = np.random.default_rng(21)
    for trial in range(40):
        p = [1, 3][trial % 2]
        wb, hb = [(4, 4), (8, 12), (32, 16), (128, 128), (64, 8)][trial % 5]
        scale = [1, 3, 40, 2000][trial % 4]
        t = rng.integers(-scale, scale + 1, size=(p, hb, wb))
        t[rng.random(t.shape) < 0.6] = 0
        blob, info = oracle.encode_block(t)
        dinfo = {}
        q = fr.decode_block(blob, p, wb, hb, dinfo)
        assert np.array_equal(q, t)
        d = 1 + int(np.abs(t).max()).bit_length()
        assert info.d == d == dinfo["d"]
        # symbols per plane / type, cell by cell
        segs = []
        for b in range(d - 1, -1, -1):
            seg = []
            for tt in range(p):
                bits_ = (t[tt] < 0).astype(int) if b == d - 1 else (np.abs(t[tt]) >> b) & 1
                syms = []
                for band in range(hb // 4):
                    for cg in range(wb // 4):
                        for half in range(2):
                            blk = bits_[4 * band + 2 * half:4 * band + 2 * half + 2, 4 * cg:4 * cg + 4]
                            syms.append(int(sum(int(blk[r, c]) << (c + 4 * r) for r in range(2) for c in range(4))))
                present = any(syms)
                assert ((info.masks[tt] >> b) & 1) == (0 if present else 1)
                if present:
                    seg += syms
            if seg:
                segs.append(seg)
        if not segs:
            continue
        hist = np.bincount(np.concatenate(segs), minlength=256)
        assert info.czr == int(np.argmin(hist))  # argmin returns the smallest index on ties
        runs = [L for s in segs for L in _runs(s) if L >= 2]
        F = np.zeros(40, dtype=np.int64)
        for L in runs:
            F[L.bit_length()] += 1
        assert list(info.run_hist) == F.tolist()
        # Eq. 3 (as read) minimised over [2, max(2, ceil(log2 p n))]
        beta = max(2, (p * wb * hb // 8 - 1).bit_length())
        costs = [sum(int(F[i]) * -(-i // w) * (w + info.l_provisional) for i in range(40))
                 for w in range(2, beta + 1)]
        assert info.wz == 2 + int(np.argmin(costs))
        assert info.wz == dinfo["wz"] and info.czr == dinfo["czr"]


# ---------------------------------------------------------------- round trip / levels
@pytest.mark.parametrize("case", CASES, ids=lambda c: "x".join(map(str, c)))
def test_lossless_roundtrip_and_level_decode(case):
    w, h, c, bits, lv, q, kind = case
    img = synth.random_image(w, h, c, bits, seed=w + 3 * h, kind=kind)
    ct = 1 if c == 3 else 0
    blob = oracle.encode_tile(img, lv, bits=bits, ct=ct, qstep=1)
    assert np.array_equal(oracle.decode_tile(blob, 0), img)
    top = (1 << bits) - 1
    for z in range(1, lv + 1):
        # decode at level z = clamp(inverse colour transform(LL_z)) (Sec. 4)
        llz = oracle.forward_dump(img, z, bits=bits, ct=ct)
        planes = np.stack([d["LL"] for d in llz], axis=-1).astype(np.int64)
        if ct:
            y, cb, cr = planes[..., 0], planes[..., 1], planes[..., 2]
            g = y - np.floor_divide(cb + cr, 4)
            planes = np.stack([cr + g, g, cb + g], axis=-1)
        exp = np.clip(planes, 0, top).astype(img.dtype)
        assert np.array_equal(oracle.decode_tile(blob, z), exp)


def _inv_colour(planes, ct):
    """Inverse colour transform written from each transform's definition."""
    if ct == 1:
        y, cb, cr = planes[..., 0], planes[..., 1], planes[..., 2]
        g = y - np.floor_divide(cb + cr, 4)
        return np.stack([cr + g, g, cb + g], axis=-1)
    if ct == 2:
        y, co, cg = planes[..., 0], planes[..., 1], planes[..., 2]
        t = y - np.floor_divide(cg, 2)
        g = cg + t
        b = t - np.floor_divide(co, 2)
        return np.stack([b + co, g, b], axis=-1)
    return planes


GENERAL = [
    # (w, h, c, bits, levels, qstep, ct, kind): alternative colour transform,
    # 9-bit RGB (27-bit pixels), 4-byte samples up to 24 bits, many channels
    (150, 97, 3, 8, 4, 1, 2, "uniform"), (64, 40, 3, 9, 3, 1, 2, "ramp"), (120, 88, 3, 9, 3, 1, 1, "uniform"),
    (77, 50, 3, 12, 3, 3, 2, "uniform"), (60, 45, 1, 24, 3, 1, 0, "uniform"), (70, 33, 3, 20, 4, 1, 1, "ramp"),
    (40, 40, 3, 24, 2, 5, 2, "uniform"), (50, 30, 16, 8, 3, 1, 0, "uniform"), (20, 12, 64, 10, 2, 1, 0, "ramp"),
]


@pytest.mark.parametrize("case", GENERAL, ids=lambda c: "x".join(map(str, c)))
def test_generality_roundtrip_levels_and_reader(case):
    w, h, c, bits, lv, q, ct, kind = case
    img = synth.random_image(w, h, c, bits, seed=w * 5 + h, kind=kind)
    blob = oracle.encode_tile(img, lv, bits=bits, ct=ct, qstep=q)
    hdr, coefs = fr.tile_coefficients(blob)
    assert (hdr["ct"], hdr["channels"], hdr["bits"], hdr["bytes_per_sample"]) == (ct, c, bits, img.itemsize)
    fd = oracle.forward_dump(img, lv, bits=bits, ct=ct, qstep=q)
    for ch in range(c):
        assert np.array_equal(coefs[ch]["LL"], fd[ch]["LL"])
    top = (1 << bits) - 1
    if q == 1:
        assert np.array_equal(oracle.decode_tile(blob, 0), img)
    for z in range(1, lv + 1):
        if q > 1 and z < lv:
            continue  # lossy: only the coarsest LL is exact
        llz = oracle.forward_dump(img, z, bits=bits, ct=ct)
        planes = np.stack([d["LL"] for d in llz], axis=-1).astype(np.int64)
        exp = np.clip(_inv_colour(planes, ct), 0, top).astype(img.dtype)
        assert np.array_equal(oracle.decode_tile(blob, z), exp)


def test_generality_limits_rejected():
    ok = synth.random_image(8, 8, 3, 8, seed=1)
    with pytest.raises(oracle.OracleError):
        oracle.encode_tile(ok[:, :, :2], 1, ct=2)  # colour transforms need 3 channels
    with pytest.raises(oracle.OracleError):
        oracle.encode_tile(ok, 1, ct=3)
    with pytest.raises(oracle.OracleError):
        oracle.encode_tile(synth.random_image(8, 8, 1, 24, seed=2), 1, bits=25)
    with pytest.raises(oracle.OracleError):
        oracle.encode_tile(np.zeros((4, 4, 65), np.uint8), 1, ct=0)


def test_constant_image_blocks_are_header_only():
    img = np.full((300, 260, 3), 217, dtype=np.uint8)
    blob = oracle.encode_tile(img, 4)
    hdr, blocks = fr.parse_tile(blob)
    for (lvl, *_), data in blocks:
        if lvl > 0:
            assert data == bytes([0b00001111])  # d=1 (00001) + three masks "1"
    assert np.array_equal(oracle.decode_tile(blob), img)


def test_lossy_quantiser_and_reconstruction():
    rng = np.random.default_rng(7)
    img = synth.he_like(96, 80, 5)
    for step in (2, 3, 4, 7):
        qd = oracle.forward_dump(img, 3, qstep=step)
        fd = oracle.forward_dump(img, 3, qstep=1)
        for ch in range(3):
            assert np.array_equal(qd[ch]["LL"], fd[ch]["LL"])
            for l in range(1, 4):
                for nm in ("HL", "LH", "HH"):
                    c = fd[ch][nm][l].astype(np.int64)
                    assert np.array_equal(qd[ch][nm][l], np.sign(c) * (np.abs(c) // step))
        blob = oracle.encode_tile(img, 3, qstep=step)
        hdr, coefs = fr.tile_coefficients(blob)
        assert hdr["qstep"] == step
        dec = oracle.decode_tile(blob)
        err = np.abs(dec.astype(np.int64) - img.astype(np.int64))
        assert err.max() <= 4 * step + 4
    _ = rng


def _read_dequant_golden():
    values, tiles = [], []
    with open(os.path.join(GOLDEN, "dequant_examples.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            parts = line.split()
            if parts[0] == "tile":
                tiles.append(tuple(int(v) for v in parts[1:]))
            else:
                values.append(tuple(int(v) for v in parts))
    return values, tiles


def test_dequantiser_worked_values_and_midpoint():
    """Reconstruction of the dead-zone quantiser (Sec. 3, JPEG2000-style):
    hand-worked values for steps 2, 3, 4, 7, both signs and q = 0; and for
    every c the reconstruction is the middle of c's bin, floor((|q| + 1/2) step),
    with the sign of c (exact rational arithmetic, no use of the formula)."""
    from fractions import Fraction
    values, _ = _read_dequant_golden()
    for step, q, rec in values:
        assert oracle.dequantise(q, step) == rec, (step, q)
    for step in (1, 2, 3, 4, 5, 7, 8, 16):
        for c in range(-300, 301):
            q = oracle.quantise(c, step)
            # q is the bin index: |q| step <= |c| < (|q| + 1) step, sign of c
            assert abs(q) * step <= abs(c) < (abs(q) + 1) * step
            assert q == 0 or (q > 0) == (c > 0)
            rec = oracle.dequantise(q, step)
            if step == 1:
                assert rec == c
            elif q == 0:
                assert rec == 0
            else:
                mid = (Fraction(abs(q)) + Fraction(1, 2)) * step
                assert abs(rec) == int(mid) and (rec > 0) == (q > 0)
                assert oracle.quantise(rec, step) == q  # stays in its bin


def test_lossy_tile_decode_worked_examples():
    """Hand-worked lossy decodes of 2x1 tiles (one level, one channel): the
    dequantised high-pass coefficient, inverse lifting and clamp, end to end
    through the oracle's encoder and decoder."""
    _, tiles = _read_dequant_golden()
    for step, a, b, ra, rb in tiles:
        img = np.array([[a, b]], dtype=np.uint8)
        blob = oracle.encode_tile(img, 1, bits=8, ct=0, qstep=step)
        assert oracle.decode_tile(blob)[:, :, 0].tolist() == [[ra, rb]], (step, a, b)


def test_c1_workload_roundtrip():
    for seed in (101, 102, 103):
        img = synth.he_like(256, 256, seed)
        blob = oracle.encode_tile(img, 3)
        assert np.array_equal(oracle.decode_tile(blob), img)
        assert len(blob) < img.nbytes


# ---------------------------------------------------------------- quality-progressive decode
def _drop_planes(q, r):
    """Definition of the reduced-quality coefficient: magnitude bits below r
    unknown; a non-zero kept part is placed at the middle of its range."""
    if r == 0:
        return q
    mag = np.abs(q) >> r << r
    mag = np.where(mag != 0, mag + (1 << (r - 1)), 0)
    return np.sign(q) * mag


@pytest.mark.parametrize("kind", ["he8_lossless", "he8_step4", "gray12", "sparse"])
def test_progressive_block_decode_matches_truncated_reader(kind):
    """Blocks decoded with r planes left out equal the independent reader's
    exact coefficients with the low r magnitude bits replaced per the
    definition (Sec. 4, decompression: the seek table lets a decoder drop LSB planes)."""
    if kind == "he8_lossless":
        img, lv, q = synth.he_like(150, 140, 31), 3, 1
    elif kind == "he8_step4":
        img, lv, q = synth.he_like(150, 140, 32), 3, 4
    elif kind == "gray12":
        img, lv, q = synth.random_image(130, 70, 1, 12, seed=33, kind="ramp"), 2, 1
    else:
        img, lv, q = synth.random_image(140, 100, 3, 8, seed=34, kind="sparse"), 3, 1
    bits = 12 if kind == "gray12" else 8
    blob = oracle.encode_tile(img, lv, bits=bits, qstep=q)
    hdr, blocks = fr.parse_tile(blob)
    n_changed = 0
    for g, data in blocks:
        p, wb, hb = g[4], g[5], g[6]
        exact = fr.decode_block(data, p, wb, hb)
        for r in (1, 2, 3, 5, 9, 31):
            got = oracle.decode_block(data, p, wb, hb, drop=r).astype(np.int64)
            exp = _drop_planes(exact, r)
            assert np.array_equal(got, exp), (g[:4], r)
            n_changed += int((got != exact).sum())
    assert n_changed > 0


def test_progressive_tile_decode_limits_and_monotone_error():
    img = synth.he_like(200, 160, 35)
    blob = oracle.encode_tile(img, 4)
    assert np.array_equal(oracle.decode_tile(blob, 0, drop=0), img)
    # every magnitude plane dropped: all coefficients 0, and the inverse
    # colour transform of (0, 0, 0) is black
    for z in (0, 2):
        assert not oracle.decode_tile(blob, z, drop=31).any()
    errs = []
    for r in (0, 1, 2, 3, 4, 6):
        d = oracle.decode_tile(blob, 0, drop=r).astype(np.int64)
        errs.append(np.abs(d - img.astype(np.int64)).mean())
    assert errs[0] == 0 and all(a <= b + 1e-9 for a, b in zip(errs, errs[1:])), errs
    assert oracle.decode_status(blob, 0, drop=32) == -1


# ---------------------------------------------------------------- robustness
def test_corrupt_and_truncated_streams_are_rejected_without_crash():
    img = synth.he_like(64, 48, 9)
    blob = oracle.encode_tile(img, 2)
    for cut in (0, 10, 23, 24, 40, len(blob) // 2, len(blob) - 1):
        assert oracle.decode_status(blob[:cut]) != oracle.OK
    rng = np.random.default_rng(2)
    hdr_len = 24 + 4 * oracle.read_header(blob)["nblocks"]
    bad = 0
    for _ in range(200):
        b = bytearray(blob)
        pos = int(rng.integers(hdr_len, len(b)))
        b[pos] ^= 1 << int(rng.integers(0, 8))
        st = oracle.decode_status(bytes(b))
        bad += st != oracle.OK
    assert bad > 40  # many single-bit flips are detected; none may crash
