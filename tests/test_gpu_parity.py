"""GPU parity: the HIP library against the CPU oracle, through the C ABI.

Integer codec: every comparison is exact (coefficients, code lengths,
bitstream bytes, decoded pixels).
"""
import numpy as np
import pytest

import oracle
from paper_2005_08713_amd import isx, synth

pytestmark = pytest.mark.gpu

SMALL = [
    # (w, h, c, bits, levels, qstep, kind)
    (1, 1, 1, 8, 0, 1, "uniform"), (4, 4, 1, 8, 0, 1, "uniform"), (5, 3, 1, 8, 2, 1, "uniform"),
    (37, 23, 3, 8, 3, 1, "uniform"), (64, 64, 1, 12, 2, 1, "uniform"),
    (130, 257, 3, 8, 5, 1, "ramp"), (33, 17, 1, 16, 6, 1, "uniform"), (50, 50, 3, 8, 3, 4, "uniform"),
    (40, 9, 3, 8, 4, 3, "checker"), (16, 16, 1, 1, 2, 1, "sparse"), (129, 3, 1, 10, 3, 1, "max"),
    (200, 150, 3, 8, 4, 1, "sparse"), (1, 40, 3, 8, 6, 2, "uniform"), (257, 257, 1, 8, 1, 1, "uniform"),
    (300, 260, 3, 8, 4, 1, "const"), (140, 131, 3, 16, 3, 1, "uniform"), (2, 2, 1, 8, 1, 1, "uniform"),
    (511, 7, 3, 8, 5, 4, "uniform"), (3, 511, 3, 8, 5, 1, "ramp"), (128, 128, 3, 8, 15, 1, "uniform"),
]


def _img(case, seed=0):
    w, h, c, bits, lv, q, kind = case
    return synth.random_image(w, h, c, bits, seed=w * 7 + h + seed, kind=kind)


def _ct(c):
    return 1 if c == 3 else 0


@pytest.mark.parametrize("case", SMALL, ids=lambda c: "x".join(map(str, c)))
def test_forward_coefficients_match_oracle(case):
    w, h, c, bits, lv, q, kind = case
    img = _img(case)
    print("forward", case, flush=True)
    got = isx.debug_forward(img, lv, bits=bits, ct=_ct(c), qstep=q)
    ref = oracle.forward_dump(img, lv, bits=bits, ct=_ct(c), qstep=q)
    for ch in range(c):
        assert np.array_equal(got[ch]["LL"], ref[ch]["LL"]), (ch, "LL")
        for l in range(1, lv + 1):
            for nm in ("HL", "LH", "HH"):
                assert np.array_equal(got[ch][nm][l], ref[ch][nm][l]), (ch, nm, l)


def test_huffman_lengths_match_oracle():
    rng = np.random.default_rng(4)
    for trial in range(60):
        m = int(rng.integers(1, 257))
        f = np.zeros(256, dtype=np.uint64)
        idx = rng.choice(256, size=m, replace=False)
        f[idx] = rng.integers(1, [2, 10, 1000, 100000][trial % 4], size=m)
        got = isx.debug_huffman(f, 0)
        assert np.array_equal(got, oracle.huffman_lengths(f)), trial
    # length-limited fallback (package-merge) on Fibonacci weights
    f = np.zeros(256, dtype=np.uint64)
    a, b = 1, 1
    for s in range(30):
        f[s * 7 % 256] = a
        a, b = b, a + b
    for lim in (14, 12, 10):
        assert np.array_equal(isx.debug_huffman(f, lim), oracle.huffman_lengths(f, limit=lim))
    # unlimited on the same weights (one merge per round), and tie-heavy cases
    # where leaves and internal nodes of equal weight meet
    assert np.array_equal(isx.debug_huffman(f, 0), oracle.huffman_lengths(f))
    for g in (np.ones(256, dtype=np.uint64),
              np.array([1 << (k % 12) for k in range(256)], dtype=np.uint64),
              np.array([(k % 3) + 1 for k in range(256)], dtype=np.uint64),
              np.array([1, 1, 2, 2, 4, 4, 8, 8] + [0] * 248, dtype=np.uint64)):
        assert np.array_equal(isx.debug_huffman(g, 0), oracle.huffman_lengths(g))
    for trial in range(20):
        f = rng.integers(0, 5000, size=256).astype(np.uint64)
        f[rng.random(256) < 0.3] = 0
        assert np.array_equal(isx.debug_huffman(f, 14), oracle.huffman_lengths(f, limit=14))


@pytest.mark.parametrize("case", SMALL, ids=lambda c: "x".join(map(str, c)))
def test_encode_bitstream_matches_oracle(case):
    w, h, c, bits, lv, q, kind = case
    img = _img(case, 1)
    print("encode", case, flush=True)
    got = isx.encode_image(img, lv, bits=bits, ct=_ct(c), qstep=q)
    ref = oracle.encode_tile(img, lv, bits=bits, ct=_ct(c), qstep=q)
    assert len(got) == len(ref)
    assert got == ref


@pytest.mark.parametrize("case", SMALL, ids=lambda c: "x".join(map(str, c)))
def test_decode_matches_oracle_at_every_level(case):
    w, h, c, bits, lv, q, kind = case
    img = _img(case, 2)
    print("decode", case, flush=True)
    blob = oracle.encode_tile(img, lv, bits=bits, ct=_ct(c), qstep=q)
    levels = list(range(lv + 1))
    got = isx.decode_streams([blob] * len(levels), levels=levels)
    for z, g in zip(levels, got):
        assert np.array_equal(g, oracle.decode_tile(blob, z)), z
    if q == 1:
        assert np.array_equal(got[0], img.reshape(got[0].shape))


def test_c1_workload_seeds():
    for seed in (101, 102, 103):
        img = synth.he_like(256, 256, seed)
        print("C1 seed", seed, flush=True)
        got = isx.encode_image(img, 3)
        assert got == oracle.encode_tile(img, 3)
        dec = isx.decode_streams([got])[0]
        assert np.array_equal(dec, img)


def test_batch_of_uneven_tiles_matches_per_tile_oracle():
    tiles = synth.tile_batch(24, seed=7, content_seed_base=7000, sides=(128, 64, 32), max_side=200)
    imgs = [t["pixels"] for t in tiles]
    levels = [t["levels"] for t in tiles]
    qs = [t["qstep"] for t in tiles]
    print("batch encode", flush=True)
    got = isx.encode_images(imgs, levels, qs)
    for i, t in enumerate(tiles):
        assert got[i] == oracle.encode_tile(t["pixels"], t["levels"], qstep=t["qstep"]), i
    zs = [i % (t["levels"] + 1) for i, t in enumerate(tiles)]
    print("batch decode", flush=True)
    dec = isx.decode_streams(got, levels=zs)
    for i, t in enumerate(tiles):
        assert np.array_equal(dec[i], oracle.decode_tile(got[i], zs[i])), i


def test_mixed_depth_batch_matches_per_tile_oracle():
    """Tiles of 8 and 16 bits and different level counts in one plan: the
    per-block kernels are sized by the plan's largest plane bound, which the
    8-bit tiles do not reach."""
    imgs = [synth.he_like(200, 150, 31),
            synth.random_image(170, 130, 1, 16, 32, kind="uniform"),
            synth.he_like(96, 72, 33),
            synth.random_image(140, 90, 3, 16, 34, kind="max")]
    levels = [3, 4, 1, 2]
    qs = [1, 1, 4, 2]
    print("mixed-depth batch encode", flush=True)
    got = isx.encode_images(imgs, levels, qs)
    for i, img in enumerate(imgs):
        assert got[i] == oracle.encode_tile(img, levels[i], qstep=qs[i]), i
    print("mixed-depth batch decode", flush=True)
    dec = isx.decode_streams(got)
    for i, img in enumerate(imgs):
        assert np.array_equal(dec[i], oracle.decode_tile(got[i], 0)), i
        if qs[i] == 1:
            assert np.array_equal(dec[i].reshape(img.shape), img), i


def test_corrupt_segments_detected_like_oracle():
    """Bit flips in seek tables and segment payloads: the GPU decoder reports
    an error exactly when the oracle does, and decodes the same pixels when
    neither does (most flips of a single code bit still give a valid token
    sequence for a while; the run, length and end checks catch them)."""
    from tests import format_reader as fr
    rng = np.random.default_rng(77)
    cases = [(96, 80, 3, 3, 1, 901), (64, 64, 1, 2, 1, 902), (140, 130, 3, 4, 4, 903)]
    blobs, base = [], []
    for w, h, c, lv, q, seed in cases:
        img = synth.he_like(w, h, seed, sigma=(60.0, 300.0)) if c == 3 else \
            synth.random_image(w, h, 1, 8, seed=seed, kind="ramp")
        blob = oracle.encode_tile(img, lv, qstep=q)
        hdr, blocks = fr.parse_tile(blob)
        off = 24 + 4 * hdr["nblocks"]
        ranges = []
        for g, data in blocks:
            r = fr.block_payload_bits(data, g[4], g[5], g[6])
            if r is not None and r[2] > r[0]:
                ranges.append((off * 8 + r[0], off * 8 + r[2]))
            off += len(data)
        for k in range(24):
            lo, hi = ranges[int(rng.integers(len(ranges)))]
            bit = int(rng.integers(lo, hi))
            b = bytearray(blob)
            b[bit >> 3] ^= 0x80 >> (bit & 7)
            blobs.append(bytes(b))
            base.append(blob)
    got, st = isx.decode_streams(blobs, return_status=True)
    n_err = 0
    for i, blob in enumerate(blobs):
        ost = oracle.decode_status(blob)
        assert (st[i] != 0) == (ost != 0), (i, st[i], ost)
        if ost == 0:
            assert np.array_equal(got[i], oracle.decode_tile(blob, 0)), i
        else:
            n_err += 1
    assert n_err > len(blobs) // 4


def test_corrupt_code_trees_detected_like_oracle():
    """Bit flips inside the serialised code trees of block headers (one or
    two bits, or a byte's worth): the GPU decoder rejects a stream exactly
    when the oracle does, and otherwise decodes the same pixels.  Flips turn
    leaves into internal nodes and back, so trees end early, run past the
    header, grow past 32 levels or repeat symbols."""
    from tests import format_reader as fr
    rng = np.random.default_rng(78)
    cases = [(96, 80, 3, 3, 1, 911), (64, 64, 1, 2, 1, 912), (140, 130, 3, 4, 4, 913), (40, 36, 1, 1, 1, 914)]
    blobs = []
    for w, h, c, lv, q, seed in cases:
        img = synth.he_like(w, h, seed, sigma=(60.0, 300.0)) if c == 3 else \
            synth.random_image(w, h, 1, 8, seed=seed, kind="uniform" if seed % 2 else "ramp")
        blob = oracle.encode_tile(img, lv, qstep=q)
        hdr, blocks = fr.parse_tile(blob)
        off = 24 + 4 * hdr["nblocks"]
        trees = []
        for g, data in blocks:
            r = fr.block_payload_bits(data, g[4], g[5], g[6])
            if r is not None:
                d = data[0] >> 3
                t0 = 5 + g[4] * d + 12
                trees.append((off * 8 + t0, off * 8 + r[0]))
            off += len(data)
        for k in range(30):
            lo, hi = trees[int(rng.integers(len(trees)))]
            b = bytearray(blob)
            nflip = [1, 2, 8][k % 3]
            for bit in rng.integers(lo, hi, size=nflip):
                b[int(bit) >> 3] ^= 0x80 >> (int(bit) & 7)
            blobs.append(bytes(b))
    print("corrupt trees", len(blobs), flush=True)
    got, st = isx.decode_streams(blobs, return_status=True)
    n_err = 0
    for i, blob in enumerate(blobs):
        ost = oracle.decode_status(blob)
        assert (st[i] != 0) == (ost != 0), (i, st[i], ost)
        if ost == 0:
            assert np.array_equal(got[i], oracle.decode_tile(blob, 0)), i
        else:
            n_err += 1
    assert n_err > len(blobs) // 2


def test_progressive_decode_matches_oracle():
    """Quality-progressive decode (r magnitude planes left out of every block,
    midpoint reconstruction) at several resolution levels, in one mixed
    batch, equals the oracle."""
    cases = [
        (synth.he_like(300, 260, 41), 4, 1, 8),
        (synth.he_like(257, 129, 42), 3, 4, 8),
        (synth.random_image(140, 131, 1, 12, seed=43, kind="ramp").astype(np.uint16), 3, 1, 12),
        (synth.random_image(200, 150, 3, 8, seed=44, kind="sparse"), 4, 1, 8),
    ]
    blobs, levels, drops, exp = [], [], [], []
    for img, lv, q, bits in cases:
        blob = oracle.encode_tile(img, lv, bits=bits, qstep=q)
        for z, r in [(0, 0), (0, 1), (0, 3), (1, 2), (lv, 4), (0, 9), (2, 31)]:
            blobs.append(blob)
            levels.append(z)
            drops.append(r)
            exp.append(oracle.decode_tile(blob, z, drop=r))
    got = isx.decode_streams(blobs, levels=levels, drop=drops)
    for i, (g, e) in enumerate(zip(got, exp)):
        assert np.array_equal(g, e), (i, levels[i], drops[i])


GENERAL = [
    # (w, h, c, bits, levels, qstep, ct, kind): YCoCg-R, 9-bit RGB, 4-byte
    # samples with up to 24 bits, 16 and 64 channels
    (150, 97, 3, 8, 4, 1, 2, "uniform"), (64, 40, 3, 9, 3, 1, 2, "ramp"), (120, 88, 3, 9, 3, 1, 1, "uniform"),
    (77, 50, 3, 12, 3, 3, 2, "uniform"), (60, 45, 1, 24, 3, 1, 0, "uniform"), (70, 33, 3, 20, 4, 1, 1, "ramp"),
    (40, 40, 3, 24, 2, 5, 2, "uniform"), (50, 30, 16, 8, 3, 1, 0, "uniform"), (20, 12, 64, 10, 2, 1, 0, "ramp"),
    (300, 140, 3, 8, 5, 1, 2, "sparse"), (33, 31, 5, 16, 2, 2, 0, "uniform"), (1, 1, 3, 24, 0, 1, 2, "max"),
]


@pytest.mark.parametrize("case", GENERAL, ids=lambda c: "x".join(map(str, c)))
def test_generality_matches_oracle(case):
    """Forward coefficients, stream bytes, every resolution level and a
    reduced-quality decode equal the oracle's for the alternative colour
    transform, deep samples and many channels."""
    print("general", case, flush=True)
    _check_everything(case)


INTERIOR = [
    # (w, h, c, bits, levels, qstep, ct, kind): images of several 64x64
    # transform tiles with interior tiles (no reflection in the window), ragged
    # right and bottom tiles, and steps that are not powers of two; the output
    # formats cover 1, 2, 3 and 4 bytes per pixel and two channel groups
    (640, 456, 3, 8, 3, 1, 1, "uniform"), (517, 389, 3, 8, 5, 7, 1, "sparse"),
    (520, 390, 3, 8, 4, 3, 2, "ramp"), (600, 330, 1, 16, 3, 5, 0, "uniform"),
    (330, 300, 2, 8, 2, 1, 0, "uniform"), (300, 280, 1, 24, 3, 1, 0, "uniform"),
    (400, 200, 4, 8, 2, 2, 0, "uniform"), (384, 320, 1, 8, 1, 1, 0, "checker"),
]


@pytest.mark.parametrize("case", INTERIOR, ids=lambda c: "x".join(map(str, c)))
def test_interior_tiles_match_oracle(case):
    """The same checks on images large enough for the transform kernels' fast
    paths (aligned interior windows, whole-row output staging)."""
    print("interior", case, flush=True)
    _check_everything(case)


def _check_everything(case):
    w, h, c, bits, lv, q, ct, kind = case
    img = synth.random_image(w, h, c, bits, seed=w * 5 + h, kind=kind)
    got = isx.debug_forward(img, lv, bits=bits, ct=ct, qstep=q)
    ref = oracle.forward_dump(img, lv, bits=bits, ct=ct, qstep=q)
    for ch in range(c):
        assert np.array_equal(got[ch]["LL"], ref[ch]["LL"]), (ch, "LL")
        for l in range(1, lv + 1):
            for nm in ("HL", "LH", "HH"):
                assert np.array_equal(got[ch][nm][l], ref[ch][nm][l]), (ch, nm, l)
    blob = isx.encode_image(img, lv, bits=bits, ct=ct, qstep=q)
    assert blob == oracle.encode_tile(img, lv, bits=bits, ct=ct, qstep=q)
    levels = list(range(lv + 1))
    dec = isx.decode_streams([blob] * len(levels), levels=levels)
    for z, g in zip(levels, dec):
        assert g.dtype == img.dtype
        assert np.array_equal(g, oracle.decode_tile(blob, z)), z
    if q == 1:
        assert np.array_equal(dec[0], img.reshape(dec[0].shape))
    r = min(3, bits)
    prog = isx.decode_streams([blob], drop=r)[0]
    assert np.array_equal(prog, oracle.decode_tile(blob, 0, drop=r))



@pytest.mark.parametrize("case", [
    # encode side: level-1 bands are held as int16 up to 13 significant bits
    (96, 80, 3, 13, 2, 1, "checker"), (96, 80, 1, 13, 3, 1, "max"), (96, 80, 3, 14, 2, 1, "checker"),
    (70, 66, 1, 14, 3, 1, "max"),
    # level-2 bands: int16 up to 11 significant bits (2x2 checkers give the
    # largest level-2 coefficients), int32 from 12
    (96, 80, 3, 11, 3, 1, "checker2"), (96, 80, 1, 11, 3, 1, "checker2"), (96, 80, 3, 12, 3, 1, "checker2"),
    (70, 66, 1, 12, 3, 1, "checker2"),
    # decode side: 8-bit, 5 levels (plane bound 13): int16 up to step 8, int32 from step 9
    (160, 144, 3, 8, 5, 7, "checker"), (160, 144, 3, 8, 5, 8, "checker"), (160, 144, 3, 8, 5, 9, "checker"),
    (150, 130, 3, 8, 5, 8, "uniform"),
], ids=lambda c: "x".join(map(str, c)))
def test_int16_band_bounds_match_oracle(case):
    """Both sides of the int16 band rules of levels 1 and 2: images with the
    largest level-1 or level-2 coefficients the bit depth allows
    (checkerboards, alternating extremes) and steps on both sides of the
    decoder's dequantisation bound, encoded and decoded at every level
    against the oracle."""
    w, h, c, bits, lv, q, kind = case
    img = _img(case, 3)
    print("int16 bound", case, flush=True)
    got = isx.encode_image(img, lv, bits=bits, ct=_ct(c), qstep=q)
    ref = oracle.encode_tile(img, lv, bits=bits, ct=_ct(c), qstep=q)
    assert got == ref
    levels = list(range(lv + 1))
    dec = isx.decode_streams([ref] * len(levels), levels=levels)
    for z, g in zip(levels, dec):
        assert np.array_equal(g, oracle.decode_tile(ref, z)), z
    if q == 1:
        assert np.array_equal(dec[0], img.reshape(dec[0].shape))
