"""GPU parity of region decode on whole-slide pyramids: every region equals
the oracle's crop of the whole decode at its level, sample for sample, at
every level, at the image edges, for odd origins, single pixels, the whole
image, lossy streams, reduced quality, other sample types and colour
transforms, and many regions of one stream in one call."""
import numpy as np
import pytest

import oracle
from paper_2005_08713_amd import isx, synth

pytestmark = pytest.mark.gpu


def _regions(w, h, lv, rng, n_random=6):
    out = []
    for z in range(lv + 1):
        ow, oh = isx.out_size(w, h, z)
        out += [(z, 0, 0, ow, oh), (z, 0, 0, 1, 1), (z, ow - 1, oh - 1, 1, 1),
                (z, ow // 2, 0, ow - ow // 2, min(oh, 3))]
        for _ in range(n_random):
            x0, y0 = int(rng.integers(0, ow)), int(rng.integers(0, oh))
            out.append((z, x0, y0, int(rng.integers(1, ow - x0 + 1)), int(rng.integers(1, oh - y0 + 1))))
    return out


CASES = [
    # (w, h, c, bits, levels, qstep, ct, kind)
    (700, 530, 3, 8, 4, 1, 1, "he"), (700, 530, 3, 8, 4, 4, 1, "he"), (513, 777, 1, 12, 5, 1, 0, "rad"),
    (300, 260, 3, 9, 3, 1, 2, "uniform"), (260, 140, 5, 8, 3, 2, 0, "uniform"), (129, 1, 1, 8, 3, 1, 0, "ramp"),
    (1000, 300, 3, 8, 0, 1, 1, "he"), (257, 260, 3, 8, 7, 1, 1, "he"),
]


def _image(case, seed):
    w, h, c, bits, lv, q, ct, kind = case
    if kind == "he":
        return synth.he_like(w, h, seed, sigma=(40.0, 200.0))
    if kind == "rad":
        return synth.rad_like(w, h, seed, bits=bits)
    return synth.random_image(w, h, c, bits, seed, kind)


@pytest.mark.parametrize("case", CASES, ids=lambda c: "x".join(map(str, c)))
def test_regions_equal_crops_of_the_oracle_decode(case):
    w, h, c, bits, lv, q, ct, kind = case
    img = _image(case, w + h)
    blob = oracle.encode_tile(img, lv, bits=bits, ct=ct, qstep=q)
    rng = np.random.default_rng(w * 3 + h)
    regs = _regions(w, h, lv, rng)
    print("regions", case, len(regs), flush=True)
    got = isx.decode_regions(blob, regs)
    full = {z: oracle.decode_tile(blob, z) for z in range(lv + 1)}
    for (z, x0, y0, rw, rh), g in zip(regs, got):
        assert np.array_equal(g, full[z][y0:y0 + rh, x0:x0 + rw]), (z, x0, y0, rw, rh)


def test_regions_at_reduced_quality():
    img = synth.he_like(600, 450, 77, sigma=(40.0, 200.0))
    blob = oracle.encode_tile(img, 5)
    regs = [(0, 100, 37, 300, 211, 2), (1, 0, 0, 300, 225, 5), (2, 31, 17, 40, 60, 1), (5, 0, 0, 19, 15, 3),
            (0, 599, 449, 1, 1, 31)]
    print("progressive regions", flush=True)
    got = isx.decode_regions(blob, regs)
    for (z, x0, y0, rw, rh, r), g in zip(regs, got):
        assert np.array_equal(g, oracle.decode_region(blob, z, x0, y0, rw, rh, drop=r)), (z, r)


def test_whole_slide_regions_match_the_full_gpu_decode():
    """A 4000 x 3000 slide as one pyramid (6 levels): viewport regions at
    every zoom equal the corresponding crops of the GPU's whole decode
    (itself equal to the oracle's at the smaller sizes above), and a few
    equal the oracle's."""
    img = synth.he_like(4000, 3000, 91, sigma=(100.0, 600.0))
    print("slide encode", flush=True)
    blob = isx.encode_image(img, 6)
    rng = np.random.default_rng(5)
    regs = []
    for z in range(7):
        ow, oh = isx.out_size(4000, 3000, z)
        for _ in range(4):
            rw, rh = min(ow, 512), min(oh, 512)
            regs.append((z, int(rng.integers(0, ow - rw + 1)), int(rng.integers(0, oh - rh + 1)), rw, rh))
    print("slide regions", len(regs), flush=True)
    got = isx.decode_regions(blob, regs)
    fulls = isx.decode_streams([blob] * 7, levels=list(range(7)))
    assert np.array_equal(fulls[0], img)
    for (z, x0, y0, rw, rh), g in zip(regs, got):
        assert np.array_equal(g, fulls[z][y0:y0 + rh, x0:x0 + rw]), (z, x0, y0)
    for (z, x0, y0, rw, rh), g in list(zip(regs, got))[12::5]:
        assert np.array_equal(g, oracle.decode_region(blob, z, x0, y0, rw, rh)), (z, x0, y0)


def test_block_table_mismatch_is_reported_not_decoded():
    """Offsets that disagree with the stream's own size table give an error
    status for that job only; the other job of the call still decodes."""
    import torch
    img = synth.he_like(300, 300, 5)
    blob = oracle.encode_tile(img, 3)
    d = isx._parse_header(blob)
    good = isx.stream_block_offsets(blob[:24 + 4 * isx.struct_u32(blob, 20)])
    bad = good.copy()
    bad[1:-1] += 1  # every block shifted by one byte
    jobs = [isx.region_job(d, good, 0, 10, 10, 100, 100, in_bytes=len(blob)),
            isx.region_job(d, bad, 0, 10, 10, 100, 100, in_bytes=len(blob), out_offset=100 * 100 * 3)]
    dec = isx.Decoder(jobs, 2 * 100 * 100 * 3)
    dec.run(torch.from_numpy(np.frombuffer(blob, np.uint8).copy()).cuda())
    torch.cuda.synchronize()
    st = dec.status.cpu().numpy()
    assert st[0] == isx.OK and st[1] == isx.E_TRUNCATED
    out = dec.out.cpu().numpy()[:100 * 100 * 3].reshape(100, 100, 3)
    assert np.array_equal(out, img[10:110, 10:110])
