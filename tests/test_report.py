"""The compression report's own encoders (CPU): the PNG writer yields files
that an independent reader decodes to the input, and the comparison runs
end to end with the oracle standing in for the codec under test."""
import io
import struct
import zlib

import numpy as np
import pytest

import oracle
from paper_2005_08713_amd import report, synth


def _png_decode(blob: bytes) -> np.ndarray:
    """PNG reader written from the specification: chunks, inflate, the five
    row filters undone byte by byte (pure Python, small images only)."""
    assert blob[:8] == b"\x89PNG\r\n\x1a\n"
    pos, idat, hdr = 8, b"", None
    while pos < len(blob):
        n, kind = struct.unpack(">I4s", blob[pos:pos + 8])
        data = blob[pos + 8:pos + 8 + n]
        assert struct.unpack(">I", blob[pos + 8 + n:pos + 12 + n])[0] == zlib.crc32(kind + data) & 0xFFFFFFFF
        if kind == b"IHDR":
            hdr = struct.unpack(">IIBBBBB", data)
        elif kind == b"IDAT":
            idat += data
        pos += 12 + n
    w, h, depth, ctype = hdr[:4]
    c = 1 if ctype == 0 else 3
    bpp = c * depth // 8
    stride = w * bpp
    raw = zlib.decompress(idat)
    rows, prev = [], [0] * stride
    for y in range(h):
        t = raw[y * (stride + 1)]
        f = raw[y * (stride + 1) + 1:(y + 1) * (stride + 1)]
        cur = []
        for i in range(stride):
            a = cur[i - bpp] if i >= bpp else 0
            b = prev[i]
            cc = prev[i - bpp] if i >= bpp else 0
            if t == 0:
                p = 0
            elif t == 1:
                p = a
            elif t == 2:
                p = b
            elif t == 3:
                p = (a + b) // 2
            else:
                q = a + b - cc
                pa, pb, pc = abs(q - a), abs(q - b), abs(q - cc)
                p = a if pa <= pb and pa <= pc else (b if pb <= pc else cc)
            cur.append((f[i] + p) & 0xFF)
        rows.append(cur)
        prev = cur
    a = np.array(rows, dtype=np.uint8).reshape(h, w, c, depth // 8)
    if depth == 16:
        return (a[..., 0].astype(np.uint16) << 8) | a[..., 1]
    return a[..., 0]


@pytest.mark.parametrize("img", [
    synth.random_image(23, 9, 3, 8, 1, "uniform"), synth.random_image(17, 12, 1, 16, 2, "ramp"),
    synth.he_like(31, 20, 3, bits=9), synth.rad_like(40, 33, 4, bits=14)[:, :, None],
    synth.random_image(1, 1, 3, 16, 5, "max"), synth.random_image(19, 7, 1, 8, 6, "checker")])
def test_png_writer_round_trips_through_an_independent_reader(img):
    blob = report.png_encode(img)
    got = _png_decode(blob)
    assert np.array_equal(got, img.reshape(got.shape))


def test_png_writer_is_read_by_pillow():
    from PIL import Image
    for img in (synth.he_like(64, 48, 7), synth.rad_like(50, 40, 8)):
        back = np.asarray(Image.open(io.BytesIO(report.png_encode(img))))
        assert np.array_equal(back, img)


def test_comparison_end_to_end_with_the_oracle():
    rows = []
    for name, img, bits, lv in report.workloads(scale=16):
        r = report.compare(img, bits, lv, lambda a, l, b: oracle.encode_tile(a, l, bits=b),
                           lambda blob: oracle.decode_tile(blob))
        assert r["raw"] == (img.size * bits + 7) // 8
        assert 0 < r["ours"] < r["raw"] and 0 < r["j2k"] < r["raw"] and 0 < r["png"] < r["raw"]
        rows.append((name, r))
    text = report.table(rows)
    assert text.count("\n") == len(rows) + 1
