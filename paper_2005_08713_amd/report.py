"""Lossless compression report: this codec against the JPEG2000 and PNG
encoders available on the machine, on seeded synthetic stand-ins for the
paper's workloads (Sec. 5 compares lossless file sizes against JPEG2000 and
PNG on radiology and histopathology images; those images are not available).

* JPEG2000: Pillow's OpenJPEG encoder, reversible 5/3 wavelet, as many
  resolutions as this codec's levels + 1, 64x64 code blocks, raw codestream.
  RGB8 is tried with and without the reversible colour transform and the
  smaller result is kept.  Pillow has no 16-bit RGB mode, so deeper RGB is
  coded as three single-channel 16-bit images and their sizes are summed.
* PNG: written here from the PNG specification (IHDR / IDAT / IEND, filter
  type chosen per row by the smallest sum of absolute filtered byte values,
  zlib deflate at a chosen level), so that 16-bit RGB is covered too.

The codec under test is passed in as ``encode(img, levels, bits) -> bytes``;
run as a program it uses the GPU library.  Sizes are the only figures that
compare like with like; the times are context (different machines and
parallelism: the GPU against one CPU thread).
"""
from __future__ import annotations

import io
import struct
import time
import zlib

import numpy as np

# ------------------------------------------------------------------ PNG
_PNG_SIG = b"\x89PNG\r\n\x1a\n"


def _chunk(kind: bytes, data: bytes) -> bytes:
    return struct.pack(">I", len(data)) + kind + data + struct.pack(">I", zlib.crc32(kind + data) & 0xFFFFFFFF)


def _paeth(a, b, c):
    p = a + b - c
    pa, pb, pc = np.abs(p - a), np.abs(p - b), np.abs(p - c)
    return np.where((pa <= pb) & (pa <= pc), a, np.where(pb <= pc, b, c))


def png_filter_rows(raw: np.ndarray, bpp: int) -> bytes:
    """Filter each scanline (uint8, H x rowbytes) with the type among the five
    of the PNG specification whose output has the smallest sum of absolute
    values (bytes read as signed), the usual adaptive choice; returns the
    filtered stream with one type byte per row."""
    h, n = raw.shape
    x = raw.astype(np.int32)
    up = np.zeros_like(x)
    up[1:] = x[:-1]
    left = np.zeros_like(x)
    left[:, bpp:] = x[:, :-bpp]
    ul = np.zeros_like(x)
    ul[1:, bpp:] = x[:-1, :-bpp]
    cands = [x, x - left, x - up, x - ((left + up) >> 1), x - _paeth(left, up, ul)]
    cands = [(c & 0xFF).astype(np.uint8) for c in cands]
    cost = np.stack([np.abs(c.view(np.int8).astype(np.int32)).sum(axis=1) for c in cands])
    best = np.argmin(cost, axis=0)
    out = np.empty((h, n + 1), dtype=np.uint8)
    out[:, 0] = best
    for t in range(5):
        rows = best == t
        out[rows, 1:] = cands[t][rows]
    return out.tobytes()


def png_encode(img: np.ndarray, level: int = 6) -> bytes:
    """PNG file of a grey (H x W or H x W x 1) or RGB (H x W x 3) uint8 /
    uint16 image; 16-bit samples are stored big endian."""
    a = np.ascontiguousarray(img)
    if a.ndim == 2:
        a = a[:, :, None]
    h, w, c = a.shape
    if c not in (1, 3) or a.dtype not in (np.uint8, np.uint16):
        raise ValueError("PNG here takes 1 or 3 channels of uint8 / uint16")
    depth = 8 * a.itemsize
    raw = a.astype(a.dtype.newbyteorder(">")).view(np.uint8).reshape(h, w * c * a.itemsize)
    ihdr = struct.pack(">IIBBBBB", w, h, depth, 0 if c == 1 else 2, 0, 0, 0)
    body = zlib.compress(png_filter_rows(raw, c * a.itemsize), level)
    return _PNG_SIG + _chunk(b"IHDR", ihdr) + _chunk(b"IDAT", body) + _chunk(b"IEND", b"")


# ------------------------------------------------------------------ JPEG2000
def j2k_encode(img: np.ndarray, levels: int) -> bytes | list:
    """Smallest lossless JPEG2000 codestream(s) Pillow/OpenJPEG makes of img;
    a list of per-channel codestreams for 16-bit RGB."""
    from PIL import Image
    a = np.ascontiguousarray(img)
    if a.ndim == 3 and a.shape[2] == 1:
        a = a[:, :, 0]
    opts = dict(irreversible=False, no_jp2=True, codeblock_size=(64, 64),
                num_resolutions=min(levels + 1, 1 + int(np.log2(max(2, min(a.shape[:2]))))))

    def one(x, mct=0):
        b = io.BytesIO()
        Image.fromarray(x).save(b, "JPEG2000", mct=mct, **opts)
        return b.getvalue()

    if a.ndim == 2:
        return one(a)
    if a.dtype == np.uint8:
        return min((one(a, 0), one(a, 1)), key=len)
    return [one(np.ascontiguousarray(a[:, :, k])) for k in range(a.shape[2])]


def _nbytes(x):
    return sum(len(p) for p in x) if isinstance(x, list) else len(x)


# ------------------------------------------------------------------ workloads
def workloads(scale: int = 1):
    """(name, image, bits, levels): stand-ins for the paper's CR/DX/MG
    radiographs and its 8- and 9-bit histopathology scans."""
    from . import synth
    s = scale
    return [
        ("CR 12-bit 2048x2560", synth.rad_like(2048 // s, 2560 // s, 11, bits=12), 12, 5),
        ("DX 14-bit 3000x3000", synth.rad_like(3000 // s, 3000 // s, 12, bits=14), 14, 5),
        ("MG 14-bit 2560x3328", synth.rad_like(2560 // s, 3328 // s, 13, bits=14), 14, 5),
        ("HP RGB 8-bit 2048x2048", synth.he_like(2048 // s, 2048 // s, 14, sigma=(60.0, 300.0)), 8, 5),
        ("HP RGB 9-bit 2048x2048", synth.he_like(2048 // s, 2048 // s, 15, sigma=(60.0, 300.0), bits=9), 9, 5),
    ]


def compare(img: np.ndarray, bits: int, levels: int, encode, decode=None, png_level: int = 6) -> dict:
    """Sizes (bytes) and encode times (s) of this codec, JPEG2000 and PNG on one image."""
    raw = (img.size * bits + 7) // 8  # packed samples, independent of the container type
    t = time.perf_counter()
    ours = encode(img, levels, bits)
    t_ours = time.perf_counter() - t
    if decode is not None:
        back = decode(ours)
        if not np.array_equal(back.reshape(img.shape), img):
            raise AssertionError("lossless round trip failed")
    t = time.perf_counter()
    j2k = j2k_encode(img, levels)
    t_j2k = time.perf_counter() - t
    t = time.perf_counter()
    png = png_encode(img, png_level)
    t_png = time.perf_counter() - t
    r = {"raw": raw, "ours": len(ours), "j2k": _nbytes(j2k), "png": len(png),
         "t_ours": t_ours, "t_j2k": t_j2k, "t_png": t_png}
    r["vs_j2k"] = r["ours"] / r["j2k"] - 1.0
    r["vs_png"] = r["ours"] / r["png"] - 1.0
    return r


def table(rows) -> str:
    out = ["| workload | packed MB | this codec | JPEG2000 | PNG | vs JPEG2000 | vs PNG | enc ms (GPU / OpenJPEG / PNG) |",
           "|---|---|---|---|---|---|---|---|"]
    for name, r in rows:
        out.append(f"| {name} | {r['raw'] / 1e6:.1f} | {r['raw'] / r['ours']:.3f}:1 | {r['raw'] / r['j2k']:.3f}:1 | "
                   f"{r['raw'] / r['png']:.3f}:1 | {100 * r['vs_j2k']:+.1f}% | {100 * r['vs_png']:+.1f}% | "
                   f"{1e3 * r['t_ours']:.1f} / {1e3 * r['t_j2k']:.0f} / {1e3 * r['t_png']:.0f} |")
    return "\n".join(out)


def main():
    import argparse
    import torch
    from . import isx
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--scale", type=int, default=1, help="divide every workload side by this")
    args = ap.parse_args()

    def encode(img, levels, bits):
        d_pix, a = isx._as_device_pixels(img)
        h, w, c = a.shape
        enc = isx.Encoder([isx.tile_desc(w, h, c, a.itemsize, bits, levels)])
        enc.run(d_pix)  # warm-up: first launch and code-object load
        torch.cuda.synchronize()
        t = time.perf_counter()
        enc.run(d_pix)
        torch.cuda.synchronize()
        encode.gpu_s = time.perf_counter() - t
        return enc.streams()[0]

    def decode(blob):
        return isx.decode_streams([blob])[0]

    rows = []
    for name, img, bits, lv in workloads(args.scale):
        r = compare(img, bits, lv, encode, decode)
        r["t_ours"] = encode.gpu_s
        rows.append((name, r))
        print(name, {k: (round(v, 4) if isinstance(v, float) else v) for k, v in r.items()}, flush=True)
    total = {k: sum(r[k] for _, r in rows) for k in ("raw", "ours", "j2k", "png")}
    print(table(rows))
    print(f"total: this codec {100 * (total['ours'] / total['j2k'] - 1):+.1f}% vs JPEG2000, "
          f"{100 * (total['ours'] / total['png'] - 1):+.1f}% vs PNG")


if __name__ == "__main__":
    main()
