"""Independent pure-Python reader of the codec's bitstream (test checker).

Written from the format as read from the paper (Sec. 4, Eq. 1-3, Fig. 3
caption) without using the oracle: it parses the tile container and every
block (d, masks, C_zr, wz, recursive tree, seek table, segments), decodes the
tokens and scatters the 4x2 area symbols back to coefficients by walking the
blocks cell by cell (not through the k -> (row, col, plane) formula the
oracle uses).  Tests compare what it recovers with the oracle's forward
transform, which pins the oracle's encoder against the format.
"""
from __future__ import annotations

import struct

import numpy as np


class Bits:
    def __init__(self, data: bytes, start_bit: int = 0, end_bit: int | None = None):
        self.data = data
        self.pos = start_bit
        self.end = len(data) * 8 if end_bit is None else end_bit

    def get(self, n: int) -> int:
        v = 0
        for _ in range(n):
            if self.pos >= self.end:
                raise ValueError("read past end")
            byte = self.data[self.pos >> 3]
            v = (v << 1) | ((byte >> (7 - (self.pos & 7))) & 1)
            self.pos += 1
        return v


def parse_tree(bits: Bits):
    """Returns a dict codeword-string -> symbol (Fig. 3: 0 internal, 1+8 leaf)."""
    table = {}

    def rec(prefix):
        if bits.get(1):
            table[prefix] = bits.get(8)
        else:
            rec(prefix + "0")
            rec(prefix + "1")

    rec("")
    return table


def block_geometry(w, h, channels, levels):
    """Block list: (level, chan, bx, by, p, wb, hb, extents[(w,h)...])."""
    sizes = [(w, h)]
    for _ in range(levels):
        pw, ph = sizes[-1]
        sizes.append(((pw + 1) // 2, (ph + 1) // 2))
    out = []
    lw, lh = sizes[levels]
    for c in range(channels):
        for by in range(-(-lh // 128)):
            for bx in range(-(-lw // 128)):
                cw, ch = min(128, lw - 128 * bx), min(128, lh - 128 * by)
                out.append((0, c, bx, by, 1, -(-cw // 4) * 4, -(-ch // 4) * 4, [(cw, ch)]))
    for lv in range(levels, 0, -1):
        pw, ph = sizes[lv - 1]
        gw, gh, hw, hh = (pw + 1) // 2, (ph + 1) // 2, pw // 2, ph // 2
        for c in range(channels):
            for by in range(-(-gh // 128)):
                for bx in range(-(-gw // 128)):
                    cw, ch = min(128, gw - 128 * bx), min(128, gh - 128 * by)
                    hwc = max(0, min(128, hw - 128 * bx))
                    hhc = max(0, min(128, hh - 128 * by))
                    if hwc == 0 and hhc == 0:
                        continue
                    ext = [(cw, hhc), (hwc, ch), (hwc, hhc)]
                    out.append((lv, c, bx, by, 3, -(-cw // 4) * 4, -(-ch // 4) * 4, ext))
    return out


def decode_block(data: bytes, p: int, wb: int, hb: int, info: dict | None = None):
    """Decode one block into an int array (p, hb, wb) of quantised coefficients."""
    n = wb * hb // 8
    bits = Bits(data)
    d = bits.get(5)
    masks = [bits.get(d) for _ in range(p)]
    # plane b is present for type t if its mask bit is 0; mask is MSB-first
    present = [[((masks[t] >> b) & 1) == 0 for b in range(d)] for t in range(p)]
    planes = [b for b in range(d - 1, -1, -1) if any(present[t][b] for t in range(p))]
    coef_bits = np.zeros((p, d, hb, wb), dtype=np.int64)
    if info is not None:
        info.update(d=d, masks=masks, planes=planes)
    if not planes:
        return np.zeros((p, hb, wb), dtype=np.int64)
    czr = bits.get(8)
    wz = bits.get(4)
    table = parse_tree(bits)
    t = (p * n).bit_length() - 1 + 5
    seglens = [bits.get(t) for _ in planes]
    if info is not None:
        info.update(czr=czr, wz=wz, table=table, seglens=seglens)
    base = (1 << wz) - 1
    pos = bits.pos
    for b, sl in zip(planes, seglens):
        kept = [tt for tt in range(p) if present[tt][b]]
        m = n * len(kept)
        sb = Bits(data, pos, pos + sl)
        syms = []
        run = 0
        while len(syms) + run < m:
            if "" in table:
                s = table[""]
            else:
                code = ""
                while code not in table:
                    code += str(sb.get(1))
                s = table[code]
            if s == czr:
                c = sb.get(wz)
                if c:
                    run = run * base + c
                    continue
            syms.extend([0] * run)
            run = 0
            syms.append(s)
        syms.extend([0] * run)
        assert len(syms) == m and sb.pos == pos + sl, "segment length mismatch"
        pos += sl
        # scatter: walk the 4-row bands and 4-column groups (Eq. 1 as read)
        for i, tt in enumerate(kept):
            seg = syms[i * n:(i + 1) * n]
            k = 0
            for band in range(hb // 4):
                for cg in range(wb // 4):
                    for half in range(2):  # upper 4x2 area, then lower
                        s = seg[k]
                        k += 1
                        for bit in range(8):
                            if (s >> bit) & 1:
                                r = 4 * band + 2 * half + bit // 4
                                col = 4 * cg + bit % 4
                                coef_bits[tt, b, r, col] = 1
    mag = np.zeros((p, hb, wb), dtype=np.int64)
    for b in range(d - 1):
        mag |= coef_bits[:, b] << b
    sign = coef_bits[:, d - 1]
    return np.where(sign == 1, -mag, mag)


def block_payload_bits(data: bytes, p: int, wb: int, hb: int):
    """(first bit of the seek table, first payload bit, end of the payload)
    of one block, or None when the block keeps no bit plane."""
    n = wb * hb // 8
    bits = Bits(data)
    d = bits.get(5)
    masks = [bits.get(d) for _ in range(p)]
    planes = [b for b in range(d) if any(((masks[t] >> b) & 1) == 0 for t in range(p))]
    if not planes:
        return None
    bits.get(8)
    bits.get(4)
    parse_tree(bits)
    seek = bits.pos
    t = (p * n).bit_length() - 1 + 5
    total = sum(bits.get(t) for _ in planes)
    return seek, bits.pos, bits.pos + total


def parse_tile(blob: bytes):
    """Returns (header dict, list of (geometry, block bytes))."""
    assert blob[:4] == b"ISX1" and blob[4] == 1
    ct, ch, bits_, bps, lv = blob[5], blob[6], blob[7], blob[8], blob[9]
    q, w, h, nb = struct.unpack_from("<HIII", blob, 10)
    sizes = struct.unpack_from("<%dI" % nb, blob, 24)
    geo = block_geometry(w, h, ch, lv)
    assert len(geo) == nb
    pos = 24 + 4 * nb
    blocks = []
    for g, s in zip(geo, sizes):
        blocks.append((g, blob[pos:pos + s]))
        pos += s
    assert pos == len(blob)
    hdr = dict(ct=ct, channels=ch, bits=bits_, bytes_per_sample=bps, levels=lv, qstep=q,
               width=w, height=h, nblocks=nb)
    return hdr, blocks


def tile_coefficients(blob: bytes):
    """Decode every block; returns per channel {'LL': arr, ('LH'|'HL'|'HH', l): arr}."""
    hdr, blocks = parse_tile(blob)
    w, h, lv = hdr["width"], hdr["height"], hdr["levels"]
    sizes = [(w, h)]
    for _ in range(lv):
        pw, ph = sizes[-1]
        sizes.append(((pw + 1) // 2, (ph + 1) // 2))
    res = []
    for _ in range(hdr["channels"]):
        d = {"LL": np.zeros((sizes[lv][1], sizes[lv][0]), dtype=np.int64)}
        for l in range(1, lv + 1):
            pw, ph = sizes[l - 1]
            d[("HL", l)] = np.zeros(((ph + 1) // 2, pw // 2), dtype=np.int64)
            d[("LH", l)] = np.zeros((ph // 2, (pw + 1) // 2), dtype=np.int64)
            d[("HH", l)] = np.zeros((ph // 2, pw // 2), dtype=np.int64)
        res.append(d)
    for (lvl, c, bx, by, p, wb, hb, ext), data in blocks:
        q = decode_block(data, p, wb, hb)
        names = ["LL"] if lvl == 0 else [("LH", lvl), ("HL", lvl), ("HH", lvl)]
        for t, nm in enumerate(names):
            tw, th = ext[t]
            if tw and th:
                res[c][nm][128 * by:128 * by + th, 128 * bx:128 * bx + tw] = q[t, :th, :tw]
                # padding must decode to zero
                assert not q[t, th:, :].any() and not q[t, :, tw:].any()
    return hdr, res
