"""CPU oracle of the codec: TEST INFRASTRUCTURE ONLY.

Plain scalar C (``isx_oracle.c``) reached through ctypes.  Only the tests,
the smoke check and the benchmark's CPU-baseline leg may import this
package; the product library never does, and the two share no code.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "isx_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, E_INVALID, E_CAPACITY, E_CORRUPT, E_TRUNCATED, E_UNSUPPORTED, E_NOMEM = 0, -1, -2, -3, -4, -5, -6


def build(force: bool = True) -> str:
    """Compile the oracle with the host C compiler (plain -O2, no intrinsics)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared",
                               "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


class BlockInfo(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("p", ctypes.c_int32), ("wb", ctypes.c_int32),
                ("hb", ctypes.c_int32), ("n_segments", ctypes.c_int32), ("czr", ctypes.c_int32),
                ("wz", ctypes.c_int32), ("l_provisional", ctypes.c_int32),
                ("limited", ctypes.c_int32), ("tbits", ctypes.c_int32),
                ("masks", ctypes.c_uint32 * 3), ("lengths", ctypes.c_uint8 * 256),
                ("freq", ctypes.c_uint64 * 256), ("seg_bits", ctypes.c_uint32 * 32),
                ("run_hist", ctypes.c_uint64 * 40), ("total_bits", ctypes.c_uint64)]


def build_sanitized(path: str) -> str:
    """Compile the oracle with AddressSanitizer and UndefinedBehaviorSanitizer
    (every report fatal) into `path`; a process loads it through
    ISX_ORACLE_LIB, with the ASan runtime preloaded."""
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-Wall", "-Wno-alloc-size-larger-than",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-fno-omit-frame-pointer", "-shared", "-fPIC", "-o", path, _SRC])
    return path


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("ISX_ORACLE_LIB") or _LIB
        if path == _LIB and (not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
            build()
        L = ctypes.CDLL(path)
        P = ctypes.c_void_p
        i32, i64, u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
        L.oracle_encode_tile.restype = i64
        L.oracle_encode_tile.argtypes = [P, i32, i32, i32, i32, i32, i32, i32, i32, i32, P, u64]
        L.oracle_decode_tile.restype = i32
        L.oracle_decode_tile.argtypes = [P, u64, i32, P, i32]
        L.oracle_decode_tile_q.restype = i32
        L.oracle_decode_tile_q.argtypes = [P, u64, i32, i32, P, i32]
        L.oracle_read_header.restype = i32
        L.oracle_read_header.argtypes = [P, u64, P]
        L.oracle_forward_dump.restype = i64
        L.oracle_forward_dump.argtypes = [P, i32, i32, i32, i32, i32, i32, i32, i32, i32, P, i64]
        L.oracle_lift53_forward_1d.restype = None
        L.oracle_lift53_forward_1d.argtypes = [P, i32, P, P]
        L.oracle_lift53_inverse_1d.restype = None
        L.oracle_lift53_inverse_1d.argtypes = [P, P, i32, P]
        L.oracle_quantise.restype = i32
        L.oracle_quantise.argtypes = [i32, i32]
        L.oracle_dequantise.restype = i32
        L.oracle_dequantise.argtypes = [i32, i32]
        L.oracle_rct_forward.restype = None
        L.oracle_rct_forward.argtypes = [i32, i32, i32, P]
        L.oracle_rct_inverse.restype = None
        L.oracle_rct_inverse.argtypes = [i32, i32, i32, P]
        L.oracle_rct_selftest_u8.restype = i64
        L.oracle_ycocg_selftest_u8.restype = i64
        L.oracle_ycocg_forward.restype = None
        L.oracle_ycocg_forward.argtypes = [i32, i32, i32, P]
        L.oracle_ycocg_inverse.restype = None
        L.oracle_ycocg_inverse.argtypes = [i32, i32, i32, P]
        L.oracle_area_coord.restype = None
        L.oracle_area_coord.argtypes = [i32, i32, i32, i32, P]
        L.oracle_huffman_lengths.restype = i32
        L.oracle_huffman_lengths.argtypes = [P, i32, P]
        L.oracle_canonical_codes.restype = None
        L.oracle_canonical_codes.argtypes = [P, P]
        L.oracle_encode_block.restype = i64
        L.oracle_encode_block.argtypes = [P, i32, i32, i32, P, u64, P]
        L.oracle_decode_block.restype = i32
        L.oracle_decode_block.argtypes = [P, u64, i32, i32, i32, P]
        L.oracle_decode_block_q.restype = i32
        L.oracle_decode_block_q.argtypes = [P, u64, i32, i32, i32, i32, P]
        L.oracle_count_blocks.restype = i32
        L.oracle_count_blocks.argtypes = [i32, i32, i32, i32]
        L.oracle_block_geometry.restype = i32
        L.oracle_block_geometry.argtypes = [i32, i32, i32, i32, P, i32]
        L.oracle_blockinfo_size.restype = i32
        assert L.oracle_blockinfo_size() == ctypes.sizeof(BlockInfo)
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _as_hwc(pixels: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(pixels)
    if a.ndim == 2:
        a = a[:, :, None]
    if a.dtype not in (np.uint8, np.uint16, np.uint32):
        raise TypeError("pixels must be uint8, uint16 or uint32")
    return a


def max_encoded_bytes(w: int, h: int, channels: int, levels: int, bits: int) -> int:
    """Generous host bound for the oracle's output buffer."""
    nb = lib().oracle_count_blocks(w, h, channels, levels)
    coeffs = w * h * channels
    return 24 + 4 * nb + nb * 4096 + coeffs * (bits + 16) * 2


def encode_tile(pixels: np.ndarray, levels: int, bits: int | None = None, ct: int | None = None,
                qstep: int = 1) -> bytes:
    a = _as_hwc(pixels)
    h, w, c = a.shape
    bps = a.itemsize
    if bits is None:
        bits = 8 * bps
    if ct is None:
        ct = 1 if c == 3 else 0
    nb = lib().oracle_count_blocks(w, h, c, levels)
    for cap in (64 + 8 * nb + 2 * w * h * c * bps + 512 * nb, max_encoded_bytes(w, h, c, levels, bits)):
        out = np.zeros(cap, dtype=np.uint8)
        n = lib().oracle_encode_tile(_ptr(a), w, h, w * c * bps, c, bps, bits, levels, ct, qstep,
                                     _ptr(out), cap)
        if n != E_CAPACITY:
            break
    if n < 0:
        raise OracleError(int(n))
    return out[:n].tobytes()


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__(f"oracle error {code}")
        self.code = code


def read_header(blob: bytes) -> dict:
    b = np.frombuffer(blob, dtype=np.uint8)
    o = np.zeros(9, dtype=np.int32)
    rc = lib().oracle_read_header(_ptr(b), len(b), _ptr(o))
    if rc:
        raise OracleError(rc)
    keys = ["width", "height", "channels", "bytes_per_sample", "bits", "levels", "ct", "qstep",
            "nblocks"]
    return dict(zip(keys, map(int, o)))


def decode_tile(blob: bytes, level: int = 0, drop: int = 0) -> np.ndarray:
    """Decode at resolution level `level`; `drop` = number of least significant
    magnitude planes left out of every block (quality-progressive decode)."""
    hd = read_header(blob)
    w, h, c, bps = hd["width"], hd["height"], hd["channels"], hd["bytes_per_sample"]
    ow, oh = -(-w // (1 << level)), -(-h // (1 << level))
    dt = {1: np.uint8, 2: np.uint16, 4: np.uint32}[bps]
    out = np.zeros((oh, ow, c), dtype=dt)
    b = np.frombuffer(blob, dtype=np.uint8)
    rc = lib().oracle_decode_tile_q(_ptr(b), len(b), level, drop, _ptr(out), ow * c * bps)
    if rc:
        raise OracleError(rc)
    return out


def decode_region(blob: bytes, level: int, x0: int, y0: int, w: int, h: int, drop: int = 0) -> np.ndarray:
    """Region [x0, x0+w) x [y0, y0+h) of the level-`level` image.  By
    definition this is the crop of the whole decode at that level (Sec. 4, decompression:
    a viewer shows part of one scale); no other arithmetic."""
    full = decode_tile(blob, level, drop)
    if not (0 <= x0 and 0 <= y0 and w >= 1 and h >= 1 and x0 + w <= full.shape[1] and y0 + h <= full.shape[0]):
        raise OracleError(E_INVALID)
    return full[y0:y0 + h, x0:x0 + w].copy()


def decode_status(blob: bytes, level: int = 0, drop: int = 0) -> int:
    """Decode and return only the status code (for robustness tests)."""
    try:
        decode_tile(blob, level, drop)
    except OracleError as e:
        return e.code
    return OK


def forward_dump(pixels: np.ndarray, levels: int, bits: int | None = None, ct: int | None = None,
                 qstep: int = 1):
    """Per channel: {'LL': array, 'HL': [l=1..L], 'LH': [...], 'HH': [...]} (quantised)."""
    a = _as_hwc(pixels)
    h, w, c = a.shape
    bps = a.itemsize
    if bits is None:
        bits = 8 * bps
    if ct is None:
        ct = 1 if c == 3 else 0
    cap = w * h * c + 16
    out = np.zeros(cap, dtype=np.int32)
    n = lib().oracle_forward_dump(_ptr(a), w, h, w * c * bps, c, bps, bits, levels, ct, qstep,
                                  _ptr(out), cap)
    if n < 0:
        raise OracleError(int(n))
    res = []
    k = 0
    sizes = []
    cw, ch = w, h
    for lv in range(1, levels + 1):
        sizes.append((cw, ch))
        cw, ch = (cw + 1) // 2, (ch + 1) // 2
    for _ in range(c):
        d = {"LL": None, "HL": [None] * (levels + 1), "LH": [None] * (levels + 1),
             "HH": [None] * (levels + 1)}
        d["LL"] = out[k:k + cw * ch].reshape(ch, cw).copy()
        k += cw * ch
        for lv in range(levels, 0, -1):
            pw, ph = sizes[lv - 1]
            for name, (bw, bh) in (("HL", (pw // 2, (ph + 1) // 2)), ("LH", ((pw + 1) // 2, ph // 2)),
                                   ("HH", (pw // 2, ph // 2))):
                d[name][lv] = out[k:k + bw * bh].reshape(bh, bw).copy()
                k += bw * bh
        res.append(d)
    assert k == n
    return res


def lift_forward_1d(x):
    x = np.ascontiguousarray(x, dtype=np.int32)
    n = len(x)
    lo = np.zeros((n + 1) // 2, dtype=np.int32)
    hi = np.zeros(max(n // 2, 1), dtype=np.int32)
    lib().oracle_lift53_forward_1d(_ptr(x), n, _ptr(lo), _ptr(hi))
    return lo, hi[:n // 2]


def lift_inverse_1d(lo, hi, n):
    lo = np.ascontiguousarray(lo, dtype=np.int32)
    hi = np.ascontiguousarray(np.concatenate([hi, [0]]), dtype=np.int32)
    x = np.zeros(n, dtype=np.int32)
    lib().oracle_lift53_inverse_1d(_ptr(lo), _ptr(hi), n, _ptr(x))
    return x


def quantise(c: int, step: int) -> int:
    return int(lib().oracle_quantise(int(c), int(step)))


def dequantise(q: int, step: int) -> int:
    return int(lib().oracle_dequantise(int(q), int(step)))


def rct_forward(r, g, b):
    o = np.zeros(3, dtype=np.int32)
    lib().oracle_rct_forward(int(r), int(g), int(b), _ptr(o))
    return tuple(int(v) for v in o)


def rct_inverse(y, cb, cr):
    o = np.zeros(3, dtype=np.int32)
    lib().oracle_rct_inverse(int(y), int(cb), int(cr), _ptr(o))
    return tuple(int(v) for v in o)


def rct_selftest_u8() -> int:
    return int(lib().oracle_rct_selftest_u8())


def ycocg_forward(r, g, b):
    o = np.zeros(3, dtype=np.int32)
    lib().oracle_ycocg_forward(int(r), int(g), int(b), _ptr(o))
    return tuple(int(v) for v in o)


def ycocg_inverse(y, co, cg):
    o = np.zeros(3, dtype=np.int32)
    lib().oracle_ycocg_inverse(int(y), int(co), int(cg), _ptr(o))
    return tuple(int(v) for v in o)


def ycocg_selftest_u8() -> int:
    return int(lib().oracle_ycocg_selftest_u8())


def area_coord(k, wb, hb, d):
    o = np.zeros(3, dtype=np.int32)
    lib().oracle_area_coord(k, wb, hb, d, _ptr(o))
    return tuple(int(v) for v in o)


def huffman_lengths(freq, limit: int = 0) -> np.ndarray:
    f = np.zeros(256, dtype=np.uint64)
    f[:len(freq)] = freq
    ln = np.zeros(256, dtype=np.uint8)
    rc = lib().oracle_huffman_lengths(_ptr(f), limit, _ptr(ln))
    if rc:
        raise OracleError(rc)
    return ln


def canonical_codes(lengths) -> np.ndarray:
    ln = np.ascontiguousarray(lengths, dtype=np.uint8)
    code = np.zeros(256, dtype=np.uint32)
    lib().oracle_canonical_codes(_ptr(ln), _ptr(code))
    return code


def encode_block(types: np.ndarray):
    """types: int32 array (p, Hb, Wb) of quantised coefficients."""
    t = np.ascontiguousarray(types, dtype=np.int32)
    p, hb, wb = t.shape
    cap = 64 + p * hb * wb * 8
    out = np.zeros(cap, dtype=np.uint8)
    info = BlockInfo()
    n = lib().oracle_encode_block(_ptr(t), p, wb, hb, _ptr(out), cap, ctypes.byref(info))
    if n < 0:
        raise OracleError(int(n))
    return out[:n].tobytes(), info


def decode_block(blob: bytes, p: int, wb: int, hb: int, drop: int = 0) -> np.ndarray:
    b = np.frombuffer(blob, dtype=np.uint8)
    out = np.zeros((p, hb, wb), dtype=np.int32)
    rc = lib().oracle_decode_block_q(_ptr(b), len(b), p, wb, hb, drop, _ptr(out))
    if rc:
        raise OracleError(rc)
    return out


def block_geometry(w, h, channels, levels) -> np.ndarray:
    n = lib().oracle_count_blocks(w, h, channels, levels)
    out = np.zeros((max(n, 1), 13), dtype=np.int32)
    lib().oracle_block_geometry(w, h, channels, levels, _ptr(out), n)
    return out[:n]
