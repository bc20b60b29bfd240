"""Python binding of libisx.so (ctypes): argument marshalling only.

Every step of the codec runs in the HIP kernels of libisx; this module only
packs descriptors, allocates device buffers with torch and passes pointers
and the current HIP stream.  It raises if the library is missing: there is
no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libisx.so")

OK, E_INVALID_ARG, E_CAPACITY, E_CORRUPT, E_TRUNCATED, E_UNSUPPORTED, E_WORKSPACE, E_HIP = (
    0, -1, -2, -3, -4, -5, -6, -7)
CT_NONE, CT_RCT, CT_YCOCG = 0, 1, 2


class TileDesc(ctypes.Structure):
    _fields_ = [("pixel_offset", ctypes.c_uint64), ("width", ctypes.c_uint32),
                ("height", ctypes.c_uint32), ("row_stride_bytes", ctypes.c_uint32),
                ("channels", ctypes.c_uint8), ("bytes_per_sample", ctypes.c_uint8),
                ("bits", ctypes.c_uint8), ("levels", ctypes.c_uint8),
                ("colour_transform", ctypes.c_uint8), ("reserved0", ctypes.c_uint8 * 3),
                ("qstep", ctypes.c_uint16), ("reserved1", ctypes.c_uint16)]


class DecodeJob(ctypes.Structure):
    _fields_ = [("tile", TileDesc), ("in_offset", ctypes.c_uint64), ("in_bytes", ctypes.c_uint64),
                ("out_offset", ctypes.c_uint64), ("out_row_stride_bytes", ctypes.c_uint32),
                ("target_level", ctypes.c_uint8), ("drop_bitplanes", ctypes.c_uint8),
                ("reserved", ctypes.c_uint16)]


class RegionJob(ctypes.Structure):
    _fields_ = [("job", DecodeJob), ("x0", ctypes.c_uint32), ("y0", ctypes.c_uint32),
                ("width", ctypes.c_uint32), ("height", ctypes.c_uint32),
                ("h_block_offsets", ctypes.c_void_p)]


class Tuning(ctypes.Structure):
    _fields_ = [("transform_tile", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("seg_waves_per_cu", ctypes.c_int32), ("seg_wave_group", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 4)]


def tuning(transform_tile=0, blocks_per_cu=0, seg_waves_per_cu=0, seg_wave_group=0) -> Tuning:
    t = Tuning()
    t.transform_tile, t.blocks_per_cu = int(transform_tile), int(blocks_per_cu)
    t.seg_waves_per_cu, t.seg_wave_group = int(seg_waves_per_cu), int(seg_wave_group)
    return t


assert ctypes.sizeof(TileDesc) == 32 and ctypes.sizeof(DecodeJob) == 64 and ctypes.sizeof(RegionJob) == 88

_lib = None


class IsxError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        super().__init__(f"{what}: {status_string(code)} ({code})" if _lib else f"{what}: {code}")
        self.code = code


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libisx.so not built ({LIB_PATH}); run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        P, u64, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int32
        sig = {
            "isx_max_encoded_bytes": (u64, [P, i32]),
            "isx_encode_workspace_bytes": (u64, [P, i32]),
            "isx_decode_workspace_bytes": (u64, [P, i32]),
            "isx_tile_block_count": (ctypes.c_int64, [P]),
            "isx_encode_tiles": (i32, [P, i32, P, P, u64, P, P, P, P, u64, P]),
            "isx_decode_tiles": (i32, [P, P, i32, P, P, P, u64, P]),
            "isx_encode_plan_bytes": (u64, [P, i32]),
            "isx_encode_plan_build": (i32, [P, i32, P, u64]),
            "isx_encode_run": (i32, [P, P, P, P, u64, P, P, P, P, u64, P]),
            "isx_decode_plan_bytes": (u64, [P, i32]),
            "isx_decode_plan_build": (i32, [P, i32, P, u64]),
            "isx_decode_run": (i32, [P, P, P, P, P, P, u64, P]),
            "isx_status_string": (ctypes.c_char_p, [i32]),
            "isx_debug_forward": (i32, [P, P, P, P, u64, P]),
            "isx_debug_huffman": (i32, [P, i32, P, P]),
            "isx_stage_count": (i32, [i32]),
            "isx_stage_name": (ctypes.c_char_p, [i32, i32]),
            "isx_encode_run_stages": (i32, [P, P, P, P, u64, P, P, P, P, u64, P, i32, i32]),
            "isx_decode_run_stages": (i32, [P, P, P, P, P, P, u64, P, i32, i32]),
            "isx_encode_plan_build_tuned": (i32, [P, i32, P, P, u64]),
            "isx_decode_plan_build_tuned": (i32, [P, i32, P, P, u64]),
            "isx_stream_block_offsets": (i32, [P, u64, P, u64]),
            "isx_region_workspace_bytes": (u64, [P, i32]),
            "isx_region_plan_bytes": (u64, [P, i32]),
            "isx_region_plan_build": (i32, [P, i32, P, P, u64]),
            "isx_decode_regions": (i32, [P, P, i32, P, P, P, u64, P]),
            "isx_read_tile_header": (i32, [P, u64, P]),
            "isx_decode_run_noalloc": (i32, [P, P, P, P, P, P]),
            "isx_plan_info": (i32, [P, P, P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


EXPORTS = ["isx_max_encoded_bytes", "isx_encode_workspace_bytes", "isx_decode_workspace_bytes",
           "isx_tile_block_count", "isx_encode_tiles", "isx_decode_tiles", "isx_encode_plan_bytes",
           "isx_encode_plan_build", "isx_encode_run", "isx_decode_plan_bytes",
           "isx_decode_plan_build", "isx_decode_run", "isx_status_string", "isx_debug_forward",
           "isx_debug_huffman", "isx_stage_count", "isx_stage_name", "isx_encode_run_stages",
           "isx_decode_run_stages", "isx_encode_plan_build_tuned", "isx_decode_plan_build_tuned",
           "isx_stream_block_offsets", "isx_region_workspace_bytes", "isx_region_plan_bytes",
           "isx_region_plan_build", "isx_decode_regions", "isx_read_tile_header",
           "isx_decode_run_noalloc", "isx_plan_info"]

NOALLOC_SCRATCH_BYTES = 64 << 20  # ISX_NOALLOC_SCRATCH_BYTES


def status_string(code: int) -> str:
    return lib().isx_status_string(int(code)).decode()


def _check(rc: int, what: str):
    if rc != OK:
        raise IsxError(rc, what)


def _torch():
    import torch
    return torch


def _stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def tile_desc(width, height, channels, bytes_per_sample, bits, levels, ct=None, qstep=1,
              pixel_offset=0, row_stride=None) -> TileDesc:
    d = TileDesc()
    d.pixel_offset = pixel_offset
    d.width, d.height = width, height
    d.row_stride_bytes = row_stride if row_stride is not None else width * channels * bytes_per_sample
    d.channels, d.bytes_per_sample, d.bits, d.levels = channels, bytes_per_sample, bits, levels
    d.colour_transform = (CT_RCT if channels == 3 else CT_NONE) if ct is None else ct
    d.qstep = qstep
    return d


def desc_array(descs):
    arr = (TileDesc * len(descs))()
    for i, d in enumerate(descs):
        arr[i] = d
    return arr


def block_count(desc: TileDesc) -> int:
    return int(lib().isx_tile_block_count(ctypes.byref(desc)))


class Encoder:
    """Encoder for a fixed batch of tile shapes: plan built and uploaded once,
    workspace and output arena allocated once (torch, on `device`)."""

    def __init__(self, descs, device="cuda", tune=None):
        torch = _torch()
        L = lib()
        self.n = len(descs)
        self.descs = desc_array(descs)
        pb = L.isx_encode_plan_bytes(self.descs, self.n)
        if pb == 0:
            raise IsxError(E_INVALID_ARG, "encode plan")
        self.h_plan = (ctypes.c_uint8 * pb)()
        self.tune = tune if tune is not None else tuning()
        _check(L.isx_encode_plan_build_tuned(self.descs, self.n, ctypes.byref(self.tune), self.h_plan,
                                             pb), "encode plan")
        self.graph = None
        self.d_plan = torch.frombuffer(bytearray(self.h_plan), dtype=torch.uint8).to(device)
        self.ws_bytes = int(L.isx_encode_workspace_bytes(self.descs, self.n))
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)
        self.capacity = int(L.isx_max_encoded_bytes(self.descs, self.n))
        self.out = torch.empty(self.capacity, dtype=torch.uint8, device=device)
        self.offsets = torch.zeros(self.n, dtype=torch.int64, device=device)
        self.sizes = torch.zeros(self.n, dtype=torch.int64, device=device)
        self.status = torch.full((self.n,), 1, dtype=torch.int32, device=device)

    def run(self, d_pixels, stream=None):
        """Enqueue the encode of the batch read from the uint8 device tensor d_pixels."""
        rc = lib().isx_encode_run(self.h_plan, _ptr(self.d_plan), _ptr(d_pixels), _ptr(self.out),
                                  self.capacity, _ptr(self.offsets), _ptr(self.sizes),
                                  _ptr(self.status), _ptr(self.ws), self.ws_bytes,
                                  _stream_ptr(stream))
        _check(rc, "isx_encode_run")

    def run_stages(self, d_pixels, first, count, stream=None):
        rc = lib().isx_encode_run_stages(self.h_plan, _ptr(self.d_plan), _ptr(d_pixels),
                                         _ptr(self.out), self.capacity, _ptr(self.offsets),
                                         _ptr(self.sizes), _ptr(self.status), _ptr(self.ws),
                                         self.ws_bytes, _stream_ptr(stream), first, count)
        _check(rc, "isx_encode_run_stages")

    def capture(self, d_pixels):
        """Capture one full encode of d_pixels into a HIP graph (replayed by replay())."""
        self.graph = _capture(lambda: self.run(d_pixels))

    def replay(self):
        self.graph.replay()

    def streams(self):
        """Host copies of the encoded tiles (after the stream has completed)."""
        st = self.status.cpu().numpy()
        off = self.offsets.cpu().numpy()
        sz = self.sizes.cpu().numpy()
        total = int(off[-1] + sz[-1]) if self.n else 0
        host = self.out[:total].cpu().numpy()
        res = []
        for i in range(self.n):
            if st[i] != OK:
                raise IsxError(int(st[i]), f"tile {i}")
            res.append(host[off[i]:off[i] + sz[i]].tobytes())
        return res


class Decoder:
    """Decoder for a fixed list of jobs (plan uploaded once): whole-tile
    DecodeJobs, or RegionJobs (their block-offset arrays must stay alive
    until the constructor returns)."""

    def __init__(self, jobs, out_bytes, device="cuda", tune=None, out=None):
        torch = _torch()
        L = lib()
        self.n = len(jobs)
        regions = self.n > 0 and isinstance(jobs[0], RegionJob)
        self.jobs = ((RegionJob if regions else DecodeJob) * self.n)()
        for i, j in enumerate(jobs):
            self.jobs[i] = j
        self.tune = tune if tune is not None else tuning()
        if regions:
            pb = L.isx_region_plan_bytes(self.jobs, self.n)
            if pb == 0:
                raise IsxError(E_INVALID_ARG, "region plan")
            self.h_plan = (ctypes.c_uint8 * pb)()
            _check(L.isx_region_plan_build(self.jobs, self.n, ctypes.byref(self.tune), self.h_plan, pb),
                   "region plan")
            self.ws_bytes = int(L.isx_region_workspace_bytes(self.jobs, self.n))
        else:
            pb = L.isx_decode_plan_bytes(self.jobs, self.n)
            if pb == 0:
                raise IsxError(E_INVALID_ARG, "decode plan")
            self.h_plan = (ctypes.c_uint8 * pb)()
            _check(L.isx_decode_plan_build_tuned(self.jobs, self.n, ctypes.byref(self.tune), self.h_plan,
                                                 pb), "decode plan")
            self.ws_bytes = int(L.isx_decode_workspace_bytes(self.jobs, self.n))
        self.graph = None
        self.d_plan = torch.frombuffer(bytearray(self.h_plan), dtype=torch.uint8).to(device)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)
        self.out = out if out is not None else torch.zeros(max(1, out_bytes), dtype=torch.uint8,
                                                           device=device)
        self.status = torch.full((self.n,), 1, dtype=torch.int32, device=device)

    def run(self, d_encoded, stream=None):
        rc = lib().isx_decode_run(self.h_plan, _ptr(self.d_plan), _ptr(d_encoded), _ptr(self.out),
                                  _ptr(self.status), _ptr(self.ws), self.ws_bytes,
                                  _stream_ptr(stream))
        _check(rc, "isx_decode_run")

    def run_noalloc(self, d_encoded, stream=None):
        """The same decode through isx_decode_run_noalloc: the library's fixed
        device workspace instead of self.ws (returns the library's status)."""
        return int(lib().isx_decode_run_noalloc(self.h_plan, _ptr(self.d_plan), _ptr(d_encoded),
                                                _ptr(self.out), _ptr(self.status), _stream_ptr(stream)))

    def run_stages(self, d_encoded, first, count, stream=None):
        rc = lib().isx_decode_run_stages(self.h_plan, _ptr(self.d_plan), _ptr(d_encoded),
                                         _ptr(self.out), _ptr(self.status), _ptr(self.ws),
                                         self.ws_bytes, _stream_ptr(stream), first, count)
        _check(rc, "isx_decode_run_stages")

    def capture(self, d_encoded):
        """Capture one full decode of d_encoded into a HIP graph."""
        self.graph = _capture(lambda: self.run(d_encoded))

    def replay(self):
        self.graph.replay()


_capture_stream = None


def _capture(fn):
    """Record the kernels `fn` enqueues into a torch CUDA(HIP) graph.  The
    library enqueues kernels only (no copies, no memsets) on the current
    stream, which torch points at its capture stream (one side stream for
    every capture of the process)."""
    global _capture_stream
    torch = _torch()
    if _capture_stream is None:
        _capture_stream = torch.cuda.Stream()
    s = _capture_stream
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fn()  # warm-up outside the graph
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    return g


def stage_names(mode):
    L = lib()
    return [L.isx_stage_name(mode, i).decode() for i in range(L.isx_stage_count(mode))]


def out_size(w, h, level):
    for _ in range(level):
        w, h = (w + 1) // 2, (h + 1) // 2
    return w, h


# ------------------------------------------------------------------ convenience
def _as_device_pixels(img: np.ndarray, device="cuda"):
    torch = _torch()
    a = np.ascontiguousarray(img)
    if a.ndim == 2:
        a = a[:, :, None]
    return torch.from_numpy(a.view(np.uint8).reshape(-1).copy()).to(device), a


def encode_image(img: np.ndarray, levels: int, bits=None, ct=None, qstep=1, device="cuda") -> bytes:
    """Encode one image (numpy, HxW[xC], uint8/uint16/uint32) on the GPU; returns the
    tile stream.  uint32 samples need an explicit ``bits`` (at most 24)."""
    torch = _torch()
    d_pix, a = _as_device_pixels(img, device)
    h, w, c = a.shape
    bps = a.itemsize
    d = tile_desc(w, h, c, bps, bits or 8 * bps, levels, ct=ct, qstep=qstep)
    enc = Encoder([d], device)
    enc.run(d_pix)
    torch.cuda.synchronize()
    return enc.streams()[0]


def encode_images(imgs, levels, qsteps=None, device="cuda", bits=None):
    """Encode a batch of images in one call (one plan, one launch sequence)."""
    torch = _torch()
    descs, chunks, off = [], [], 0
    for i, img in enumerate(imgs):
        a = np.ascontiguousarray(img)
        if a.ndim == 2:
            a = a[:, :, None]
        h, w, c = a.shape
        bps = a.itemsize
        lv = levels[i] if isinstance(levels, (list, tuple)) else levels
        q = qsteps[i] if qsteps is not None else 1
        descs.append(tile_desc(w, h, c, bps, bits or 8 * bps, lv, qstep=q, pixel_offset=off))
        b = a.view(np.uint8).reshape(-1)
        chunks.append(b)
        off += len(b)
        pad = (-off) % 16
        if pad:
            chunks.append(np.zeros(pad, np.uint8))
            off += pad
    d_pix = torch.from_numpy(np.concatenate(chunks)).to(device)
    enc = Encoder(descs, device)
    enc.run(d_pix)
    torch.cuda.synchronize()
    return enc.streams()


def read_tile_header(blob: bytes) -> TileDesc:
    """Tile parameters of an encoded stream (the library's host parser of its
    24-byte header)."""
    d = TileDesc()
    head = np.frombuffer(blob[:24], np.uint8)
    _check(lib().isx_read_tile_header(head.ctypes.data_as(ctypes.c_void_p), len(head), ctypes.byref(d)),
           "isx_read_tile_header")
    return d


_parse_header = read_tile_header


def encode_tiles(d_pixels, descs, d_out, d_offsets, d_sizes, d_status, d_ws, stream=None) -> int:
    """One isx_encode_tiles call (plan built and copied by the library) on
    caller-owned torch device buffers; returns the library's status."""
    arr = desc_array(descs)
    return int(lib().isx_encode_tiles(arr, len(descs), _ptr(d_pixels), _ptr(d_out), d_out.numel(),
                                      _ptr(d_offsets), _ptr(d_sizes), _ptr(d_status), _ptr(d_ws),
                                      d_ws.numel(), _stream_ptr(stream)))


def decode_tiles(d_encoded, jobs, d_out, d_status, d_ws, stream=None) -> int:
    """One isx_decode_tiles call on caller-owned torch device buffers."""
    arr = (DecodeJob * len(jobs))()
    for i, j in enumerate(jobs):
        arr[i] = j
    return int(lib().isx_decode_tiles(_ptr(d_encoded), arr, len(jobs), _ptr(d_out), _ptr(d_status),
                                      _ptr(d_ws), d_ws.numel(), _stream_ptr(stream)))


def encode_workspace_bytes(descs) -> int:
    return int(lib().isx_encode_workspace_bytes(desc_array(descs), len(descs)))


def decode_workspace_bytes(jobs) -> int:
    arr = (DecodeJob * len(jobs))()
    for i, j in enumerate(jobs):
        arr[i] = j
    return int(lib().isx_decode_workspace_bytes(arr, len(jobs)))


def max_encoded_bytes(descs) -> int:
    return int(lib().isx_max_encoded_bytes(desc_array(descs), len(descs)))


def decode_streams(blobs, levels=None, device="cuda", return_status=False, drop=None):
    """Decode a batch of tile streams on the GPU (one call); returns numpy images.
    `levels` / `drop`: one value, or one per stream (resolution level z and
    magnitude planes left out)."""
    torch = _torch()
    jobs, outs, in_off, out_off = [], [], 0, 0
    parts = []
    for i, blob in enumerate(blobs):
        d = _parse_header(blob)
        z = 0 if levels is None else (levels[i] if isinstance(levels, (list, tuple)) else levels)
        ow, oh = out_size(d.width, d.height, z)
        j = DecodeJob()
        j.tile = d
        j.in_offset, j.in_bytes = in_off, len(blob)
        j.out_offset = out_off
        j.out_row_stride_bytes = ow * d.channels * d.bytes_per_sample
        j.target_level = z
        if drop is not None:
            j.drop_bitplanes = drop[i] if isinstance(drop, (list, tuple)) else drop
        jobs.append(j)
        outs.append((out_off, oh, ow, d.channels, d.bytes_per_sample))
        parts.append(np.frombuffer(blob, np.uint8))
        in_off += len(blob)
        pad = (-in_off) % 256
        if pad:
            parts.append(np.zeros(pad, np.uint8))
            in_off += pad
        out_off += oh * ow * d.channels * d.bytes_per_sample
        out_off += (-out_off) % 16
    d_enc = torch.from_numpy(np.concatenate(parts)).to(device)
    dec = Decoder(jobs, out_off, device)
    dec.run(d_enc)
    torch.cuda.synchronize()
    host = dec.out.cpu().numpy()
    st = dec.status.cpu().numpy()
    res = []
    for (o, oh, ow, c, bps), s in zip(outs, st):
        n = oh * ow * c * bps
        a = host[o:o + n].view({1: np.uint8, 2: np.uint16, 4: np.uint32}[bps]).reshape(oh, ow, c)
        res.append(a.copy())
    if return_status:
        return res, [int(x) for x in st]
    for i, s in enumerate(st):
        if s != OK:
            raise IsxError(int(s), f"decode job {i}")
    return res


def stream_block_offsets(head: bytes) -> np.ndarray:
    """Byte offset of every block of a stream, then its length (uint64), from
    the stream's first 24 + 4 * blocks bytes (the library's host parser)."""
    import struct
    if len(head) < 24:
        raise IsxError(E_TRUNCATED, "stream head")
    nb = struct.unpack_from("<I", head, 20)[0]
    out = np.zeros(nb + 1, dtype=np.uint64)
    buf = np.frombuffer(head, np.uint8)
    _check(lib().isx_stream_block_offsets(buf.ctypes.data_as(ctypes.c_void_p), len(head),
                                          out.ctypes.data_as(ctypes.c_void_p), nb + 1),
           "isx_stream_block_offsets")
    return out


def region_job(desc: TileDesc, offsets: np.ndarray, level, x0, y0, w, h, in_offset=0, in_bytes=None,
               out_offset=0, drop=0) -> RegionJob:
    """Region [x0, x0+w) x [y0, y0+h) of the level-`level` image of one stream."""
    r = RegionJob()
    r.job.tile = desc
    r.job.in_offset = in_offset
    r.job.in_bytes = int(offsets[-1]) if in_bytes is None else in_bytes
    r.job.out_offset = out_offset
    r.job.out_row_stride_bytes = w * desc.channels * desc.bytes_per_sample
    r.job.target_level, r.job.drop_bitplanes = level, drop
    r.x0, r.y0, r.width, r.height = x0, y0, w, h
    r.h_block_offsets = offsets.ctypes.data
    return r


def decode_regions(blob: bytes, regions, device="cuda", return_status=False):
    """Decode regions (level, x0, y0, w, h[, drop]) of one stream in one call;
    returns numpy images."""
    torch = _torch()
    d = _parse_header(blob)
    offs = stream_block_offsets(blob[:24 + 4 * struct_u32(blob, 20)])
    jobs, outs, off = [], [], 0
    bps = d.bytes_per_sample
    for reg in regions:
        z, x0, y0, w, h = reg[:5]
        drop = reg[5] if len(reg) > 5 else 0
        jobs.append(region_job(d, offs, z, x0, y0, w, h, in_bytes=len(blob), out_offset=off, drop=drop))
        outs.append((off, h, w))
        off += h * w * d.channels * bps
        off += (-off) % 16
    d_enc = torch.from_numpy(np.frombuffer(blob, np.uint8).copy()).to(device)
    dec = Decoder(jobs, off, device)
    dec.run(d_enc)
    torch.cuda.synchronize()
    host = dec.out.cpu().numpy()
    st = [int(x) for x in dec.status.cpu().numpy()]
    dt = {1: np.uint8, 2: np.uint16, 4: np.uint32}[bps]
    res = [host[o:o + h * w * d.channels * bps].view(dt).reshape(h, w, d.channels).copy() for o, h, w in outs]
    if return_status:
        return res, st
    for i, s in enumerate(st):
        if s != OK:
            raise IsxError(s, f"region job {i}")
    return res


def struct_u32(blob: bytes, off: int) -> int:
    return int.from_bytes(blob[off:off + 4], "little")


def debug_forward(img: np.ndarray, levels, bits=None, ct=None, qstep=1, device="cuda"):
    """Quantised coefficient bands per channel, as the GPU forward transform wrote them."""
    torch = _torch()
    d_pix, a = _as_device_pixels(img, device)
    h, w, c = a.shape
    bps = a.itemsize
    d = tile_desc(w, h, c, bps, bits or 8 * bps, levels, ct=ct, qstep=qstep)
    L = lib()
    ws_bytes = int(L.isx_encode_workspace_bytes(ctypes.byref(d), 1))
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=device)
    coeffs = torch.zeros(w * h * c + 16, dtype=torch.int32, device=device)
    _check(L.isx_debug_forward(ctypes.byref(d), _ptr(d_pix), _ptr(coeffs), _ptr(ws), ws_bytes,
                               _stream_ptr()), "isx_debug_forward")
    torch.cuda.synchronize()
    flat = coeffs.cpu().numpy()
    sizes = []
    cw, ch = w, h
    for _ in range(levels):
        sizes.append((cw, ch))
        cw, ch = (cw + 1) // 2, (ch + 1) // 2
    res, k = [], 0
    for _ in range(c):
        dd = {"LL": flat[k:k + cw * ch].reshape(ch, cw).copy(), "HL": [None] * (levels + 1),
              "LH": [None] * (levels + 1), "HH": [None] * (levels + 1)}
        k += cw * ch
        for lv in range(levels, 0, -1):
            pw, ph = sizes[lv - 1]
            for name, (bw, bh) in (("HL", (pw // 2, (ph + 1) // 2)), ("LH", ((pw + 1) // 2, ph // 2)),
                                   ("HH", (pw // 2, ph // 2))):
                dd[name][lv] = flat[k:k + bw * bh].reshape(bh, bw).copy()
                k += bw * bh
        res.append(dd)
    return res


def debug_huffman(freq, limit=0, device="cuda"):
    torch = _torch()
    f = torch.tensor(np.asarray(freq, dtype=np.uint32).astype(np.int64), dtype=torch.int32,
                     device=device)
    out = torch.zeros(256, dtype=torch.uint8, device=device)
    _check(lib().isx_debug_huffman(_ptr(f), int(limit), _ptr(out), _stream_ptr()),
           "isx_debug_huffman")
    torch.cuda.synchronize()
    return out.cpu().numpy()
