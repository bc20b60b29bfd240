"""Autotuner for the batched encode/decode launches.

Searches the launch parameters of a plan (isx_tuning: LDS transform-tile
shape and persistent workgroups per CU for the per-block kernels) by timing
real runs of the caller's batch with HIP events, checks that every candidate
produces byte-identical streams and identical pixels, and caches the winner
in a JSON file keyed by the GPU architecture and a summary of the batch.
"""
from __future__ import annotations

import json
import os

import numpy as np

from . import isx

CANDIDATES = [(32, 0), (16, 0), (32, 2), (32, 4), (32, 8), (16, 4), (16, 8)]


def cache_path() -> str:
    return os.environ.get("ISX_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "isx", "tune.json"))


def batch_key(descs) -> str:
    """Arch + a coarse summary of the batch (tile-size class, levels, bits)."""
    import torch
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    sides = np.array([max(d.width, d.height) for d in descs])
    cls = ",".join(str(int(x)) for x in np.percentile(sides, [10, 50, 90]).round(-1))
    lv = ",".join(str(x) for x in sorted({d.levels for d in descs}))
    bits = ",".join(str(x) for x in sorted({d.bits for d in descs}))
    nb = int(np.log2(max(1, len(descs))))
    return f"{arch}|n2^{nb}|side[{cls}]|lv[{lv}]|bits[{bits}]"


def _load():
    p = cache_path()
    if os.path.exists(p):
        with open(p) as f:
            return json.load(f)
    return {}


def _store(c):
    p = cache_path()
    os.makedirs(os.path.dirname(p), exist_ok=True)
    tmp = p + ".tmp"
    with open(tmp, "w") as f:
        json.dump(c, f, indent=1, sort_keys=True)
    os.replace(tmp, p)


def _time(fn, reps):
    import torch
    fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def tune(descs, d_pixels, reps: int = 3, candidates=CANDIDATES, use_cache: bool = True, log=None):
    """Returns {'encode': (tq, bpc), 'decode': (tq, bpc), 'timings': {...}}."""
    import torch
    key = batch_key(descs)
    cache = _load() if use_cache else {}
    if key in cache:
        return cache[key]
    ref_streams, ref_pixels = None, None
    enc_t, dec_t = {}, {}
    for tq, bpc in candidates:
        t = isx.tuning(tq, bpc)
        enc = isx.Encoder(descs, tune=t)
        enc.run(d_pixels)
        torch.cuda.synchronize()
        streams = enc.streams()
        if ref_streams is None:
            ref_streams = streams
        elif streams != ref_streams:
            raise RuntimeError(f"tuning {tq, bpc} changed the encoded bytes")
        jobs, out_off = [], 0
        offs = enc.offsets.cpu().numpy()
        for i, d in enumerate(descs):
            j = isx.DecodeJob()
            j.tile = d
            j.in_offset, j.in_bytes = int(offs[i]), len(streams[i])
            j.out_offset = out_off
            j.out_row_stride_bytes = d.width * d.channels * d.bytes_per_sample
            j.target_level = 0
            jobs.append(j)
            out_off += d.width * d.height * d.channels * d.bytes_per_sample
        dec = isx.Decoder(jobs, out_off, tune=t)
        dec.run(enc.out)
        torch.cuda.synchronize()
        if int(dec.status.abs().sum().item()) != 0:
            raise RuntimeError("decode failed during tuning")
        px = dec.out[:out_off].clone()
        if ref_pixels is None:
            ref_pixels = px
        elif not torch.equal(px, ref_pixels):
            raise RuntimeError(f"tuning {tq, bpc} changed the decoded pixels")
        enc_t[(tq, bpc)] = _time(lambda: enc.run(d_pixels), reps)
        dec_t[(tq, bpc)] = _time(lambda: dec.run(enc.out), reps)
        if log:
            log(f"[tune] tq={tq} bpc={bpc} encode {enc_t[(tq, bpc)]:.3f} ms decode {dec_t[(tq, bpc)]:.3f} ms")
        del enc, dec
    best_e = min(enc_t, key=enc_t.get)
    best_d = min(dec_t, key=dec_t.get)
    res = {"encode": list(best_e), "decode": list(best_d),
           "timings_ms": {f"{k[0]}/{k[1]}": [round(enc_t[k], 4), round(dec_t[k], 4)] for k in enc_t}}
    if use_cache:
        cache[key] = res
        _store(cache)
    return res
