"""Autotuner for the batched encode/decode launches.

Searches the launch parameters of a plan (isx_tuning: LDS transform-tile
shape, persistent workgroups per CU for the per-block kernels, the segment
decoder's waves per workgroup and, in its one-wave form, waves per CU) by timing
real runs of the caller's batch with HIP events, checks that every candidate
produces byte-identical streams and identical pixels, and caches the winner
in a JSON file keyed by the GPU architecture and a summary of the batch.
"""
from __future__ import annotations

import json
import os

import numpy as np

from . import isx

# (transform tile, blocks per CU, segment-decoder waves per CU, segment-decoder
# waves per workgroup; 0 = default)
CANDIDATES = [(32, 0, 0, 0), (16, 0, 0, 0), (32, 2, 0, 0), (32, 4, 0, 0), (32, 8, 0, 0), (16, 4, 0, 0),
              (16, 8, 0, 0), (32, 0, 0, 1), (32, 0, 8, 1), (32, 0, 0, 4)]


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
    """Returns {'encode': (tq, bpc, swpc, swg), 'decode': (tq, bpc, swpc, swg), 'timings': {...}}."""
    import torch
    key = batch_key(descs)
    cache = _load() if use_cache else {}
    if key in cache:
        return cache[key]
    ref_streams, ref_pixels = None, None
    enc_t, dec_t = {}, {}
    for cand in candidates:
        cand = tuple(cand) + (0,) * (4 - len(cand))
        tq, bpc, swpc, swg = cand
        t = isx.tuning(tq, bpc, swpc, swg)
        enc = isx.Encoder(descs, tune=t)
        enc.run(d_pixels)
        torch.cuda.synchronize()
        streams = enc.streams()
        if ref_streams is None:
            ref_streams = streams
        elif streams != ref_streams:
            raise RuntimeError(f"tuning {cand} changed the encoded bytes")
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
            raise RuntimeError(f"tuning {cand} changed the decoded pixels")
        enc_t[cand] = _time(lambda: enc.run(d_pixels), reps)
        dec_t[cand] = _time(lambda: dec.run(enc.out), reps)
        if log:
            log(f"[tune] tq={tq} bpc={bpc} swpc={swpc} swg={swg} encode {enc_t[cand]:.3f} ms decode {dec_t[cand]:.3f} ms")
        del enc, dec
    best_e = min(enc_t, key=enc_t.get)
    best_d = min(dec_t, key=dec_t.get)
    res = {"encode": list(best_e), "decode": list(best_d),
           "timings_ms": {"/".join(str(x) for x in k): [round(enc_t[k], 4), round(dec_t[k], 4)] for k in enc_t}}
    if use_cache:
        cache[key] = res
        _store(cache)
    return res
