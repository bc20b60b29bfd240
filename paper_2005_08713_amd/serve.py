"""Tile-decode serving with continuous batching over an HBM-resident slide.

Two layouts of the same slide:

* ``Slide``: cut into square tiles, each encoded on its own (Sec. 4: separate
  blocks per scale let any tile be decoded at any resolution level).  A
  request (z, X, Y) for the 512x512 view at zoom z decodes the 2^z x 2^z
  source tiles (X 2^z + i, Y 2^z + j), each to level z (only its coarser
  blocks), straight into its place in the request's output buffer.
* ``PyramidSlide``: the whole slide as ONE stream, one non-redundant wavelet
  pyramid (or, beyond 65535 pixels a side, a grid of such streams).  The same
  request is one region job per stream it touches: the 512x512 window
  [512 X, 512 X + 512) x [512 Y, 512 Y + 512) of the level-z image, decoded
  from the blocks under its halo at levels z+1 .. L only.

The server loop admits arrived requests into a free batch slot as long as the
slot's workspace and output memory allow, launches the whole batch as one
isx_decode_run on the slot's stream, and keeps going while earlier batches
run; completed batches release their slot.  Latency = completion - arrival.
"""
from __future__ import annotations

import ctypes
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import isx


@dataclass
class Request:
    rid: int
    z: int
    X: int
    Y: int
    arrival: float = 0.0
    done: float = -1.0
    slot: int = -1
    out_off: int = 0


class Slide:
    """Encoded tiles of a slide, resident in HBM, with a host index."""

    def __init__(self, tiles_x, tiles_y, tile=512, levels=6, seed=501, batch=256, device="cuda",
                 log=None):
        import torch
        from .synth import SlideGen
        self.tx, self.ty, self.tile, self.levels = tiles_x, tiles_y, tile, levels
        self.n = tiles_x * tiles_y
        gen = SlideGen(tiles_x, tiles_y, tile, seed, device)
        self.gen = gen
        desc = [isx.tile_desc(tile, tile, 3, 1, 8, levels, pixel_offset=i * tile * tile * 3)
                for i in range(batch)]
        enc = isx.Encoder(desc, device)
        parts, self.offsets, self.sizes = [], np.zeros(self.n, np.int64), np.zeros(self.n, np.int64)
        total = 0
        t0 = time.perf_counter()
        for b0 in range(0, self.n, batch):
            ids = list(range(b0, min(self.n, b0 + batch)))
            px = gen.tiles(ids, b0 // batch)
            if len(ids) < batch:
                pad = torch.zeros((batch - len(ids),) + px.shape[1:], dtype=px.dtype, device=device)
                px = torch.cat([px, pad])
            enc.run(px.reshape(-1))
            torch.cuda.synchronize()
            st = enc.status.cpu().numpy()
            if (st[:len(ids)] != 0).any():
                raise RuntimeError("slide encode failed")
            off = enc.offsets.cpu().numpy()
            sz = enc.sizes.cpu().numpy()
            end = int(off[len(ids) - 1] + sz[len(ids) - 1])
            parts.append(enc.out[:end].clone())
            for k, i in enumerate(ids):
                self.offsets[i] = total + off[k]
                self.sizes[i] = sz[k]
            total += (end + 255) // 256 * 256
            if parts[-1].numel() % 256:
                parts.append(torch.zeros(256 - parts[-1].numel() % 256, dtype=torch.uint8, device=device))
            if log and (b0 // batch) % 16 == 0:
                log(f"[slide] encoded {min(self.n, b0 + batch)}/{self.n} tiles, {total / 1e9:.2f} GB")
        self.arena = torch.cat(parts)
        self.encode_s = time.perf_counter() - t0
        self.raw_bytes = self.n * tile * tile * 3
        self.desc = isx.tile_desc(tile, tile, 3, 1, 8, levels)

    def sources(self, z, X, Y):
        """Source tiles of request (z, X, Y): list of (tile id, i, j)."""
        s = 1 << z
        out = []
        for j in range(s):
            for i in range(s):
                tx, ty = X * s + i, Y * s + j
                if tx < self.tx and ty < self.ty:
                    out.append((ty * self.tx + tx, i, j))
        return out

    def grid(self, z):
        s = 1 << z
        return -(-self.tx // s), -(-self.ty // s)

    def source_arrays(self, z, X, Y):
        """Vectorised sources(): (tile ids, i, j) arrays."""
        s = 1 << z
        jj, ii = np.divmod(np.arange(s * s), s)
        tx, ty = X * s + ii, Y * s + jj
        ok = (tx < self.tx) & (ty < self.ty)
        return (ty * self.tx + tx)[ok], ii[ok], jj[ok]

    def source_count(self, z, X, Y):
        s = 1 << z
        return max(0, min(s, self.tx - X * s)) * max(0, min(s, self.ty - Y * s))


class PyramidSlide:
    """The slide of ``Slide`` (same generator, seed and tile batches, so the
    same pixels) encoded as non-redundant wavelet pyramids: one stream for the
    whole slide, or a grid of streams of `sub` = (sx, sy) tiles each when the
    slide is larger than one stream allows (65535 pixels a side).  The level-z
    slide image is the sub-pyramids' level-z images side by side (every
    sub-pyramid but the last of a row or column spans a multiple of 2^levels
    pixels).  Host index per stream: the byte offset of every block (from
    its size table)."""

    def __init__(self, tiles_x, tiles_y, tile=512, levels=6, seed=501, batch=256, device="cuda", log=None,
                 sub=None, keep_image=None):
        import torch
        from .synth import SlideGen
        self.tx, self.ty, self.tile, self.levels = tiles_x, tiles_y, tile, levels
        self.n = tiles_x * tiles_y
        W, H = tiles_x * tile, tiles_y * tile
        self.W, self.H = W, H
        sx, sy = sub if sub else (tiles_x, tiles_y)
        if (sx * tile) % (1 << levels) or (sy * tile) % (1 << levels):
            raise ValueError("sub-pyramid sides must be multiples of 2^levels")
        self.sx, self.sy = sx, sy
        self.gx, self.gy = -(-tiles_x // sx), -(-tiles_y // sy)
        if keep_image is None:
            keep_image = self.gx * self.gy == 1
        gen = SlideGen(tiles_x, tiles_y, tile, seed, device)
        self.gen = gen
        t0 = time.perf_counter()
        imgs = []
        for j in range(self.gy):
            for i in range(self.gx):
                w = (min(tiles_x, (i + 1) * sx) - i * sx) * tile
                h = (min(tiles_y, (j + 1) * sy) - j * sy) * tile
                imgs.append(torch.empty((h, w, 3), dtype=torch.uint8, device=device))
        for b0 in range(0, self.n, batch):
            ids = list(range(b0, min(self.n, b0 + batch)))
            px = gen.tiles(ids, b0 // batch)
            for k, t in enumerate(ids):
                X, Y = t % tiles_x, t // tiles_x
                im = imgs[(Y // sy) * self.gx + X // sx]
                x, y = (X % sx) * tile, (Y % sy) * tile
                im[y:y + tile, x:x + tile] = px[k]
        torch.cuda.synchronize()
        self.descs, self.offs, self.sizes, self.block_offsets = [], [], [], []
        parts, total = [], 0
        self.encode_only_s = 0.0
        for k, im in enumerate(imgs):
            h, w = im.shape[:2]
            d = isx.tile_desc(w, h, 3, 1, 8, levels)
            enc = isx.Encoder([d], device)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            enc.run(im.reshape(-1))
            torch.cuda.synchronize()
            self.encode_only_s += time.perf_counter() - t1
            if int(enc.status[0]) != 0:
                raise RuntimeError("pyramid encode failed")
            size = int(enc.sizes[0])
            blob = enc.out[int(enc.offsets[0]):int(enc.offsets[0]) + size].clone()
            del enc
            nb = int.from_bytes(blob[20:24].cpu().numpy().tobytes(), "little")
            self.block_offsets.append(isx.stream_block_offsets(blob[:24 + 4 * nb].cpu().numpy().tobytes()))
            self.descs.append(d)
            self.offs.append(total)
            self.sizes.append(size)
            parts.append(blob)
            pad = (-size) % 256
            if pad:
                parts.append(torch.zeros(pad, dtype=torch.uint8, device=device))
            total += size + pad
            if not keep_image:
                imgs[k] = None
                del im
        self.arena = torch.cat(parts)
        del parts
        self.size = int(sum(self.sizes))
        self.image = imgs[0] if keep_image and len(imgs) == 1 else None
        # single-stream names kept for callers of a one-stream slide
        self.desc = self.descs[0]
        self.offsets = self.block_offsets[0]
        self.encode_s = time.perf_counter() - t0
        self.raw_bytes = W * H * 3
        if log:
            log(f"[pyramid] {W}x{H} slide encoded as {len(self.descs)} stream(s) of up to "
                f"{sx * tile}x{sy * tile}: {self.size / 1e9:.3f} GB, "
                f"{sum(len(o) - 1 for o in self.block_offsets)} blocks, encode {self.encode_only_s * 1e3:.1f} ms")

    def grid(self, z):
        s = 1 << z
        return -(-self.tx // s), -(-self.ty // s)

    def region(self, z, X, Y):
        """(x0, y0, w, h) of view (z, X, Y) in the level-z slide image."""
        ow, oh = self.level_size(z)
        x0, y0 = X * self.tile, Y * self.tile
        return x0, y0, min(self.tile, ow - x0), min(self.tile, oh - y0)

    def level_size(self, z):
        ow = sum(isx.out_size(self.descs[i].width, 1, z)[0] for i in range(self.gx))
        oh = sum(isx.out_size(1, self.descs[j * self.gx].height, z)[1] for j in range(self.gy))
        return ow, oh

    def parts(self, z, X, Y):
        """The sub-pyramid regions of view (z, X, Y): (stream k, x0, y0, w, h
        in that stream's level-z image, dx, dy in the view)."""
        vx0, vy0, vw, vh = self.region(z, X, Y)
        if vw <= 0 or vh <= 0:
            return []
        sw, sh = (self.sx * self.tile) >> z, (self.sy * self.tile) >> z
        out = []
        for j in range(vy0 // sh, min(self.gy, (vy0 + vh - 1) // sh + 1)):
            for i in range(vx0 // sw, min(self.gx, (vx0 + vw - 1) // sw + 1)):
                k = j * self.gx + i
                kw, kh = isx.out_size(self.descs[k].width, self.descs[k].height, z)
                ax0, ay0 = i * sw, j * sh
                x0, y0 = max(vx0, ax0), max(vy0, ay0)
                x1, y1 = min(vx0 + vw, ax0 + kw), min(vy0 + vh, ay0 + kh)
                if x1 > x0 and y1 > y0:
                    out.append((k, x0 - ax0, y0 - ay0, x1 - x0, y1 - y0, x0 - vx0, y0 - vy0))
        return out


def viewer_trace(slide, n_viewers=32, steps=200, zmax=6, vw=4, vh=3, seed=502):
    """Requests of viewers doing random walks: pan w.p. 0.8, zoom +-1 w.p. 0.2;
    each step requests the newly visible tiles of the viewport."""
    rng = np.random.Generator(np.random.PCG64(seed))
    state = []
    for _ in range(n_viewers):
        z = int(rng.integers(0, zmax + 1))
        gx, gy = slide.grid(z)
        state.append([z, int(rng.integers(0, max(1, gx - vw + 1))), int(rng.integers(0, max(1, gy - vh + 1)))])
    seen = [set() for _ in range(n_viewers)]
    reqs = []
    for _ in range(steps):
        for v in range(n_viewers):
            z, x, y = state[v]
            if rng.uniform() < 0.8:
                dx, dy = [(1, 0), (-1, 0), (0, 1), (0, -1)][int(rng.integers(0, 4))]
                x, y = x + dx, y + dy
            else:
                nz = min(zmax, max(0, z + (1 if rng.uniform() < 0.5 else -1)))
                if nz > z:
                    x, y = x // 2, y // 2
                elif nz < z:
                    x, y = x * 2, y * 2
                z = nz
            gx, gy = slide.grid(z)
            x = min(max(0, x), max(0, gx - vw))
            y = min(max(0, y), max(0, gy - vh))
            state[v] = [z, x, y]
            vis = {(z, x + i, y + j) for i in range(vw) for j in range(vh) if x + i < gx and y + j < gy}
            for t in sorted(vis - seen[v]):
                reqs.append(t)
            seen[v] = vis
    return reqs


def poisson_arrivals(n, lam, seed=502):
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / lam, size=n))


JOB_DTYPE = np.dtype([("pixel_offset", "<u8"), ("width", "<u4"), ("height", "<u4"),
                      ("row_stride", "<u4"), ("channels", "u1"), ("bps", "u1"), ("bits", "u1"),
                      ("levels", "u1"), ("ct", "u1"), ("r0", "u1", (3,)), ("qstep", "<u2"),
                      ("r1", "<u2"), ("in_offset", "<u8"), ("in_bytes", "<u8"),
                      ("out_offset", "<u8"), ("out_stride", "<u4"), ("target", "u1"),
                      ("drop", "u1"), ("res", "<u2")])
assert JOB_DTYPE.itemsize == 64
REGION_DTYPE = np.dtype([("job", JOB_DTYPE), ("x0", "<u4"), ("y0", "<u4"), ("w", "<u4"), ("h", "<u4"),
                         ("offsets", "<u8")])
assert REGION_DTYPE.itemsize == 88


def _fill_tile(a, d):
    a["width"], a["height"], a["row_stride"] = d.width, d.height, d.row_stride_bytes
    a["channels"], a["bps"], a["bits"], a["levels"] = d.channels, d.bytes_per_sample, d.bits, d.levels
    a["ct"], a["qstep"] = d.colour_transform, d.qstep


class _Slot:
    def __init__(self, ws_bytes, out_bytes, max_jobs, plan_bytes, device):
        import torch
        self.stream = torch.cuda.Stream()
        self.ws = torch.empty(ws_bytes, dtype=torch.uint8, device=device)
        self.out = torch.zeros(out_bytes, dtype=torch.uint8, device=device)
        self.status = torch.zeros(max_jobs, dtype=torch.int32, device=device)
        self.h_plan = torch.empty(plan_bytes, dtype=torch.uint8).pin_memory()
        self.d_plan = torch.empty(plan_bytes, dtype=torch.uint8, device=device)
        self.event = None
        self.reqs = []
        self.busy = False


class Server:
    """Continuous-batching decode server over a Slide.

    Memory: `slots` batch slots, each with `ws_bytes` of decode workspace and
    room for `max_reqs` 512x512x3 outputs; a batch is formed from arrived
    requests in order while its jobs' workspace (library figure) fits."""

    def __init__(self, slide, slots=3, ws_bytes=256 << 20, max_reqs=64, device="cuda",
                 tune=None):
        self.slide = slide
        self.pyr = isinstance(slide, PyramidSlide)
        L = isx.lib()
        if self.pyr:
            self._plan_bytes, self._ws_bytes = L.isx_region_plan_bytes, L.isx_region_workspace_bytes
            self._build = lambda jp, n, hp, pb: L.isx_region_plan_build(jp, n, ctypes.byref(self.tune), hp, pb)
        else:
            self._plan_bytes, self._ws_bytes = L.isx_decode_plan_bytes, L.isx_decode_workspace_bytes
            self._build = lambda jp, n, hp, pb: L.isx_decode_plan_build_tuned(jp, n, ctypes.byref(self.tune),
                                                                              hp, pb)
        self.t = slide.tile
        self.req_bytes = self.t * self.t * 3
        if self.pyr:  # per-stream fields of the region jobs
            self._sub_w = np.array([d.width for d in slide.descs], dtype=np.int64)
            self._sub_h = np.array([d.height for d in slide.descs], dtype=np.int64)
            self._sub_off = np.array(slide.offs, dtype=np.int64)
            self._sub_size = np.array(slide.sizes, dtype=np.int64)
            self._sub_bofs = np.array([o.ctypes.data for o in slide.block_offsets], dtype=np.uint64)
        self.max_reqs = max_reqs
        self.max_jobs = 16384  # decode jobs (source tiles) per batch
        self.tune = tune if tune is not None else isx.tuning()
        # plan bytes upper bound for max_jobs jobs
        if self.pyr:  # the widest batch: views that cross sub-pyramid edges, at every zoom
            pb = 0
            for z in range(slide.levels + 1):
                gx, gy = slide.grid(z)
                for X, Y in ((0, 0), (min(1, gx - 1), min(1, gy - 1)), (gx // 2, gy // 2)):
                    probe = self._jobs([Request(0, z, X, Y)] * max_reqs)
                    if len(probe):
                        pb = max(pb, int(self._plan_bytes(probe.ctypes.data, len(probe))))
            pb *= 4
        else:
            probe = self._jobs([Request(0, 0, 0, 0)], dummy=self.max_jobs)
            pb = int(self._plan_bytes(probe.ctypes.data, len(probe)))
        self.plan_cap = pb + (1 << 16)
        self.ws_cap = ws_bytes
        self.slots = [_Slot(ws_bytes, max_reqs * self.req_bytes, self.max_jobs, self.plan_cap, device)
                      for _ in range(slots)]
        self.ws_est = {}

    def _jobs(self, reqs, dummy=0):
        """Decode jobs (a numpy array laid out as isx_decode_job, or as
        isx_region_job for a pyramid) for requests."""
        d = self.slide.desc
        if self.pyr:
            sl = self.slide
            rows = [(r, p) for r in reqs for p in sl.parts(r.z, r.X, r.Y)]
            a = np.zeros(len(rows), dtype=REGION_DTYPE)
            job = a["job"]
            _fill_tile(job, d)  # shared fields; the sizes per stream below
            if rows:
                P = np.array([p for _, p in rows], dtype=np.int64)
                k = P[:, 0]
                job["width"] = self._sub_w[k]
                job["height"] = self._sub_h[k]
                job["row_stride"] = self._sub_w[k] * 3
                job["in_offset"] = self._sub_off[k]
                job["in_bytes"] = self._sub_size[k]
                job["out_offset"] = np.array([r.out_off for r, _ in rows], dtype=np.int64) + (P[:, 6] * self.t + P[:, 5]) * 3
                job["target"] = [r.z for r, _ in rows]
                a["offsets"] = self._sub_bofs[k]
                a["x0"], a["y0"], a["w"], a["h"] = P[:, 1], P[:, 2], P[:, 3], P[:, 4]
            job["out_stride"] = self.t * 3
            return a
        if dummy:
            a = np.zeros(dummy, dtype=JOB_DTYPE)
            _fill_tile(a, d)
            a["in_bytes"] = 1
            a["out_stride"] = self.t * 3
            return a
        parts = []
        for r in reqs:
            ids, ii, jj = self.slide.source_arrays(r.z, r.X, r.Y)
            a = np.zeros(len(ids), dtype=JOB_DTYPE)
            _fill_tile(a, d)
            sub = self.t >> r.z
            a["in_offset"] = self.slide.offsets[ids]
            a["in_bytes"] = self.slide.sizes[ids]
            a["out_offset"] = r.out_off + (jj * sub * self.t + ii * sub) * 3
            a["out_stride"] = self.t * 3
            a["target"] = r.z
            parts.append(a)
        return np.concatenate(parts) if parts else np.zeros(0, dtype=JOB_DTYPE)

    def req_ws(self, z):
        """Workspace of one request at zoom z (cached library figure)."""
        if z not in self.ws_est:
            # the largest of a corner view (all sources present) and an
            # interior view (the widest halo cover of a pyramid region)
            gx, gy = self.slide.grid(z)
            est = 0
            for X, Y in ((0, 0), (min(1, gx - 1), min(1, gy - 1)), (gx // 2, gy // 2), (gx - 1, gy - 1)):
                jobs = self._jobs([Request(0, z, X, Y)])
                est = max(est, int(self._ws_bytes(jobs.ctypes.data, len(jobs))))
            self.ws_est[z] = est
        return self.ws_est[z]

    def covered(self, r) -> bool:
        """Does the view lie wholly inside the slide?"""
        if self.pyr:
            return sum(p[3] * p[4] for p in self.slide.parts(r.z, r.X, r.Y)) == self.t * self.t
        return self.slide.source_count(r.z, r.X, r.Y) == (1 << (2 * r.z))

    def view_pixels(self, r) -> int:
        if self.pyr:
            return sum(p[3] * p[4] for p in self.slide.parts(r.z, r.X, r.Y))
        return (self.t >> r.z) ** 2 * self.slide.source_count(r.z, r.X, r.Y)

    def launch(self, slot: _Slot, reqs):
        import torch
        L = isx.lib()
        for k, r in enumerate(reqs):
            r.out_off = k * self.req_bytes
        jobs = self._jobs(reqs)
        n = len(jobs)
        jp = jobs.ctypes.data
        # one planning pass: build into the slot's buffer, read the sizes back
        hp = (ctypes.c_uint8 * self.plan_cap).from_address(slot.h_plan.data_ptr())
        rc = self._build(jp, n, hp, self.plan_cap)
        if rc:
            raise isx.IsxError(rc, "serve plan (or plan beyond the slot's buffer)")
        pbv, need = ctypes.c_uint64(), ctypes.c_uint64()
        rc = L.isx_plan_info(hp, ctypes.byref(pbv), ctypes.byref(need))
        if rc:
            raise isx.IsxError(rc, "serve plan info")
        pb = int(pbv.value)
        if int(need.value) > self.ws_cap:
            raise RuntimeError("batch exceeds the slot workspace")
        with torch.cuda.stream(slot.stream):
            for r in reqs:  # views that run off the slide: clear the part no source covers
                if not self.covered(r):
                    slot.out[r.out_off:r.out_off + self.req_bytes].zero_()
            slot.d_plan[:pb].copy_(slot.h_plan[:pb], non_blocking=True)
            rc = L.isx_decode_run(hp, isx._ptr(slot.d_plan), isx._ptr(self.slide.arena), isx._ptr(slot.out),
                                  isx._ptr(slot.status), isx._ptr(slot.ws), slot.ws.numel(),
                                  ctypes.c_void_p(slot.stream.cuda_stream))
            if rc:
                raise isx.IsxError(rc, "serve decode")
            slot.event = torch.cuda.Event(enable_timing=True)
            slot.event.record(slot.stream)
        slot.reqs = reqs
        slot.busy = True
        slot.njobs = n

    def run(self, reqs, log=None, check=None):
        """Serve `reqs` (with .arrival in seconds from start); returns stats.

        A request's completion time is its batch's device event: the time
        origin is a reference event recorded on an idle stream and waited
        for, so device event times convert to the host clock of the arrivals
        (late by at most the wait's own latency, never early)."""
        import torch
        pending = deque(sorted(reqs, key=lambda r: r.arrival))
        ready = deque()
        torch.cuda.synchronize()
        ref = torch.cuda.Event(enable_timing=True)
        ref.record(self.slots[0].stream)
        ref.synchronize()
        t0 = time.perf_counter()
        done = 0
        batches = 0
        px = 0
        while done < len(reqs):
            now = time.perf_counter() - t0
            # completions
            for s in self.slots:
                if s.busy and s.event.query():
                    tdone = ref.elapsed_time(s.event) * 1e-3
                    st = s.status[:s.njobs].cpu()
                    if int(st.abs().sum()) != 0:
                        raise RuntimeError("decode error in a served batch")
                    for r in s.reqs:
                        r.done = tdone
                        px += self.view_pixels(r)
                    if check:
                        check(s, s.reqs)
                    done += len(s.reqs)
                    s.busy = False
            while pending and pending[0].arrival <= now:
                ready.append(pending.popleft())
            free = [s for s in self.slots if not s.busy]
            if ready and free:
                batch, ws, nj = [], 0, 0
                while ready and len(batch) < self.max_reqs:
                    need = self.req_ws(ready[0].z)
                    jobs = 4 if self.pyr else 1 << (2 * ready[0].z)
                    if batch and (ws + need > self.ws_cap * 0.9 or nj + jobs > self.max_jobs):
                        break
                    ws += need
                    nj += jobs
                    batch.append(ready.popleft())
                self.launch(free[0], batch)
                batches += 1
            elif not ready and pending:
                wait = pending[0].arrival - (time.perf_counter() - t0)
                if wait > 2e-4 and not any(s.busy for s in self.slots):
                    time.sleep(wait - 1e-4)
        wall = max(time.perf_counter() - t0, max(r.done for r in reqs))
        lat = np.array([r.done - r.arrival for r in reqs]) * 1e3
        return {"requests": len(reqs), "batches": batches, "wall_s": wall,
                "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "mean_ms": float(lat.mean()), "decoded_mpx_s": px / 1e6 / wall,
                "offered_rps": len(reqs) / max(reqs[-1].arrival, 1e-9), "served_rps": len(reqs) / wall}

    def decode_alone(self, r: Request):
        """Decode one request by itself (slot 0), returns its output bytes (host)."""
        import torch
        s = self.slots[0]
        while s.busy:
            if s.event.query():
                s.busy = False
        self.launch(s, [r])
        s.event.synchronize()
        s.busy = False
        return s.out[:self.req_bytes].cpu().numpy().copy()
