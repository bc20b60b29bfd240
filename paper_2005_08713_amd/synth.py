"""Seeded synthetic inputs shaped like the paper's workloads.

The paper benchmarks on histopathology scans (RGB, 8-9 bits per channel) and
on radiology images (CR/DX/MG, 12-16 bit single channel) whose datasets are
not available here (Sec. 5).  These generators produce stand-ins with the
same shapes, value ranges and spatial structure:

* ``he_like``  -- H&E-stained tissue on a bright background, RGB uint8
  (or 9-bit RGB in uint16, as the paper's pathology scans).
* ``rad_like`` -- a smooth radial gradient with blob structures and Poisson
  counting noise, single channel uint16 with 12 (or more) significant bits.
* ``tile_batch`` -- a batch of RGB tiles of uneven size (square 512/256/128
  tiles plus ragged edge tiles), with per-tile wavelet levels and
  lossless/quantised mode, as produced when a slide is cut into tiles.

This module holds none of the codec's arithmetic; it only draws numbers.
Both the GPU library and the CPU oracle are fed the arrays it returns.
"""
from __future__ import annotations

import numpy as np

PINK = np.array([232.0, 150.0, 190.0])
PURPLE = np.array([130.0, 70.0, 160.0])


def _blob_field(rng, w, h, nblobs, sig_lo, sig_hi, amp_lo, amp_hi):
    """Sum of separable isotropic Gaussian blobs evaluated on a w x h grid."""
    xs = np.arange(w, dtype=np.float64)
    ys = np.arange(h, dtype=np.float64)
    field = np.zeros((h, w), dtype=np.float64)
    for _ in range(nblobs):
        cx = rng.uniform(0, w)
        cy = rng.uniform(0, h)
        sig = rng.uniform(sig_lo, sig_hi)
        amp = rng.uniform(amp_lo, amp_hi)
        gx = np.exp(-((xs - cx) ** 2) / (2.0 * sig * sig))
        gy = np.exp(-((ys - cy) ** 2) / (2.0 * sig * sig))
        field += amp * np.outer(gy, gx)
    return field


def he_like(width: int, height: int, seed: int, sigma=(20.0, 60.0),
            tissue: float = 0.40, bits: int = 8) -> np.ndarray:
    """H&E-like RGB image, shape (height, width, 3): uint8, or uint16 for
    bits > 8 (the 9-bit-per-channel scans).

    Background ~U{230..245} per pixel and channel; tissue where an 8-blob
    field exceeds its (1-tissue) quantile, coloured by a second 8-blob field
    mixing pink and purple stain colours; additive N(0, 2^2) noise.  For
    bits > 8 the background and stain colours are scaled by 2^(bits-8) and
    the noise by the same factor before rounding.
    """
    if bits != 8:
        return _he_like_deep(width, height, seed, sigma, tissue, bits)
    rng = np.random.Generator(np.random.PCG64(seed))
    img = rng.integers(230, 246, size=(height, width, 3)).astype(np.float64)
    f = _blob_field(rng, width, height, 8, sigma[0], sigma[1], 0.5, 1.0)
    thr = np.quantile(f, 1.0 - tissue)
    mask = f > thr
    hfield = _blob_field(rng, width, height, 8, sigma[0], sigma[1], 0.5, 1.0)
    lo, hi = hfield.min(), hfield.max()
    hmix = (hfield - lo) / (hi - lo) if hi > lo else np.zeros_like(hfield)
    colour = np.rint((1.0 - hmix)[..., None] * PINK + hmix[..., None] * PURPLE)
    img[mask] = colour[mask]
    img += rng.normal(0.0, 2.0, size=img.shape)
    return np.clip(np.rint(img), 0, 255).astype(np.uint8)


def _he_like_deep(width, height, seed, sigma, tissue, bits):
    rng = np.random.Generator(np.random.PCG64(seed))
    k = float(1 << (bits - 8))
    img = rng.uniform(230.0, 246.0, size=(height, width, 3)) * k
    f = _blob_field(rng, width, height, 8, sigma[0], sigma[1], 0.5, 1.0)
    mask = f > np.quantile(f, 1.0 - tissue)
    hfield = _blob_field(rng, width, height, 8, sigma[0], sigma[1], 0.5, 1.0)
    lo, hi = hfield.min(), hfield.max()
    hmix = (hfield - lo) / (hi - lo) if hi > lo else np.zeros_like(hfield)
    colour = ((1.0 - hmix)[..., None] * PINK + hmix[..., None] * PURPLE) * k
    img[mask] = colour[mask]
    img += rng.normal(0.0, 2.0 * k, size=img.shape)
    return np.clip(np.rint(img), 0, (1 << bits) - 1).astype(np.uint16 if bits <= 16 else np.uint32)


def rad_like(width: int, height: int, seed: int, bits: int = 12) -> np.ndarray:
    """Radiology-like uint16 image (12 significant bits), shape (height, width).

    lambda = 2000 + 300 (1 - 2 r / r_max) plus 20 Gaussian blobs with
    amplitude ~U(-600, 1200) and sigma ~U(50, 800) px (scaled down for
    images smaller than 8192 px), clipped to [1, 4000]; Poisson counts
    clipped to [0, 4095].  For another ``bits`` the intensity field is
    scaled by 2^(bits-12) before the Poisson draw and the counts are clipped
    to [0, 2^bits - 1].
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    ys, xs = np.mgrid[0:height, 0:width].astype(np.float64)
    cx, cy = (width - 1) / 2.0, (height - 1) / 2.0
    r = np.hypot(xs - cx, ys - cy)
    rmax = max(r.max(), 1.0)
    lam = 2000.0 + 300.0 * (1.0 - 2.0 * r / rmax)
    del xs, ys, r
    scale = min(1.0, max(width, height) / 8192.0)
    lam += _blob_field(rng, width, height, 20, 50.0 * scale + 1.0,
                       800.0 * scale + 2.0, -600.0, 1200.0)
    lam = np.clip(lam, 1.0, 4000.0)
    if bits != 12:
        lam *= 2.0 ** (bits - 12)
    counts = rng.poisson(lam)
    return np.clip(counts, 0, (1 << bits) - 1).astype(np.uint16)


def random_image(width: int, height: int, channels: int, bits: int,
                 seed: int, kind: str = "uniform") -> np.ndarray:
    """Adversarial / generic test images of any bit depth.

    kind: 'uniform' (iid uniform over [0, 2^bits)), 'const', 'max'
    (all samples 2^bits-1), 'checker' (alternating 0 / max), 'checker2'
    (2x2 squares alternating 0 / max, channel k shifted by k squares),
    'ramp', 'sparse' (mostly zero with a few random samples).
    Returns uint8 for bits <= 8, uint16 for bits <= 16, else uint32; shape (h, w, c).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    top = (1 << bits) - 1
    dt = np.uint8 if bits <= 8 else (np.uint16 if bits <= 16 else np.uint32)
    shape = (height, width, channels)
    if kind == "uniform":
        a = rng.integers(0, top + 1, size=shape)
    elif kind == "const":
        a = np.full(shape, rng.integers(0, top + 1))
    elif kind == "max":
        a = np.full(shape, top)
    elif kind == "checker":
        yy, xx = np.mgrid[0:height, 0:width]
        a = np.repeat((((yy + xx) & 1) * top)[..., None], channels, axis=2)
    elif kind == "checker2":
        yy, xx = np.mgrid[0:height, 0:width]
        a = np.stack([(((yy >> 1) + (xx >> 1) + k) & 1) * top for k in range(channels)], axis=2)
    elif kind == "ramp":
        yy, xx = np.mgrid[0:height, 0:width]
        a = np.repeat(((yy * 7 + xx * 3) % (top + 1))[..., None], channels, axis=2)
    elif kind == "sparse":
        a = np.zeros(shape, dtype=np.int64)
        n = max(1, (height * width * channels) // 50)
        idx = rng.integers(0, height * width * channels, size=n)
        a.reshape(-1)[idx] = rng.integers(0, top + 1, size=n)
    else:
        raise ValueError(kind)
    return a.astype(dt)


def _he_tile(args):
    w, h, seed, sc = args
    return he_like(w, h, seed, sigma=(max(1.0, 20.0 * sc), max(2.0, 60.0 * sc)))


def tile_batch(n_tiles: int, seed: int, content_seed_base: int,
               sides=(512, 256, 128), edge_frac: float = 0.15,
               levels=(3, 4, 5), qstep: int = 4, max_side: int = 511, workers: int = 1):
    """Mixed batch of RGB uint8 tiles as cut from a slide.

    Returns a list of dicts {pixels, levels, qstep}.  85% of tiles are
    square with side drawn uniformly from ``sides``; the rest are edge tiles
    with width and height ~U{1..max_side}.  Levels ~U(levels); mode is
    lossless (qstep 1) or quantised (``qstep``) with probability 1/2.  Tile i
    has content seed ``content_seed_base + i`` and blob sigma scaled by
    side/256.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    specs = []
    for i in range(n_tiles):
        if rng.uniform() < edge_frac:
            w = int(rng.integers(1, max_side + 1))
            h = int(rng.integers(1, max_side + 1))
        else:
            s = int(sides[int(rng.integers(0, len(sides)))])
            w = h = s
        lv = int(levels[int(rng.integers(0, len(levels)))])
        q = 1 if rng.uniform() < 0.5 else int(qstep)
        specs.append((w, h, lv, q))
    jobs = [(w, h, content_seed_base + i, max(w, h) / 256.0) for i, (w, h, _, _) in enumerate(specs)]
    if workers > 1:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(workers) as pool:
            pixels = pool.map(_he_tile, jobs, chunksize=8)
    else:
        pixels = [_he_tile(j) for j in jobs]
    return [{"pixels": px, "levels": lv, "qstep": q}
            for px, (w, h, lv, q) in zip(pixels, specs)]


# --------------------------------------------------------------------------
# Whole-slide generator on the GPU (torch), for the served-slide workload.
class SlideGen:
    """H&E-like slide of tiles_x x tiles_y square tiles, generated tile batch
    by tile batch on the GPU.

    Recipe (same structure as ``he_like``): 8 Gaussian blobs per 4096^2 area
    (sigma ~U(100, 600) px, amplitude ~U(0.5, 1)) form the tissue field,
    thresholded at its 60% quantile (40% tissue); a second blob set mixes
    pink and purple stain colours; background ~U{230..245}; N(0, 2^2) noise.
    The two fields are evaluated on a 32-px grid (blobs only within 4 sigma)
    and bilinearly upsampled per tile.  Blob parameters come from numpy
    PCG64(seed); the per-pixel background and noise of tile batch b come from
    a torch generator seeded with seed * 1000 + b.
    """

    def __init__(self, tiles_x: int, tiles_y: int, tile: int = 512, seed: int = 501, device="cuda"):
        import torch
        self.tx, self.ty, self.tile, self.seed, self.device = tiles_x, tiles_y, tile, seed, device
        W, H = tiles_x * tile, tiles_y * tile
        self.step = 32
        gw, gh = W // self.step + 2, H // self.step + 2
        rng = np.random.Generator(np.random.PCG64(seed))
        nb = max(1, int(round(8 * W * H / 4096.0 ** 2)))
        fields = []
        for _ in range(2):
            f = torch.zeros((gh, gw), dtype=torch.float32, device=device)
            cx = rng.uniform(0, W, nb)
            cy = rng.uniform(0, H, nb)
            sg = rng.uniform(100, 600, nb)
            am = rng.uniform(0.5, 1.0, nb)
            for x, y, s, a in zip(cx, cy, sg, am):
                x0 = max(0, int((x - 4 * s) / self.step)); x1 = min(gw, int((x + 4 * s) / self.step) + 1)
                y0 = max(0, int((y - 4 * s) / self.step)); y1 = min(gh, int((y + 4 * s) / self.step) + 1)
                if x1 <= x0 or y1 <= y0:
                    continue
                xs = torch.arange(x0, x1, device=device, dtype=torch.float32) * self.step
                ys = torch.arange(y0, y1, device=device, dtype=torch.float32) * self.step
                gx = torch.exp(-(xs - x) ** 2 / (2 * s * s))
                gy = torch.exp(-(ys - y) ** 2 / (2 * s * s))
                f[y0:y1, x0:x1] += float(a) * torch.outer(gy, gx)
            fields.append(f)
        self.tissue, self.stain = fields
        flat = self.tissue.flatten()
        if flat.numel() > 4_000_000:
            idx = torch.linspace(0, flat.numel() - 1, 4_000_000, device=device).long()
            flat = flat[idx]
        self.thr = float(torch.quantile(flat, 0.60))
        lo, hi = float(self.stain.min()), float(self.stain.max())
        self.stain = (self.stain - lo) / max(hi - lo, 1e-12)

    def tiles(self, ids, batch_index: int):
        """uint8 tensor (len(ids), tile, tile, 3) for tile ids (ty * tiles_x + tx)."""
        import torch
        import torch.nn.functional as F
        T, st = self.tile, self.step
        k = T // st
        g = torch.Generator(device=self.device)
        g.manual_seed(self.seed * 1000 + batch_index)
        out = torch.empty((len(ids), T, T, 3), dtype=torch.uint8, device=self.device)
        pink = torch.tensor([232.0, 150.0, 190.0], device=self.device)
        purple = torch.tensor([130.0, 70.0, 160.0], device=self.device)
        for n, tid in enumerate(ids):
            tx, ty = tid % self.tx, tid // self.tx
            fa = self.tissue[ty * k:ty * k + k + 1, tx * k:tx * k + k + 1][None, None]
            fb = self.stain[ty * k:ty * k + k + 1, tx * k:tx * k + k + 1][None, None]
            fa = F.interpolate(fa, size=(T + 1, T + 1), mode="bilinear", align_corners=True)[0, 0, :T, :T]
            fb = F.interpolate(fb, size=(T + 1, T + 1), mode="bilinear", align_corners=True)[0, 0, :T, :T]
            img = torch.randint(230, 246, (T, T, 3), generator=g, device=self.device).float()
            col = torch.round((1 - fb)[..., None] * pink + fb[..., None] * purple)
            img = torch.where((fa > self.thr)[..., None], col, img)
            img = img + 2.0 * torch.randn((T, T, 3), generator=g, device=self.device)
            out[n] = torch.clamp(torch.round(img), 0, 255).to(torch.uint8)
        return out
