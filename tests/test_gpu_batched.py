"""GPU tests of the batched production pattern: one plan for many uneven
tiles, launch parameters (LDS tile shape, persistent workgroups per CU) that
must not change a single output byte, HIP-graph capture and replay, and the
autotuner."""
import os

import numpy as np
import pytest

import oracle
from paper_2005_08713_amd import isx, synth

pytestmark = pytest.mark.gpu


def _batch(n=40, seed=11):
    tiles = synth.tile_batch(n, seed=seed, content_seed_base=seed * 1000, sides=(128, 64, 32),
                             max_side=200)
    return tiles


def _upload(tiles):
    import torch
    descs, chunks, off = [], [], 0
    for t in tiles:
        a = t["pixels"]
        h, w, c = a.shape
        descs.append(isx.tile_desc(w, h, c, 1, 8, t["levels"], qstep=t["qstep"], pixel_offset=off))
        chunks.append(a.reshape(-1))
        off += a.size
        pad = (-off) % 16
        chunks.append(np.zeros(pad, np.uint8))
        off += pad
    return descs, torch.from_numpy(np.concatenate(chunks)).cuda()


def _jobs(descs, enc, streams, levels=None):
    offs = enc.offsets.cpu().numpy()
    jobs, out_off, outs = [], 0, []
    for i, d in enumerate(descs):
        z = 0 if levels is None else levels[i]
        ow, oh = isx.out_size(d.width, d.height, z)
        j = isx.DecodeJob()
        j.tile = d
        j.in_offset, j.in_bytes = int(offs[i]), len(streams[i])
        j.out_offset, j.out_row_stride_bytes, j.target_level = out_off, ow * d.channels, z
        jobs.append(j)
        outs.append((out_off, oh, ow, d.channels))
        out_off += oh * ow * d.channels
    return jobs, out_off, outs


def test_tunings_give_identical_bytes_and_pixels():
    import torch
    tiles = _batch()
    descs, d_pix = _upload(tiles)
    ref = None
    # the last four force the segment decoder's waves per segment (the
    # default picks four for a batch this small)
    for tun in [(32, 0, 0), (16, 0, 0), (32, 1, 0), (16, 3, 0), (32, 8, 0), (32, 0, 1, 1), (32, 0, 7, 1),
                (32, 0, 0, 1), (32, 0, 3, 1), (16, 3, 0, 2), (32, 0, 0, 4)]:
        print("tuning", tun, flush=True)
        enc = isx.Encoder(descs, tune=isx.tuning(*tun))
        enc.run(d_pix)
        torch.cuda.synchronize()
        streams = enc.streams()
        if ref is None:
            ref = streams
            for t, s in zip(tiles, streams):
                assert s == oracle.encode_tile(t["pixels"], t["levels"], qstep=t["qstep"])
        assert streams == ref
        zs = [i % (t["levels"] + 1) for i, t in enumerate(tiles)]
        jobs, nbytes, outs = _jobs(descs, enc, streams, zs)
        dec = isx.Decoder(jobs, nbytes, tune=isx.tuning(*tun))
        dec.run(enc.out)
        torch.cuda.synchronize()
        assert int(dec.status.abs().sum().item()) == 0
        host = dec.out.cpu().numpy()
        for i, (o, oh, ow, c) in enumerate(outs):
            got = host[o:o + oh * ow * c].reshape(oh, ow, c)
            assert np.array_equal(got, oracle.decode_tile(ref[i], zs[i])), (tun, i)


def test_graph_replay_matches_eager_every_time():
    import torch
    tiles = _batch(24, seed=12)
    descs, d_pix = _upload(tiles)
    eager = isx.Encoder(descs)
    eager.run(d_pix)
    torch.cuda.synchronize()
    ref = eager.streams()
    g = isx.Encoder(descs, tune=isx.tuning(32, 4))
    g.capture(d_pix)
    jobs, nbytes, outs = _jobs(descs, g, ref)
    dec = isx.Decoder(jobs, nbytes)
    dec.capture(g.out)
    for rep in range(4):
        print("replay", rep, flush=True)
        g.out.zero_()
        dec.out.zero_()
        g.replay()
        # unrelated eager work between replays, on the same stream
        x = torch.randn(1 << 20, device="cuda")
        _ = (x * 2).sum().item()
        eager.run(d_pix)
        dec.replay()
        torch.cuda.synchronize()
        assert g.streams() == ref
        host = dec.out.cpu().numpy()
        for i, (o, oh, ow, c) in enumerate(outs):
            assert np.array_equal(host[o:o + oh * ow * c].reshape(oh, ow, c), tiles[i]["pixels"]) \
                or tiles[i]["qstep"] != 1


def test_autotuner_picks_a_valid_setting(tmp_path, monkeypatch):
    from paper_2005_08713_amd import autotune
    monkeypatch.setenv("ISX_TUNE_CACHE", str(tmp_path / "tune.json"))
    tiles = _batch(16, seed=13)
    descs, d_pix = _upload(tiles)
    res = autotune.tune(descs, d_pix, reps=1, candidates=[(32, 0), (16, 0), (32, 4), (32, 0, 8, 1)])
    ok = [(32, 0, 0, 0), (16, 0, 0, 0), (32, 4, 0, 0), (32, 0, 8, 1)]
    assert tuple(res["encode"]) in ok
    assert tuple(res["decode"]) in ok
    assert os.path.exists(tmp_path / "tune.json")
    again = autotune.tune(descs, d_pix, reps=1)
    assert again == res


def test_serving_results_identical_alone_and_in_the_mix():
    """Requests decoded inside mixed continuous batches equal the same request
    decoded alone, and equal the oracle's stitched level-z decodes."""
    import torch
    from paper_2005_08713_amd import serve
    slide = serve.Slide(6, 5, tile=512, levels=6, seed=7, batch=16)
    srv = serve.Server(slide, slots=3, ws_bytes=192 << 20, max_reqs=16)
    trace = serve.viewer_trace(slide, n_viewers=8, steps=6, zmax=3, seed=9)
    reqs = [serve.Request(i, z, X, Y) for i, (z, X, Y) in enumerate(trace[:60])]
    times = serve.poisson_arrivals(len(reqs), 4000.0, seed=3)
    for r, t in zip(reqs, times):
        r.arrival = float(t)
    got = {}

    def check(slot, rs):
        host = slot.out.cpu().numpy()
        for r in rs:
            got[r.rid] = host[r.out_off:r.out_off + srv.req_bytes].copy()

    stats = srv.run(reqs, check=check)
    print("serve stats", stats, flush=True)
    assert stats["batches"] >= 2 and len(got) == len(reqs)
    # each result the same alone
    for r in reqs[::7]:
        alone = srv.decode_alone(serve.Request(r.rid, r.z, r.X, r.Y))
        assert np.array_equal(alone, got[r.rid]), r
    # and equal to the oracle on the stitched sources (a few requests)
    enc = slide.arena.cpu().numpy()
    for r in reqs[:4]:
        exp = np.zeros((512, 512, 3), np.uint8)
        sub = 512 >> r.z
        for tid, i, j in slide.sources(r.z, r.X, r.Y):
            blob = enc[slide.offsets[tid]:slide.offsets[tid] + slide.sizes[tid]].tobytes()
            exp[j * sub:(j + 1) * sub, i * sub:(i + 1) * sub] = oracle.decode_tile(blob, r.z)
        assert np.array_equal(got[r.rid].reshape(512, 512, 3), exp), r
    # the slide's own pixels round-trip at zoom 0
    px = slide.gen.tiles([0], 0)[0].cpu().numpy()
    blob = enc[slide.offsets[0]:slide.offsets[0] + slide.sizes[0]].tobytes()
    assert np.array_equal(oracle.decode_tile(blob, 0), px)


def test_pyramid_serving_regions_match_the_oracle():
    """The same slide as one pyramid: served views equal the oracle's crops
    of the level-z decode, equal the same view decoded alone, and at zoom 0
    equal the slide's pixels."""
    import torch
    from paper_2005_08713_amd import serve
    pyr = serve.PyramidSlide(5, 4, tile=256, levels=5, seed=7, batch=8)
    srv = serve.Server(pyr, slots=3, ws_bytes=96 << 20, max_reqs=16)
    trace = serve.viewer_trace(pyr, n_viewers=6, steps=6, zmax=4, seed=9)
    reqs = [serve.Request(i, z, X, Y) for i, (z, X, Y) in enumerate(trace[:48])]
    times = serve.poisson_arrivals(len(reqs), 4000.0, seed=3)
    for r, t in zip(reqs, times):
        r.arrival = float(t)
    got = {}

    def check(slot, rs):
        host = slot.out.cpu().numpy()
        for r in rs:
            got[r.rid] = host[r.out_off:r.out_off + srv.req_bytes].copy()

    stats = srv.run(reqs, check=check)
    print("pyramid serve stats", stats, flush=True)
    assert stats["batches"] >= 2 and len(got) == len(reqs)
    blob = pyr.arena.cpu().numpy().tobytes()
    full = {}
    img = pyr.image.cpu().numpy()
    for r in reqs[::3]:
        x0, y0, w, h = pyr.region(r.z, r.X, r.Y)
        if r.z not in full:
            full[r.z] = oracle.decode_tile(blob, r.z)
        exp = np.zeros((256, 256, 3), np.uint8)
        exp[:h, :w] = full[r.z][y0:y0 + h, x0:x0 + w]
        assert np.array_equal(got[r.rid].reshape(256, 256, 3), exp), r
        if r.z == 0:
            assert np.array_equal(exp[:h, :w], img[y0:y0 + h, x0:x0 + w])
    for r in reqs[1::9]:
        assert np.array_equal(srv.decode_alone(serve.Request(r.rid, r.z, r.X, r.Y)), got[r.rid]), r


def test_pyramid_grid_serving_regions_match_the_oracle():
    """A slide as a grid of pyramid streams (2 x 2 sub-pyramids, the last
    column narrower): served views, which cross the streams' edges at every
    zoom, equal the stitched crops of the oracle's level-z decodes of the
    streams they touch, and the same view decoded alone; at zoom 0 every view
    equals the generator's tile pixels."""
    from paper_2005_08713_amd import serve
    pyr = serve.PyramidSlide(6, 4, tile=128, levels=4, seed=11, batch=8, sub=(4, 2))
    assert (pyr.gx, pyr.gy) == (2, 2) and pyr.image is None
    srv = serve.Server(pyr, slots=3, ws_bytes=96 << 20, max_reqs=16)
    trace = serve.viewer_trace(pyr, n_viewers=6, steps=8, zmax=4, seed=13)
    extra = [(z, X, Y) for z in range(5) for X in range(pyr.grid(z)[0]) for Y in range(pyr.grid(z)[1])]
    sample = trace[:40] + extra
    reqs = [serve.Request(i, z, X, Y) for i, (z, X, Y) in enumerate(sample)]
    times = serve.poisson_arrivals(len(reqs), 4000.0, seed=5)
    for r, t in zip(reqs, times):
        r.arrival = float(t)
    got = {}

    def check(slot, rs):
        host = slot.out.cpu().numpy()
        for r in rs:
            got[r.rid] = host[r.out_off:r.out_off + srv.req_bytes].copy()

    print("pyramid grid serve", len(reqs), "requests", flush=True)
    srv.run(reqs, check=check)
    assert len(got) == len(reqs)
    arena = pyr.arena.cpu().numpy()
    full = {}

    def level(k, z):
        if (k, z) not in full:
            o, n = pyr.offs[k], pyr.sizes[k]
            full[(k, z)] = oracle.decode_tile(arena[o:o + n].tobytes(), z)
        return full[(k, z)]

    T = pyr.tile
    # the tile pixels, generated again batch by batch as the slide was
    tiles = {}
    for b0 in range(0, pyr.n, 8):
        ids = list(range(b0, min(pyr.n, b0 + 8)))
        px = pyr.gen.tiles(ids, b0 // 8).cpu().numpy()
        for k, t in enumerate(ids):
            tiles[t] = px[k]
    for r in reqs:
        exp = np.zeros((T, T, 3), np.uint8)
        parts = pyr.parts(r.z, r.X, r.Y)
        assert parts, r
        for (k, x0, y0, w, h, dx, dy) in parts:
            exp[dy:dy + h, dx:dx + w] = level(k, r.z)[y0:y0 + h, x0:x0 + w]
        assert np.array_equal(got[r.rid].reshape(T, T, 3), exp), r
        if r.z == 0:
            assert np.array_equal(exp, tiles[r.Y * pyr.tx + r.X]), r
    for r in reqs[1::7]:
        assert np.array_equal(srv.decode_alone(serve.Request(r.rid, r.z, r.X, r.Y)), got[r.rid]), r
