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
    for tq, bpc in [(32, 0), (16, 0), (32, 1), (16, 3), (32, 8)]:
        print("tuning", tq, bpc, flush=True)
        enc = isx.Encoder(descs, tune=isx.tuning(tq, bpc))
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
        dec = isx.Decoder(jobs, nbytes, tune=isx.tuning(tq, bpc))
        dec.run(enc.out)
        torch.cuda.synchronize()
        assert int(dec.status.abs().sum().item()) == 0
        host = dec.out.cpu().numpy()
        for i, (o, oh, ow, c) in enumerate(outs):
            got = host[o:o + oh * ow * c].reshape(oh, ow, c)
            assert np.array_equal(got, oracle.decode_tile(ref[i], zs[i])), (tq, bpc, i)


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
    res = autotune.tune(descs, d_pix, reps=1, candidates=[(32, 0), (16, 0), (32, 4)])
    assert tuple(res["encode"]) in [(32, 0), (16, 0), (32, 4)]
    assert os.path.exists(tmp_path / "tune.json")
    again = autotune.tune(descs, d_pix, reps=1)
    assert again == res
