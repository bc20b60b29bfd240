"""GPU tests of the two work entry points, called directly through the C ABI
(isx_encode_tiles / isx_decode_tiles: plan built and copied by the library),
and full-size parity of the single-image workloads against the oracle.

Integer codec: every comparison is exact.
"""
import numpy as np
import pytest

import oracle
from paper_2005_08713_amd import isx, synth

pytestmark = pytest.mark.gpu


def _batch():
    """Mixed tiles: 8- and 16-bit, 1 and 3 channels, ragged sizes, lossless
    and quantised, 0-6 levels."""
    specs = [(300, 200, 3, 8, 4, 1, "he"), (37, 23, 3, 8, 3, 4, "uniform"), (1, 1, 1, 8, 0, 1, "uniform"),
             (129, 257, 1, 12, 5, 1, "uniform"), (64, 64, 3, 8, 6, 3, "sparse"), (511, 9, 1, 16, 2, 1, "ramp")]
    imgs, descs, chunks, off = [], [], [], 0
    for i, (w, h, c, bits, lv, q, kind) in enumerate(specs):
        img = synth.he_like(w, h, 900 + i) if kind == "he" else synth.random_image(w, h, c, bits, 900 + i, kind)
        if img.ndim == 2:
            img = img[:, :, None]
        bps = img.itemsize
        descs.append(isx.tile_desc(w, h, c, bps, bits, lv, qstep=q, pixel_offset=off))
        b = img.view(np.uint8).reshape(-1)
        chunks.append(b)
        off += len(b)
        pad = (-off) % 16
        chunks.append(np.zeros(pad, np.uint8))
        off += pad
        imgs.append((img, lv, bits, q))
    return imgs, descs, np.concatenate(chunks)


def test_encode_tiles_and_decode_tiles_direct_match_oracle():
    import torch
    imgs, descs, host_pix = _batch()
    print("boundary batch", [(d.width, d.height, d.channels, d.bits, d.levels, d.qstep) for d in descs],
          flush=True)
    d_pix = torch.from_numpy(host_pix).cuda()
    cap = isx.max_encoded_bytes(descs)
    d_out = torch.zeros(cap, dtype=torch.uint8, device="cuda")
    d_off = torch.zeros(len(descs), dtype=torch.int64, device="cuda")
    d_sz = torch.zeros(len(descs), dtype=torch.int64, device="cuda")
    d_st = torch.full((len(descs),), 1, dtype=torch.int32, device="cuda")
    d_ws = torch.empty(isx.encode_workspace_bytes(descs), dtype=torch.uint8, device="cuda")
    assert isx.encode_tiles(d_pix, descs, d_out, d_off, d_sz, d_st, d_ws) == isx.OK
    # a second call on the same buffers (the first call's plan bytes are released by then)
    assert isx.encode_tiles(d_pix, descs, d_out, d_off, d_sz, d_st, d_ws) == isx.OK
    torch.cuda.synchronize()
    assert d_st.cpu().tolist() == [0] * len(descs)
    off, sz = d_off.cpu().numpy(), d_sz.cpu().numpy()
    host = d_out.cpu().numpy()
    streams = [host[o:o + s].tobytes() for o, s in zip(off, sz)]
    for (img, lv, bits, q), blob in zip(imgs, streams):
        assert blob == oracle.encode_tile(img, lv, bits=bits, qstep=q)

    # decode every tile at full resolution and at its coarsest level, jobs built
    # from the library's header reader
    jobs, outs, o = [], [], 0
    for i, blob in enumerate(streams):
        d = isx.read_tile_header(blob)
        for z in sorted({0, d.levels}):
            ow, oh = isx.out_size(d.width, d.height, z)
            j = isx.DecodeJob()
            j.tile = d
            j.in_offset, j.in_bytes = int(off[i]), int(sz[i])
            j.out_offset, j.out_row_stride_bytes, j.target_level = o, ow * d.channels * d.bytes_per_sample, z
            jobs.append(j)
            outs.append((i, z, o, oh, ow, d.channels, d.bytes_per_sample))
            o += oh * ow * d.channels * d.bytes_per_sample
            o += (-o) % 16
    d_dec = torch.zeros(o, dtype=torch.uint8, device="cuda")
    d_dst = torch.full((len(jobs),), 1, dtype=torch.int32, device="cuda")
    d_dws = torch.empty(isx.decode_workspace_bytes(jobs), dtype=torch.uint8, device="cuda")
    assert isx.decode_tiles(d_out, jobs, d_dec, d_dst, d_dws) == isx.OK
    torch.cuda.synchronize()
    assert d_dst.cpu().tolist() == [0] * len(jobs)
    hd = d_dec.cpu().numpy()
    for i, z, o, oh, ow, c, bps in outs:
        got = hd[o:o + oh * ow * c * bps].view({1: np.uint8, 2: np.uint16}[bps]).reshape(oh, ow, c)
        assert np.array_equal(got, oracle.decode_tile(streams[i], z)), (i, z)
        if z == 0 and imgs[i][3] == 1:
            assert np.array_equal(got, imgs[i][0])


def test_convenience_calls_refuse_graph_capture_and_small_workspace():
    import torch
    imgs, descs, host_pix = _batch()
    d_pix = torch.from_numpy(host_pix).cuda()
    cap = isx.max_encoded_bytes(descs)
    d_out = torch.zeros(cap, dtype=torch.uint8, device="cuda")
    d_off = torch.zeros(len(descs), dtype=torch.int64, device="cuda")
    d_sz = torch.zeros(len(descs), dtype=torch.int64, device="cuda")
    d_st = torch.full((len(descs),), 1, dtype=torch.int32, device="cuda")
    need = isx.encode_workspace_bytes(descs)
    small = torch.empty(need - 256, dtype=torch.uint8, device="cuda")
    assert isx.encode_tiles(d_pix, descs, d_out, d_off, d_sz, d_st, small) == isx.E_WORKSPACE
    d_ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    rcs = []
    with torch.cuda.graph(g, stream=s):
        rcs.append(isx.encode_tiles(d_pix, descs, d_out, d_off, d_sz, d_st, d_ws))
    assert rcs == [isx.E_UNSUPPORTED]
    torch.cuda.synchronize()
    # the library still works normally afterwards
    assert isx.encode_tiles(d_pix, descs, d_out, d_off, d_sz, d_st, d_ws) == isx.OK
    torch.cuda.synchronize()
    assert d_st.cpu().tolist() == [0] * len(descs)


def _roundtrip_full_size(imgs_modes, levels, bits):
    """Encode the images as one batch (the launch shape bench.py times), then
    decode them as one batch; compare streams and pixels with the oracle."""
    import torch
    descs, chunks, off = [], [], 0
    for img, q in imgs_modes:
        h, w, c = img.shape
        descs.append(isx.tile_desc(w, h, c, img.itemsize, bits, levels, qstep=q, pixel_offset=off))
        chunks.append(img.view(np.uint8).reshape(-1))
        off += img.nbytes
    enc = isx.Encoder(descs)
    d_pix = torch.from_numpy(np.concatenate(chunks)).cuda()
    enc.run(d_pix)
    torch.cuda.synchronize()
    streams = enc.streams()
    offs = enc.offsets.cpu().numpy()
    jobs, o = [], 0
    for i, d in enumerate(descs):
        j = isx.DecodeJob()
        j.tile = d
        j.in_offset, j.in_bytes = int(offs[i]), len(streams[i])
        j.out_offset, j.out_row_stride_bytes = o, d.width * d.channels * d.bytes_per_sample
        jobs.append(j)
        o += d.width * d.height * d.channels * d.bytes_per_sample
    dec = isx.Decoder(jobs, o)
    dec.run(enc.out)
    torch.cuda.synchronize()
    assert dec.status.cpu().tolist() == [0] * len(jobs)
    host = dec.out.cpu().numpy()
    o = 0
    for (img, q), blob in zip(imgs_modes, streams):
        print("oracle", img.shape, img.dtype, "q", q, flush=True)
        ref = oracle.encode_tile(img, levels, bits=bits, qstep=q)
        assert blob == ref, "stream differs from the oracle"
        got = host[o:o + img.nbytes].view(img.dtype).reshape(img.shape)
        if q == 1:
            assert np.array_equal(got, img)
        else:
            assert np.array_equal(got, oracle.decode_tile(ref, 0))
        o += img.nbytes


def test_full_size_high_bit_depth_matches_oracle():
    """8192x8192 single-channel uint16 with 12 significant bits, 6 levels,
    lossless (the radiology-like workload): stream equal to the oracle's,
    decode equal to the input."""
    print("generating 8192x8192 12-bit image", flush=True)
    img = synth.rad_like(8192, 8192, 301)[:, :, None]
    _roundtrip_full_size([(img, 1)], 6, 12)


def test_full_size_rgb_both_modes_match_oracle():
    """4096x4096 RGB uint8 H&E-like region, 5 levels, lossless and step 4 in
    one batch (the benchmark's step): streams and pixels equal to the oracle."""
    print("generating 4096x4096 RGB image", flush=True)
    img = synth.he_like(4096, 4096, 201, sigma=(100.0, 600.0), tissue=0.40)
    _roundtrip_full_size([(img, 1), (img, 4)], 5, 8)
