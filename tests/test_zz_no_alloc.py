"""GPU test of isx_decode_run_noalloc (the decode entry point that takes its
workspace from the library's fixed device array instead of an argument):
two calls in a row, the second with a smaller input, each equal to
isx_decode_run on the same plan and to the oracle.  Integer codec: every
comparison is exact."""
import numpy as np
import pytest

import oracle
from paper_2005_08713_amd import isx, synth

pytestmark = pytest.mark.gpu


def _jobs(streams, descs, offs, levels):
    jobs, shapes, o = [], [], 0
    for blob, d, off, z in zip(streams, descs, offs, levels):
        ow, oh = isx.out_size(d.width, d.height, z)
        j = isx.DecodeJob()
        j.tile = isx.read_tile_header(blob)
        j.in_offset, j.in_bytes = int(off), len(blob)
        j.out_offset, j.out_row_stride_bytes, j.target_level = o, ow * d.channels, z
        jobs.append(j)
        shapes.append((o, oh, ow, d.channels))
        o += oh * ow * d.channels
        o += (-o) % 16
    return jobs, shapes, o


def _case(imgs, levels, qsteps, targets):
    import torch
    descs, chunks, off = [], [], 0
    for img, lv, q in zip(imgs, levels, qsteps):
        h, w, c = img.shape
        descs.append(isx.tile_desc(w, h, c, 1, 8, lv, qstep=q, pixel_offset=off))
        chunks.append(img.reshape(-1))
        off += img.size
        pad = (-off) % 16
        chunks.append(np.zeros(pad, np.uint8))
        off += pad
    d_pix = torch.from_numpy(np.concatenate(chunks)).cuda()
    enc = isx.Encoder(descs)
    enc.run(d_pix)
    torch.cuda.synchronize()
    streams = enc.streams()
    for img, lv, q, blob in zip(imgs, levels, qsteps, streams):
        assert blob == oracle.encode_tile(img, lv, qstep=q)
    offs = enc.offsets.cpu().numpy()
    jobs, shapes, nbytes = _jobs(streams, descs, offs, targets)
    return enc, streams, jobs, shapes, nbytes


def _decode_both(enc, jobs, nbytes):
    import torch
    ref = isx.Decoder(jobs, nbytes)
    assert ref.ws_bytes <= isx.NOALLOC_SCRATCH_BYTES
    ref.run(enc.out)
    torch.cuda.synchronize()
    assert ref.status.cpu().tolist() == [0] * len(jobs)
    na = isx.Decoder(jobs, nbytes)
    na.out.fill_(0x5A)
    na.status.fill_(1)
    assert na.run_noalloc(enc.out) == isx.OK
    torch.cuda.synchronize()
    assert na.status.cpu().tolist() == [0] * len(jobs)
    return ref.out.cpu().numpy(), na.out.cpu().numpy()


def _check(streams, shapes, targets, a, b):
    for blob, (o, oh, ow, c), z in zip(streams, shapes, targets):
        n = oh * ow * c
        assert np.array_equal(a[o:o + n], b[o:o + n])
        assert np.array_equal(b[o:o + n].reshape(oh, ow, c), oracle.decode_tile(blob, z))


def test_noalloc_decode_matches_decode_run_twice_second_smaller():
    # first call: three tiles (lossless and step 3, full size and level 2)
    imgs = [synth.he_like(700, 530, 71), synth.he_like(301, 257, 72), synth.he_like(128, 128, 73)]
    levels, qsteps, targets = [4, 5, 3], [1, 3, 1], [0, 0, 2]
    print("noalloc call 1", [i.shape for i in imgs], flush=True)
    enc, streams, jobs, shapes, nbytes = _case(imgs, levels, qsteps, targets)
    a, b = _decode_both(enc, jobs, nbytes)
    _check(streams, shapes, targets, a, b)
    # second call, smaller input: one ragged tile, quantised, level 1
    imgs2 = [synth.he_like(131, 67, 74)]
    print("noalloc call 2", [i.shape for i in imgs2], flush=True)
    enc2, streams2, jobs2, shapes2, nbytes2 = _case(imgs2, [3], [4], [1])
    a2, b2 = _decode_both(enc2, jobs2, nbytes2)
    _check(streams2, shapes2, [1], a2, b2)


def test_noalloc_rejects_a_plan_beyond_its_workspace():
    import torch
    w = h = 2048  # a 2048x2048 RGB decode needs about 86 MB of workspace
    d = isx.tile_desc(w, h, 3, 1, 8, 5)
    j = isx.DecodeJob()
    j.tile, j.in_offset, j.in_bytes = d, 0, 1 << 20
    j.out_offset, j.out_row_stride_bytes, j.target_level = 0, w * 3, 0
    assert isx.decode_workspace_bytes([j]) > isx.NOALLOC_SCRATCH_BYTES
    dec = isx.Decoder([j], 16)
    src = torch.zeros(1 << 20, dtype=torch.uint8, device="cuda")
    assert dec.run_noalloc(src) == isx.E_WORKSPACE
    torch.cuda.synchronize()
    assert dec.status.cpu().tolist() == [1]  # nothing was launched
