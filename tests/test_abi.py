"""Host-side checks of the C-ABI library: it loads, exports every symbol the
header declares, and its pure host entry points validate and size correctly
(no device calls here)."""
import ctypes
import os
import re

import pytest

from paper_2005_08713_amd import isx

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    with open(os.path.join(ROOT, "include", "isx.h")) as f:
        text = f.read()
    return sorted(set(re.findall(r"\b(isx_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = isx.lib()
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n
    assert sorted(isx.EXPORTS) == names


def test_status_strings():
    assert isx.status_string(0) == "ok"
    assert "corrupt" in isx.status_string(-3)


def test_block_counts_match_oracle_geometry():
    import oracle
    for (w, h, c, lv) in [(1, 1, 1, 0), (256, 256, 3, 3), (257, 129, 3, 5), (4096, 4096, 3, 5),
                          (8192, 8192, 1, 6), (1, 300, 1, 6), (511, 3, 3, 4)]:
        d = isx.tile_desc(w, h, c, 1, 8, lv)
        assert isx.block_count(d) == oracle.lib().oracle_count_blocks(w, h, c, lv)


def test_host_validation_rejects_bad_descriptors():
    L = isx.lib()
    bad = [isx.tile_desc(0, 5, 1, 1, 8, 1), isx.tile_desc(5, 5, 65, 1, 8, 1),
           isx.tile_desc(5, 5, 1, 1, 9, 1), isx.tile_desc(5, 5, 1, 3, 8, 1),
           isx.tile_desc(5, 5, 1, 1, 8, 16), isx.tile_desc(5, 5, 2, 1, 8, 1, ct=1),
           isx.tile_desc(5, 5, 1, 1, 8, 1, qstep=0), isx.tile_desc(5, 5, 2, 1, 8, 1, ct=2),
           isx.tile_desc(5, 5, 3, 1, 8, 1, ct=3), isx.tile_desc(5, 5, 1, 4, 25, 1),
           isx.tile_desc(5, 5, 1, 2, 17, 1), isx.tile_desc(5, 5, 1, 4, 0, 1)]
    for d in bad:
        assert L.isx_encode_workspace_bytes(ctypes.byref(d), 1) == 0
        assert L.isx_max_encoded_bytes(ctypes.byref(d), 1) == 0
    d = isx.tile_desc(64, 64, 3, 1, 8, 3)
    assert L.isx_encode_workspace_bytes(ctypes.byref(d), 1) > 64 * 64 * 3 * 4
    # the widest accepted descriptors plan; misaligned 16/32-bit samples do not
    for ok in (isx.tile_desc(5, 5, 64, 1, 8, 2), isx.tile_desc(5, 5, 1, 4, 24, 2),
               isx.tile_desc(5, 5, 3, 2, 16, 2, ct=2)):
        assert L.isx_encode_plan_bytes(ctypes.byref(ok), 1) > 0
    for mis in (isx.tile_desc(5, 5, 1, 4, 24, 2, pixel_offset=2), isx.tile_desc(5, 5, 1, 2, 9, 1, row_stride=11)):
        assert L.isx_encode_plan_bytes(ctypes.byref(mis), 1) == 0
    j = isx.DecodeJob()
    j.tile, j.in_bytes, j.out_row_stride_bytes = isx.tile_desc(8, 8, 1, 2, 16, 1), 4096, 16
    arr = (isx.DecodeJob * 1)(j)
    assert L.isx_decode_plan_bytes(arr, 1) > 0
    for off, stride in ((1, 16), (0, 17)):
        arr[0].out_offset, arr[0].out_row_stride_bytes = off, stride
        assert L.isx_decode_plan_bytes(arr, 1) == 0
    # a call with a null device pointer fails on the host before any launch
    rc = L.isx_encode_tiles(ctypes.byref(d), 1, None, None, 0, None, None, None, None, 0, None)
    assert rc == isx.E_INVALID_ARG


def test_max_encoded_bytes_covers_oracle_output():
    import numpy as np
    import oracle
    from paper_2005_08713_amd import synth
    for (w, h, c, bits, lv, kind) in [(64, 64, 3, 8, 3, "uniform"), (33, 17, 1, 16, 6, "uniform"),
                                      (40, 9, 3, 8, 4, "checker")]:
        img = synth.random_image(w, h, c, bits, 3, kind)
        blob = oracle.encode_tile(img, lv, bits=bits)
        d = isx.tile_desc(w, h, c, img.itemsize, bits, lv)
        assert isx.lib().isx_max_encoded_bytes(ctypes.byref(d), 1) >= len(blob)


def test_stream_block_offsets_and_region_validation():
    """The host parser of a stream's size table, and the limits of region
    jobs, checked on the CPU (plans only, no device call)."""
    import numpy as np
    import oracle
    from paper_2005_08713_amd import synth
    L = isx.lib()
    img = synth.he_like(300, 200, 4)
    blob = oracle.encode_tile(img, 3)
    nb = int.from_bytes(blob[20:24], "little")
    offs = isx.stream_block_offsets(blob[:24 + 4 * nb])
    sizes = np.frombuffer(blob[24:24 + 4 * nb], np.uint32).astype(np.uint64)
    assert offs[0] == 24 + 4 * nb and offs[-1] == len(blob)
    assert np.array_equal(np.diff(offs), sizes)
    with pytest.raises(isx.IsxError):
        isx.stream_block_offsets(blob[:24 + 4 * nb - 1])
    with pytest.raises(isx.IsxError):
        isx.stream_block_offsets(b"JPEG" + blob[4:24 + 4 * nb])
    d = isx._parse_header(blob)

    def plan_bytes(z, x0, y0, w, h, stride=None):
        r = isx.region_job(d, offs, z, x0, y0, w, h)
        if stride is not None:
            r.job.out_row_stride_bytes = stride
        return L.isx_region_plan_bytes((isx.RegionJob * 1)(r), 1)

    assert plan_bytes(0, 0, 0, 300, 200) > 0
    assert plan_bytes(3, 37, 24, 1, 1) > 0
    assert plan_bytes(1, 149, 99, 1, 1) > 0
    for bad in [(0, 0, 0, 301, 200), (0, 300, 0, 1, 1), (1, 0, 0, 151, 1), (0, 5, 5, 0, 3), (4, 0, 0, 1, 1)]:
        assert plan_bytes(*bad) == 0, bad
    assert plan_bytes(0, 0, 0, 100, 100, stride=299) == 0
    r = isx.region_job(d, offs, 0, 0, 0, 10, 10)
    r.h_block_offsets = None
    assert L.isx_region_plan_bytes((isx.RegionJob * 1)(r), 1) == 0
    # a small region reads fewer blocks and a smaller workspace than the whole tile
    small = isx.region_job(d, offs, 0, 10, 10, 20, 20)
    whole = isx.region_job(d, offs, 0, 0, 0, 300, 200)
    assert L.isx_region_workspace_bytes((isx.RegionJob * 1)(small), 1) < \
        L.isx_region_workspace_bytes((isx.RegionJob * 1)(whole), 1)


def test_read_tile_header_matches_oracle_and_rejects_bad_heads():
    """isx_read_tile_header (host) returns the parameters the oracle wrote into
    the 24-byte header, a decodable `tile`, and rejects short, foreign and
    inconsistent heads without touching *out."""
    import numpy as np
    import oracle
    from paper_2005_08713_amd import synth
    L = isx.lib()
    cases = [(synth.he_like(70, 45, 3), 3, 8, None, 4),
             (synth.random_image(33, 17, 1, 12, 5, "uniform"), 6, 12, None, 1),
             (synth.random_image(9, 40, 3, 8, 6, "checker"), 2, 8, 2, 3)]
    for img, lv, bits, ct, q in cases:
        blob = oracle.encode_tile(img, lv, bits=bits, ct=ct, qstep=q)
        ref = oracle.read_header(blob)
        d = isx.read_tile_header(blob)
        assert (d.width, d.height, d.channels, d.bytes_per_sample, d.bits, d.levels,
                d.colour_transform, d.qstep) == (ref["width"], ref["height"], ref["channels"],
                                                 ref["bytes_per_sample"], ref["bits"], ref["levels"],
                                                 ref["ct"], ref["qstep"])
        assert d.pixel_offset == 0 and d.row_stride_bytes == d.width * d.channels * d.bytes_per_sample
        assert isx.block_count(d) == ref["nblocks"]
    blob = oracle.encode_tile(synth.he_like(40, 30, 1), 2)
    out = isx.TileDesc()
    out.width = 777

    def rc(head):
        b = np.frombuffer(bytes(head), np.uint8)
        return L.isx_read_tile_header(b.ctypes.data_as(ctypes.c_void_p), len(b), ctypes.byref(out))

    assert rc(blob[:23]) == isx.E_TRUNCATED
    assert rc(b"JPEG" + blob[4:24]) == isx.E_CORRUPT
    assert rc(blob[:4] + b"\x02" + blob[5:24]) == isx.E_CORRUPT            # version
    assert rc(blob[:20] + (12345).to_bytes(4, "little")) == isx.E_CORRUPT  # block count
    assert rc(blob[:6] + b"\x00" + blob[7:24]) == isx.E_CORRUPT            # zero channels
    assert out.width == 777
    assert L.isx_read_tile_header(None, 24, ctypes.byref(out)) == isx.E_INVALID_ARG


def test_noalloc_decode_validates_on_the_host():
    """isx_decode_run_noalloc refuses null pointers, a non-decode plan and a
    plan beyond its fixed workspace before touching the device."""
    L = isx.lib()
    d = isx.tile_desc(2048, 2048, 3, 1, 8, 5)
    j = isx.DecodeJob()
    j.tile, j.in_bytes, j.out_row_stride_bytes = d, 1 << 20, 2048 * 3
    arr = (isx.DecodeJob * 1)(j)
    pb = L.isx_decode_plan_bytes(arr, 1)
    plan = (ctypes.c_uint8 * pb)()
    assert L.isx_decode_plan_build(arr, 1, plan, pb) == isx.OK
    assert L.isx_decode_workspace_bytes(arr, 1) > isx.NOALLOC_SCRATCH_BYTES
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: every check here is on the host
    assert L.isx_decode_run_noalloc(plan, fake, fake, fake, fake, None) == isx.E_WORKSPACE
    assert L.isx_decode_run_noalloc(plan, None, fake, fake, fake, None) == isx.E_INVALID_ARG
    assert L.isx_decode_run_noalloc(None, fake, fake, fake, fake, None) == isx.E_INVALID_ARG
    e = isx.tile_desc(64, 64, 3, 1, 8, 3)
    eb = L.isx_encode_plan_bytes(ctypes.byref(e), 1)
    eplan = (ctypes.c_uint8 * eb)()
    assert L.isx_encode_plan_build(ctypes.byref(e), 1, eplan, eb) == isx.OK
    assert L.isx_decode_run_noalloc(eplan, fake, fake, fake, fake, None) == isx.E_INVALID_ARG


def test_tuning_ranges_are_checked_on_the_host():
    L = isx.lib()
    d = isx.tile_desc(64, 64, 3, 1, 8, 3)
    pb = L.isx_encode_plan_bytes(ctypes.byref(d), 1)
    buf = (ctypes.c_uint8 * pb)()
    for t, ok in [((32, 0, 0), True), ((32, 0, 11), True), ((16, 64, 1), True), ((32, 0, 12), False),
                  ((32, 0, -1), False), ((24, 0, 0), False), ((32, 65, 0), False), ((32, 0, 0, 1), True),
                  ((32, 0, 0, 2), True), ((32, 0, 0, 4), True), ((32, 0, 0, 3), False), ((32, 0, 0, 8), False),
                  ((32, 0, 0, -1), False)]:
        tu = isx.tuning(*t)
        rc = L.isx_encode_plan_build_tuned(ctypes.byref(d), 1, ctypes.byref(tu), buf, pb)
        assert (rc == isx.OK) == ok, t
