// isx_common.h -- internal data layout of libisx (device + host).
//
// Plan = host-built description of a batch of tiles (encode) or decode jobs:
// a PlanHdr, one TileGeo per tile/job and per-level work lists.  It is copied
// to the device once per call (or once per replayed shape) and the kernels
// derive every block's geometry from it.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace isx {

constexpr int kBlock = 128;        // Sec. 4: wavelet data partitioned in 128x128 blocks
constexpr int kMaxLevels = 15;
constexpr int kMaxChannels = 64;
constexpr int kMaxPlanes = 31;     // d is a 5-bit field; magnitudes < 2^30
constexpr int kNumWz = 14;         // counter widths 2..15 tracked per segment
constexpr uint32_t kPlanMagic = 0x4e4c5058u;  // "XPLN"

enum { MODE_ENCODE = 0, MODE_DECODE = 1 };

struct LevelGeo {          // level l (1..levels) of a tile
    uint32_t w, h;         // size of LL_{l-1}, the input of level l
    uint32_t gx, gy;       // H-block grid over ceil(w/2) x ceil(h/2)
    uint32_t corner_empty; // the last grid cell (per channel) has no coefficient
    uint32_t blocks_per_chan;
    uint32_t group_start;  // first tile-local block index of this level's H-blocks
    uint32_t pitch[3];     // element pitch of the LH, HL, HH bands (type order)
    uint32_t pad;
    uint64_t off[3];       // int32-element offset of LH, HL, HH of channel 0 from ws base
    // decode: the part of this level's bands held in the arena (band
    // coordinates, block aligned), the same window for LL_l, LH, HL and HH;
    // the whole band for a full decode, a region's halo cover otherwise
    uint32_t wx0, wy0, ww, wh;
};

struct TileGeo {
    uint64_t pix_offset;   // encode: input pixels; decode: output pixels (bytes)
    uint32_t pix_stride;   // bytes per row
    uint32_t width, height;
    uint8_t channels, bps, bits, levels;
    uint8_t ct, target_level, dmax, first_level;  // first_level: lowest level reconstructed
    uint8_t coef16;        // bit l-1: level l's LH, HL, HH held as int16 in their (int32-sized) arena regions (l <= 2)
    uint8_t pad8[3];
    uint32_t qstep;
    uint32_t qmul, qsh;    // n / qstep = (t + ((n - t) >> 1)) >> qsh, t = mulhi(qmul, n), for qstep > 1
    uint64_t enc_offset;   // decode: encoded tile offset in d_encoded
    uint64_t enc_bytes;    // decode: bytes available
    uint64_t chan_elems;   // int32 elements between channels of the coefficient arena
    uint64_t tmp_off[2];   // int32-element offsets of the LL ping-pong buffers (odd, even levels)
    uint64_t tmp_chan[2];  // elements between channels in each ping-pong buffer
    uint32_t tmp_pitch[2];
    uint64_t ll_off;       // int32-element offset of LL_levels (channel 0)
    uint32_t ll_pitch, ll_w, ll_h, ll_gx, ll_gy;
    uint32_t block_base;   // first global block index of this tile/job
    uint32_t nblocks;      // blocks handled in this call (decode: prefix to target level)
    uint32_t nblocks_stream;  // blocks of the complete stream
    uint32_t slot_base;    // first global plane slot
    uint32_t drop;         // decode: magnitude planes left out (quality-progressive)
    uint64_t sym_base;     // byte offset of this tile's symbol area (ws)
    // decode: output region [rx0, rx1) x [ry0, ry1) of the level-z image
    // (the whole image for a full decode), window origin of the LL_levels
    // arena, and the plan offset of the selected-block list (0: the blocks
    // are the stream prefix 0 .. nblocks-1)
    uint32_t rx0, ry0, rx1, ry1;
    uint32_t ll_wx0, ll_wy0;
    uint64_t sel_off;
    LevelGeo lv[kMaxLevels + 1];  // index 1..levels
};

struct WorkItem {          // transform work: one tile at one level
    uint32_t tile;
    uint32_t wg_start;     // first workgroup index of this item
    uint32_t ntx, nty;     // spatial tiles
    uint32_t nch;          // channel groups (workgroups per spatial tile)
    uint32_t qx0, qy0;     // decode: quad origin of the first spatial tile
    uint32_t pad;
};

struct SelBlock {          // a block of a region decode: stream index, bytes
    uint32_t local;        // index in the tile's block order
    uint32_t len;          // its byte length (checked against the stream)
    uint64_t off;          // its byte offset from the stream start
};

struct PlanHdr {
    uint32_t magic, mode, n_tiles, total_blocks;
    uint32_t total_slots, max_levels, max_nblocks, max_dmax;  // max_dmax: largest plane bound of any tile
    uint64_t plan_bytes;
    uint64_t ws_bytes;
    // workspace regions (byte offsets from ws base)
    uint64_t ws_blockdesc, ws_acc, ws_seghist, ws_segstat, ws_blkstat, ws_blkplan, ws_tileout,
        ws_lut, ws_items;
    // plan regions (byte offsets from plan base)
    uint64_t tiles_off, work_off;
    uint32_t lvl_first[kMaxLevels + 2];  // per level: first WorkItem index
    uint32_t lvl_count[kMaxLevels + 2];  // per level: number of WorkItems
    uint32_t lvl_wgs[kMaxLevels + 2];    // per level: total workgroups
    uint32_t fin_first, fin_count, fin_wgs, pad1;  // decode: final-output work list
    uint32_t tq;        // transform tile: quads per side (16 or 32)
    uint32_t blk_grid;  // workgroups of the per-block kernels (== total_blocks unless persistent)
    uint32_t num_cus, blocks_per_cu;
    uint32_t seg_waves_per_cu;  // segment decoder: persistent waves per CU
    uint32_t seg_nw;            // segment decoder: waves per workgroup (1, 2 or 4)
    uint32_t seg_big_bits;      // segment decoder: a segment of at least this many bits is a large item
    uint32_t seg_whole_words;   // segment decoder: staging words of a whole-block item (0 = none)
    uint32_t pack_nw;           // packer: waves per item (1, or 4 for plans of few segments)
    uint64_t list_off;      // plan offset of the block list (u32): large blocks, then small ones
    uint32_t n_big, n_small;  // blocks with > 768 4x4 cells / with <= 768
};

struct BlockDesc {
    uint32_t tile;
    uint32_t local;        // index within the tile's stream
    uint8_t level, chan, p, drop;  // drop: decode, magnitude planes left out
    uint16_t bx, by;
    uint16_t wb, hb;       // padded block size (multiples of 4, <= 128)
    uint8_t tw[3], th[3];  // extent of each type inside the cell (<= 128)
    uint8_t c16;           // coefficients held as int16: off[] counts int16 elements
    uint8_t pad1;
    uint32_t pitch[3];
    uint64_t off[3];       // int32-element offset of each type's cell origin (ws)
    uint64_t sym_off;      // byte offset of the block's symbols (ws)
    uint32_t slot;         // first plane slot
    uint32_t dmax;
    uint64_t byte_off;     // decode: absolute byte offset of the block in d_encoded
    uint32_t byte_len;     // decode: block length in bytes
    uint32_t pad2;
};

struct BlkAcc {            // filled by the forward transform (atomicOr)
    uint32_t or_mag[3];    // OR of |q| per type
    uint32_t neg;          // bit t: type t has a negative coefficient
};

struct SegStat {           // per (block, plane)
    uint32_t zir;          // zeros inside runs (length >= 2)
    uint32_t dig[kNumWz];  // sum over runs of the digit count for wz = 2 + i
    uint32_t pad;
};

struct BlkStat {
    uint32_t F[16];        // maximal zero runs with bit length i
    uint32_t nruns;
    uint32_t err;
    uint32_t pad[2];
};

struct BlkPlan {
    uint32_t code[256];
    uint8_t len[256];
    uint8_t order[256];    // symbols in canonical (length, symbol) order
    uint32_t m;            // leaves of the code
    uint32_t d, czr, wz, nseg, tbits, p, n;
    uint32_t masks[3];
    uint32_t hdr_bits;
    uint32_t bytes;
    uint32_t limited;
    uint32_t err;
    uint32_t pad;
    uint8_t seg_plane[32];
    uint32_t seg_bits[32];
    uint32_t seg_M[32];
    uint64_t byte_off;     // within the tile stream
    uint64_t seg_bitpos[32];  // decode: absolute bit position of each segment
};

// decode code tables, per block: prefix table of 2^kLutK uint16 entries, then
// the left-aligned codes (uint32[256]), lengths and symbols (uint8[256] each)
constexpr int kLutK = 10;
constexpr uint32_t kLutBytes16 = (1u << kLutK) * 2;
constexpr uint32_t kLutStride = kLutBytes16 + 1024 + 256 + 256;
constexpr uint32_t kMaxSeg = 3 * 128 * 128 / 8;  // symbols in the largest segment
constexpr uint32_t kSegWords = 1662;             // segment bits staged in LDS, 53 Kbit (larger: read from HBM)
constexpr uint32_t kHalfWords = 480;             // the same, per wave, where two waves split a workgroup's LDS
constexpr uint32_t kBigSegBits = 16384;          // queue class of a segment
constexpr uint32_t kSmallSegBits = 4096;         // a block of only such segments is one decode item
constexpr uint32_t kWholeBlock = 31;             // segment field of such an item (segments are 0..30)
constexpr uint32_t kSegWavesPerCu = 11;  // one-wave workgroups of 14.5 KB LDS each
// Segment work queue header: the large-list length, the small-list length
// and the take counter, each in a 128-byte line of its own (atomics of
// thousands of waves on one shared line contend); the lists follow.
constexpr uint32_t kQBig = 0, kQSmall = 32, kQTake = 64, kItemsHdr = 384;
struct TileOut {
    uint64_t size;
    uint64_t offset;
    int32_t status;
    uint32_t pad[3];
};

// ---------------------------------------------------------------- helpers
__host__ __device__ inline uint32_t div_up(uint32_t a, uint32_t b) { return (a + b - 1) / b; }
__host__ __device__ inline uint32_t round4(uint32_t a) { return (a + 3u) & ~3u; }
// Hand-over between the lanes of a one-wave workgroup through LDS: the LDS
// operations of a wave take effect in program order, so keeping the compiled
// accesses in order is all it needs (no wait for memory, no barrier).
__device__ inline void wave_sync() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); }

__host__ __device__ inline uint32_t bitlen32(uint32_t v) { return v ? 32u - (uint32_t)__builtin_clz(v) : 0u; }
// Bytes between the bitplanes of a block's symbol area (p*n symbols per
// plane, padded to 16 bytes so each plane is written with 16-byte stores).
__host__ __device__ inline uint32_t plane_stride(uint32_t pn) { return (pn + 15u) & ~15u; }
__host__ __device__ inline uint64_t block_sym_bytes(const BlockDesc &B, uint32_t dmax)
{
    return (uint64_t)plane_stride((uint32_t)B.p * B.wb * B.hb / 8) * dmax;
}

// Geometry of tile-local block `local` (Sec. 4 blocks; group order LL, then
// H-blocks of level L .. 1; channel-major, then raster; the empty corner cell
// of a level is skipped).
__host__ __device__ inline void block_geometry(const TileGeo &T, uint32_t local, BlockDesc &B)
{
    uint32_t nll = T.ll_gx * T.ll_gy;
    B.local = local;
    B.c16 = 0;
    if (local < nll * T.channels) {
        uint32_t c = local / nll, r = local % nll;
        uint32_t by = r / T.ll_gx, bx = r % T.ll_gx;
        uint32_t cw = T.ll_w - bx * kBlock; if (cw > (uint32_t)kBlock) cw = kBlock;
        uint32_t ch = T.ll_h - by * kBlock; if (ch > (uint32_t)kBlock) ch = kBlock;
        B.level = 0; B.chan = (uint8_t)c; B.p = 1; B.bx = (uint16_t)bx; B.by = (uint16_t)by;
        B.wb = (uint16_t)round4(cw); B.hb = (uint16_t)round4(ch);
        B.tw[0] = (uint8_t)(cw & 0xff); B.th[0] = (uint8_t)(ch & 0xff);
        B.tw[1] = B.th[1] = B.tw[2] = B.th[2] = 0;
        if (cw == 128) B.tw[0] = 128;
        if (ch == 128) B.th[0] = 128;
        B.pitch[0] = T.ll_pitch; B.pitch[1] = B.pitch[2] = 0;
        B.off[0] = T.ll_off + (uint64_t)c * T.chan_elems + (uint64_t)(by * kBlock - T.ll_wy0) * T.ll_pitch +
                   (bx * kBlock - T.ll_wx0);
        B.off[1] = B.off[2] = 0;
        return;
    }
    uint32_t l = T.levels;
    for (; l >= 1; l--) {
        const LevelGeo &G = T.lv[l];
        if (local < G.group_start + G.blocks_per_chan * T.channels) break;
    }
    const LevelGeo &G = T.lv[l];
    uint32_t r0 = local - G.group_start;
    uint32_t c = r0 / G.blocks_per_chan, r = r0 % G.blocks_per_chan;
    uint32_t by = r / G.gx, bx = r % G.gx;
    uint32_t gw = (G.w + 1) / 2, gh = (G.h + 1) / 2, hw = G.w / 2, hh = G.h / 2;
    uint32_t cw = gw - bx * kBlock; if (cw > (uint32_t)kBlock) cw = kBlock;
    uint32_t ch = gh - by * kBlock; if (ch > (uint32_t)kBlock) ch = kBlock;
    int32_t hwc = (int32_t)hw - (int32_t)(bx * kBlock); if (hwc < 0) hwc = 0; if (hwc > kBlock) hwc = kBlock;
    int32_t hhc = (int32_t)hh - (int32_t)(by * kBlock); if (hhc < 0) hhc = 0; if (hhc > kBlock) hhc = kBlock;
    B.level = (uint8_t)l; B.chan = (uint8_t)c; B.p = 3; B.bx = (uint16_t)bx; B.by = (uint16_t)by;
    B.wb = (uint16_t)round4(cw); B.hb = (uint16_t)round4(ch);
    uint32_t tw[3] = {cw, (uint32_t)hwc, (uint32_t)hwc};
    uint32_t th[3] = {(uint32_t)hhc, ch, (uint32_t)hhc};
    const bool c16 = l <= 2 && ((T.coef16 >> (l - 1)) & 1u);  // the level's bands held as int16
    for (int t = 0; t < 3; t++) {
        B.tw[t] = (uint8_t)(tw[t] >= 128 ? 128 : tw[t]);
        B.th[t] = (uint8_t)(th[t] >= 128 ? 128 : th[t]);
        B.pitch[t] = G.pitch[t];
        const uint64_t band = G.off[t] + (uint64_t)c * T.chan_elems;  // int32 elements
        const uint64_t org = (uint64_t)(by * kBlock - G.wy0) * G.pitch[t] + (bx * kBlock - G.wx0);
        B.off[t] = c16 ? 2 * band + org : band + org;
    }
    B.c16 = c16 ? 1 : 0;
}

// The 8 XCDs of the chip receive a launch's workgroups round-robin, and each
// has its own L2.  Remapping the workgroup index this way gives every XCD one
// contiguous range of the logical grid, so neighbouring tiles (which share
// halo cache lines) and the channels of one tile run behind the same L2.
constexpr uint32_t kXcds = 8;
__device__ inline uint32_t xcd_remap(uint32_t b, uint32_t n)
{
    const uint32_t per = n / kXcds, rem = n % kXcds, x = b % kXcds;
    return x * per + (x < rem ? x : rem) + b / kXcds;
}

// Whole-sample symmetric extension of index i into [0, n).
__host__ __device__ inline int reflect_idx(int i, int n)
{
    if (n <= 1) return 0;
    int per = 2 * n - 2;
    i %= per;
    if (i < 0) i += per;
    return i >= n ? per - i : i;
}

// ---------------------------------------------------------------- stages
enum EncStage {
    ENC_PREP = 0,
    ENC_FWD0 = 1,  // forward level l is stage ENC_FWD0 + l (l = 0..15)
    ENC_SYM = ENC_FWD0 + kMaxLevels + 1,
    ENC_CODE,
    ENC_BOFF,
    ENC_TOFF,
    ENC_FIN,
    ENC_PACK,
    ENC_NSTAGES
};
enum DecStage {
    DEC_PREP = 0,
    DEC_HDR,
    DEC_SEG,
    DEC_REASM,
    DEC_INV15,                     // inverse of level 15 .. level 2 (intermediate outputs)
    DEC_FINAL = DEC_INV15 + kMaxLevels,  // inverse of level z+1 fused with the output stage
    DEC_NSTAGES
};

// ---------------------------------------------------------------- launchers
// (defined in the .hip files; all asynchronous on `stream`)
hipError_t launch_encode(const PlanHdr &H, const uint8_t *d_plan, const uint8_t *d_pixels,
                         uint8_t *d_out, uint64_t out_capacity, uint64_t *d_tile_offsets,
                         uint64_t *d_tile_sizes, int32_t *d_status, uint8_t *d_ws,
                         hipStream_t stream, int first, int last);
hipError_t launch_forward_only(const PlanHdr &H, const uint8_t *d_plan, const uint8_t *d_pixels,
                               uint8_t *d_ws, hipStream_t stream);
hipError_t launch_decode(const PlanHdr &H, const uint8_t *d_plan, const uint8_t *d_encoded,
                         uint8_t *d_pixels_out, int32_t *d_status, uint8_t *d_ws,
                         hipStream_t stream, int first, int last);
hipError_t launch_debug_huffman(const uint32_t *d_freq, int limit, uint8_t *d_len,
                                hipStream_t stream);

}  // namespace isx
