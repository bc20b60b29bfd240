// isx_api.hip -- host side of libisx: argument validation, planning
// (geometry, workspace layout, work lists) and the C ABI of include/isx.h.
#include <string.h>

#include <mutex>
#include <vector>

#include "isx.h"
#include "isx_common.h"

using namespace isx;

namespace {

constexpr uint64_t kAlign = 256;
constexpr uint64_t kPlanRegion = 1ull << 20;  // plan copy kept at the start of the workspace (convenience API)

uint64_t al(uint64_t v, uint64_t a = kAlign) { return (v + a - 1) / a * a; }

int validate_desc(const isx_tile_desc &d)
{
    if (d.width < 1 || d.height < 1 || d.width > 65535 || d.height > 65535) return ISX_E_INVALID_ARG;
    if (d.channels < 1 || d.channels > kMaxChannels) return ISX_E_INVALID_ARG;
    if (d.bytes_per_sample != 1 && d.bytes_per_sample != 2 && d.bytes_per_sample != 4) return ISX_E_INVALID_ARG;
    // 4-byte samples carry at most 24 bits: every coefficient then fits 32 bits
    if (d.bits < 1 || d.bits > (d.bytes_per_sample == 4 ? 24 : 8 * d.bytes_per_sample)) return ISX_E_INVALID_ARG;
    if (d.levels > kMaxLevels) return ISX_E_INVALID_ARG;
    if (d.colour_transform > ISX_CT_YCOCG) return ISX_E_INVALID_ARG;
    if (d.colour_transform != ISX_CT_NONE && d.channels != 3) return ISX_E_INVALID_ARG;
    if (d.qstep < 1) return ISX_E_INVALID_ARG;
    return ISX_OK;
}

// Magnitude bound of level l's high-pass outputs (the recursion below).
double highpass_bound(uint32_t bits, uint32_t level)
{
    const double M0 = (double)((1u << bits) - 1);
    double A = M0, e = 0.0, h = 0.0;
    for (uint32_t l = 1; l <= level; l++) {
        h = 4.0 * A + 2.0;
        e = 2.25 * e + 2.5;
        A = 2.9584 * M0 + e;
    }
    return h;
}

// Upper bound of the number of bitplanes d of any block (1 + bit length of
// the largest coefficient magnitude).  With M0 = 2^bits - 1 bounding every
// colour-transformed sample: the integer LL of level l stays within
// 1.72^2 M0 (L1 norm of the iterated 2-D 5/3 low-pass, < 1.7157^2 for every
// depth) plus an accumulated rounding error e_l <= 2.25 e_{l-1} + 2.5; a
// level's high-pass outputs are at most 4 A + 2 for inputs bounded by A.
uint32_t dmax_bound(uint32_t bits, uint32_t levels)
{
    double M0 = (double)((1u << bits) - 1);
    double A = M0, e = 0.0, mx = M0;
    for (uint32_t l = 1; l <= levels; l++) {
        double h = 4.0 * A + 2.0;
        if (h > mx) mx = h;
        e = 2.25 * e + 2.5;
        A = 2.9584 * M0 + e;
        if (A > mx) mx = A;
    }
    uint64_t m = (uint64_t)mx + 1;
    uint32_t d = 1;
    while (m) { d++; m >>= 1; }
    if (d > (uint32_t)kMaxPlanes) d = kMaxPlanes;
    return d;
}

struct TileBuild {
    TileGeo g;
    uint64_t arena_elems = 0, tmp_elems[2] = {0, 0}, sym_bytes = 0;
    std::vector<SelBlock> sel;  // region decode: the blocks it reads, in stream order
    // decode: range [kx0, kx1) x [ky0, ky1) of LL_k needed, k = z .. levels
    uint32_t kx0[kMaxLevels + 1] = {}, kx1[kMaxLevels + 1] = {}, ky0[kMaxLevels + 1] = {},
             ky1[kMaxLevels + 1] = {};
};

struct RegionIn {           // region decode: [x0, x1) x [y0, y1) of the level-z image
    uint32_t x0, y0, x1, y1;
    const uint64_t *offs;   // byte offset of every block, then the stream length
};

// Geometry of one tile; offsets are relative (filled in later).  For a
// decode to level z it also fixes the arena windows: the whole bands, or for
// a region the blocks under its halo at every level.
int tile_geometry(const isx_tile_desc &d, int target_level, TileBuild &tb, const RegionIn *reg = nullptr)
{
    TileGeo &T = tb.g;
    memset(&T, 0, sizeof(T));
    tb.arena_elems = 0; tb.tmp_elems[0] = tb.tmp_elems[1] = 0; tb.sym_bytes = 0;
    tb.sel.clear();
    memset(tb.kx0, 0, sizeof(tb.kx0)); memset(tb.kx1, 0, sizeof(tb.kx1));
    memset(tb.ky0, 0, sizeof(tb.ky0)); memset(tb.ky1, 0, sizeof(tb.ky1));
    T.pix_offset = d.pixel_offset;
    T.pix_stride = d.row_stride_bytes;
    T.width = d.width; T.height = d.height;
    T.channels = d.channels; T.bps = d.bytes_per_sample; T.bits = d.bits; T.levels = d.levels;
    T.ct = d.colour_transform; T.target_level = (uint8_t)target_level; T.qstep = d.qstep;
    {   // division by the invariant step (Granlund and Montgomery 1994): with
        // l = ceil(log2 step), qmul = floor(2^32 (2^l - step) / step) + 1
        uint32_t l = 0;
        while ((1ull << l) < d.qstep) l++;
        T.qmul = (uint32_t)(((1ull << 32) * ((1ull << l) - d.qstep)) / d.qstep + 1);
        T.qsh = l ? l - 1 : 0;
    }
    T.dmax = (uint8_t)dmax_bound(d.bits, d.levels);
    T.first_level = (uint8_t)(target_level + 1);
    uint32_t w = d.width, h = d.height;
    for (uint32_t l = 1; l <= d.levels; l++) {
        T.lv[l].w = w; T.lv[l].h = h;
        w = (w + 1) / 2; h = (h + 1) / 2;
    }
    T.ll_w = w; T.ll_h = h;
    T.ll_gx = div_up(w, kBlock); T.ll_gy = div_up(h, kBlock);
    uint32_t start = T.ll_gx * T.ll_gy * d.channels;
    uint32_t prefix_needed = start;  // blocks needed for target level
    for (uint32_t l = d.levels; l >= 1; l--) {
        LevelGeo &G = T.lv[l];
        uint32_t gw = (G.w + 1) / 2, gh = (G.h + 1) / 2, hw = G.w / 2, hh = G.h / 2;
        G.gx = div_up(gw, kBlock); G.gy = div_up(gh, kBlock);
        uint32_t bx = G.gx - 1, by = G.gy - 1;
        G.corner_empty = ((int64_t)hw - (int64_t)bx * kBlock <= 0) && ((int64_t)hh - (int64_t)by * kBlock <= 0);
        G.blocks_per_chan = G.gx * G.gy - G.corner_empty;
        G.group_start = start;
        start += G.blocks_per_chan * d.channels;
        if ((int)l > target_level) prefix_needed = start;
    }
    T.nblocks_stream = start;
    T.nblocks = prefix_needed;
    // windows.  K_k is the range of LL_k the decode needs (k = z: the
    // output).  Undoing level k at sample n reads band samples floor(n/2)-1
    // .. floor(n/2)+1 (Sec. 3: the 5/3 lifting steps reach one neighbour
    // each); K_k keeps one more on either side.  The window of level k is
    // K_k widened to whole 128-blocks.
    const uint32_t z = (uint32_t)target_level, L = d.levels;
    auto ll_size = [&](uint32_t k, bool xdim) -> uint32_t {
        if (k == 0) return xdim ? T.width : T.height;
        if (k < L) return xdim ? T.lv[k + 1].w : T.lv[k + 1].h;
        return xdim ? T.ll_w : T.ll_h;
    };
    uint32_t a0 = reg ? reg->x0 : 0, a1 = reg ? reg->x1 : ll_size(z, true);
    uint32_t b0 = reg ? reg->y0 : 0, b1 = reg ? reg->y1 : ll_size(z, false);
    T.rx0 = a0; T.rx1 = a1; T.ry0 = b0; T.ry1 = b1;
    tb.kx0[z] = a0; tb.kx1[z] = a1; tb.ky0[z] = b0; tb.ky1[z] = b1;
    auto cover = [](uint32_t lo, uint32_t hi, uint32_t n, uint32_t &o, uint32_t &len) {
        o = lo / kBlock * kBlock;
        uint32_t e = div_up(hi, kBlock) * kBlock;
        len = (e < n ? e : n) - o;
    };
    for (uint32_t k = z + 1; k <= L; k++) {
        const uint32_t nx = ll_size(k, true), ny = ll_size(k, false);
        a0 = a0 / 2 >= 2 ? a0 / 2 - 2 : 0; a1 = a1 / 2 + 2 < nx ? a1 / 2 + 2 : nx;
        b0 = b0 / 2 >= 2 ? b0 / 2 - 2 : 0; b1 = b1 / 2 + 2 < ny ? b1 / 2 + 2 : ny;
        tb.kx0[k] = a0; tb.kx1[k] = a1; tb.ky0[k] = b0; tb.ky1[k] = b1;
        LevelGeo &G = T.lv[k];
        cover(a0, a1, nx, G.wx0, G.ww);
        cover(b0, b1, ny, G.wy0, G.wh);
    }
    uint32_t ll_ww, ll_wh;
    if (L > z) {
        T.ll_wx0 = T.lv[L].wx0; T.ll_wy0 = T.lv[L].wy0; ll_ww = T.lv[L].ww; ll_wh = T.lv[L].wh;
    } else {
        cover(a0, a1, T.ll_w, T.ll_wx0, ll_ww);
        cover(b0, b1, T.ll_h, T.ll_wy0, ll_wh);
    }
    // per-channel arena layout (int32 elements); a decode to level z only
    // needs the bands of levels z+1 .. L
    uint64_t off = 0;
    T.ll_pitch = round4(ll_ww);
    T.ll_off = off;
    off = al(off + (uint64_t)T.ll_pitch * ll_wh, 64);
    for (uint32_t l = z + 1; l <= L; l++) {
        LevelGeo &G = T.lv[l];
        uint32_t bw[3] = {(G.w + 1) / 2, G.w / 2, G.w / 2};
        uint32_t bh[3] = {G.h / 2, (G.h + 1) / 2, G.h / 2};
        for (int t = 0; t < 3; t++) {
            if (reg) { G.pitch[t] = round4(G.ww); bh[t] = G.wh; }
            else G.pitch[t] = round4(bw[t] ? bw[t] : 1);
            G.off[t] = off;
            off = al(off + (uint64_t)G.pitch[t] * bh[t], 64);
        }
    }
    T.chan_elems = al(off, 64);
    tb.arena_elems = T.chan_elems * d.channels;
    // LL ping-pong for the intermediate LL_k, k in [z+1, L-1] (held in the
    // window of level k): odd k in buffer 0, even k in buffer 1, each sized
    // for the largest window of its parity
    for (uint32_t k = z + 1; k + 1 <= L; k++) {
        int which = (k & 1) ? 0 : 1;
        uint32_t p = round4(T.lv[k].ww);
        if (p > T.tmp_pitch[which]) T.tmp_pitch[which] = p;
    }
    for (uint32_t k = z + 1; k + 1 <= L; k++) {
        int which = (k & 1) ? 0 : 1;
        uint64_t e = al((uint64_t)T.tmp_pitch[which] * T.lv[k].wh, 64);
        if (e > T.tmp_chan[which]) T.tmp_chan[which] = e;
    }
    for (int which = 0; which < 2; which++) tb.tmp_elems[which] = T.tmp_chan[which] * d.channels;
    // region decode: the blocks under the windows, in stream order
    if (reg) {
        std::vector<uint32_t> locals;
        const uint32_t nll = T.ll_gx * T.ll_gy;
        for (uint32_t c = 0; c < d.channels; c++)
            for (uint32_t by = T.ll_wy0 / kBlock; by < div_up(T.ll_wy0 + ll_wh, kBlock); by++)
                for (uint32_t bx = T.ll_wx0 / kBlock; bx < div_up(T.ll_wx0 + ll_ww, kBlock); bx++)
                    locals.push_back(c * nll + by * T.ll_gx + bx);
        for (uint32_t l = L; l > z; l--) {
            const LevelGeo &G = T.lv[l];
            for (uint32_t c = 0; c < d.channels; c++)
                for (uint32_t by = G.wy0 / kBlock; by < div_up(G.wy0 + G.wh, kBlock); by++)
                    for (uint32_t bx = G.wx0 / kBlock; bx < div_up(G.wx0 + G.ww, kBlock); bx++) {
                        if (G.corner_empty && bx == G.gx - 1 && by == G.gy - 1) continue;
                        locals.push_back(G.group_start + c * G.blocks_per_chan + by * G.gx + bx);
                    }
        }
        tb.sel.clear();
        for (uint32_t local : locals) {
            const uint64_t o = reg->offs[local], e = reg->offs[local + 1];
            if (e < o || e - o > 0xffffffffull) return ISX_E_INVALID_ARG;
            tb.sel.push_back({local, (uint32_t)(e - o), o});
        }
        T.nblocks = (uint32_t)tb.sel.size();
    }
    // symbols
    uint64_t sb = 0;
    for (uint32_t i = 0; i < T.nblocks; i++) {
        BlockDesc B;
        block_geometry(T, reg ? tb.sel[i].local : i, B);
        sb += block_sym_bytes(B, T.dmax);
    }
    tb.sym_bytes = sb;
    return ISX_OK;
}

// A plan: the header, and the plan bytes in `bytes`, or written straight
// into a caller's buffer (dst, cap), or not at all (sizes only).
struct Plan {
    std::vector<uint8_t> bytes;
    PlanHdr H;
    uint8_t *dst = nullptr;
    uint64_t cap = 0;
    bool sizes_only = false;
    bool wide_coeffs = false;  // keep every band int32 (coefficient dumps)
};

int device_cus()
{
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) return 256;
    return v;
}

int build_plan(int mode, const isx_tile_desc *descs, const isx_decode_job *jobs, int32_t n, Plan &P,
               const isx_tuning *tune = nullptr, const isx_region_job *regions = nullptr)
{
    if (mode == MODE_DECODE && !jobs && !regions) return ISX_E_INVALID_ARG;
    auto job_at = [&](int32_t i) -> const isx_decode_job & { return regions ? regions[i].job : jobs[i]; };
    if (n < 1) return ISX_E_INVALID_ARG;
    // per-thread scratch kept between calls: planning large batches often
    // (a serving loop) then touches no fresh pages
    static thread_local std::vector<TileBuild> tls_tb;
    static thread_local std::vector<WorkItem> tls_items;
    static thread_local std::vector<uint32_t> tls_big, tls_small;
    if (tls_tb.size() < (size_t)n) tls_tb.resize((size_t)n);
    TileBuild *tb = tls_tb.data();
    PlanHdr &H = P.H;
    memset(&H, 0, sizeof(H));
    H.magic = kPlanMagic;
    H.mode = (uint32_t)mode;
    H.n_tiles = (uint32_t)n;
    H.tq = 32;
    H.blocks_per_cu = 0;
    H.seg_waves_per_cu = kSegWavesPerCu;
    if (tune) {
        if (tune->transform_tile != 0 && tune->transform_tile != 16 && tune->transform_tile != 32)
            return ISX_E_INVALID_ARG;
        if (tune->blocks_per_cu < 0 || tune->blocks_per_cu > 64) return ISX_E_INVALID_ARG;
        if (tune->seg_waves_per_cu < 0 || tune->seg_waves_per_cu > (int32_t)kSegWavesPerCu) return ISX_E_INVALID_ARG;
        if (tune->seg_waves_per_cu) H.seg_waves_per_cu = (uint32_t)tune->seg_waves_per_cu;
        if (tune->seg_wave_group != 0 && tune->seg_wave_group != 1 && tune->seg_wave_group != 2 &&
            tune->seg_wave_group != 4)
            return ISX_E_INVALID_ARG;
        if (tune->transform_tile) H.tq = (uint32_t)tune->transform_tile;
        H.blocks_per_cu = (uint32_t)tune->blocks_per_cu;
    }
    H.num_cus = (uint32_t)device_cus();
    uint64_t total_blocks = 0, total_slots = 0;
    for (int32_t i = 0; i < n; i++) {
        const isx_tile_desc &d = mode == MODE_ENCODE ? descs[i] : job_at(i).tile;
        int rc = validate_desc(d);
        if (rc) return rc;
        int z = 0;
        if (mode == MODE_DECODE) {
            const isx_decode_job &j = job_at(i);
            if (j.target_level > d.levels) return ISX_E_INVALID_ARG;
            if (j.drop_bitplanes > 31) return ISX_E_INVALID_ARG;
            z = j.target_level;
        } else if (d.row_stride_bytes < (uint64_t)d.width * d.channels * d.bytes_per_sample) {
            return ISX_E_INVALID_ARG;
        } else if (d.bytes_per_sample > 1 && ((d.pixel_offset | d.row_stride_bytes) & (d.bytes_per_sample - 1u))) {
            return ISX_E_INVALID_ARG;  // 16/32-bit samples are read as aligned words
        }
        RegionIn rg{}, *rgp = nullptr;
        uint32_t ow = d.width, oh = d.height;
        for (int k = 0; k < z; k++) { ow = (ow + 1) / 2; oh = (oh + 1) / 2; }
        if (regions) {
            const isx_region_job &R = regions[i];
            if (!R.h_block_offsets || R.width < 1 || R.height < 1 || R.x0 >= ow || R.y0 >= oh ||
                R.width > ow - R.x0 || R.height > oh - R.y0)
                return ISX_E_INVALID_ARG;
            rg = {R.x0, R.y0, R.x0 + R.width, R.y0 + R.height, R.h_block_offsets};
            rgp = &rg;
            ow = R.width;  // output row width
        }
        // consecutive tiles of one shape (a served batch, a slide) share
        // their geometry: computed once, copied after
        const isx_tile_desc *dp = i ? &(mode == MODE_ENCODE ? descs[i - 1] : job_at(i - 1).tile) : nullptr;
        const bool same = dp && !regions && dp->width == d.width && dp->height == d.height &&
                          dp->row_stride_bytes == d.row_stride_bytes && dp->channels == d.channels &&
                          dp->bytes_per_sample == d.bytes_per_sample && dp->bits == d.bits &&
                          dp->levels == d.levels && dp->colour_transform == d.colour_transform &&
                          dp->qstep == d.qstep && tb[i - 1].g.target_level == (uint8_t)z;
        if (same) {
            tb[i] = tb[i - 1];
            tb[i].g.pix_offset = d.pixel_offset;
        } else {
            rc = tile_geometry(d, z, tb[i], rgp);
            if (rc) return rc;
        }
        TileGeo &T = tb[i].g;
        if (mode == MODE_DECODE) {
            const isx_decode_job &j = job_at(i);
            if (j.out_row_stride_bytes < (uint64_t)ow * T.channels * T.bps) return ISX_E_INVALID_ARG;
            if (T.bps > 1 && ((j.out_offset | j.out_row_stride_bytes) & (T.bps - 1u))) return ISX_E_INVALID_ARG;
            T.pix_offset = j.out_offset;
            T.pix_stride = j.out_row_stride_bytes;
            T.enc_offset = j.in_offset;
            T.enc_bytes = j.in_bytes;
            T.drop = j.drop_bitplanes;
        } else {
            T.drop = 0;
        }
        T.block_base = (uint32_t)total_blocks;
        T.slot_base = (uint32_t)total_slots;
        total_blocks += T.nblocks;
        total_slots += (uint64_t)T.nblocks * T.dmax;
        if (total_blocks > 0x7fffffffull || total_slots > 0x7fffffffull) return ISX_E_UNSUPPORTED;
        if (T.levels > H.max_levels) H.max_levels = T.levels;
        if (T.nblocks > H.max_nblocks) H.max_nblocks = T.nblocks;
        if (T.dmax > H.max_dmax) H.max_dmax = T.dmax;
    }
    if (mode == MODE_DECODE && total_blocks >= (1ull << 27)) return ISX_E_UNSUPPORTED;  // segment item = block << 5 | segment
    H.total_blocks = (uint32_t)total_blocks;
    H.total_slots = (uint32_t)total_slots;
    // Segment decoder workgroups: two waves (large segments decoded by both,
    // small ones by each wave alone: sixteen waves per CU where one-wave
    // workgroups fit eleven); four waves for a decode with few segments (a
    // served view, one small tile), so that the lone segments finish sooner.
    // total_slots bounds the segment count.
    H.seg_nw = mode == MODE_DECODE && total_slots <= 4ull * H.num_cus ? 4u : 2u;
    if (tune && tune->seg_wave_group) H.seg_nw = (uint32_t)tune->seg_wave_group;
    // the packer likewise: four waves per segment when there are few
    H.pack_nw = mode == MODE_ENCODE && total_slots <= 4ull * H.num_cus ? 4u : 1u;
    // Large segments are queued first.  With two waves per workgroup they
    // are the ones that a lone wave's half of the LDS could not stage (the
    // small ones are decoded a wave each); a whole-block item must fit the
    // staging of the wave that takes it.
    const bool latency_form = total_slots <= 8ull * H.num_cus;
    H.seg_big_bits = H.seg_nw == 2 ? (kHalfWords - 3) * 32u : kBigSegBits;
    H.seg_whole_words = H.seg_nw == 1 ? kSegWords : (H.seg_nw == 2 && !latency_form ? kHalfWords : 0u);
    H.blk_grid = H.total_blocks;
    if (H.blocks_per_cu) {
        uint64_t g = (uint64_t)H.num_cus * H.blocks_per_cu;
        if (g < H.blk_grid) H.blk_grid = (uint32_t)g;
    }
    // workspace: global regions, then per-tile arenas
    uint64_t o = kPlanRegion;
    H.ws_blockdesc = o; o = al(o + total_blocks * sizeof(BlockDesc));
    H.ws_acc = o; o = al(o + total_blocks * sizeof(BlkAcc));
    H.ws_blkstat = o; o = al(o + total_blocks * sizeof(BlkStat));
    H.ws_blkplan = o; o = al(o + total_blocks * sizeof(BlkPlan));
    if (mode == MODE_ENCODE) {
        H.ws_seghist = o; o = al(o + total_slots * 256 * sizeof(uint16_t));
        H.ws_segstat = o; o = al(o + total_slots * sizeof(SegStat));
    }
    if (mode == MODE_DECODE) {
        H.ws_lut = o; o = al(o + total_blocks * kLutStride);
        H.ws_items = o; o = al(o + kItemsHdr + 2 * total_blocks * 32 * sizeof(uint32_t));
    }
    H.ws_tileout = o; o = al(o + (uint64_t)n * sizeof(TileOut));
    for (int32_t i = 0; i < n; i++) {
        TileGeo &T = tb[i].g;
        // The LH, HL and HH bands of levels 1 and 2 (fifteen sixteenths of the
        // coefficients) are held as int16 by the strip kernels when every
        // value fits (bit l-1 of coef16 for level l): an encode's quantised
        // level-l outputs are within the high-pass bound of the bit-depth
        // recursion (level 1: 4 (2^bits - 1) + 2), and a decode's
        // dequantised ones within (2^(dmax-1) - 1) step + step/2 at every
        // level, since the decoder rejects a block deeper than dmax planes.
        T.coef16 = 0;
        if (H.tq == 32 && !P.wide_coeffs) {
            for (uint32_t l = 1; l <= 2 && l <= T.levels; l++) {
                const bool fits = mode == MODE_ENCODE
                                      ? highpass_bound(T.bits, l) <= 32767.0
                                      : ((1ull << (T.dmax - 1)) - 1) * T.qstep + T.qstep / 2 <= 32767u;
                if (fits) T.coef16 |= (uint8_t)(1u << (l - 1));
            }
        }
        uint64_t base = o / 4;  // int32 elements
        T.ll_off += base;
        for (uint32_t l = 1; l <= T.levels; l++)
            for (int t = 0; t < 3; t++) T.lv[l].off[t] += base;
        o = al(o + tb[i].arena_elems * 4);
        T.tmp_off[0] = o / 4; o = al(o + tb[i].tmp_elems[0] * 4);
        T.tmp_off[1] = o / 4; o = al(o + tb[i].tmp_elems[1] * 4);
        T.sym_base = o; o = al(o + tb[i].sym_bytes);
    }
    H.ws_bytes = o;
    // work lists
    std::vector<WorkItem> &items = tls_items;
    items.clear();
    auto add_level = [&](int lvl, bool inverse) {
        H.lvl_first[lvl] = (uint32_t)items.size();
        uint32_t wg = 0;
        for (int32_t i = 0; i < n; i++) {
            const TileGeo &T = tb[i].g;
            uint32_t w, h;
            if (lvl == 0) {
                if (inverse || T.levels != 0) continue;
                w = T.width; h = T.height;
            } else {
                if (T.levels < lvl) continue;
                if (inverse && lvl < (int)T.target_level + 2) continue;
                w = T.lv[lvl].w; h = T.lv[lvl].h;
            }
            WorkItem it;
            memset(&it, 0, sizeof(it));
            it.tile = (uint32_t)i;
            it.wg_start = wg;
            uint32_t span = lvl == 0 ? 64u : 2u * H.tq;  // level-0 copies use 64x64 tiles
            it.ntx = div_up(w, span); it.nty = div_up(h, span);
            if (inverse) {  // tiles over the range of LL_{lvl-1} the decode needs
                const TileBuild &B = tb[i];
                it.qx0 = B.kx0[lvl - 1] / 2; it.qy0 = B.ky0[lvl - 1] / 2;
                it.ntx = div_up(B.kx1[lvl - 1] - 2 * it.qx0, span);
                it.nty = div_up(B.ky1[lvl - 1] - 2 * it.qy0, span);
            }
            it.nch = T.channels;
            wg += it.ntx * it.nty * it.nch;
            items.push_back(it);
        }
        H.lvl_count[lvl] = (uint32_t)items.size() - H.lvl_first[lvl];
        H.lvl_wgs[lvl] = wg;
    };
    if (mode == MODE_ENCODE) {
        for (int l = 0; l <= (int)H.max_levels; l++) add_level(l, false);
    } else {
        for (int l = 1; l <= (int)H.max_levels; l++) add_level(l, true);
        H.fin_first = (uint32_t)items.size();
        uint32_t wg = 0;
        for (int32_t i = 0; i < n; i++) {
            const TileGeo &T = tb[i].g;
            WorkItem it;
            memset(&it, 0, sizeof(it));
            it.tile = (uint32_t)i;
            it.wg_start = wg;
            it.qx0 = T.rx0 / 2; it.qy0 = T.ry0 / 2;
            it.ntx = div_up(T.rx1 - 2 * it.qx0, 2 * H.tq); it.nty = div_up(T.ry1 - 2 * it.qy0, 2 * H.tq);
            it.nch = T.ct ? 1 : div_up(T.channels, 3);
            wg += it.ntx * it.nty * it.nch;
            items.push_back(it);
        }
        H.fin_count = (uint32_t)items.size() - H.fin_first;
        H.fin_wgs = wg;
    }
    // block lists by size class (symbol kernel launch shape)
    std::vector<uint32_t> &big = tls_big, &small = tls_small;
    big.clear();
    small.clear();
    for (int32_t i = 0; i < n; i++) {
        const TileGeo &T = tb[i].g;
        for (uint32_t b = 0; b < T.nblocks; b++) {
            BlockDesc B;
            block_geometry(T, tb[i].sel.empty() ? b : tb[i].sel[b].local, B);
            uint32_t cells = (uint32_t)B.p * B.wb * B.hb / 16;
            (cells > 768 ? big : small).push_back(T.block_base + b);
        }
    }
    H.n_big = (uint32_t)big.size();
    H.n_small = (uint32_t)small.size();
    H.tiles_off = al(sizeof(PlanHdr), 64);
    H.work_off = al(H.tiles_off + (uint64_t)n * sizeof(TileGeo), 64);
    H.list_off = al(H.work_off + items.size() * sizeof(WorkItem), 64);
    H.plan_bytes = H.list_off + (big.size() + small.size()) * sizeof(uint32_t);
    // region decode: each job's selected blocks
    for (int32_t i = 0; i < n; i++) {
        if (tb[i].sel.empty()) continue;
        H.plan_bytes = al(H.plan_bytes, 64);
        tb[i].g.sel_off = H.plan_bytes;
        H.plan_bytes += tb[i].sel.size() * sizeof(SelBlock);
    }
    if (H.plan_bytes > kPlanRegion) {
        // large batches keep the plan after the workspace regions
        uint64_t extra = al(H.plan_bytes);
        H.ws_bytes += extra;
    }
    if (P.sizes_only) return ISX_OK;
    uint8_t *out;
    if (P.dst) {
        if (P.cap < H.plan_bytes) return ISX_E_INVALID_ARG;
        out = P.dst;
        memset(out, 0, H.plan_bytes);
    } else {
        P.bytes.assign(H.plan_bytes, 0);
        out = P.bytes.data();
    }
    memcpy(out, &H, sizeof(H));
    for (int32_t i = 0; i < n; i++) memcpy(out + H.tiles_off + (uint64_t)i * sizeof(TileGeo), &tb[i].g, sizeof(TileGeo));
    if (!items.empty()) memcpy(out + H.work_off, items.data(), items.size() * sizeof(WorkItem));
    if (!big.empty()) memcpy(out + H.list_off, big.data(), big.size() * sizeof(uint32_t));
    if (!small.empty())
        memcpy(out + H.list_off + big.size() * sizeof(uint32_t), small.data(), small.size() * sizeof(uint32_t));
    for (int32_t i = 0; i < n; i++)
        if (!tb[i].sel.empty())
            memcpy(out + tb[i].g.sel_off, tb[i].sel.data(), tb[i].sel.size() * sizeof(SelBlock));
    return ISX_OK;
}

// Device address of the plan copy inside the workspace (convenience API).
uint64_t plan_ws_offset(const PlanHdr &H)
{
    if (H.plan_bytes <= kPlanRegion) return 0;
    return H.ws_bytes - al(H.plan_bytes);
}

// Host bytes of a plan copy in flight: freed by a host function that the
// stream runs after the copy, so the source outlives the copy whether or not
// the runtime stages pageable memory before hipMemcpyAsync returns.
void release_plan_bytes(void *p) { delete static_cast<std::vector<uint8_t> *>(p); }

// The convenience entry points copy their plan into the workspace on
// `stream`.  They refuse a stream under capture: a captured copy would keep a
// host pointer whose lifetime the graph does not control (capture-safe
// callers use the plan / run entry points, which enqueue kernels only).
int upload_plan(Plan &P, uint8_t *d_ws, hipStream_t stream, uint8_t **d_plan)
{
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(stream, &cs) != hipSuccess) return ISX_E_HIP;
    if (cs != hipStreamCaptureStatusNone) return ISX_E_UNSUPPORTED;
    *d_plan = d_ws + plan_ws_offset(P.H);
    auto *held = new std::vector<uint8_t>(P.bytes);
    hipError_t e = hipMemcpyAsync(*d_plan, held->data(), held->size(), hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) {
        delete held;
        return ISX_E_HIP;
    }
    e = hipLaunchHostFunc(stream, release_plan_bytes, held);
    if (e != hipSuccess) {
        // the copy is queued and its source must stay valid: wait for it
        (void)hipStreamSynchronize(stream);
        delete held;
        return ISX_E_HIP;
    }
    return ISX_OK;
}

// Workspace of isx_decode_run_noalloc: a fixed array in the library's device
// memory (each GPU that loads the library holds its own copy until the
// process ends).  Host code never passes `scratch` itself to a kernel: in host
// code the name is a stand-in, not a device address; the address is looked up
// per device with hipGetSymbolAddress and kept in g_scratch.
static __device__ __align__(256) uint8_t scratch[ISX_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint8_t *g_scratch[kMaxDevices];

// Device address of `scratch` on the current device (looked up once per
// device, with that device current); nullptr on a HIP error.
uint8_t *scratch_ptr()
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
        g_scratch[dev] = (uint8_t *)p;
    }
    return g_scratch[dev];
}

}  // namespace

extern "C" {

const char *isx_status_string(int32_t code)
{
    switch (code) {
    case ISX_OK: return "ok";
    case ISX_E_INVALID_ARG: return "invalid argument";
    case ISX_E_CAPACITY: return "output capacity exceeded";
    case ISX_E_CORRUPT: return "corrupt stream";
    case ISX_E_TRUNCATED: return "truncated stream";
    case ISX_E_UNSUPPORTED: return "unsupported parameters";
    case ISX_E_WORKSPACE: return "workspace too small";
    case ISX_E_HIP: return "HIP runtime error";
    case ISX_E_PENDING: return "pending";
    default: return "unknown status";
    }
}

int64_t isx_tile_block_count(const isx_tile_desc *h_desc)
{
    if (!h_desc || validate_desc(*h_desc)) return ISX_E_INVALID_ARG;
    TileBuild tb;
    tile_geometry(*h_desc, 0, tb);
    return tb.g.nblocks_stream;
}

uint64_t isx_max_encoded_bytes(const isx_tile_desc *h_descs, int32_t n_tiles)
{
    if (!h_descs || n_tiles < 1) return 0;
    uint64_t total = 0;
    for (int32_t i = 0; i < n_tiles; i++) {
        if (validate_desc(h_descs[i])) return 0;
        TileBuild tb;
        tile_geometry(h_descs[i], 0, tb);
        const TileGeo &T = tb.g;
        uint64_t t = 24 + 4ull * T.nblocks_stream;
        for (uint32_t b = 0; b < T.nblocks_stream; b++) {
            BlockDesc B;
            block_geometry(T, b, B);
            uint64_t S = (uint64_t)B.p * B.wb * B.hb / 8 * T.dmax;  // symbols
            // header <= 3200 bits; payload <= 8 bits per token + wz (<= 13)
            // per C_zr token (< S/2 + S/256 of them): < 15 S bits
            t += 400 + (15 * S + 7) / 8;
        }
        total += al(t);
    }
    return total;
}

uint64_t isx_encode_workspace_bytes(const isx_tile_desc *h_descs, int32_t n_tiles)
{
    Plan P;
    P.sizes_only = true;
    if (!h_descs || build_plan(MODE_ENCODE, h_descs, nullptr, n_tiles, P)) return 0;
    return P.H.ws_bytes;
}

uint64_t isx_decode_workspace_bytes(const isx_decode_job *h_jobs, int32_t n_jobs)
{
    Plan P;
    P.sizes_only = true;
    if (!h_jobs || build_plan(MODE_DECODE, nullptr, h_jobs, n_jobs, P)) return 0;
    return P.H.ws_bytes;
}

uint64_t isx_encode_plan_bytes(const isx_tile_desc *h_descs, int32_t n_tiles)
{
    Plan P;
    P.sizes_only = true;
    if (!h_descs || build_plan(MODE_ENCODE, h_descs, nullptr, n_tiles, P)) return 0;
    return P.H.plan_bytes;
}

int32_t isx_encode_plan_build(const isx_tile_desc *h_descs, int32_t n_tiles, void *h_plan, uint64_t plan_bytes)
{
    Plan P;
    if (!h_descs || !h_plan) return ISX_E_INVALID_ARG;
    P.dst = (uint8_t *)h_plan;
    P.cap = plan_bytes;
    int rc = build_plan(MODE_ENCODE, h_descs, nullptr, n_tiles, P);
    if (rc) return rc;
    return ISX_OK;
}

int32_t isx_encode_plan_build_tuned(const isx_tile_desc *h_descs, int32_t n_tiles, const isx_tuning *tuning,
                                    void *h_plan, uint64_t plan_bytes)
{
    Plan P;
    if (!h_descs || !h_plan) return ISX_E_INVALID_ARG;
    P.dst = (uint8_t *)h_plan;
    P.cap = plan_bytes;
    int rc = build_plan(MODE_ENCODE, h_descs, nullptr, n_tiles, P, tuning);
    if (rc) return rc;
    return ISX_OK;
}

int32_t isx_decode_plan_build_tuned(const isx_decode_job *h_jobs, int32_t n_jobs, const isx_tuning *tuning,
                                    void *h_plan, uint64_t plan_bytes)
{
    Plan P;
    if (!h_jobs || !h_plan) return ISX_E_INVALID_ARG;
    P.dst = (uint8_t *)h_plan;
    P.cap = plan_bytes;
    int rc = build_plan(MODE_DECODE, nullptr, h_jobs, n_jobs, P, tuning);
    if (rc) return rc;
    return ISX_OK;
}

uint64_t isx_decode_plan_bytes(const isx_decode_job *h_jobs, int32_t n_jobs)
{
    Plan P;
    P.sizes_only = true;
    if (!h_jobs || build_plan(MODE_DECODE, nullptr, h_jobs, n_jobs, P)) return 0;
    return P.H.plan_bytes;
}

int32_t isx_decode_plan_build(const isx_decode_job *h_jobs, int32_t n_jobs, void *h_plan, uint64_t plan_bytes)
{
    Plan P;
    if (!h_jobs || !h_plan) return ISX_E_INVALID_ARG;
    P.dst = (uint8_t *)h_plan;
    P.cap = plan_bytes;
    int rc = build_plan(MODE_DECODE, nullptr, h_jobs, n_jobs, P);
    if (rc) return rc;
    return ISX_OK;
}

static int check_plan(const void *h_plan, int mode)
{
    if (!h_plan) return ISX_E_INVALID_ARG;
    const PlanHdr *H = (const PlanHdr *)h_plan;
    if (H->magic != kPlanMagic || H->mode != (uint32_t)mode) return ISX_E_INVALID_ARG;
    return ISX_OK;
}

int32_t isx_plan_info(const void *h_plan, uint64_t *plan_bytes, uint64_t *workspace_bytes)
{
    if (!h_plan || !plan_bytes || !workspace_bytes) return ISX_E_INVALID_ARG;
    const PlanHdr *H = (const PlanHdr *)h_plan;
    if (H->magic != kPlanMagic || (H->mode != MODE_ENCODE && H->mode != MODE_DECODE)) return ISX_E_INVALID_ARG;
    *plan_bytes = H->plan_bytes;
    *workspace_bytes = H->ws_bytes;
    return ISX_OK;
}

int32_t isx_encode_run(const void *h_plan, const void *d_plan, const void *d_pixels, void *d_out,
                       uint64_t out_capacity, uint64_t *d_tile_offsets, uint64_t *d_tile_sizes,
                       int32_t *d_status, void *d_workspace, uint64_t workspace_bytes, void *stream)
{
    int rc = check_plan(h_plan, MODE_ENCODE);
    if (rc) return rc;
    const PlanHdr &H = *(const PlanHdr *)h_plan;
    if (!d_plan || !d_pixels || !d_out || !d_tile_offsets || !d_tile_sizes || !d_status || !d_workspace)
        return ISX_E_INVALID_ARG;
    if (workspace_bytes < H.ws_bytes) return ISX_E_WORKSPACE;
    hipError_t e = launch_encode(H, (const uint8_t *)d_plan, (const uint8_t *)d_pixels, (uint8_t *)d_out,
                                 out_capacity, d_tile_offsets, d_tile_sizes, d_status, (uint8_t *)d_workspace,
                                 (hipStream_t)stream, 0, ENC_NSTAGES - 1);
    return e == hipSuccess ? ISX_OK : ISX_E_HIP;
}

int32_t isx_decode_run(const void *h_plan, const void *d_plan, const void *d_encoded, void *d_pixels_out,
                       int32_t *d_status, void *d_workspace, uint64_t workspace_bytes, void *stream)
{
    int rc = check_plan(h_plan, MODE_DECODE);
    if (rc) return rc;
    const PlanHdr &H = *(const PlanHdr *)h_plan;
    if (!d_plan || !d_encoded || !d_pixels_out || !d_status || !d_workspace) return ISX_E_INVALID_ARG;
    if (workspace_bytes < H.ws_bytes) return ISX_E_WORKSPACE;
    hipError_t e = launch_decode(H, (const uint8_t *)d_plan, (const uint8_t *)d_encoded, (uint8_t *)d_pixels_out,
                                 d_status, (uint8_t *)d_workspace, (hipStream_t)stream, 0, DEC_NSTAGES - 1);
    return e == hipSuccess ? ISX_OK : ISX_E_HIP;
}

int32_t isx_decode_run_noalloc(const void *h_plan, const void *d_plan, const void *d_encoded, void *d_pixels_out,
                               int32_t *d_status, void *stream)
{
    int rc = check_plan(h_plan, MODE_DECODE);
    if (rc) return rc;
    const PlanHdr &H = *(const PlanHdr *)h_plan;
    if (!d_plan || !d_encoded || !d_pixels_out || !d_status) return ISX_E_INVALID_ARG;
    if (H.ws_bytes > ISX_NOALLOC_SCRATCH_BYTES) return ISX_E_WORKSPACE;
    uint8_t *ws = scratch_ptr();
    if (!ws) return ISX_E_HIP;
    // the stages clear every counter and queue they use with kernels; no
    // other state of a previous call is read
    hipError_t e = launch_decode(H, (const uint8_t *)d_plan, (const uint8_t *)d_encoded, (uint8_t *)d_pixels_out,
                                 d_status, ws, (hipStream_t)stream, 0, DEC_NSTAGES - 1);
    return e == hipSuccess ? ISX_OK : ISX_E_HIP;
}

int32_t isx_stage_count(int32_t mode)
{
    return mode == 0 ? (int32_t)ENC_NSTAGES : (mode == 1 ? (int32_t)DEC_NSTAGES : ISX_E_INVALID_ARG);
}

const char *isx_stage_name(int32_t mode, int32_t stage)
{
    static const char *fwd[16] = {"forward_l0", "forward_l1", "forward_l2", "forward_l3", "forward_l4",
                                  "forward_l5", "forward_l6", "forward_l7", "forward_l8", "forward_l9",
                                  "forward_l10", "forward_l11", "forward_l12", "forward_l13", "forward_l14",
                                  "forward_l15"};
    static const char *inv[16] = {"inverse_final", "inverse_l1", "inverse_l2", "inverse_l3", "inverse_l4",
                                  "inverse_l5", "inverse_l6", "inverse_l7", "inverse_l8", "inverse_l9",
                                  "inverse_l10", "inverse_l11", "inverse_l12", "inverse_l13", "inverse_l14",
                                  "inverse_l15"};
    if (mode == 0) {
        if (stage == ENC_PREP) return "enc_prep";
        if (stage >= ENC_FWD0 && stage <= ENC_FWD0 + kMaxLevels) return fwd[stage - ENC_FWD0];
        if (stage == ENC_SYM) return "enc_symbols";
        if (stage == ENC_CODE) return "enc_code";
        if (stage == ENC_BOFF) return "enc_block_offsets";
        if (stage == ENC_TOFF) return "enc_tile_offsets";
        if (stage == ENC_FIN) return "enc_tile_finish";
        if (stage == ENC_PACK) return "enc_pack";
    } else if (mode == 1) {
        if (stage == DEC_PREP) return "dec_prep";
        if (stage == DEC_HDR) return "dec_header";
        if (stage == DEC_SEG) return "dec_segments";
        if (stage == DEC_REASM) return "dec_reassemble";
        if (stage >= DEC_INV15 && stage <= DEC_FINAL) return inv[DEC_FINAL - stage];
    }
    return "";
}

int32_t isx_encode_run_stages(const void *h_plan, const void *d_plan, const void *d_pixels, void *d_out,
                              uint64_t out_capacity, uint64_t *d_tile_offsets, uint64_t *d_tile_sizes,
                              int32_t *d_status, void *d_workspace, uint64_t workspace_bytes, void *stream,
                              int32_t first, int32_t count)
{
    int rc = check_plan(h_plan, MODE_ENCODE);
    if (rc) return rc;
    const PlanHdr &H = *(const PlanHdr *)h_plan;
    if (!d_plan || !d_pixels || !d_out || !d_tile_offsets || !d_tile_sizes || !d_status || !d_workspace)
        return ISX_E_INVALID_ARG;
    if (first < 0 || count < 0 || first + count > (int32_t)ENC_NSTAGES) return ISX_E_INVALID_ARG;
    if (workspace_bytes < H.ws_bytes) return ISX_E_WORKSPACE;
    if (!count) return ISX_OK;
    hipError_t e = launch_encode(H, (const uint8_t *)d_plan, (const uint8_t *)d_pixels, (uint8_t *)d_out,
                                 out_capacity, d_tile_offsets, d_tile_sizes, d_status, (uint8_t *)d_workspace,
                                 (hipStream_t)stream, first, first + count - 1);
    return e == hipSuccess ? ISX_OK : ISX_E_HIP;
}

int32_t isx_decode_run_stages(const void *h_plan, const void *d_plan, const void *d_encoded, void *d_pixels_out,
                              int32_t *d_status, void *d_workspace, uint64_t workspace_bytes, void *stream,
                              int32_t first, int32_t count)
{
    int rc = check_plan(h_plan, MODE_DECODE);
    if (rc) return rc;
    const PlanHdr &H = *(const PlanHdr *)h_plan;
    if (!d_plan || !d_encoded || !d_pixels_out || !d_status || !d_workspace) return ISX_E_INVALID_ARG;
    if (first < 0 || count < 0 || first + count > (int32_t)DEC_NSTAGES) return ISX_E_INVALID_ARG;
    if (workspace_bytes < H.ws_bytes) return ISX_E_WORKSPACE;
    if (!count) return ISX_OK;
    hipError_t e = launch_decode(H, (const uint8_t *)d_plan, (const uint8_t *)d_encoded, (uint8_t *)d_pixels_out,
                                 d_status, (uint8_t *)d_workspace, (hipStream_t)stream, first, first + count - 1);
    return e == hipSuccess ? ISX_OK : ISX_E_HIP;
}

int32_t isx_encode_tiles(const isx_tile_desc *h_descs, int32_t n_tiles, const void *d_pixels, void *d_out,
                         uint64_t out_capacity, uint64_t *d_tile_offsets, uint64_t *d_tile_sizes,
                         int32_t *d_status, void *d_workspace, uint64_t workspace_bytes, void *stream)
{
    if (!h_descs) return ISX_E_INVALID_ARG;
    Plan P;
    int rc = build_plan(MODE_ENCODE, h_descs, nullptr, n_tiles, P);
    if (rc) return rc;
    if (!d_pixels || !d_out || !d_tile_offsets || !d_tile_sizes || !d_status || !d_workspace)
        return ISX_E_INVALID_ARG;
    if (workspace_bytes < P.H.ws_bytes) return ISX_E_WORKSPACE;
    uint8_t *d_plan;
    rc = upload_plan(P, (uint8_t *)d_workspace, (hipStream_t)stream, &d_plan);
    if (rc) return rc;
    return isx_encode_run(P.bytes.data(), d_plan, d_pixels, d_out, out_capacity, d_tile_offsets, d_tile_sizes,
                          d_status, d_workspace, workspace_bytes, stream);
}

int32_t isx_decode_tiles(const void *d_encoded, const isx_decode_job *h_jobs, int32_t n_jobs, void *d_pixels_out,
                         int32_t *d_status, void *d_workspace, uint64_t workspace_bytes, void *stream)
{
    if (!h_jobs) return ISX_E_INVALID_ARG;
    Plan P;
    int rc = build_plan(MODE_DECODE, nullptr, h_jobs, n_jobs, P);
    if (rc) return rc;
    if (!d_encoded || !d_pixels_out || !d_status || !d_workspace) return ISX_E_INVALID_ARG;
    if (workspace_bytes < P.H.ws_bytes) return ISX_E_WORKSPACE;
    uint8_t *d_plan;
    rc = upload_plan(P, (uint8_t *)d_workspace, (hipStream_t)stream, &d_plan);
    if (rc) return rc;
    return isx_decode_run(P.bytes.data(), d_plan, d_encoded, d_pixels_out, d_status, d_workspace,
                          workspace_bytes, stream);
}

int32_t isx_read_tile_header(const void *h_bytes, uint64_t len, isx_tile_desc *out)
{
    if (!h_bytes || !out) return ISX_E_INVALID_ARG;
    const uint8_t *h = (const uint8_t *)h_bytes;
    if (len < 24) return ISX_E_TRUNCATED;
    if (h[0] != 'I' || h[1] != 'S' || h[2] != 'X' || h[3] != '1' || h[4] != 1) return ISX_E_CORRUPT;
    auto u32 = [&](uint64_t o) {
        return (uint32_t)h[o] | ((uint32_t)h[o + 1] << 8) | ((uint32_t)h[o + 2] << 16) | ((uint32_t)h[o + 3] << 24);
    };
    isx_tile_desc d;
    memset(&d, 0, sizeof(d));
    d.colour_transform = h[5];
    d.channels = h[6];
    d.bits = h[7];
    d.bytes_per_sample = h[8];
    d.levels = h[9];
    d.qstep = (uint16_t)(h[10] | (h[11] << 8));
    const uint32_t w = u32(12), ht = u32(16), nb = u32(20);
    if (w > 65535 || ht > 65535) return ISX_E_CORRUPT;
    d.width = w;
    d.height = ht;
    d.pixel_offset = 0;
    d.row_stride_bytes = w * d.channels * d.bytes_per_sample;
    if (validate_desc(d)) return ISX_E_CORRUPT;
    TileBuild tb;
    tile_geometry(d, 0, tb);
    if (tb.g.nblocks_stream != nb) return ISX_E_CORRUPT;
    *out = d;
    return ISX_OK;
}

int32_t isx_stream_block_offsets(const void *h_head, uint64_t head_bytes, uint64_t *h_offsets, uint64_t n_offsets)
{
    if (!h_head || !h_offsets) return ISX_E_INVALID_ARG;
    const uint8_t *h = (const uint8_t *)h_head;
    if (head_bytes < 24) return ISX_E_TRUNCATED;
    if (h[0] != 'I' || h[1] != 'S' || h[2] != 'X' || h[3] != '1' || h[4] != 1) return ISX_E_CORRUPT;
    auto u32 = [&](uint64_t o) {
        return (uint32_t)h[o] | ((uint32_t)h[o + 1] << 8) | ((uint32_t)h[o + 2] << 16) | ((uint32_t)h[o + 3] << 24);
    };
    const uint64_t nb = u32(20);
    if (n_offsets < nb + 1) return ISX_E_INVALID_ARG;
    if (head_bytes < 24 + 4 * nb) return ISX_E_TRUNCATED;
    uint64_t off = 24 + 4 * nb;
    for (uint64_t b = 0; b < nb; b++) {
        h_offsets[b] = off;
        off += u32(24 + 4 * b);
    }
    h_offsets[nb] = off;
    return ISX_OK;
}

uint64_t isx_region_workspace_bytes(const isx_region_job *h_jobs, int32_t n_jobs)
{
    Plan P;
    P.sizes_only = true;
    if (!h_jobs || build_plan(MODE_DECODE, nullptr, nullptr, n_jobs, P, nullptr, h_jobs)) return 0;
    return P.H.ws_bytes;
}

uint64_t isx_region_plan_bytes(const isx_region_job *h_jobs, int32_t n_jobs)
{
    Plan P;
    P.sizes_only = true;
    if (!h_jobs || build_plan(MODE_DECODE, nullptr, nullptr, n_jobs, P, nullptr, h_jobs)) return 0;
    return P.H.plan_bytes;
}

int32_t isx_region_plan_build(const isx_region_job *h_jobs, int32_t n_jobs, const isx_tuning *tuning, void *h_plan,
                              uint64_t plan_bytes)
{
    Plan P;
    if (!h_jobs || !h_plan) return ISX_E_INVALID_ARG;
    P.dst = (uint8_t *)h_plan;
    P.cap = plan_bytes;
    int rc = build_plan(MODE_DECODE, nullptr, nullptr, n_jobs, P, tuning, h_jobs);
    if (rc) return rc;
    return ISX_OK;
}

int32_t isx_decode_regions(const void *d_encoded, const isx_region_job *h_jobs, int32_t n_jobs, void *d_pixels_out,
                           int32_t *d_status, void *d_workspace, uint64_t workspace_bytes, void *stream)
{
    if (!h_jobs) return ISX_E_INVALID_ARG;
    Plan P;
    int rc = build_plan(MODE_DECODE, nullptr, nullptr, n_jobs, P, nullptr, h_jobs);
    if (rc) return rc;
    if (!d_encoded || !d_pixels_out || !d_status || !d_workspace) return ISX_E_INVALID_ARG;
    if (workspace_bytes < P.H.ws_bytes) return ISX_E_WORKSPACE;
    uint8_t *d_plan;
    rc = upload_plan(P, (uint8_t *)d_workspace, (hipStream_t)stream, &d_plan);
    if (rc) return rc;
    return isx_decode_run(P.bytes.data(), d_plan, d_encoded, d_pixels_out, d_status, d_workspace,
                          workspace_bytes, stream);
}

int32_t isx_debug_forward(const isx_tile_desc *h_desc, const void *d_pixels, int32_t *d_coeffs,
                          void *d_workspace, uint64_t workspace_bytes, void *stream)
{
    if (!h_desc || !d_pixels || !d_coeffs || !d_workspace) return ISX_E_INVALID_ARG;
    Plan P;
    P.wide_coeffs = true;
    int rc = build_plan(MODE_ENCODE, h_desc, nullptr, 1, P);
    if (rc) return rc;
    if (workspace_bytes < P.H.ws_bytes) return ISX_E_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    uint8_t *d_plan;
    rc = upload_plan(P, (uint8_t *)d_workspace, s, &d_plan);
    if (rc) return rc;
    if (launch_forward_only(P.H, d_plan, (const uint8_t *)d_pixels, (uint8_t *)d_workspace, s) != hipSuccess)
        return ISX_E_HIP;
    const TileGeo &T = *(const TileGeo *)(P.bytes.data() + P.H.tiles_off);
    const int32_t *wsi = (const int32_t *)d_workspace;
    uint64_t k = 0;
    for (uint32_t c = 0; c < T.channels; c++) {
        struct BandRef { uint64_t off; uint32_t pitch, w, h; };
        std::vector<BandRef> list;
        list.push_back({T.ll_off + c * T.chan_elems, T.ll_pitch, T.ll_w, T.ll_h});
        for (uint32_t l = T.levels; l >= 1; l--) {
            const LevelGeo &G = T.lv[l];
            // HL, LH, HH
            list.push_back({G.off[1] + c * T.chan_elems, G.pitch[1], G.w / 2, (G.h + 1) / 2});
            list.push_back({G.off[0] + c * T.chan_elems, G.pitch[0], (G.w + 1) / 2, G.h / 2});
            list.push_back({G.off[2] + c * T.chan_elems, G.pitch[2], G.w / 2, G.h / 2});
        }
        for (const BandRef &b : list) {
            if (b.w && b.h) {
                hipError_t e = hipMemcpy2DAsync(d_coeffs + k, (size_t)b.w * 4, wsi + b.off, (size_t)b.pitch * 4,
                                                (size_t)b.w * 4, b.h, hipMemcpyDeviceToDevice, s);
                if (e != hipSuccess) return ISX_E_HIP;
            }
            k += (uint64_t)b.w * b.h;
        }
    }
    return ISX_OK;
}

int32_t isx_debug_huffman(const uint32_t *d_freq, int32_t limit, uint8_t *d_len, void *stream)
{
    if (!d_freq || !d_len) return ISX_E_INVALID_ARG;
    if (limit != 0 && (limit < 8 || limit > 15)) return ISX_E_INVALID_ARG;
    return launch_debug_huffman(d_freq, limit, d_len, (hipStream_t)stream) == hipSuccess ? ISX_OK : ISX_E_HIP;
}

}  // extern "C"
