// k_transform.hip -- colour transform + multi-level 2-D 5/3 integer lifting
// (forward and inverse) for gfx950.
//
// Forward level l (Sec. 4: 5/3 Le Gall integer lifting, recursive on LL;
// rows first, then columns):
//   d[n] = x[2n+1] - floor((x[2n] + x[2n+2]) / 2)
//   s[n] = x[2n]   + floor((d[n-1] + d[n] + 2) / 4)
// with whole-sample symmetric extension at the borders.  A workgroup owns a
// 32x32-quad output tile (64x64 input samples); it stages the input plus a
// 2/1-sample halo (reflected at the image border) in LDS, lifts the rows,
// then the columns, and writes the four subbands.  Level 1 reads the
// interleaved uint8/uint16 pixels and applies the reversible colour
// transform on load (Sec. 3's optional colour stage).  The high-pass bands
// are quantised on store (Sec. 3: JPEG2000-style dead-zone quantiser) and the
// OR of the magnitudes / any-negative flags of every coefficient block are
// accumulated here (wave reduction + one atomicOr per wave), which gives each
// block's bit depth d and empty-plane masks without another pass.
//
// Inverse level: the same tiling over the output; the window holds the
// interleaved subband samples (reflected in the interleaved domain, which is
// exact because each lifting step is a symmetric filter); columns are undone
// first, then rows.  The final level of a decode job also applies the inverse
// colour transform, clamps to [0, 2^bits - 1] and stores interleaved pixels.
#include "isx_common.h"

namespace isx {

__device__ inline int32_t floor_half(int32_t v) { return v >> 1; }           // arithmetic shift = floor
__device__ inline int32_t floor_quarter_r(int32_t v) { return (v + 2) >> 2; }  // floor((v+2)/4)

__device__ inline const WorkItem &find_item(const WorkItem *items, uint32_t first, uint32_t count,
                                            uint32_t wg)
{
    uint32_t lo = 0, hi = count;  // last item with wg_start <= wg
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (items[first + mid].wg_start <= wg) lo = mid; else hi = mid;
    }
    return items[first + lo];
}

__device__ inline int32_t load_sample(const uint8_t *pix, const TileGeo &T, int x, int y, int c)
{
    const uint8_t *row = pix + T.pix_offset + (uint64_t)y * T.pix_stride;
    uint32_t e = ((uint32_t)x * T.channels + c) * T.bps;
    if (T.bps == 1) return row[e];
    return (int32_t)row[e] | ((int32_t)row[e + 1] << 8);
}

// Sample of channel c after the colour transform (Y = floor((R+2G+B)/4),
// Cb = B - G, Cr = R - G when ct = RCT).
__device__ inline int32_t load_colour(const uint8_t *pix, const TileGeo &T, int x, int y, int c)
{
    if (T.ct == 0) return load_sample(pix, T, x, y, c);
    int32_t r = load_sample(pix, T, x, y, 0), g = load_sample(pix, T, x, y, 1), b = load_sample(pix, T, x, y, 2);
    if (c == 0) return (r + 2 * g + b) >> 2;
    if (c == 1) return b - g;
    return r - g;
}

__device__ inline uint32_t wave_or(uint32_t v)
{
    for (int o = 32; o >= 1; o >>= 1) v |= __shfl_xor(v, o, 64);
    return v;
}

// One forward 2-D level over a 32x32-quad tile, one channel per workgroup.
__global__ void __launch_bounds__(256) k_fwd_level(PlanHdr H, const uint8_t *__restrict__ plan,
                                                   const uint8_t *__restrict__ pix,
                                                   uint8_t *__restrict__ ws, int level)
{
    __shared__ int32_t win[kWin * kWinPitch];
    const TileGeo *tiles = (const TileGeo *)(plan + H.tiles_off);
    const WorkItem *items = (const WorkItem *)(plan + H.work_off);
    const WorkItem &W = find_item(items, H.lvl_first[level], H.lvl_count[level], blockIdx.x);
    const TileGeo &T = tiles[W.tile];
    uint32_t r = blockIdx.x - W.wg_start;
    uint32_t nsp = W.ntx * W.nty;
    int c = (int)(r / nsp);
    uint32_t sp = r % nsp;
    int qx0 = (int)(sp % W.ntx) * kTQ, qy0 = (int)(sp / W.ntx) * kTQ;
    const LevelGeo &G = T.lv[level];
    int w = (int)G.w, h = (int)G.h;
    int32_t *wsi = (int32_t *)ws;
    // source LL_{level-1}
    const int32_t *src = nullptr;
    uint32_t spitch = 0;
    if (level > 1) {
        int k = level - 1, which = (k & 1) ? 0 : 1;
        src = wsi + T.tmp_off[which] + (uint64_t)c * T.tmp_chan[which];
        spitch = T.tmp_pitch[which];
    }
    // stage window rows [2qy0-2, 2qy0+65], cols [2qx0-2, 2qx0+65] (reflected)
    for (int i = threadIdx.x; i < kWin * kWin; i += blockDim.x) {
        int lr = i / kWin, lc = i % kWin;
        int gy = reflect_idx(2 * qy0 - 2 + lr, h), gx = reflect_idx(2 * qx0 - 2 + lc, w);
        int32_t v = (level == 1) ? load_colour(pix, T, gx, gy, c) : src[(uint64_t)gy * spitch + gx];
        win[lr * kWinPitch + lc] = v;
    }
    __syncthreads();
    // rows: predict at odd columns 1..65, update at even columns 2..64 (all 68 rows)
    for (int i = threadIdx.x; i < kWin * 33; i += blockDim.x) {
        int lr = i / 33, lc = 1 + 2 * (i % 33);
        int32_t *row = win + lr * kWinPitch;
        row[lc] -= floor_half(row[lc - 1] + row[lc + 1]);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kWin * 32; i += blockDim.x) {
        int lr = i / 32, lc = 2 + 2 * (i % 32);
        int32_t *row = win + lr * kWinPitch;
        row[lc] += floor_quarter_r(row[lc - 1] + row[lc + 1]);
    }
    __syncthreads();
    // columns 2..65: predict at odd rows 1..65, update at even rows 2..64
    for (int i = threadIdx.x; i < 33 * 64; i += blockDim.x) {
        int lc = 2 + (i % 64), lr = 1 + 2 * (i / 64);
        win[lr * kWinPitch + lc] -= floor_half(win[(lr - 1) * kWinPitch + lc] + win[(lr + 1) * kWinPitch + lc]);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 32 * 64; i += blockDim.x) {
        int lc = 2 + (i % 64), lr = 2 + 2 * (i / 64);
        win[lr * kWinPitch + lc] += floor_quarter_r(win[(lr - 1) * kWinPitch + lc] + win[(lr + 1) * kWinPitch + lc]);
    }
    __syncthreads();
    // outputs
    int llw = (w + 1) / 2, llh = (h + 1) / 2, hw = w / 2, hh = h / 2;
    bool last = (level == T.levels);
    int32_t *llout;
    uint32_t llpitch;
    if (last) {
        llout = wsi + T.ll_off + (uint64_t)c * T.chan_elems;
        llpitch = T.ll_pitch;
    } else {
        int which = (level & 1) ? 0 : 1;
        llout = wsi + T.tmp_off[which] + (uint64_t)c * T.tmp_chan[which];
        llpitch = T.tmp_pitch[which];
    }
    int32_t *lh = wsi + G.off[0] + (uint64_t)c * T.chan_elems;
    int32_t *hl = wsi + G.off[1] + (uint64_t)c * T.chan_elems;
    int32_t *hhb = wsi + G.off[2] + (uint64_t)c * T.chan_elems;
    uint32_t step = T.qstep;
    uint32_t orm[3] = {0, 0, 0}, neg = 0, llor = 0;
    for (int i = threadIdx.x; i < kTQ * kTQ; i += blockDim.x) {
        int ii = i % kTQ, jj = i / kTQ;
        int qx = qx0 + ii, qy = qy0 + jj;
        int32_t vLL = win[(2 + 2 * jj) * kWinPitch + 2 + 2 * ii];
        int32_t vHL = win[(2 + 2 * jj) * kWinPitch + 3 + 2 * ii];
        int32_t vLH = win[(3 + 2 * jj) * kWinPitch + 2 + 2 * ii];
        int32_t vHH = win[(3 + 2 * jj) * kWinPitch + 3 + 2 * ii];
        if (step > 1) {
            vHL = vHL < 0 ? -(int32_t)((uint32_t)(-vHL) / step) : (int32_t)((uint32_t)vHL / step);
            vLH = vLH < 0 ? -(int32_t)((uint32_t)(-vLH) / step) : (int32_t)((uint32_t)vLH / step);
            vHH = vHH < 0 ? -(int32_t)((uint32_t)(-vHH) / step) : (int32_t)((uint32_t)vHH / step);
        }
        if (qx < llw && qy < llh) {
            llout[(uint64_t)qy * llpitch + qx] = vLL;
            if (last) { llor |= (uint32_t)(vLL < 0 ? -vLL : vLL); neg |= (vLL < 0) ? 8u : 0u; }
        }
        if (qx < llw && qy < hh) {
            lh[(uint64_t)qy * G.pitch[0] + qx] = vLH;
            orm[0] |= (uint32_t)(vLH < 0 ? -vLH : vLH); neg |= (vLH < 0) ? 1u : 0u;
        }
        if (qx < hw && qy < llh) {
            hl[(uint64_t)qy * G.pitch[1] + qx] = vHL;
            orm[1] |= (uint32_t)(vHL < 0 ? -vHL : vHL); neg |= (vHL < 0) ? 2u : 0u;
        }
        if (qx < hw && qy < hh) {
            hhb[(uint64_t)qy * G.pitch[2] + qx] = vHH;
            orm[2] |= (uint32_t)(vHH < 0 ? -vHH : vHH); neg |= (vHH < 0) ? 4u : 0u;
        }
    }
    // per-block accumulation (the whole 32x32-quad tile lies in one 128 cell)
    orm[0] = wave_or(orm[0]); orm[1] = wave_or(orm[1]); orm[2] = wave_or(orm[2]);
    neg = wave_or(neg); llor = wave_or(llor);
    if ((threadIdx.x & 63) == 0) {
        BlkAcc *acc = (BlkAcc *)(ws + H.ws_acc);
        int bx = qx0 / kBlock, by = qy0 / kBlock;
        int32_t hwc = hw - bx * kBlock, hhc = hh - by * kBlock;
        if (hwc > 0 || hhc > 0) {  // the cell holds at least one H coefficient
            uint32_t local = G.group_start + (uint32_t)c * G.blocks_per_chan + (uint32_t)by * G.gx + bx;
            BlkAcc *a = acc + T.block_base + local;
            if (orm[0]) atomicOr(&a->or_mag[0], orm[0]);
            if (orm[1]) atomicOr(&a->or_mag[1], orm[1]);
            if (orm[2]) atomicOr(&a->or_mag[2], orm[2]);
            if (neg & 7u) atomicOr(&a->neg, neg & 7u);
        }
        if (last) {
            uint32_t local = (uint32_t)c * T.ll_gx * T.ll_gy + (uint32_t)by * T.ll_gx + bx;
            BlkAcc *a = acc + T.block_base + local;
            if (llor) atomicOr(&a->or_mag[0], llor);
            if (neg & 8u) atomicOr(&a->neg, 1u);
        }
    }
}

// Levels = 0: the LL band is the (colour transformed) image itself.
__global__ void __launch_bounds__(256) k_fwd_level0(PlanHdr H, const uint8_t *__restrict__ plan,
                                                    const uint8_t *__restrict__ pix,
                                                    uint8_t *__restrict__ ws)
{
    const TileGeo *tiles = (const TileGeo *)(plan + H.tiles_off);
    const WorkItem *items = (const WorkItem *)(plan + H.work_off);
    const WorkItem &W = find_item(items, H.lvl_first[0], H.lvl_count[0], blockIdx.x);
    const TileGeo &T = tiles[W.tile];
    uint32_t r = blockIdx.x - W.wg_start;
    uint32_t nsp = W.ntx * W.nty;
    int c = (int)(r / nsp);
    uint32_t sp = r % nsp;
    int x0 = (int)(sp % W.ntx) * 64, y0 = (int)(sp / W.ntx) * 64;
    int32_t *ll = (int32_t *)ws + T.ll_off + (uint64_t)c * T.chan_elems;
    uint32_t orv = 0, neg = 0;
    for (int i = threadIdx.x; i < 64 * 64; i += blockDim.x) {
        int x = x0 + (i % 64), y = y0 + (i / 64);
        if (x < (int)T.width && y < (int)T.height) {
            int32_t v = load_colour(pix, T, x, y, c);
            ll[(uint64_t)y * T.ll_pitch + x] = v;
            orv |= (uint32_t)(v < 0 ? -v : v);
            neg |= v < 0;
        }
    }
    orv = wave_or(orv); neg = wave_or(neg);
    if ((threadIdx.x & 63) == 0) {
        BlkAcc *acc = (BlkAcc *)(ws + H.ws_acc);
        uint32_t local = (uint32_t)c * T.ll_gx * T.ll_gy + (uint32_t)(y0 / kBlock) * T.ll_gx + x0 / kBlock;
        BlkAcc *a = acc + T.block_base + local;
        if (orv) atomicOr(&a->or_mag[0], orv);
        if (neg) atomicOr(&a->neg, 1u);
    }
}

// ------------------------------------------------------------------ inverse
// Stage the interleaved window of level `level` for channel c: position
// (gy, gx) of LL_{level-1}, reflected, maps to LL/HL/LH/HH by parity.
__device__ inline void stage_inverse(const TileGeo &T, int level, int c, int qx0, int qy0,
                                     const int32_t *wsi, int32_t *win)
{
    const LevelGeo &G = T.lv[level];
    int w = (int)G.w, h = (int)G.h;
    const int32_t *ll;
    uint32_t llp;
    if (level == T.levels) { ll = wsi + T.ll_off + (uint64_t)c * T.chan_elems; llp = T.ll_pitch; }
    else {
        int which = (level & 1) ? 0 : 1;
        ll = wsi + T.tmp_off[which] + (uint64_t)c * T.tmp_chan[which];
        llp = T.tmp_pitch[which];
    }
    const int32_t *lh = wsi + G.off[0] + (uint64_t)c * T.chan_elems;
    const int32_t *hl = wsi + G.off[1] + (uint64_t)c * T.chan_elems;
    const int32_t *hh = wsi + G.off[2] + (uint64_t)c * T.chan_elems;
    for (int i = threadIdx.x; i < kWin * kWin; i += blockDim.x) {
        int lr = i / kWin, lc = i % kWin;
        int gy = reflect_idx(2 * qy0 - 2 + lr, h), gx = reflect_idx(2 * qx0 - 2 + lc, w);
        int32_t v;
        if (h == 1) gy = 0;
        if (w == 1) gx = 0;
        int py = gy & 1, px = gx & 1;
        if (!py && !px) v = ll[(uint64_t)(gy >> 1) * llp + (gx >> 1)];
        else if (!py && px) v = hl[(uint64_t)(gy >> 1) * G.pitch[1] + (gx >> 1)];
        else if (py && !px) v = lh[(uint64_t)(gy >> 1) * G.pitch[0] + (gx >> 1)];
        else v = hh[(uint64_t)(gy >> 1) * G.pitch[2] + (gx >> 1)];
        win[lr * kWinPitch + lc] = v;
    }
}

// Undo the lifting in the window: columns (unless the level has one row),
// then rows (unless it has one column).  Valid output: [2, 66) x [2, 66).
__device__ inline void inverse_window(int32_t *win, bool do_cols, bool do_rows)
{
    if (do_cols) {
        // undo update at even rows 2..66, columns 1..67
        for (int i = threadIdx.x; i < 33 * 67; i += blockDim.x) {
            int lc = 1 + (i % 67), lr = 2 + 2 * (i / 67);
            win[lr * kWinPitch + lc] -= floor_quarter_r(win[(lr - 1) * kWinPitch + lc] + win[(lr + 1) * kWinPitch + lc]);
        }
        __syncthreads();
        // undo predict at odd rows 3..65
        for (int i = threadIdx.x; i < 32 * 67; i += blockDim.x) {
            int lc = 1 + (i % 67), lr = 3 + 2 * (i / 67);
            win[lr * kWinPitch + lc] += floor_half(win[(lr - 1) * kWinPitch + lc] + win[(lr + 1) * kWinPitch + lc]);
        }
        __syncthreads();
    }
    if (do_rows) {
        for (int i = threadIdx.x; i < 64 * 33; i += blockDim.x) {
            int lr = 2 + (i / 33), lc = 2 + 2 * (i % 33);
            int32_t *row = win + lr * kWinPitch;
            row[lc] -= floor_quarter_r(row[lc - 1] + row[lc + 1]);
        }
        __syncthreads();
        for (int i = threadIdx.x; i < 64 * 32; i += blockDim.x) {
            int lr = 2 + (i / 32), lc = 3 + 2 * (i % 32);
            int32_t *row = win + lr * kWinPitch;
            row[lc] += floor_half(row[lc - 1] + row[lc + 1]);
        }
        __syncthreads();
    }
}

// Inverse of level `level` into LL_{level-1} (an intermediate level).
__global__ void __launch_bounds__(256) k_inv_level(PlanHdr H, const uint8_t *__restrict__ plan,
                                                   uint8_t *__restrict__ ws, int level)
{
    __shared__ int32_t win[kWin * kWinPitch];
    const TileGeo *tiles = (const TileGeo *)(plan + H.tiles_off);
    const WorkItem *items = (const WorkItem *)(plan + H.work_off);
    const WorkItem &W = find_item(items, H.lvl_first[level], H.lvl_count[level], blockIdx.x);
    const TileGeo &T = tiles[W.tile];
    uint32_t r = blockIdx.x - W.wg_start;
    uint32_t nsp = W.ntx * W.nty;
    int c = (int)(r / nsp);
    uint32_t sp = r % nsp;
    int qx0 = (int)(sp % W.ntx) * kTQ, qy0 = (int)(sp / W.ntx) * kTQ;
    int32_t *wsi = (int32_t *)ws;
    const LevelGeo &G = T.lv[level];
    stage_inverse(T, level, c, qx0, qy0, wsi, win);
    __syncthreads();
    inverse_window(win, G.h > 1, G.w > 1);
    int k = level - 1, which = (k & 1) ? 0 : 1;
    int32_t *dst = wsi + T.tmp_off[which] + (uint64_t)c * T.tmp_chan[which];
    uint32_t dp = T.tmp_pitch[which];
    for (int i = threadIdx.x; i < 64 * 64; i += blockDim.x) {
        int x = 2 * qx0 + (i % 64), y = 2 * qy0 + (i / 64);
        if (x < (int)G.w && y < (int)G.h) dst[(uint64_t)y * dp + x] = win[(2 + i / 64) * kWinPitch + 2 + (i % 64)];
    }
}

__device__ inline void store_pixel(uint8_t *pix, const TileGeo &T, int x, int y, int c, int32_t v)
{
    int32_t top = (1 << T.bits) - 1;
    v = v < 0 ? 0 : (v > top ? top : v);
    uint8_t *row = pix + T.pix_offset + (uint64_t)y * T.pix_stride;
    uint32_t e = ((uint32_t)x * T.channels + c) * T.bps;
    row[e] = (uint8_t)(v & 0xff);
    if (T.bps == 2) row[e + 1] = (uint8_t)(v >> 8);
}

// Final stage of a decode job: LL_z (z = target level) -> inverse colour
// transform -> clamp -> interleaved pixels.  If z < levels this fuses the
// inverse of level z+1; all channels are handled by one workgroup.
__global__ void __launch_bounds__(256) k_inv_final(PlanHdr H, const uint8_t *__restrict__ plan,
                                                   uint8_t *__restrict__ ws,
                                                   uint8_t *__restrict__ pix,
                                                   const int32_t *__restrict__ status)
{
    __shared__ int32_t win[3][kWin * kWinPitch];
    const TileGeo *tiles = (const TileGeo *)(plan + H.tiles_off);
    const WorkItem *items = (const WorkItem *)(plan + H.work_off);
    const WorkItem &W = find_item(items, H.fin_first, H.fin_count, blockIdx.x);
    const TileGeo &T = tiles[W.tile];
    uint32_t r = blockIdx.x - W.wg_start;
    uint32_t nsp = W.ntx * W.nty;
    int cg = (int)(r / nsp);
    uint32_t sp = r % nsp;
    int qx0 = (int)(sp % W.ntx) * kTQ, qy0 = (int)(sp / W.ntx) * kTQ;
    int32_t *wsi = (int32_t *)ws;
    int z = T.target_level;
    int c0 = cg * 3, nc = (int)T.channels - c0;
    if (nc > 3) nc = 3;
    int ow, oh;
    if (z < T.levels) {
        const LevelGeo &G = T.lv[z + 1];
        ow = (int)G.w; oh = (int)G.h;
        for (int k = 0; k < nc; k++) stage_inverse(T, z + 1, c0 + k, qx0, qy0, wsi, win[k]);
        __syncthreads();
        for (int k = 0; k < nc; k++) inverse_window(win[k], G.h > 1, G.w > 1);
    } else {
        ow = (int)T.ll_w; oh = (int)T.ll_h;
        for (int k = 0; k < nc; k++) {
            const int32_t *ll = wsi + T.ll_off + (uint64_t)(c0 + k) * T.chan_elems;
            for (int i = threadIdx.x; i < 64 * 64; i += blockDim.x) {
                int x = 2 * qx0 + (i % 64), y = 2 * qy0 + (i / 64);
                if (x < ow && y < oh) win[k][(2 + i / 64) * kWinPitch + 2 + (i % 64)] = ll[(uint64_t)y * T.ll_pitch + x];
            }
        }
        __syncthreads();
    }
    for (int i = threadIdx.x; i < 64 * 64; i += blockDim.x) {
        int x = 2 * qx0 + (i % 64), y = 2 * qy0 + (i / 64);
        if (x >= ow || y >= oh) continue;
        int li = (2 + i / 64) * kWinPitch + 2 + (i % 64);
        if (T.ct == 1) {
            int32_t Y = win[0][li], cb = win[1][li], cr = win[2][li];
            int32_t g = Y - ((cb + cr) >> 2);
            store_pixel(pix, T, x, y, 0, cr + g);
            store_pixel(pix, T, x, y, 1, g);
            store_pixel(pix, T, x, y, 2, cb + g);
        } else {
            for (int k = 0; k < nc; k++) store_pixel(pix, T, x, y, c0 + k, win[k][li]);
        }
    }
    (void)status;
}

// ------------------------------------------------------------------ launch
hipError_t launch_forward_level(const PlanHdr &H, const uint8_t *d_plan, const uint8_t *d_pixels,
                                uint8_t *d_ws, int level, hipStream_t stream)
{
    if (level > (int)H.max_levels || !H.lvl_wgs[level]) return hipSuccess;
    if (level == 0)
        hipLaunchKernelGGL(k_fwd_level0, dim3(H.lvl_wgs[0]), dim3(256), 0, stream, H, d_plan, d_pixels, d_ws);
    else
        hipLaunchKernelGGL(k_fwd_level, dim3(H.lvl_wgs[level]), dim3(256), 0, stream, H, d_plan, d_pixels, d_ws, level);
    return hipGetLastError();
}

hipError_t launch_inverse_level(const PlanHdr &H, const uint8_t *d_plan, uint8_t *d_ws,
                                uint8_t *d_pixels_out, const int32_t *d_status, int level,
                                hipStream_t stream)
{
    if (level == 0) {
        if (H.fin_wgs)
            hipLaunchKernelGGL(k_inv_final, dim3(H.fin_wgs), dim3(256), 0, stream, H, d_plan, d_ws, d_pixels_out, d_status);
    } else if (level <= (int)H.max_levels && H.lvl_wgs[level]) {
        hipLaunchKernelGGL(k_inv_level, dim3(H.lvl_wgs[level]), dim3(256), 0, stream, H, d_plan, d_ws, level);
    }
    return hipGetLastError();
}

}  // namespace isx
