// k_transform.hip -- colour transform + multi-level 2-D 5/3 integer lifting
// (forward and inverse) for gfx950.
//
// Forward level l (Sec. 4: 5/3 Le Gall integer lifting, recursive on LL;
// rows first, then columns):
//   d[n] = x[2n+1] - floor((x[2n] + x[2n+2]) / 2)
//   s[n] = x[2n]   + floor((d[n-1] + d[n] + 2) / 4)
// with whole-sample symmetric extension at the borders.  A workgroup owns a
// TQ x TQ-quad output tile (2TQ x 2TQ input samples); it stages the input
// plus a 2-sample halo (reflected at the image border) in LDS, lifts the
// rows, then the columns, and writes the four subbands.  Two implementations:
// element-wise LDS passes (TQ = 16) and, for TQ = 32, the strip kernels at
// the end of this file, which lift whole lines in registers.  Level 1 reads the
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

// One sample: 1, 2 or 4 bytes, little endian (16/32-bit samples are aligned;
// 4-byte samples hold at most 24 bits).
__device__ inline int32_t sample_at(const uint8_t *px, uint32_t bps, uint32_t c)
{
    if (bps == 1) return px[c];
    if (bps == 2) return ((const uint16_t *)px)[c];
    return (int32_t)((const uint32_t *)px)[c];
}

// Colour-transformed channel c of one pixel: RCT (Y = floor((R+2G+B)/4),
// Cb = B - G, Cr = R - G) or YCoCg-R (Co = R - B, t = B + floor(Co/2),
// Cg = G - t, Y = t + floor(Cg/2)); arithmetic shifts are floors.
__device__ inline int32_t colour_fwd(int32_t R, int32_t G, int32_t B, uint32_t ct, int c)
{
    if (ct == 1) return c == 0 ? ((R + 2 * G + B) >> 2) : (c == 1 ? B - G : R - G);
    const int32_t co = R - B, t = B + (co >> 1), cg = G - t;
    return c == 0 ? t + (cg >> 1) : (c == 1 ? co : cg);
}

// Inverse colour transform in place (a, b, c) = (Y, Cb, Cr) or (Y, Co, Cg) ->
// (R, G, B); ct = 0 leaves the channels.
__device__ inline void colour_inv(uint32_t ct, int32_t &a, int32_t &b, int32_t &c)
{
    if (ct == 1) {
        const int32_t g = a - ((b + c) >> 2);
        const int32_t R = c + g, B = b + g;
        a = R; b = g; c = B;
    } else if (ct == 2) {
        const int32_t t = a - (c >> 1), g = c + t, B = t - (b >> 1);
        a = B + b; b = g; c = B;
    }
}

__device__ inline int32_t load_sample(const uint8_t *pix, const TileGeo &T, int x, int y, int c)
{
    const uint8_t *px = pix + T.pix_offset + (uint64_t)y * T.pix_stride + (uint64_t)x * T.channels * T.bps;
    return sample_at(px, T.bps, (uint32_t)c);
}

__device__ inline int32_t load_colour(const uint8_t *pix, const TileGeo &T, int x, int y, int c)
{
    if (T.ct == 0) return load_sample(pix, T, x, y, c);
    return colour_fwd(load_sample(pix, T, x, y, 0), load_sample(pix, T, x, y, 1), load_sample(pix, T, x, y, 2),
                      T.ct, c);
}

__device__ inline uint32_t wave_or(uint32_t v)
{
    for (int o = 32; o >= 1; o >>= 1) v |= __shfl_xor(v, o, 64);
    return v;
}

// One forward 2-D level over a TQ x TQ-quad tile, one channel per workgroup
// (the channels of a tile are adjacent workgroups, so the pixels they share
// are served from L2).  LDS window: (2TQ + 4)^2 samples.
template <int TQ>
__global__ void __launch_bounds__(256) k_fwd_level(PlanHdr H, const uint8_t *__restrict__ plan,
                                                   const uint8_t *__restrict__ pix,
                                                   uint8_t *__restrict__ ws, int level)
{
    constexpr int WN = 2 * TQ + 4, WP = WN + 1, T2 = 2 * TQ;
    __shared__ int32_t win[WN * WP];
    __shared__ int32_t rmap[WN], cmap[WN];
    const TileGeo *tiles = (const TileGeo *)(plan + H.tiles_off);
    const WorkItem *items = (const WorkItem *)(plan + H.work_off);
    const uint32_t bid = xcd_remap(blockIdx.x, gridDim.x);
    const WorkItem &W = find_item(items, H.lvl_first[level], H.lvl_count[level], bid);
    const TileGeo &T = tiles[W.tile];
    uint32_t r = bid - W.wg_start;
    int c = (int)(r % W.nch);
    uint32_t sp = r / W.nch;
    int qx0 = (int)(sp % W.ntx) * TQ, qy0 = (int)(sp / W.ntx) * TQ;
    const LevelGeo &G = T.lv[level];
    int w = (int)G.w, h = (int)G.h;
    int32_t *wsi = (int32_t *)ws;
    if (threadIdx.x < WN) rmap[threadIdx.x] = reflect_idx(2 * qy0 - 2 + (int)threadIdx.x, h);
    else if (threadIdx.x < 2 * WN) cmap[threadIdx.x - WN] = reflect_idx(2 * qx0 - 2 + (int)threadIdx.x - WN, w);
    __syncthreads();
    // stage window rows [2qy0-2, 2qy0+2TQ+1], same columns (reflected); all
    // of a thread's loads are issued before its LDS stores
    constexpr int NI = (WN * WN + 255) / 256;
    int32_t vals[NI];
    if (level == 1) {
        const uint32_t C = T.channels, bps = T.bps;
        if (bps == 1 && T.ct == 1) {
            // one branch-free loop per channel, so the loads of all samples
            // are scheduled together
            auto rgb = [&](auto f) {
#pragma unroll
                for (int k = 0; k < NI; k++) {
                    const int i = (int)threadIdx.x + 256 * k;
                    if (i >= WN * WN) break;
                    const int lr = i / WN, lc = i % WN;
                    const uint8_t *px =
                        pix + T.pix_offset + (uint64_t)rmap[lr] * T.pix_stride + (uint32_t)cmap[lc] * C;
                    vals[k] = f((int32_t)px[0], (int32_t)px[1], (int32_t)px[2]);
                }
            };
            if (c == 0) rgb([](int32_t R, int32_t Gc, int32_t Bc) { return (R + 2 * Gc + Bc) >> 2; });
            else if (c == 1) rgb([](int32_t, int32_t Gc, int32_t Bc) { return Bc - Gc; });
            else rgb([](int32_t R, int32_t Gc, int32_t) { return R - Gc; });
        } else {
#pragma unroll
            for (int k = 0; k < NI; k++) {
                const int i = (int)threadIdx.x + 256 * k;
                if (i >= WN * WN) break;
                const int lr = i / WN, lc = i % WN;
                const uint8_t *px = pix + T.pix_offset + (uint64_t)rmap[lr] * T.pix_stride + (uint32_t)cmap[lc] * C * bps;
                vals[k] = T.ct ? colour_fwd(sample_at(px, bps, 0), sample_at(px, bps, 1), sample_at(px, bps, 2), T.ct, c)
                               : sample_at(px, bps, (uint32_t)c);
            }
        }
    } else {
        int k = level - 1, which = (k & 1) ? 0 : 1;
        const int32_t *src = wsi + T.tmp_off[which] + (uint64_t)c * T.tmp_chan[which];
        const uint32_t spitch = T.tmp_pitch[which];
#pragma unroll
        for (int k2 = 0; k2 < NI; k2++) {
            const int i = (int)threadIdx.x + 256 * k2;
            if (i >= WN * WN) break;
            const int lr = i / WN, lc = i % WN;
            vals[k2] = src[(uint64_t)rmap[lr] * spitch + cmap[lc]];
        }
    }
#pragma unroll
    for (int k = 0; k < NI; k++) {
        const int i = (int)threadIdx.x + 256 * k;
        if (i >= WN * WN) break;
        win[(i / WN) * WP + (i % WN)] = vals[k];
    }
    __syncthreads();
    // rows: predict at odd columns 1..2TQ+1, update at even columns 2..2TQ (all rows)
    for (int i = threadIdx.x; i < WN * (TQ + 1); i += blockDim.x) {
        int lr = i / (TQ + 1), lc = 1 + 2 * (i % (TQ + 1));
        int32_t *row = win + lr * WP;
        row[lc] -= floor_half(row[lc - 1] + row[lc + 1]);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < WN * TQ; i += blockDim.x) {
        int lr = i / TQ, lc = 2 + 2 * (i % TQ);
        int32_t *row = win + lr * WP;
        row[lc] += floor_quarter_r(row[lc - 1] + row[lc + 1]);
    }
    __syncthreads();
    // columns 2..2TQ+1: predict at odd rows 1..2TQ+1, update at even rows 2..2TQ
    for (int i = threadIdx.x; i < (TQ + 1) * T2; i += blockDim.x) {
        int lc = 2 + (i % T2), lr = 1 + 2 * (i / T2);
        win[lr * WP + lc] -= floor_half(win[(lr - 1) * WP + lc] + win[(lr + 1) * WP + lc]);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < TQ * T2; i += blockDim.x) {
        int lc = 2 + (i % T2), lr = 2 + 2 * (i / T2);
        win[lr * WP + lc] += floor_quarter_r(win[(lr - 1) * WP + lc] + win[(lr + 1) * WP + lc]);
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
    for (int i = threadIdx.x; i < TQ * TQ; i += blockDim.x) {
        int ii = i % TQ, jj = i / TQ;
        int qx = qx0 + ii, qy = qy0 + jj;
        int32_t vLL = win[(2 + 2 * jj) * WP + 2 + 2 * ii];
        int32_t vHL = win[(2 + 2 * jj) * WP + 3 + 2 * ii];
        int32_t vLH = win[(3 + 2 * jj) * WP + 2 + 2 * ii];
        int32_t vHH = win[(3 + 2 * jj) * WP + 3 + 2 * ii];
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
    // per-block accumulation (the whole quad tile lies in one 128 cell)
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
    const uint32_t bid = xcd_remap(blockIdx.x, gridDim.x);
    const WorkItem &W = find_item(items, H.lvl_first[0], H.lvl_count[0], bid);
    const TileGeo &T = tiles[W.tile];
    uint32_t r = bid - W.wg_start;
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
// rmap/cmap hold the reflected coordinates of the window rows/columns.
template <int TQ, int KB>
__device__ inline void stage_inverse(const TileGeo &T, int level, int c, const int32_t *rmap,
                                     const int32_t *cmap, const int32_t *wsi, int32_t *win)
{
    constexpr int WN = 2 * TQ + 4, WP = WN + 1;
    const LevelGeo &G = T.lv[level];
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
    if (KB == 0) {  // element by element (fewest registers)
        for (int i = threadIdx.x; i < WN * WN; i += blockDim.x) {
            int lr = i / WN, lc = i % WN;
            int gy = rmap[lr], gx = cmap[lc];
            int py = gy & 1, px = gx & 1;
            uint64_t ry = (uint64_t)(gy >> 1);
            int32_t v;
            if (!py) v = !px ? ll[ry * llp + (gx >> 1)] : hl[ry * G.pitch[1] + (gx >> 1)];
            else v = !px ? lh[ry * G.pitch[0] + (gx >> 1)] : hh[ry * G.pitch[2] + (gx >> 1)];
            win[lr * WP + lc] = v;
        }
        return;
    }
    // band by band (window row/column parity = band type, as the window
    // starts at an even position and reflection keeps parity): a wave reads
    // consecutive elements of one band row; KB loads in flight per thread
    constexpr int HN = WN / 2, NB = HN * HN, NT = 4 * NB, KBn = KB > 0 ? KB : 1;
    for (int base = 0; base < NT; base += 256 * KBn) {
        int32_t v[KBn];
        int dst[KBn];
#pragma unroll
        for (int k = 0; k < KBn; k++) {
            const int i = base + (int)threadIdx.x + 256 * k;
            dst[k] = -1;
            if (i < NT) {
                const int b = i / NB, j = i - b * NB;  // 0 LL, 1 HL, 2 LH, 3 HH
                const int br = j / HN, bc = j - br * HN;
                const int lr = 2 * br + (b >> 1), lc = 2 * bc + (b & 1);
                const int32_t *src = b == 0 ? ll : (b == 1 ? hl : (b == 2 ? lh : hh));
                const uint32_t pitch = b == 0 ? llp : G.pitch[b == 1 ? 1 : (b == 2 ? 0 : 2)];
                v[k] = src[(uint64_t)(rmap[lr] >> 1) * pitch + (cmap[lc] >> 1)];
                dst[k] = lr * WP + lc;
            }
        }
#pragma unroll
        for (int k = 0; k < KBn; k++)
            if (dst[k] >= 0) win[dst[k]] = v[k];
    }
}

// Undo the lifting in the window: columns (unless the level has one row),
// then rows (unless it has one column).  Valid output: [2, 2TQ+2)^2.
template <int TQ>
__device__ inline void inverse_window(int32_t *win, bool do_cols, bool do_rows)
{
    constexpr int WN = 2 * TQ + 4, WP = WN + 1, T2 = 2 * TQ, NC = WN - 1;
    if (do_cols) {
        // undo update at even rows 2..2TQ+2, columns 1..2TQ+3
        for (int i = threadIdx.x; i < (TQ + 1) * NC; i += blockDim.x) {
            int lc = 1 + (i % NC), lr = 2 + 2 * (i / NC);
            win[lr * WP + lc] -= floor_quarter_r(win[(lr - 1) * WP + lc] + win[(lr + 1) * WP + lc]);
        }
        __syncthreads();
        // undo predict at odd rows 3..2TQ+1
        for (int i = threadIdx.x; i < TQ * NC; i += blockDim.x) {
            int lc = 1 + (i % NC), lr = 3 + 2 * (i / NC);
            win[lr * WP + lc] += floor_half(win[(lr - 1) * WP + lc] + win[(lr + 1) * WP + lc]);
        }
        __syncthreads();
    }
    if (do_rows) {
        for (int i = threadIdx.x; i < T2 * (TQ + 1); i += blockDim.x) {
            int lr = 2 + (i / (TQ + 1)), lc = 2 + 2 * (i % (TQ + 1));
            int32_t *row = win + lr * WP;
            row[lc] -= floor_quarter_r(row[lc - 1] + row[lc + 1]);
        }
        __syncthreads();
        for (int i = threadIdx.x; i < T2 * TQ; i += blockDim.x) {
            int lr = 2 + (i / TQ), lc = 3 + 2 * (i % TQ);
            int32_t *row = win + lr * WP;
            row[lc] += floor_half(row[lc - 1] + row[lc + 1]);
        }
        __syncthreads();
    }
}

// Interleaved coordinate g (reflected into the image) -> band index relative
// to the level's arena window, clamped into it, with g's parity in bit 0.
// Positions the window does not hold only feed outputs nobody reads.
__device__ inline int32_t win_idx(int g, uint32_t o, uint32_t n)
{
    int r = (g >> 1) - (int)o;
    r = r < 0 ? 0 : (r >= (int)n ? (int)n - 1 : r);
    return (r << 1) | (g & 1);
}

template <int TQ>
__device__ inline void fill_maps(int32_t *rmap, int32_t *cmap, int qx0, int qy0, int w, int h, const LevelGeo &G)
{
    constexpr int WN = 2 * TQ + 4;
    if (threadIdx.x < WN)
        rmap[threadIdx.x] = win_idx(reflect_idx(2 * qy0 - 2 + (int)threadIdx.x, h), G.wy0, G.wh);
    else if (threadIdx.x < 2 * WN)
        cmap[threadIdx.x - WN] = win_idx(reflect_idx(2 * qx0 - 2 + (int)threadIdx.x - WN, w), G.wx0, G.ww);
}

// Inverse of level `level` into LL_{level-1} (an intermediate level).
template <int TQ>
__global__ void __launch_bounds__(256) k_inv_level(PlanHdr H, const uint8_t *__restrict__ plan,
                                                   uint8_t *__restrict__ ws, int level)
{
    constexpr int WN = 2 * TQ + 4, WP = WN + 1, T2 = 2 * TQ;
    __shared__ int32_t win[WN * WP];
    __shared__ int32_t rmap[WN], cmap[WN];
    const TileGeo *tiles = (const TileGeo *)(plan + H.tiles_off);
    const WorkItem *items = (const WorkItem *)(plan + H.work_off);
    const uint32_t bid = xcd_remap(blockIdx.x, gridDim.x);
    const WorkItem &W = find_item(items, H.lvl_first[level], H.lvl_count[level], bid);
    const TileGeo &T = tiles[W.tile];
    uint32_t r = bid - W.wg_start;
    int c = (int)(r % W.nch);
    uint32_t sp = r / W.nch;
    int qx0 = (int)(W.qx0 + (sp % W.ntx) * TQ), qy0 = (int)(W.qy0 + (sp / W.ntx) * TQ);
    int32_t *wsi = (int32_t *)ws;
    const LevelGeo &G = T.lv[level];
    fill_maps<TQ>(rmap, cmap, qx0, qy0, (int)G.w, (int)G.h, G);
    __syncthreads();
    stage_inverse<TQ, 6>(T, level, c, rmap, cmap, wsi, win);
    __syncthreads();
    inverse_window<TQ>(win, G.h > 1, G.w > 1);
    // LL_{level-1} is the low band of level-1: store the part inside that
    // level's window
    int k = level - 1, which = (k & 1) ? 0 : 1;
    const LevelGeo &D = T.lv[k];
    int32_t *dst = wsi + T.tmp_off[which] + (uint64_t)c * T.tmp_chan[which];
    uint32_t dp = T.tmp_pitch[which];
    for (int i = threadIdx.x; i < T2 * T2; i += blockDim.x) {
        int x = 2 * qx0 + (i % T2) - (int)D.wx0, y = 2 * qy0 + (i / T2) - (int)D.wy0;
        if ((uint32_t)x < D.ww && (uint32_t)y < D.wh)
            dst[(uint64_t)y * dp + x] = win[(2 + i / T2) * WP + 2 + (i % T2)];
    }
}

// Final stage of a decode job: LL_z (z = target level) -> inverse colour
// transform -> clamp -> interleaved pixels.  If z < levels this fuses the
// inverse of level z+1.  The channels of a group (3 with the colour
// transform) go through one LDS window in turn; each thread keeps its output
// samples per channel in registers, then converts and stores 4 horizontally
// adjacent pixels at a time.
template <int TQ>
__global__ void __launch_bounds__(256) k_inv_final(PlanHdr H, const uint8_t *__restrict__ plan,
                                                   uint8_t *__restrict__ ws,
                                                   uint8_t *__restrict__ pix,
                                                   const int32_t *__restrict__ status)
{
    constexpr int WN = 2 * TQ + 4, WP = WN + 1, T2 = 2 * TQ;
    constexpr int TPR = T2 / 4;          // threads per output row (4 pixels each)
    constexpr int RSTEP = 256 / TPR;     // rows between a thread's rows
    constexpr int NR = T2 / RSTEP;       // rows per thread
    __shared__ int32_t win[WN * WP];
    __shared__ int32_t rmap[WN], cmap[WN];
    const TileGeo *tiles = (const TileGeo *)(plan + H.tiles_off);
    const WorkItem *items = (const WorkItem *)(plan + H.work_off);
    const uint32_t bid = xcd_remap(blockIdx.x, gridDim.x);
    const WorkItem &W = find_item(items, H.fin_first, H.fin_count, bid);
    const TileGeo &T = tiles[W.tile];
    uint32_t r = bid - W.wg_start;
    int cg = (int)(r % W.nch);
    uint32_t sp = r / W.nch;
    int qx0 = (int)(W.qx0 + (sp % W.ntx) * TQ), qy0 = (int)(W.qy0 + (sp / W.ntx) * TQ);
    int32_t *wsi = (int32_t *)ws;
    int z = T.target_level;
    int c0 = cg * 3, nc = (int)T.channels - c0;
    if (nc > 3) nc = 3;
    int ow, oh;
    const bool fused = z < T.levels;
    if (fused) { ow = (int)T.lv[z + 1].w; oh = (int)T.lv[z + 1].h; }
    else { ow = (int)T.ll_w; oh = (int)T.ll_h; }
    if (fused) fill_maps<TQ>(rmap, cmap, qx0, qy0, ow, oh, T.lv[z + 1]);
    // output region of the level-z image (all of it for a full decode)
    const int rx0 = (int)T.rx0, ry0 = (int)T.ry0, rx1 = (int)T.rx1, ry1 = (int)T.ry1;
    const int tx = (threadIdx.x % TPR) * 4, ty = threadIdx.x / TPR;
    int32_t v[3][NR][4];
#pragma unroll
    for (int k = 0; k < 3; k++) {
        if (k >= nc) {
#pragma unroll
            for (int rr = 0; rr < NR; rr++)
#pragma unroll
                for (int xx = 0; xx < 4; xx++) v[k][rr][xx] = 0;
            continue;
        }
        __syncthreads();
        if (fused) {
            stage_inverse<TQ, 0>(T, z + 1, c0 + k, rmap, cmap, wsi, win);
            __syncthreads();
            inverse_window<TQ>(win, oh > 1, ow > 1);
        } else {
            const int32_t *ll = wsi + T.ll_off + (uint64_t)(c0 + k) * T.chan_elems;
            for (int i = threadIdx.x; i < T2 * T2; i += blockDim.x) {
                int x = 2 * qx0 + (i % T2), y = 2 * qy0 + (i / T2);
                if (x >= rx0 && x < rx1 && y >= ry0 && y < ry1)
                    win[(2 + i / T2) * WP + 2 + (i % T2)] =
                        ll[(uint64_t)(y - (int)T.ll_wy0) * T.ll_pitch + (x - (int)T.ll_wx0)];
            }
            __syncthreads();
        }
#pragma unroll
        for (int rr = 0; rr < NR; rr++)
#pragma unroll
            for (int xx = 0; xx < 4; xx++) v[k][rr][xx] = win[(2 + ty + RSTEP * rr) * WP + 2 + tx + xx];
    }
    const int32_t top = (1 << T.bits) - 1;
    const uint32_t C = T.channels, bps = T.bps;
    // RGB u8 rows whose start is 4-byte aligned: stage each output row in LDS
    // (the window is free now) and store whole dwords, contiguous per row
    // (a region starting at an odd column takes the per-pixel path)
    const uint64_t rowbase0 = T.pix_offset + (uint64_t)(2 * qx0 - rx0) * 3;
    const bool staged = bps == 1 && C == 3 && 2 * qx0 >= rx0 && ((rowbase0 | T.pix_stride) & 3u) == 0 &&
                        (((uintptr_t)pix) & 3u) == 0;
    if (staged) {
        __syncthreads();
        uint8_t *ob = (uint8_t *)win;  // T2 rows x (T2 * 3) bytes
#pragma unroll
        for (int rr = 0; rr < NR; rr++) {
            int ly = ty + RSTEP * rr;
#pragma unroll
            for (int xx = 0; xx < 4; xx++) {
                int32_t o0 = v[0][rr][xx], o1 = v[1][rr][xx], o2 = v[2][rr][xx];
                colour_inv(T.ct, o0, o1, o2);
                o0 = o0 < 0 ? 0 : (o0 > top ? top : o0);
                o1 = o1 < 0 ? 0 : (o1 > top ? top : o1);
                o2 = o2 < 0 ? 0 : (o2 > top ? top : o2);
                uint8_t *q = ob + ly * (T2 * 3) + (tx + xx) * 3;
                q[0] = (uint8_t)o0; q[1] = (uint8_t)o1; q[2] = (uint8_t)o2;
            }
        }
        __syncthreads();
        const int nx = min(T2, rx1 - 2 * qx0);  // valid pixels in the row
        const int nbytes = nx * 3;
        const int ndw = nbytes / 4;
        for (int i = threadIdx.x; i < T2 * (T2 * 3 / 4); i += blockDim.x) {
            int ly = i / (T2 * 3 / 4), k = i % (T2 * 3 / 4);
            int y = 2 * qy0 + ly;
            if (y < ry0 || y >= ry1) continue;
            uint8_t *row = pix + rowbase0 + (uint64_t)(y - ry0) * T.pix_stride;
            const uint8_t *src = ob + ly * (T2 * 3);
            if (k < ndw) ((uint32_t *)row)[k] = ((const uint32_t *)src)[k];
            else if (k == ndw) for (int b = 4 * ndw; b < nbytes; b++) row[b] = src[b];
        }
        return;
    }
#pragma unroll
    for (int rr = 0; rr < NR; rr++) {
        int y = 2 * qy0 + ty + RSTEP * rr;
        if (y < ry0 || y >= ry1) continue;
        int x0 = 2 * qx0 + tx;
        int32_t o[3][4];
#pragma unroll
        for (int xx = 0; xx < 4; xx++) {
#pragma unroll
            for (int k = 0; k < 3; k++) o[k][xx] = v[k][rr][xx];
            colour_inv(T.ct, o[0][xx], o[1][xx], o[2][xx]);
#pragma unroll
            for (int k = 0; k < 3; k++) o[k][xx] = o[k][xx] < 0 ? 0 : (o[k][xx] > top ? top : o[k][xx]);
        }
        uint8_t *row = pix + T.pix_offset + (uint64_t)(y - ry0) * T.pix_stride;  // region row
        if (bps == 1 && C == 3 && x0 >= rx0 && x0 + 3 < rx1 &&
            ((((uintptr_t)(row + (uint32_t)(x0 - rx0) * 3)) & 3u) == 0)) {
            uint32_t *d = (uint32_t *)(row + (uint32_t)(x0 - rx0) * 3);
            d[0] = (uint32_t)o[0][0] | ((uint32_t)o[1][0] << 8) | ((uint32_t)o[2][0] << 16) | ((uint32_t)o[0][1] << 24);
            d[1] = (uint32_t)o[1][1] | ((uint32_t)o[2][1] << 8) | ((uint32_t)o[0][2] << 16) | ((uint32_t)o[1][2] << 24);
            d[2] = (uint32_t)o[2][2] | ((uint32_t)o[0][3] << 8) | ((uint32_t)o[1][3] << 16) | ((uint32_t)o[2][3] << 24);
        } else {
            for (int xx = 0; xx < 4; xx++) {
                int x = x0 + xx;
                if (x < rx0) continue;
                if (x >= rx1) break;
#pragma unroll
                for (int k = 0; k < 3; k++) {
                    if (k >= nc) break;
                    uint32_t e = ((uint32_t)(x - rx0) * C + c0 + k) * bps;
                    if (bps == 1) row[e] = (uint8_t)o[k][xx];
                    else if (bps == 2) *(uint16_t *)(row + e) = (uint16_t)o[k][xx];
                    else *(uint32_t *)(row + e) = (uint32_t)o[k][xx];
                }
            }
        }
    }
    (void)status;
}

// ------------------------------------------------------------------ strips
// The 32x32-quad tile kernels below lift whole lines in registers.  The
// window is split into four strips of 16 outputs, one per wave.  In a row
// pass each lane owns one window row of its wave's strip; in a column pass
// each lane owns one window column.  A line of a strip takes 19 window
// samples and gives the 16 outputs at window positions 16s+2 .. 16s+17
// (s = strip), which is the 2-sample halo of the 5/3 filter on each side.
namespace strips {
constexpr int TQ = 32, WN = 2 * TQ + 4, WP = WN + 1;  // odd pitch: a column is bank-conflict free

// Forward lifting of the samples at positions p .. p+18 (p even): outputs at
// p+2 .. p+17, low-pass s at even positions, high-pass d at odd ones.
__device__ inline void lift_fwd16(const int32_t (&x)[19], int32_t (&o)[16])
{
    int32_t d[9];  // d at p+1, p+3, .., p+17
#pragma unroll
    for (int k = 0; k < 9; k++) d[k] = x[2 * k + 1] - floor_half(x[2 * k] + x[2 * k + 2]);
#pragma unroll
    for (int k = 0; k < 8; k++) {
        o[2 * k] = x[2 * k + 2] + floor_quarter_r(d[k] + d[k + 1]);
        o[2 * k + 1] = d[k + 1];
    }
}

// Inverse lifting of the interleaved coefficients at positions p+1 .. p+19
// (x[j] at p+1+j: odd j hold s, even j hold d): samples at p+2 .. p+17.
__device__ inline void lift_inv16(const int32_t (&x)[19], int32_t (&o)[16])
{
    int32_t e[9];  // samples at p+2, p+4, .., p+18
#pragma unroll
    for (int k = 0; k < 9; k++) e[k] = x[2 * k + 1] - floor_quarter_r(x[2 * k] + x[2 * k + 2]);
#pragma unroll
    for (int k = 0; k < 8; k++) {
        o[2 * k] = e[k];
        o[2 * k + 1] = x[2 * k + 2] + floor_half(e[k] + e[k + 1]);
    }
}

// Forward row lifting at one position from the raw samples p[-2..2] of its
// row (for window rows the row pass leaves out).
__device__ inline int32_t row_lift_fwd_at(const int32_t *p, bool odd)
{
    const int32_t xm2 = p[-2], xm1 = p[-1], x0 = p[0], xp1 = p[1], xp2 = p[2];
    const int32_t hv = x0 - floor_half(xm1 + xp1);
    const int32_t dm = xm1 - floor_half(xm2 + x0), dp = xp1 - floor_half(x0 + xp2);
    const int32_t lv = x0 + floor_quarter_r(dm + dp);
    return odd ? hv : lv;
}

// Inverse column lifting at one position from the coefficients p[-2WP..2WP]
// of its column (for window columns the column pass leaves out).
__device__ inline int32_t col_lift_inv_at(const int32_t *p, bool odd)
{
    const int32_t xm2 = p[-2 * WP], xm1 = p[-WP], x0 = p[0], xp1 = p[WP], xp2 = p[2 * WP];
    const int32_t ev = x0 - floor_quarter_r(xm1 + xp1);
    const int32_t em = xm1 - floor_quarter_r(xm2 + x0), ep = xp1 - floor_quarter_r(x0 + xp2);
    const int32_t ov = x0 + floor_half(em + ep);
    return odd ? ov : ev;
}

// |v| / step with the sign of v (dead-zone quantiser), the division by the
// tile's precomputed multiplier.
__device__ inline int32_t quantise(int32_t v, uint32_t qmul, uint32_t qsh)
{
    const uint32_t a = v < 0 ? 0u - (uint32_t)v : (uint32_t)v;
    const uint32_t t = __umulhi(qmul, a);
    const uint32_t q = (t + ((a - t) >> 1)) >> qsh;
    return v < 0 ? -(int32_t)q : (int32_t)q;
}

// Interleaved RGB u8: the colour-transformed channel of 4 pixels held in 3
// little-endian dwords.
template <int CT, int CH>
__device__ inline int32_t rgb_channel(uint32_t R, uint32_t G, uint32_t B)
{
    const int32_t r = (int32_t)R, g = (int32_t)G, b = (int32_t)B;
    if (CT == 1) return CH == 0 ? ((r + 2 * g + b) >> 2) : (CH == 1 ? b - g : r - g);
    const int32_t co = r - b, t = b + (co >> 1), cg = g - t;
    return CH == 0 ? t + (cg >> 1) : (CH == 1 ? co : cg);
}

// Window of a tile at level 1 from interleaved RGB u8 pixels: each task
// loads 12 bytes (4 pixels) of a window row; the window starts at pixel
// 2 qx0 - 2 and the loads at 2 qx0 - 4, so every load is dword aligned.
//
// Any tile, including the image borders: the window's rows come through the
// reflected row map, and a group of 4 window columns whose pixels all lie
// inside the image is loaded as 12 bytes; the groups at the left and right
// borders gather their 4 pixels through the reflected column map, byte by
// byte, into the same 3-dword form.  `tb` is the tile's first pixel row and
// dword aligned, as is the stride.
// AL: every row starts 4-byte aligned; else a group's 12 bytes come from the
// four aligned words around them, shifted into place.  Kept out of line: the
// twelve variants inlined into the kernel make it several times larger and
// slower (instruction cache).
template <int CT, int CH, bool AL>
__device__ __noinline__ void stage_rgb8(const uint8_t *tb, uint32_t stride, const int32_t *rmap, const int32_t *cmap,
                                  int qx0, int w, int32_t *win)
{
    constexpr int NG = 18, NT = WN * NG, NK = (NT + 255) / 256;
    uint32_t d[NK][3];
#pragma unroll
    for (int k = 0; k < NK; k++) {
        const int t = (int)threadIdx.x + 256 * k;
        if (t < NT) {
            const int lr = t / NG, g = t - lr * NG;
            const uint8_t *row = tb + (uint64_t)rmap[lr] * stride;
            const int p0 = 2 * qx0 - 4 + 4 * g;
            if (p0 >= 0 && p0 + 3 < w) {
                if (AL) {
                    const uint32_t *p = (const uint32_t *)(row + 3 * p0);
                    d[k][0] = p[0]; d[k][1] = p[1]; d[k][2] = p[2];
                } else {
                    // the aligned words holding bytes 3 p0 .. 3 p0 + 11 (the
                    // fourth only when they straddle it: it holds the last
                    // byte, so it lies in the same page)
                    const uint8_t *pb = row + 3 * p0;
                    const uint32_t m = (uint32_t)(uintptr_t)pb & 3u;
                    const uint32_t *p = (const uint32_t *)(pb - m);
                    const uint32_t a0 = p[0], a1 = p[1], a2 = p[2];
                    const uint32_t a3 = m ? p[3] : 0u;
                    d[k][0] = __builtin_amdgcn_alignbyte(a1, a0, m);
                    d[k][1] = __builtin_amdgcn_alignbyte(a2, a1, m);
                    d[k][2] = __builtin_amdgcn_alignbyte(a3, a2, m);
                }
            } else {
                uint32_t q[3] = {0, 0, 0};
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    int lc = 4 * g - 2 + e;
                    lc = lc < 0 ? 0 : (lc > WN - 1 ? WN - 1 : lc);  // outside the window: never stored
                    const uint8_t *px = row + 3 * cmap[lc];
#pragma unroll
                    for (int c = 0; c < 3; c++) {
                        const int b = 3 * e + c;
                        q[b >> 2] |= (uint32_t)px[c] << (8 * (b & 3));
                    }
                }
                d[k][0] = q[0]; d[k][1] = q[1]; d[k][2] = q[2];
            }
        }
    }
#pragma unroll
    for (int k = 0; k < NK; k++) {
        const int t = (int)threadIdx.x + 256 * k;
        if (t < NT) {
            const int lr = t / NG, g = t - lr * NG;
            const uint32_t a = d[k][0], b = d[k][1], c = d[k][2];
            int32_t v[4];
            v[0] = rgb_channel<CT, CH>(a & 0xff, (a >> 8) & 0xff, (a >> 16) & 0xff);
            v[1] = rgb_channel<CT, CH>(a >> 24, b & 0xff, (b >> 8) & 0xff);
            v[2] = rgb_channel<CT, CH>((b >> 16) & 0xff, b >> 24, c & 0xff);
            v[3] = rgb_channel<CT, CH>((c >> 8) & 0xff, (c >> 16) & 0xff, c >> 24);
            int32_t *row = win + lr * WP + 4 * g - 2;
            if (g > 0) { row[0] = v[0]; row[1] = v[1]; }          // columns -2, -1 are outside
            if (g < NG - 1) { row[2] = v[2]; row[3] = v[3]; }     // columns 68, 69 are outside
        }
    }
}
}  // namespace strips

// One forward 2-D level over a 32x32-quad tile of one channel, by strips:
// stage the reflected 68x68 window, lift window rows 1..64 (a lane per row),
// then window columns 2..65 (a lane per column) and store the coefficients
// from the column pass: a wave stores 32 consecutive coefficients of two
// bands per instruction.  Rows 0, 65 and 66 are row-lifted where the column
// pass needs them.  Same results as the element-wise kernel above.
__global__ void __launch_bounds__(256) k_fwd_strips(PlanHdr H, const uint8_t *__restrict__ plan,
                                                    const uint8_t *__restrict__ pix,
                                                    uint8_t *__restrict__ ws, int level)
{
    using namespace strips;
    __shared__ __align__(16) int32_t win[WN * WP];
    __shared__ int32_t rmap[WN], cmap[WN];
    const TileGeo *tiles = (const TileGeo *)(plan + H.tiles_off);
    const WorkItem *items = (const WorkItem *)(plan + H.work_off);
    const uint32_t bid = xcd_remap(blockIdx.x, gridDim.x);
    const WorkItem &W = find_item(items, H.lvl_first[level], H.lvl_count[level], bid);
    const TileGeo &T = tiles[W.tile];
    const uint32_t r = bid - W.wg_start;
    const int c = (int)(r % W.nch);
    const uint32_t sp = r / W.nch;
    const int qx0 = (int)(sp % W.ntx) * TQ, qy0 = (int)(sp / W.ntx) * TQ;
    const LevelGeo &G = T.lv[level];
    const int w = (int)G.w, h = (int)G.h;
    int32_t *wsi = (int32_t *)ws;
    const int lane = (int)(threadIdx.x & 63);
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if (threadIdx.x < WN) rmap[threadIdx.x] = reflect_idx(2 * qy0 - 2 + (int)threadIdx.x, h);
    else if (threadIdx.x < 2 * WN) cmap[threadIdx.x - WN] = reflect_idx(2 * qx0 - 2 + (int)threadIdx.x - WN, w);
    __syncthreads();
    // ---- stage the window (rows and columns 0..67)
    if (level == 1) {
        const uint32_t C = T.channels, bps = T.bps;
        const uint8_t *tb = pix + T.pix_offset;
        const bool fast = bps == 1 && C == 3 && T.ct != 0;
        const bool al = ((((uintptr_t)tb) | T.pix_stride) & 3u) == 0;
        if (fast && al) {
            if (T.ct == 1) {
                if (c == 0) stage_rgb8<1, 0, true>(tb, T.pix_stride, rmap, cmap, qx0, w, win);
                else if (c == 1) stage_rgb8<1, 1, true>(tb, T.pix_stride, rmap, cmap, qx0, w, win);
                else stage_rgb8<1, 2, true>(tb, T.pix_stride, rmap, cmap, qx0, w, win);
            } else {
                if (c == 0) stage_rgb8<2, 0, true>(tb, T.pix_stride, rmap, cmap, qx0, w, win);
                else if (c == 1) stage_rgb8<2, 1, true>(tb, T.pix_stride, rmap, cmap, qx0, w, win);
                else stage_rgb8<2, 2, true>(tb, T.pix_stride, rmap, cmap, qx0, w, win);
            }
        } else if (fast) {
            if (T.ct == 1) {
                if (c == 0) stage_rgb8<1, 0, false>(tb, T.pix_stride, rmap, cmap, qx0, w, win);
                else if (c == 1) stage_rgb8<1, 1, false>(tb, T.pix_stride, rmap, cmap, qx0, w, win);
                else stage_rgb8<1, 2, false>(tb, T.pix_stride, rmap, cmap, qx0, w, win);
            } else {
                if (c == 0) stage_rgb8<2, 0, false>(tb, T.pix_stride, rmap, cmap, qx0, w, win);
                else if (c == 1) stage_rgb8<2, 1, false>(tb, T.pix_stride, rmap, cmap, qx0, w, win);
                else stage_rgb8<2, 2, false>(tb, T.pix_stride, rmap, cmap, qx0, w, win);
            }
        } else {
            // any format, or a tile at the image border: element by element,
            // six loads in flight per thread
            constexpr int NI = (WN * WN + 255) / 256, KB = 6;
            for (int k0 = 0; k0 < NI; k0 += KB) {
                int32_t vals[KB];
#pragma unroll
                for (int k = 0; k < KB; k++) {
                    const int i = (int)threadIdx.x + 256 * (k0 + k);
                    if (i < WN * WN) {
                        const int lr = i / WN, lc = i % WN;
                        const uint8_t *px = tb + (uint64_t)rmap[lr] * T.pix_stride + (uint32_t)cmap[lc] * C * bps;
                        vals[k] = T.ct ? colour_fwd(sample_at(px, bps, 0), sample_at(px, bps, 1), sample_at(px, bps, 2),
                                                    T.ct, c)
                                       : sample_at(px, bps, (uint32_t)c);
                    }
                }
#pragma unroll
                for (int k = 0; k < KB; k++) {
                    const int i = (int)threadIdx.x + 256 * (k0 + k);
                    if (i < WN * WN) win[(i / WN) * WP + (i % WN)] = vals[k];
                }
            }
        }
    } else {
        // LL of the previous level: a lane per window column (0..63), a wave
        // per fourth row; then columns 64..67
        const int which = ((level - 1) & 1) ? 0 : 1;
        const int32_t *src = wsi + T.tmp_off[which] + (uint64_t)c * T.tmp_chan[which];
        const uint32_t spitch = T.tmp_pitch[which];
        constexpr int NR = WN / 4;
        int32_t v[NR];
        const int32_t *sc = src + cmap[lane];
#pragma unroll
        for (int k = 0; k < NR; k++) v[k] = sc[(uint64_t)rmap[wv + 4 * k] * spitch];
        int32_t e[2];
#pragma unroll
        for (int k = 0; k < 2; k++) {
            const int t = (int)threadIdx.x + 256 * k;
            if (t < 4 * WN) e[k] = src[(uint64_t)rmap[t >> 2] * spitch + cmap[64 + (t & 3)]];
        }
#pragma unroll
        for (int k = 0; k < NR; k++) win[(wv + 4 * k) * WP + lane] = v[k];
#pragma unroll
        for (int k = 0; k < 2; k++) {
            const int t = (int)threadIdx.x + 256 * k;
            if (t < 4 * WN) win[(t >> 2) * WP + 64 + (t & 3)] = e[k];
        }
    }
    __syncthreads();
    // ---- row pass: window rows 1..64, columns 16wv .. 16wv+18 -> 16wv+2 ..
    {
        int32_t x[19], o[16];
        int32_t *row = win + (1 + lane) * WP + 16 * wv;
#pragma unroll
        for (int j = 0; j < 19; j++) x[j] = row[j];
        lift_fwd16(x, o);
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 16; j++) row[2 + j] = o[j];
    }
    __syncthreads();
    // ---- column pass: window column 2 + lane, rows 16wv .. 16wv+18
    const int cc = 2 + lane;
    const bool odd = (lane & 1) != 0;  // column parity: high-pass column
    int32_t o[16];
    {
        int32_t x[19];
        const int32_t *col = win + 16 * wv * WP + cc;
#pragma unroll
        for (int j = 0; j < 19; j++) x[j] = col[j * WP];
        if (wv == 0) x[0] = row_lift_fwd_at(win + cc, odd);
        if (wv == 3) {
            x[17] = row_lift_fwd_at(win + 65 * WP + cc, odd);
            x[18] = row_lift_fwd_at(win + 66 * WP + cc, odd);
        }
        lift_fwd16(x, o);
    }
    // ---- outputs: even window rows of the strip give L rows, odd ones H rows
    const int llw = (w + 1) / 2, llh = (h + 1) / 2, hw = w / 2, hh = h / 2;
    const bool last = (level == T.levels);
    int32_t *llout;
    uint32_t llpitch;
    if (last) {
        llout = wsi + T.ll_off + (uint64_t)c * T.chan_elems;
        llpitch = T.ll_pitch;
    } else {
        const int which = (level & 1) ? 0 : 1;
        llout = wsi + T.tmp_off[which] + (uint64_t)c * T.tmp_chan[which];
        llpitch = T.tmp_pitch[which];
    }
    const int qx = qx0 + (lane >> 1);
    const bool xin = qx < (odd ? hw : llw);
    const uint32_t step = T.qstep, qmul = T.qmul, qsh = T.qsh;
    // OR of the magnitudes per row parity; the OR of the values themselves
    // has its sign bit set iff one of them is negative
    uint32_t or_e = 0, or_o = 0, sg_e = 0, sg_o = 0;
    const int qyb = qy0 + 8 * wv;
#pragma unroll
    for (int j = 0; j < 16; j++) {
        const int qy = qyb + (j >> 1);
        int32_t v = o[j];
        if (j & 1) {
            if (step > 1) v = quantise(v, qmul, qsh);
            if (xin && qy < hh) {
                or_o |= v < 0 ? 0u - (uint32_t)v : (uint32_t)v;
                sg_o |= (uint32_t)v;
            }
        } else {
            if (step > 1 && odd) v = quantise(v, qmul, qsh);
            if (xin && qy < llh) {
                or_e |= v < 0 ? 0u - (uint32_t)v : (uint32_t)v;
                sg_e |= (uint32_t)v;
            }
        }
        o[j] = v;
    }
    uint32_t negs = (sg_e >> 31) | ((sg_o >> 31) << 1);
    // the four 32x32 bands of the tile go through LDS (the window is free
    // once every column pass has read it) and out in 16-byte pieces: a wave
    // stores eight whole band rows per instruction
    constexpr int BP = 36, BS = 32 * BP + 4;  // row and band pitch of the staging (16-byte rows)
    __syncthreads();
    {
        int32_t *stg = win + (odd ? BS : 0) + (lane >> 1);  // LL | HL, then + 2 BS: LH | HH
#pragma unroll
        for (int j = 0; j < 16; j++) stg[((j & 1) ? 2 * BS : 0) + (8 * wv + (j >> 1)) * BP] = o[j];
    }
    __syncthreads();
    {
        int32_t *const bptr[4] = {llout, wsi + G.off[1] + (uint64_t)c * T.chan_elems,
                                  wsi + G.off[0] + (uint64_t)c * T.chan_elems,
                                  wsi + G.off[2] + (uint64_t)c * T.chan_elems};
        const uint32_t bpitch[4] = {llpitch, G.pitch[1], G.pitch[0], G.pitch[2]};
        const int bw[4] = {llw, hw, llw, hw}, bh[4] = {llh, llh, hh, hh};
        const bool b16 = level <= 2 && ((T.coef16 >> (level - 1)) & 1u);  // the level's H bands as int16
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const int b = k;  // band of this pass: thread t stores row t >> 3, piece t & 7
            const int row = (int)threadIdx.x >> 3, part = (int)threadIdx.x & 7;
            const int qy = qy0 + row, qxs = qx0 + 4 * part;
            if (qy >= bh[b] || qxs >= bw[b]) continue;
            const int32_t *src = win + b * BS + row * BP + 4 * part;
            if (b16 && b > 0) {
                int16_t *dst = (int16_t *)bptr[b] + (uint64_t)qy * bpitch[b] + qxs;
                if (qxs + 3 < bw[b])
                    *(short4 *)dst = make_short4((short)src[0], (short)src[1], (short)src[2], (short)src[3]);
                else
                    for (int e = 0; e < 4 && qxs + e < bw[b]; e++) dst[e] = (int16_t)src[e];
                continue;
            }
            int32_t *dst = bptr[b] + (uint64_t)qy * bpitch[b] + qxs;
            if (qxs + 3 < bw[b]) *(int4 *)dst = *(const int4 *)src;
            else
                for (int e = 0; e < 4 && qxs + e < bw[b]; e++) dst[e] = src[e];
        }
    }
    // per-block accumulation over the lanes of one column parity (the whole
    // quad tile lies in one 128 cell): lane 0 gets LL and LH, lane 1 HL and HH
#pragma unroll
    for (int s = 2; s <= 32; s <<= 1) {
        or_e |= __shfl_xor(or_e, s, 64);
        or_o |= __shfl_xor(or_o, s, 64);
        negs |= __shfl_xor(negs, s, 64);
    }
    if (lane < 2) {
        BlkAcc *acc = (BlkAcc *)(ws + H.ws_acc);
        const int bx = qx0 / kBlock, by = qy0 / kBlock;
        const int32_t hwc = hw - bx * kBlock, hhc = hh - by * kBlock;
        if (hwc > 0 || hhc > 0) {  // the cell holds at least one H coefficient
            const uint32_t local = G.group_start + (uint32_t)c * G.blocks_per_chan + (uint32_t)by * G.gx + bx;
            BlkAcc *a = acc + T.block_base + local;
            if (lane == 0) {
                if (or_o) atomicOr(&a->or_mag[0], or_o);
                if (negs & 2u) atomicOr(&a->neg, 1u);
            } else {
                if (or_e) atomicOr(&a->or_mag[1], or_e);
                if (or_o) atomicOr(&a->or_mag[2], or_o);
                const uint32_t nb = ((negs & 1u) ? 2u : 0u) | ((negs & 2u) ? 4u : 0u);
                if (nb) atomicOr(&a->neg, nb);
            }
        }
        if (last && lane == 0) {
            const uint32_t local = (uint32_t)c * T.ll_gx * T.ll_gy + (uint32_t)by * T.ll_gx + bx;
            BlkAcc *a = acc + T.block_base + local;
            if (or_e) atomicOr(&a->or_mag[0], or_e);
            if (negs & 1u) atomicOr(&a->neg, 1u);
        }
    }
}

// Inverse of level `level` for one channel over the window of the maps rmap /
// cmap, by strips, in three steps so that a caller can have the next
// channel's loads in flight while it finishes the current one:
//  1. inv_strips_load: the column pass's coefficients of window column
//     2 + lane, rows 1 + 16wv .. 19 + 16wv, straight from the bands into
//     registers, and one coefficient of the halo columns 1, 66, 67;
//  2. inv_strips_cols: the column lifting, its outputs (and the raw halo)
//     into the window;
//  3. after a barrier, inv_strips_rows: the row pass of window row 2 + lane,
//     columns 16wv + 2 .. 16wv + 17, lifting the halo columns where needed.
struct InvLoad {
    int32_t x[19];
    int32_t hv;
    int hdst;
};

// b16: the LH, HL and HH bands are held as int16 (level 1 of a tile whose
// level-1 values fit); LL is int32.
__device__ inline int32_t band_at(const int32_t *base, bool is16, uint64_t i)
{
    // one 32-bit load either way (lanes of one instruction may read bands
    // of both kinds): an int16 element comes with its 4-byte-aligned
    // neighbour, which lies inside the row's padded pitch
    const uint8_t *b = (const uint8_t *)base;
    const int32_t w = *(const int32_t *)(b + (is16 ? 2 * (i & ~1ull) : 4 * i));
    const uint32_t sh = is16 ? 16u - 16u * (uint32_t)(i & 1) : 0u;
    return is16 ? (int32_t)((uint32_t)w << sh) >> 16 : w;
}

// The 32-bit words of 19 consecutive window rows of one column: even rows
// from pE, odd rows from pO (row strides sE, sO bytes); P0 = parity of the
// first row.
template <int P0>
__device__ inline void load_rows19(const uint8_t *pE, const uint8_t *pO, uint64_t sE, uint64_t sO, int32_t (&x)[19])
{
#pragma unroll
    for (int j = 0; j < 19; j++) {
        if (((j + P0) & 1) == 0) {
            x[j] = *(const int32_t *)pE;
            pE += sE;
        } else {
            x[j] = *(const int32_t *)pO;
            pO += sO;
        }
    }
}

__device__ inline void inv_strips_load(const TileGeo &T, int level, int ch, const int32_t *rmap, const int32_t *cmap,
                                       const int32_t *wsi, int lane, int wv, bool b16, InvLoad &L)
{
    using namespace strips;
    const LevelGeo &G = T.lv[level];
    const int32_t *ll;
    uint32_t llp;
    if (level == T.levels) { ll = wsi + T.ll_off + (uint64_t)ch * T.chan_elems; llp = T.ll_pitch; }
    else {
        const int which = (level & 1) ? 0 : 1;
        ll = wsi + T.tmp_off[which] + (uint64_t)ch * T.tmp_chan[which];
        llp = T.tmp_pitch[which];
    }
    const int32_t *lh = wsi + G.off[0] + (uint64_t)ch * T.chan_elems;
    const int32_t *hl = wsi + G.off[1] + (uint64_t)ch * T.chan_elems;
    const int32_t *hh = wsi + G.off[2] + (uint64_t)ch * T.chan_elems;
    // halo columns, window rows 0..67
    const int t = (int)threadIdx.x;
    L.hv = 0;
    L.hdst = -1;
    if (t < 3 * WN) {
        const int k = t / WN, lr = t - k * WN;
        const int lc = k == 0 ? 1 : 65 + k;
        const int gy = rmap[lr], gx = cmap[lc];
        const int32_t *src = (gy & 1) ? ((gx & 1) ? hh : lh) : ((gx & 1) ? hl : ll);
        const uint32_t pitch = (gy & 1) ? G.pitch[(gx & 1) ? 2 : 0] : ((gx & 1) ? G.pitch[1] : llp);
        L.hv = band_at(src, b16 && ((gy | gx) & 1), (uint64_t)(gy >> 1) * pitch + (gx >> 1));
        L.hdst = lr * WP + lc;
    }
    // window column 2 + lane: even rows LL | HL, odd rows LH | HH
    const int gx = cmap[2 + lane];
    const bool xo = (gx & 1) != 0;
    const int32_t *pe = xo ? hl : ll;
    const int32_t *po = xo ? hh : lh;
    const uint32_t pitch_e = xo ? G.pitch[1] : llp, pitch_o = G.pitch[xo ? 2 : 0];
    const bool e16 = b16 && xo;
    const int a = 1 + 16 * wv;
    const int gy0 = __builtin_amdgcn_readfirstlane(rmap[a]);
    if (__all(lane >= 19 || rmap[a + lane] == gy0 + lane)) {
        // the strip's 19 rows are consecutive (no reflection): each lane
        // walks one pointer through the even rows and one through the odd
        // rows of its column instead of computing every address (pitches
        // are multiples of 4, so an int16 element keeps its half of the
        // 32-bit word in every row)
        const int p0 = gy0 & 1;
        const uint32_t xe = (uint32_t)(gx >> 1);
        const uint64_t ie = (uint64_t)((gy0 + p0) >> 1) * pitch_e + xe;
        const uint64_t io = (uint64_t)((gy0 + 1 - p0) >> 1) * pitch_o + xe;
        const uint8_t *pE = (const uint8_t *)pe + (e16 ? 2 * (ie & ~1ull) : 4 * ie);
        const uint8_t *pO = (const uint8_t *)po + (b16 ? 2 * (io & ~1ull) : 4 * io);
        const uint64_t sE = (uint64_t)pitch_e * (e16 ? 2u : 4u), sO = (uint64_t)pitch_o * (b16 ? 2u : 4u);
        if (p0) load_rows19<1>(pE, pO, sE, sO, L.x);
        else load_rows19<0>(pE, pO, sE, sO, L.x);
        if (b16) {
            // int16 elements: the low half of the word for even ones
            const uint32_t lE = e16 ? 16u - 16u * (xe & 1u) : 0u, rE = e16 ? 16u : 0u;
            const uint32_t lO = 16u - 16u * (xe & 1u);
#pragma unroll
            for (int j = 0; j < 19; j++) {
                if (((j + p0) & 1) == 0) L.x[j] = (int32_t)((uint32_t)L.x[j] << lE) >> rE;
                else L.x[j] = (int32_t)((uint32_t)L.x[j] << lO) >> 16;
            }
        }
        return;
    }
#pragma unroll
    for (int j = 0; j < 19; j++) {
        const int gy = __builtin_amdgcn_readfirstlane(rmap[1 + 16 * wv + j]);
        if (gy & 1) L.x[j] = band_at(po, b16, (uint64_t)(gy >> 1) * pitch_o + (gx >> 1));
        else L.x[j] = band_at(pe, e16, (uint64_t)(gy >> 1) * pitch_e + (gx >> 1));
    }
}

__device__ inline void inv_strips_cols(const InvLoad &L, int32_t *win, int lane, int wv, bool do_cols)
{
    using namespace strips;
    if (L.hdst >= 0) win[L.hdst] = L.hv;
    int32_t y[16];
    if (do_cols) lift_inv16(L.x, y);
    else {
#pragma unroll
        for (int j = 0; j < 16; j++) y[j] = L.x[j + 1];
    }
    int32_t *colw = win + (2 + 16 * wv) * WP + 2 + lane;
#pragma unroll
    for (int j = 0; j < 16; j++) colw[j * WP] = y[j];
}

__device__ inline void inv_strips_rows(const int32_t *win, int lane, int wv, bool do_cols, bool do_rows,
                                       int32_t (&o)[16])
{
    using namespace strips;
    int32_t x[19];
    const int32_t *rw = win + (2 + lane) * WP;
#pragma unroll
    for (int j = 0; j < 19; j++) x[j] = rw[1 + 16 * wv + j];
    if (do_cols) {  // the halo columns were left raw by the column pass
        const bool ro = (lane & 1) != 0;  // window row parity
        if (wv == 0) x[0] = col_lift_inv_at(rw + 1, ro);
        if (wv == 3) {
            x[17] = col_lift_inv_at(rw + 66, ro);
            x[18] = col_lift_inv_at(rw + 67, ro);
        }
    }
    if (do_rows) lift_inv16(x, o);
    else {
#pragma unroll
        for (int j = 0; j < 16; j++) o[j] = x[j + 1];
    }
}

// Inverse of level `level` into LL_{level-1} (an intermediate level), by
// strips; the outputs go back through the window so that a wave stores whole
// rows.
__global__ void __launch_bounds__(256) k_inv_level_strips(PlanHdr H, const uint8_t *__restrict__ plan,
                                                          uint8_t *__restrict__ ws, int level)
{
    using namespace strips;
    __shared__ __align__(16) int32_t win[WN * WP];
    __shared__ int32_t rmap[WN], cmap[WN];
    const TileGeo *tiles = (const TileGeo *)(plan + H.tiles_off);
    const WorkItem *items = (const WorkItem *)(plan + H.work_off);
    const uint32_t bid = xcd_remap(blockIdx.x, gridDim.x);
    const WorkItem &W = find_item(items, H.lvl_first[level], H.lvl_count[level], bid);
    const TileGeo &T = tiles[W.tile];
    const uint32_t r = bid - W.wg_start;
    const int c = (int)(r % W.nch);
    const uint32_t sp = r / W.nch;
    const int qx0 = (int)(W.qx0 + (sp % W.ntx) * TQ), qy0 = (int)(W.qy0 + (sp / W.ntx) * TQ);
    int32_t *wsi = (int32_t *)ws;
    const LevelGeo &G = T.lv[level];
    const int lane = (int)(threadIdx.x & 63);
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    fill_maps<TQ>(rmap, cmap, qx0, qy0, (int)G.w, (int)G.h, G);
    __syncthreads();
    int32_t o[16];
    {
        InvLoad L;
        inv_strips_load(T, level, c, rmap, cmap, wsi, lane, wv, level <= 2 && ((T.coef16 >> (level - 1)) & 1u), L);
        inv_strips_cols(L, win, lane, wv, G.h > 1);
    }
    __syncthreads();
    inv_strips_rows(win, lane, wv, G.h > 1, G.w > 1, o);
    // the 64x64 outputs go through LDS (rows of 68 words, 16-byte aligned)
    constexpr int OP = 68;
    __syncthreads();
    {
        int32_t *rowp = win + lane * OP + 16 * wv;
#pragma unroll
        for (int j = 0; j < 16; j++) rowp[j] = o[j];
    }
    __syncthreads();
    // LL_{level-1} is the low band of level-1: store the part inside that
    // level's window; 16-byte pieces (a wave stores four whole rows) when the
    // tile's columns are 4-aligned in it, else a lane per column
    const int k = level - 1, which = (k & 1) ? 0 : 1;
    const LevelGeo &D = T.lv[k];
    int32_t *dst = wsi + T.tmp_off[which] + (uint64_t)c * T.tmp_chan[which];
    const uint32_t dp = T.tmp_pitch[which];
    const int xb = 2 * qx0 - (int)D.wx0, yb = 2 * qy0 - (int)D.wy0;
    if (((xb | (int)dp) & 3) == 0) {
#pragma unroll
        for (int m = 0; m < 4; m++) {
            const int ch = (int)threadIdx.x + 256 * m, row = ch >> 4, part = ch & 15;
            const int y = yb + row, x = xb + 4 * part;
            if ((uint32_t)y >= D.wh) continue;
            const int32_t *src = win + row * OP + 4 * part;
            int32_t *d = dst + (uint64_t)y * dp;
            if (x >= 0 && x + 3 < (int)D.ww) *(int4 *)(d + x) = *(const int4 *)src;
            else
                for (int e = 0; e < 4; e++)
                    if ((uint32_t)(x + e) < D.ww) d[x + e] = src[e];
        }
    } else {
        const int x = xb + lane;
#pragma unroll
        for (int m = 0; m < 16; m++) {
            const int ly = wv + 4 * m;
            const int y = yb + ly;
            if ((uint32_t)x < D.ww && (uint32_t)y < D.wh) dst[(uint64_t)y * dp + x] = win[ly * OP + lane];
        }
    }
}

// Final stage of a decode job by strips: LL_z (z = target level), fusing the
// inverse of level z+1 if z < levels, then the inverse colour transform,
// clamping and the interleaved pixel stores.  The channels of a group (3
// with the colour transform) go through the window in turn; a thread keeps
// its 16 pixels of one output row per channel in registers.  Formats of at
// most 4 bytes per pixel in one channel group are staged in LDS as output
// bytes and stored by whole rows.
__global__ void __launch_bounds__(256) k_inv_final_strips(PlanHdr H, const uint8_t *__restrict__ plan,
                                                          uint8_t *__restrict__ ws, uint8_t *__restrict__ pix)
{
    using namespace strips;
    __shared__ __align__(16) int32_t win[WN * WP];
    __shared__ int32_t rmap[WN], cmap[WN];
    const TileGeo *tiles = (const TileGeo *)(plan + H.tiles_off);
    const WorkItem *items = (const WorkItem *)(plan + H.work_off);
    const uint32_t bid = xcd_remap(blockIdx.x, gridDim.x);
    const WorkItem &W = find_item(items, H.fin_first, H.fin_count, bid);
    const TileGeo &T = tiles[W.tile];
    const uint32_t r = bid - W.wg_start;
    const int cg = (int)(r % W.nch);
    const uint32_t sp = r / W.nch;
    const int qx0 = (int)(W.qx0 + (sp % W.ntx) * TQ), qy0 = (int)(W.qy0 + (sp / W.ntx) * TQ);
    int32_t *wsi = (int32_t *)ws;
    const int lane = (int)(threadIdx.x & 63);
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int z = T.target_level;
    const int c0 = cg * 3;
    const int nc = min((int)T.channels - c0, 3);
    const bool fused = z < T.levels;
    int ow = 0, oh = 0;
    if (fused) {
        ow = (int)T.lv[z + 1].w; oh = (int)T.lv[z + 1].h;
        fill_maps<TQ>(rmap, cmap, qx0, qy0, ow, oh, T.lv[z + 1]);
        __syncthreads();
    }
    // output region of the level-z image (all of it for a full decode)
    const int rx0 = (int)T.rx0, ry0 = (int)T.ry0, rx1 = (int)T.rx1, ry1 = (int)T.ry1;
    const int y = 2 * qy0 + lane;      // this thread's output row
    const int xs = 2 * qx0 + 16 * wv;  // its first output column
    int32_t v[3][16];
    InvLoad L;  // the coefficients of the channel the window takes next
    const bool b16 = z < 2 && ((T.coef16 >> z) & 1u);  // level z + 1's H bands as int16
    if (fused) inv_strips_load(T, z + 1, c0, rmap, cmap, wsi, lane, wv, b16, L);
#pragma unroll
    for (int k = 0; k < 3; k++) {
        if (k >= nc) {
#pragma unroll
            for (int j = 0; j < 16; j++) v[k][j] = 0;
            continue;
        }
        if (fused) {
            if (k) __syncthreads();  // the previous row pass has read the window
            inv_strips_cols(L, win, lane, wv, oh > 1);
            // the next channel's loads are in flight during this row pass
            if (k + 1 < nc) inv_strips_load(T, z + 1, c0 + k + 1, rmap, cmap, wsi, lane, wv, b16, L);
            __syncthreads();
            inv_strips_rows(win, lane, wv, oh > 1, ow > 1, v[k]);
        } else {
            const int32_t *ll = wsi + T.ll_off + (uint64_t)(c0 + k) * T.chan_elems;
            const bool yin = y >= ry0 && y < ry1;
#pragma unroll
            for (int j = 0; j < 16; j++) {
                const int x = xs + j;
                v[k][j] = (yin && x >= rx0 && x < rx1)
                              ? ll[(uint64_t)(y - (int)T.ll_wy0) * T.ll_pitch + (x - (int)T.ll_wx0)] : 0;
            }
        }
    }
    const int32_t top = (1 << T.bits) - 1;
#pragma unroll
    for (int j = 0; j < 16; j++) {
        if (T.ct) colour_inv(T.ct, v[0][j], v[1][j], v[2][j]);
#pragma unroll
        for (int k = 0; k < 3; k++) v[k][j] = v[k][j] < 0 ? 0 : (v[k][j] > top ? top : v[k][j]);
    }
    const uint32_t C = T.channels, bps = T.bps, sb = C * bps;
    const uint64_t rowbase0 = T.pix_offset + (uint64_t)(2 * qx0 - rx0) * sb;
    // rows that do not start 4-byte aligned (odd widths of 1- and 3-byte
    // pixels) are stored as aligned words assembled from the staged bytes
    const bool al4 = ((rowbase0 | T.pix_stride | (uint64_t)(uintptr_t)pix) & 3u) == 0;
    const bool staged = nc == (int)C && (al4 ? sb <= 4 : sb <= 3) && 2 * qx0 >= rx0;
    if (staged) {
        __syncthreads();  // every row pass has read the window
        uint8_t *ob = (uint8_t *)win;  // 64 rows x 64 * sb bytes
        const int RB = 64 * (int)sb;
        uint8_t *mine = ob + lane * RB + 16 * wv * (int)sb;
        if (sb == 3) {
            uint32_t dw[12];
#pragma unroll
            for (int i = 0; i < 12; i++) dw[i] = 0;
#pragma unroll
            for (int j = 0; j < 16; j++)
#pragma unroll
                for (int k = 0; k < 3; k++) {
                    const int b = 3 * j + k;
                    dw[b >> 2] |= (uint32_t)v[k][j] << (8 * (b & 3));
                }
            uint4 *q = (uint4 *)mine;
            q[0] = make_uint4(dw[0], dw[1], dw[2], dw[3]);
            q[1] = make_uint4(dw[4], dw[5], dw[6], dw[7]);
            q[2] = make_uint4(dw[8], dw[9], dw[10], dw[11]);
        } else {
#pragma unroll
            for (int j = 0; j < 16; j++)
#pragma unroll
                for (int k = 0; k < 3; k++) {  // constant indices keep v in registers
                    if (k >= nc) break;
                    uint8_t *q = mine + (j * (int)C + k) * (int)bps;
                    if (bps == 1) *q = (uint8_t)v[k][j];
                    else if (bps == 2) *(uint16_t *)q = (uint16_t)v[k][j];
                    else *(uint32_t *)q = (uint32_t)v[k][j];
                }
        }
        __syncthreads();
        const int nbytes = min(64, rx1 - 2 * qx0) * (int)sb;
        if (!al4) {
            // a row's bytes [0, nbytes) start at an address m bytes past a
            // word boundary; aligned word i of the destination holds bytes
            // 4i - m .. 4i - m + 3, the top m bytes of staged word i - 1 and
            // the low 4 - m of word i.  16 lanes per row, four words each
            // (RB <= 192 bytes: at most 49 words).
            const int k = lane & 15;
            const int nst = RB / 4;
#pragma unroll
            for (int mm = 0; mm < 4; mm++) {
                const int ly = 4 * (wv + 4 * mm) + (lane >> 4);
                const int yy = 2 * qy0 + ly;
                if (yy < ry0 || yy >= ry1) continue;
                uint8_t *rdst = pix + rowbase0 + (uint64_t)(yy - ry0) * T.pix_stride;
                const uint32_t m = (uint32_t)(uintptr_t)rdst & 3u;
                uint32_t *wdst = (uint32_t *)(rdst - m);
                const uint32_t *ls = (const uint32_t *)(ob + ly * RB);
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    const int i = 4 * k + e;
                    const int b0 = 4 * i - (int)m;  // row byte of the word's first byte
                    if (b0 >= nbytes) break;
                    const uint32_t lo = i > 0 ? ls[i - 1] : 0u, hi = i < nst ? ls[i] : 0u;
                    const uint32_t v = m ? __builtin_amdgcn_alignbyte(hi, lo, 4u - m) : hi;
                    if (b0 >= 0 && b0 + 4 <= nbytes) wdst[i] = v;
                    else
                        for (int q = 0; q < 4; q++)
                            if (b0 + q >= 0 && b0 + q < nbytes) rdst[b0 + q] = (uint8_t)(v >> (8 * q));
                }
            }
            return;
        }
        // 16-byte pieces: 16 lanes per row, four rows per wave and pass
        const int nq = RB / 16;
        const bool a16 = ((rowbase0 | T.pix_stride | (uint64_t)(uintptr_t)pix) & 15u) == 0;
        const int k = lane & 15;
#pragma unroll
        for (int m = 0; m < 4; m++) {
            const int ly = 4 * (wv + 4 * m) + (lane >> 4);
            const int yy = 2 * qy0 + ly;
            const int nb = min(16, nbytes - 16 * k);
            if (k >= nq || nb <= 0 || yy < ry0 || yy >= ry1) continue;
            uint8_t *dst = pix + rowbase0 + (uint64_t)(yy - ry0) * T.pix_stride + 16 * k;
            const uint8_t *src = ob + ly * RB + 16 * k;
            if (nb == 16 && a16) *(uint4 *)dst = *(const uint4 *)src;
            else {
                const int nw = nb >> 2;
                for (int i = 0; i < nw; i++) ((uint32_t *)dst)[i] = ((const uint32_t *)src)[i];
                for (int b = 4 * nw; b < nb; b++) dst[b] = src[b];
            }
        }
        return;
    }
    if (y < ry0 || y >= ry1) return;
    uint8_t *row = pix + T.pix_offset + (uint64_t)(y - ry0) * T.pix_stride;  // region row
#pragma unroll
    for (int j = 0; j < 16; j++) {
        const int x = xs + j;
        if (x < rx0 || x >= rx1) continue;
#pragma unroll
        for (int k = 0; k < 3; k++) {
            if (k >= nc) break;
            const uint32_t e = ((uint32_t)(x - rx0) * C + c0 + k) * bps;
            if (bps == 1) row[e] = (uint8_t)v[k][j];
            else if (bps == 2) *(uint16_t *)(row + e) = (uint16_t)v[k][j];
            else *(uint32_t *)(row + e) = (uint32_t)v[k][j];
        }
    }
}

// ------------------------------------------------------------------ launch
hipError_t launch_forward_level(const PlanHdr &H, const uint8_t *d_plan, const uint8_t *d_pixels,
                                uint8_t *d_ws, int level, hipStream_t stream)
{
    if (level > (int)H.max_levels || !H.lvl_wgs[level]) return hipSuccess;
    if (level == 0)
        hipLaunchKernelGGL(k_fwd_level0, dim3(H.lvl_wgs[0]), dim3(256), 0, stream, H, d_plan, d_pixels, d_ws);
    else if (H.tq == 16)
        hipLaunchKernelGGL(k_fwd_level<16>, dim3(H.lvl_wgs[level]), dim3(256), 0, stream, H, d_plan, d_pixels, d_ws, level);
    else
        hipLaunchKernelGGL(k_fwd_strips, dim3(H.lvl_wgs[level]), dim3(256), 0, stream, H, d_plan, d_pixels, d_ws, level);
    return hipGetLastError();
}

hipError_t launch_inverse_level(const PlanHdr &H, const uint8_t *d_plan, uint8_t *d_ws,
                                uint8_t *d_pixels_out, const int32_t *d_status, int level,
                                hipStream_t stream)
{
    if (level == 0) {
        if (!H.fin_wgs) return hipSuccess;
        if (H.tq == 16)
            hipLaunchKernelGGL(k_inv_final<16>, dim3(H.fin_wgs), dim3(256), 0, stream, H, d_plan, d_ws, d_pixels_out, d_status);
        else
            hipLaunchKernelGGL(k_inv_final_strips, dim3(H.fin_wgs), dim3(256), 0, stream, H, d_plan, d_ws, d_pixels_out);
    } else if (level <= (int)H.max_levels && H.lvl_wgs[level]) {
        if (H.tq == 16)
            hipLaunchKernelGGL(k_inv_level<16>, dim3(H.lvl_wgs[level]), dim3(256), 0, stream, H, d_plan, d_ws, level);
        else
            hipLaunchKernelGGL(k_inv_level_strips, dim3(H.lvl_wgs[level]), dim3(256), 0, stream, H, d_plan, d_ws, level);
    }
    return hipGetLastError();
}

}  // namespace isx
