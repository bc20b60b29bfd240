// k_decode.hip -- decoder of the codec for gfx950: the encode pipeline in
// reverse (Sec. 4: "traversing the pipeline in reverse"; lower resolutions by
// decoding only the coarser blocks).
//
//  k_dec_prep      per job: tile header and block-size table checks, block
//                  descriptors and byte offsets (scan) of the blocks needed
//                  for the target level.
//  k_dec_header    per block: d, masks, C_zr, wz, recursive code tree (Fig. 3:
//                  0 = internal node, 1 + 8 bits = leaf), seek table; builds a
//                  4096-entry prefix table plus the sorted left-aligned codes
//                  (any valid tree is accepted, not only canonical ones).
//  k_dec_segments  per segment: tokens -> symbols (runs of zeros from the
//                  bijective-base counters, a literal C_zr from a zero counter).
//  k_dec_reasm     per block: symbols -> signed-magnitude bits -> integers ->
//                  dequantised coefficients in the band arrays.
// Every read of the stream is bounded by the job's input region; an error
// marks the job's status and never makes a kernel leave its buffers.
#include "isx_common.h"

namespace isx {

#define D_OK 0
#define D_CORRUPT (-3)
#define D_TRUNC (-4)

constexpr uint16_t kLutLong = 0x4000;

__device__ inline uint32_t rd_byte(const uint8_t *base, uint64_t len, uint64_t i)
{
    return i < len ? base[i] : 0u;
}

template <int NT>
__device__ inline uint64_t dblock_excl_sum(uint64_t v, uint64_t *sh, uint64_t *total)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint64_t x = v;
    for (int o = 1; o < 64; o <<= 1) {
        uint64_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) sh[wave] = x;
    __syncthreads();
    uint64_t base = 0, tot = 0;
    for (int w = 0; w < NT / 64; w++) {
        if (w < wave) base += sh[w];
        tot += sh[w];
    }
    __syncthreads();
    if (total) *total = tot;
    return base + x - v;
}

__global__ void __launch_bounds__(256) k_dec_prep(PlanHdr H, const uint8_t *__restrict__ plan,
                                                  const uint8_t *__restrict__ enc,
                                                  uint8_t *__restrict__ ws,
                                                  int32_t *__restrict__ status)
{
    __shared__ uint64_t sh[8];
    __shared__ int32_t s_st;
    const uint32_t job = blockIdx.x;
    const TileGeo &T = ((const TileGeo *)(plan + H.tiles_off))[job];
    BlockDesc *descs = (BlockDesc *)(ws + H.ws_blockdesc);
    const uint8_t *base = enc + T.enc_offset;
    const uint64_t avail = T.enc_bytes;
    if (threadIdx.x == 0) {
        int32_t st = D_OK;
        if (avail < 24) st = D_TRUNC;
        else {
            uint8_t h[24];
            for (int i = 0; i < 24; i++) h[i] = base[i];
            uint32_t q = h[10] | (h[11] << 8);
            uint32_t w = h[12] | (h[13] << 8) | (h[14] << 16) | ((uint32_t)h[15] << 24);
            uint32_t hh = h[16] | (h[17] << 8) | (h[18] << 16) | ((uint32_t)h[19] << 24);
            uint32_t nb = h[20] | (h[21] << 8) | (h[22] << 16) | ((uint32_t)h[23] << 24);
            if (h[0] != 'I' || h[1] != 'S' || h[2] != 'X' || h[3] != '1' || h[4] != 1 || h[5] != T.ct ||
                h[6] != T.channels || h[7] != T.bits || h[8] != T.bps || h[9] != T.levels || q != T.qstep ||
                w != T.width || hh != T.height || nb != T.nblocks_stream)
                st = D_CORRUPT;
            else if (avail < 24 + 4ull * nb) st = D_TRUNC;
        }
        s_st = st;
    }
    __syncthreads();
    int32_t st = s_st;
    uint64_t carry = 24 + 4ull * T.nblocks_stream, scarry = 0;
    uint32_t bad = 0;
    for (uint32_t b0 = 0; b0 < T.nblocks; b0 += 256) {
        uint32_t local = b0 + threadIdx.x;
        BlockDesc B;
        uint64_t sz = 0, ssz = 0;
        if (local < T.nblocks) {
            block_geometry(T, local, B);
            ssz = ((uint64_t)B.p * B.wb * B.hb / 8 * T.dmax + 15) & ~15ull;
            if (st == D_OK) {
                uint64_t o = 24 + 4ull * local;
                sz = (uint64_t)base[o] | ((uint64_t)base[o + 1] << 8) | ((uint64_t)base[o + 2] << 16) |
                     ((uint64_t)base[o + 3] << 24);
            }
        }
        uint64_t tot, stot;
        uint64_t ex = dblock_excl_sum<256>(sz, sh, &tot);
        uint64_t sex = dblock_excl_sum<256>(ssz, sh, &stot);
        if (local < T.nblocks) {
            uint64_t off = carry + ex;
            B.tile = job;
            B.sym_off = T.sym_base + scarry + sex;
            B.slot = T.slot_base + local * T.dmax;
            B.dmax = T.dmax;
            if (st == D_OK && off + sz <= avail && sz > 0) {
                B.byte_off = T.enc_offset + off;
                B.byte_len = (uint32_t)sz;
            } else {
                B.byte_off = 0;
                B.byte_len = 0;
                if (st == D_OK) bad = 1;
            }
            descs[T.block_base + local] = B;
        }
        carry += tot;
        scarry += stot;
    }
    bad = __syncthreads_or(bad);
    if (threadIdx.x == 0) status[job] = (st == D_OK && bad) ? D_TRUNC : st;
}

// ------------------------------------------------------------------ header
__global__ void __launch_bounds__(64) k_dec_header(PlanHdr H, const uint8_t *__restrict__ enc,
                                                   uint8_t *__restrict__ ws,
                                                   int32_t *__restrict__ status)
{
    __shared__ uint8_t hb[512];
    __shared__ uint32_t s_info[8];
    __shared__ uint32_t s_acode[256];
    __shared__ uint8_t s_len[256], s_sym[256];
    const uint32_t blk = blockIdx.x, lane = threadIdx.x;
    const BlockDesc &B = ((const BlockDesc *)(ws + H.ws_blockdesc))[blk];
    BlkPlan &P = ((BlkPlan *)(ws + H.ws_blkplan))[blk];
    uint16_t *lut = (uint16_t *)(ws + H.ws_lut + (uint64_t)blk * kLutBytes);
    DecLeaves *LV = (DecLeaves *)((uint8_t *)lut + (1u << kLutK) * 2);
    if (status[B.tile] != D_OK || B.byte_len == 0) {
        if (lane == 0) { P.nseg = 0; P.err = 1; P.d = 1; }
        return;
    }
    const uint8_t *src = enc + B.byte_off;
    const uint32_t blen = B.byte_len;
    for (uint32_t i = lane; i < 512; i += 64) hb[i] = (uint8_t)rd_byte(src, blen, i);
    __syncthreads();
    const uint32_t p = B.p, n = (uint32_t)B.wb * B.hb / 8;
    if (lane == 0) {
        uint64_t pos = 0;
        const uint64_t lim = (uint64_t)blen * 8;
        int32_t err = 0;
        auto get = [&](uint32_t nb) -> uint32_t {
            uint32_t v = 0;
            for (uint32_t i = 0; i < nb; i++) {
                uint32_t bit = 0;
                if (pos < lim && pos < 4096) bit = (hb[pos >> 3] >> (7 - (pos & 7))) & 1u;
                else err = D_TRUNC;
                v = (v << 1) | bit;
                pos++;
            }
            return v;
        };
        uint32_t d = get(5);
        uint32_t masks[3] = {0, 0, 0};
        for (uint32_t t = 0; t < p; t++) masks[t] = get(d);
        if (!err && (d < 1 || d > B.dmax)) err = D_CORRUPT;
        uint32_t nseg = 0;
        if (!err) {
            for (int b = (int)d - 1; b >= 0; b--) {
                uint32_t pm = 0;
                for (uint32_t t = 0; t < p; t++) pm |= (((masks[t] >> b) & 1u) ^ 1u) << t;
                if (pm) {
                    P.seg_plane[nseg] = (uint8_t)b;
                    P.seg_M[nseg] = n * __popc(pm);
                    nseg++;
                }
            }
        }
        uint32_t czr = 0, wz = 0, m = 0, single = 0;
        if (!err && nseg) {
            czr = get(8);
            wz = get(4);
            uint32_t beta = bitlen32(p * n - 1), wzhi = beta > 2 ? beta : 2;
            if (wz < 2 || wz > wzhi) err = D_CORRUPT;
            // recursive tree, pre-order; explicit stack of pending right children
            uint32_t stk_code[33], stk_len[33];
            int sp = 0;
            uint32_t code = 0, len = 0, nodes = 0;
            uint32_t seen[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            while (!err) {
                if (++nodes > 511) { err = D_CORRUPT; break; }
                uint32_t bit = get(1);
                if (err) break;
                if (!bit) {
                    if (len >= 32) { err = D_CORRUPT; break; }
                    stk_code[sp] = (code << 1) | 1u;
                    stk_len[sp] = len + 1;
                    sp++;
                    code <<= 1;
                    len++;
                } else {
                    uint32_t s = get(8);
                    if (err) break;
                    if ((seen[s >> 5] >> (s & 31)) & 1u) { err = D_CORRUPT; break; }
                    seen[s >> 5] |= 1u << (s & 31);
                    s_acode[m] = len ? (code << (32 - len)) : 0u;
                    s_len[m] = (uint8_t)len;
                    s_sym[m] = (uint8_t)s;
                    m++;
                    if (sp == 0) break;
                    sp--;
                    code = stk_code[sp];
                    len = stk_len[sp];
                }
            }
            single = (m == 1);
            const uint32_t tb = bitlen32(p * n) - 1 + 5;
            uint64_t acc = 0;
            for (uint32_t s = 0; s < nseg && !err; s++) {
                P.seg_bits[s] = get(tb);
                acc += P.seg_bits[s];
            }
            if (!err) {
                uint64_t start = (uint64_t)B.byte_off * 8 + pos;
                if (pos + acc > lim) err = D_TRUNC;
                for (uint32_t s = 0; s < nseg; s++) {
                    P.seg_bitpos[s] = start;
                    start += P.seg_bits[s];
                }
            }
        }
        P.d = d; P.nseg = err ? 0 : nseg; P.czr = czr; P.wz = wz; P.m = m; P.p = p; P.n = n;
        for (uint32_t t = 0; t < 3; t++) P.masks[t] = masks[t];
        P.err = err ? 1 : 0;
        s_info[0] = err ? 0 : nseg;
        s_info[1] = m;
        s_info[2] = single;
        if (err) atomicMin(&status[B.tile], err);
    }
    __syncthreads();
    const uint32_t nseg = s_info[0], m = s_info[1];
    if (!nseg) return;
    // prefix table: entry = sym | len << 8, or kLutLong for codes longer than K
    for (uint32_t j = lane; j < m; j += 64) {
        LV->acode[j] = s_acode[j];
        LV->len[j] = s_len[j];
        LV->sym[j] = s_sym[j];
        uint32_t L = s_len[j];
        uint32_t a = s_acode[j] >> (32 - kLutK);
        if (L <= (uint32_t)kLutK) {
            uint32_t cnt = 1u << (kLutK - L);
            uint16_t e = (uint16_t)(s_sym[j] | (L << 8));
            for (uint32_t k = 0; k < cnt; k++) lut[a + k] = e;
        } else {
            lut[a] = kLutLong;
        }
    }
    if (lane == 0) { LV->m = m; LV->single = s_info[2]; }
}

// ------------------------------------------------------------------ segments
// Bounded MSB-first bit reader over one block.
struct BitRd {
    const uint8_t *base;  // stream start (d_encoded)
    uint64_t lo, hi;      // allowed byte range [lo, hi)
    uint64_t bytepos;     // next byte to load
    uint64_t buf;         // MSB aligned
    uint32_t nb;          // valid bits in buf
    __device__ inline void init(const uint8_t *b, uint64_t lo_, uint64_t hi_, uint64_t bitpos)
    {
        base = b; lo = lo_; hi = hi_;
        bytepos = bitpos >> 3;
        buf = 0; nb = 0;
        refill();
        uint32_t skip = (uint32_t)(bitpos & 7);
        buf <<= skip;
        nb -= skip;
    }
    __device__ inline void refill()
    {
        while (nb <= 56) {
            uint64_t v = (bytepos >= lo && bytepos < hi) ? base[bytepos] : 0;
            buf |= v << (56 - nb);
            nb += 8;
            bytepos++;
        }
    }
    __device__ inline uint32_t peek32() { return (uint32_t)(buf >> 32); }
    __device__ inline void skip(uint32_t k) { buf <<= k; nb -= k; if (nb <= 56) refill(); }
};

__global__ void __launch_bounds__(64) k_dec_segments(PlanHdr H, const uint8_t *__restrict__ enc,
                                                     uint8_t *__restrict__ ws,
                                                     int32_t *__restrict__ status)
{
    __shared__ uint16_t lut[1 << kLutK];
    __shared__ uint32_t acode[256];
    __shared__ uint8_t llen[256], lsym[256];
    const uint32_t blk = blockIdx.x, lane = threadIdx.x;
    const BlockDesc &B = ((const BlockDesc *)(ws + H.ws_blockdesc))[blk];
    const BlkPlan &P = ((const BlkPlan *)(ws + H.ws_blkplan))[blk];
    const uint32_t nseg = P.nseg;
    if (!nseg || status[B.tile] != D_OK) return;
    const uint16_t *glut = (const uint16_t *)(ws + H.ws_lut + (uint64_t)blk * kLutBytes);
    const DecLeaves *LV = (const DecLeaves *)((const uint8_t *)glut + (1u << kLutK) * 2);
    for (uint32_t i = lane; i < (1u << kLutK); i += 64) lut[i] = glut[i];
    const uint32_t m = LV->m;
    for (uint32_t j = lane; j < m; j += 64) { acode[j] = LV->acode[j]; llen[j] = LV->len[j]; lsym[j] = LV->sym[j]; }
    // zero the symbol planes of the present segments
    const uint32_t pn = P.p * P.n;
    for (uint32_t s = 0; s < nseg; s++) {
        uint32_t *dst = (uint32_t *)(ws + B.sym_off + (uint64_t)P.seg_plane[s] * pn);
        uint32_t nw = (P.seg_M[s] + 3) / 4;
        if ((((uintptr_t)dst) & 3u) == 0) {
            for (uint32_t i = lane; i < nw; i += 64) dst[i] = 0;
        } else {
            uint8_t *db = (uint8_t *)dst;
            for (uint32_t i = lane; i < P.seg_M[s]; i += 64) db[i] = 0;
        }
    }
    __syncthreads();
    if (lane >= nseg) return;
    const uint32_t s = lane;
    const uint32_t M = P.seg_M[s];
    uint8_t *out = ws + B.sym_off + (uint64_t)P.seg_plane[s] * pn;
    const uint64_t start = P.seg_bitpos[s], end = start + P.seg_bits[s];
    BitRd r;
    r.init(enc, B.byte_off, B.byte_off + B.byte_len, start);
    uint64_t pos = start;
    const uint32_t czr = P.czr, wz = P.wz, Bb = (1u << wz) - 1u;
    const bool single = (m == 1);
    uint32_t k = 0, run = 0;
    bool in_run = false;
    int32_t err = 0;
    while (k + run < M) {
        uint32_t v, L;
        if (single) { v = lsym[0]; L = 0; }
        else {
            uint32_t pk = r.peek32();
            uint16_t e = lut[pk >> (32 - kLutK)];
            if (!(e & kLutLong)) { v = e & 0xffu; L = (e >> 8) & 0x3fu; }
            else {
                uint32_t lo = 0, hi = m;  // last leaf with acode <= pk
                while (hi - lo > 1) { uint32_t mid = (lo + hi) >> 1; if (acode[mid] <= pk) lo = mid; else hi = mid; }
                v = lsym[lo]; L = llen[lo];
            }
        }
        if (pos + L > end) { err = D_CORRUPT; break; }
        r.skip(L); pos += L;
        if (v == czr) {
            if (pos + wz > end) { err = D_CORRUPT; break; }
            uint32_t c = r.peek32() >> (32 - wz);
            r.skip(wz); pos += wz;
            if (c) {
                run = run * Bb + c;
                in_run = true;
                if (k + run > M) { err = D_CORRUPT; break; }
                continue;
            }
        }
        if (in_run) {
            if (run < 2) { err = D_CORRUPT; break; }
            k += run; run = 0; in_run = false;
        }
        if (k >= M) { err = D_CORRUPT; break; }
        if (v) out[k] = (uint8_t)v;
        k++;
    }
    if (!err && in_run) {
        if (run < 2) err = D_CORRUPT;
        else k += run;
    }
    if (!err && (k != M || pos != end)) err = D_CORRUPT;
    if (err) atomicMin(&status[B.tile], err);
}

// ------------------------------------------------------------------ reassembly
__global__ void __launch_bounds__(1024) k_dec_reasm(PlanHdr H, const uint8_t *__restrict__ plan,
                                                    uint8_t *__restrict__ ws,
                                                    const int32_t *__restrict__ status)
{
    const uint32_t blk = blockIdx.x, tid = threadIdx.x;
    const BlockDesc &B = ((const BlockDesc *)(ws + H.ws_blockdesc))[blk];
    const BlkPlan &P = ((const BlkPlan *)(ws + H.ws_blkplan))[blk];
    if (status[B.tile] != D_OK) return;
    const TileGeo &T = ((const TileGeo *)(plan + H.tiles_off))[B.tile];
    const uint32_t p = B.p, wb = B.wb, hb = B.hb, n = wb * hb / 8, cpt = n / 2, wq = wb / 4;
    const uint32_t d = P.d, nseg = P.nseg;
    const uint32_t step = (B.level == 0) ? 1u : T.qstep;
    int32_t *wsi = (int32_t *)ws;
    for (uint32_t cell = tid; cell < p * cpt; cell += blockDim.x) {
        uint32_t t = cell / cpt, ci = cell % cpt;
        uint32_t mag[16];
#pragma unroll
        for (int i = 0; i < 16; i++) mag[i] = 0;
        uint32_t sgn = 0;
        for (uint32_t s = 0; s < nseg; s++) {
            uint32_t b = P.seg_plane[s];
            uint32_t pm = 0;
            for (uint32_t u = 0; u < p; u++) pm |= (((P.masks[u] >> b) & 1u) ^ 1u) << u;
            if (!((pm >> t) & 1u)) continue;
            uint32_t rank = __popc(pm & ((1u << t) - 1u));
            uint32_t v = *(const uint16_t *)(ws + B.sym_off + (uint64_t)b * p * n + rank * n + 2 * ci);
            if (b == d - 1) sgn = v;
            else {
#pragma unroll
                for (int i = 0; i < 16; i++) mag[i] |= ((v >> i) & 1u) << b;
            }
        }
        uint32_t band = ci / wq, cg = ci % wq;
        uint32_t r0 = 4 * band, c0 = 4 * cg;
        const uint32_t tw = B.tw[t], th = B.th[t];
        for (int rr = 0; rr < 4; rr++) {
            uint32_t row = r0 + rr;
            if (row >= th) break;
            int32_t *dst = wsi + B.off[t] + (uint64_t)row * B.pitch[t] + c0;
            for (int cc = 0; cc < 4; cc++) {
                if (c0 + cc >= tw) break;
                int i = rr * 4 + cc;
                int32_t q = (int32_t)mag[i];
                if (step > 1 && q) q = q * (int32_t)step + (int32_t)(step / 2);
                dst[cc] = ((sgn >> i) & 1u) ? -q : q;
            }
        }
    }
}

// ------------------------------------------------------------------ launch
hipError_t launch_inverse_levels(const PlanHdr &H, const uint8_t *d_plan, uint8_t *d_ws,
                                 uint8_t *d_pixels_out, const int32_t *d_status, hipStream_t stream);

hipError_t launch_decode(const PlanHdr &H, const uint8_t *d_plan, const uint8_t *d_encoded,
                         uint8_t *d_pixels_out, int32_t *d_status, uint8_t *d_ws,
                         hipStream_t stream)
{
    hipLaunchKernelGGL(k_dec_prep, dim3(H.n_tiles), dim3(256), 0, stream, H, d_plan, d_encoded, d_ws, d_status);
    if (H.total_blocks) {
        hipLaunchKernelGGL(k_dec_header, dim3(H.total_blocks), dim3(64), 0, stream, H, d_encoded, d_ws, d_status);
        hipLaunchKernelGGL(k_dec_segments, dim3(H.total_blocks), dim3(64), 0, stream, H, d_encoded, d_ws, d_status);
        hipLaunchKernelGGL(k_dec_reasm, dim3(H.total_blocks), dim3(1024), 0, stream, H, d_plan, d_ws, d_status);
    }
    return launch_inverse_levels(H, d_plan, d_ws, d_pixels_out, d_status, stream);
}

}  // namespace isx
