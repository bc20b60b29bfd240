// k_decode.hip -- decoder of the codec for gfx950: the encode pipeline run
// backwards (Sec. 4, decompression; lower resolutions by decoding only the coarser blocks).
//
//  k_dec_prep      per job: tile header and block-size table checks, block
//                  descriptors and byte offsets (scan) of the blocks needed
//                  for the target level.
//  k_dec_header    per block (one wave, scalar parse): d, masks, C_zr, wz,
//                  recursive code tree (Fig. 3: 0 = internal node, 1 + 8 bits
//                  = leaf), seek table; builds the prefix table plus the
//                  sorted left-aligned codes (any valid tree is accepted, not
//                  only canonical ones) and queues one item per segment.
//  k_dec_segments  per segment (persistent waves over the queue): tokens ->
//                  symbols (runs of zeros from the bijective-base counters, a
//                  literal C_zr from a zero counter).
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

template <int NT>  // 256, or 1024 for tiles of many blocks
__global__ void __launch_bounds__(NT) k_dec_prep(PlanHdr H, const uint8_t *__restrict__ plan,
                                                 const uint8_t *__restrict__ enc,
                                                 uint8_t *__restrict__ ws,
                                                 int32_t *__restrict__ status)
{
    __shared__ uint64_t sh[NT / 64];
    __shared__ int32_t s_st;
    const uint32_t job = blockIdx.x;
    const TileGeo &T = ((const TileGeo *)(plan + H.tiles_off))[job];
    BlockDesc *descs = (BlockDesc *)(ws + H.ws_blockdesc);
    const uint8_t *base = enc + T.enc_offset;
    const uint64_t avail = T.enc_bytes;
    if (job == 0)  // segment queue
        for (uint32_t i = threadIdx.x; i < kItemsHdr / 4; i += blockDim.x) ((uint32_t *)(ws + H.ws_items))[i] = 0;
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
    // region decode: the plan lists the blocks with their byte ranges (from
    // the stream's size table, read by the host); each is checked here
    // against the size table in the stream
    const SelBlock *sel = T.sel_off ? (const SelBlock *)(plan + T.sel_off) : nullptr;
    const uint64_t table_end = 24 + 4ull * T.nblocks_stream;
    uint64_t carry = table_end, scarry = 0;
    uint32_t bad = 0;
    for (uint32_t b0 = 0; b0 < T.nblocks; b0 += NT) {
        const uint32_t i = b0 + threadIdx.x;
        const uint32_t local = (sel && i < T.nblocks) ? sel[i].local : i;
        BlockDesc B;
        uint64_t sz = 0, ssz = 0;
        if (i < T.nblocks) {
            block_geometry(T, local, B);
            B.drop = (uint8_t)T.drop;
            ssz = block_sym_bytes(B, T.dmax);
            if (st == D_OK) {
                uint64_t o = 24 + 4ull * local;
                sz = (uint64_t)base[o] | ((uint64_t)base[o + 1] << 8) | ((uint64_t)base[o + 2] << 16) |
                     ((uint64_t)base[o + 3] << 24);
            }
        }
        uint64_t tot, stot;
        uint64_t ex = sel ? 0 : dblock_excl_sum<NT>(sz, sh, &tot);
        uint64_t sex = dblock_excl_sum<NT>(ssz, sh, &stot);
        if (i < T.nblocks) {
            uint64_t off = sel ? sel[i].off : carry + ex;
            bool ok = sz > 0 && off >= table_end && off + sz <= avail;
            if (sel && sz != sel[i].len) ok = false;
            B.tile = job;
            B.sym_off = T.sym_base + scarry + sex;
            B.slot = T.slot_base + i * T.dmax;
            B.dmax = T.dmax;
            if (st == D_OK && ok) {
                B.byte_off = T.enc_offset + off;
                B.byte_len = (uint32_t)sz;
            } else {
                B.byte_off = 0;
                B.byte_len = 0;
                if (st == D_OK) bad = 1;
            }
            descs[T.block_base + i] = B;
        }
        if (!sel) carry += tot;
        scarry += stot;
    }
    bad = __syncthreads_or(bad);
    if (threadIdx.x == 0) status[job] = (st == D_OK && bad) ? D_TRUNC : st;
}

// ------------------------------------------------------------------ header
// Wave-uniform reader of the staged header words (big-endian, in LDS): every
// value goes through readfirstlane, so the parse runs on the scalar unit.
// `buf` holds `avail` >= 32 valid bits, left-aligned; the next word is loaded
// one refill ahead.
__device__ inline uint32_t rfl(uint32_t x) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)x); }

struct UBits {
    const uint32_t *w;
    uint32_t nw;
    uint64_t buf;
    uint32_t avail, nx, pos;
    uint32_t pre;  // next word (vector register until used)
    __device__ inline uint32_t load(uint32_t i) const { return i < nw ? w[i] : 0u; }
    __device__ inline void init(const uint32_t *words, uint32_t n)
    {
        w = words; nw = n;
        buf = ((uint64_t)rfl(load(0)) << 32) | rfl(load(1));
        pre = load(2);
        avail = 64; nx = 3; pos = 0;
    }
    // restart at bit `b` of the words
    __device__ inline void init_at(const uint32_t *words, uint32_t n, uint32_t b)
    {
        w = words; nw = n;
        const uint32_t i = b >> 5, o = b & 31u;
        const uint64_t x = ((uint64_t)rfl(load(i)) << 32) | rfl(load(i + 1));
        buf = x << o;
        avail = 64 - o;
        pre = load(i + 2);
        nx = i + 3;
        pos = b;
    }
    __device__ inline uint32_t peek() const { return (uint32_t)(buf >> 32); }
    __device__ inline void skip(uint32_t k)  // k <= 32
    {
        buf <<= k;
        avail -= k;
        pos += k;
        if (avail <= 32) {
            buf |= (uint64_t)rfl(pre) << (32 - avail);
            avail += 32;
            pre = load(nx++);
        }
    }
    __device__ inline uint32_t get(uint32_t k)  // k <= 32
    {
        uint32_t v = k ? peek() >> (32 - k) : 0u;
        skip(k);
        return v;
    }
};

// 64 header bits from bit b on (words w[b / 32 ..] big-endian, MSB first).
__device__ inline uint64_t hbits64(const uint32_t *w, uint32_t b)
{
    const uint32_t i = b >> 5, o = b & 31u;
    const uint64_t x = ((uint64_t)w[i] << 32) | w[i + 1];
    return o ? (x << o) | ((uint64_t)w[i + 2] >> (32 - o)) : x;
}

// Token walk over one 64-bit chunk of the serialised tree (0 = internal
// node, one bit; 1 + 8 bits = leaf): from the token start `pos` < 64, the
// first token start at or after bit 64, minus 64 (0..8).
__device__ inline uint32_t tree_chunk_exit(uint64_t W, uint32_t pos)
{
    while (pos < 64) {
        const uint64_t rest = W << pos;
        if (!rest) return 0;  // internal nodes up to the chunk end
        pos += (uint32_t)__builtin_clzll(rest) + 9;
    }
    return pos - 64;
}

// Per block, one wave: header (layout of Fig. 3 as read: d, masks, C_zr, wz,
// pre-order code tree with 0 = internal node and 1 + 8 bits = leaf, seek
// table), then the prefix table and sorted left-aligned codes of the tree
// (any valid tree is accepted, not only canonical ones), then one work item
// per kept segment, appended to the large- or small-segment list.
__global__ void __launch_bounds__(64) k_dec_header(PlanHdr H, const uint8_t *__restrict__ enc,
                                                   uint8_t *__restrict__ ws,
                                                   int32_t *__restrict__ status)
{
    __shared__ uint32_t hw[136];
    __shared__ uint16_t s_lzb[256], s_lend[256];  // per tokenised leaf: 0-tokens before it, end bit
    __shared__ uint8_t s_lsym[256];
    __shared__ uint32_t s_acode[256];
    __shared__ uint8_t s_len[256], s_sym[256];
    __shared__ uint32_t s_bits[32], s_M[32];
    __shared__ uint64_t s_pos[32];
    __shared__ uint8_t s_plane[32];
    __shared__ uint32_t s_seen[8];
    const uint32_t lane = threadIdx.x;
    const uint32_t blk = blockIdx.x;
    const BlockDesc &B = ((const BlockDesc *)(ws + H.ws_blockdesc))[blk];
    BlkPlan &P = ((BlkPlan *)(ws + H.ws_blkplan))[blk];
    const uint32_t blen = B.byte_len;
    const int32_t tst = __builtin_amdgcn_readfirstlane(status[B.tile]);
    if (tst != D_OK || blen == 0) {
        if (lane == 0) { P.nseg = 0; P.err = 1; P.d = 1; }
        return;
    }
    const uint8_t *src = enc + B.byte_off;
    // the first 512 bytes hold any header (<= ~400 bytes)
    for (uint32_t i = lane; i < 128; i += 64) {
        uint32_t x = 0;
        for (int k = 0; k < 4; k++) x = (x << 8) | rd_byte(src, blen, 4 * i + k);
        hw[i] = x;
    }
    if (lane < 8) hw[128 + lane] = 0;
    __syncthreads();
    const uint32_t p = B.p, n = (uint32_t)B.wb * B.hb / 8;
    const uint32_t lim = (blen < 512 ? blen : 512) * 8;
    UBits r;
    r.init(hw, 136);
    int32_t err = 0;
    const uint32_t d = r.get(5);
    uint32_t masks[3] = {0, 0, 0};
    if (d >= 1 && d <= B.dmax) {
        for (uint32_t t = 0; t < p; t++) masks[t] = r.get(d);
    } else {
        err = D_CORRUPT;
    }
    uint32_t nseg = 0;
    if (!err) {
        for (int b = (int)d - 1; b >= 0; b--) {
            uint32_t pm = 0;
            for (uint32_t t = 0; t < p; t++) pm |= (((masks[t] >> b) & 1u) ^ 1u) << t;
            if (pm) {
                s_plane[nseg] = (uint8_t)b;
                s_M[nseg] = n * __popc(pm);
                nseg++;
            }
        }
    }
    uint32_t czr = 0, wz = 0, m = 0;
    if (!err && nseg) {
        czr = r.get(8);
        wz = r.get(4);
        const uint32_t beta = bitlen32(p * n - 1), wzhi = beta > 2 ? beta : 2;
        if (wz < 2 || wz > wzhi) err = D_CORRUPT;
        // The tree, in two steps.  (1) Tokens in parallel: lane c takes bits
        // [64c, 64c + 64) of the tree; for each of the 9 places its first
        // token can start (a leaf from the previous chunk reaches up to 8
        // bits in) it finds where its last token ends; composing these maps
        // over the lanes gives every lane its true first token, and each
        // lane lists its leaves with the number of 0-tokens (internal
        // nodes) before them.  (2) The pre-order walk itself, on the scalar
        // unit, leaf by leaf: a run of z internal nodes deepens the current
        // node by z; after a leaf with left-aligned code A and depth d the
        // next node is at A + 2^(32-d), depth 32 - ctz.  Every violation
        // (a node deeper than 32, more than 511 nodes, bits past the header,
        // a 257th leaf, a repeated symbol, no closing leaf) is the same
        // error, so the checks are grouped.
        const uint32_t t0 = r.pos;
        if (lane < 8) s_seen[lane] = 0;
        const uint64_t W = hbits64(hw, t0 + 64 * lane);
        uint64_t f = 0;  // 9 exits, 4 bits each
#pragma unroll 1
        for (uint32_t e = 0; e < 9; e++) f |= (uint64_t)tree_chunk_exit(W, e) << (4 * e);
        // inclusive scan of the maps (F_c = f_c o ... o f_0), then the entry
        // of chunk c = F_{c-1}(0)
        uint64_t F = f;
        for (int o = 1; o < 64; o <<= 1) {
            const uint64_t G = __shfl_up(F, o, 64);
            if ((int)lane >= o) {
                uint64_t h = 0;
#pragma unroll
                for (uint32_t e = 0; e < 9; e++) h |= ((F >> (4 * ((G >> (4 * e)) & 15u))) & 15u) << (4 * e);
                F = h;
            }
        }
        const uint64_t Fp = __shfl_up(F, 1, 64);
        uint32_t pos = lane == 0 ? 0u : (uint32_t)(Fp & 15u);
        // this lane's leaves (at most 8 in 64 bits)
        uint32_t lq[8], lz[8], nl = 0, nz = 0;
#pragma unroll
        for (int k = 0; k < 8; k++) { lq[k] = 0; lz[k] = 0; }
#pragma unroll
        for (int k = 0; k < 8; k++) {
            if (pos < 64) {
                const uint64_t rest = W << pos;
                const uint32_t z = rest ? (uint32_t)__builtin_clzll(rest) : 64u - pos;
                if (pos + z < 64) {
                    nz += z;
                    lq[k] = pos + z;
                    lz[k] = nz;
                    nl++;
                    pos += z + 9;
                } else {
                    nz += 64 - pos;
                    pos = 64;
                }
            }
        }
        if (pos < 64) nz += 64 - pos;  // unreachable: 8 leaves fill 72 bits
        uint32_t Lx = nl, Zx = nz;  // inclusive scans over the lanes
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t a = __shfl_up(Lx, o, 64), b = __shfl_up(Zx, o, 64);
            if ((int)lane >= o) { Lx += a; Zx += b; }
        }
        const uint32_t NL = __builtin_amdgcn_readlane(Lx, 63);
        const uint32_t Lpre = Lx - nl, Zpre = Zx - nz;
#pragma unroll
        for (int k = 0; k < 8; k++) {
            const uint32_t j = Lpre + (uint32_t)k;
            if ((uint32_t)k < nl && j < 256) {
                const uint32_t a = t0 + 64 * lane + lq[k];
                s_lzb[j] = (uint16_t)(Zpre + lz[k]);
                s_lend[j] = (uint16_t)(a + 9);
                s_lsym[j] = (uint8_t)(hbits64(hw, a + 1) >> 56);
            }
        }
        __syncthreads();
        // leaf j's record in lane j % 64 of R[j / 64]: the 0-tokens since the
        // previous leaf (bits 0-5, at most 63: more is a depth error anyway),
        // its symbol (6-13), a node-count or header-end violation (14), the
        // bit after it (15-27), and bit 31 for "no such leaf"
        uint32_t R0, R1, R2, R3;
        {
            const uint32_t nlc = NL < 256 ? NL : 256;
            auto rec = [&](uint32_t j) -> uint32_t {
                if (j >= nlc) return 1u << 31;
                const uint32_t zb = s_lzb[j], end = s_lend[j];
                const uint32_t z = zb - (j ? (uint32_t)s_lzb[j - 1] : 0u);
                const uint32_t bad = (zb + j + 1 > 511 || end > lim) ? 1u : 0u;
                return (z < 63 ? z : 63u) | ((uint32_t)s_lsym[j] << 6) | (bad << 14) | (end << 15);
            };
            R0 = rec(lane); R1 = rec(64 + lane); R2 = rec(128 + lane); R3 = rec(192 + lane);
        }
        __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): the records are in registers
        // the walk: leaf j's code and depth go to lane j % 64 of Aq, Dq (q =
        // j / 64).  The serial part carries only what the next leaf needs:
        // its depth (the deepest open right branch, 32 - ctz of the running
        // code, plus the leaf's 0-tokens) and the running code.  Where the
        // tree closes (a lone leaf of depth 0, or the carry out of the
        // rightmost leaf) and whether a leaf up to there breaks a rule is
        // found afterwards, 64 leaves at a time; leaves after the close are
        // computed but never read.
        uint32_t A0 = 0, A1 = 0, A2 = 0, A3 = 0, D0 = 0, D1 = 0, D2 = 0, D3 = 0;
        uint32_t A = 0, base = 0;
        auto walk = [&](uint32_t Rq, uint32_t &Aq, uint32_t &Dq) {
#pragma unroll 16
            for (uint32_t ln = 0; ln < 64; ln++) {
                const uint32_t d = base + (__builtin_amdgcn_readlane(Rq, ln) & 63u);
                const bool mine = lane == ln;
                Aq = mine ? A : Aq;
                Dq = mine ? d : Dq;
                A += d ? 1u << ((32u - d) & 31u) : 0u;
                base = A ? 32u - (uint32_t)__builtin_ctz(A) : base;
            }
        };
        // per group of 64 leaves: walk it, then look for the close; groups
        // after the close are not walked (and not checked)
        uint32_t close = 256u;
        bool bad = false;
        auto check = [&](uint32_t q, uint32_t Rv, uint32_t Av, uint32_t Dv) {
            const uint32_t An = Av + (Dv ? 1u << ((32u - Dv) & 31u) : 0u);
            const bool fail = (Rv >> 31) != 0u || ((Rv >> 14) & 1u) != 0u || Dv > 32u;
            const bool stop = !fail && (Dv == 0u || An < Av);
            const uint64_t sm = __ballot(stop), fm = __ballot(fail);
            // leaves of this group at or before the close
            const uint64_t upto = sm ? (2ull << __builtin_ctzll(sm)) - 1ull : ~0ull;
            bad |= (fm & upto) != 0ull;
            if (sm) close = 64u * q + (uint32_t)__builtin_ctzll(sm);
        };
        walk(R0, A0, D0);
        check(0, R0, A0, D0);
        if (close == 256u) { walk(R1, A1, D1); check(1, R1, A1, D1); }
        if (close == 256u) { walk(R2, A2, D2); check(2, R2, A2, D2); }
        if (close == 256u) { walk(R3, A3, D3); check(3, R3, A3, D3); }
        m = close < 256u ? close + 1u : 0u;
        if (bad || close == 256u) err = D_CORRUPT;  // a violation, or 256 leaves and open: a symbol repeats
        uint32_t tend = t0;
        if (!err) {
            const uint32_t q = (m - 1) >> 6, ln = (m - 1) & 63u;
            const uint32_t Rl = q == 0 ? R0 : (q == 1 ? R1 : (q == 2 ? R2 : R3));
            tend = ((uint32_t)__builtin_amdgcn_readlane(Rl, ln) >> 15) & 0x1fffu;
#pragma unroll
            for (uint32_t k = 0; k < 4; k++) {
                const uint32_t j = 64 * k + lane;
                const uint32_t Av = k == 0 ? A0 : (k == 1 ? A1 : (k == 2 ? A2 : A3));
                const uint32_t Dv = k == 0 ? D0 : (k == 1 ? D1 : (k == 2 ? D2 : D3));
                const uint32_t Rv = k == 0 ? R0 : (k == 1 ? R1 : (k == 2 ? R2 : R3));
                if (j < m) {
                    s_acode[j] = Av;
                    s_len[j] = (uint8_t)Dv;
                    s_sym[j] = (uint8_t)((Rv >> 6) & 255u);
                }
            }
        }
        if (!err) r.init_at(hw, 136, tend);
        __syncthreads();
        if (!err) {  // repeated symbols
            bool dup = false;
            for (uint32_t j = lane; j < m; j += 64) {
                const uint32_t v = s_sym[j];
                dup |= (atomicOr(&s_seen[v >> 5], 1u << (v & 31)) >> (v & 31)) & 1u;
            }
            if (__any(dup)) err = D_CORRUPT;
        }
        const uint32_t tb = bitlen32(p * n) - 1 + 5;
        uint64_t acc = 0;
        for (uint32_t s = 0; s < nseg && !err; s++) {
            if (r.pos + tb > lim) { err = D_TRUNC; break; }
            const uint32_t v = r.get(tb);
            s_bits[s] = v;
            acc += v;
        }
        if (!err) {
            uint64_t start = B.byte_off * 8 + r.pos;
            if (r.pos + acc > (uint64_t)blen * 8) err = D_TRUNC;
            for (uint32_t s = 0; s < nseg; s++) {
                s_pos[s] = start;
                start += s_bits[s];
            }
        }
    } else if (!err && r.pos > blen * 8) {
        err = D_TRUNC;
    }
    if (err) nseg = 0;
    // quality-progressive decode: the segments of magnitude planes b < drop
    // (the trailing ones) are neither queued nor read back
    uint32_t nkeep = nseg;
    while (nkeep > 0 && s_plane[nkeep - 1] < B.drop && s_plane[nkeep - 1] != d - 1) nkeep--;
    __syncthreads();
    if (lane == 0) {
        P.d = d; P.nseg = nkeep; P.czr = czr; P.wz = wz; P.m = m; P.p = p; P.n = n;
        P.err = err ? 1 : 0;
        for (uint32_t t = 0; t < 3; t++) P.masks[t] = masks[t];
        if (err) atomicMin(&status[B.tile], err);
    }
    if (!nkeep) return;
    if (lane < nseg) {
        P.seg_plane[lane] = s_plane[lane];
        P.seg_M[lane] = s_M[lane];
        P.seg_bits[lane] = s_bits[lane];
        P.seg_bitpos[lane] = s_pos[lane];
    }
    // prefix table: entry e belongs to the last leaf whose left-aligned code
    // is <= e << (32 - K): sym | len << 8; for codes longer than K, kLutLong |
    // the first candidate leaf | the number of candidates << 8 (the leaves
    // whose codes start with e; 0 = 64 or more), so that a long code is found
    // by a search over those leaves only
    uint8_t *tab = ws + H.ws_lut + (uint64_t)blk * kLutStride;
    {
        constexpr uint32_t per = (1u << kLutK) / 64;
        const uint32_t e0 = lane * per;
        uint32_t lo = 0, hi = m;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (s_acode[mid] <= (e0 << (32 - kLutK))) lo = mid; else hi = mid;
        }
        uint32_t j = lo, jh = lo;
        uint32_t packed[per / 2];
#pragma unroll
        for (uint32_t k = 0; k < per; k++) {
            const uint32_t key = (e0 + k) << (32 - kLutK);
            const uint32_t keyhi = key | ((1u << (32 - kLutK)) - 1u);
            while (j + 1 < m && s_acode[j + 1] <= key) j++;
            if (jh < j) jh = j;
            while (jh + 1 < m && s_acode[jh + 1] <= keyhi) jh++;
            const uint32_t L = s_len[j], cnt = jh - j + 1;
            const uint32_t e = (L <= (uint32_t)kLutK) ? (s_sym[j] | (L << 8))
                                                      : (kLutLong | j | ((cnt < 64 ? cnt : 0u) << 8));
            if (k & 1) packed[k / 2] |= e << 16; else packed[k / 2] = e;
        }
        uint4 *dst = (uint4 *)(tab + (uint64_t)e0 * 2);
#pragma unroll
        for (uint32_t k = 0; k < per / 8; k++)
            dst[k] = make_uint4(packed[4 * k], packed[4 * k + 1], packed[4 * k + 2], packed[4 * k + 3]);
    }
    uint32_t *acode = (uint32_t *)(tab + kLutBytes16);
    uint8_t *llen = tab + kLutBytes16 + 1024, *lsym = llen + 256;
    for (uint32_t j = lane; j < 256; j += 64) {
        acode[j] = j < m ? s_acode[j] : 0xffffffffu;
        llen[j] = j < m ? s_len[j] : 0;
        lsym[j] = j < m ? s_sym[j] : 0;
    }
    // work items: large segments (at least seg_big_bits) first in the
    // decode order.  A small block
    // (at most 1536 symbols per plane: 64x64-coefficient types, or smaller)
    // whose kept segments are all short and fit the LDS staging together is
    // one item (segment field kWholeBlock): one wave decodes its segments
    // one after the other with the tables and bits loaded once.  Large
    // blocks keep one item per segment, decoded side by side.
    uint32_t *ctr = (uint32_t *)(ws + H.ws_items);
    {
        const uint32_t bl = lane < nkeep ? s_bits[lane] : 0u;
        uint32_t mx = bl, sum = bl;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            mx = max(mx, (uint32_t)__shfl_xor(mx, o, 64));
            sum += __shfl_xor(sum, o, 64);
        }
        const bool small_block = p * n <= 1536u && mx < kSmallSegBits;
        // (seg_whole_words: the staging of the wave that takes such an
        // item; 0 in the latency form, where the segments of a block run
        // side by side)
        if (H.seg_whole_words && nkeep >= 2 && small_block && sum + 64 <= (H.seg_whole_words - 2) * 32u) {
            if (lane == 0) {
                const uint32_t sb1 = atomicAdd(&ctr[kQSmall], 1u);
                uint32_t *list = (uint32_t *)(ws + H.ws_items + kItemsHdr);
                list[H.total_blocks * 32ull + sb1] = (blk << 5) | kWholeBlock;
            }
            return;
        }
    }
    const bool big = lane < nkeep && s_bits[lane] >= H.seg_big_bits;
    const uint64_t bm = __ballot(big);
    const uint32_t nbig = __popcll(bm), nsmall = nkeep - nbig;
    uint32_t bb = 0, sb = 0;
    if (lane == 0) {
        if (nbig) bb = atomicAdd(&ctr[kQBig], nbig);
        if (nsmall) sb = atomicAdd(&ctr[kQSmall], nsmall);
    }
    bb = __shfl(bb, 0, 64);
    sb = __shfl(sb, 0, 64);
    if (lane < nkeep) {
        const uint64_t below = (1ull << lane) - 1ull;
        const uint32_t item = (blk << 5) | lane;
        uint32_t *list = (uint32_t *)(ws + H.ws_items + kItemsHdr);
        if (big) list[bb + __popcll(bm & below)] = item;
        else list[H.total_blocks * 32ull + sb + (lane - __popcll(bm & below))] = item;
    }
}

// ------------------------------------------------------------------ segments
// Bit cursors over one segment; positions are relative to the segment start
// and only move forward between seeks.  A cursor holds three consecutive
// stream words (MSB first): bit r lies in the first, a, at an offset k < 32;
// the third, n, is fetched when the window moves on, so that its latency
// overlaps the next token's table lookup instead of adding to it.
struct CurLds {
    const uint32_t *w;  // staged words, from the word holding the first bit (w[nw], w[nw + 1] are zero)
    uint32_t off;       // bit offset of the segment start in w[0]
    uint32_t nw;        // staged words
    uint32_t wi, a, b, n;
    __device__ inline uint32_t ld(uint32_t i) const { return w[i <= nw + 1 ? i : nw + 1]; }
    __device__ inline void seek(uint32_t r)
    {
        wi = (r + off) >> 5;
        a = ld(wi); b = ld(wi + 1); n = ld(wi + 2);
    }
    __device__ inline void step() { a = b; b = n; wi++; n = ld(wi + 2); }
};

// big-endian word `wi` of the stream, bytes outside [lo, hi) read as 0
__device__ inline uint32_t stream_word(const uint8_t *enc, uint64_t lo, uint64_t hi, uint64_t wi)
{
    const uint64_t b = wi * 4;
    if (b >= lo && b + 4 <= hi) return __builtin_bswap32(*(const uint32_t *)(enc + b));
    uint32_t x = 0;
    for (int k = 0; k < 4; k++) x = (x << 8) | ((b + k >= lo && b + k < hi) ? enc[b + k] : 0u);
    return x;
}

struct CurGlb {
    const uint8_t *enc;
    uint64_t lo, hi, w0;  // readable bytes; word of the first bit
    uint32_t off;
    uint32_t wi, a, b, n;
    __device__ inline uint32_t ld(uint32_t i) const { return stream_word(enc, lo, hi, w0 + i); }
    __device__ inline void seek(uint32_t r)
    {
        wi = (r + off) >> 5;
        a = ld(wi); b = ld(wi + 1); n = ld(wi + 2);
    }
    __device__ inline void step() { a = b; b = n; wi++; n = ld(wi + 2); }
};

// moves the window to bit r; returns r's offset in a
template <class Cur>
__device__ inline uint32_t cur_at(Cur &C, uint32_t r)
{
    uint32_t k = r + C.off - (C.wi << 5);
    while (k >= 32) {
        C.step();
        k -= 32;
    }
    return k;
}
// the 32 bits from offset k < 64 of the window
template <class Cur>
__device__ inline uint32_t cur_win(const Cur &C, uint32_t k)
{
    const uint64_t x = k < 32 ? (((uint64_t)C.a << 32) | C.b) : (((uint64_t)C.b << 32) | C.n);
    return (uint32_t)((x << (k & 31)) >> 32);
}

struct DecTab {
    const uint16_t *lut;
    const uint32_t *acode;
    const uint8_t *llen, *lsym;
    uint32_t m, czr, wz;
};

// One token at r: returns the symbol; c = counter of a C_zr symbol (else 0),
// adv = bits taken.
template <class Cur>
__device__ inline uint32_t dec_token(Cur &C, const DecTab &T, uint32_t r, uint32_t &c, uint32_t &adv)
{
    const uint32_t k = cur_at(C, r);
    const uint32_t w = (uint32_t)(((((uint64_t)C.a << 32) | C.b) << k) >> 32);
    const uint32_t e = T.lut[w >> (32 - kLutK)];
    uint32_t v, L, cw;
    if (!(e & kLutLong)) {
        v = e & 0xffu;
        L = (e >> 8) & 0x3fu;
        cw = w << L;
    } else {
        // the leaves whose codes start with this prefix
        const uint32_t n = (e >> 8) & 0x3fu;
        uint32_t lo = e & 0xffu, hi = n ? lo + n : T.m;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (T.acode[mid] <= w) lo = mid; else hi = mid;
        }
        v = T.lsym[lo];
        L = T.llen[lo];
        cw = cur_win(C, k + L);
    }
    const bool z = (v == T.czr);
    c = z ? (cw >> (32 - T.wz)) : 0u;
    adv = L + (z ? T.wz : 0u);
    return v;
}

// Run-length bookkeeping of a token range as an affine map on (pos, R):
// pos = output position, R = value of the pending run of C_zr digits.
// Values saturate at kSat = 2^18: a segment holds at most 6144 symbols, so a
// saturated value always ends as a corrupt-stream error, and every per-token
// product (R < 2^18 times 2^wz - 1 < 2^13) stays in 32 bits.
constexpr uint32_t kSat = 1u << 18;
__device__ inline uint32_t sadd(uint32_t a, uint32_t b) { return min(a + b, kSat); }  // a, b <= kSat
__device__ inline uint32_t smul(uint32_t a, uint32_t b)
{
    const uint64_t r = (uint64_t)a * b;
    return r > kSat ? kSat : (uint32_t)r;
}
// R * (2^wz - 1) + c, saturated (R <= kSat, wz <= 13, c < 2^wz)
__device__ inline uint32_t run_push(uint32_t R, uint32_t c, uint32_t wz)
{
    return min((R << wz) - R + c, kSat);
}
struct RunXf {
    uint32_t lit;  // the range holds a literal symbol
    uint32_t P0;   // B^(digits before the first literal)
    uint32_t V0;   // value of those digits
    uint32_t mid;  // output symbols from the first literal up to the trailing digits
    uint32_t V1;   // value of the trailing digits (pending run)
};
__device__ inline RunXf xf_id() { RunXf f = {0, 1, 0, 0, 0}; return f; }
__device__ inline RunXf xf_combine(const RunXf &a, const RunXf &b)
{
    RunXf r;
    if (!a.lit) {
        r.lit = b.lit; r.P0 = smul(a.P0, b.P0); r.V0 = sadd(smul(a.V0, b.P0), b.V0);
        r.mid = b.mid; r.V1 = b.V1;
    } else if (!b.lit) {
        r.lit = 1; r.P0 = a.P0; r.V0 = a.V0; r.mid = a.mid; r.V1 = sadd(smul(a.V1, b.P0), b.V0);
    } else {
        r.lit = 1; r.P0 = a.P0; r.V0 = a.V0;
        r.mid = sadd(sadd(a.mid, sadd(smul(a.V1, b.P0), b.V0)), b.mid);
        r.V1 = b.V1;
    }
    return r;
}
// append one token (a C_zr digit when dig, else an output symbol); no branches
__device__ inline void xf_push(RunXf &f, bool dig, uint32_t c, uint32_t wz)
{
    const bool lit = f.lit != 0;
    const uint32_t R = lit ? f.V1 : f.V0;
    const uint32_t Rn = run_push(R, c, wz);
    const uint32_t P0n = run_push(f.P0, 0, wz);
    const uint32_t midl = lit ? min(f.mid + f.V1 + 1u, kSat) : 1u;
    const bool first = dig && !lit;
    f.V0 = first ? Rn : f.V0;
    f.P0 = first ? P0n : f.P0;
    f.V1 = dig ? (lit ? Rn : f.V1) : 0u;
    f.mid = dig ? f.mid : midl;
    f.lit = dig ? f.lit : 1u;
}

// Tokens from r up to the first token start at or after lim, appended to f.
// Once f holds a literal only mid and V1 change (a digit extends the pending
// run, a symbol closes it), so the rest of the range takes a shorter update.
template <class Cur>
__device__ inline uint32_t run_tokens(Cur &C, const DecTab &T, uint32_t r, uint32_t lim, RunXf &f)
{
    const uint32_t czr = T.czr, wz = T.wz;
    while (r < lim && !f.lit) {
        uint32_t c, adv;
        const uint32_t v = dec_token(C, T, r, c, adv);
        r += adv;
        xf_push(f, v == czr && c, c, wz);
    }
    uint32_t mid = f.mid, V1 = f.V1;
    while (r < lim) {
        uint32_t c, adv;
        const uint32_t v = dec_token(C, T, r, c, adv);
        r += adv;
        const bool dig = v == czr && c;
        mid = dig ? mid : min(mid + V1 + 1u, kSat);
        V1 = dig ? run_push(V1, c, wz) : 0u;
    }
    f.mid = mid;
    f.V1 = V1;
    return r;
}

// Phase-1 bits before the first and the second resynchronisation point.
constexpr uint32_t kSyncWin = 128, kSyncWin2 = 384;

// Decode of one segment by a workgroup of NW waves (G = 64 NW lanes): the
// segment's N bits are split into G chunks.  Phase 1: every lane decodes its
// chunk from the chunk start (speculatively, for lanes > 0), keeping the run
// maps of the tokens before the first token start sw1 at or after kSyncWin
// bits, from sw1 to the first token start sw2 at or after kSyncWin2 bits,
// and from sw2 on, and its exit (first token start at or after the chunk
// end).  Phase 2: a lane whose start differs from its left neighbour's exit
// decodes again from that exit; on reaching sw1, or else sw2, the rest of
// phase 1 stands (Huffman codes resynchronise), else it decodes the whole
// chunk; repeated until no lane changes.  A scan of the run maps over the
// lanes gives each lane its output position and pending run; phase 3 decodes
// again and writes the non-zero symbols into a zeroed copy of the plane in
// LDS (runs write nothing), which the workgroup then stores to the plane
// with whole-line 16-byte stores.  More waves per segment (NW = 2 or 4)
// shorten a segment's decode: the lanes' chunks halve or quarter, and the
// waves exchange their edge values through LDS at barriers.

// workgroup-wide hand-over between lanes: a wave's own LDS order, or a barrier
template <int NW>
__device__ inline void wg_sync()
{
    if (NW == 1) wave_sync();
    else __syncthreads();
}

// Stores the M symbols staged in LDS to the plane (both 16-byte aligned, the
// plane's stride padded to 16 bytes) with the whole workgroup.
template <int NW>
__device__ inline void store_plane(const uint8_t *pl, uint8_t *out, uint32_t M)
{
    const uint4 *src = (const uint4 *)pl;
    uint4 *dst = (uint4 *)out;
    const uint32_t M16 = (M + 15) / 16;
    for (uint32_t i = NW == 1 ? (threadIdx.x & 63) : threadIdx.x; i < M16; i += 64 * NW) dst[i] = src[i];
}
template <int NW>
__device__ inline void zero_lds_plane(uint8_t *pl, uint32_t M)
{
    uint4 *d = (uint4 *)pl;
    const uint32_t M16 = (M + 15) / 16;
    for (uint32_t i = NW == 1 ? (threadIdx.x & 63) : threadIdx.x; i < M16; i += 64 * NW) d[i] = make_uint4(0, 0, 0, 0);
}

// values the waves of a workgroup exchange
struct WaveX {
    uint32_t exit[4], any[4];
    uint32_t tot[4][5];  // each wave's run-map total (lit, P0, V0, mid, V1)
};

template <int NW, class Cur>
__device__ int32_t decode_segment(Cur C, const DecTab &T, uint32_t N, uint32_t M, uint8_t *pl, uint8_t *out,
                                  WaveX &X)
{
    constexpr uint32_t G = 64 * NW;
    // g: the thread's index in the group (one wave of a two-wave workgroup
    // may decode alone)
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = NW == 1 ? lane : threadIdx.x;
    const uint32_t wz = T.wz, czr = T.czr;
    uint32_t chunk = (N + G - 1) / G;
    chunk = (chunk + 31) & ~31u;
    if (chunk < 32) chunk = 32;
    const uint32_t cs = g * chunk;
    const bool active = cs < N;
    const uint32_t ce = active ? (cs + chunk < N ? cs + chunk : N) : cs;
    // phase 1
    RunXf fpre = xf_id(), G1 = xf_id(), G2 = xf_id();
    const uint32_t l1 = (cs + kSyncWin < ce) ? cs + kSyncWin : ce;
    C.seek(cs);
    const uint32_t sw1 = run_tokens(C, T, cs, l1, fpre);
    const uint32_t l2 = (cs + kSyncWin2 < ce) ? cs + kSyncWin2 : ce;
    const uint32_t sw2 = run_tokens(C, T, sw1, l2, G1);
    const uint32_t exit1 = run_tokens(C, T, sw2, ce, G2);
    const RunXf G12 = xf_combine(G1, G2);
    RunXf f = xf_combine(fpre, G12);
    uint32_t start = cs, exitc = exit1;
    // phase 2
    for (uint32_t it = 0; it < G; it++) {
        uint32_t left = __shfl_up(exitc, 1, 64);
        if (NW > 1) {
            if (lane == 63) X.exit[wave] = exitc;
            __syncthreads();
            if (lane == 0 && wave > 0) left = X.exit[wave - 1];
        }
        const uint32_t want = (g == 0) ? 0u : left;
        const bool chg = active && want != start;
        bool anyc = __any(chg);
        if (NW > 1) {
            if (lane == 0) X.any[wave] = anyc ? 1u : 0u;
            __syncthreads();
            anyc = false;
#pragma unroll
            for (int w = 0; w < NW; w++) anyc |= X.any[w] != 0;
            __syncthreads();  // every wave has read X before it is written again
        }
        if (!anyc) break;
        if (chg) {
            start = want;
            C.seek(want);
            RunXf Pm = xf_id();
            uint32_t q = run_tokens(C, T, want, min(sw1, ce), Pm);
            if (q == sw1) {
                f = xf_combine(Pm, G12);
                exitc = exit1;
            } else {
                q = run_tokens(C, T, q, min(sw2, ce), Pm);
                if (q == sw2) {
                    f = xf_combine(Pm, G2);
                    exitc = exit1;
                } else {
                    q = run_tokens(C, T, q, ce, Pm);
                    f = Pm;
                    exitc = q;
                }
            }
        }
    }
    if (!active) f = xf_id();
    // exclusive scan of the run maps: within each wave, then across the waves
    RunXf x = f;
    for (int o = 1; o < 64; o <<= 1) {
        RunXf y;
        y.lit = __shfl_up(x.lit, o, 64); y.P0 = __shfl_up(x.P0, o, 64); y.V0 = __shfl_up(x.V0, o, 64);
        y.mid = __shfl_up(x.mid, o, 64); y.V1 = __shfl_up(x.V1, o, 64);
        if ((int)lane >= o) x = xf_combine(y, x);
    }
    RunXf wpre = xf_id();  // the waves before this one
    if (NW > 1) {
        if (lane == 63) {
            X.tot[wave][0] = x.lit; X.tot[wave][1] = x.P0; X.tot[wave][2] = x.V0;
            X.tot[wave][3] = x.mid; X.tot[wave][4] = x.V1;
        }
        __syncthreads();
        for (uint32_t w = 0; w < wave; w++) {
            RunXf t;
            t.lit = X.tot[w][0]; t.P0 = X.tot[w][1]; t.V0 = X.tot[w][2]; t.mid = X.tot[w][3]; t.V1 = X.tot[w][4];
            wpre = xf_combine(wpre, t);
        }
        x = xf_combine(wpre, x);
    }
    RunXf ex;
    ex.lit = __shfl_up(x.lit, 1, 64); ex.P0 = __shfl_up(x.P0, 1, 64); ex.V0 = __shfl_up(x.V0, 1, 64);
    ex.mid = __shfl_up(x.mid, 1, 64); ex.V1 = __shfl_up(x.V1, 1, 64);
    if (lane == 0) ex = wpre;
    uint32_t op, run;
    if (ex.lit) { op = sadd(ex.V0, ex.mid); run = ex.V1; }
    else { op = 0; run = ex.V0; }
    zero_lds_plane<NW>(pl, M);
    wg_sync<NW>();
    // phase 3: write the non-zero symbols into the LDS plane
    int32_t err = 0;
    const bool last = active && (g == G - 1 || cs + chunk >= N);
    if (active) {
        uint32_t q = start;
        bool bad = false;
        C.seek(start);
        while (q < ce) {
            uint32_t c, adv;
            const uint32_t v = dec_token(C, T, q, c, adv);
            q += adv;
            const bool dig = (v == czr) && c;
            const uint32_t opr = sadd(op, run);
            bad |= !dig && (run == 1 || opr >= M);
            if (!dig && v && opr < M) pl[opr] = (uint8_t)v;
            op = dig ? op : opr + 1;
            run = dig ? run_push(run, c, wz) : 0u;
        }
        if (last) {
            if (run) {
                bad |= run < 2;
                op = sadd(op, run);
            }
            bad |= (q != N || op != M);
        }
        if (bad) err = D_CORRUPT;
    }
    wg_sync<NW>();
    store_plane<NW>(pl, out, M);
    if (N == 0 && g == 0 && M != 0) err = D_CORRUPT;
    return err;
}

struct SegShared {
    uint16_t lut[1 << kLutK];
    alignas(16) uint8_t plane[kMaxSeg];  // one segment's symbols
    uint32_t bits[kSegWords + 2];
};
// one wave's part where the two waves of a workgroup decode on their own
struct SegHalf {
    uint16_t lut[1 << kLutK];
    alignas(16) uint8_t plane[kMaxSeg];
    uint32_t bits[kHalfWords + 2];
};
template <int NW>
union SegLds {
    SegShared all;
    SegHalf half[NW == 2 ? 2 : 1];
};

// One queue item (a segment, or all kept segments of a small block) with the
// NW waves of the group: the prefix table and the bits (up to CAP words) to
// LDS, then per segment the three phases and the plane store.  t is the
// thread's index in the group.
template <int NW, uint32_t CAP>
__device__ __forceinline__ void dec_item(const PlanHdr &H, const uint8_t *__restrict__ enc, uint8_t *__restrict__ ws,
                         int32_t *__restrict__ status, uint32_t item, uint16_t *lut, uint8_t *plane,
                         uint32_t *bits, WaveX &X)
{
    constexpr uint32_t NT = 64 * NW;
    const uint32_t t = NW == 1 ? (threadIdx.x & 63) : threadIdx.x;
    const uint32_t blk = item >> 5, s = item & 31;
    const BlockDesc &B = ((const BlockDesc *)(ws + H.ws_blockdesc))[blk];
    const BlkPlan &P = ((const BlkPlan *)(ws + H.ws_blkplan))[blk];
    // segments [s0, s1) of the block: one, or all kept ones of a block item
    const bool whole = s == kWholeBlock;
    const uint32_t s0 = whole ? 0u : s;
    const uint32_t s1 = whole ? __builtin_amdgcn_readfirstlane(P.nseg) : s + 1;
    const uint64_t S0 = P.seg_bitpos[s0];
    const uint64_t Send = P.seg_bitpos[s1 - 1] + P.seg_bits[s1 - 1];
    const uint32_t Nall = (uint32_t)(Send - S0);
    const uint32_t pstride = plane_stride((uint32_t)B.p * B.wb * B.hb / 8);
    bool toolong = false;
    for (uint32_t k = s0; k < s1; k++) toolong |= P.seg_M[k] > kMaxSeg;
    if (toolong) {  // not reachable for 128-grid blocks
        if (t == 0) atomicMin(&status[B.tile], D_CORRUPT);
        return;
    }
    const uint8_t *tab = ws + H.ws_lut + (uint64_t)blk * kLutStride;
    wg_sync<NW>();  // the group's previous item is done with the LDS
    {
        // prefix table (kLutBytes16 / 16 pieces of 16 bytes): all loads
        // of a thread first.  The leaf tables that resolve the long codes
        // stay in global memory (read through the L1 cache).
        constexpr uint32_t NQ = kLutBytes16 / 16;
        static_assert(kLutBytes16 % 16 == 0, "table copy layout");
        const uint4 *src = (const uint4 *)tab;
        uint4 *dst = (uint4 *)lut;
        if constexpr (NQ % NT == 0) {
            constexpr uint32_t NR = NQ / NT;
            uint4 a[NR];
#pragma unroll
            for (uint32_t r = 0; r < NR; r++) a[r] = src[t + NT * r];
#pragma unroll
            for (uint32_t r = 0; r < NR; r++) dst[t + NT * r] = a[r];
        } else {
            static_assert(NT > NQ, "table copy layout");
            if (t < NQ) dst[t] = src[t];
        }
    }
    const uint64_t lo = B.byte_off, hi = B.byte_off + B.byte_len;
    const uint64_t w0 = S0 >> 5;
    const uint32_t nw = Nall ? (uint32_t)(((S0 + Nall - 1) >> 5) + 2 - w0) : 0u;
    const bool staged = nw <= CAP;
    if (staged) {
        // words w0 .. w0+nw-1 from 16-byte loads (4 per thread in
        // flight); a chunk not wholly inside the block falls back to bytes
        const bool al16 = (((uintptr_t)enc) & 15u) == 0;
        const uint64_t c0 = (w0 * 4) & ~15ull, c1 = (w0 + nw) * 4;
        const uint32_t nch = (uint32_t)((c1 - c0 + 15) / 16);
        for (uint32_t base = 0; base < nch; base += 4 * NT) {
            uint4 q[4];
#pragma unroll
            for (int k = 0; k < 4; k++) {
                const uint32_t ci = base + t + NT * k;
                const uint64_t cb = c0 + 16ull * ci;
                if (ci < nch && al16 && cb >= lo && cb + 16 <= hi) q[k] = *(const uint4 *)(enc + cb);
                else if (ci < nch) {
                    q[k].x = __builtin_bswap32(stream_word(enc, lo, hi, cb / 4));
                    q[k].y = __builtin_bswap32(stream_word(enc, lo, hi, cb / 4 + 1));
                    q[k].z = __builtin_bswap32(stream_word(enc, lo, hi, cb / 4 + 2));
                    q[k].w = __builtin_bswap32(stream_word(enc, lo, hi, cb / 4 + 3));
                }
            }
#pragma unroll
            for (int k = 0; k < 4; k++) {
                const uint32_t ci = base + t + NT * k;
                if (ci >= nch) continue;
                const int64_t r0 = (int64_t)((c0 / 4) + 4ull * ci) - (int64_t)w0;  // staged index of q[k].x
                if (r0 >= 0 && r0 + 3 < (int64_t)nw) {
                    bits[r0] = __builtin_bswap32(q[k].x);
                    bits[r0 + 1] = __builtin_bswap32(q[k].y);
                    bits[r0 + 2] = __builtin_bswap32(q[k].z);
                    bits[r0 + 3] = __builtin_bswap32(q[k].w);
                } else {
                    if (r0 >= 0 && r0 < (int64_t)nw) bits[r0] = __builtin_bswap32(q[k].x);
                    if (r0 + 1 >= 0 && r0 + 1 < (int64_t)nw) bits[r0 + 1] = __builtin_bswap32(q[k].y);
                    if (r0 + 2 >= 0 && r0 + 2 < (int64_t)nw) bits[r0 + 2] = __builtin_bswap32(q[k].z);
                    if (r0 + 3 >= 0 && r0 + 3 < (int64_t)nw) bits[r0 + 3] = __builtin_bswap32(q[k].w);
                }
            }
        }
        if (t < 2) bits[nw + t] = 0u;
    }
    wg_sync<NW>();
    DecTab T;
    T.lut = lut;
    T.acode = (const uint32_t *)(tab + kLutBytes16);
    T.llen = tab + kLutBytes16 + 1024;
    T.lsym = T.llen + 256;
    T.m = P.m; T.czr = P.czr; T.wz = P.wz;
    int32_t err = 0;
    for (uint32_t k = s0; k < s1; k++) {
        const uint32_t M = P.seg_M[k], N = P.seg_bits[k];
        const uint64_t Sk = P.seg_bitpos[k];
        uint8_t *out = ws + B.sym_off + (uint64_t)P.seg_plane[k] * pstride;
        int32_t e = 0;
        if (T.m == 1 && T.lsym[0] != T.czr) {
            // zero-length codewords: the segment is M copies of the leaf
            if (N != 0) e = D_CORRUPT;
            const uint32_t fill = T.lsym[0] * 0x01010101u;
            uint32_t *pw = (uint32_t *)plane;
            wg_sync<NW>();  // the previous segment's plane has been stored
            for (uint32_t i = t; i < (M + 15) / 16 * 4; i += NT) {
                const uint32_t b = 4 * i;
                pw[i] = b + 4 <= M ? fill : (b < M ? fill & ((1u << (8 * (M - b))) - 1u) : 0u);
            }
            wg_sync<NW>();
            store_plane<NW>(plane, out, M);
        } else if (staged) {
            const uint32_t wk = (uint32_t)((Sk >> 5) - w0);
            CurLds src;
            src.w = bits + wk; src.off = (uint32_t)(Sk & 31); src.nw = nw - wk;
            wg_sync<NW>();  // the previous segment's plane has been stored
            e = decode_segment<NW>(src, T, N, M, plane, out, X);
        } else {
            CurGlb src;
            src.enc = enc; src.lo = lo; src.hi = hi; src.w0 = Sk >> 5; src.off = (uint32_t)(Sk & 31);
            wg_sync<NW>();
            e = decode_segment<NW>(src, T, N, M, plane, out, X);
        }
        err = e ? e : err;
    }
    if (err) atomicMin(&status[B.tile], err);
}

// Persistent workgroups of NW waves taking (block, segment) items from the
// two lists (large segments first).  The default form (NW = 2): two waves
// share 14.5 KB for a large segment and decode it together; once the large
// list is drained each of them takes small items on its own in half of the
// workgroup's LDS (20 KB per workgroup: eight per CU, sixteen waves, as many
// as their registers allow).  NW = 4: four waves decode every item together
// (the latency form for plans of few segments).  NW = 1: one wave per item,
// 14.5 KB of LDS each, eleven per CU (selectable by the launch tuning).
template <int NW>
__global__ void __launch_bounds__(64 * NW, NW == 2 ? 4 : 1) k_dec_segments(PlanHdr H, const uint8_t *__restrict__ enc,
                                                          uint8_t *__restrict__ ws,
                                                          int32_t *__restrict__ status)
{
    __shared__ SegLds<NW> S;
    __shared__ WaveX X;
    __shared__ uint32_t s_item;
    __shared__ int32_t s_status;
    const uint32_t tid = threadIdx.x;
    uint32_t *ctr = (uint32_t *)(ws + H.ws_items);
    const uint32_t nbig = __builtin_amdgcn_readfirstlane(ctr[kQBig]);
    const uint32_t ntot = nbig + __builtin_amdgcn_readfirstlane(ctr[kQSmall]);
    const uint32_t *list = (const uint32_t *)(ws + H.ws_items + kItemsHdr);
    const uint32_t *small = list + H.total_blocks * 32ull;
    for (;;) {
        uint32_t idx = 0;
        if (tid == 0) idx = atomicAdd(&ctr[kQTake], 1u);
        if (NW > 1) {
            __syncthreads();  // the previous item is done with S and s_item
            if (tid == 0) s_item = idx;
            __syncthreads();
            idx = s_item;
        }
        idx = __builtin_amdgcn_readfirstlane(idx);
        if (idx >= ntot) break;
        if constexpr (NW == 2) {
            if (idx >= nbig) {
                // the large list is drained (the take counter only grows):
                // from here on each wave takes small items alone, wave 0
                // starting with this one.  No barrier follows; the
                // barriers above saw both waves done with S.all.
                const uint32_t w = tid >> 6;
                SegHalf &Hf = S.half[w];
                uint32_t id = idx;
                if (w != 0) {
                    id = 0;
                    if ((tid & 63) == 0) id = atomicAdd(&ctr[kQTake], 1u);
                    id = __builtin_amdgcn_readfirstlane(id);
                }
                while (id < ntot) {
                    const uint32_t item = __builtin_amdgcn_readfirstlane(small[id - nbig]);
                    const BlockDesc &B = ((const BlockDesc *)(ws + H.ws_blockdesc))[item >> 5];
                    if (__builtin_amdgcn_readfirstlane(status[B.tile]) == D_OK)
                        dec_item<1, kHalfWords>(H, enc, ws, status, item, Hf.lut, Hf.plane, Hf.bits, X);
                    id = 0;
                    if ((tid & 63) == 0) id = atomicAdd(&ctr[kQTake], 1u);
                    id = __builtin_amdgcn_readfirstlane(id);
                }
                return;
            }
        }
        const uint32_t item = __builtin_amdgcn_readfirstlane(idx < nbig ? list[idx] : small[idx - nbig]);
        const BlockDesc &B = ((const BlockDesc *)(ws + H.ws_blockdesc))[item >> 5];
        // the tile's status, as one thread read it (other workgroups may set
        // it meanwhile, and every wave must take the same branch)
        int32_t st;
        if (NW > 1) {
            if (tid == 0) s_status = status[B.tile];
            __syncthreads();
            st = s_status;
        } else {
            st = status[B.tile];
        }
        if (__builtin_amdgcn_readfirstlane(st) != D_OK) continue;
        dec_item<NW, kSegWords>(H, enc, ws, status, item, S.all.lut, S.all.plane, S.all.bits, X);
    }
}

// ------------------------------------------------------------------ reassembly
// 16x16 bit-matrix transpose: bit j of r[i] moves to bit i of r[j] (rows of
// 16 bits in the low halves), by the recursive block transpose (blocks of 8,
// 4, 2 and 1 bits swapped between rows i and i + s).
__device__ inline void transpose16(uint32_t (&r)[16])
{
#pragma unroll
    for (int s = 8, k = 0; s >= 1; s >>= 1, k++) {
        const uint32_t m = k == 0 ? 0x00ffu : (k == 1 ? 0x0f0fu : (k == 2 ? 0x3333u : 0x5555u));
#pragma unroll
        for (int i = 0; i < 16; i++) {
            if (i & s) continue;
            const uint32_t x = ((r[i] >> s) ^ r[i + s]) & m;
            r[i + s] ^= x;
            r[i] ^= x << s;
        }
    }
}

// Reassembly of NC (1 or 2) consecutive cells ci .. ci + NC - 1 of type t
// (4x4 coefficients each): the 16 low magnitude planes and the sign plane
// (d - 1) in flight together (a plane the type skips, or above the block's
// depth, is not read and counts as 0: the condition is the same for a wave's
// cells of one type), then one 16x16 bit-matrix transpose per cell turns
// plane words into magnitudes; dequantised, signed and stored.
// The same transpose for two cells at once: each word holds a plane word of
// the first cell in its low half and of the second in its high half (the
// masks keep every exchange inside its half).
__device__ inline void transpose16x2(uint32_t (&r)[16])
{
#pragma unroll
    for (int s = 8, k = 0; s >= 1; s >>= 1, k++) {
        const uint32_t m = k == 0 ? 0x00ff00ffu : (k == 1 ? 0x0f0f0f0fu : (k == 2 ? 0x33333333u : 0x55555555u));
#pragma unroll
        for (int i = 0; i < 16; i++) {
            if (i & s) continue;
            const uint32_t x = ((r[i] >> s) ^ r[i + s]) & m;
            r[i + s] ^= x;
            r[i] ^= x << s;
        }
    }
}

typedef uint16_t u16x2 __attribute__((ext_vector_type(2)));

template <int NC>
__device__ __forceinline__ void reasm_cells(const BlockDesc &B, uint8_t *ws, const uint8_t *sym,
                                   const uint32_t (*s_off)[3], uint32_t t, uint32_t ci, uint32_t d,
                                   uint32_t wq, uint32_t step, bool c16)
{
    auto ld = [&](uint32_t o) -> uint32_t {
        return NC == 2 ? *(const uint32_t *)(sym + o + 2 * ci) : (uint32_t)*(const uint16_t *)(sym + o + 2 * ci);
    };
    const uint32_t tw = B.tw[t], th = B.th[t];
    const uint64_t toff = B.off[t];
    const uint32_t tpitch = B.pitch[t];
    // both cells in one band row, whole, int16: each row's 8 coefficients
    // in one 16-byte store (8 int16 elements, aligned)
    const bool row16 =
        NC == 2 && c16 && ((toff | tpitch) & 7u) == 0 && (ci % wq) + 1 < wq && 4 * ((ci % wq) + 1) + 3 < tw;
    uint32_t mag[NC][16], sgn[NC];
    bool split = true;
    if constexpr (NC == 2) {
        if (d <= 17) {
            // magnitudes of at most 16 bits: the two cells' plane words
            // stay packed in one register through the transpose
            uint32_t pw[16];
#pragma unroll
            for (int b = 0; b < 16; b++) {
                const uint32_t o = (uint32_t)b + 1 < d ? s_off[b][t] : ~0u;
                pw[b] = o != ~0u ? ld(o) : 0u;
            }
            uint32_t sg;
            {
                const uint32_t o = d ? s_off[d - 1][t] : ~0u;
                const uint32_t v = ld(o != ~0u ? o : 0u);
                sg = o != ~0u ? v : 0u;
            }
            transpose16x2(pw);
            if (B.drop) {  // midpoint of the dropped magnitude bits (no carry out of a half)
                const uint32_t half = 1u << (B.drop - 1);
#pragma unroll
                for (int i = 0; i < 16; i++)
                    pw[i] += ((pw[i] & 0xffffu) ? half : 0u) + ((pw[i] >> 16) ? half << 16 : 0u);
            }
            if (row16) {
                // dequantised and signed as 16-bit pairs: (q*step + step/2
                // for q != 0), then two's complement where the sign bit is set
                const u16x2 stp = (u16x2)(uint16_t)step, hlf = (u16x2)(uint16_t)(step / 2), one = (u16x2)1;
                uint32_t v[16];
#pragma unroll
                for (int i = 0; i < 16; i++) {
                    u16x2 q = __builtin_bit_cast(u16x2, pw[i]);
                    if (step > 1) q = q * stp + __builtin_elementwise_min(q, one) * hlf;
                    const uint32_t s1 = (sg >> i) & 0x00010001u;  // sign bits, one per half
                    const u16x2 m = __builtin_bit_cast(u16x2, __builtin_bit_cast(uint32_t, q) ^ (s1 * 0xffffu));
                    v[i] = __builtin_bit_cast(uint32_t, m + __builtin_bit_cast(u16x2, s1));
                }
                const uint32_t r0 = 4 * (ci / wq), c0 = 4 * (ci % wq);
#pragma unroll
                for (int rr = 0; rr < 4; rr++) {
                    const uint32_t row = r0 + rr;
                    if (row >= th) continue;
                    int16_t *dst = (int16_t *)ws + toff + (uint64_t)row * tpitch + c0;
                    const uint32_t *q = v + 4 * rr;
                    // low halves: the first cell's row, high halves: the second's
                    *(uint4 *)dst = make_uint4(__builtin_amdgcn_perm(q[1], q[0], 0x05040100u),
                                               __builtin_amdgcn_perm(q[3], q[2], 0x05040100u),
                                               __builtin_amdgcn_perm(q[1], q[0], 0x07060302u),
                                               __builtin_amdgcn_perm(q[3], q[2], 0x07060302u));
                }
                return;
            }
#pragma unroll
            for (int i = 0; i < 16; i++) {
                mag[0][i] = pw[i] & 0xffffu;
                mag[NC - 1][i] = pw[i] >> 16;
            }
            sgn[0] = sg & 0xffffu;
            sgn[NC - 1] = sg >> 16;
            split = false;
        }
    }
    if (split) {
#pragma unroll
        for (int b = 0; b < 16; b++) {
            const uint32_t o = (uint32_t)b + 1 < d ? s_off[b][t] : ~0u;
            uint32_t v = 0;
            if (o != ~0u) v = ld(o);
#pragma unroll
            for (int k = 0; k < NC; k++) mag[k][b] = (v >> (16 * k)) & 0xffffu;
        }
        {
            const uint32_t o = d ? s_off[d - 1][t] : ~0u;
            const uint32_t v = ld(o != ~0u ? o : 0u);
#pragma unroll
            for (int k = 0; k < NC; k++) sgn[k] = o != ~0u ? (v >> (16 * k)) & 0xffffu : 0u;
        }
#pragma unroll
        for (int k = 0; k < NC; k++) transpose16(mag[k]);
        // magnitude planes 16 .. d-2 (samples deeper than 16 bits)
        for (uint32_t b = 16; b + 1 < d; b++) {
            const uint32_t o = s_off[b][t];
            if (o == ~0u) continue;
            const uint32_t v = ld(o);
#pragma unroll
            for (int k = 0; k < NC; k++)
#pragma unroll
                for (int i = 0; i < 16; i++) mag[k][i] |= ((v >> (16 * k + i)) & 1u) << b;
        }
        if (B.drop) {  // midpoint of the dropped magnitude bits
            const uint32_t half = 1u << (B.drop - 1);
#pragma unroll
            for (int k = 0; k < NC; k++)
#pragma unroll
                for (int i = 0; i < 16; i++) mag[k][i] += mag[k][i] ? half : 0u;
        }
    }
    auto coef = [&](int k, int i) -> int32_t {
        int32_t q = (int32_t)mag[k][i];
        if (step > 1 && q) q = q * (int32_t)step + (int32_t)(step / 2);
        return ((sgn[k] >> i) & 1u) ? -q : q;
    };
    if (row16) {
        const uint32_t r0 = 4 * (ci / wq), c0 = 4 * (ci % wq);
#pragma unroll
        for (int rr = 0; rr < 4; rr++) {
            const uint32_t row = r0 + rr;
            if (row >= th) continue;
            int16_t *dst = (int16_t *)ws + toff + (uint64_t)row * tpitch + c0;
            const uint32_t w0 = (uint16_t)coef(0, rr * 4) | ((uint32_t)(uint16_t)coef(0, rr * 4 + 1) << 16);
            const uint32_t w1 = (uint16_t)coef(0, rr * 4 + 2) | ((uint32_t)(uint16_t)coef(0, rr * 4 + 3) << 16);
            const uint32_t w2 = (uint16_t)coef(NC - 1, rr * 4) | ((uint32_t)(uint16_t)coef(NC - 1, rr * 4 + 1) << 16);
            const uint32_t w3 = (uint16_t)coef(NC - 1, rr * 4 + 2) | ((uint32_t)(uint16_t)coef(NC - 1, rr * 4 + 3) << 16);
            *(uint4 *)dst = make_uint4(w0, w1, w2, w3);
        }
        return;
    }
#pragma unroll
    for (int k = 0; k < NC; k++) {
        const uint32_t band = (ci + k) / wq, cg = (ci + k) % wq;
        const uint32_t r0 = 4 * band, c0 = 4 * cg;
#pragma unroll
        for (int rr = 0; rr < 4; rr++) {
            const uint32_t row = r0 + rr;
            if (row >= th || c0 >= tw) continue;
            int32_t o[4];
#pragma unroll
            for (int cc = 0; cc < 4; cc++) o[cc] = coef(k, rr * 4 + cc);
            if (c16) {  // coefficients held as int16 (their bound fits)
                int16_t *dst = (int16_t *)ws + toff + (uint64_t)row * tpitch + c0;
                if (c0 + 3 < tw) *(short4 *)dst = make_short4((short)o[0], (short)o[1], (short)o[2], (short)o[3]);
                else
                    for (int cc = 0; cc < 4 && c0 + cc < tw; cc++) dst[cc] = (int16_t)o[cc];
                continue;
            }
            int32_t *dst = (int32_t *)ws + toff + (uint64_t)row * tpitch + c0;
            if (c0 + 3 < tw) *(int4 *)dst = make_int4(o[0], o[1], o[2], o[3]);
            else
                for (int cc = 0; cc < 4 && c0 + cc < tw; cc++) dst[cc] = o[cc];
        }
    }
}

// Blocks of the plan's list [list0, list0 + nlist): NT = 1024 threads for the
// blocks of more than 768 cells, 256 for the others.
template <int NT>
__global__ void __launch_bounds__(NT) k_dec_reasm(PlanHdr H, const uint8_t *__restrict__ plan,
                                                  uint8_t *__restrict__ ws,
                                                  const int32_t *__restrict__ status, uint32_t list0,
                                                  uint32_t nlist)
{
    // per plane b of the block and type t: the byte offset of the type's
    // symbols in the plane (~0: not decoded for the type), so that the cell
    // loop issues only independent symbol loads
    __shared__ uint32_t s_off[32][3];
    const uint32_t tid = threadIdx.x;
    const uint32_t *list = (const uint32_t *)(plan + H.list_off) + list0;
    for (uint32_t li = blockIdx.x; li < nlist; li += gridDim.x) {
    const uint32_t blk = list[li];
    const BlockDesc &B = ((const BlockDesc *)(ws + H.ws_blockdesc))[blk];
    const BlkPlan &P = ((const BlkPlan *)(ws + H.ws_blkplan))[blk];
    if (status[B.tile] != D_OK) continue;
    const TileGeo &T = ((const TileGeo *)(plan + H.tiles_off))[B.tile];
    const uint32_t p = B.p, wb = B.wb, hb = B.hb, n = wb * hb / 8, cpt = n / 2, wq = wb / 4;
    const uint32_t d = P.d, nseg = P.nseg;
    const uint32_t step = (B.level == 0) ? 1u : T.qstep;
    const bool c16 = B.c16 != 0;
    const uint8_t *sym = ws + B.sym_off;
    const uint32_t pstr = plane_stride(p * n);
    __syncthreads();  // the previous block's table has been read
    if (tid < 96) (&s_off[0][0])[tid] = ~0u;
    __syncthreads();
    if (tid < nseg) {
        const uint32_t b = P.seg_plane[tid];
        uint32_t pm = 0;
        for (uint32_t u = 0; u < p; u++) pm |= (((P.masks[u] >> b) & 1u) ^ 1u) << u;
        for (uint32_t u = 0; u < 3; u++)
            s_off[b][u] = ((pm >> u) & 1u) ? b * pstr + (uint32_t)__popc(pm & ((1u << u) - 1u)) * n : ~0u;
    }
    __syncthreads();
    if ((cpt & 1u) == 0 && (n & 3u) == 0) {
        // two horizontally consecutive cells per thread: their symbols are
        // adjacent in every plane, one 32-bit load per plane
        for (uint32_t pr = tid; pr < p * cpt / 2; pr += blockDim.x) {
            const uint32_t cell = 2 * pr, t = cell / cpt;
            reasm_cells<2>(B, ws, sym, s_off, t, cell % cpt, d, wq, step, c16);
        }
    } else {
        for (uint32_t cell = tid; cell < p * cpt; cell += blockDim.x)
            reasm_cells<1>(B, ws, sym, s_off, cell / cpt, cell % cpt, d, wq, step, c16);
    }
    }
}

// ------------------------------------------------------------------ launch
hipError_t launch_inverse_level(const PlanHdr &H, const uint8_t *d_plan, uint8_t *d_ws,
                                uint8_t *d_pixels_out, const int32_t *d_status, int level,
                                hipStream_t stream);

// Stages (in order): prep, block headers, segments, reassembly, inverse
// levels 15..1 (intermediate outputs), final output stage.
hipError_t launch_decode(const PlanHdr &H, const uint8_t *d_plan, const uint8_t *d_encoded,
                         uint8_t *d_pixels_out, int32_t *d_status, uint8_t *d_ws,
                         hipStream_t stream, int first, int last)
{
    for (int st = first; st <= last; st++) {
        if (st == DEC_PREP) {
            if (H.max_nblocks > 512)
                hipLaunchKernelGGL(k_dec_prep<1024>, dim3(H.n_tiles), dim3(1024), 0, stream, H, d_plan, d_encoded, d_ws,
                                   d_status);
            else
                hipLaunchKernelGGL(k_dec_prep<256>, dim3(H.n_tiles), dim3(256), 0, stream, H, d_plan, d_encoded, d_ws,
                                   d_status);
        } else if (st == DEC_HDR) {
            if (H.total_blocks)
                hipLaunchKernelGGL(k_dec_header, dim3(H.total_blocks), dim3(64), 0, stream, H, d_encoded, d_ws, d_status);
        } else if (st == DEC_SEG) {
            if (H.total_blocks) {
                // no more waves than the plan can queue segments (a block
                // queues at most one per plane, at most its tile's plane bound)
                const uint32_t slots = std::max<uint32_t>(H.total_slots, 1u);
                if (H.seg_nw == 4)  // four workgroups of four waves per CU (registers)
                    hipLaunchKernelGGL(k_dec_segments<4>, dim3(std::min<uint32_t>(H.num_cus * 4, slots)), dim3(256), 0,
                                       stream, H, d_encoded, d_ws, d_status);
                else if (H.seg_nw == 2)
                    hipLaunchKernelGGL(k_dec_segments<2>, dim3(std::min<uint32_t>(H.num_cus * 8, slots)), dim3(128), 0,
                                       stream, H, d_encoded, d_ws, d_status);
                else
                    hipLaunchKernelGGL(k_dec_segments<1>, dim3(std::min<uint32_t>(H.num_cus * H.seg_waves_per_cu, slots)),
                                       dim3(64), 0, stream, H, d_encoded, d_ws, d_status);
            }
        } else if (st == DEC_REASM) {
            if (H.seg_nw == 4 && H.n_big + H.n_small) {
                // a plan of few blocks: all of them in one launch
                hipLaunchKernelGGL(k_dec_reasm<1024>, dim3(H.n_big + H.n_small), dim3(1024), 0, stream, H, d_plan, d_ws,
                                   d_status, 0u, H.n_big + H.n_small);
            } else {
                if (H.n_big) {
                    const uint32_t g =
                        H.blocks_per_cu ? std::min<uint32_t>(H.n_big, H.num_cus * H.blocks_per_cu) : H.n_big;
                    hipLaunchKernelGGL(k_dec_reasm<1024>, dim3(g), dim3(1024), 0, stream, H, d_plan, d_ws, d_status,
                                       0u, H.n_big);
                }
                if (H.n_small) {
                    const uint32_t g =
                        H.blocks_per_cu ? std::min<uint32_t>(H.n_small, H.num_cus * H.blocks_per_cu * 4) : H.n_small;
                    hipLaunchKernelGGL(k_dec_reasm<256>, dim3(g), dim3(256), 0, stream, H, d_plan, d_ws, d_status,
                                       H.n_big, H.n_small);
                }
            }
        } else if (st >= DEC_INV15 && st <= DEC_FINAL) {
            int level = DEC_FINAL - st;  // 15..1, then 0 = final stage
            hipError_t e = launch_inverse_level(H, d_plan, d_ws, d_pixels_out, d_status, level, stream);
            if (e != hipSuccess) return e;
        }
    }
    return hipGetLastError();
}

}  // namespace isx
