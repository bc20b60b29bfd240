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
            ssz = block_sym_bytes(B, T.dmax);
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
// Bits of the block header staged in LDS, read through a 64-bit window.
struct LdsBits {
    const uint32_t *w;  // big-endian words
    uint32_t nwords;
    uint64_t pos;       // next bit
    uint64_t win;       // bits [wpos, wpos + 64)
    uint64_t wpos;
    __device__ inline uint32_t word(uint64_t i) const { return i < nwords ? w[i] : 0u; }
    __device__ inline void seek(uint64_t p)
    {
        pos = p;
        wpos = p & ~31ull;
        win = ((uint64_t)word(wpos >> 5) << 32) | word((wpos >> 5) + 1);
    }
    __device__ inline uint32_t get(uint32_t n)  // n <= 32
    {
        if (!n) return 0;
        while (pos - wpos > 32) { wpos += 32; win = (win << 32) | word((wpos >> 5) + 1); }
        uint32_t off = (uint32_t)(pos - wpos);
        uint64_t v = (win << off) >> (64 - n);
        pos += n;
        return (uint32_t)v;
    }
};

// ------------------------------------------------------------------ segments
// Window over the stream (MSB-first): `buf` holds nb >= 33 valid bits of the
// stream from the current position, `pre` the next 32-bit word; loads are
// bounded to [lo, hi) bytes.
struct BitRd {
    const uint8_t *base;
    uint64_t lo, hi;
    uint64_t buf;
    uint32_t nb;
    uint64_t nextw;
    uint32_t pre;
    __device__ inline uint32_t load(uint64_t wi) const
    {
        uint64_t b = wi * 4;
        if (b >= lo && b + 4 <= hi) return __builtin_bswap32(*(const uint32_t *)(base + b));
        uint32_t x = 0;
        for (int k = 0; k < 4; k++) x = (x << 8) | ((b + k >= lo && b + k < hi) ? base[b + k] : 0u);
        return x;
    }
    __device__ inline void seek(uint64_t pos)
    {
        uint64_t w = pos >> 5;
        uint32_t o = (uint32_t)(pos & 31);
        buf = (((uint64_t)load(w) << 32) | load(w + 1)) << o;
        nb = 64 - o;
        nextw = w + 2;
        pre = load(nextw);
    }
    __device__ inline uint32_t peek() const { return (uint32_t)(buf >> 32); }
    __device__ inline void skip(uint32_t k)  // k <= 32
    {
        buf <<= k;
        nb -= k;
        if (nb < 32) {
            buf |= (uint64_t)pre << (32 - nb);
            nb += 32;
            nextw++;
            pre = load(nextw);
        }
    }
};

// Run-length bookkeeping of a token range as an affine map on (pos, R):
// pos = output position, R = value of the pending run of C_zr digits.
constexpr uint32_t kSat = 1u << 30;
__device__ inline uint32_t smul(uint32_t a, uint32_t b) { uint64_t r = (uint64_t)a * b; return r > kSat ? kSat : (uint32_t)r; }
__device__ inline uint32_t sadd(uint32_t a, uint32_t b) { uint32_t r = a + b; return r > kSat ? kSat : r; }
struct RunXf {
    uint32_t lit;  // the range holds a literal symbol
    uint32_t P0;   // B^(digits before the first literal)
    uint32_t V0;   // value of those digits
    uint32_t mid;  // output symbols from the first literal up to the trailing digits
    uint32_t V1;   // value of the trailing digits (pending run)
};
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

struct SegCtx {
    const uint16_t *lut;
    const uint32_t *acode;
    const uint8_t *llen, *lsym;
    uint32_t m, czr, wz, single;
};

// One token at the reader's position: returns the symbol, advances pos;
// *cnt = counter (valid when the symbol is C_zr).
__device__ inline uint32_t next_token(const SegCtx &C, BitRd &R, uint64_t &pos, uint32_t *cnt)
{
    uint32_t v, L;
    if (C.single) { v = C.lsym[0]; L = 0; }
    else {
        uint32_t pk = R.peek();
        uint16_t e = C.lut[pk >> (32 - kLutK)];
        if (!(e & kLutLong)) { v = e & 0xffu; L = (e >> 8) & 0x3fu; }
        else {
            uint32_t lo = 0, hi = C.m;
            while (hi - lo > 1) { uint32_t mid = (lo + hi) >> 1; if (C.acode[mid] <= pk) lo = mid; else hi = mid; }
            v = C.lsym[lo]; L = C.llen[lo];
        }
    }
    R.skip(L);
    pos += L;
    *cnt = 0;
    if (v == C.czr) {
        *cnt = R.peek() >> (32 - C.wz);
        R.skip(C.wz);
        pos += C.wz;
    }
    return v;
}

constexpr int kSyncBits = 128;  // token starts remembered per chunk (re-sync window)
constexpr int kDecWaves = 8;
constexpr uint32_t kMaxSeg = 3 * 128 * 128 / 8;  // symbols in the largest segment

struct DecShared {
    uint32_t hw[132];          // first 512 bytes of the block (header), big-endian words
    uint16_t lut[1 << kLutK];
    uint32_t acode[256];
    uint8_t llen[256], lsym[256];
    uint32_t vis[kDecWaves][64][kSyncBits / 32];
    uint32_t nseg, czr, wz, m, err;
    uint8_t seg_plane[32];
    uint32_t seg_M[32], seg_bits[32];
    uint64_t seg_bitpos[32];
};

// Block header (Fig. 3 layout as read): d, masks, C_zr, wz, pre-order code
// tree, seek table.  Lane 0 only.  Fills S and the block plan's d/masks/
// segments (used by the reassembly).
__device__ void parse_header(const BlockDesc &B, BlkPlan &P, DecShared &S)
{
    const uint32_t p = B.p, n = (uint32_t)B.wb * B.hb / 8;
    const uint32_t blen = B.byte_len;
    const uint64_t lim = (uint64_t)(blen < 512 ? blen : 512) * 8;
    LdsBits r;
    r.w = S.hw; r.nwords = 130;
    r.seek(0);
    int32_t err = 0;
    uint32_t d = r.get(5);
    uint32_t masks[3] = {0, 0, 0};
    if (d >= 1 && d <= B.dmax)
        for (uint32_t t = 0; t < p; t++) masks[t] = r.get(d);
    else err = D_CORRUPT;
    uint32_t nseg = 0;
    if (!err) {
        for (int b = (int)d - 1; b >= 0; b--) {
            uint32_t pm = 0;
            for (uint32_t t = 0; t < p; t++) pm |= (((masks[t] >> b) & 1u) ^ 1u) << t;
            if (pm) {
                S.seg_plane[nseg] = (uint8_t)b;
                S.seg_M[nseg] = n * __popc(pm);
                nseg++;
            }
        }
    }
    uint32_t czr = 0, wz = 0, m = 0;
    if (!err && nseg) {
        czr = r.get(8);
        wz = r.get(4);
        uint32_t beta = bitlen32(p * n - 1), wzhi = beta > 2 ? beta : 2;
        if (wz < 2 || wz > wzhi) err = D_CORRUPT;
        // pre-order tree: 0 = internal, 1 + 8-bit symbol = leaf.  Walk with
        // the left-aligned code A and depth of the current node; after a leaf
        // the next node is at A + 2^(32-depth), depth 32 - ctz.
        uint64_t A = 0;
        uint32_t depth = 0, nodes = 0;
        uint32_t seen[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        while (!err) {
            if (++nodes > 511 || r.pos + 1 > lim) { err = D_CORRUPT; break; }
            if (!r.get(1)) {
                if (depth >= 32) { err = D_CORRUPT; break; }
                depth++;
                continue;
            }
            if (r.pos + 8 > lim) { err = D_CORRUPT; break; }
            uint32_t sym = r.get(8);
            if ((seen[sym >> 5] >> (sym & 31)) & 1u) { err = D_CORRUPT; break; }
            seen[sym >> 5] |= 1u << (sym & 31);
            S.acode[m] = (uint32_t)A;
            S.llen[m] = (uint8_t)depth;
            S.lsym[m] = (uint8_t)sym;
            m++;
            if (depth == 0) break;  // a lone leaf is the whole tree
            A += 1ull << (32 - depth);
            if (A >= (1ull << 32)) break;  // the rightmost leaf closes the tree
            depth = 32 - (uint32_t)__builtin_ctzll(A);
        }
        const uint32_t tb = bitlen32(p * n) - 1 + 5;
        uint64_t acc = 0;
        for (uint32_t s = 0; s < nseg && !err; s++) {
            if (r.pos + tb > lim) { err = D_TRUNC; break; }
            S.seg_bits[s] = r.get(tb);
            acc += S.seg_bits[s];
        }
        if (!err) {
            uint64_t start = (uint64_t)B.byte_off * 8 + r.pos;
            if (r.pos + acc > (uint64_t)blen * 8) err = D_TRUNC;
            for (uint32_t s = 0; s < nseg; s++) {
                S.seg_bitpos[s] = start;
                start += S.seg_bits[s];
            }
        }
    } else if (!err && r.pos > (uint64_t)blen * 8) {
        err = D_TRUNC;
    }
    S.nseg = err ? 0 : nseg; S.czr = czr; S.wz = wz; S.m = m; S.err = (uint32_t)err;
    P.d = d; P.nseg = err ? 0 : nseg; P.p = p; P.n = n; P.err = err ? 1 : 0;
    for (uint32_t t = 0; t < 3; t++) P.masks[t] = masks[t];
    for (uint32_t s = 0; s < nseg && !err; s++) { P.seg_plane[s] = S.seg_plane[s]; P.seg_M[s] = S.seg_M[s]; }
}

// Entropy decode of a block: header, prefix table (4096 entries in LDS:
// entry e belongs to the last leaf whose left-aligned code is <= e << 20),
// then one wave per segment, the segment's bits split into 64 chunks.
// Phase 1: every lane decodes its chunk from the chunk start (speculatively,
// for lanes > 0) and remembers its token starts in the first kSyncBits bits.
// Phase 2: a lane whose start differs from its left neighbour's exit
// re-decodes from that exit until it reaches a remembered token start (then
// its old exit stands) or its chunk end; repeated until no lane changes
// (Huffman codes resynchronise within a few tokens).  Phase 3: per-chunk run
// maps, a wave scan gives each lane its output position and pending run.
// Phase 4: decode again and write the non-zero symbols (the plane was zeroed
// first, so runs write nothing).
__global__ void __launch_bounds__(64 * kDecWaves) k_dec_blocks(PlanHdr H, const uint8_t *__restrict__ enc,
                                                               uint8_t *__restrict__ ws,
                                                               int32_t *__restrict__ status)
{
    __shared__ DecShared S;
    // per-wave staging of one segment's symbol plane (M <= 3 * 2048 bytes)
    __shared__ uint4 stg[kDecWaves][kMaxSeg / 16];
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (uint32_t blk = blockIdx.x; blk < H.total_blocks; blk += gridDim.x) {
    const BlockDesc &B = ((const BlockDesc *)(ws + H.ws_blockdesc))[blk];
    BlkPlan &P = ((BlkPlan *)(ws + H.ws_blkplan))[blk];
    const uint8_t *src = enc + B.byte_off;
    const uint32_t blen = B.byte_len;
    __syncthreads();  // the previous block is done with S
    for (uint32_t i = tid; i < 128; i += blockDim.x) {
        uint32_t x = 0;
        for (int k = 0; k < 4; k++) x = (x << 8) | rd_byte(src, blen, 4 * i + k);
        S.hw[i] = x;
    }
    if (tid < 4) S.hw[128 + tid] = 0;
    __syncthreads();
    if (tid == 0) {
        // the tile status is read once, so the whole workgroup takes the
        // same branch below
        if (status[B.tile] != D_OK || blen == 0) {
            P.nseg = 0; P.err = 1; P.d = 1;
            S.nseg = 0;
        } else {
            parse_header(B, P, S);
            if (S.err) atomicMin(&status[B.tile], (int32_t)S.err);
        }
    }
    __syncthreads();
    const uint32_t nseg = S.nseg, m = S.m;
    if (!nseg) continue;
    {
        const uint32_t per = (1u << kLutK) / (64 * kDecWaves);
        const uint32_t e0 = tid * per;
        uint32_t lo = 0, hi = m;
        while (hi - lo > 1) {
            uint32_t mid = (lo + hi) >> 1;
            if (S.acode[mid] <= (e0 << (32 - kLutK))) lo = mid; else hi = mid;
        }
        uint32_t j = lo;
        for (uint32_t e = e0; e < e0 + per; e++) {
            uint32_t key = e << (32 - kLutK);
            while (j + 1 < m && S.acode[j + 1] <= key) j++;
            uint32_t L = S.llen[j];
            S.lut[e] = (L <= (uint32_t)kLutK) ? (uint16_t)(S.lsym[j] | (L << 8)) : kLutLong;
        }
    }
    __syncthreads();
    SegCtx C;
    C.lut = S.lut; C.acode = S.acode; C.llen = S.llen; C.lsym = S.lsym; C.m = m;
    C.czr = S.czr; C.wz = S.wz; C.single = (m == 1);
    const uint32_t Bb = (1u << S.wz) - 1u;
    const uint32_t pstride = plane_stride((uint32_t)B.p * B.wb * B.hb / 8);
    BitRd R;
    R.base = enc; R.lo = B.byte_off; R.hi = B.byte_off + B.byte_len;
    int32_t err = 0;
    for (uint32_t s = wave; s < nseg; s += kDecWaves) {
        const uint32_t M = S.seg_M[s];
        if (M > kMaxSeg) { err = D_CORRUPT; continue; }  // not reachable for 128-grid blocks
        uint4 *gout = (uint4 *)(ws + B.sym_off + (uint64_t)S.seg_plane[s] * pstride);
        uint8_t *out = (uint8_t *)stg[wave];
        const uint32_t M16 = (M + 15) / 16;
        for (uint32_t i = lane; i < M16; i += 64) stg[wave][i] = make_uint4(0, 0, 0, 0);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        const uint64_t S0 = S.seg_bitpos[s], N = S.seg_bits[s], SE = S0 + N;
        if (C.single && S.lsym[0] != C.czr) {
            // zero-length codewords: the segment is M copies of the leaf
            if (N != 0) err = D_CORRUPT;
            else if (S.lsym[0]) for (uint32_t i = lane; i < M; i += 64) out[i] = S.lsym[0];
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            for (uint32_t i = lane; i < M16; i += 64) gout[i] = stg[wave][i];
            continue;
        }
        uint64_t chunk = (N + 63) / 64;
        chunk = (chunk + 31) & ~31ull;
        if (chunk < 32) chunk = 32;
        const uint64_t cs = S0 + lane * chunk;
        const bool active = cs < SE;
        const uint64_t ce = active ? (cs + chunk < SE ? cs + chunk : SE) : cs;
        // phase 1
        uint32_t *mv = S.vis[wave][lane];
#pragma unroll
        for (int k = 0; k < kSyncBits / 32; k++) mv[k] = 0;
        uint64_t start = cs, exit1 = cs;
        if (active) {
            uint64_t pos = cs;
            R.seek(pos);
            while (pos < ce) {
                uint64_t rel = pos - cs;
                if (rel < kSyncBits) mv[rel >> 5] |= 1u << (rel & 31);
                uint32_t c;
                next_token(C, R, pos, &c);
            }
            exit1 = pos;
        }
        uint64_t exitc = exit1;
        // phase 2
        for (int it = 0; it < 64; it++) {
            uint64_t left = __shfl_up(exitc, 1, 64);
            uint64_t want = (lane == 0) ? S0 : left;
            bool chg = active && want != start;
            if (!__any(chg)) break;
            if (chg) {
                start = want;
                uint64_t pos = want;
                bool synced = false;
                if (pos < ce) R.seek(pos);
                while (pos < ce) {
                    uint64_t rel = pos - cs;
                    if (rel < kSyncBits && ((mv[rel >> 5] >> (rel & 31)) & 1u)) { synced = true; break; }
                    uint32_t c;
                    next_token(C, R, pos, &c);
                }
                exitc = synced ? exit1 : pos;
            }
        }
        // phase 3: run maps and their scan
        RunXf f = {0, 1, 0, 0, 0};
        if (active && start < ce) {
            uint64_t pos = start;
            R.seek(pos);
            while (pos < ce) {
                uint32_t c;
                uint32_t v = next_token(C, R, pos, &c);
                if (v == C.czr && c) {
                    if (!f.lit) { f.V0 = sadd(smul(f.V0, Bb), c); f.P0 = smul(f.P0, Bb); }
                    else f.V1 = sadd(smul(f.V1, Bb), c);
                } else {
                    if (!f.lit) { f.lit = 1; f.mid = 1; }
                    else { f.mid = sadd(f.mid, sadd(f.V1, 1)); f.V1 = 0; }
                }
            }
        }
        RunXf x = f;
        for (int o = 1; o < 64; o <<= 1) {
            RunXf y;
            y.lit = __shfl_up(x.lit, o, 64); y.P0 = __shfl_up(x.P0, o, 64); y.V0 = __shfl_up(x.V0, o, 64);
            y.mid = __shfl_up(x.mid, o, 64); y.V1 = __shfl_up(x.V1, o, 64);
            if ((int)lane >= o) x = xf_combine(y, x);
        }
        RunXf ex;
        ex.lit = __shfl_up(x.lit, 1, 64); ex.P0 = __shfl_up(x.P0, 1, 64); ex.V0 = __shfl_up(x.V0, 1, 64);
        ex.mid = __shfl_up(x.mid, 1, 64); ex.V1 = __shfl_up(x.V1, 1, 64);
        if (lane == 0) { ex.lit = 0; ex.P0 = 1; ex.V0 = 0; ex.mid = 0; ex.V1 = 0; }
        uint32_t opos, orun;
        if (ex.lit) { opos = sadd(ex.V0, ex.mid); orun = ex.V1; }
        else { opos = 0; orun = ex.V0; }
        // phase 4: write
        const bool last = active && (lane == 63 || cs + chunk >= SE);
        if (active) {
            uint64_t pos = start;
            uint32_t op = opos, run = orun;
            if (pos < ce) R.seek(pos);
            while (pos < ce) {
                uint32_t c;
                uint32_t v = next_token(C, R, pos, &c);
                if (v == C.czr && c) { run = sadd(smul(run, Bb), c); continue; }
                if (run) {
                    if (run < 2) { err = D_CORRUPT; break; }
                    op = sadd(op, run);
                    run = 0;
                }
                if (op >= M) { err = D_CORRUPT; break; }
                if (v) out[op] = (uint8_t)v;
                op++;
            }
            if (last && !err) {
                if (run) {
                    if (run < 2) err = D_CORRUPT;
                    op = sadd(op, run);
                }
                if (pos != SE || op != M) err = D_CORRUPT;
            }
        }
        if (N == 0 && lane == 0 && M != 0) err = D_CORRUPT;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        for (uint32_t i = lane; i < M16; i += 64) gout[i] = stg[wave][i];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
    if (err) atomicMin(&status[B.tile], err);
    }
}

// ------------------------------------------------------------------ reassembly
__global__ void __launch_bounds__(1024) k_dec_reasm(PlanHdr H, const uint8_t *__restrict__ plan,
                                                    uint8_t *__restrict__ ws,
                                                    const int32_t *__restrict__ status)
{
    const uint32_t tid = threadIdx.x;
    for (uint32_t blk = blockIdx.x; blk < H.total_blocks; blk += gridDim.x) {
    const BlockDesc &B = ((const BlockDesc *)(ws + H.ws_blockdesc))[blk];
    const BlkPlan &P = ((const BlkPlan *)(ws + H.ws_blkplan))[blk];
    if (status[B.tile] != D_OK) continue;
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
            uint32_t v = *(const uint16_t *)(ws + B.sym_off + (uint64_t)b * plane_stride(p * n) + rank * n + 2 * ci);
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
            hipLaunchKernelGGL(k_dec_prep, dim3(H.n_tiles), dim3(256), 0, stream, H, d_plan, d_encoded, d_ws, d_status);
        } else if (st == DEC_SEG) {
            if (H.total_blocks)
                hipLaunchKernelGGL(k_dec_blocks, dim3(H.blk_grid), dim3(64 * kDecWaves), 0, stream, H, d_encoded, d_ws,
                                   d_status);
        } else if (st == DEC_REASM) {
            if (H.total_blocks)
                hipLaunchKernelGGL(k_dec_reasm, dim3(H.blk_grid), dim3(1024), 0, stream, H, d_plan, d_ws, d_status);
        } else if (st >= DEC_INV15 && st <= DEC_FINAL) {
            int level = DEC_FINAL - st;  // 15..1, then 0 = final stage
            hipError_t e = launch_inverse_level(H, d_plan, d_ws, d_pixels_out, d_status, level, stream);
            if (e != hipSuccess) return e;
        }
    }
    return hipGetLastError();
}

}  // namespace isx
