// k_encode.hip -- per-block entropy coder of the codec (Sec. 4, Eq. 1-3,
// Fig. 3) for gfx950: symbols, statistics, code construction, offsets and the
// bit packer.
//
// Per block (one workgroup each):
//  k_enc_symbols  d from the OR of the magnitudes (collected by the forward
//                 transform), the 4x2-area symbols of every kept bitplane
//                 (Eq. 1 order: 4-row bands, 4-column groups, upper area then
//                 lower area; Eq. 2 bit weights), a 256-bin histogram per
//                 segment, and the maximal zero runs of each segment via a
//                 workgroup prefix-max scan of the last non-zero position.
//  k_enc_code     C_zr = least frequent symbol (smallest on ties), a
//                 provisional Huffman code to get l, the counter width wz
//                 minimising Eq. 3, the final Huffman code (two-queue merge,
//                 (f, symbol) order, leaf first on ties), canonical codes,
//                 exact segment lengths (seek table), header and block sizes.
//  k_enc_pack     one workgroup per block header and per segment: token bit
//                 lengths, a prefix sum to bit offsets, MSB-first packing into
//                 an LDS window, written once to the final position in HBM.
// Per tile: block offsets (scan), tile offsets (scan), tile header.
#include <algorithm>

#include "isx_common.h"

namespace isx {

#define ISX_STATUS_OK 0
#define ISX_STATUS_CAPACITY (-2)
#define ISX_STATUS_CORRUPT (-3)
#define ISX_STATUS_TRUNC (-4)
#define ISX_STATUS_UNSUP (-5)

// ---------------------------------------------------------------- scans
template <int NT>
__device__ inline uint64_t block_excl_sum_u64(uint64_t v, uint64_t *sh /* NT/64 + 1 */, uint64_t *total)
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

template <int NT>
__device__ inline int32_t block_excl_max_i32(int32_t v, int32_t *sh)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int32_t x = v;
    for (int o = 1; o < 64; o <<= 1) {
        int32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x = max(x, y);
    }
    int32_t ex = __shfl_up(x, 1, 64);
    if (lane == 0) ex = -1;
    if (lane == 63) sh[wave] = x;
    __syncthreads();
    int32_t base = -1;
    for (int w = 0; w < wave; w++) base = max(base, sh[w]);
    __syncthreads();
    return max(base, ex);
}

// Digits of L in bijective base B = 2^w - 1.
__device__ inline uint32_t bij_digits(uint32_t L, uint32_t B)
{
    uint32_t m = 1, t = B, p = B;
    while (L > t) { p *= B; t += p; m++; }
    return m;
}

// ---------------------------------------------------------------- prep
// Per tile: block descriptors, symbol-area offsets, zeroed accumulators.
template <int NT>  // 256, or 1024 for tiles of many blocks
__global__ void __launch_bounds__(NT) k_prep_blocks(PlanHdr H, const uint8_t *__restrict__ plan,
                                                    uint8_t *__restrict__ ws)
{
    __shared__ uint64_t sh[NT / 64 + 1];
    const TileGeo &T = ((const TileGeo *)(plan + H.tiles_off))[blockIdx.x];
    BlockDesc *descs = (BlockDesc *)(ws + H.ws_blockdesc);
    BlkAcc *acc = (BlkAcc *)(ws + H.ws_acc);
    uint64_t carry = 0;
    for (uint32_t base = 0; base < T.nblocks; base += NT) {
        uint32_t local = base + threadIdx.x;
        BlockDesc B;
        uint64_t sz = 0;
        if (local < T.nblocks) {
            block_geometry(T, local, B);
            sz = block_sym_bytes(B, T.dmax);
        }
        uint64_t tot;
        uint64_t ex = block_excl_sum_u64<NT>(sz, sh, &tot);
        if (local < T.nblocks) {
            B.tile = blockIdx.x;
            B.sym_off = T.sym_base + carry + ex;
            B.slot = T.slot_base + local * T.dmax;
            B.dmax = T.dmax;
            B.byte_off = 0;
            B.byte_len = 0;
            descs[T.block_base + local] = B;
            BlkAcc z = {{0, 0, 0}, 0};
            acc[T.block_base + local] = z;
        }
        carry += tot;
    }
}

// ---------------------------------------------------------------- symbols
constexpr int kCellsPT = 3;  // 3 cells per thread: 1024 threads cover a 128x128 H-block (3 types)

// Blocks are split in two classes by size: more than 768 4x4 cells (1024
// threads) and at most 768 cells (256 threads); the plan lists the blocks of
// each class, large ones first.
constexpr int kPG = 4;  // phase B: planes per group (one set of barriers per group)

// 16x16 bit-matrix transpose: bit j of r[i] moves to bit i of r[j] (rows of
// 16 bits in the low halves).  Four rounds swap blocks of 8, 4, 2 and 1 bits
// between rows i and i + s (the recursive block transpose).
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

// The same for two cells at once: each word holds a row of the first cell in
// its low half and of the second in its high half (the masks keep every
// exchange inside its half).
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

template <int kSymNT>
__global__ void __launch_bounds__(kSymNT, 8) k_enc_symbols(PlanHdr H, const uint8_t *__restrict__ plan,
                                                        uint8_t *__restrict__ ws, uint32_t list0,
                                                        uint32_t nlist)
{
    constexpr int NW = kSymNT / 64;
    // phase-B statistics, double-buffered by group parity: a group's buffers
    // are read out after its second barrier and cleared during the next
    // group, so consecutive groups never touch the same words unsynchronised
    __shared__ uint32_t hist[2][kPG][256];
    __shared__ int32_t wmax[kPG][NW];
    __shared__ uint32_t s_zero[2][kPG], s_zir[2][kPG], s_pruns[2][kPG], s_dig[2][kPG][kNumWz];
    __shared__ uint32_t s_F[16];
    __shared__ uint32_t s_gb[2][kPG];  // the group's planes, for the read-out
    const uint32_t *list = (const uint32_t *)(plan + H.list_off) + list0;
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
    for (uint32_t i = tid; i < 2 * kPG * 256; i += kSymNT) (&hist[0][0][0])[i] = 0;
    for (uint32_t li = blockIdx.x; li < nlist; li += gridDim.x) {
    const uint32_t blk = list[li];
    __syncthreads();
    const BlockDesc B = ((const BlockDesc *)(ws + H.ws_blockdesc))[blk];
    const BlkAcc A = ((const BlkAcc *)(ws + H.ws_acc))[blk];
    BlkPlan &P = ((BlkPlan *)(ws + H.ws_blkplan))[blk];
    BlkStat &S = ((BlkStat *)(ws + H.ws_blkstat))[blk];
    uint16_t *seghist = (uint16_t *)(ws + H.ws_seghist);
    SegStat *segstat = (SegStat *)(ws + H.ws_segstat);
    const int32_t *wsi = (const int32_t *)ws;
    const uint32_t p = B.p, wb = B.wb, hb = B.hb, n = wb * hb / 8, cpt = n / 2, wq = wb / 4;

    uint32_t orall = A.or_mag[0] | A.or_mag[1] | A.or_mag[2];
    uint32_t d = 1 + bitlen32(orall);
    uint32_t err = 0;
    if (d > B.dmax) { err = 1; d = B.dmax; }
    uint32_t pres[3];
    for (int t = 0; t < 3; t++)
        pres[t] = (t < (int)p) ? ((A.or_mag[t] & ((1u << (d - 1)) - 1u)) | (((A.neg >> t) & 1u) << (d - 1))) : 0u;

    // phase A: every cell (4x4 coefficients) once -- its signed-magnitude
    // bits go straight to the block's symbol planes (the 16-bit pair of 4x2
    // area symbols of each kept plane, Eq. 1-2); consecutive threads take
    // consecutive cells so the 2-byte stores coalesce
    const uint32_t ncell = p * cpt;
    const uint32_t pstr = plane_stride(p * n);
    uint8_t *symb = ws + B.sym_off;
    const BlockDesc &Bg = ((const BlockDesc *)(ws + H.ws_blockdesc))[blk];
    const bool c16 = Bg.c16 != 0;  // coefficients held as int16
    // two horizontally adjacent cells per thread where their symbols are
    // adjacent, 4-byte aligned, in every plane and magnitudes fit 16 bits:
    // both cells' magnitudes go packed (first cell in the low halves)
    // through one 16x16 bit transpose and each plane gets one 32-bit store
    // (int16 blocks only: the int32 rows' loads would not fit the registers)
    const bool pairs = c16 && (cpt & 1u) == 0 && (wq & 1u) == 0 && (n & 3u) == 0 && d <= 17;
#pragma unroll 1
    for (int k = 0; pairs && k < (kCellsPT + 1) / 2; k++) {
        const uint32_t pr = (uint32_t)k * kSymNT + tid;
        if (2 * pr >= ncell) break;
        const uint32_t cell = 2 * pr, t = cell / cpt, ci = cell % cpt;
        const uint32_t band = ci / wq, cg = ci % wq;
        const uint32_t r0 = 4 * band, c0 = 4 * cg;
        const uint32_t tw = Bg.tw[t], th = Bg.th[t];
        const uint64_t toff = Bg.off[t];
        const uint32_t tpitch = Bg.pitch[t];
        uint32_t pw[16], sg = 0;
#pragma unroll
        for (int rr = 0; rr < 4; rr++) {
            const uint32_t row = r0 + rr;
            int32_t v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            if (row < th && c0 < tw) {
                const int16_t *src = (const int16_t *)ws + toff + (uint64_t)row * tpitch + c0;
                if (c0 + 7 < tw && ((toff + (uint64_t)row * tpitch + c0) & 7u) == 0) {
                    const uint4 q = *(const uint4 *)src;
                    const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
                    for (int e = 0; e < 4; e++) {
                        v[2 * e] = (int32_t)(w[e] << 16) >> 16;
                        v[2 * e + 1] = (int32_t)w[e] >> 16;
                    }
                } else {
#pragma unroll
                    for (int cc = 0; cc < 8; cc++) v[cc] = (c0 + cc < tw) ? src[cc] : 0;
                }
            }
#pragma unroll
            for (int cc = 0; cc < 4; cc++) {
                const int32_t a = v[cc], b = v[4 + cc];
                pw[rr * 4 + cc] = (uint32_t)(a < 0 ? -a : a) | ((uint32_t)(b < 0 ? -b : b) << 16);
                sg |= ((a < 0 ? 1u : 0u) | (b < 0 ? 0x10000u : 0u)) << (rr * 4 + cc);
            }
        }
        auto put2 = [&](int b, uint32_t v) {
            const uint32_t pm = ((pres[0] >> b) & 1u) | (((pres[1] >> b) & 1u) << 1) | (((pres[2] >> b) & 1u) << 2);
            if (!((pm >> t) & 1u)) return;
            const uint32_t rank = __popc(pm & ((1u << t) - 1u));
            *(uint32_t *)(symb + (uint64_t)b * pstr + rank * n + 2 * ci) = v;
        };
        put2((int)d - 1, sg);
        transpose16x2(pw);
#pragma unroll
        for (int b = 0; b < 16; b++)
            if (b + 1 < (int)d) put2(b, pw[b]);
    }
#pragma unroll 1
    for (int k = 0; !pairs && k < kCellsPT; k++) {
        const uint32_t cell = (uint32_t)k * kSymNT + tid;
        if (cell >= ncell) break;
        const uint32_t t = cell / cpt, ci = cell % cpt;
        const uint32_t band = ci / wq, cg = ci % wq;
        const uint32_t r0 = 4 * band, c0 = 4 * cg;
        // per-type fields read through the global copy (a runtime index into
        // a register copy would put the whole descriptor in scratch)
        const uint32_t tw = Bg.tw[t], th = Bg.th[t];
        const uint64_t toff = Bg.off[t];
        const uint32_t tpitch = Bg.pitch[t];
        uint32_t mag[16], sgn = 0;
#pragma unroll
        for (int rr = 0; rr < 4; rr++) {
            const uint32_t row = r0 + rr;
            int32_t v[4] = {0, 0, 0, 0};
            if (row < th && c0 < tw && c16) {
                const int16_t *src = (const int16_t *)ws + toff + (uint64_t)row * tpitch + c0;
                if (c0 + 3 < tw) {
                    const short4 q = *(const short4 *)src;
                    v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
                } else {
#pragma unroll
                    for (int cc = 0; cc < 4; cc++) v[cc] = (c0 + cc < tw) ? src[cc] : 0;
                }
            } else if (row < th && c0 < tw) {
                const int32_t *src = wsi + toff + (uint64_t)row * tpitch + c0;
                if (c0 + 3 < tw) {
                    const int4 q = *(const int4 *)src;
                    v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
                } else {
#pragma unroll
                    for (int cc = 0; cc < 4; cc++) v[cc] = (c0 + cc < tw) ? src[cc] : 0;
                }
            }
#pragma unroll
            for (int cc = 0; cc < 4; cc++) {
                mag[rr * 4 + cc] = (uint32_t)(v[cc] < 0 ? -v[cc] : v[cc]);
                sgn |= (v[cc] < 0 ? 1u : 0u) << (rr * 4 + cc);
            }
        }
        auto put_plane = [&](int b, uint32_t v) {
            const uint32_t pm = ((pres[0] >> b) & 1u) | (((pres[1] >> b) & 1u) << 1) | (((pres[2] >> b) & 1u) << 2);
            if (!((pm >> t) & 1u)) return;
            const uint32_t rank = __popc(pm & ((1u << t) - 1u));
            *(uint16_t *)(symb + (uint64_t)b * pstr + rank * n + 2 * ci) = (uint16_t)v;
        };
        put_plane((int)d - 1, sgn);
        // magnitude planes 16 .. d-2 (samples deeper than 16 bits): bit gathers
        for (int b = (int)d - 2; b >= 16; b--) {
            uint32_t v = 0;
#pragma unroll
            for (int i = 0; i < 16; i++) v |= ((mag[i] >> b) & 1u) << i;
            put_plane(b, v);
        }
        // planes 0 .. 15: one 16x16 bit-matrix transpose of the low halves
#pragma unroll
        for (int i = 0; i < 16; i++) mag[i] &= 0xffffu;
        transpose16(mag);
#pragma unroll
        for (int b = 0; b < 16; b++)
            if (b + 1 < (int)d) put_plane(b, mag[b]);
    }
    // phase B reads the planes back with a thread-contiguous cell layout
    uint32_t ctype[kCellsPT], cci[kCellsPT];
#pragma unroll
    for (int k = 0; k < kCellsPT; k++) {
        const uint32_t cell = tid * kCellsPT + k;
        ctype[k] = cell < ncell ? cell / cpt : 3u;
        cci[k] = cell < ncell ? cell % cpt : 0u;
    }
    __threadfence_block();
    // kept planes (a plane where no type is present is removed, Sec. 4)
    uint32_t keep = 0;
    for (int b = (int)d - 1; b >= 0; b--) {
        const uint32_t pm = ((pres[0] >> b) & 1u) | (((pres[1] >> b) & 1u) << 1) | (((pres[2] >> b) & 1u) << 2);
        if (pm) keep |= 1u << b;
    }
    for (uint32_t i = tid; i < 2 * kPG * (3 + kNumWz); i += kSymNT) {
        const uint32_t g = i / (3 + kNumWz), f = i % (3 + kNumWz);
        uint32_t *row = f == 0 ? &s_zero[0][0] : (f == 1 ? &s_zir[0][0] : (f == 2 ? &s_pruns[0][0] : &s_dig[0][0][f - 3]));
        row[f < 3 ? g : g * kNumWz] = 0;
    }
    if (tid < 16) s_F[tid] = 0;
    __syncthreads();

    uint32_t nseg = 0, nruns = 0, par = 0;
    while (keep) {
        // the group: up to kPG planes from the top
        uint32_t gb[kPG], gn = 0;
        {
            uint32_t r = keep;
#pragma unroll
            for (int g = 0; g < kPG; g++) {
                gb[g] = r ? 31u - (uint32_t)__builtin_clz(r) : 0u;
                if (r) { r &= ~(1u << gb[g]); gn++; }
            }
            keep = r;
        }
        if (tid < kPG) s_gb[par][tid] = gb[0];
#pragma unroll
        for (int g = 1; g < kPG; g++)
            if (tid == (uint32_t)g) s_gb[par][g] = gb[g];
        // the group's symbols of the thread's cells, all loads in flight at
        // once (a cell the plane skips reads the plane start and is masked
        // out); both passes use them
        uint32_t sy[kPG][kCellsPT];
#pragma unroll
        for (int g = 0; g < kPG; g++) {
            const uint32_t b = gb[g];
            const uint32_t pm = ((pres[0] >> b) & 1u) | (((pres[1] >> b) & 1u) << 1) | (((pres[2] >> b) & 1u) << 2);
            const uint8_t *segp = symb + (uint64_t)b * pstr;
#pragma unroll
            for (int k = 0; k < kCellsPT; k++) {
                const uint32_t t = ctype[k];
                const bool in = (uint32_t)g < gn && t <= 2 && ((pm >> t) & 1u);
                const uint32_t ps = in ? __popc(pm & ((1u << t) - 1u)) * n + 2 * cci[k] : 0u;
                const uint32_t v = *(const uint16_t *)(segp + ps);
                sy[g][k] = in ? (0x10000u | v) : 0u;
            }
        }
        // pass 1: histograms, zero counts, and the wave-level scan of the
        // last non-zero position
        int32_t ex[kPG];
#pragma unroll
        for (int g = 0; g < kPG; g++) {
            ex[g] = -1;
            if ((uint32_t)g >= gn) continue;
            const uint32_t b = gb[g];
            const uint32_t pm = ((pres[0] >> b) & 1u) | (((pres[1] >> b) & 1u) << 1) | (((pres[2] >> b) & 1u) << 2);
            int32_t lastnz = -1;
            uint32_t zeros = 0;
#pragma unroll
            for (int k = 0; k < kCellsPT; k++) {
                if (!(sy[g][k] >> 16)) continue;
                const uint32_t t = ctype[k];
                const uint32_t ps = __popc(pm & ((1u << t) - 1u)) * n + 2 * cci[k];
                const uint32_t top = sy[g][k] & 0xffu, bot = (sy[g][k] >> 8) & 0xffu;
                if (top) { atomicAdd(&hist[par][g][top], 1u); lastnz = (int32_t)ps; } else zeros++;
                if (bot) { atomicAdd(&hist[par][g][bot], 1u); lastnz = (int32_t)ps + 1; } else zeros++;
            }
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) zeros += __shfl_xor(zeros, o, 64);
            if (lane == 0 && zeros) atomicAdd(&s_zero[par][g], zeros);
            int32_t x = lastnz;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int32_t y = __shfl_up(x, o, 64);
                if ((int)lane >= o) x = max(x, y);
            }
            ex[g] = __shfl_up(x, 1, 64);
            if (lane == 0) ex[g] = -1;
            if (lane == 63) wmax[g][wave] = x;
        }
        __syncthreads();
        // the previous group's small statistics are read out: clear them
        if (tid < kPG * (3 + kNumWz)) {
            const uint32_t g = tid / (3 + kNumWz), f = tid % (3 + kNumWz);
            if (f == 0) s_zero[par ^ 1][g] = 0;
            else if (f == 1) s_zir[par ^ 1][g] = 0;
            else if (f == 2) s_pruns[par ^ 1][g] = 0;
            else s_dig[par ^ 1][g][f - 3] = 0;
        }
        // pass 2: runs terminated inside this thread (by a non-zero symbol
        // or the segment end), per-thread sums, then one atomic per wave
#pragma unroll
        for (int g = 0; g < kPG; g++) {
            if ((uint32_t)g >= gn) continue;
            const uint32_t b = gb[g];
            const uint32_t pm = ((pres[0] >> b) & 1u) | (((pres[1] >> b) & 1u) << 1) | (((pres[2] >> b) & 1u) << 2);
            const uint32_t M = n * __popc(pm);
            int32_t cur = ex[g];
            for (uint32_t w = 0; w < wave; w++) cur = max(cur, wmax[g][w]);
            uint32_t rz = 0, rn = 0;
#pragma unroll
            for (int k = 0; k < kCellsPT; k++) {
                if (!(sy[g][k] >> 16)) continue;
                const uint32_t t = ctype[k];
                const uint32_t ps0 = __popc(pm & ((1u << t) - 1u)) * n + 2 * cci[k];
#pragma unroll
                for (int h = 0; h < 2; h++) {
                    const uint32_t sv = h ? ((sy[g][k] >> 8) & 0xffu) : (sy[g][k] & 0xffu);
                    const int32_t ps = (int32_t)ps0 + h;
                    const bool endseg = (uint32_t)ps == M - 1;
                    if (sv || endseg) {
                        const int32_t L = sv ? (ps - cur - 1) : (ps - cur);
                        if (L >= 2) {
                            atomicAdd(&s_F[bitlen32((uint32_t)L)], 1u);
                            rz += (uint32_t)L;
                            rn++;
                            // digits beyond the first, for the widths whose base 2^w-1 < L
                            for (int i = 0; i < kNumWz && ((1u << (i + 2)) - 1u) < (uint32_t)L; i++)
                                atomicAdd(&s_dig[par][g][i], bij_digits((uint32_t)L, (1u << (i + 2)) - 1u) - 1u);
                        }
                        if (sv) cur = ps;
                    }
                }
            }
            if (__any(rn)) {
#pragma unroll
                for (int o = 32; o >= 1; o >>= 1) {
                    rz += __shfl_xor(rz, o, 64);
                    rn += __shfl_xor(rn, o, 64);
                }
                if (lane == 0 && rn) {
                    atomicAdd(&s_zir[par][g], rz);
                    atomicAdd(&s_pruns[par][g], rn);
                }
            }
        }
        __syncthreads();
        // write-out of the group: per plane the 256-bin histogram (bin 0 =
        // zero symbols), the run sums per counter width and the plane list
        for (uint32_t i = tid; i < gn * 256; i += kSymNT) {
            const uint32_t g = i >> 8, sidx = i & 255u;
            const uint32_t hv = sidx ? hist[par][g][sidx] : s_zero[par][g];
            seghist[(uint64_t)(B.slot + s_gb[par][g]) * 256 + sidx] = (uint16_t)hv;
            hist[par][g][sidx] = 0;
        }
        for (uint32_t i = tid; i < gn * kNumWz; i += kSymNT) {
            const uint32_t g = i / kNumWz, k = i % kNumWz;
            segstat[B.slot + s_gb[par][g]].dig[k] = s_dig[par][g][k] + s_pruns[par][g];
        }
        if (tid < gn) {
            const uint32_t b = s_gb[par][tid];
            segstat[B.slot + b].zir = s_zir[par][tid];
            P.seg_plane[nseg + tid] = (uint8_t)b;
            P.seg_M[nseg + tid] = n * (((pres[0] >> b) & 1u) + ((pres[1] >> b) & 1u) + ((pres[2] >> b) & 1u));
        }
        if (tid == 0)
            for (uint32_t g = 0; g < gn; g++) nruns += s_pruns[par][g];
        nseg += gn;
        par ^= 1u;
    }
    __syncthreads();
    if (tid < 16) S.F[tid] = s_F[tid];
    if (tid == 0) {
        S.nruns = nruns;
        S.err = err;
        P.d = d;
        P.nseg = nseg;
        P.p = p;
        P.n = n;
        P.err = err;
        for (uint32_t t = 0; t < 3; t++) P.masks[t] = (t < p) ? (~pres[t] & ((1u << d) - 1u)) : 0u;
    }
    }
}

// ---------------------------------------------------------------- Huffman
// Code lengths of the per-block Huffman code (Sec. 3 / Sec. 4): leaves with
// f > 0 sorted by (f, symbol); two-queue merge taking the leaf on equal
// weight; length = depth.  One wave per block, no workgroup barriers: lane l
// holds the symbols l, l + 64, l + 128 and l + 192; lanes hand values over
// through LDS with wave_sync.
//
// The merge runs in rounds.  With s the sum of the two smallest candidates
// (the next internal weight), every candidate of weight <= s precedes every
// internal node created from now on (leaves win ties, older internal nodes
// precede newer ones), so the sequential merge pairs these candidates two by
// two in their merged order before it looks at a new node: one round makes
// all floor(T/2) of those merges at once (T = candidates <= s).  This gives
// the same tree as the one-at-a-time merge; blocks take about ten rounds.
// A node is merged only in a round after the one that made it, so depths
// follow top-down, a round at a time from the last (whose one node is the
// root).

struct HuffW {
    uint32_t w[512];       // sorted leaf weights, then internal nodes in creation order
    uint16_t par[512];
    uint16_t srt[256];     // symbol of sorted leaf r
    uint16_t ord[512];     // a round's candidates in merged order
    uint16_t rfirst[256];  // first internal node of each round
    uint8_t dep[512];
};

// Ascending bitonic sort of 256 keys held as a[j] = element j * 64 + lane.
__device__ inline void wave_sort256(uint32_t (&a)[4])
{
    const uint32_t lane = threadIdx.x & 63;
#pragma unroll
    for (uint32_t k = 2; k <= 256; k <<= 1) {
#pragma unroll
        for (uint32_t d = k >> 1; d > 0; d >>= 1) {
            uint32_t o[4];
#pragma unroll
            for (int j = 0; j < 4; j++)
                o[j] = d >= 64 ? a[j ^ (int)(d >> 6)] : (uint32_t)__shfl_xor((int)a[j], (int)d, 64);
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const uint32_t i = (uint32_t)j * 64 + lane;
                const bool keep_min = ((i & d) == 0) == ((i & k) == 0);
                a[j] = keep_min ? min(a[j], o[j]) : max(a[j], o[j]);
            }
        }
    }
}

// The leaves with f > 0 in (f, symbol) order: S.srt, S.w.  Returns m.
__device__ inline uint32_t sort_leaves(const uint32_t *f, HuffW &S)
{
    const uint32_t lane = threadIdx.x & 63;
    uint32_t a[4], m = 0;
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const uint32_t s = (uint32_t)j * 64 + lane, fv = f[s];
        a[j] = fv ? (fv << 8) | s : 0xffffffffu;  // f < 2^24
        m += (uint32_t)__popcll(__ballot(fv > 0));
    }
    if (m <= 1) return m;
    wave_sort256(a);
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const uint32_t i = (uint32_t)j * 64 + lane;
        if (i < m) {
            S.srt[i] = (uint16_t)(a[j] & 0xffu);
            S.w[i] = a[j] >> 8;
        }
    }
    wave_sync();
    return m;
}

__device__ void huff_lengths(const uint32_t *f, uint8_t *len, HuffW &S)
{
    const uint32_t lane = threadIdx.x & 63;
    constexpr uint32_t INF = 0xffffffffu;
#pragma unroll
    for (int j = 0; j < 4; j++) len[j * 64 + lane] = 0;
    const uint32_t m = sort_leaves(f, S);
    if (m <= 1) { wave_sync(); return; }
    uint32_t qa = 0, qb = 0, ne = 0, nr = 0;  // leaf head, internal head, internal count, rounds
    while (ne + 1 < m) {
        // the two smallest candidates (leaf first on ties)
        const uint32_t x0 = qa < m ? S.w[qa] : INF, x1 = qa + 1 < m ? S.w[qa + 1] : INF;
        const uint32_t y0 = qb < ne ? S.w[m + qb] : INF, y1 = qb + 1 < ne ? S.w[m + qb + 1] : INF;
        uint32_t sum;
        if (x0 <= y0) sum = x0 + (x1 <= y0 ? x1 : y0);
        else sum = y0 + (x0 <= y1 ? x0 : y1);
        // candidates <= sum in each queue (both sorted)
        uint32_t cl = 0, ci = 0;
#pragma unroll
        for (int c = 0; c < 4; c++) {
            const uint32_t t = lane + 64u * c;
            cl += (uint32_t)__popcll(__ballot(qa + t < m && S.w[qa + t] <= sum));
            ci += (uint32_t)__popcll(__ballot(qb + t < ne && S.w[m + qb + t] <= sum));
        }
        const uint32_t T = cl + ci, P = T / 2;
        // merged order: a leaf goes before internal nodes of equal weight
#pragma unroll
        for (int c = 0; c < 4; c++) {
            const uint32_t t = lane + 64u * c;
            if (t < cl) {
                const uint32_t x = S.w[qa + t];
                uint32_t lo = 0, hi = ci;  // internal nodes < x
                while (lo < hi) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if (S.w[m + qb + mid] < x) lo = mid + 1; else hi = mid;
                }
                S.ord[t + lo] = (uint16_t)(qa + t);
            }
            if (t < ci) {
                const uint32_t y = S.w[m + qb + t];
                uint32_t lo = 0, hi = cl;  // leaves <= y
                while (lo < hi) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if (S.w[qa + mid] <= y) lo = mid + 1; else hi = mid;
                }
                S.ord[t + lo] = (uint16_t)(m + qb + t);
            }
        }
        wave_sync();
        if (lane == 0) S.rfirst[nr] = (uint16_t)(m + ne);
#pragma unroll
        for (int c = 0; c < 2; c++) {  // P <= 128
            const uint32_t t = lane + 64u * c;
            if (t < P) {
                const uint32_t a = S.ord[2 * t], b = S.ord[2 * t + 1];
                const uint32_t id = m + ne + t;
                S.w[id] = S.w[a] + S.w[b];
                S.par[a] = (uint16_t)id;
                S.par[b] = (uint16_t)id;
            }
        }
        // leaves among the consumed 2P candidates
        const uint32_t lastleaf = (T & 1u) ? (S.ord[T - 1] < m ? 1u : 0u) : 0u;
        wave_sync();
        const uint32_t nl = cl - lastleaf;
        qa += nl;
        qb += 2 * P - nl;
        ne += P;
        nr++;
    }
    // depths: the root (the last round's one node) at 0, then each earlier
    // round's nodes one below their parents
    if (lane == 0) S.dep[m + ne - 1] = 0;
    wave_sync();
    for (int r = (int)nr - 2; r >= 0; r--) {
        const uint32_t a = S.rfirst[r], b = S.rfirst[r + 1];
#pragma unroll
        for (int c = 0; c < 2; c++) {
            const uint32_t id = a + lane + 64u * c;
            if (id < b) S.dep[id] = (uint8_t)(S.dep[S.par[id]] + 1);
        }
        wave_sync();
    }
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const uint32_t i = (uint32_t)j * 64 + lane;
        if (i < m) len[S.srt[i]] = (uint8_t)(S.dep[S.par[i]] + 1);
    }
    wave_sync();
}

// Length-limited optimal code by package-merge (fallback when a seek-table
// entry of t bits cannot hold a segment length).  Lane 0 runs it; lengths
// are added level by level while backtracking the chosen items.
struct PMScratch {
    uint32_t wa[512], wb[512];
    uint32_t flag[16][16];  // per level: bit i = item i is a package
};

__device__ void package_merge_lengths(const uint32_t *f, int limit, uint8_t *len, HuffW &S, PMScratch &Q)
{
    const uint32_t lane = threadIdx.x & 63;
#pragma unroll
    for (int j = 0; j < 4; j++) len[j * 64 + lane] = 0;
    const uint32_t m = sort_leaves(f, S);
    if (m <= 1) { wave_sync(); return; }
    if (lane == 0) {
        uint32_t *prev = Q.wa, *cur = Q.wb;
        for (uint32_t i = 0; i < m; i++) prev[i] = S.w[i];
        uint32_t nprev = m;
        for (int lvl = 0; lvl < 16; lvl++)
            for (int i = 0; i < 16; i++) Q.flag[lvl][i] = 0;
        // level index j = limit (finest) ... 1; flags stored for j = 1..limit-1
        for (int j = limit - 1; j >= 1; j--) {
            uint32_t npk = nprev / 2, a = 0, b = 0, nc = 0;
            while (a < m || b < npk) {
                bool coin;
                uint32_t wpk = (b < npk) ? prev[2 * b] + prev[2 * b + 1] : 0;
                if (a >= m) coin = false;
                else if (b >= npk) coin = true;
                else coin = S.w[a] <= wpk;
                if (coin) { cur[nc] = S.w[a]; a++; }
                else { cur[nc] = wpk; Q.flag[j][nc >> 5] |= 1u << (nc & 31); b++; }
                nc++;
            }
            uint32_t *t = prev; prev = cur; cur = t; nprev = nc;
        }
        // backtrack from level 1: choose the first 2(m-1) items
        uint32_t take = 2 * (m - 1);
        for (int j = 1; j <= limit; j++) {
            uint32_t leaves = 0, pk = 0;
            for (uint32_t i = 0; i < take; i++) {
                bool isp = (j < limit) && ((Q.flag[j][i >> 5] >> (i & 31)) & 1u);
                if (isp) pk++; else leaves++;
            }
            for (uint32_t i = 0; i < leaves; i++) len[S.srt[i]]++;
            take = 2 * pk;
            if (!take) break;
        }
    }
    wave_sync();
}

// Canonical codes (RFC 1951 Sec. 3.2.2: by length, then symbol, counting
// up) and the leaf order, a length at a time: a symbol's rank among the
// symbols of its length is the count of those with a smaller index (ballots).
__device__ void canonical(const uint8_t *len, uint32_t *code, uint8_t *order)
{
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t lt = (1ull << lane) - 1ull;
    uint32_t l[4], cd[4] = {0, 0, 0, 0}, mx = 0;
#pragma unroll
    for (int j = 0; j < 4; j++) {
        l[j] = len[j * 64 + lane];
        mx = max(mx, l[j]);
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) mx = max(mx, (uint32_t)__shfl_xor((int)mx, o, 64));
    uint32_t first = 0, below = 0, prev = 0;
    for (uint32_t L = 1; L <= mx; L++) {
        first = (first + prev) << 1;  // first code of length L (0 for L = 1)
        uint32_t acc = 0;
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const uint64_t b = __ballot(l[j] == L);
            if (l[j] == L) {
                const uint32_t r = acc + (uint32_t)__popcll(b & lt);
                cd[j] = first + r;
                order[below + r] = (uint8_t)(j * 64 + lane);
            }
            acc += (uint32_t)__popcll(b);
        }
        below += acc;
        prev = acc;
    }
#pragma unroll
    for (int j = 0; j < 4; j++) code[j * 64 + lane] = cd[j];
}

struct CodeShared {
    uint32_t f[256];
    uint8_t len[256];
    uint32_t segbits[32];
    uint32_t plane[32];             // kept planes, segment order
    uint32_t zir[32];               // per segment: zeros inside runs
    uint16_t dig[32][kNumWz];       // per segment: run digits per counter width (< 8 * 3073)
    HuffW hs;
};

// Bits of every segment under the current code: symbol counts times code
// lengths, C_zr counted once per run digit plus once per literal C_zr.
__device__ void seg_lengths(CodeShared &C, const uint16_t *seghist, uint32_t slot, uint32_t nseg, uint32_t czr,
                            uint32_t wz)
{
    const uint32_t lane = threadIdx.x & 63;
    uint32_t cost[4];
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const uint32_t s = (uint32_t)j * 64 + lane;
        cost[j] = C.len[s] + (s == czr ? wz : 0u);
    }
    const uint32_t zcost = C.len[czr] + wz;
    uint32_t sg = 0;
    // four segments at a time: their 16 histogram loads in flight together,
    // their four wave sums interleaved
    for (; sg + 4 <= nseg; sg += 4) {
        uint32_t cnt[4][4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const uint16_t *h = seghist + (uint64_t)(slot + C.plane[sg + u]) * 256;
#pragma unroll
            for (int j = 0; j < 4; j++) cnt[u][j] = h[j * 64 + lane];
        }
        uint32_t add[4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            add[u] = 0;
#pragma unroll
            for (int j = 0; j < 4; j++) {
                uint32_t c = cnt[u][j];
                if (j == 0 && lane == 0) c -= C.zir[sg + u];
                add[u] += c * cost[j];
            }
            if (lane == 0) add[u] += C.dig[sg + u][wz - 2] * zcost;
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1)
#pragma unroll
            for (int u = 0; u < 4; u++) add[u] += __shfl_xor(add[u], o, 64);
        if (lane == 0)
#pragma unroll
            for (int u = 0; u < 4; u++) C.segbits[sg + u] = add[u];
    }
    for (; sg < nseg; sg++) {
        const uint16_t *h = seghist + (uint64_t)(slot + C.plane[sg]) * 256;
        uint32_t add = 0;
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const uint32_t s = (uint32_t)j * 64 + lane;
            uint32_t cnt = h[s];
            if (s == 0) cnt -= C.zir[sg];
            add += cnt * cost[j];
        }
        if (lane == 0) add += C.dig[sg][wz - 2] * zcost;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) add += __shfl_xor(add, o, 64);
        if (lane == 0) C.segbits[sg] = add;
    }
    wave_sync();
}

// One wave per block (12 per CU: 13.2 KB of LDS each), looping over the
// blocks of the grid.
__global__ void __launch_bounds__(64) k_enc_code(PlanHdr H, uint8_t *__restrict__ ws)
{
    __shared__ CodeShared C;
    __shared__ PMScratch Q;
    const uint32_t lane = threadIdx.x;
    for (uint32_t blk = blockIdx.x; blk < H.total_blocks; blk += gridDim.x) {
    wave_sync();
    const BlockDesc &B = ((const BlockDesc *)(ws + H.ws_blockdesc))[blk];
    BlkPlan &P = ((BlkPlan *)(ws + H.ws_blkplan))[blk];
    const BlkStat &S = ((const BlkStat *)(ws + H.ws_blkstat))[blk];
    const uint16_t *seghist = (const uint16_t *)(ws + H.ws_seghist);
    const SegStat *segstat = (const SegStat *)(ws + H.ws_segstat);
    const uint32_t nseg = P.nseg, d = P.d, p = P.p, n = P.n;
    const uint32_t tb = bitlen32(p * n) - 1 + 5;  // t = floor(log2(p w h / 8)) + 5
    if (nseg == 0) {
        if (lane == 0) {
            P.czr = 0; P.wz = 0; P.m = 0; P.tbits = tb; P.limited = 0;
            P.hdr_bits = 5 + p * d;
            P.bytes = (P.hdr_bits + 7) / 8;
        }
        continue;
    }
    // segment statistics to LDS
    const uint32_t slot = B.slot;
    if (lane < nseg) C.plane[lane] = P.seg_plane[lane];
    wave_sync();
    for (uint32_t i = lane; i < nseg * (kNumWz + 1); i += 64) {
        const uint32_t sg = i / (kNumWz + 1), k = i % (kNumWz + 1);
        const SegStat &st = segstat[slot + C.plane[sg]];
        if (k == kNumWz) C.zir[sg] = st.zir;
        else C.dig[sg][k] = (uint16_t)st.dig[k];
    }
    // block histogram
    uint32_t h[4] = {0, 0, 0, 0};
    {
        // four segments' loads in flight at a time
        uint32_t sg = 0;
        for (; sg + 4 <= nseg; sg += 4) {
            uint32_t v[4][4];
#pragma unroll
            for (int u = 0; u < 4; u++) {
                const uint16_t *hs = seghist + (uint64_t)(slot + C.plane[sg + u]) * 256;
#pragma unroll
                for (int j = 0; j < 4; j++) v[u][j] = hs[j * 64 + lane];
            }
#pragma unroll
            for (int u = 0; u < 4; u++)
#pragma unroll
                for (int j = 0; j < 4; j++) h[j] += v[u][j];
        }
        for (; sg < nseg; sg++) {
            const uint16_t *hs = seghist + (uint64_t)(slot + C.plane[sg]) * 256;
#pragma unroll
            for (int j = 0; j < 4; j++) h[j] += hs[j * 64 + lane];
        }
    }
    wave_sync();
    uint32_t Z = 0;
    for (uint32_t sg = 0; sg < nseg; sg++) Z += C.zir[sg];
    // C_zr: least frequent symbol, smallest value on ties (Sec. 4)
    uint64_t key = ~0ull;
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const uint64_t kj = ((uint64_t)h[j] << 8) | (uint32_t)(j * 64 + lane);
        key = kj < key ? kj : key;
    }
    for (int o = 32; o >= 1; o >>= 1) { uint64_t y = __shfl_xor(key, o, 64); key = y < key ? y : key; }
    const uint32_t czr = (uint32_t)(key & 0xff);
    uint32_t lit[4];
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const uint32_t s = (uint32_t)j * 64 + lane;
        lit[j] = h[j] - (s == 0 ? Z : 0u);
        C.f[s] = lit[j] + (s == czr ? S.nruns : 0u);
    }
    wave_sync();
    // provisional code (each run one C_zr token) -> l
    huff_lengths(C.f, C.len, C.hs);
    const uint32_t l = C.len[czr];
    // counter width: Eq. 3 as read, minimised over [2, max(2, beta)]; lane
    // w - 2 prices width w, smallest width on ties
    const uint32_t beta = bitlen32(p * n - 1);
    const uint32_t wzhi = beta > 2 ? beta : 2;
    uint32_t wz, D = 0;
    {
        const uint32_t w = lane + 2;
        uint64_t key2 = ~0ull;
        if (w <= wzhi) {
            uint64_t cost = 0;
            for (uint32_t i = 1; i < 16; i++) cost += (uint64_t)S.F[i] * ((i + w - 1) / w) * (w + l);
            key2 = (cost << 6) | lane;  // cost < 2^56: counts < 2^24, factors < 2^6 each
        }
        for (int o = 32; o >= 1; o >>= 1) { uint64_t y = __shfl_xor(key2, o, 64); key2 = y < key2 ? y : key2; }
        wz = (uint32_t)(key2 & 63u) + 2;
        for (uint32_t sg = 0; sg < nseg; sg++) D += C.dig[sg][wz - 2];
    }
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const uint32_t s = (uint32_t)j * 64 + lane;
        C.f[s] = lit[j] + (s == czr ? D : 0u);
    }
    wave_sync();
    huff_lengths(C.f, C.len, C.hs);
    seg_lengths(C, seghist, slot, nseg, czr, wz);
    // seek-table overflow -> length-limited fallback
    uint32_t limited = 0;
    if (__any(lane < nseg && C.segbits[lane] >= (1u << tb))) {
        package_merge_lengths(C.f, 14, C.len, C.hs, Q);
        seg_lengths(C, seghist, slot, nseg, czr, wz);
        limited = 1;
    }
    canonical(C.len, P.code, P.order);
    uint32_t m = 0;
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const uint32_t s = (uint32_t)j * 64 + lane;
        const bool has = C.f[s] > 0;
        m += (uint32_t)__popcll(__ballot(has));
        P.len[s] = C.len[s];
    }
#pragma unroll
    for (int j = 0; j < 4; j++)  // single leaf: code length 0
        if (m == 1 && C.f[j * 64 + lane] > 0) P.order[0] = (uint8_t)(j * 64 + lane);
    if (lane < nseg) P.seg_bits[lane] = C.segbits[lane];
    if (lane == 0) {
        uint32_t over = 0, sum = 0;
        for (uint32_t sg = 0; sg < nseg; sg++) { sum += C.segbits[sg]; over |= C.segbits[sg] >= (1u << tb); }
        P.czr = czr; P.wz = wz; P.m = m; P.tbits = tb; P.limited = limited;
        P.hdr_bits = 5 + p * d + 8 + 4 + (10 * m - 1) + nseg * tb;
        P.bytes = (P.hdr_bits + sum + 7) / 8;
        if (over) P.err = 2;
    }
    }
}

// ---------------------------------------------------------------- offsets
// Four consecutive blocks per thread and iteration: one workgroup scan per
// 1024 blocks.
constexpr uint32_t kPrepPT = 4;

__global__ void __launch_bounds__(256) k_enc_block_offsets(PlanHdr H, const uint8_t *__restrict__ plan,
                                                           uint8_t *__restrict__ ws)
{
    __shared__ uint64_t sh[8];
    const TileGeo &T = ((const TileGeo *)(plan + H.tiles_off))[blockIdx.x];
    BlkPlan *plans = (BlkPlan *)(ws + H.ws_blkplan);
    TileOut *to = (TileOut *)(ws + H.ws_tileout);
    uint64_t carry = 24 + 4ull * T.nblocks_stream;
    uint32_t err = 0;
    for (uint32_t base = 0; base < T.nblocks; base += 256 * kPrepPT) {
        const uint32_t l0 = base + threadIdx.x * kPrepPT;
        uint64_t sz[kPrepPT], own = 0;
#pragma unroll
        for (uint32_t k = 0; k < kPrepPT; k++) {
            sz[k] = 0;
            if (l0 + k < T.nblocks) {
                sz[k] = plans[T.block_base + l0 + k].bytes;
                err |= plans[T.block_base + l0 + k].err;
            }
            own += sz[k];
        }
        uint64_t tot;
        uint64_t ex = block_excl_sum_u64<256>(own, sh, &tot);
#pragma unroll
        for (uint32_t k = 0; k < kPrepPT; k++) {
            if (l0 + k < T.nblocks) plans[T.block_base + l0 + k].byte_off = carry + ex;
            ex += sz[k];
        }
        carry += tot;
    }
    err = __syncthreads_or(err);
    if (threadIdx.x == 0) {
        to[blockIdx.x].size = carry;
        to[blockIdx.x].status = err ? ISX_STATUS_UNSUP : ISX_STATUS_OK;
    }
}

__global__ void __launch_bounds__(1024) k_enc_tile_offsets(PlanHdr H, uint8_t *__restrict__ ws,
                                                           uint64_t capacity,
                                                           uint64_t *__restrict__ d_off,
                                                           uint64_t *__restrict__ d_size,
                                                           int32_t *__restrict__ d_status)
{
    __shared__ uint64_t sh[16];
    TileOut *to = (TileOut *)(ws + H.ws_tileout);
    uint64_t carry = 0;
    for (uint32_t base = 0; base < H.n_tiles; base += 1024) {
        uint32_t i = base + threadIdx.x;
        uint64_t sz = 0;
        if (i < H.n_tiles) sz = (to[i].size + 255) & ~255ull;
        uint64_t tot;
        uint64_t ex = block_excl_sum_u64<1024>(sz, sh, &tot);
        if (i < H.n_tiles) {
            uint64_t off = carry + ex;
            int32_t st = to[i].status;
            if (st == ISX_STATUS_OK && off + ((to[i].size + 3) & ~3ull) > capacity) st = ISX_STATUS_CAPACITY;
            to[i].offset = off;
            to[i].status = st;
            d_off[i] = off;
            d_size[i] = to[i].size;
            d_status[i] = st;
        }
        carry += tot;
    }
}

// Workgroups [0, n_tiles): tile header (little endian) + block size table.
// The rest, one wave per block: zero the words that the packers OR into --
// the first and last word of every block header and every segment
// (neighbouring regions share those words; all other words are written whole
// by exactly one packer).
__global__ void __launch_bounds__(256) k_enc_tile_finish(PlanHdr H, const uint8_t *__restrict__ plan,
                                                         const uint8_t *__restrict__ ws,
                                                         uint8_t *__restrict__ out)
{
    const BlkPlan *plans = (const BlkPlan *)(ws + H.ws_blkplan);
    const TileOut *tos = (const TileOut *)(ws + H.ws_tileout);
    if (blockIdx.x < H.n_tiles) {
        const TileGeo &T = ((const TileGeo *)(plan + H.tiles_off))[blockIdx.x];
        const TileOut &O = tos[blockIdx.x];
        if (O.status != ISX_STATUS_OK) return;
        uint32_t *w = (uint32_t *)(out + O.offset);
        uint32_t hdrw = 6 + T.nblocks_stream;
        for (uint32_t i = threadIdx.x; i < hdrw; i += blockDim.x) {
            uint32_t x = 0;
            if (i == 0) x = 0x31585349u;  // "ISX1"
            else if (i == 1) x = 1u | ((uint32_t)T.ct << 8) | ((uint32_t)T.channels << 16) | ((uint32_t)T.bits << 24);
            else if (i == 2) x = (uint32_t)T.bps | ((uint32_t)T.levels << 8) | ((uint32_t)T.qstep << 16);
            else if (i == 3) x = T.width;
            else if (i == 4) x = T.height;
            else if (i == 5) x = T.nblocks_stream;
            else x = plans[T.block_base + (i - 6)].bytes;
            w[i] = x;
        }
        return;
    }
    const uint32_t blk = (blockIdx.x - H.n_tiles) * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (blk >= H.total_blocks) return;
    const BlockDesc &B = ((const BlockDesc *)(ws + H.ws_blockdesc))[blk];
    const TileOut &O = tos[B.tile];
    if (O.status != ISX_STATUS_OK) return;
    const BlkPlan &P = plans[blk];
    uint32_t *w = (uint32_t *)(out + O.offset);
    const uint64_t a = P.byte_off * 8, e0 = a + P.hdr_bits;
    // segment s starts after the header and segments 0 .. s-1 (wave scan)
    const uint32_t nseg = P.nseg;
    const uint32_t nb = lane < nseg ? P.seg_bits[lane] : 0u;
    uint32_t x = nb;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if ((int)lane >= o) x += y;
    }
    const uint64_t st = e0 + (x - nb);
    if (nb) {
        w[st >> 5] = 0;
        w[(st + nb - 1) >> 5] = 0;
    }
    if (lane == 0) {
        w[a >> 5] = 0;
        w[(e0 - 1) >> 5] = 0;
    }
    // the byte padding after the last region
    const uint64_t eall = e0 + (uint64_t)__shfl(x, 63, 64);
    const uint64_t end = (P.byte_off + P.bytes) * 8;
    if (lane == 0 && end > eall) w[(end - 1) >> 5] = 0;
}

// ---------------------------------------------------------------- pack
// One workgroup per item (a block header, or one segment).  A segment is
// packed in rounds of 8 symbols per lane: the lanes' token bits are counted,
// scanned across the lanes, written into a staging area in LDS, and the
// round's complete words are stored to the stream; the last, partial word
// is carried into the next round.  The throughput form is one wave per item
// (rounds of 512 symbols, scans within the wave: the per-item cost of small
// segments is one wave's); a plan of few segments (one small tile) packs
// each with four waves (rounds of 2048 symbols, the waves' totals combined
// through LDS), so that its longest segment takes a quarter of the rounds.
constexpr uint32_t kPackK = 8;                    // symbols per lane and round
constexpr uint32_t kPackRound = 64 * kPackK;      // symbols per round
// Staging words of one round.  Per symbol at most one literal token (a code
// of at most 32 bits plus a counter of at most 13 bits, wz <= 13); a zero run
// is emitted at its end, at most 45 bits per two of its symbols, except the
// run that began in an earlier round (at most 8 digit tokens for runs of at
// most 6144 zeros); plus the carried partial word and the put's second word.
// Rounds of nw waves take nw times the symbols.
constexpr uint32_t pack_stage(int nw) { return (kPackRound * (uint32_t)nw * 45 + 8 * 45 + 31) / 32 + 3; }

__device__ inline void put_bits(uint32_t *st, uint32_t pos, uint32_t val, uint32_t nb)
{
    if (!nb) return;
    if (nb < 32) val &= (1u << nb) - 1u;
    uint32_t wi = pos >> 5, o = pos & 31u;
    uint64_t x = (uint64_t)val << (64u - nb - o);
    uint32_t hi = (uint32_t)(x >> 32), lo = (uint32_t)x;
    if (hi) atomicOr(&st[wi], hi);
    if (lo) atomicOr(&st[wi + 1], lo);
}

// Store staging words [0, n) at stream word w0 (big-endian).  The item's
// first word (when `first_shared`) and the word `last_shared` (when <= n-1)
// are shared with the neighbouring region and ORed in; every other word
// belongs to this item alone.
__device__ inline void store_words(const uint32_t *st, uint32_t n, uint64_t w0, bool first_shared,
                                   uint32_t last_shared, uint32_t *outw, uint32_t nt = 64)
{
    for (uint32_t i = threadIdx.x; i < n; i += nt) {
        const uint32_t v = st[i];
        if ((i == 0 && first_shared) || i == last_shared) {
            if (v) atomicOr(&outw[w0 + i], __builtin_bswap32(v));
        } else {
            outw[w0 + i] = __builtin_bswap32(v);
        }
    }
}

__device__ inline uint32_t wave_excl_sum(uint32_t v, uint32_t &total)
{
    const uint32_t lane = threadIdx.x & 63;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if ((int)lane >= o) x += y;
    }
    total = __shfl(x, 63, 64);
    return x - v;
}

__device__ inline int32_t wave_excl_max(int32_t v, int32_t &total)
{
    const uint32_t lane = threadIdx.x & 63;
    int32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t y = __shfl_up(x, o, 64);
        if ((int)lane >= o) x = max(x, y);
    }
    total = __shfl(x, 63, 64);
    const int32_t ex = __shfl_up(x, 1, 64);
    return lane == 0 ? INT32_MIN : ex;
}

template <int NW>
struct PackShared {
    uint32_t st[pack_stage(NW)];
    uint32_t code[256];
    uint8_t len[256];
    uint8_t cost[256];  // bits of a literal: its code, plus the counter for C_zr
    int32_t wmax[NW];   // per wave: its last non-zero position (NW > 1)
    uint32_t wsum[NW];  // per wave: its token bits (NW > 1)
};

// Exclusive max / sum over the NW waves' lanes in thread order, and the
// total; for NW > 1 through LDS at a barrier that every thread reaches.
template <int NW>
__device__ inline int32_t group_excl_max(int32_t v, int32_t &total, int32_t *sh)
{
    int32_t wt;
    const int32_t ex = wave_excl_max(v, wt);
    if (NW == 1) {
        total = wt;
        return ex;
    }
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) sh[wave] = wt;
    __syncthreads();
    int32_t before = INT32_MIN, all = INT32_MIN;
#pragma unroll
    for (int w = 0; w < NW; w++) {
        const int32_t x = sh[w];
        if ((uint32_t)w < wave) before = max(before, x);
        all = max(all, x);
    }
    total = all;
    return max(before, ex);
}
template <int NW>
__device__ inline uint32_t group_excl_sum(uint32_t v, uint32_t &total, uint32_t *sh)
{
    uint32_t wt;
    const uint32_t ex = wave_excl_sum(v, wt);
    if (NW == 1) {
        total = wt;
        return ex;
    }
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) sh[wave] = wt;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < NW; w++) {
        const uint32_t x = sh[w];
        if ((uint32_t)w < wave) before += x;
        all += x;
    }
    total = all;
    return before + ex;
}

// Item y of block blk: y = 0 the block header, y = 1.. segment y-1.  The
// longest items (the last segments: low, dense planes) come first in the
// grid, the headers last.
template <int NW>
__global__ void __launch_bounds__(64 * NW) k_enc_pack(PlanHdr H, const uint8_t *__restrict__ ws,
                                                      uint8_t *__restrict__ out)
{
    constexpr uint32_t NT = 64 * NW;
    __shared__ PackShared<NW> S;
    const uint32_t blk = blockIdx.x, y = gridDim.y - 1u - blockIdx.y;
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
    const BlockDesc &B = ((const BlockDesc *)(ws + H.ws_blockdesc))[blk];
    const BlkPlan &P = ((const BlkPlan *)(ws + H.ws_blkplan))[blk];
    const uint32_t nseg = __builtin_amdgcn_readfirstlane(P.nseg);
    if (y > nseg) return;
    const TileOut &O = ((const TileOut *)(ws + H.ws_tileout))[B.tile];
    if (__builtin_amdgcn_readfirstlane(O.status) != ISX_STATUS_OK) return;
    uint32_t *st = S.st;
    uint32_t *outw = (uint32_t *)out;
    const uint64_t bit0 = (O.offset + P.byte_off) * 8;
    const uint32_t hdr_bits = P.hdr_bits;
    if (y == 0) {
        // header: d | masks | C_zr | wz | tree | seek table (Fig. 3)
        const uint32_t o = (uint32_t)(bit0 & 31u);
        const uint32_t nw = (o + hdr_bits + 31) >> 5;
        for (uint32_t i = tid; i < nw + 1; i += NT) st[i] = 0;
        __syncthreads();
        const uint32_t d = P.d, p = P.p;
        if (tid == 0) {
            put_bits(st, o, d, 5);
            for (uint32_t t = 0; t < p; t++) put_bits(st, o + 5 + t * d, P.masks[t], d);
            if (nseg) {
                put_bits(st, o + 5 + p * d, P.czr, 8);
                put_bits(st, o + 13 + p * d, P.wz, 4);
            }
        }
        if (nseg && wave == 0) {
            // pre-order tree: leaf j (canonical order) is preceded by zj
            // internal-node zeros; lane takes leaves 4 lane .. 4 lane + 3
            const uint32_t tree0 = o + 17 + p * d;
            const uint32_t m = P.m;
            uint32_t z[4], sy[4], sum = 0;
#pragma unroll
            for (uint32_t k = 0; k < 4; k++) {
                const uint32_t j = 4 * lane + k;
                z[k] = 0; sy[k] = 0;
                if (j < m) {
                    const uint32_t sym = P.order[j], lj = P.len[sym];
                    if (j == 0) z[k] = lj;
                    else {
                        const uint32_t ps = P.order[j - 1];
                        z[k] = lj - P.len[ps] + (uint32_t)__builtin_ctz(~P.code[ps]);  // trailing ones
                    }
                    sy[k] = sym;
                    sum += z[k] + 9;
                }
            }
            uint32_t tot;
            uint32_t ex = wave_excl_sum(sum, tot);
#pragma unroll
            for (uint32_t k = 0; k < 4; k++) {
                if (4 * lane + k < m) {
                    put_bits(st, tree0 + ex + z[k], 0x100u | sy[k], 9);
                    ex += z[k] + 9;
                }
            }
            const uint32_t seek0 = tree0 + 10 * m - 1;
            if (lane < nseg) put_bits(st, seek0 + lane * P.tbits, P.seg_bits[lane], P.tbits);
        }
        __syncthreads();
        const uint32_t tail = ((o + hdr_bits) & 31u) ? nw - 1 : ~0u;
        store_words(st, nw, bit0 >> 5, o != 0, tail, outw, NT);
        return;
    }
    // segment s = y-1: it starts after the header and segments 0 .. s-1
    const uint32_t s = y - 1;
    const uint32_t czr = P.czr, wz = P.wz;
    const uint32_t M = P.seg_M[s];
    uint32_t start;
    {
        uint32_t t;
        (void)wave_excl_sum(lane < s ? P.seg_bits[lane & 31u] : 0u, t);
        start = hdr_bits + t;
    }
    const uint64_t abit = bit0 + start;
    const uint32_t o = (uint32_t)(abit & 31u);
    const uint64_t w0 = abit >> 5;
#pragma unroll
    for (uint32_t k = 0; k < 256 / NT; k++) {
        const uint32_t sy = tid + NT * k, lv = P.len[sy];
        S.code[sy] = P.code[sy];
        S.len[sy] = (uint8_t)lv;
        S.cost[sy] = (uint8_t)(lv + (sy == czr ? wz : 0u));
    }
    for (uint32_t i = tid; i < pack_stage(NW); i += NT) st[i] = 0;
    const uint8_t *syms = ws + B.sym_off + (uint64_t)P.seg_plane[s] * plane_stride(P.p * P.n);
    __syncthreads();
    const uint32_t Bb = (1u << wz) - 1u;
    const uint32_t lz = S.len[czr];
    const uint32_t tokz = lz + wz;
    const uint32_t len0 = S.len[0];
    const uint32_t lit0 = len0 + (czr == 0 ? wz : 0u);
    const uint32_t code0 = S.code[0], codez = S.code[czr];
    // nd(L) = 1 + #{k >= 1 : B + B^2 + ... + B^k < L}; 8 digits cover L <= 6144
    uint32_t thr[7];
    {
        uint64_t pw = Bb, t = Bb;
#pragma unroll
        for (int k = 0; k < 7; k++) {
            thr[k] = t > 0xffffffffull ? 0xffffffffu : (uint32_t)t;
            pw *= Bb;
            t += pw;
        }
    }
    int32_t cur = -1;     // position of the last non-zero symbol before the round
    uint32_t bp = o;      // bit position of the round's first token in the staging
    uint64_t wdone = 0;   // stream words stored so far (staging word 0 = stream word w0 + wdone)
    for (uint32_t r0 = 0; r0 < M; r0 += kPackRound * NW) {
        const uint32_t lo = r0 + kPackK * tid;
        const uint32_t hi = min(lo + kPackK, M);
        // 8 symbols of the lane (the plane stride is a multiple of 16 bytes,
        // so the 8-byte load stays in the plane); symbols >= hi read as 0
        uint2 q = make_uint2(0, 0);
        if (lo < M) q = *(const uint2 *)(syms + lo);
        if (hi - lo < 8 && lo < M) {
            const uint32_t nb = hi - lo;  // 1..7
            if (nb < 4) { q.x &= (1u << (8 * nb)) - 1u; q.y = 0; }
            else if (nb > 4) q.y &= (1u << (8 * (nb - 4))) - 1u;
            else q.y = 0;
        }
        int32_t lastnz = -1;
        if (q.y) lastnz = (int32_t)(lo + 4 + (31u - (uint32_t)__builtin_clz(q.y)) / 8u);
        else if (q.x) lastnz = (int32_t)(lo + (31u - (uint32_t)__builtin_clz(q.x)) / 8u);
        int32_t mx;
        const int32_t prev = max(cur, group_excl_max<NW>(lastnz, mx, S.wmax));
#define LOC(i) ((((i) < 4 ? q.x : q.y) >> (8 * ((i) & 3))) & 0xffu)
        // token bits: a symbol that ends a zero run (non-zero, or the
        // segment's last) emits the run (one zero literal for length 1, else
        // nd(L) digit tokens) and then itself when non-zero.  Symbols past
        // the segment read as 0 and end nothing.  nd(L) is 1 up to L = B
        // (most runs); the longer ones count their thresholds.
        uint32_t bits = 0;
        {
            int32_t c = prev;
#pragma unroll
            for (uint32_t i = 0; i < kPackK; i++) {
                const uint32_t v = LOC(i);
                const int32_t ps = (int32_t)(lo + i);
                const bool nz = v != 0;
                const int32_t L = nz ? (ps - c - 1) : ((uint32_t)ps == M - 1 ? ps - c : 0);
                if (L > 0) {
                    uint32_t nd = 1;
                    if ((uint32_t)L > thr[0]) {
                        nd = 2;
#pragma unroll
                        for (int k = 1; k < 7; k++) nd += thr[k] < (uint32_t)L;
                    }
                    bits += L == 1 ? lit0 : nd * tokz;
                }
                if (nz) bits += S.cost[v];
                c = nz ? ps : c;
            }
        }
        uint32_t rbits;
        const uint32_t off = group_excl_sum<NW>(bits, rbits, S.wsum);
        {
            uint32_t b = bp + off;
            int32_t c = prev;
#pragma unroll
            for (uint32_t i = 0; i < kPackK; i++) {
                const uint32_t v = LOC(i);
                const int32_t ps = (int32_t)(lo + i);
                const bool nz = v != 0;
                const int32_t L = nz ? (ps - c - 1) : ((uint32_t)ps == M - 1 ? ps - c : 0);
                c = nz ? ps : c;
                if (L == 1) {
                    put_bits(st, b, code0, len0);  // literal zero (counter 0 when it is C_zr)
                    b += lit0;
                } else if (L >= 2) {
                    // bijective base-(2^wz - 1) digits, most significant first
                    uint32_t dg[8], nd = 0, x = (uint32_t)L;
                    while (x > 0 && nd < 8) { uint32_t qq = (x - 1) / Bb; dg[nd++] = x - qq * Bb; x = qq; }
                    for (int k = (int)nd - 1; k >= 0; k--) {
                        put_bits(st, b, codez, lz);
                        put_bits(st, b + lz, dg[k], wz);
                        b += tokz;
                    }
                }
                if (nz) {
                    const uint32_t lv = S.len[v];
                    put_bits(st, b, S.code[v], lv);
                    b += lv + (v == czr ? wz : 0u);
                }
            }
        }
#undef LOC
        __syncthreads();
        // the round's complete words go out; the partial one is carried
        const uint32_t end = bp + rbits;
        const uint32_t nfull = end >> 5;
        store_words(st, nfull, w0 + wdone, wdone == 0 && o != 0, ~0u, outw, NT);
        __syncthreads();
        const uint32_t carry = st[nfull];
        const uint32_t used = (end + 63) >> 5;  // words the round may have touched
        for (uint32_t i = tid; i < used; i += NT) st[i] = 0;
        __syncthreads();
        if (tid == 0) st[0] = carry;
        __syncthreads();
        bp = end & 31u;
        wdone += nfull;
        cur = max(cur, mx);
    }
    // the segment's last, partial word is shared with what follows it
    if (bp && tid == 0 && st[0]) atomicOr(&outw[w0 + wdone], __builtin_bswap32(st[0]));
}

// ---------------------------------------------------------------- launch
hipError_t launch_forward_level(const PlanHdr &H, const uint8_t *d_plan, const uint8_t *d_pixels,
                                uint8_t *d_ws, int level, hipStream_t stream);

hipError_t launch_forward_only(const PlanHdr &H, const uint8_t *d_plan, const uint8_t *d_pixels,
                               uint8_t *d_ws, hipStream_t stream)
{
    return launch_encode(H, d_plan, d_pixels, nullptr, 0, nullptr, nullptr, nullptr, d_ws, stream,
                         ENC_PREP, ENC_FWD0 + kMaxLevels);
}

// Stages (in order): prep, forward levels 0..15, symbols, code, block
// offsets, tile offsets, tile finish, pack.  Stages without work launch nothing.
hipError_t launch_encode(const PlanHdr &H, const uint8_t *d_plan, const uint8_t *d_pixels,
                         uint8_t *d_out, uint64_t out_capacity, uint64_t *d_tile_offsets,
                         uint64_t *d_tile_sizes, int32_t *d_status, uint8_t *d_ws,
                         hipStream_t stream, int first, int last)
{
    for (int st = first; st <= last; st++) {
        if (st == ENC_PREP) {
            if (H.max_nblocks > 512)
                hipLaunchKernelGGL(k_prep_blocks<1024>, dim3(H.n_tiles), dim3(1024), 0, stream, H, d_plan, d_ws);
            else
                hipLaunchKernelGGL(k_prep_blocks<256>, dim3(H.n_tiles), dim3(256), 0, stream, H, d_plan, d_ws);
        } else if (st >= ENC_FWD0 && st <= ENC_FWD0 + kMaxLevels) {
            hipError_t e = launch_forward_level(H, d_plan, d_pixels, d_ws, st - ENC_FWD0, stream);
            if (e != hipSuccess) return e;
        } else if (st == ENC_SYM) {
            if (H.pack_nw == 4 && H.n_big + H.n_small) {
                // a plan of few blocks: all of them in one launch (a second
                // launch for the small blocks would add its whole latency)
                hipLaunchKernelGGL(k_enc_symbols<1024>, dim3(H.n_big + H.n_small), dim3(1024), 0, stream, H, d_plan,
                                   d_ws, 0u, H.n_big + H.n_small);
            } else {
                if (H.n_big) {
                    uint32_t g = H.blocks_per_cu ? std::min<uint32_t>(H.n_big, H.num_cus * H.blocks_per_cu) : H.n_big;
                    hipLaunchKernelGGL(k_enc_symbols<1024>, dim3(g), dim3(1024), 0, stream, H, d_plan, d_ws, 0u,
                                       H.n_big);
                }
                if (H.n_small) {
                    uint32_t g =
                        H.blocks_per_cu ? std::min<uint32_t>(H.n_small, H.num_cus * H.blocks_per_cu * 4) : H.n_small;
                    hipLaunchKernelGGL(k_enc_symbols<256>, dim3(g), dim3(256), 0, stream, H, d_plan, d_ws, H.n_big,
                                       H.n_small);
                }
            }
        } else if (st == ENC_CODE) {
            if (H.total_blocks) hipLaunchKernelGGL(k_enc_code, dim3(H.blk_grid), dim3(64), 0, stream, H, d_ws);
        } else if (st == ENC_BOFF) {
            hipLaunchKernelGGL(k_enc_block_offsets, dim3(H.n_tiles), dim3(256), 0, stream, H, d_plan, d_ws);
        } else if (st == ENC_TOFF) {
            hipLaunchKernelGGL(k_enc_tile_offsets, dim3(1), dim3(1024), 0, stream, H, d_ws, out_capacity,
                               d_tile_offsets, d_tile_sizes, d_status);
        } else if (st == ENC_FIN) {
            hipLaunchKernelGGL(k_enc_tile_finish, dim3(H.n_tiles + (H.total_blocks + 3) / 4), dim3(256), 0, stream, H,
                               d_plan, d_ws, d_out);
        } else if (st == ENC_PACK) {
            // item y = 0 is the header, y = 1 .. nseg the segments; nseg <= d <= the tile's plane bound
            if (H.total_blocks && H.pack_nw == 4)
                hipLaunchKernelGGL(k_enc_pack<4>, dim3(H.total_blocks, H.max_dmax + 1), dim3(256), 0, stream, H, d_ws,
                                   d_out);
            else if (H.total_blocks)
                hipLaunchKernelGGL(k_enc_pack<1>, dim3(H.total_blocks, H.max_dmax + 1), dim3(64), 0, stream, H, d_ws,
                                   d_out);
        }
    }
    return hipGetLastError();
}

// Debug: Huffman lengths of one frequency table, as the block coder builds them.
__global__ void __launch_bounds__(64) k_debug_huffman(const uint32_t *freq, int limit, uint8_t *out)
{
    __shared__ uint32_t f[256];
    __shared__ uint8_t len[256];
    __shared__ HuffW hs;
    __shared__ PMScratch q;
    for (int j = 0; j < 4; j++) f[j * 64 + threadIdx.x] = freq[j * 64 + threadIdx.x];
    wave_sync();
    if (limit <= 0) huff_lengths(f, len, hs);
    else package_merge_lengths(f, limit, len, hs, q);
    for (int j = 0; j < 4; j++) out[j * 64 + threadIdx.x] = len[j * 64 + threadIdx.x];
}

hipError_t launch_debug_huffman(const uint32_t *d_freq, int limit, uint8_t *d_len, hipStream_t stream)
{
    hipLaunchKernelGGL(k_debug_huffman, dim3(1), dim3(64), 0, stream, d_freq, limit, d_len);
    return hipGetLastError();
}

}  // namespace isx
