/*
 * isx_oracle.c -- plain, slow, scalar CPU reference of the codec in
 * "Fast Compression Method for Medical Images on the Web" (Hulsken, 2020).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The product path (the
 * HIP library) never calls it and shares no code, header or table with it.
 *
 * The paper leaves many details open (its figures and MATLAB code are not
 * available); every reading taken here is marked "Reading:" at the place it
 * is used.  What is computed, stage by stage (Sec. 3 Fig. 1, Sec. 4):
 *
 *   pixels -> reversible colour transform (Sec. 3: optional; Sec. 4:
 *   named as a standard stage and not specified)
 *   -> recursive 2-D 5/3 Le Gall integer lifting (Sec. 4)
 *   -> quantisation of the high-pass bands (Sec. 3, JPEG2000-style)
 *   -> 128x128 coefficient blocks (Sec. 4; Fig. 3 caption)
 *   -> signed-magnitude bitplanes, 4x2 areas in snake order (Sec. 4 Eq. 1)
 *   -> one byte symbol per area (Sec. 4 Eq. 2)
 *   -> empty-bitplane removal with per-type masks, zero-run coding with the
 *      least frequent symbol and an optimised counter width (Sec. 4 Eq. 3)
 *   -> per-block Huffman code (Sec. 3; Sec. 4), counters raw big-endian
 *   -> block header with masks, tree and seek table (Fig. 3 caption).
 *
 * Parity status per function is stated in its comment ("pinned by ...").
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* status codes of the oracle (its own numbering; same meaning as the  */
/* library's, written twice on purpose)                                 */
#define OR_OK 0
#define OR_E_INVALID (-1)
#define OR_E_CAPACITY (-2)
#define OR_E_CORRUPT (-3)
#define OR_E_TRUNCATED (-4)
#define OR_E_UNSUPPORTED (-5)
#define OR_E_NOMEM (-6)

#define OR_BLOCK 128      /* Sec. 4: wavelet data partitioned in 128*128 blocks */
#define OR_MAX_LEVELS 15
#define OR_MAX_CHANNELS 64
#define OR_LIMITED_LEN 14 /* length limit of the fallback code (seek-table overflow) */

/* floor(a / b) for b > 0, written out (C division truncates toward zero). */
static int64_t floor_div(int64_t a, int64_t b)
{
    int64_t q = a / b;
    if ((a % b) != 0 && a < 0) q -= 1;
    return q;
}

static int bit_length(uint64_t v)
{
    int n = 0;
    while (v) { n++; v >>= 1; }
    return n;
}

static int roundup4(int v) { return (v + 3) / 4 * 4; }

/* ================================================================== */
/* Colour transform.  Reading: the paper only says the stage is optional */
/* and standard (Sec. 3, Sec. 4); the reversible component transform of  */
/* JPEG2000 lineage the paper compares to is used:                       */
/*   Y = floor((R + 2G + B) / 4),  Cb = B - G,  Cr = R - G               */
/* and its exact inverse G = Y - floor((Cb + Cr)/4), R = Cr + G,         */
/* B = Cb + G.  Pinned by: exhaustive inverse(forward) over all RGB8     */
/* triples, gray -> (v,0,0), hand-worked values.                          */
/* ================================================================== */
void oracle_rct_forward(int32_t r, int32_t g, int32_t b, int32_t out[3])
{
    out[0] = (int32_t)floor_div((int64_t)r + 2 * (int64_t)g + b, 4);
    out[1] = b - g;
    out[2] = r - g;
}

void oracle_rct_inverse(int32_t y, int32_t cb, int32_t cr, int32_t out[3])
{
    int32_t g = y - (int32_t)floor_div((int64_t)cb + cr, 4);
    out[0] = cr + g; /* R */
    out[1] = g;      /* G */
    out[2] = cb + g; /* B */
}

/* ================================================================== */
/* Alternative reversible colour transform (the generality row of the   */
/* build: the paper asks for arbitrary channels and bit depths; Sec. 3  */
/* leaves the colour transform open).  Reading: YCoCg-R, the lifting    */
/* form of YCoCg, exactly reversible in integers:                        */
/*   Co = R - B, t = B + floor(Co/2), Cg = G - t, Y = t + floor(Cg/2)    */
/* inverse: t = Y - floor(Cg/2), G = Cg + t, B = t - floor(Co/2),        */
/* R = B + Co.  Stream channel order Y, Co, Cg.  Pinned by: exhaustive   */
/* inverse(forward) over all RGB8 triples, hand-worked values, and its   */
/* relation to the real YCoCg matrix (Y within 1 of R/4 + G/2 + B/4).    */
/* ================================================================== */
void oracle_ycocg_forward(int32_t r, int32_t g, int32_t b, int32_t out[3])
{
    int32_t co = r - b;
    int32_t t = b + (int32_t)floor_div(co, 2);
    int32_t cg = g - t;
    out[0] = t + (int32_t)floor_div(cg, 2);
    out[1] = co;
    out[2] = cg;
}

void oracle_ycocg_inverse(int32_t y, int32_t co, int32_t cg, int32_t out[3])
{
    int32_t t = y - (int32_t)floor_div(cg, 2);
    int32_t g = cg + t;
    int32_t b = t - (int32_t)floor_div(co, 2);
    out[0] = b + co; /* R */
    out[1] = g;      /* G */
    out[2] = b;      /* B */
}

int64_t oracle_ycocg_selftest_u8(void)
{
    int64_t bad = 0;
    for (int r = 0; r < 256; r++)
        for (int g = 0; g < 256; g++)
            for (int b = 0; b < 256; b++) {
                int32_t f[3], v[3];
                oracle_ycocg_forward(r, g, b, f);
                oracle_ycocg_inverse(f[0], f[1], f[2], v);
                if (v[0] != r || v[1] != g || v[2] != b) bad++;
            }
    return bad;
}

/* Exhaustive inverse(forward) check over all 2^24 RGB8 triples; returns the
 * number of triples that do not round-trip. */
int64_t oracle_rct_selftest_u8(void)
{
    int64_t bad = 0;
    for (int r = 0; r < 256; r++)
        for (int g = 0; g < 256; g++)
            for (int b = 0; b < 256; b++) {
                int32_t f[3], v[3];
                oracle_rct_forward(r, g, b, f);
                oracle_rct_inverse(f[0], f[1], f[2], v);
                if (v[0] != r || v[1] != g || v[2] != b) bad++;
            }
    return bad;
}

/* ================================================================== */
/* 1-D 5/3 Le Gall integer lifting (Sec. 4 names the MATLAB 5/3 integer */
/* lifting).  Reading (MATLAB's exact code is not available): the       */
/* reversible 5/3 of JPEG2000 with whole-sample symmetric extension:     */
/*   d[n] = x[2n+1] - floor((x[2n] + x[2n+2]) / 2)                       */
/*   s[n] = x[2n]   + floor((d[n-1] + d[n] + 2) / 4)                     */
/* with x[N] := x[N-2], d[-1] := d[0] and, for odd N, the missing last   */
/* d[(N-1)/2] := d[(N-3)/2].  Low band = even samples (ceil(N/2)),       */
/* high band = odd samples (floor(N/2)); N = 1 passes x[0] to the low    */
/* band.  Pinned by: perfect reconstruction, and agreement within the   */
/* rounding bound with the real-valued Le Gall analysis filters          */
/* (-1,2,6,2,-1)/8 and (-1,2,-1)/2 on a symmetrically extended signal.  */
/* ================================================================== */
void oracle_lift53_forward_1d(const int32_t *x, int32_t n, int32_t *low, int32_t *high)
{
    int nl = (n + 1) / 2, nh = n / 2;
    if (n <= 0) return;
    if (n == 1) { low[0] = x[0]; return; }
    /* predict step: high band */
    for (int k = 0; k < nh; k++) {
        int64_t left = x[2 * k];
        int64_t right = (2 * k + 2 < n) ? x[2 * k + 2] : x[n - 2]; /* x[N] := x[N-2] */
        high[k] = (int32_t)(x[2 * k + 1] - floor_div(left + right, 2));
    }
    /* update step: low band */
    for (int k = 0; k < nl; k++) {
        int64_t dm1 = (k - 1 >= 0) ? high[k - 1] : high[0];    /* d[-1] := d[0] */
        int64_t d0 = (k < nh) ? high[k] : high[nh - 1];         /* odd N: missing last d */
        low[k] = (int32_t)(x[2 * k] + floor_div(dm1 + d0 + 2, 4));
    }
}

void oracle_lift53_inverse_1d(const int32_t *low, const int32_t *high, int32_t n, int32_t *x)
{
    int nl = (n + 1) / 2, nh = n / 2;
    if (n <= 0) return;
    if (n == 1) { x[0] = low[0]; return; }
    /* undo the update step: even samples */
    for (int k = 0; k < nl; k++) {
        int64_t dm1 = (k - 1 >= 0) ? high[k - 1] : high[0];
        int64_t d0 = (k < nh) ? high[k] : high[nh - 1];
        x[2 * k] = (int32_t)(low[k] - floor_div(dm1 + d0 + 2, 4));
    }
    /* undo the predict step: odd samples */
    for (int k = 0; k < nh; k++) {
        int64_t left = x[2 * k];
        int64_t right = (2 * k + 2 < n) ? x[2 * k + 2] : x[n - 2];
        x[2 * k + 1] = (int32_t)(high[k] + floor_div(left + right, 2));
    }
}

/* ================================================================== */
/* One 2-D level (Sec. 4; Sec. 3: the wavelet transform is recursive).  */
/* Reading: rows first, then columns (the order is not in the paper).   */
/* Subbands of a w x h input: LL ceil(w/2) x ceil(h/2); HL (horizontal  */
/* high, vertical low) floor(w/2) x ceil(h/2); LH ceil(w/2) x floor(h/2);*/
/* HH floor(w/2) x floor(h/2).  Outputs are dense row-major arrays.     */
/* ================================================================== */
static int dwt2_forward_level(const int32_t *src, int w, int h,
                              int32_t *ll, int32_t *hl, int32_t *lh, int32_t *hh)
{
    int wl = (w + 1) / 2, wh = w / 2, hl_ = (h + 1) / 2, hh_ = h / 2;
    int32_t *rows = (int32_t *)malloc(sizeof(int32_t) * (size_t)w * h);
    int32_t *line = (int32_t *)malloc(sizeof(int32_t) * (size_t)(w > h ? w : h));
    int32_t *lo = (int32_t *)malloc(sizeof(int32_t) * (size_t)(w > h ? w : h));
    int32_t *hi = (int32_t *)malloc(sizeof(int32_t) * (size_t)(w > h ? w : h) + 4);
    if (!rows || !line || !lo || !hi) { free(rows); free(line); free(lo); free(hi); return OR_E_NOMEM; }
    /* horizontal pass: each row -> [low | high] */
    for (int y = 0; y < h; y++) {
        for (int x = 0; x < w; x++) line[x] = src[(size_t)y * w + x];
        oracle_lift53_forward_1d(line, w, lo, hi);
        for (int x = 0; x < wl; x++) rows[(size_t)y * w + x] = lo[x];
        for (int x = 0; x < wh; x++) rows[(size_t)y * w + wl + x] = hi[x];
    }
    /* vertical pass: each column -> [low ; high] */
    for (int x = 0; x < w; x++) {
        for (int y = 0; y < h; y++) line[y] = rows[(size_t)y * w + x];
        oracle_lift53_forward_1d(line, h, lo, hi);
        for (int y = 0; y < hl_; y++) {
            if (x < wl) ll[(size_t)y * wl + x] = lo[y];
            else hl[(size_t)y * wh + (x - wl)] = lo[y];
        }
        for (int y = 0; y < hh_; y++) {
            if (x < wl) lh[(size_t)y * wl + x] = hi[y];
            else hh[(size_t)y * wh + (x - wl)] = hi[y];
        }
    }
    free(rows); free(line); free(lo); free(hi);
    return OR_OK;
}

/* Inverse of one 2-D level: columns first, then rows. */
static int dwt2_inverse_level(const int32_t *ll, const int32_t *hl, const int32_t *lh,
                              const int32_t *hh, int w, int h, int32_t *dst)
{
    int wl = (w + 1) / 2, wh = w / 2, hl_ = (h + 1) / 2, hh_ = h / 2;
    int32_t *rows = (int32_t *)malloc(sizeof(int32_t) * (size_t)w * h);
    int m = (w > h ? w : h);
    int32_t *line = (int32_t *)malloc(sizeof(int32_t) * (size_t)m);
    int32_t *lo = (int32_t *)malloc(sizeof(int32_t) * (size_t)m);
    int32_t *hi = (int32_t *)malloc(sizeof(int32_t) * (size_t)m + 4);
    if (!rows || !line || !lo || !hi) { free(rows); free(line); free(lo); free(hi); return OR_E_NOMEM; }
    for (int x = 0; x < w; x++) {
        for (int y = 0; y < hl_; y++)
            lo[y] = (x < wl) ? ll[(size_t)y * wl + x] : hl[(size_t)y * wh + (x - wl)];
        for (int y = 0; y < hh_; y++)
            hi[y] = (x < wl) ? lh[(size_t)y * wl + x] : hh[(size_t)y * wh + (x - wl)];
        oracle_lift53_inverse_1d(lo, hi, h, line);
        for (int y = 0; y < h; y++) rows[(size_t)y * w + x] = line[y];
    }
    for (int y = 0; y < h; y++) {
        for (int x = 0; x < wl; x++) lo[x] = rows[(size_t)y * w + x];
        for (int x = 0; x < wh; x++) hi[x] = rows[(size_t)y * w + wl + x];
        oracle_lift53_inverse_1d(lo, hi, w, line);
        for (int x = 0; x < w; x++) dst[(size_t)y * w + x] = line[x];
    }
    free(rows); free(line); free(lo); free(hi);
    return OR_OK;
}

/* ================================================================== */
/* Per-channel coefficient pyramid.                                    */
/* ================================================================== */
typedef struct {
    int w, h;
    int32_t *v; /* dense row-major, w*h */
} Band;

typedef struct {
    int levels;
    int w0, h0;                 /* channel size */
    Band ll;                    /* coarsest LL (LL_levels) */
    Band hl[OR_MAX_LEVELS + 1]; /* index 1..levels */
    Band lh[OR_MAX_LEVELS + 1];
    Band hh[OR_MAX_LEVELS + 1];
} Pyramid;

static void band_free(Band *b) { free(b->v); b->v = NULL; }

static int band_alloc(Band *b, int w, int h)
{
    b->w = w; b->h = h;
    b->v = (int32_t *)calloc((size_t)(w > 0 ? w : 1) * (size_t)(h > 0 ? h : 1), sizeof(int32_t));
    return b->v ? OR_OK : OR_E_NOMEM;
}

static void pyramid_free(Pyramid *p)
{
    band_free(&p->ll);
    for (int l = 1; l <= OR_MAX_LEVELS; l++) { band_free(&p->hl[l]); band_free(&p->lh[l]); band_free(&p->hh[l]); }
}

/* level-l subband sizes: LL_{l-1} is (w, h) */
static void level_sizes(int w0, int h0, int l, int *w, int *h)
{
    int a = w0, b = h0;
    for (int i = 1; i < l; i++) { a = (a + 1) / 2; b = (b + 1) / 2; }
    *w = a; *h = b;
}

/* Recursive forward transform of one channel plane (Sec. 3: recursive). */
static int pyramid_forward(const int32_t *plane, int w, int h, int levels, Pyramid *p)
{
    memset(p, 0, sizeof(*p));
    p->levels = levels; p->w0 = w; p->h0 = h;
    int cw = w, ch = h;
    int32_t *cur = (int32_t *)malloc(sizeof(int32_t) * (size_t)w * h);
    if (!cur) return OR_E_NOMEM;
    memcpy(cur, plane, sizeof(int32_t) * (size_t)w * h);
    for (int l = 1; l <= levels; l++) {
        int wl = (cw + 1) / 2, wh = cw / 2, hl_ = (ch + 1) / 2, hh_ = ch / 2;
        int32_t *nxt = (int32_t *)malloc(sizeof(int32_t) * (size_t)wl * hl_);
        if (!nxt || band_alloc(&p->hl[l], wh, hl_) || band_alloc(&p->lh[l], wl, hh_) ||
            band_alloc(&p->hh[l], wh, hh_)) { free(nxt); free(cur); return OR_E_NOMEM; }
        int rc = dwt2_forward_level(cur, cw, ch, nxt, p->hl[l].v, p->lh[l].v, p->hh[l].v);
        free(cur);
        if (rc) { free(nxt); return rc; }
        cur = nxt; cw = wl; ch = hl_;
    }
    p->ll.w = cw; p->ll.h = ch; p->ll.v = cur;
    return OR_OK;
}

/* Inverse from the coarsest level down to level z: returns LL_z (caller frees). */
static int32_t *pyramid_inverse(const Pyramid *p, int z, int *ow, int *oh)
{
    int cw = p->ll.w, ch = p->ll.h;
    int32_t *cur = (int32_t *)malloc(sizeof(int32_t) * (size_t)cw * ch);
    if (!cur) return NULL;
    memcpy(cur, p->ll.v, sizeof(int32_t) * (size_t)cw * ch);
    for (int l = p->levels; l > z; l--) {
        int w, h;
        level_sizes(p->w0, p->h0, l, &w, &h);
        int32_t *nxt = (int32_t *)malloc(sizeof(int32_t) * (size_t)w * h);
        if (!nxt) { free(cur); return NULL; }
        if (dwt2_inverse_level(cur, p->hl[l].v, p->lh[l].v, p->hh[l].v, w, h, nxt)) {
            free(nxt); free(cur); return NULL;
        }
        free(cur);
        cur = nxt; cw = w; ch = h;
    }
    *ow = cw; *oh = ch;
    return cur;
}

/* ================================================================== */
/* Quantisation (Sec. 3: lossy images use the quantisation of JPEG2000). */
/* Reading: dead-zone scalar quantiser with step D on the               */
/* HL, LH and HH bands of every level (LL always D = 1):                 */
/*   q = sign(c) floor(|c| / D);  c' = 0 if q = 0 else                   */
/*   sign(q) (|q| D + floor(D/2)).  D = 1 is the identity.               */
/* ================================================================== */
static int32_t quantise(int32_t c, int32_t step)
{
    if (step <= 1) return c;
    int64_t a = c < 0 ? -(int64_t)c : c;
    int64_t q = a / step;
    return (int32_t)(c < 0 ? -q : q);
}

static int32_t dequantise(int32_t q, int32_t step)
{
    if (step <= 1 || q == 0) return q;
    int64_t a = q < 0 ? -(int64_t)q : q;
    int64_t r = a * step + step / 2;
    return (int32_t)(q < 0 ? -r : r);
}

/* The two maps above, exported for their pins (worked values and the
 * midpoint property of the reconstruction). */
int32_t oracle_quantise(int32_t c, int32_t step) { return quantise(c, step); }
int32_t oracle_dequantise(int32_t q, int32_t step) { return dequantise(q, step); }

/* ================================================================== */
/* MSB-first bit writer / reader (Fig. 3 caption: fields are not byte    */
/* aligned; Sec. 4: counters stored big-endian).                         */
/* ================================================================== */
typedef struct {
    uint8_t *buf;
    uint64_t cap_bits;
    uint64_t pos;
    int overflow;
} BitWriter;

static void bw_put(BitWriter *w, uint64_t value, int nbits)
{
    for (int i = nbits - 1; i >= 0; i--) {
        int bit = (int)((value >> i) & 1u);
        if (w->pos >= w->cap_bits) { w->overflow = 1; return; }
        if (bit) w->buf[w->pos >> 3] |= (uint8_t)(0x80u >> (w->pos & 7));
        w->pos++;
    }
}

typedef struct {
    const uint8_t *buf;
    uint64_t len_bits;
    uint64_t pos;
    int err;
} BitReader;

static uint64_t br_get(BitReader *r, int nbits)
{
    uint64_t v = 0;
    for (int i = 0; i < nbits; i++) {
        if (r->pos >= r->len_bits) { r->err = 1; return 0; }
        int bit = (r->buf[r->pos >> 3] >> (7 - (r->pos & 7))) & 1;
        v = (v << 1) | (uint64_t)bit;
        r->pos++;
    }
    return v;
}

/* ================================================================== */
/* Huffman code lengths (Sec. 3 and Sec. 4: an ordinary Huffman code per */
/* block).  Reading (tie-breaks are not in                                */
/* the paper): leaves with f > 0 sorted by (f, symbol); the classical    */
/* two-queue merge, taking the leaf queue's front on equal weight; code  */
/* length = leaf depth.  One leaf -> length 0.                           */
/* Pinned by: total cost equals an independent heap-based Huffman's cost */
/* (cost is unique over tie-breaks), Kraft sum = 1.                      */
/* ================================================================== */
static void huffman_lengths(const uint64_t freq[256], uint8_t len[256])
{
    int leaves[256], m = 0;
    memset(len, 0, 256);
    for (int s = 0; s < 256; s++) if (freq[s] > 0) leaves[m++] = s;
    if (m == 0) return;
    if (m == 1) { len[leaves[0]] = 0; return; }
    /* insertion sort by (f, symbol) */
    for (int i = 1; i < m; i++) {
        int v = leaves[i], j = i - 1;
        while (j >= 0 && (freq[leaves[j]] > freq[v] || (freq[leaves[j]] == freq[v] && leaves[j] > v))) {
            leaves[j + 1] = leaves[j]; j--;
        }
        leaves[j + 1] = v;
    }
    /* nodes 0..m-1 are leaves (sorted order), m..2m-2 internal */
    uint64_t weight[511];
    int parent[511];
    for (int i = 0; i < m; i++) { weight[i] = freq[leaves[i]]; parent[i] = -1; }
    int qa = 0;            /* leaf queue front */
    int qb = m, qb_end = m; /* internal queue [qb, qb_end) */
    for (int step = 0; step < m - 1; step++) {
        int pick[2];
        for (int t = 0; t < 2; t++) {
            int take_leaf;
            if (qa >= m) take_leaf = 0;
            else if (qb >= qb_end) take_leaf = 1;
            else take_leaf = weight[qa] <= weight[qb]; /* leaf preferred on tie */
            pick[t] = take_leaf ? qa++ : qb++;
        }
        weight[qb_end] = weight[pick[0]] + weight[pick[1]];
        parent[qb_end] = -1;
        parent[pick[0]] = qb_end;
        parent[pick[1]] = qb_end;
        qb_end++;
    }
    for (int i = 0; i < m; i++) {
        int depth = 0, v = i;
        while (parent[v] >= 0) { depth++; v = parent[v]; }
        len[leaves[i]] = (uint8_t)depth;
    }
}

/* ================================================================== */
/* Length-limited fallback code (only used when a seek-table entry of   */
/* t bits cannot hold a segment length, Fig. 3 caption).  Reading: the   */
/* optimal code with lengths <= 14 from the textbook package-merge       */
/* method (Larmore & Hirschberg 1990): coin denominations 2^-1..2^-L,    */
/* one coin per symbol per denomination with numismatic value f; at each */
/* denomination, package adjacent pairs of the finer list and merge with */
/* the symbol coins (ties: symbol coin first, symbol coins in (f,        */
/* symbol) order); the first 2(m-1) items of the coarsest list are       */
/* chosen and a symbol's length is the number of its coins chosen.       */
/* Pinned by: exhaustive search over length-limited codes for small      */
/* alphabets (cost equal), lengths <= limit, Kraft sum = 1.              */
/* ================================================================== */
typedef struct {
    uint64_t w;
    uint8_t cnt[256]; /* coins of each symbol contained in this item */
} PMItem;

static int package_merge_lengths(const uint64_t freq[256], int limit, uint8_t len[256])
{
    int leaves[256], m = 0;
    memset(len, 0, 256);
    for (int s = 0; s < 256; s++) if (freq[s] > 0) leaves[m++] = s;
    if (m == 0) return OR_OK;
    if (m == 1) return OR_OK;
    if ((1 << limit) < m) return OR_E_UNSUPPORTED;
    for (int i = 1; i < m; i++) {
        int v = leaves[i], j = i - 1;
        while (j >= 0 && (freq[leaves[j]] > freq[v] || (freq[leaves[j]] == freq[v] && leaves[j] > v))) {
            leaves[j + 1] = leaves[j]; j--;
        }
        leaves[j + 1] = v;
    }
    PMItem *prev = (PMItem *)calloc((size_t)2 * m, sizeof(PMItem));
    PMItem *cur = (PMItem *)calloc((size_t)2 * m, sizeof(PMItem));
    if (!prev || !cur) { free(prev); free(cur); return OR_E_NOMEM; }
    int nprev = 0;
    /* finest denomination 2^-limit: the symbol coins alone */
    for (int i = 0; i < m; i++) { prev[i].w = freq[leaves[i]]; prev[i].cnt[leaves[i]] = 1; }
    nprev = m;
    for (int level = limit - 1; level >= 1; level--) {
        /* packages of adjacent pairs of the finer list */
        int npk = nprev / 2;
        int a = 0, b = 0, ncur = 0;
        while (a < m || b < npk) {
            int take_coin;
            uint64_t wb = 0;
            if (b < npk) wb = prev[2 * b].w + prev[2 * b + 1].w;
            if (a >= m) take_coin = 0;
            else if (b >= npk) take_coin = 1;
            else take_coin = freq[leaves[a]] <= wb;
            PMItem *o = &cur[ncur++];
            memset(o, 0, sizeof(*o));
            if (take_coin) {
                o->w = freq[leaves[a]];
                o->cnt[leaves[a]] = 1;
                a++;
            } else {
                o->w = wb;
                for (int s = 0; s < 256; s++) o->cnt[s] = (uint8_t)(prev[2 * b].cnt[s] + prev[2 * b + 1].cnt[s]);
                b++;
            }
        }
        PMItem *t = prev; prev = cur; cur = t; nprev = ncur;
    }
    for (int i = 0; i < 2 * (m - 1); i++)
        for (int s = 0; s < 256; s++) len[s] = (uint8_t)(len[s] + prev[i].cnt[s]);
    free(prev); free(cur);
    return OR_OK;
}

/* Canonical codes from lengths (Reading: sort by (length, symbol) and   */
/* count up, as in RFC 1951 Sec. 3.2.2).  One leaf: code length 0.      */
static void canonical_codes(const uint8_t len[256], uint32_t code[256])
{
    int bl_count[64] = {0};
    uint32_t next_code[64] = {0};
    int maxlen = 0;
    for (int s = 0; s < 256; s++) if (len[s]) { bl_count[len[s]]++; if (len[s] > maxlen) maxlen = len[s]; }
    uint32_t c = 0;
    for (int bits = 1; bits <= maxlen; bits++) {
        c = (c + (uint32_t)bl_count[bits - 1]) << 1;
        next_code[bits] = c;
    }
    for (int s = 0; s < 256; s++) { code[s] = 0; if (len[s]) code[s] = next_code[len[s]]++; }
}

/* Code tree built explicitly from the codewords, serialised pre-order  */
/* (Fig. 3 caption: 0 = internal node, 1 + 8-bit symbol = leaf).        */
/* Reading: the left child is bit 0; internal nodes: left then right.   */
typedef struct { int child[2]; int sym; } TNode;

static int tree_from_codes(const uint8_t len[256], const uint32_t code[256], TNode *nodes)
{
    int nn = 1;
    nodes[0].child[0] = nodes[0].child[1] = -1; nodes[0].sym = -1;
    for (int s = 0; s < 256; s++) {
        if (!len[s]) continue;
        int v = 0;
        for (int i = len[s] - 1; i >= 0; i--) {
            int bit = (code[s] >> i) & 1;
            if (nodes[v].child[bit] < 0) {
                nodes[nn].child[0] = nodes[nn].child[1] = -1; nodes[nn].sym = -1;
                nodes[v].child[bit] = nn++;
            }
            v = nodes[v].child[bit];
        }
        nodes[v].sym = s;
    }
    return nn;
}

static void tree_write(BitWriter *w, const TNode *nodes, int v)
{
    if (nodes[v].sym >= 0 && nodes[v].child[0] < 0) {
        bw_put(w, 1, 1);
        bw_put(w, (uint64_t)nodes[v].sym, 8);
        return;
    }
    bw_put(w, 0, 1);
    tree_write(w, nodes, nodes[v].child[0]);
    tree_write(w, nodes, nodes[v].child[1]);
}

/* ================================================================== */
/* Area order T(k) (Sec. 4 Eq. 1, Fig. 2(c): a snake order).  Eq. 1 is  */
/* garbled as printed (its plane index leaves [0,d-1] after one plane    */
/* and its row index collides).  Reading that keeps its readable parts:  */
/* with n = Wb*Hb/8 areas per plane and k' = k mod n,                    */
/*   row(k) = 2 (k mod 2) + 4 floor(k' / (Wb/2))                         */
/*   col(k) = 4 (floor(k'/2) mod (Wb/4))                                 */
/*   b(k)   = d - 1 - floor(k / n)                                       */
/* i.e. plane by plane from the sign plane down (Sec. 4: sign first,     */
/* then magnitude MSB to LSB), 4-row bands top to bottom, 4-column       */
/* groups left to right, and in each 4x4 cell the upper 4x2 area before  */
/* the lower one.  Pinned by: bijection onto all (area, plane) pairs.    */
/* ================================================================== */
void oracle_area_coord(int32_t k, int32_t wb, int32_t hb, int32_t d, int32_t out[3])
{
    int32_t n = wb * hb / 8;
    int32_t kk = k % n;
    out[0] = 2 * (k % 2) + 4 * (kk / (wb / 2));
    out[1] = 4 * ((kk / 2) % (wb / 4));
    out[2] = d - 1 - k / n;
}

/* Bit b of the signed-magnitude representation (Sec. 4: sign plane      */
/* first, then magnitude bits MSB..LSB).  Reading: plane d-1 is the sign */
/* (1 = negative; zero has sign 0), planes d-2..0 are magnitude bits.    */
static int smr_bit(int32_t v, int b, int d)
{
    if (b == d - 1) return v < 0;
    uint32_t a = v < 0 ? (uint32_t)(-(int64_t)v) : (uint32_t)v;
    return (int)((a >> b) & 1u);
}

/* Symbol of the 4x2 area with top-left (i, j) in plane b (Sec. 4 Eq. 2:  */
/* S = sum over m in {i,i+1}, n in {j..j+3} of B(m,n,b) 2^((n-j)+4(m-i))).*/
/* Reading: the caption of Fig. 2 describes a clockwise bit order but     */
/* Eq. 2 is raster;                                                       */
/* Eq. 2 is followed.  Samples outside the type's extent are zero pad.    */
typedef struct {
    const int32_t *v; /* top-left of the region inside its band */
    int stride;
    int w, h;         /* region extent (may be 0) */
} TypeView;

static int32_t view_get(const TypeView *t, int r, int c)
{
    if (r >= t->h || c >= t->w) return 0;
    return t->v[(size_t)r * t->stride + c];
}

static int area_symbol(const TypeView *t, const int32_t *qv, int i, int j, int b, int d)
{
    (void)t;
    int s = 0;
    for (int m = i; m <= i + 1; m++)
        for (int nn = j; nn <= j + 3; nn++) {
            int bit = smr_bit(qv[m * 128 + nn], b, d);
            s += bit << ((nn - j) + 4 * (m - i));
        }
    return s;
}

/* Number of digits of L in bijective base B (digits 1..B). */
static int bij_digits(uint64_t L, uint64_t B)
{
    int m = 0;
    while (L > 0) { uint64_t q = (L - 1) / B; m++; L = q; }
    return m;
}

/* Digits of L in bijective base B, most significant first. */
static int bij_encode(uint64_t L, uint64_t B, uint32_t *dig)
{
    uint32_t tmp[64];
    int m = 0;
    while (L > 0) {
        uint64_t q = (L - 1) / B;
        tmp[m++] = (uint32_t)(L - q * B);
        L = q;
    }
    for (int i = 0; i < m; i++) dig[i] = tmp[m - 1 - i];
    return m;
}

/* Per-block analysis exported for tests. */
typedef struct {
    int32_t d;
    int32_t p;
    int32_t wb, hb;
    int32_t n_segments;
    int32_t czr;
    int32_t wz;
    int32_t l_provisional;
    int32_t limited; /* 1 if the length-limited fallback was used */
    int32_t tbits;
    uint32_t masks[3];
    uint8_t lengths[256];
    uint64_t freq[256];
    uint32_t seg_bits[32];
    uint64_t run_hist[40]; /* F_i: maximal zero runs with bit_length(L) = i */
    uint64_t total_bits;
} BlockInfo;

/* ================================================================== */
/* Encode one coefficient block (Sec. 4; Fig. 3).  types[0..p-1] are   */
/* the multiplexed types (LH, HL, HH for an H-block, caption order; LL  */
/* alone for an LL-block), already quantised.  Reading of the layout    */
/* (the field figure is missing): all MSB-first, not byte aligned:      */
/*   d (5 bits) | p masks of d bits (plane d-1 first; 1 = plane removed) */
/*   | if any plane is kept: C_zr (8) | wz (4) | tree | one t-bit        */
/*   seek-table entry per segment holding the segment's length in bits | */
/*   segments in plane order | zero pad to a byte.                      */
/* A segment is one bitplane: the kept types' symbols concatenated in    */
/* type order, each in T(k) order.  Zero runs never cross segments.      */
/* ================================================================== */
static int encode_block(const TypeView *types, int p, int wb, int hb,
                        BitWriter *out, BlockInfo *info)
{
    int n = wb * hb / 8;
    /* zero-padded copies of the (already quantised) types, 128 x 128 */
    int32_t *q = (int32_t *)calloc((size_t)3 * 128 * 128, sizeof(int32_t));
    if (!q) return OR_E_NOMEM;
    uint64_t maxmag = 0;
    for (int t = 0; t < p; t++)
        for (int r = 0; r < hb; r++)
            for (int c = 0; c < wb; c++) {
                int32_t v = view_get(&types[t], r, c);
                q[(size_t)t * 128 * 128 + r * 128 + c] = v;
                uint64_t a = v < 0 ? (uint64_t)(-(int64_t)v) : (uint64_t)v;
                if (a > maxmag) maxmag = a;
            }
    /* Reading: d is per block: 1 + bit length of the largest magnitude. */
    int d = 1 + bit_length(maxmag);
    if (d > 31) { free(q); return OR_E_UNSUPPORTED; }

    /* symbols of every (type, plane) in T(k) order */
    uint8_t *sym = (uint8_t *)malloc((size_t)p * d * n);
    if (!sym) { free(q); return OR_E_NOMEM; }
    int present[3][32];
    for (int t = 0; t < p; t++) {
        for (int bi = 0; bi < d; bi++) present[t][bi] = 0;
        for (int64_t k = 0; k < (int64_t)n * d; k++) {
            int32_t co[3];
            oracle_area_coord((int32_t)k, wb, hb, d, co);
            int s = area_symbol(&types[t], q + (size_t)t * 128 * 128, co[0], co[1], co[2], d);
            sym[((size_t)t * d + co[2]) * n + (k % n)] = (uint8_t)s;
            if (s) present[t][co[2]] = 1;
        }
    }
    free(q);

    /* Empty bitplanes removed, recorded in one d-bit mask per type (Sec. 4). */
    uint32_t masks[3] = {0, 0, 0};
    for (int t = 0; t < p; t++)
        for (int bi = d - 1; bi >= 0; bi--)
            masks[t] = (masks[t] << 1) | (present[t][bi] ? 0u : 1u);

    /* segments, plane d-1 first */
    int seg_plane[32], nseg = 0;
    for (int bi = d - 1; bi >= 0; bi--) {
        int any = 0;
        for (int t = 0; t < p; t++) any |= present[t][bi];
        if (any) seg_plane[nseg++] = bi;
    }
    uint8_t *segsym[32];
    int seglen[32];
    for (int s = 0; s < nseg; s++) {
        int bi = seg_plane[s], L = 0;
        segsym[s] = (uint8_t *)malloc((size_t)p * n);
        for (int t = 0; t < p; t++)
            if (present[t][bi]) {
                memcpy(segsym[s] + L, sym + ((size_t)t * d + bi) * n, (size_t)n);
                L += n;
            }
        seglen[s] = L;
    }
    free(sym);

    int tbits = bit_length((uint64_t)(p * n)) - 1 + 5; /* t = floor(log2(p w h / 8)) + 5 */
    if (info) {
        memset(info, 0, sizeof(*info));
        info->d = d; info->p = p; info->wb = wb; info->hb = hb;
        info->n_segments = nseg; info->tbits = tbits;
        for (int t = 0; t < p; t++) info->masks[t] = masks[t];
        info->czr = -1; info->wz = 0;
    }

    bw_put(out, (uint64_t)d, 5);
    for (int t = 0; t < p; t++) bw_put(out, masks[t], d);
    if (nseg == 0) {
        if (info) info->total_bits = out->pos;
        return OR_OK;
    }

    /* Symbol histogram of the kept planes, before run substitution. */
    uint64_t hist[256] = {0};
    for (int s = 0; s < nseg; s++)
        for (int k = 0; k < seglen[s]; k++) hist[segsym[s][k]]++;
    /* Zero-run symbol: the least frequent symbol of the block (Sec. 4).
     * Reading: all 256 values are candidates, ties go to the smallest. */
    int czr = 0;
    for (int v = 1; v < 256; v++) if (hist[v] < hist[czr]) czr = v;

    /* maximal zero runs (length >= 2) inside segments */
    uint64_t runs_F[40] = {0};
    uint64_t nruns = 0, zeros_in_runs = 0;
    for (int s = 0; s < nseg; s++) {
        int k = 0;
        while (k < seglen[s]) {
            if (segsym[s][k] != 0) { k++; continue; }
            int e = k;
            while (e < seglen[s] && segsym[s][e] == 0) e++;
            int L = e - k;
            if (L >= 2) { runs_F[bit_length((uint64_t)L)]++; nruns++; zeros_in_runs += (uint64_t)L; }
            k = e;
        }
    }
    /* literal occurrences of each value (zeros inside runs are not symbols) */
    uint64_t lit[256];
    for (int v = 0; v < 256; v++) lit[v] = hist[v];
    lit[0] -= zeros_in_runs;

    /* Provisional code: each run counted once as a C_zr token (Reading of
     * Eq. 3's l: the code length of C_zr). */
    uint64_t fprov[256];
    for (int v = 0; v < 256; v++) fprov[v] = lit[v];
    fprov[czr] += nruns;
    uint8_t lprov[256];
    huffman_lengths(fprov, lprov);
    int l = lprov[czr];

    /* Counter width (Sec. 4 Eq. 3, garbled as printed).  Reading:
     * minimise sum_i F_i ceil(i / wz) (wz + l) over wz in [2, max(2, beta)],
     * beta = ceil(log2(p n)) (the segment holds at most p n symbols);
     * ties to the smallest wz. */
    int beta = bit_length((uint64_t)(p * n - 1));
    int wz_hi = beta > 2 ? beta : 2;
    int wz = 2;
    uint64_t best = UINT64_MAX;
    for (int w = 2; w <= wz_hi; w++) {
        uint64_t cost = 0;
        for (int i = 1; i < 40; i++) cost += runs_F[i] * (uint64_t)((i + w - 1) / w) * (uint64_t)(w + l);
        if (cost < best) { best = cost; wz = w; }
    }
    uint64_t B = ((uint64_t)1 << wz) - 1;

    /* Final code: C_zr frequency = literal C_zr + every run digit (Sec. 4:
     * the symbol frequencies count the zero runs). */
    uint64_t f[256];
    for (int v = 0; v < 256; v++) f[v] = lit[v];
    for (int s = 0; s < nseg; s++) {
        int k = 0;
        while (k < seglen[s]) {
            if (segsym[s][k] != 0) { k++; continue; }
            int e = k;
            while (e < seglen[s] && segsym[s][e] == 0) e++;
            if (e - k >= 2) f[czr] += (uint64_t)bij_digits((uint64_t)(e - k), B);
            k = e;
        }
    }
    uint8_t len[256];
    huffman_lengths(f, len);

    /* segment lengths in bits; seek-table entries must fit t bits */
    uint32_t segbits[32];
    int limited = 0;
    for (int pass = 0; pass < 2; pass++) {
        int overflow = 0;
        for (int s = 0; s < nseg; s++) {
            uint64_t bits = 0;
            int k = 0;
            while (k < seglen[s]) {
                int v = segsym[s][k];
                if (v != 0) { bits += len[v] + (v == czr ? (uint64_t)wz : 0); k++; continue; }
                int e = k;
                while (e < seglen[s] && segsym[s][e] == 0) e++;
                if (e - k == 1) bits += len[0] + (czr == 0 ? (uint64_t)wz : 0);
                else bits += (uint64_t)bij_digits((uint64_t)(e - k), B) * (len[czr] + (uint64_t)wz);
                k = e;
            }
            if (bits >= ((uint64_t)1 << tbits)) overflow = 1;
            segbits[s] = (uint32_t)bits;
        }
        if (!overflow) break;
        if (pass == 1) {
            for (int s = 0; s < nseg; s++) free(segsym[s]);
            return OR_E_UNSUPPORTED;
        }
        /* Reading (seek-table overflow): rebuild an optimal code limited to
         * 14 bits, keep C_zr and wz. */
        if (package_merge_lengths(f, OR_LIMITED_LEN, len)) {
            for (int s = 0; s < nseg; s++) free(segsym[s]);
            return OR_E_UNSUPPORTED;
        }
        limited = 1;
    }
    uint32_t code[256];
    canonical_codes(len, code);

    /* header */
    bw_put(out, (uint64_t)czr, 8);
    bw_put(out, (uint64_t)wz, 4);
    TNode nodes[520];
    tree_from_codes(len, code, nodes);
    if (nodes[0].child[0] < 0 && nodes[0].child[1] < 0) {
        /* single leaf: the tree is that leaf alone (code length 0) */
        int only = -1;
        for (int v = 0; v < 256; v++) if (f[v] > 0) only = v;
        bw_put(out, 1, 1);
        bw_put(out, (uint64_t)only, 8);
    } else {
        tree_write(out, nodes, 0);
    }
    for (int s = 0; s < nseg; s++) bw_put(out, segbits[s], tbits);

    /* segments: Huffman codewords, counters raw big-endian (Sec. 4) */
    for (int s = 0; s < nseg; s++) {
        int k = 0;
        while (k < seglen[s]) {
            int v = segsym[s][k];
            if (v != 0) {
                bw_put(out, code[v], len[v]);
                if (v == czr) bw_put(out, 0, wz); /* literal C_zr: a run of length zero */
                k++;
                continue;
            }
            int e = k;
            while (e < seglen[s] && segsym[s][e] == 0) e++;
            if (e - k == 1) {
                bw_put(out, code[0], len[0]);
                if (czr == 0) bw_put(out, 0, wz);
            } else {
                /* Reading: run length written as bijective base-(2^wz - 1)
                 * digits, most significant first, each as (C_zr, digit). */
                uint32_t dig[64];
                int md = bij_encode((uint64_t)(e - k), B, dig);
                for (int i = 0; i < md; i++) {
                    bw_put(out, code[czr], len[czr]);
                    bw_put(out, dig[i], wz);
                }
            }
            k = e;
        }
    }
    if (info) {
        info->czr = czr; info->wz = wz; info->l_provisional = l; info->limited = limited;
        memcpy(info->lengths, len, 256);
        memcpy(info->freq, f, sizeof(f));
        for (int s = 0; s < nseg; s++) info->seg_bits[s] = segbits[s];
        memcpy(info->run_hist, runs_F, sizeof(runs_F));
        info->total_bits = out->pos;
    }
    for (int s = 0; s < nseg; s++) free(segsym[s]);
    return OR_OK;
}

/* ================================================================== */
/* Decode one block into (dequantisation is done by the caller) the    */
/* zero-padded types.  Exact inverse of encode_block.  Rejects: d out   */
/* of [1,31], wz out of range, malformed tree (depth > 32, > 256 leaves, */
/* duplicate leaf), a codeword or counter reading past its segment, a   */
/* run of length < 2, a segment decoding to more or fewer symbols than  */
/* it holds or not ending exactly at its seek-table length, seek sum    */
/* past the block end.                                                  */
/* ================================================================== */
static int tree_read(BitReader *r, TNode *nodes, int *nn, int depth, int *nleaves, uint8_t *seen)
{
    if (depth > 32 || *nn >= 511) return OR_E_CORRUPT;
    int v = (*nn)++;
    nodes[v].child[0] = nodes[v].child[1] = -1; nodes[v].sym = -1;
    int bit = (int)br_get(r, 1);
    if (r->err) return OR_E_TRUNCATED;
    if (bit) {
        int s = (int)br_get(r, 8);
        if (r->err) return OR_E_TRUNCATED;
        if (seen[s]) return OR_E_CORRUPT;
        seen[s] = 1;
        nodes[v].sym = s;
        (*nleaves)++;
        return OR_OK;
    }
    int rc;
    int c0 = *nn;
    if ((rc = tree_read(r, nodes, nn, depth + 1, nleaves, seen))) return rc;
    nodes[v].child[0] = c0;
    int c1 = *nn;
    if ((rc = tree_read(r, nodes, nn, depth + 1, nleaves, seen))) return rc;
    nodes[v].child[1] = c1;
    return OR_OK;
}

/* Quality-progressive decode (Sec. 4, decompression: the seek table lets a decoder drop
 * any number of the least significant planes of a block).  Reading: `drop`
 * = r removes the magnitude planes b < r of every block (the sign plane is
 * always kept); their segments are skipped through the seek table and not
 * checked.  A coefficient whose kept magnitude bits are not all zero is
 * reconstructed at the midpoint of its unknown range, |q| = kept + 2^(r-1);
 * otherwise it is 0.  r = 0 is the exact decode. */
static int decode_block(const uint8_t *buf, uint64_t nbytes, int p, int wb, int hb,
                        int32_t *q /* p x 128 x 128 out */, int drop)
{
    int n = wb * hb / 8;
    BitReader r = {buf, nbytes * 8, 0, 0};
    int d = (int)br_get(&r, 5);
    if (r.err) return OR_E_TRUNCATED;
    if (d < 1 || d > 31) return OR_E_CORRUPT;
    uint32_t masks[3] = {0, 0, 0};
    for (int t = 0; t < p; t++) masks[t] = (uint32_t)br_get(&r, d);
    if (r.err) return OR_E_TRUNCATED;
    int present[3][32];
    for (int t = 0; t < p; t++)
        for (int bi = 0; bi < d; bi++) present[t][bi] = !((masks[t] >> bi) & 1u);
    int seg_plane[32], nseg = 0;
    for (int bi = d - 1; bi >= 0; bi--) {
        int any = 0;
        for (int t = 0; t < p; t++) any |= present[t][bi];
        if (any) seg_plane[nseg++] = bi;
    }
    memset(q, 0, sizeof(int32_t) * (size_t)p * 128 * 128);
    if (nseg == 0) return OR_OK;

    int czr = (int)br_get(&r, 8);
    int wz = (int)br_get(&r, 4);
    if (r.err) return OR_E_TRUNCATED;
    int beta = bit_length((uint64_t)(p * n - 1));
    int wz_hi = beta > 2 ? beta : 2;
    if (wz < 2 || wz > wz_hi) return OR_E_CORRUPT;
    uint64_t B = ((uint64_t)1 << wz) - 1;
    TNode nodes[520];
    int nn = 0, nleaves = 0;
    uint8_t seen[256] = {0};
    int rc = tree_read(&r, nodes, &nn, 0, &nleaves, seen);
    if (rc) return rc;
    int single = (nodes[0].child[0] < 0);
    int tbits = bit_length((uint64_t)(p * n)) - 1 + 5;
    uint64_t seglen_bits[32];
    for (int s = 0; s < nseg; s++) seglen_bits[s] = br_get(&r, tbits);
    if (r.err) return OR_E_TRUNCATED;
    uint64_t start = r.pos, total = 0;
    for (int s = 0; s < nseg; s++) total += seglen_bits[s];
    if (start + total > r.len_bits) return OR_E_TRUNCATED;

    uint8_t *seg = (uint8_t *)malloc((size_t)p * n);
    if (!seg) return OR_E_NOMEM;
    uint64_t pos_bits = start;
    for (int s = 0; s < nseg; s++) {
        int bi = seg_plane[s];
        int M = 0;
        for (int t = 0; t < p; t++) if (present[t][bi]) M += n;
        if (bi < drop && bi != d - 1) { /* dropped magnitude plane */
            pos_bits += seglen_bits[s];
            continue;
        }
        BitReader sr = {buf, pos_bits + seglen_bits[s], pos_bits, 0};
        int k = 0;
        uint64_t run = 0;
        int in_run = 0;
        while ((uint64_t)k + run < (uint64_t)M) {
            int v;
            if (single) v = nodes[0].sym;
            else {
                int node = 0;
                while (nodes[node].child[0] >= 0) {
                    int bit = (int)br_get(&sr, 1);
                    if (sr.err) { free(seg); return OR_E_CORRUPT; }
                    node = nodes[node].child[bit];
                }
                v = nodes[node].sym;
            }
            if (v == czr) {
                uint64_t c = br_get(&sr, wz);
                if (sr.err) { free(seg); return OR_E_CORRUPT; }
                if (c != 0) {
                    run = run * B + c;
                    in_run = 1;
                    if ((uint64_t)k + run > (uint64_t)M) { free(seg); return OR_E_CORRUPT; }
                    continue;
                }
            }
            if (in_run) {
                if (run < 2) { free(seg); return OR_E_CORRUPT; }
                for (uint64_t i = 0; i < run; i++) seg[k++] = 0;
                run = 0; in_run = 0;
            }
            if (k >= M) { free(seg); return OR_E_CORRUPT; }
            seg[k++] = (uint8_t)v;
        }
        if (in_run) {
            if (run < 2) { free(seg); return OR_E_CORRUPT; }
            for (uint64_t i = 0; i < run; i++) seg[k++] = 0;
        }
        if (k != M || sr.pos != pos_bits + seglen_bits[s]) { free(seg); return OR_E_CORRUPT; }
        /* scatter: symbols back to bits of the coefficients (Eq. 1, Eq. 2) */
        int off = 0;
        for (int t = 0; t < p; t++) {
            if (!present[t][bi]) continue;
            for (int kk = 0; kk < n; kk++) {
                int32_t co[3];
                oracle_area_coord(kk, wb, hb, 1, co); /* row/col only */
                int sv = seg[off + kk];
                for (int m = 0; m < 2; m++)
                    for (int c = 0; c < 4; c++)
                        if ((sv >> (c + 4 * m)) & 1) {
                            int32_t *cell = &q[(size_t)t * 128 * 128 + (co[0] + m) * 128 + co[1] + c];
                            if (bi == d - 1) *cell |= (int32_t)0x80000000u; /* sign flag */
                            else *cell |= (int32_t)(1u << bi);
                        }
            }
            off += n;
        }
        pos_bits += seglen_bits[s];
    }
    free(seg);
    /* signed-magnitude -> integer */
    for (size_t i = 0; i < (size_t)p * 128 * 128; i++) {
        uint32_t u = (uint32_t)q[i];
        int32_t mag = (int32_t)(u & 0x7fffffffu);
        if (drop > 0 && mag != 0) mag += (int32_t)1 << (drop - 1);
        q[i] = (u & 0x80000000u) ? -mag : mag;
    }
    return OR_OK;
}

/* ================================================================== */
/* Block geometry (Sec. 4: 128x128 blocks; Fig. 3 caption: a block holds */
/* LL coefficients or multiplexed LH, HL, HH).  Reading: a 128-grid      */
/* anchored at each subband's origin; the H-block grid covers the        */
/* ceil(w/2) x ceil(h/2) extent of the level; a cell holds LH, HL, HH in */
/* that order, each zero padded to Wb x Hb = roundup4 of the cell size;  */
/* a cell where all three types are empty emits no block.  Blocks of a   */
/* tile: LL blocks, then H-blocks of level L, ..., level 1; within each  */
/* group channel-major, then block rows, then block columns.             */
/* ================================================================== */
typedef struct {
    int level;    /* 0 for the LL group */
    int chan;
    int bx, by;
    int p;
    int wb, hb;
    int tw[3], th[3]; /* type extents inside the cell */
} BlockGeo;

static int enumerate_blocks(int w, int h, int channels, int levels, BlockGeo *out, int cap)
{
    int nb = 0;
    int lw, lh;
    level_sizes(w, h, levels + 1, &lw, &lh); /* size of LL_levels */
    for (int c = 0; c < channels; c++)
        for (int by = 0; by * OR_BLOCK < lh; by++)
            for (int bx = 0; bx * OR_BLOCK < lw; bx++) {
                if (out && nb < cap) {
                    BlockGeo *g = &out[nb];
                    memset(g, 0, sizeof(*g));
                    g->level = 0; g->chan = c; g->bx = bx; g->by = by; g->p = 1;
                    int cw = lw - bx * OR_BLOCK; if (cw > OR_BLOCK) cw = OR_BLOCK;
                    int ch = lh - by * OR_BLOCK; if (ch > OR_BLOCK) ch = OR_BLOCK;
                    g->tw[0] = cw; g->th[0] = ch;
                    g->wb = roundup4(cw); g->hb = roundup4(ch);
                }
                nb++;
            }
    for (int l = levels; l >= 1; l--) {
        int pw, ph;
        level_sizes(w, h, l, &pw, &ph);
        int gw = (pw + 1) / 2, gh = (ph + 1) / 2, hw = pw / 2, hh = ph / 2;
        for (int c = 0; c < channels; c++)
            for (int by = 0; by * OR_BLOCK < gh; by++)
                for (int bx = 0; bx * OR_BLOCK < gw; bx++) {
                    int cw = gw - bx * OR_BLOCK; if (cw > OR_BLOCK) cw = OR_BLOCK;
                    int ch = gh - by * OR_BLOCK; if (ch > OR_BLOCK) ch = OR_BLOCK;
                    int hwc = hw - bx * OR_BLOCK; if (hwc < 0) hwc = 0; if (hwc > OR_BLOCK) hwc = OR_BLOCK;
                    int hhc = hh - by * OR_BLOCK; if (hhc < 0) hhc = 0; if (hhc > OR_BLOCK) hhc = OR_BLOCK;
                    if (hwc == 0 && hhc == 0) continue; /* LH, HL and HH all empty */
                    if (out && nb < cap) {
                        BlockGeo *g = &out[nb];
                        memset(g, 0, sizeof(*g));
                        g->level = l; g->chan = c; g->bx = bx; g->by = by; g->p = 3;
                        g->tw[0] = cw;  g->th[0] = hhc; /* LH */
                        g->tw[1] = hwc; g->th[1] = ch;  /* HL */
                        g->tw[2] = hwc; g->th[2] = hhc; /* HH */
                        g->wb = roundup4(cw); g->hb = roundup4(ch);
                    }
                    nb++;
                }
    }
    return nb;
}

int32_t oracle_count_blocks(int32_t w, int32_t h, int32_t channels, int32_t levels)
{
    return enumerate_blocks(w, h, channels, levels, NULL, 0);
}

/* ================================================================== */
/* Tile container.  Not in the paper (the iSyntax container is only      */
/* named).  Ours, little endian, byte aligned:                           */
/*   "ISX1" | version u8 (=1) | ct u8 | channels u8 | bits u8 |          */
/*   bytes/sample u8 | levels u8 | qstep u16 | width u32 | height u32 |  */
/*   nblocks u32 | nblocks x u32 block byte sizes | blocks              */
/* ================================================================== */
#define OR_HDR 24

static void put_le(uint8_t *p, uint64_t v, int nbytes)
{
    for (int i = 0; i < nbytes; i++) p[i] = (uint8_t)(v >> (8 * i));
}

static uint64_t get_le(const uint8_t *p, int nbytes)
{
    uint64_t v = 0;
    for (int i = 0; i < nbytes; i++) v |= (uint64_t)p[i] << (8 * i);
    return v;
}

static int validate_params(int w, int h, int channels, int bps, int bits, int levels, int ct, int qstep)
{
    if (w < 1 || h < 1 || w > 65535 || h > 65535) return OR_E_INVALID;
    if (channels < 1 || channels > OR_MAX_CHANNELS) return OR_E_INVALID;
    /* Reading: samples of 1, 2 or 4 bytes; 4-byte samples carry at most 24
     * significant bits, so that every coefficient stays within 32 bits */
    if (bps != 1 && bps != 2 && bps != 4) return OR_E_INVALID;
    if (bits < 1 || bits > (bps == 4 ? 24 : 8 * bps)) return OR_E_INVALID;
    if (levels < 0 || levels > OR_MAX_LEVELS) return OR_E_INVALID;
    if (ct < 0 || ct > 2) return OR_E_INVALID;
    if (ct != 0 && channels != 3) return OR_E_INVALID;
    if (qstep < 1 || qstep > 65535) return OR_E_INVALID;
    return OR_OK;
}

/* Forward transform of a whole tile into per-channel pyramids (after the
 * colour transform and the quantiser). */
static int tile_forward(const uint8_t *pix, int w, int h, int stride, int channels, int bps,
                        int bits, int levels, int ct, int qstep, Pyramid *pyr)
{
    int32_t *planes = (int32_t *)malloc(sizeof(int32_t) * (size_t)w * h * channels);
    if (!planes) return OR_E_NOMEM;
    for (int y = 0; y < h; y++)
        for (int x = 0; x < w; x++) {
            int32_t s[OR_MAX_CHANNELS] = {0};
            for (int c = 0; c < channels; c++) {
                const uint8_t *e = pix + (size_t)y * stride + ((size_t)x * channels + c) * bps;
                uint32_t u = e[0];
                for (int k = 1; k < bps; k++) u |= (uint32_t)e[k] << (8 * k);
                if (u >= (1u << bits)) { free(planes); return OR_E_INVALID; }
                s[c] = (int32_t)u;
            }
            if (ct == 1 || ct == 2) {
                int32_t f[3];
                if (ct == 1) oracle_rct_forward(s[0], s[1], s[2], f);
                else oracle_ycocg_forward(s[0], s[1], s[2], f);
                s[0] = f[0]; s[1] = f[1]; s[2] = f[2];
            }
            for (int c = 0; c < channels; c++) planes[((size_t)c * h + y) * w + x] = s[c];
        }
    for (int c = 0; c < channels; c++) {
        int rc = pyramid_forward(planes + (size_t)c * w * h, w, h, levels, &pyr[c]);
        if (rc) { free(planes); return rc; }
        for (int l = 1; l <= levels; l++) {
            Band *bands[3] = {&pyr[c].hl[l], &pyr[c].lh[l], &pyr[c].hh[l]};
            for (int bi = 0; bi < 3; bi++)
                for (size_t i = 0; i < (size_t)bands[bi]->w * bands[bi]->h; i++)
                    bands[bi]->v[i] = quantise(bands[bi]->v[i], qstep);
        }
    }
    free(planes);
    return OR_OK;
}

static void block_views(const Pyramid *py, const BlockGeo *g, TypeView *tv)
{
    int x0 = g->bx * OR_BLOCK, y0 = g->by * OR_BLOCK;
    if (g->level == 0) {
        tv[0].v = py->ll.v + (size_t)y0 * py->ll.w + x0;
        tv[0].stride = py->ll.w; tv[0].w = g->tw[0]; tv[0].h = g->th[0];
        return;
    }
    const Band *bands[3] = {&py->lh[g->level], &py->hl[g->level], &py->hh[g->level]};
    for (int t = 0; t < 3; t++) {
        tv[t].stride = bands[t]->w;
        tv[t].w = g->tw[t]; tv[t].h = g->th[t];
        tv[t].v = (tv[t].w > 0 && tv[t].h > 0) ? bands[t]->v + (size_t)y0 * bands[t]->w + x0 : bands[t]->v;
    }
}

/* Encode one tile.  Returns the byte count written, or a negative code. */
int64_t oracle_encode_tile(const uint8_t *pixels, int32_t width, int32_t height,
                           int32_t row_stride, int32_t channels, int32_t bytes_per_sample,
                           int32_t bits, int32_t levels, int32_t ct, int32_t qstep,
                           uint8_t *out, uint64_t out_cap)
{
    int rc = validate_params(width, height, channels, bytes_per_sample, bits, levels, ct, qstep);
    if (rc) return rc;
    if (row_stride < width * channels * bytes_per_sample) return OR_E_INVALID;
    Pyramid pyr[OR_MAX_CHANNELS];
    memset(pyr, 0, sizeof(pyr));
    rc = tile_forward(pixels, width, height, row_stride, channels, bytes_per_sample, bits, levels,
                      ct, qstep, pyr);
    if (rc) { for (int c = 0; c < channels; c++) pyramid_free(&pyr[c]); return rc; }
    int nb = enumerate_blocks(width, height, channels, levels, NULL, 0);
    BlockGeo *geo = (BlockGeo *)malloc(sizeof(BlockGeo) * (size_t)nb);
    uint64_t hdr = OR_HDR + 4ull * nb;
    if (!geo) { for (int c = 0; c < channels; c++) pyramid_free(&pyr[c]); return OR_E_NOMEM; }
    enumerate_blocks(width, height, channels, levels, geo, nb);
    if (out_cap < hdr) { free(geo); for (int c = 0; c < channels; c++) pyramid_free(&pyr[c]); return OR_E_CAPACITY; }
    memset(out, 0, (size_t)out_cap);
    uint64_t pos = hdr;
    for (int i = 0; i < nb; i++) {
        TypeView tv[3];
        block_views(&pyr[geo[i].chan], &geo[i], tv);
        if (pos > out_cap) { rc = OR_E_CAPACITY; break; }
        BitWriter bw = {out + pos, (out_cap - pos) * 8, 0, 0};
        rc = encode_block(tv, geo[i].p, geo[i].wb, geo[i].hb, &bw, NULL);
        if (rc) break;
        if (bw.overflow) { rc = OR_E_CAPACITY; break; }
        uint64_t nbytes = (bw.pos + 7) / 8;
        put_le(out + OR_HDR + 4 * (size_t)i, nbytes, 4);
        pos += nbytes;
    }
    free(geo);
    for (int c = 0; c < channels; c++) pyramid_free(&pyr[c]);
    if (rc) return rc;
    memcpy(out, "ISX1", 4);
    out[4] = 1; out[5] = (uint8_t)ct; out[6] = (uint8_t)channels; out[7] = (uint8_t)bits;
    out[8] = (uint8_t)bytes_per_sample; out[9] = (uint8_t)levels;
    put_le(out + 10, (uint64_t)qstep, 2);
    put_le(out + 12, (uint64_t)width, 4);
    put_le(out + 16, (uint64_t)height, 4);
    put_le(out + 20, (uint64_t)nb, 4);
    return (int64_t)pos;
}

/* Parse a tile header: fills the seven parameters (w,h,ch,bps,bits,levels,
 * ct,qstep,nblocks); returns OR_OK or a negative code. */
int32_t oracle_read_header(const uint8_t *in, uint64_t len, int32_t out[9])
{
    if (len < OR_HDR) return OR_E_TRUNCATED;
    if (memcmp(in, "ISX1", 4) != 0 || in[4] != 1) return OR_E_CORRUPT;
    int ct = in[5], ch = in[6], bits = in[7], bps = in[8], lv = in[9];
    int q = (int)get_le(in + 10, 2), w = (int)get_le(in + 12, 4), h = (int)get_le(in + 16, 4);
    uint64_t nbw = get_le(in + 20, 4);
    if (w < 1 || h < 1 || w > 65535 || h > 65535) return OR_E_CORRUPT;
    if (validate_params(w, h, ch, bps, bits, lv, ct, q)) return OR_E_CORRUPT;
    int nb = enumerate_blocks(w, h, ch, lv, NULL, 0);
    if (nbw != (uint64_t)nb) return OR_E_CORRUPT;
    out[0] = w; out[1] = h; out[2] = ch; out[3] = bps; out[4] = bits; out[5] = lv;
    out[6] = ct; out[7] = q; out[8] = nb;
    return OR_OK;
}

/* Decode one tile at resolution level z (0 = full size).  Output is the
 * ceil(W/2^z) x ceil(H/2^z) image (Sec. 4: lower resolutions by discarding
 * the high-pass blocks of the finer levels) interleaved, same sample type
 * as the source.  Reading: samples are clamped to [0, 2^bits - 1] after
 * the inverse colour transform (a no-op for a lossless full-size decode). */
int32_t oracle_decode_tile_q(const uint8_t *in, uint64_t len, int32_t z, int32_t drop,
                             uint8_t *out, int32_t out_row_stride)
{
    int32_t hd[9];
    if (drop < 0 || drop > 31) return OR_E_INVALID;
    int rc = oracle_read_header(in, len, hd);
    if (rc) return rc;
    int w = hd[0], h = hd[1], ch = hd[2], bps = hd[3], bits = hd[4], lv = hd[5], ct = hd[6], qs = hd[7], nb = hd[8];
    if (z < 0 || z > lv) return OR_E_INVALID;
    uint64_t hdr = OR_HDR + 4ull * nb;
    if (len < hdr) return OR_E_TRUNCATED;
    BlockGeo *geo = (BlockGeo *)malloc(sizeof(BlockGeo) * (size_t)(nb > 0 ? nb : 1));
    int32_t *q = (int32_t *)malloc(sizeof(int32_t) * 3 * 128 * 128);
    Pyramid pyr[OR_MAX_CHANNELS];
    memset(pyr, 0, sizeof(pyr));
    if (!geo || !q) { free(geo); free(q); return OR_E_NOMEM; }
    enumerate_blocks(w, h, ch, lv, geo, nb);
    /* allocate the bands */
    for (int c = 0; c < ch && !rc; c++) {
        pyr[c].levels = lv; pyr[c].w0 = w; pyr[c].h0 = h;
        int lw, lh;
        level_sizes(w, h, lv + 1, &lw, &lh);
        rc = band_alloc(&pyr[c].ll, lw, lh);
        for (int l = 1; l <= lv && !rc; l++) {
            int pw, ph;
            level_sizes(w, h, l, &pw, &ph);
            rc = band_alloc(&pyr[c].hl[l], pw / 2, (ph + 1) / 2);
            if (!rc) rc = band_alloc(&pyr[c].lh[l], (pw + 1) / 2, ph / 2);
            if (!rc) rc = band_alloc(&pyr[c].hh[l], pw / 2, ph / 2);
        }
    }
    uint64_t pos = hdr;
    for (int i = 0; i < nb && !rc; i++) {
        uint64_t sz = get_le(in + OR_HDR + 4 * (size_t)i, 4);
        if (geo[i].level != 0 && geo[i].level <= z) break; /* finer levels not needed */
        if (pos + sz > len) { rc = OR_E_TRUNCATED; break; }
        const BlockGeo *g = &geo[i];
        rc = decode_block(in + pos, sz, g->p, g->wb, g->hb, q, drop);
        if (rc) break;
        TypeView tv[3];
        block_views(&pyr[g->chan], g, tv);
        int step = g->level == 0 ? 1 : qs;
        for (int t = 0; t < g->p; t++)
            for (int r = 0; r < tv[t].h; r++)
                for (int c = 0; c < tv[t].w; c++)
                    ((int32_t *)tv[t].v)[(size_t)r * tv[t].stride + c] =
                        dequantise(q[(size_t)t * 128 * 128 + r * 128 + c], step);
        pos += sz;
    }
    free(q); free(geo);
    if (rc) { for (int c = 0; c < ch; c++) pyramid_free(&pyr[c]); return rc; }
    int ow = 0, oh = 0;
    int32_t *planes[OR_MAX_CHANNELS] = {0};
    for (int c = 0; c < ch; c++) {
        planes[c] = pyramid_inverse(&pyr[c], z, &ow, &oh);
        if (!planes[c]) rc = OR_E_NOMEM;
    }
    if (!rc) {
        int32_t top = (1 << bits) - 1;
        for (int y = 0; y < oh; y++)
            for (int x = 0; x < ow; x++) {
                int32_t s[OR_MAX_CHANNELS];
                for (int c = 0; c < ch; c++) s[c] = planes[c][(size_t)y * ow + x];
                if (ct == 1 || ct == 2) {
                    int32_t v[3];
                    if (ct == 1) oracle_rct_inverse(s[0], s[1], s[2], v);
                    else oracle_ycocg_inverse(s[0], s[1], s[2], v);
                    s[0] = v[0]; s[1] = v[1]; s[2] = v[2];
                }
                for (int c = 0; c < ch; c++) {
                    int32_t v = s[c] < 0 ? 0 : (s[c] > top ? top : s[c]);
                    uint8_t *e = out + (size_t)y * out_row_stride + ((size_t)x * ch + c) * bps;
                    for (int k = 0; k < bps; k++) e[k] = (uint8_t)((uint32_t)v >> (8 * k));
                }
            }
    }
    for (int c = 0; c < ch; c++) { free(planes[c]); pyramid_free(&pyr[c]); }
    return rc;
}

/* Exact decode at level z (drop = 0). */
int32_t oracle_decode_tile(const uint8_t *in, uint64_t len, int32_t z,
                           uint8_t *out, int32_t out_row_stride)
{
    return oracle_decode_tile_q(in, len, z, 0, out, out_row_stride);
}

/* ================================================================== */
/* Debug exports used by the tests.                                      */
/* ================================================================== */

/* Forward transform dump: for channel c, writes LL_L then, for l = L..1,
 * HL_l, LH_l, HH_l, each dense row-major, into out (int32).  Returns the
 * number of int32 written or a negative code. */
int64_t oracle_forward_dump(const uint8_t *pixels, int32_t width, int32_t height,
                            int32_t row_stride, int32_t channels, int32_t bytes_per_sample,
                            int32_t bits, int32_t levels, int32_t ct, int32_t qstep,
                            int32_t *out, int64_t cap)
{
    int rc = validate_params(width, height, channels, bytes_per_sample, bits, levels, ct, qstep);
    if (rc) return rc;
    Pyramid pyr[OR_MAX_CHANNELS];
    memset(pyr, 0, sizeof(pyr));
    rc = tile_forward(pixels, width, height, row_stride, channels, bytes_per_sample, bits, levels,
                      ct, qstep, pyr);
    int64_t k = 0;
    for (int c = 0; c < channels && !rc; c++) {
        const Band *list[1 + 3 * OR_MAX_LEVELS];
        int nl = 0;
        list[nl++] = &pyr[c].ll;
        for (int l = levels; l >= 1; l--) { list[nl++] = &pyr[c].hl[l]; list[nl++] = &pyr[c].lh[l]; list[nl++] = &pyr[c].hh[l]; }
        for (int i = 0; i < nl; i++) {
            int64_t cnt = (int64_t)list[i]->w * list[i]->h;
            if (k + cnt > cap) { rc = OR_E_CAPACITY; break; }
            memcpy(out + k, list[i]->v, sizeof(int32_t) * (size_t)cnt);
            k += cnt;
        }
    }
    for (int c = 0; c < channels; c++) pyramid_free(&pyr[c]);
    return rc ? rc : k;
}

/* Code lengths of the per-block Huffman code (limit 0 = unlimited two-queue
 * construction, else package-merge with that limit). */
int32_t oracle_huffman_lengths(const uint64_t *freq, int32_t limit, uint8_t *len)
{
    if (limit <= 0) { huffman_lengths(freq, len); return OR_OK; }
    return package_merge_lengths(freq, limit, len);
}

void oracle_canonical_codes(const uint8_t *len, uint32_t *code) { canonical_codes(len, code); }

/* Encode a single block given its p types as dense Wb x Hb arrays (already
 * quantised); writes the block bytes and analysis info.  Returns the byte
 * count or a negative code. */
int64_t oracle_encode_block(const int32_t *types, int32_t p, int32_t wb, int32_t hb,
                            uint8_t *out, uint64_t cap, BlockInfo *info)
{
    if (p != 1 && p != 3) return OR_E_INVALID;
    if (wb < 4 || hb < 4 || wb > 128 || hb > 128 || wb % 4 || hb % 4) return OR_E_INVALID;
    TypeView tv[3];
    for (int t = 0; t < p; t++) {
        tv[t].v = types + (size_t)t * wb * hb;
        tv[t].stride = wb; tv[t].w = wb; tv[t].h = hb;
    }
    memset(out, 0, (size_t)cap);
    BitWriter bw = {out, cap * 8, 0, 0};
    int rc = encode_block(tv, p, wb, hb, &bw, info);
    if (rc) return rc;
    if (bw.overflow) return OR_E_CAPACITY;
    return (int64_t)((bw.pos + 7) / 8);
}

/* Decode a single block into p dense Wb x Hb arrays. */
int32_t oracle_decode_block_q(const uint8_t *in, uint64_t len, int32_t p, int32_t wb, int32_t hb,
                              int32_t drop, int32_t *types)
{
    if (p != 1 && p != 3) return OR_E_INVALID;
    if (drop < 0 || drop > 31) return OR_E_INVALID;
    if (wb < 4 || hb < 4 || wb > 128 || hb > 128 || wb % 4 || hb % 4) return OR_E_INVALID;
    int32_t *q = (int32_t *)malloc(sizeof(int32_t) * 3 * 128 * 128);
    if (!q) return OR_E_NOMEM;
    int rc = decode_block(in, len, p, wb, hb, q, drop);
    if (!rc)
        for (int t = 0; t < p; t++)
            for (int r = 0; r < hb; r++)
                for (int c = 0; c < wb; c++)
                    types[(size_t)t * wb * hb + r * wb + c] = q[(size_t)t * 128 * 128 + r * 128 + c];
    free(q);
    return rc;
}

int32_t oracle_decode_block(const uint8_t *in, uint64_t len, int32_t p, int32_t wb, int32_t hb,
                            int32_t *types)
{
    return oracle_decode_block_q(in, len, p, wb, hb, 0, types);
}

int32_t oracle_blockinfo_size(void) { return (int32_t)sizeof(BlockInfo); }

/* Block geometry dump: 12 int32 per block (level, chan, bx, by, p, wb, hb,
 * tw0, th0, tw1, th1, tw2) + th2 -> 13 values. */
int32_t oracle_block_geometry(int32_t w, int32_t h, int32_t channels, int32_t levels,
                              int32_t *out, int32_t cap_blocks)
{
    int nb = enumerate_blocks(w, h, channels, levels, NULL, 0);
    if (nb > cap_blocks) return nb;
    BlockGeo *g = (BlockGeo *)malloc(sizeof(BlockGeo) * (size_t)(nb > 0 ? nb : 1));
    if (!g) return OR_E_NOMEM;
    enumerate_blocks(w, h, channels, levels, g, nb);
    for (int i = 0; i < nb; i++) {
        int32_t *o = out + 13 * (size_t)i;
        o[0] = g[i].level; o[1] = g[i].chan; o[2] = g[i].bx; o[3] = g[i].by; o[4] = g[i].p;
        o[5] = g[i].wb; o[6] = g[i].hb;
        o[7] = g[i].tw[0]; o[8] = g[i].th[0]; o[9] = g[i].tw[1]; o[10] = g[i].th[1];
        o[11] = g[i].tw[2]; o[12] = g[i].th[2];
    }
    free(g);
    return nb;
}
