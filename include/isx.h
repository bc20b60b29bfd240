/*
 * isx.h -- C ABI of the MI355X (gfx950) codec library libisx.so.
 *
 * The codec is the one of "Fast Compression Method for Medical Images on the
 * Web" (Hulsken, 2020): reversible colour transform, recursive 2-D 5/3 integer
 * lifting wavelet (Sec. 4), quantisation of the high-pass bands (Sec. 3),
 * 128x128 coefficient blocks coded as signed-magnitude bitplanes of 4x2 areas
 * (Sec. 4 Eq. 1, Eq. 2) with empty-plane masks, zero runs (Eq. 3) and a
 * per-block Huffman code, packed as in the block layout of Fig. 3.
 *
 * Conventions for every entry point:
 *  - "d_" pointers are device (HBM) pointers on the current HIP device, "h_"
 *    pointers are host pointers.  The caller owns every buffer and keeps it
 *    alive until the work queued on `stream` has completed.
 *  - Calls are asynchronous and stream ordered: they validate their host
 *    arguments, enqueue kernels (and, for the convenience entry points, one
 *    small host-to-device copy of the plan) on `stream` and return without
 *    synchronising.  The library never allocates or frees device memory (the
 *    fixed workspace of isx_decode_run_noalloc is part of its code object).
 *  - The return value is ISX_OK or a negative status for errors detected on
 *    the host before anything was enqueued.  Errors only the device can see
 *    (corrupt streams, full output buffer) are written per tile or per job
 *    into d_status, readable after the stream has been synchronised.
 *  - Entry points are thread safe.  The only mutable global state is the
 *    per-device address table of isx_decode_run_noalloc's fixed workspace.
 */
#ifndef ISX_H
#define ISX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define ISX_OK 0
#define ISX_E_INVALID_ARG (-1)   /* bad descriptor, null pointer, size out of range    */
#define ISX_E_CAPACITY (-2)      /* (device status) output arena too small for a tile   */
#define ISX_E_CORRUPT (-3)       /* (device status) malformed encoded stream            */
#define ISX_E_TRUNCATED (-4)     /* (device status) encoded stream shorter than needed  */
#define ISX_E_UNSUPPORTED (-5)   /* parameters outside what the library implements      */
#define ISX_E_WORKSPACE (-6)     /* workspace smaller than the *_workspace_bytes figure */
#define ISX_E_HIP (-7)           /* a HIP runtime call failed                           */
#define ISX_E_PENDING 1          /* (device status) initial value before completion     */

#define ISX_CT_NONE 0
#define ISX_CT_RCT 1    /* reversible colour transform (Y, Cb, Cr), channels == 3       */
#define ISX_CT_YCOCG 2  /* YCoCg-R, the lifting form of YCoCg (Y, Co, Cg), channels == 3 */

/* One tile (image) to encode, or the parameters of an encoded tile.
 * Limits: 1 <= width, height <= 65535; 1 <= channels <= 64; bytes_per_sample
 * 1 (uint8), 2 (uint16) or 4 (uint32), little endian; 1 <= bits <=
 * 8*bytes_per_sample, at most 24 for 4-byte samples (coefficients then fit
 * 32 bits), and every sample < 2^bits; 0 <= levels <= 15; qstep >= 1
 * (1 = lossless).  16- and 32-bit samples need pixel_offset and
 * row_stride_bytes to be multiples of the sample size.
 * Pixels are interleaved: sample (x, y, c) is at byte
 *   pixel_offset + y*row_stride_bytes + (x*channels + c)*bytes_per_sample. */
typedef struct {
    uint64_t pixel_offset;     /* byte offset of the tile in the pixel arena       */
    uint32_t width, height;
    uint32_t row_stride_bytes; /* >= width*channels*bytes_per_sample               */
    uint8_t channels;
    uint8_t bytes_per_sample;
    uint8_t bits;
    uint8_t levels;
    uint8_t colour_transform;  /* ISX_CT_NONE, ISX_CT_RCT or ISX_CT_YCOCG           */
    uint8_t reserved0[3];
    uint16_t qstep;            /* dead-zone quantiser step on HL/LH/HH (Sec. 3)     */
    uint16_t reserved1;
} isx_tile_desc;               /* 32 bytes */

/* One decode job: reconstruct an encoded tile at resolution level
 * target_level (0 = full size; z gives the ceil(W/2^z) x ceil(H/2^z) image
 * built from the coarser blocks only: the decompression part of Sec. 4
 * leaves out the high-pass blocks of the finer levels).  `tile` repeats the
 * encoded tile's parameters (the host plans the workspace from them; the
 * device checks them against the stream header and reports ISX_E_CORRUPT on
 * mismatch); tile.pixel_offset and tile.row_stride_bytes are ignored; for
 * 16- and 32-bit samples out_offset and out_row_stride_bytes must be
 * multiples of the sample size.
 * drop_bitplanes = r > 0 asks for a lower-quality decode (Sec. 4, decompression: the seek
 * table of a block lets the decoder discard its least significant planes):
 * the magnitude planes b < r of every block are skipped (not decoded, not
 * checked; the sign plane is kept), and a coefficient whose kept magnitude
 * bits are not all zero is rebuilt at the midpoint of its unknown range,
 * |q| = kept + 2^(r-1); otherwise it is 0.  The output is clamped to the
 * sample range.  r = 0 is the exact decode; r > 31 is ISX_E_INVALID_ARG. */
typedef struct {
    isx_tile_desc tile;
    uint64_t in_offset;            /* byte offset of the encoded tile in d_encoded    */
    uint64_t in_bytes;             /* bytes available for it                           */
    uint64_t out_offset;           /* byte offset of the output image in d_pixels_out  */
    uint32_t out_row_stride_bytes; /* >= out_width*channels*bytes_per_sample           */
    uint8_t target_level;          /* 0 .. tile.levels                                 */
    uint8_t drop_bitplanes;        /* 0 .. 31: quality-progressive decode, see below    */
    uint16_t reserved;
} isx_decode_job;                  /* 64 bytes */

/* ---- sizes (host, pure) -------------------------------------------------- */

/* Upper bound of the encoded size of every tile, summed, including the
 * 256-byte alignment of tile starts in the output arena. 0 on invalid input. */
uint64_t isx_max_encoded_bytes(const isx_tile_desc *h_descs, int32_t n_tiles);

/* Device workspace needed by isx_encode_tiles for these tiles (bytes). */
uint64_t isx_encode_workspace_bytes(const isx_tile_desc *h_descs, int32_t n_tiles);

/* Device workspace needed by isx_decode_tiles for these jobs (bytes). */
uint64_t isx_decode_workspace_bytes(const isx_decode_job *h_jobs, int32_t n_jobs);

/* Parameters of an encoded tile, read from the first 24 bytes of its stream
 * (host memory; the header written by isx_encode_tiles).  On ISX_OK *out
 * holds the tile's width, height, channels, bytes_per_sample, bits, levels,
 * colour_transform and qstep, with pixel_offset = 0 and row_stride_bytes =
 * width * channels * bytes_per_sample: a ready `tile` for an isx_decode_job.
 * Returns ISX_E_INVALID_ARG for null pointers, ISX_E_TRUNCATED if len < 24,
 * ISX_E_CORRUPT if the magic, the version or a field is out of range or the
 * block count disagrees with the geometry (Sec. 4: 128x128 blocks per band);
 * *out is left unchanged on error. */
int32_t isx_read_tile_header(const void *h_bytes, uint64_t len, isx_tile_desc *out);

/* Number of coefficient blocks of a tile (Sec. 4: 128x128 blocks; LL blocks
 * plus one multiplexed LH/HL/HH block per non-empty grid cell per level). */
int64_t isx_tile_block_count(const isx_tile_desc *h_desc);

/* ---- encode ---------------------------------------------------------------- */

/* Encode n_tiles tiles read from the device pixel arena d_pixels.
 * Output: tile i is written to d_out[d_tile_offsets[i] .. + d_tile_sizes[i])
 * (offsets are 256-byte aligned, assigned in tile order); each tile is a
 * self-contained stream: a 24-byte little-endian header ("ISX1", version,
 * colour transform, channels, bits, bytes/sample, levels, qstep, width,
 * height, block count), the per-block byte sizes (u32 each) and the blocks,
 * each byte aligned.  d_tile_offsets, d_tile_sizes (uint64 x n_tiles) and
 * d_status (int32 x n_tiles) are device arrays written by the kernels;
 * d_status[i] is ISX_OK or ISX_E_CAPACITY (nothing of tile i written).
 * d_workspace must hold isx_encode_workspace_bytes(h_descs, n_tiles) bytes.
 * Output is bit-identical for any batch composition and any run.
 * The plan of the call is copied into the workspace by a stream-ordered copy
 * whose host source the library keeps alive until the copy has run (a host
 * function queued on `stream` releases it).  isx_encode_tiles,
 * isx_decode_tiles and isx_decode_regions return ISX_E_UNSUPPORTED if
 * `stream` is being captured into a graph; capture the plan / run entry
 * points instead. */
int32_t isx_encode_tiles(const isx_tile_desc *h_descs, int32_t n_tiles,
                         const void *d_pixels, void *d_out, uint64_t out_capacity,
                         uint64_t *d_tile_offsets, uint64_t *d_tile_sizes, int32_t *d_status,
                         void *d_workspace, uint64_t workspace_bytes, void *stream);

/* ---- decode ---------------------------------------------------------------- */

/* Decode n_jobs jobs from the device arena d_encoded (as written by
 * isx_encode_tiles) into the device pixel arena d_pixels_out (interleaved,
 * same sample type as the source).  d_status[j] (int32, device) receives
 * ISX_OK, ISX_E_CORRUPT or ISX_E_TRUNCATED.  On error the job's output
 * region holds unspecified pixels; the call never reads or writes outside
 * the regions the jobs name.  Lossless tiles decode bit-exactly; lossy
 * tiles and reduced-resolution outputs are clamped to [0, 2^bits-1]. */
int32_t isx_decode_tiles(const void *d_encoded, const isx_decode_job *h_jobs, int32_t n_jobs,
                         void *d_pixels_out, int32_t *d_status,
                         void *d_workspace, uint64_t workspace_bytes, void *stream);

/* ---- plans (for callers that replay the same shapes, e.g. in a HIP graph) --
 * isx_*_plan_bytes gives the size of a host plan; isx_*_plan_build fills it;
 * the caller copies it to device memory once and calls isx_*_run with the
 * device copy: the run entry points enqueue kernels only (no copies), so
 * they may be captured into a HIP graph. */
uint64_t isx_encode_plan_bytes(const isx_tile_desc *h_descs, int32_t n_tiles);
int32_t isx_encode_plan_build(const isx_tile_desc *h_descs, int32_t n_tiles, void *h_plan,
                              uint64_t plan_bytes);
int32_t isx_encode_run(const void *h_plan, const void *d_plan, const void *d_pixels, void *d_out,
                       uint64_t out_capacity, uint64_t *d_tile_offsets, uint64_t *d_tile_sizes,
                       int32_t *d_status, void *d_workspace, uint64_t workspace_bytes,
                       void *stream);

uint64_t isx_decode_plan_bytes(const isx_decode_job *h_jobs, int32_t n_jobs);
int32_t isx_decode_plan_build(const isx_decode_job *h_jobs, int32_t n_jobs, void *h_plan,
                              uint64_t plan_bytes);
int32_t isx_decode_run(const void *h_plan, const void *d_plan, const void *d_encoded,
                       void *d_pixels_out, int32_t *d_status, void *d_workspace,
                       uint64_t workspace_bytes, void *stream);

/* ---- decode without any allocation ------------------------------------------
 * For callers that cannot allocate memory of any kind during the call: code
 * recorded under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  isx_decode_run_noalloc is isx_decode_run with its
 * workspace taken from a fixed array of ISX_NOALLOC_SCRATCH_BYTES in the
 * library's own device memory instead of a d_workspace argument: it calls no
 * hipMalloc, hipFree, host allocator or other allocating routine (the
 * address of the array is looked up once per device, on the first call with
 * that device current).  The caller still passes the plan (h_plan and its
 * device copy d_plan, from isx_decode_plan_build or isx_region_plan_build),
 * the encoded arena, the output arena and d_status, exactly as for
 * isx_decode_run; the output is identical to isx_decode_run's.
 * Returns ISX_E_WORKSPACE if the plan needs more than
 * ISX_NOALLOC_SCRATCH_BYTES of workspace (isx_decode_workspace_bytes of its
 * jobs: 64 MiB covers one 1024x1024 RGB tile at any level count, one
 * 2048x2048 single-channel 16-bit tile, or eleven 512x512 RGB tiles of 6
 * levels), ISX_E_INVALID_ARG for a null pointer or a plan
 * that is not a decode plan, ISX_E_HIP if the runtime fails.
 * Every call on one GPU uses that GPU's one array, which keeps the contents
 * of the last call (every counter and queue the kernels need is cleared by
 * the kernels themselves): calls that overlap on one GPU (on different
 * streams, or from different threads without ordering) race and produce
 * undefined output.  Calls ordered on one stream are safe. */
#define ISX_NOALLOC_SCRATCH_BYTES (64ull << 20)
int32_t isx_decode_run_noalloc(const void *h_plan, const void *d_plan, const void *d_encoded,
                               void *d_pixels_out, int32_t *d_status, void *stream);

/* Sizes recorded in a plan built by any isx_*_plan_build call (host
 * memory): the plan's length in bytes and the workspace its runs need (the
 * same figures as isx_*_plan_bytes and isx_*_workspace_bytes for its tiles
 * or jobs, without planning them again).  A caller may build into a buffer
 * of a known capacity and read the sizes back here.  Returns ISX_OK, or
 * ISX_E_INVALID_ARG for null pointers or bytes that are not a plan of this
 * library. */
int32_t isx_plan_info(const void *h_plan, uint64_t *plan_bytes, uint64_t *workspace_bytes);

/* Launch parameters of a plan.  They change speed only: the encoded bytes and
 * decoded pixels are identical for every setting.
 *  transform_tile: quads per side of a lifting tile staged in LDS, 16 or 32
 *                  (0 = 32); 32 stages 68x68-sample windows, 16 stages 36x36.
 *  blocks_per_cu:  0 = one workgroup per coefficient block for the per-block
 *                  kernels; k > 0 = a persistent grid of k workgroups per
 *                  compute unit that loops over the blocks (1..64).
 *  seg_waves_per_cu: decode only: persistent one-wave workgroups per compute
 *                  unit of the segment decoder (0 = 11, the most its LDS
 *                  allows; 1..11); used with seg_wave_group 1.
 *  seg_wave_group: decode only: waves per segment-decoder workgroup, 1, 2 or
 *                  4 (0 = 4 for plans of at most 4 segment slots per compute
 *                  unit, else 2).  1: each wave decodes its own segments.
 *                  2: both waves decode a large segment together, each
 *                  decodes small ones alone; 8 workgroups per compute unit.
 *                  4: all four decode every segment together; 4 workgroups
 *                  per compute unit. */
typedef struct {
    int32_t transform_tile;
    int32_t blocks_per_cu;
    int32_t seg_waves_per_cu;
    int32_t seg_wave_group;
    int32_t reserved[4];
} isx_tuning;

/* As isx_*_plan_build, with explicit launch parameters (NULL = defaults).
 * Returns ISX_E_INVALID_ARG for values outside the ranges above. */
int32_t isx_encode_plan_build_tuned(const isx_tile_desc *h_descs, int32_t n_tiles,
                                    const isx_tuning *tuning, void *h_plan, uint64_t plan_bytes);
int32_t isx_decode_plan_build_tuned(const isx_decode_job *h_jobs, int32_t n_jobs,
                                    const isx_tuning *tuning, void *h_plan, uint64_t plan_bytes);

/* ---- region decode (whole-slide pyramids) ----------------------------------
 * A whole slide encoded as ONE tile is one non-redundant wavelet pyramid
 * (Sec. 3: the blocks of every scale are stored separately, Sec. 4, decompression: a viewer
 * decodes only the blocks of the scale and area it shows).  A region job
 * reconstructs the rectangle [x0, x0+width) x [y0, y0+height) of the level-z
 * image (z = job.target_level) from the blocks it depends on: at each level
 * l = z+1 .. L the inverse lifting of a sample reaches two band samples to
 * either side, so the blocks read are those covering the region's halo at
 * every level, plus the LL blocks under the coarsest halo.  The result is
 * identical, sample for sample, to cropping the full level-z decode.
 *
 * isx_stream_block_offsets reads a stream's header and size table (host
 * memory: the first 24 + 4 * block_count bytes of the stream) and writes
 * the byte offset of every block from the stream start, plus the stream
 * length, into h_offsets[0 .. block_count] (block_count + 1 entries).
 * Returns ISX_OK, ISX_E_INVALID_ARG (null pointers, n_offsets too small),
 * ISX_E_TRUNCATED (head_bytes shorter than the table) or ISX_E_CORRUPT
 * (not a stream of this codec). */
int32_t isx_stream_block_offsets(const void *h_head, uint64_t head_bytes, uint64_t *h_offsets,
                                 uint64_t n_offsets);

/* One region job.  job: the stream (tile parameters, in_offset, in_bytes),
 * the output (out_offset; out_row_stride_bytes >= width * channels *
 * bytes_per_sample), the level (target_level) and drop_bitplanes, exactly
 * as for a whole-tile decode job.  The region must lie inside the level
 * image (1 <= width, height; x0 + width <= ceil(W / 2^z), likewise y).
 * h_block_offsets: the stream's block offsets from isx_stream_block_offsets
 * (host memory, read while the plan is built, not kept).  The device checks
 * every block's size against the stream's own table and reports
 * ISX_E_TRUNCATED if they disagree. */
typedef struct {
    isx_decode_job job;
    uint32_t x0, y0;
    uint32_t width, height;
    const uint64_t *h_block_offsets;
} isx_region_job;                  /* 88 bytes */

/* Sizes and plan of a batch of region jobs (0 on invalid input).  The plan
 * is a decode plan: isx_decode_run / isx_decode_run_stages run it. */
uint64_t isx_region_workspace_bytes(const isx_region_job *h_jobs, int32_t n_jobs);
uint64_t isx_region_plan_bytes(const isx_region_job *h_jobs, int32_t n_jobs);
int32_t isx_region_plan_build(const isx_region_job *h_jobs, int32_t n_jobs, const isx_tuning *tuning,
                              void *h_plan, uint64_t plan_bytes);

/* Decode a batch of region jobs in one call (plan built and copied into the
 * workspace, then run), as isx_decode_tiles does for whole tiles. */
int32_t isx_decode_regions(const void *d_encoded, const isx_region_job *h_jobs, int32_t n_jobs,
                           void *d_pixels_out, int32_t *d_status, void *d_workspace,
                           uint64_t workspace_bytes, void *stream);

/* ---- stage-wise runs (profiling) -------------------------------------------
 * The encode and decode runs are fixed sequences of kernel stages; these
 * entry points enqueue stages [first, first + count) of the full sequence
 * (isx_*_run == all stages), so a caller can bracket each stage with events
 * on `stream`.  Stages without work for the plan enqueue nothing.  Running
 * every stage once, in order, is equivalent to one isx_*_run call.
 * mode: 0 = encode, 1 = decode.  isx_stage_count returns the number of
 * stages (or ISX_E_INVALID_ARG); isx_stage_name a static name ("" if none). */
int32_t isx_stage_count(int32_t mode);
const char *isx_stage_name(int32_t mode, int32_t stage);
int32_t isx_encode_run_stages(const void *h_plan, const void *d_plan, const void *d_pixels, void *d_out,
                              uint64_t out_capacity, uint64_t *d_tile_offsets, uint64_t *d_tile_sizes,
                              int32_t *d_status, void *d_workspace, uint64_t workspace_bytes,
                              void *stream, int32_t first, int32_t count);
int32_t isx_decode_run_stages(const void *h_plan, const void *d_plan, const void *d_encoded,
                              void *d_pixels_out, int32_t *d_status, void *d_workspace,
                              uint64_t workspace_bytes, void *stream, int32_t first, int32_t count);

/* ---- diagnostics ----------------------------------------------------------- */

/* Human-readable text of a status code (static storage). */
const char *isx_status_string(int32_t code);

/* Debug: forward transform only.  Writes, for each channel c, the quantised
 * coefficient bands LL_L then (HL_l, LH_l, HH_l) for l = L..1, each dense
 * row-major int32, into d_coeffs (device), in that order (the same order as
 * the tile's block groups).  Workspace as for isx_encode_tiles. */
int32_t isx_debug_forward(const isx_tile_desc *h_desc, const void *d_pixels, int32_t *d_coeffs,
                          void *d_workspace, uint64_t workspace_bytes, void *stream);

/* Debug: Huffman code lengths as built on the device for a 256-bin
 * frequency table (d_freq: uint32 x 256, device); limit 0 = unlimited
 * two-queue construction, 14 = the length-limited fallback.  d_len:
 * uint8 x 256 (device). */
int32_t isx_debug_huffman(const uint32_t *d_freq, int32_t limit, uint8_t *d_len, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* ISX_H */
