/*
 * ufvc.h - C ABI of the MI355X chunk video codec hot path.
 *
 * The codec follows the chunk coding of "Ultra-Fast Neural Video Compression"
 * (DCVC-UF): a chunk of T frames is patch-embedded to 1/8 resolution, encoded
 * by one chunk encoder into a single latent y, and decoded by a shared chunk
 * decoder followed by T frame-specific decoders (Sec. 3.1, 3.2).  Entropy
 * coding is single-step (Sec. 3.4): one pass predicts the mean mu and scale
 * sigma of every latent element from the hyper prior z_hat, the residual
 * r_hat = round(y - mu) is coded with tables chosen by sigma alone, and the
 * decoder recovers all of r_hat in one bit-stream interaction before adding
 * mu back.  The networks are a stand-in (plain 3x3 convolutions, weights
 * supplied by the caller); the arithmetic coder is 32-lane interleaved rANS.
 *
 * Conventions shared by every entry point
 *  - Device pointers: frames, bit-streams, symbol and index arrays passed to
 *    the coding calls are device (HBM) memory allocated and owned by the
 *    caller.  The library owns only its context, weights, tables and
 *    workspaces, all freed by ufvc_destroy.
 *  - Streams: `stream` is a hipStream_t passed as void* (NULL = the null
 *    stream).  Work is enqueued in stream order.
 *  - Frames: float32, layout [T][3][H][W] contiguous, values in [0, 1].
 *    H and W are multiples of 8 and at least 16; internally they are padded
 *    up to multiples of 16 by edge replication and cropped on output.
 *  - Errors: every call returns a ufvc_status.  Host-checkable argument
 *    errors return immediately without enqueuing work.  Errors found on the
 *    device while decoding (bad header, corrupt stream) are accumulated in a
 *    per-context device status word, read and cleared by ufvc_sync_status.
 *  - Threads: a context may be used by one host thread at a time.
 */
#ifndef UFVC_H
#define UFVC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  UFVC_OK = 0,
  UFVC_E_INVAL = -1,       /* bad argument or header mismatch */
  UFVC_E_NOSPC = -2,       /* output capacity too small; *out_len = size needed */
  UFVC_E_CORRUPT = -3,     /* bit-stream failed its integrity checks */
  UFVC_E_DEVICE = -4,      /* a HIP runtime call failed */
  UFVC_E_NOMEM = -5,       /* device allocation failed */
  UFVC_E_UNSUPPORTED = -6, /* configuration outside what the kernels support */
  UFVC_E_SCRATCH = -7      /* input larger than an allocation-free call's fixed scratch */
} ufvc_status;

/* In every mode the hyper conv runs in float32 and the entropy-parameter
 * conv in float32 arithmetic: its float32 weights are split exactly into
 * three bf16 parts and its input (the integer hyper latent) is exact in
 * bf16, so the bf16 matrix cores form every product exactly and the sums
 * stay float32, in a fixed order (Sec. 3.4). */
typedef enum {
  UFVC_FP32 = 0,      /* every other convolution in float32 (MFMA f32) */
  UFVC_BF16 = 1,      /* analysis and synthesis convs bf16 MFMA, fp32 accumulate */
  UFVC_BF16_FP8 = 2   /* as BF16, synthesis convs in FP8 E4M3 */
} ufvc_precision;

typedef struct {
  int T;               /* frames per chunk, 1..8 (one model per T, Sec. 4.1) */
  int C;               /* latent channels: 64 or 128 */
  int precision;       /* ufvc_precision */
  int seg_log2;        /* y symbols per rANS segment = 2^seg_log2, 5..24 */
  int seg_log2_z;      /* z symbols per rANS segment = 2^seg_log2_z, 5..24 */
  uint32_t model_tag;  /* written to and checked against every bit-stream */
  int autotune;        /* 1: the first call for an (H, W) bucket times every conv
                          tile configuration per layer and keeps the fastest */
  int quadtree;        /* 1: four-step progressive means over the quadtree
                          partition (Sec. 3.4, Fig. 3 (a)); 0: every mean from
                          the single pass.  See "Quadtree means" below. */
  int temporal;        /* 1: chunks are coded conditioned on the temporal
                          context of their stream (Sec. 3.1); such models code
                          through ufvc_stream objects.  See "Temporal context". */
} ufvc_config;

typedef struct ufvc_ctx ufvc_ctx;

/* Number of float32 weights ufvc_create expects for (T, C): the layers
 * a1 (C x 192T x 3 x 3), a2, a3 (C x C), h (32 x C), p (2C x 32), d1, d2, d3
 * (C x C), then for t = 0..T-1: k1_t, k2_t (C x C), k3_t (192 x C), each
 * OIHW, concatenated in that order.  A quadtree model (cfg.quadtree = 1)
 * appends the mean-step layers m1, m2, m3 (C x C x 3 x 3 each), 27 C^2 more
 * values.  Returns 0 for unsupported (T, C).
 *
 * Quadtree means (Sec. 3.4 with Fig. 3 (a)).  The latent is split into four
 * partitions: element (c, v, u) has channel group g = 4c / C and spatial
 * phase q = 2 (v mod 2) + (u mod 2), and lies in partition
 * ({0, 2, 3, 1}[q] + g) mod 4.  The single pass gives every scale and the base
 * mean of every element; partition k = 1, 2, 3 then gets the mean
 * mu_base + conv3x3(r_hat restricted to partitions < k, m_k), computed on the
 * GPU after the one-step decode of all of r_hat (and, in the encoder, before
 * partition k is quantised).  Streams of such models carry header flag bit 0
 * and decode only with a quadtree model; batches and the server take
 * single-pass models only (UNSUPPORTED otherwise).
 *
 * Temporal context (Sec. 3.1 with the Fig. 2 caption, Sec. 3.3, and the
 * prior s_i of Sec. 3.4).  A temporal model (cfg.temporal = 1) appends, after
 * the mean-step layers if any, the context network c1, c2 (C x C), and the
 * context inputs a1c (C x C), pc (2C x C) and d1c (C x C), each 3 x 3 OIHW:
 * 54 C^2 more values.  Chunk i of a stream is coded conditioned on a context
 * C_i ([h][w][C], zero for the first chunk): a1 adds conv(C_i, a1c), the
 * entropy parameters add conv(C_i, pc) (float32 arithmetic like the rest of
 * that conv), d1 adds conv(C_i, d1c), each before its activation; the joint
 * feature F_i then gives C_{i+1} = relu(conv(relu(conv(F_i, c1)), c2)).  The
 * encoder runs the chunk decoder on its own y_hat to follow the decoder's
 * contexts exactly.  Streams carry header flag bit 1; such models code only
 * through ufvc_stream objects (ufvc_encode_chunk / ufvc_decode_chunk, batches
 * and the server return UNSUPPORTED). */
size_t ufvc_weight_count(int T, int C);

/* Creates a context on the current HIP device: validates cfg, repacks the
 * host float32 `weights` (n_weights values, layout above; read only during
 * the call, still owned by the caller) into the kernels' layouts, and builds
 * the Gaussian CDF tables in FP64 on the device: the quantised distributions
 * under which r_hat is coded given sigma alone (Sec. 3.4).  Blocks until
 * done.
 * Errors: INVAL (cfg or n_weights), UNSUPPORTED (also an entropy-parameter
 * weight that three bf16 parts cannot hold exactly: non-finite, or too close
 * to the bottom of the float32 range), NOMEM, DEVICE. */
int ufvc_create(const ufvc_config* cfg, const float* weights, size_t n_weights,
                ufvc_ctx** out);

/* Frees every device allocation of the context (after a device sync). */
void ufvc_destroy(ufvc_ctx* ctx);

/* Upper bound on the coded size of one T x H x W chunk (every symbol at
 * 16 bits, plus states, padding, header and segment table). */
size_t ufvc_max_bitstream_bytes(const ufvc_ctx* ctx, int H, int W);

/* Encodes one chunk (Sec. 3.1 chunk encoder + Sec. 3.4 entropy coding).
 * frames: device [T][3][H][W] float32 with T equal to the context's T.
 * bitstream: device buffer of `capacity` bytes.  On success *out_len is the
 * coded size.  The call is stream-ordered and synchronises `stream` once at
 * the end to read the size.  NOSPC: nothing is written past the header and
 * *out_len holds the size needed. */
int ufvc_encode_chunk(ufvc_ctx* ctx, const float* frames, int T, int H, int W,
                      uint8_t* bitstream, size_t capacity, size_t* out_len,
                      void* stream);

/* Decodes one chunk into device frames_out [T][3][H][W] float32 (Sec. 3.1,
 * 3.2; r_hat decoded in one step from sigma alone, then y_hat = r_hat + mu,
 * Sec. 3.4).  bitstream: device, `len` bytes.  Asynchronous: returns after
 * enqueuing.  The header must match (T, H, W), the context's C, segment
 * sizes and model tag; mismatches set INVAL and integrity failures set
 * CORRUPT in the device status (read with ufvc_sync_status).  The kernels
 * never read outside [bitstream, bitstream + len) and always terminate; on
 * error the frames hold unspecified but finite values. */
int ufvc_decode_chunk(ufvc_ctx* ctx, const uint8_t* bitstream, size_t len,
                      int T, int H, int W, float* frames_out, void* stream);

/* Synchronises `stream`, returns the first device-side error recorded since
 * the last call (UFVC_OK if none) and clears it. */
int ufvc_sync_status(ufvc_ctx* ctx, void* stream);

/* ---- Streams of a temporal model (Sec. 3.1: the chunk context) ----
 * A stream object holds the temporal context of one video stream at one
 * size on one side (an encoder and a decoder each keep their own): C_i, the
 * context of the next chunk, in the activation type, resident on the device.
 * Chunks must be coded and decoded in stream order.  One stream object per
 * host thread at a time; it keeps its context pointer valid until destroyed.
 * ufvc_stream_create: INVAL for a model that is not temporal or a bad size,
 * NOMEM.  The context starts at zero (a stream's first chunk). */
typedef struct ufvc_stream ufvc_stream;
int ufvc_stream_create(ufvc_ctx* ctx, int H, int W, ufvc_stream** out);
void ufvc_stream_destroy(ufvc_stream* st);
/* Sets the context back to zero (the next chunk starts a new stream). */
int ufvc_stream_reset(ufvc_stream* st);
/* Copies the current context ([h][w][C], bf16 bits or float32 as the
 * model's activations) to host memory; `bytes` must equal its size.
 * Synchronises the stream's last HIP stream. */
int ufvc_stream_copy_context(ufvc_stream* st, void* host_dst, size_t bytes);
/* Encodes the stream's next chunk (frames as for ufvc_encode_chunk) with its
 * context, then forms the next context.  Synchronises `stream` once.  On
 * success the context advances; on NOSPC (nothing written past the header,
 * *out_len = size needed) it does not. */
int ufvc_encode_next(ufvc_stream* st, const float* frames, uint8_t* bitstream, size_t capacity,
                     size_t* out_len, void* stream);
/* Decodes the stream's next chunk into frames_out, then forms the next
 * context.  Asynchronous; errors as for ufvc_decode_chunk (read with
 * ufvc_sync_status on the model).  The context always advances: after a
 * decode error reset the stream. */
int ufvc_decode_next(ufvc_stream* st, const uint8_t* bitstream, size_t len, float* frames_out,
                     void* stream);

/* ---- Stage-level entry points (same kernels; used for parity testing) ---- */

/* Copies the device-built tables to host memory (the Gaussian models of
 * r_hat given sigma, Sec. 3.4): freq and cum as 64 x 65 uint16 each (row =
 * scale index, column = symbol r + 32), thresholds as 63 float32 (scale
 * index = number of thresholds <= sigma).  Synchronous. */
int ufvc_get_tables(ufvc_ctx* ctx, uint16_t* freq, uint16_t* cum, float* thresholds);

/* The arithmetic coder of the single-step entropy model on its own (Sec. 3.4:
 * every symbol's table depends on sigma alone, so all of them are coded in
 * one pass): rANS-encodes n symbols (device uint8, values 0..64) with
 * per-symbol table rows idx (device uint8, 0..63) in segments of
 * 2^seg_log2 symbols.  Output
 * (device, `capacity` bytes): uint32 seg_bytes[n_seg] then the segments, in
 * the container's segment format.  *out_len = bytes written (or needed, with
 * NOSPC).  Synchronises `stream`. */
int ufvc_rans_encode(ufvc_ctx* ctx, const uint8_t* sym, const uint8_t* idx, size_t n,
                     int seg_log2, uint8_t* out, size_t capacity, size_t* out_len,
                     void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * ufvc_rans_encode with the same arguments, kernels, output and errors, but
 * it calls no hipMalloc, hipFree or other allocating routine.  Its scratch
 * (padded copies of sym and idx, the per-segment slots, word ranges and
 * offsets) lives in one fixed 64 MiB device array per GPU, reserved when the
 * library's code is loaded there and held until the process ends; its device
 * address is looked up by the first ufvc_create on that GPU.  The scratch
 * needed is, each term rounded up to 256 bytes,
 *     2 (n + 2048) + n_seg (128 + 2^(seg_log2 + 1)) + 8 n_seg + 4 n_seg,
 * n_seg = ceil(n / 2^seg_log2); a larger input returns UFVC_E_SCRATCH without
 * enqueuing work (at seg_log2 = 13 that is about 4 bytes per symbol, so up to
 * 16.7 M symbols: a 4K latent of C = 128 has 16.6 M, a 1080p one 4.2 M).  Nothing in the scratch has to start at zero: every
 * byte a call reads was written earlier in the same call.  All calls on one
 * GPU share the array, so calls that overlap in time on one GPU (two host
 * threads, or two streams) race and must be serialised by the caller.
 * Synchronises `stream`. */
int ufvc_rans_encode_noalloc(ufvc_ctx* ctx, const uint8_t* sym, const uint8_t* idx, size_t n,
                             int seg_log2, uint8_t* out, size_t capacity, size_t* out_len,
                             void* stream);

/* Inverse of ufvc_rans_encode, all segments in one launch (the decoder's
 * single bit-stream interaction, Sec. 3.4): `in` (device, len bytes) -> sym
 * (device, n bytes), with the same per-symbol rows idx (device, n bytes).
 * Asynchronous; integrity failures set CORRUPT in the status. */
int ufvc_rans_decode(ufvc_ctx* ctx, const uint8_t* in, size_t len, const uint8_t* idx,
                     size_t n, int seg_log2, uint8_t* sym, void* stream);

/* Runs the chunk decoder and frame decoders on a caller-provided latent
 * y_hat (device float32, channels innermost [h][w][C], h = Hp/8, w = Wp/8)
 * and writes frames_out.  Asynchronous. */
int ufvc_synthesize(ufvc_ctx* ctx, const float* y_hat, int T, int H, int W,
                    float* frames_out, void* stream);

/* Workspace views left by the last encode / decode, copied to host memory
 * (synchronises the context's last stream).  Element types and layouts
 * (channels innermost, [h][w][c]):
 *   UFVC_BUF_Y      float32 [h][w][C]    analysis output y (encoder)
 *   UFVC_BUF_ZSYM   uint8   [hz][wz][32] z_hat + 32
 *   UFVC_BUF_PARAMS float32 [h][w][2C]   mu (first C) and raw scale logits
 *   UFVC_BUF_IDX    uint8   [h][w][C]    table index from sigma
 *   UFVC_BUF_SYM    uint8   [h][w][C]    r_hat + 32
 * and the synthesis activations of the last decode / synthesis, in the
 * activation type (bfloat16 bits for UFVC_BF16 and UFVC_BF16_FP8, float32
 * for UFVC_FP32), after ReLU:
 *   UFVC_BUF_D2     act     [h][w][C]    output of chunk-decoder conv d2
 *   UFVC_BUF_F      act     [h][w][C]    joint feature F (output of d3)
 *   UFVC_BUF_K1     act     [h][w][T C]  first conv of every frame head
 *   UFVC_BUF_K2     act     [h][w][T C]  second conv of every frame head
 *   UFVC_BUF_AMAX   uint32  [8]          UFVC_BF16_FP8: float32 bits of the
 *                                        amax of the outputs of d1, d2, d3,
 *                                        k1 and k2 (slots 5-7 unused)
 * `bytes` must equal the buffer size for the last (H, W). */
enum { UFVC_BUF_Y = 0, UFVC_BUF_ZSYM = 1, UFVC_BUF_PARAMS = 2, UFVC_BUF_IDX = 3,
       UFVC_BUF_SYM = 4, UFVC_BUF_D2 = 5, UFVC_BUF_F = 6, UFVC_BUF_K1 = 7, UFVC_BUF_K2 = 8,
       UFVC_BUF_AMAX = 9 };
int ufvc_copy_buffer(ufvc_ctx* ctx, int which, void* host_dst, size_t bytes);

/* ---- Frame formats around the YUV444 interface ----
 * The codec's frames are YUV444 planes (the one interface of the
 * supplementary RGB section: RGB and YUV420 video are converted to YUV444 for
 * inference and back afterwards, RGB with BT.709).  Full range, [0, 1],
 * chroma centred at 1/2; BT.709 luma weights Kr = 0.2126, Kb = 0.0722.
 * Layouts (device float32): UFVC_FMT_YUV444 and UFVC_FMT_RGB709 are
 * [T][3][H][W] planes; UFVC_FMT_YUV420 is T planar frames, each Y [H][W]
 * followed by Cb and Cr [H/2][W/2].  4:2:0 -> 4:4:4 repeats each chroma
 * sample over its 2 x 2 block, 4:4:4 -> 4:2:0 takes the block mean; RGB
 * output is clamped to [0, 1]. */
enum { UFVC_FMT_YUV444 = 0, UFVC_FMT_RGB709 = 1, UFVC_FMT_YUV420 = 2 };

/* Converts T frames of H x W (H even, W a multiple of 4) from src_fmt to
 * dst_fmt: RGB709 <-> YUV444 (src may equal dst) and YUV420 <-> YUV444
 * (distinct buffers).  Device pointers, caller-owned; asynchronous on
 * `stream`.  INVAL for bad sizes or an aliased 4:2:0 conversion,
 * UNSUPPORTED for other format pairs. */
int ufvc_convert_frames(const float* src, int src_fmt, float* dst, int dst_fmt, int T, int H,
                        int W, void* stream);

/* ---- The DC block ----
 * The paper builds every module from one primitive, the depth-wise
 * convolution (DC) block of DCVC-RT (supplementary material, DC-block
 * section; the figure with its structure is missing, so the structure is a
 * reading):  t = relu(pw1 x), x1 = x + pw2 dw3x3(t), y = x1 + pw4 relu(pw3 x1)
 * with 1 x 1 convs pw1, pw2 (C -> C), pw3 (C -> 2C), pw4 (2C -> C), one 3 x 3
 * depth-wise filter per channel (zero padding) and no biases.  One fused
 * kernel per call: bf16 operands on the matrix cores, float32 accumulation,
 * t, d, x1 (as pw3's input) and u rounded to bf16, the residual sums float32
 * until the bf16 output.
 *
 * ufvc_dcblock_create uploads one block's weights for C = 64 or 128: host
 * float32, concatenated pw1 (C x C), dw (C x 3 x 3), pw2 (C x C), pw3
 * (2C x C), pw4 (C x 2C), each (out, in) order: 6 C^2 + 9 C values, read
 * only during the call.  INVAL for other C or counts, NOMEM, DEVICE. */
typedef struct ufvc_dcblock ufvc_dcblock;
int ufvc_dcblock_create(int C, const float* weights, size_t n_weights, ufvc_dcblock** out);
/* Frees the block's weights (after a device sync). */
void ufvc_dcblock_destroy(ufvc_dcblock* b);
/* y = DC block(x) on an h x w latent: x and y are device bf16 bit patterns,
 * [h][w][C] (channels innermost), distinct caller-owned buffers.
 * Asynchronous on `stream`.  INVAL for null or aliased pointers or empty
 * sizes. */
int ufvc_dcblock_run(ufvc_dcblock* b, const uint16_t* x, uint16_t* y, int h, int w, void* stream);

/* ---- Batches: many chunks of uneven size per launch ----
 * A batch object runs encode or decode of n chunks (each with its own model,
 * i.e. its own T, and its own H x W) with one launch per pipeline stage and
 * tile configuration, instead of one launch per chunk and stage.  All models
 * must share C, precision and segment sizes.  Per batch composition (the
 * list of (model, H, W)) the object keeps a device arena and fixed-address
 * work lists; with use_graph the decode of a composition is captured into
 * a hipGraph when the composition recurs (its first decode runs eagerly) and
 * replayed from then on.  Results are bitwise identical to the
 * single-chunk calls.  Calls on one batch object must use one stream. */
typedef struct ufvc_batch ufvc_batch;
typedef struct {
  int model;            /* index into the models given to ufvc_batch_create */
  int H, W;             /* frame size; T is the model's */
  const float* frames;  /* encode: input frames, device [T][3][H][W] */
  float* frames_out;    /* decode: output frames, device [T][3][H][W] */
  uint8_t* bitstream;   /* encode: output buffer; decode: input stream (device) */
  size_t capacity;      /* encode: bytes available at bitstream */
  size_t len;           /* decode: stream bytes; encode: set to the coded size */
  int status;           /* set: UFVC_OK or this chunk's error */
} ufvc_chunk;

/* models: n_models contexts, which must outlive the batch object. */
int ufvc_batch_create(ufvc_ctx* const* models, int n_models, ufvc_batch** out);
void ufvc_batch_destroy(ufvc_batch* b);
/* Encodes every chunk; synchronises `stream` and sets len and status. */
int ufvc_encode_batch(ufvc_batch* b, ufvc_chunk* chunks, int n, void* stream);
/* Decodes every chunk; asynchronous (status via ufvc_batch_sync_status). */
int ufvc_decode_batch(ufvc_batch* b, ufvc_chunk* chunks, int n, int use_graph, void* stream);
/* Synchronises `stream` and sets each chunk's decode status. */
int ufvc_batch_sync_status(ufvc_batch* b, ufvc_chunk* chunks, int n, void* stream);
/* Launch policy of the batch's conv stages.  0: each chunk keeps its size
 * bucket's tuned tile configuration, one launch per configuration present
 * in a stage.  1 (default): one launch per stage, every chunk of the batch on
 * the configuration of the chunk with the most work in that stage (when all
 * chunks support it; else as 0).  Results are bitwise identical either way
 * (configurations never change them).  Drops the cached plans (after a
 * device sync).  INVAL for other values. */
int ufvc_batch_set_policy(ufvc_batch* b, int policy);
/* stats[0] plans built, [1] plans evicted (the cache keeps the 32 most
 * recently used compositions), [2] plans cached, [3] conv stages and [4]
 * conv launches of the most recently used plan (encode and decode stages
 * together), [5] the launch policy.  n >= 6. */
int ufvc_batch_stats(ufvc_batch* b, uint64_t* stats, int n);

/* ---- Request server: continuous batching over the batch executor ----
 * Requests (encode or decode of one chunk) arrive from any thread at any
 * time with ufvc_server_submit.  `lanes` executor threads each own a HIP
 * stream (default priority) and a batch object; whenever a lane is free it
 * forms the next batch from the queue in arrival order: the head request's
 * kind, then further queued requests of that kind, up to `max_batch`, while
 * (a) the chunks' working arena fits the lane's arena and (b) the HBM
 * footprint of all admitted, unfinished requests stays within hbm_budget
 * less the lanes' descriptor slabs.  A request's footprint is its working
 * arena plus its own device buffers (input and output).  Batches of
 * different lanes run concurrently on the device, so requests that arrive
 * while others are on the GPU join the next batch as lanes and memory free
 * up.  Model weights, CDF tables, and the callers' frames and bit-streams
 * stay resident; nothing is copied to the host except lengths and status.
 * Results are bitwise those of ufvc_encode_chunk / ufvc_decode_chunk.
 *
 * Ownership: the caller keeps every request's buffers alive and untouched
 * until its completion is polled.  Times are microseconds on a steady clock
 * since the server was created: t_submit when ufvc_server_submit ran,
 * t_admit when the request joined a batch, t_done when that batch's stream
 * had finished. */
typedef struct ufvc_server ufvc_server;
typedef struct {
  size_t hbm_budget;    /* bytes; 0 selects 64 GiB.  Each lane's share
                           (hbm_budget / lanes) is allocated at creation: a
                           slab for batch plans' descriptors (1/16 of the share,
                           at most 64 MiB) and the working arena (the rest), so
                           nothing is allocated on the request path */
  int lanes;            /* 1..8 concurrent batches */
  int max_batch;        /* 1..64 chunks per batch */
  int use_graph;        /* decode batches replay a captured hipGraph */
  int small_pixels;     /* 0: batches formed by arrival only.  > 0 (with two or
                           more lanes): lane 0 prefers requests of at most this
                           many pixels per frame (the oldest such, batched only
                           with such), so a large request cannot hold every lane */
} ufvc_server_config;
enum { UFVC_REQ_ENCODE = 0, UFVC_REQ_DECODE = 1 };
typedef struct {
  int kind;             /* UFVC_REQ_ENCODE or UFVC_REQ_DECODE */
  int model;            /* index into the server's models */
  int H, W;
  const float* frames;  /* encode: input frames, device [T][3][H][W] */
  float* frames_out;    /* decode: output frames, device [T][3][H][W] */
  uint8_t* bitstream;   /* encode: output buffer; decode: input stream (device) */
  size_t capacity;      /* encode: bytes available at bitstream */
  size_t len;           /* decode: stream bytes */
  uint64_t tag;         /* caller's cookie, returned with the completion */
} ufvc_request;
typedef struct {
  uint64_t ticket, tag;
  int status;           /* UFVC_OK, UFVC_E_NOSPC (encode), UFVC_E_CORRUPT / INVAL (decode) */
  int batch_size;       /* chunks in the batch that carried the request */
  size_t len;           /* encode: coded bytes */
  double t_submit_us, t_admit_us, t_done_us;
} ufvc_completion;
/* models: contexts that share C, precision and segment sizes, and outlive
 * the server. */
int ufvc_server_create(ufvc_ctx* const* models, int n_models, const ufvc_server_config* cfg,
                       ufvc_server** out);
/* Queues one request; never blocks on the GPU.  UFVC_E_INVAL for a bad
 * model or size or missing buffer, UFVC_E_NOSPC when its footprint alone
 * exceeds a lane's share of the budget. */
int ufvc_server_submit(ufvc_server* s, const ufvc_request* req, uint64_t* ticket);
/* Moves up to `max` completions to `out`, waiting up to timeout_ms for the
 * first; returns their number (or a negative status). */
int ufvc_server_poll(ufvc_server* s, ufvc_completion* out, int max, int timeout_ms);
/* stats[0] requests queued, [1] in flight, [2] completed, [3] batches run,
 * [4] peak admitted footprint (bytes), [5] HBM budget (bytes), [6] batch
 * plans built so far (all lanes; a plan is built for each new batch
 * composition, cached up to 32 per lane), [7] device bytes reserved for
 * the lanes at creation (arenas and descriptor slabs: the budget). */
int ufvc_server_stats(ufvc_server* s, uint64_t* stats, int n);
/* Finishes every queued and in-flight request, then frees the server
 * (unpolled completions are dropped). */
void ufvc_server_destroy(ufvc_server* s);

/* ---- Conv tile configurations (autotuner) ----
 * ufvc_get_tuning writes, for the 9 tunable conv layers of a T x H x W chunk
 * (a1 a2 a3 d1 d2 d3 k1 k2 k3), the tile configuration chosen so far, or -1
 * where the built-in default is used (n >= 9).  ufvc_tile_config describes a
 * configuration: output tile rows x columns and output channels per
 * workgroup.  Configurations never change results, only speed. */
int ufvc_get_tuning(ufvc_ctx* ctx, int H, int W, int* cfg, int n);
int ufvc_tile_config(int cfg, int* th, int* tw, int* bn);
/* Number of tile configurations (valid cfg values are 0 .. n - 1). */
int ufvc_num_tile_configs(void);
/* Test hook: every conv layer of ctx that supports configuration cfg (its
 * precision, input loader and stride, and a channel tile dividing its
 * outputs) uses it, in chunk calls and in batches planned afterwards; the
 * other layers keep their tuned or default choice.  cfg = -1 clears it.
 * Returns UFVC_E_INVAL for cfg outside -1 .. n - 1. */
int ufvc_force_tile_config(ufvc_ctx* ctx, int cfg);

/* ---- Per-stage timing ----
 * With profiling enabled, every kernel launch of the coding calls is
 * bracketed by two HIP events recorded on the caller's stream (the stream
 * the kernel runs on).  ufvc_profile_enable synchronises the device and
 * clears earlier records.  ufvc_profile_read synchronises the device, writes
 * per stage the summed elapsed milliseconds and the number of launches
 * (arrays of n >= ufvc_profile_stage_count() entries), and clears the
 * records.  Stage names are static strings owned by the library. */
int ufvc_profile_enable(ufvc_ctx* ctx, int on);
int ufvc_profile_stage_count(void);
const char* ufvc_profile_stage_name(int i);
int ufvc_profile_read(ufvc_ctx* ctx, double* total_ms, int* count, int n);

#ifdef __cplusplus
}
#endif
#endif /* UFVC_H */
