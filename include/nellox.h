/*
 * nellox.h -- C ABI of nellox, an MI355X (gfx950) implementation of parallel
 * neural local lossless compression (Zhang, Townsend, Kang, Barber,
 * "Parallel Neural Local Lossless Compression", arXiv 2201.05213).
 *
 * What the library computes
 *   An image x in {0..255}^(H x W x 3) is coded into a byte string and back
 *   (Sec. 2: a stream coder driven by an autoregressive model). The model is
 *   the local autoregressive model of Eq. (3) with horizon h: pixel (i,j)
 *   depends on rows i-h..i-1 (columns j-h..j+h) and on row i (columns
 *   j-h..j-1), zero padded, realised as a causal first convolution followed
 *   by 1x1 layers (Sec. 2.1). Its head is a 10-component discretised logistic
 *   mixture over each channel, R then G then B, each channel's weights
 *   conditioned on the earlier channels and its mean shifted linearly by them.
 *   Probabilities are quantised to 16-bit CDFs
 *       cdf_k = k + floor(clamp(F(B_k), 0, 1) * 65280),  B_k = (2k - 256)/255,
 *   so every symbol has frequency >= 1 and the total is 2^16, and coded with
 *   byte-renormalising rANS (32-bit state, L = 2^23, start state 1; a push
 *   from a state below the symbol's frequency f takes the x-th of the slots
 *   whose 16-bit reversal lies in the symbol's range, so it grows the state
 *   by about 2^16 / f; the final state is flushed as its significant bytes),
 *   one stream per lane or K = 2, 4, 8, 16 interleaved streams per lane (opts.interleave):
 *   in a wavefront step, row i - i_first goes to stream (i - i_first) mod K;
 *   or one stream per lane row (interleave -1), its pixels left to right.
 *   Decoding order (nellox_opts.order):
 *     0 raster: one pixel after the other (the sequential decoder of Sec. 2);
 *     1 wavefront: pixel (i,j) at step t = j + (h+1) i, all pixels of a step
 *       in parallel (Sec. 3, Fig. 3, Algorithm 1): W + (h+1)(H-1) steps.
 *   Patches: the image is cut into patch_h x patch_w tiles anchored at (0,0),
 *   row-major, ragged at the right/bottom edges; each tile is coded as an
 *   independent image with its own rANS stream ("lane"), and all lanes of all
 *   images of a call are decoded concurrently. patch 0 = the whole image.
 *
 * Conventions
 *   - Device pointers are HIP device memory on the current device; the
 *     caller owns every buffer and the stream (a hipStream_t passed as void*;
 *     NULL = the default stream). Calls enqueue work on that stream and
 *     return without waiting for it, except where noted.
 *   - The library owns only the model handle (device weights and a small
 *     pinned staging buffer for per-call plans).
 *   - A non-OK return means nothing was enqueued; nellox_last_error() gives
 *     a thread-local message. Data errors found by the GPU (a corrupt
 *     container, a model hash mismatch) are reported per image in the
 *     device status array of nellox_decode.
 *   - Images are uint8, H x W x 3, row-major, channel-interleaved (HWC),
 *     1 <= H, W <= 65535.
 */
#ifndef NELLOX_H
#define NELLOX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nellox_model nellox_model; /* opaque, immutable after create */

typedef enum {
  NELLOX_OK = 0,
  NELLOX_E_ARG = 1,            /* bad argument (null pointer, size out of range) */
  NELLOX_E_BLOB = 2,           /* weight blob malformed or its hash is wrong */
  NELLOX_E_CAPACITY = 3,       /* output or workspace buffer too small */
  NELLOX_E_CORRUPT = 4,        /* (device status) container damaged */
  NELLOX_E_MODEL_MISMATCH = 5, /* (device status) container made by another model */
  NELLOX_E_HIP = 6,            /* a HIP runtime call failed */
  NELLOX_E_UNSUPPORTED = 7     /* model dimensions the library has no kernel for */
} nellox_status;

typedef struct {
  int32_t order;      /* 0 raster, 1 wavefront (Algorithm 1), 2 wavefront decoded in the
                         sheared layout (ShearLoC, Sec. 3.1, Algorithm 2): the coded order
                         and the containers of 2 are those of 1; a decoder with order 2
                         gathers each pixel's context from a window of the lane's
                         sheared canvas, where every step is one column */
  int32_t patch_h;    /* patch rows; <= 0 or >= H: whole image */
  int32_t patch_w;    /* patch columns; <= 0 or >= W: whole image */
  int32_t interleave; /* rANS states per lane: 0 or 1 = one; 2, 4, 8 or 16 (wavefront
                         order only): the rows of every wavefront step are dealt to
                         the states in turn, so a decoder can search that many
                         symbols at once (with 16, every row of a 16-row group has
                         its own stream); -1 (wavefront order 1 only): one stream
                         per lane row, so every row of every step decodes at once,
                         the lane in bands of 16 rows on as many CUs (meant for
                         whole-image lanes, the paper's exact method: a row of W
                         pixels costs one stream). Each stream costs its start
                         and flush, about 4.6 bits */
} nellox_opts;

typedef struct {
  uint8_t* px; /* device pointer to H*W*3 bytes */
  int32_t H, W;
} nellox_image;

/* Weight blob (little endian): "NLXW", u32 version = 1, u32 h, u32 C,
 * u32 n_blocks, u32 n_mix = 10, u32 flags = 1, then FP32 tensors
 *   conv_w[C][3][2h+1][2h+1] (only the causal taps are read), conv_b[C],
 *   per block: w1[C][C], b1[C], w2[C][C], b2[C],
 *   head_w[100][C], head_b[100],
 * then u64 FNV-1a of all preceding bytes. Head outputs: [0,10) mixture
 * logits, [10+10c, 20+10c) means of channel c, [40+10c, 50+10c) log-scales of
 * channel c (floored at -7), [70,80) [80,90) [90,100) pre-tanh coefficients of
 * G|R, B|R, B|G. Each block computes a += W2 elu(W1 elu(a) + b1) + b2; the head
 * reads elu(a). Inputs are normalised as v/127.5 - 1.
 * `blob` is host memory; it is copied. Supported: h in {1,2,3} with
 * C <= 32 (h = 1) or C <= 64 (h = 2, 3), within the per-CU LDS budget. */
nellox_status nellox_model_create(const void* blob, size_t blob_bytes, nellox_model** out);
void nellox_model_destroy(nellox_model* m);
/* dims = {h, C, n_blocks, n_mix}; hash = the blob's FNV-1a trailer */
nellox_status nellox_model_info(const nellox_model* m, int32_t dims[4], uint64_t* hash);

/* Upper bound on the container bytes of one H x W image. */
size_t nellox_encode_bound(int32_t H, int32_t W, const nellox_opts* opts);

/* Device workspace bytes that encode, decode, nll and the debug calls need
 * for this batch (the maximum over them: the encoder's). With K streams per
 * lane about (28 + 6 K) B per pixel plus 16 K (patch_w + 4 patch_h) B per
 * lane: it grows with the sum of the lanes; 0 if the arguments are invalid. */
size_t nellox_workspace_bytes(const nellox_model* m, int32_t n, const nellox_image* imgs, const nellox_opts* opts);

/* Device workspace bytes of every call but nellox_encode for this batch:
 * nellox_decode, nellox_decode_trace, nellox_decode_prepare / _run,
 * nellox_sample, nellox_nll, nellox_debug_symbols and nellox_debug_cdf (image
 * descriptors, the lane queue, the sheared layout's context windows, 4 B of
 * per-pixel bits and the per-image partial sums); at most
 * nellox_workspace_bytes. 0 if the arguments are invalid. */
size_t nellox_decode_workspace_bytes(const nellox_model* m, int32_t n, const nellox_image* imgs,
                                     const nellox_opts* opts);

/* Encode n images (Sec. 2 stream coding; every pixel's CDF is computed in one
 * full-image pass, then each lane is rANS-coded in reverse decode order).
 * out: device buffer of out_cap bytes, at least the sum of
 * nellox_encode_bound over the images; image k's container is written at
 * out + out_offsets[k], out_offsets has n+1 device entries (the last = total).
 * ws: device workspace of ws_bytes >= nellox_workspace_bytes. */
nellox_status nellox_encode(const nellox_model* m, int32_t n, const nellox_image* imgs, const nellox_opts* opts,
                            uint8_t* out, size_t out_cap, uint64_t* out_offsets, void* ws, size_t ws_bytes,
                            void* stream);

/* Read H, W, order and patch shape from a container header in host memory. */
nellox_status nellox_peek(const uint8_t* container, size_t len, int32_t* H, int32_t* W, nellox_opts* opts);

/* Decode n containers (device buffer `in`, image k at in[in_offsets[k] ..
 * in_offsets[k+1]), exactly the container's bytes, in_offsets on the
 * device) into the preallocated images
 * out[k] (H, W from nellox_peek). opts must match the containers (order and
 * patch shape). status: n device int32, set to NELLOX_OK or a data error per
 * image. Wavefront order runs Algorithm 1 of the paper per lane, with all
 * lanes of the batch in one persistent launch. */
nellox_status nellox_decode(const nellox_model* m, int32_t n, const uint8_t* in, const uint64_t* in_offsets,
                            const nellox_opts* opts, const nellox_image* out, int32_t* status, void* ws,
                            size_t ws_bytes, void* stream);

/* As nellox_decode, for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): no
 * workspace argument, and no device or pinned allocation on the call. The
 * decoder's scratch (image descriptors, the lane queue, the sheared layout's
 * context windows) lives in a 32 MiB device array of the library, one per
 * GPU, held until the process ends; its address is looked up on the first
 * call on each device. The call refuses (NELLOX_E_CAPACITY) a batch whose
 * scratch exceeds 32 MiB (nellox_decode_workspace_bytes tells) or that has
 * more than 2,730 images. Calls on one GPU share that array: calls that
 * overlap in time on one GPU (other streams, other threads) race and must
 * not be made; every call resets what it needs (queue, windows) itself. */
nellox_status nellox_decode_static(const nellox_model* m, int32_t n, const uint8_t* in, const uint64_t* in_offsets,
                                   const nellox_opts* opts, const nellox_image* out, int32_t* status, void* stream);

/* As nellox_decode, and also writes the (start | freq << 16) the decoder used
 * for every pixel and channel to sym_dump (device, sum of H*W*3 uint32, images
 * in order) -- for bitwise comparison with nellox_debug_symbols. */
nellox_status nellox_decode_trace(const nellox_model* m, int32_t n, const uint8_t* in, const uint64_t* in_offsets,
                                  const nellox_opts* opts, const nellox_image* out, int32_t* status,
                                  uint32_t* sym_dump, void* ws, size_t ws_bytes, void* stream);

/* ---- capturable decoding (batching) ----
 * nellox_decode split in two: prepare validates the batch and writes its
 * plan (per-image descriptors) into the workspace, with a host-to-device copy;
 * run only launches kernels (no copies, no host waits), so a caller may
 * capture it in a hipGraph and replay it. The plan ties the workspace to the
 * output images: every run decodes into them, from whatever containers `in`
 * and `in_offsets` hold when it executes. A plan is plain host data. */
typedef struct {
  int32_t n, order, interleave; /* images, decoding order, rANS streams per lane */
  int32_t grid, waves;          /* launch shape: workgroups, waves per workgroup */
  int64_t n_lanes;              /* patches (lanes) of the batch */
  uint64_t model_hash;          /* the model the plan was made for */
  int64_t ws_bytes;             /* workspace bytes the plan occupies */
  int64_t desc_offset;          /* byte offset of the descriptors in the workspace */
  int64_t counter_offset;       /* byte offset of the lane-queue counter */
  int64_t ring_offset;          /* order 2: byte offset of the per-wave sheared context rings */
  int64_t ring_rows;            /* order 2: rows of a ring (tallest lane + h, padded) */
  int64_t n_bands;              /* row streams: bands of 16 lane rows (the launch's work items) */
  int64_t progress_offset;      /* row streams: byte offset of the per-band progress counters */
  int64_t band_order_offset;    /* row streams: byte offset of the bands' queue order (0: image order) */
} nellox_decode_plan;

nellox_status nellox_decode_prepare(const nellox_model* m, int32_t n, const nellox_image* out,
                                    const nellox_opts* opts, void* ws, size_t ws_bytes, nellox_decode_plan* plan,
                                    void* stream);
nellox_status nellox_decode_run(const nellox_model* m, const nellox_decode_plan* plan, const uint8_t* in,
                                const uint64_t* in_offsets, int32_t* status, void* ws, void* stream);

/* ---- sampling (the O(D) parallel generation that Sec. 5 leaves to future
 * work, run by the wavefront schedule of Sec. 3) ----
 * Draws n images from the model into the preallocated out[k] (H, W set by the
 * caller) by ancestral sampling. The symbol of channel c of pixel (y, x) of
 * image k is the v with cdf[v] <= u < cdf[v + 1]: cdf is the quantised CDF
 * row the coder uses given the pixels already drawn, u is the top 16 bits of
 * word c of the Philox4x64-10 block (Salmon, Moraes, Dror, Shaw, SC'11) with
 * counter (y W + x, 0, 0, 0) and key (seeds[k], 0). So P(v) = freq_v / 2^16
 * exactly, and an image depends on its seed, size and patch shape only (not
 * on the order, the batch or the launch). opts: order 0 raster or 1 wavefront
 * (H + (h + 1)(W - 1) steps per patch instead of H W); patch_* cut the image
 * into patches drawn independently, as the coder models them; interleave is
 * ignored. seeds: host array of n values. ws: device workspace, at least
 * nellox_workspace_bytes(m, n, out, opts) bytes (the plan is copied into it
 * on `stream`). Errors: NELLOX_E_ARG (null pointer, bad size or order),
 * NELLOX_E_CAPACITY (workspace), NELLOX_E_HIP (a launch failed). */
nellox_status nellox_sample(const nellox_model* m, int32_t n, const uint64_t* seeds, const nellox_opts* opts,
                            const nellox_image* out, void* ws, size_t ws_bytes, void* stream);

/* Continuous code length -log2 p(x) of each image under the model (Eq. 2's
 * objective): bits_per_px (nullable, device, sum of H*W floats) and
 * bits_total (device, n doubles). opts.patch_* selects the patch grid. */
nellox_status nellox_nll(const nellox_model* m, int32_t n, const nellox_image* imgs, const nellox_opts* opts,
                         float* bits_per_px, double* bits_total, void* ws, size_t ws_bytes, void* stream);

/* The encoder's symbols: (start | freq << 16) per pixel and channel (device,
 * sum of H*W*3 uint32) and its quantised ideal code length per image
 * (device, n doubles, nullable). */
nellox_status nellox_debug_symbols(const nellox_model* m, int32_t n, const nellox_image* imgs,
                                   const nellox_opts* opts, uint32_t* sym, double* ideal_bits, void* ws,
                                   size_t ws_bytes, void* stream);

/* Full quantised CDF rows of one image as the encoder computes them:
 * cdf (device) [H*W][3][257] int32, channel rows conditioned on the image's
 * own earlier channels. */
nellox_status nellox_debug_cdf(const nellox_model* m, const nellox_image* img, const nellox_opts* opts,
                               int32_t* cdf, void* ws, size_t ws_bytes, void* stream);

/* Exhaustive check of the property the quantised CDF's monotonicity rests on
 * (every symbol frequency >= 1): over every finite FP32 value in increasing
 * order, counts adjacent pairs where the device's exp2 decreases
 * (counts[0]), where its reciprocal increases on [1, FLT_MAX] (counts[1]),
 * where rcp(1 + exp2(z)) increases (counts[2]); counts[3] = pairs checked.
 * counts: 4 device uint64. */
nellox_status nellox_debug_check_monotone(uint64_t* counts, void* stream);

/* For tests of the row-stream decoder's failure path: sets how long (in
 * ticks of the 100 MHz clock) a band of rows may wait for the band above it
 * in decodes launched from now on; a band that waits longer marks its image
 * CORRUPT and finishes. ticks = 0 restores the default, 2e9 (20 s). Returns
 * the previous limit. Process-wide; not for use while other threads launch
 * decodes. */
uint64_t nellox_debug_band_wait(uint64_t ticks);

/* ---- training (the objective of Eq. 2: the model's code length, and its
 * gradient; Sec. 2.1 model) ----
 * These calls take the parameters directly instead of a model handle, so an
 * optimiser can update them between calls:
 *   dims = {h, C, n_blocks, n_mix = 10}: h in {1,2,3}, C in 1..64 (1..32 for
 *          h = 1), n_blocks >= 0, within one workgroup's LDS;
 *   params: device FP32 vector in the weight blob's tensor order
 *          (nellox_param_count(dims) floats; masked conv taps are ignored and
 *          get gradient 0);
 *   imgs: device, n images of H x W x 3 uint8, contiguous (a batch of crops).
 * Number of FP32 parameters of a model with these dims (-1 if invalid). */
int64_t nellox_param_count(const int32_t dims[4]);

/* Device workspace bytes for nellox_nll_fwd_train / nellox_nll_bwd on a
 * batch of n images of H x W (0 if the arguments are invalid). About
 * (3 (2 n_blocks + 1) C + 300) * 4 bytes per pixel. */
size_t nellox_train_workspace_bytes(const int32_t dims[4], int32_t n, int32_t H, int32_t W);

/* Forward: bits_per_img[k] (device, n doubles) = -log2 p(image k), the joint
 * mixture likelihood of every pixel summed in FP64; bits_per_px (device,
 * n*H*W floats, nullable) receives each pixel's -log2 p in FP32, images and
 * rows in order. Saves in ws what nellox_nll_bwd needs. */
nellox_status nellox_nll_fwd_train(const float* params, const int32_t dims[4], const uint8_t* imgs, int32_t n,
                                   int32_t H, int32_t W, double* bits_per_img, float* bits_per_px, void* ws,
                                   size_t ws_bytes, void* stream);

/* Backward: grad_params (device, overwritten) = sum_k grad_bits[k] *
 * d bits_k / d params, grad_bits: device, n floats. ws must still hold the
 * state of the last nellox_nll_fwd_train with the same params, dims and
 * images (no other call on ws in between): the activations and the weight
 * images come from there. Deterministic: the same inputs give the same
 * bits. */
nellox_status nellox_nll_bwd(const float* params, const int32_t dims[4], const uint8_t* imgs, int32_t n, int32_t H,
                             int32_t W, const float* grad_bits, float* grad_params, void* ws, size_t ws_bytes,
                             void* stream);

const char* nellox_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* NELLOX_H */
