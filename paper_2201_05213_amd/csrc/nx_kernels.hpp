// nx_kernels.hpp -- launch interface between the host runtime (nx_capi.cpp)
// and the kernels (nx_kernels.hip). Plain structs of device pointers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nx_layout.hpp"

namespace nx {

// status codes written to the per-image device status array (match nellox.h)
constexpr int ST_OK = 0;
constexpr int ST_CORRUPT = 4;
constexpr int ST_MISMATCH = 5;

struct PassArgs {
  const float* w;          // device weight image
  int64_t wfloats;
  int nb;
  const ImgDesc* desc;     // device copy of the plan
  int n_img;
  int64_t n_tiles;
  int mode;                // 0 symbols, 1 continuous bits, 2 full CDF rows
  uint32_t* sym;           // mode 0: (start | freq << 16) per pixel and channel
  float* bits;             // mode 0: quantised ideal bits per pixel (nullable);
                           // mode 1: continuous bits per pixel
  int32_t* cdf;            // mode 2: [pixel][3][257]
};

struct RansEncArgs {
  const ImgDesc* desc;
  int n_img;
  int64_t n_lanes;
  int64_t n_streams;       // rANS streams of the batch (n_lanes K, or the lane rows)
  int order;               // 0 raster, 1 wavefront
  int h;
  int K;                   // rANS streams per lane (ROW_STREAMS: one per lane row)
  const uint32_t* sym;
  uint8_t* slots;
  uint32_t* lane_len;      // symbols per stream (gather), then bytes per stream (encoder)
  uint32_t* rev;           // per stream, its symbols in coding order (reverse decode order);
                           // image n's streams from desc[n].rev_base, stream_rev_words each
  int32_t* after;          // per stream and step t: the stream's symbols in steps after t;
                           // from desc[n].after_base, stream_after_entries each
  int64_t max_lane_px;     // pixels of the largest lane
};

struct PackArgs {
  const ImgDesc* desc;
  int n_img;
  int64_t n_lanes;
  int64_t n_streams;       // rANS streams of the batch
  int order, h;
  int K;                   // rANS streams per lane (ROW_STREAMS: one per lane row)
  uint64_t model_hash;
  const uint8_t* slots;
  const uint32_t* lane_len;  // per stream (global stream index, image n's from desc[n].stream_base)
  uint32_t* lane_end;      // scratch: cumulative payload bytes per stream
  uint64_t* img_bytes;     // scratch: container bytes per image
  uint8_t* out;
  uint64_t* out_offsets;   // n_img + 1
  uint64_t out_cap;
  int32_t* overflow;       // set when the containers would exceed out_cap
};

struct DecArgs {
  const float* w;
  int64_t wfloats;
  int nb;
  const ImgDesc* desc;     // px = output image
  int n_img;
  int64_t n_lanes;
  int order;
  int K;                   // rANS streams per lane
  uint64_t model_hash;
  const uint8_t* in;
  const uint64_t* in_off;  // n_img + 1
  int32_t* status;         // n_img
  int32_t* counter;        // work queue head
  uint32_t* sym_dump;      // nullable: (start | freq << 16) used per pixel/channel
  uint8_t* ring;           // order 2: grid x waves context rings of ring_wave_bytes(ring_rows)
  int ring_rows;
  int32_t* progress;       // row streams: per band, the steps it has finished (zeroed by the prep)
  int64_t n_bands;         // row streams: bands of the batch (the queue's work items)
  uint64_t band_wait_ticks;  // row streams: the longest wait on the band above (100 MHz clock ticks)
  const int32_t* band_order; // row streams, nullable: queue position -> band (in image order)
};
// row streams: the default limit of a band's wait on the band above (20 s);
// a wait that exceeds it marks the image corrupt and lets the band finish
constexpr uint64_t BAND_WAIT_TICKS = 2000000000ull;

// Training objective and gradient (nx_train.hip). n images of H x W, all
// pixel tensors pixel-major.
struct TrainArgs {
  const uint8_t* imgs;     // n x H x W x 3
  int n, H, W, ntx;        // ntx = ceil(W / 16)
  int64_t npx, n_tiles;    // n H W, n H ntx
  int nb, Cp, KP;          // KP = conv inputs padded to a multiple of 16
  const float* wimg;       // forward weight image
  const float* wimgT;      // transposed weight image
  int64_t wfloats, wTfloats;
  float* bits;             // [npx] continuous bits per pixel
  float* ctx;              // [npx][KP] conv inputs (normalised taps)
  float* u;                // [2 nb + 1][npx][Cp] inputs of the 1x1 layers and the head
  float* theta;            // [npx][128] head rows
  float* delta;            // [2 nb + 1][npx][Cp] output deltas: first layer, then per block W1, W2
  float* dtheta;           // [npx][128] head-row deltas
  const float* grad_bits;  // [n] d loss / d bits of image n
};

// layer kinds of the weight-gradient launch (they set the layer's shape)
constexpr int WGRAD_FIRST = 0, WGRAD_BLOCK = 1, WGRAD_HEAD = 2;
// the head's rows go to WGRAD_HEAD_PARTS layer entries (HEAD_TILES /
// WGRAD_HEAD_PARTS row tiles each), which keeps every layer's accumulators
// at most 4 row tiles wide
constexpr int WGRAD_HEAD_PARTS = 2;
constexpr int WGRAD_MAX_LAYERS = 11;  // the head's parts, first layer, up to 8 1x1 layers

struct WgradLayer {
  const float* delta;      // [npx][ld_delta], rows 16-byte aligned
  const float* in;         // [npx][ld_in], rows 16-byte aligned
  int ld_delta, ld_in;
  int64_t w_off, b_off;    // offsets of this layer's dW [rows][cols] and db in a partial
  int kind;                // WGRAD_FIRST, WGRAD_BLOCK or WGRAD_HEAD
};

struct WgradArgs {
  WgradLayer layer[WGRAD_MAX_LAYERS];  // indexed by blockIdx.y
  int64_t npx, chunk, nchunks, ngrad;
  float* partial;          // [nchunks][ngrad]
};

struct GradReduceArgs {
  int h, C, Cp, nb, KP;
  int64_t off_conv, off_blocks, off_head, bias_conv, bias_blocks, bias_head;
  int64_t nchunks, ngrad;
  const float* partial;
  float* grad;             // parameter vector layout
};

// decoder workgroup shape: waves per workgroup and the LDS it needs beyond
// the weight image (per wave a pivot table and a mixture table)
constexpr int DECODE_WAVES = 12;
constexpr int DECODE_LDS_EXTRA = DECODE_WAVES * (256 + 16 * 36) * 4;

// host launchers (return hipError_t of the launch); h in {1,2,3}, C in {16,32,64}
bool supported(int h, int C);
hipError_t launch_pass(int h, int C, const PassArgs& a, int grid, hipStream_t s);
hipError_t launch_rans_encode(const RansEncArgs& a, hipStream_t s);
hipError_t launch_pack(const PackArgs& a, hipStream_t s);
hipError_t launch_decode_prep(int32_t* status, int n_img, int32_t* counter, hipStream_t s,
                              int32_t* progress = nullptr, int64_t n_bands = 0);
// row streams: the band decoder (four waves per workgroup, one per SIMD, one band at a time)
constexpr int ROW_WAVES = 4;
hipError_t launch_decode_rows(int h, int C, const DecArgs& a, int grid, hipStream_t s);
// raise the decoder kernels' LDS limit (once, outside any stream capture)
hipError_t prepare_decode(int h, int C, int K);
// waves per workgroup in 1..DECODE_WAVES (the LDS takes one pivot table per wave);
// prepare_decode must have run for (h, C, a.K)
hipError_t launch_decode(int h, int C, const DecArgs& a, int grid, int waves, hipStream_t s);
// ancestral sampling with the decoder's schedule (DecArgs: in, in_off, status
// and sym_dump unused; every image descriptor carries its seed)
hipError_t launch_sample(int h, int C, const DecArgs& a, int grid, int waves, hipStream_t s);
// per-image FP64 sums of per-pixel bits, in a fixed order (partials: n_img
// x REDUCE_PARTS doubles of scratch)
constexpr int REDUCE_PARTS = 64;
hipError_t launch_reduce_bits(const ImgDesc* desc, int n_img, const float* bits, double* partials, double* out,
                              hipStream_t s);

// the no-allocation decoder's scratch: STATIC_SCRATCH_BYTES of device memory
// per GPU (a file-scope array); static_scratch gives the current device's
// address, looked up on the first call per device
constexpr size_t STATIC_SCRATCH_BYTES = (size_t)32 << 20;
hipError_t static_scratch(void** ptr);

// exhaustive order check of the hardware exp2 and reciprocal (out: 4 counters)
hipError_t launch_check_monotone(unsigned long long* out, hipStream_t s);

constexpr int TRAIN_BLOCK = 16 * 64;  // threads per workgroup of the per-tile training kernels
hipError_t launch_swizzle(const float* params, int h, int C, int Cp, int nb, float* wimg, int64_t nw, float* wimgT,
                          int64_t nwT, hipStream_t s);
hipError_t launch_train_fwd(int h, int Cp, const TrainArgs& a, int grid, hipStream_t s);
hipError_t launch_train_bwd(int h, int Cp, const TrainArgs& a, int grid, hipStream_t s);
hipError_t launch_wgrad(int CT, int KT, const WgradArgs& a, int nlayers, hipStream_t s);
// resident workgroups of that launch per CU (0 if the runtime cannot tell)
int wgrad_blocks_per_cu(int CT, int KT);
hipError_t launch_grad_reduce(const GradReduceArgs& a, hipStream_t s);
hipError_t launch_bits_img(const float* bits, int n, int64_t per_img, double* out, hipStream_t s);

}  // namespace nx
