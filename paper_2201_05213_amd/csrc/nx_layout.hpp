// nx_layout.hpp -- data layouts shared by the host runtime and the kernels:
// the device weight image, per-image plan descriptors, the container header.
#pragma once
#include <stdint.h>

namespace nx {

constexpr int NMIX = 10;          // logistic mixture components
constexpr int NOUT = 10 * NMIX;   // head outputs of the model
constexpr int HEAD_TILES = 8;     // head rows padded to 8 MFMA tiles of 16
constexpr int CDF_BITS = 16;
constexpr uint32_t CDF_TOTAL = 1u << CDF_BITS;
constexpr uint32_t RANS_L = 1u << 23;  // lower bound of the normalised rANS state
constexpr uint32_t RANS_X0 = 1u;       // encoder start state

// number of causal taps of the (2h+1)x(2h+1) first kernel: h rows of 2h+1,
// plus h to the left in the pixel's own row
constexpr int n_taps(int h) { return 2 * h * (h + 1); }
constexpr int conv_chunks(int h) { return 3 * n_taps(h) / 4; }  // MFMA K-chunks of 4
constexpr int conv_quads(int h) { return (conv_chunks(h) + 3) / 4; }

// Device weight image (floats). Every MFMA A-operand block is 64 lanes x 4
// consecutive K-chunks (one 16-byte LDS read per lane covers 4 MFMAs).
//   conv:   [mt < C/16][kq < conv_quads][lane][q]   W[16mt + lane%16][k = 4(4kq+q) + lane/16]
//   1x1:    [mt < C/16][ct < C/16][lane][q]         W[16mt + lane%16][16ct + 4(lane/16) + q]
//   head:   [mt < 8][ct < C/16][lane][q]            same, with permuted/padded rows
//   biases: conv[C], per block b1[C], b2[C], head[128] (permuted rows)
struct WeightLayout {
  int h, C, nb;
  int64_t conv, layer0, layer_stride, head, bias_conv, bias_blocks, bias_head, total;
};

inline constexpr WeightLayout weight_layout(int h, int C, int nb) {
  WeightLayout L{};
  L.h = h; L.C = C; L.nb = nb;
  const int64_t mt = C / 16;
  L.conv = 0;
  L.layer0 = mt * conv_quads(h) * 256;
  L.layer_stride = mt * mt * 256;
  L.head = L.layer0 + 2 * (int64_t)nb * L.layer_stride;
  L.bias_conv = L.head + (int64_t)HEAD_TILES * mt * 256;
  L.bias_blocks = L.bias_conv + C;
  L.bias_head = L.bias_blocks + 2 * (int64_t)nb * C;
  L.total = L.bias_head + 16 * HEAD_TILES;
  return L;
}

// Per-image plan, built on the host and copied into the workspace.
struct ImgDesc {
  uint8_t* px;         // H x W x 3 image (input for encode, output for decode)
  int32_t H, W;
  int32_t ph, pw;      // effective patch shape (clamped to the image)
  int32_t nlx, nly;    // lanes per patch row / column
  int64_t lane_base;   // first global lane index of this image
  int64_t px_base;     // first global pixel index of this image
  int64_t tile_base;   // first global 16-pixel encode tile of this image
  int32_t ntx;         // encode tiles per image row = ceil(W/16)
  int32_t pad_;
  int64_t slot_base;   // byte offset of this image's first rANS lane slot
};
static_assert(sizeof(ImgDesc) == 72, "descriptor layout");

// Container header (little endian), followed by u32 lane_end[n_lanes]
// (cumulative payload bytes per lane) and the lane payloads.
constexpr int HDR_BYTES = 32;
constexpr uint8_t CONTAINER_VERSION = 1;
constexpr uint8_t CODER_RANS8 = 1;  // byte-renormalising rANS, L=2^23, M=2^16, x0=1
//  0 "NLXC" | 4 u8 version | 5 u8 order | 6 u8 h | 7 u8 coder | 8 u32 H | 12 u32 W
// 16 u16 patch_h (0 = whole) | 18 u16 patch_w (0 = whole) | 20 u64 model hash
// 28 u32 n_lanes

// Lane slot for the rANS encoder: at most 2 bytes per symbol, 4 flush bytes.
inline constexpr int64_t lane_slot_bytes(int64_t px) { return 6 * px + 8; }

}  // namespace nx
