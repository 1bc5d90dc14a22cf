// nx_layout.hpp -- data layouts shared by the host runtime and the kernels:
// the device weight image, per-image plan descriptors, the container header.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define NXHD __host__ __device__ inline

namespace nx {

constexpr int NMIX = 10;          // logistic mixture components
constexpr int NOUT = 10 * NMIX;   // head outputs of the model
constexpr int HEAD_TILES = 8;     // head rows padded to 8 MFMA tiles of 16
constexpr int CDF_BITS = 16;
constexpr uint32_t CDF_TOTAL = 1u << CDF_BITS;
constexpr uint32_t RANS_L = 1u << 23;  // lower bound of the normalised rANS state
constexpr uint32_t RANS_X0 = 1u;       // encoder start state (the decoder's end state)

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
  uint64_t seed;       // sampling: key word 0 of the image's Philox stream
  int64_t rev_base;    // encoder: first word of this image's streams in the coding-order symbol buffer
  int64_t after_base;  // encoder: first entry of this image's streams in the per-step offset table
  int64_t stream_base; // first global rANS stream index of this image (lane_base K with K streams per lane)
  int64_t band_base;   // row streams: first global band index of this image
};
static_assert(sizeof(ImgDesc) == 112, "descriptor layout");

// Row streams (opts.interleave = -1, K = 0 inside the library, 0 in the
// container's stream byte): every row of every lane is its own rANS stream,
// its symbols the row's pixels left to right, R, G, B. The stream table
// holds a lane's rows in order, lanes in order: lane (ly, lx) of a patch grid
// nlx wide with patch rows ph starts at entry ly nlx ph + lx Hl, Hl its rows.
constexpr int ROW_STREAMS = 0;
NXHD int64_t row_entry_base(int ly, int lx, int nlx, int ph, int Hl) {
  return (int64_t)ly * nlx * ph + (int64_t)lx * Hl;
}
// a lane's rows are decoded in bands of ROW_BAND rows (one 16-pixel tile),
// one workgroup each, a band waiting on the progress of the one above
constexpr int ROW_BAND = 16;
NXHD int bands_of(int Hl) { return (Hl + ROW_BAND - 1) / ROW_BAND; }
// streams and bands of an image of H rows with a grid of nlx x nly patches of ph rows
NXHD int64_t image_streams(int K, int H, int nlx, int nly) {
  return K == ROW_STREAMS ? (int64_t)nlx * H : (int64_t)nlx * nly * K;
}
NXHD int64_t image_bands(int H, int ph, int nlx, int nly) {
  const int last = H - (nly - 1) * ph;
  return (int64_t)nlx * ((int64_t)(nly - 1) * bands_of(ph) + bands_of(last));
}

// Encoder scratch per rANS stream of a lane of at most ph x pw pixels (K
// streams per lane): its symbols in coding order, 3 (ph pw / K + T) words
// rounded up to 16 (a stream holds at most ceil(n / K) + 1 rows of a step of
// n rows; T = pw + (h + 1)(ph - 1) steps with h + 1 <= 4), and per step the
// count of its symbols in later steps (T + 1 entries). Each image's streams
// take these sizes for its own patch shape, so the buffers grow with the sum
// of the lanes, not with the largest lane times their number.
NXHD int64_t stream_rev_words(int ph, int pw, int K) {
  const int64_t cap = 3 * (((int64_t)ph * pw + K - 1) / K + pw + 4 * ((int64_t)ph - 1));
  return (cap + 15) / 16 * 16;
}
NXHD int64_t stream_after_entries(int ph, int pw) { return (int64_t)pw + 4 * ((int64_t)ph - 1) + 1; }

// Sheared layout (Sec. 3.1, Algorithm 2): a decoding wave keeps the last
// RING_COLS columns of its lane's sheared canvas (column t = wavefront step
// t), as int16 numerators 2x - 255 of the normalised values (0 = padding),
// planes [column][channel][row]; rows = h zero rows on top, then the lane's
// rows, padded to a multiple of 4. The sheared kernel reads h(h+2) columns
// back, so RING_COLS > h(h+2) for every supported h.
constexpr int RING_COLS = 16;
static_assert(RING_COLS > 3 * (3 + 2), "ring too short for h = 3");
NXHD int64_t ring_rows_for(int ph_max, int h) { return ((int64_t)ph_max + h + 3) & ~(int64_t)3; }
NXHD int64_t ring_wave_bytes(int64_t rows) { return (int64_t)RING_COLS * 3 * rows * 2; }
// windows are grouped by XCD (workgroup b runs on XCD b mod RING_XCDS): a
// launch of `grid` workgroups of `waves` waves needs this many windows
constexpr int RING_XCDS = 8;
NXHD int64_t ring_windows(int grid, int waves) {
  return (int64_t)RING_XCDS * ((grid + RING_XCDS - 1) / RING_XCDS) * waves;
}

// Container header (little endian), followed by u32 end[n_lanes * K]
// (cumulative payload bytes per stream, stream k of lane q at q K + k) and
// the stream payloads (the final state's significant bytes, most significant
// first, then the renormalisation bytes in the order the decoder reads them).
constexpr int HDR_BYTES = 32;
constexpr uint8_t CONTAINER_VERSION = 2;
// coder byte = K, the rANS streams per lane: byte-renormalising rANS,
// L = 2^23, M = 2^16, start state 1, pushes from states below the symbol's
// frequency through its bit-reversal-spread slots, K in {1, 2, 4, 8, 16}
constexpr uint8_t CODER_RANS8 = 1;
constexpr int MAX_INTERLEAVE = 16;
NXHD bool valid_interleave(int k) { return k == 1 || k == 2 || k == 4 || k == 8 || k == 16; }
// the container's stream byte: K, or 0 for row streams
NXHD bool valid_stream_code(int k) { return k == ROW_STREAMS || valid_interleave(k); }
//  0 "NLXC" | 4 u8 version | 5 u8 order | 6 u8 h | 7 u8 K | 8 u32 H | 12 u32 W
// 16 u16 patch_h (0 = whole) | 18 u16 patch_w (0 = whole) | 20 u64 model hash
// 28 u32 n_lanes

// Lane slot for the rANS encoder: at most 2 bytes per symbol, at most 4 flush bytes.
inline constexpr int64_t lane_slot_bytes(int64_t px) { return 6 * px + 8; }

// ------------------------------------------------------------------ parameters
// Offsets of the model tensors in the flat FP32 parameter vector, which is the
// weight blob's tensor order: conv_w[C][3][2h+1][2h+1], conv_b[C], per block
// {w1[C][C], b1[C], w2[C][C], b2[C]}, head_w[100][C], head_b[100].
struct ParamLayout {
  int h, C, nb;
  int64_t conv_w, conv_b, blocks, block_stride, head_w, head_b, total;
};

NXHD constexpr ParamLayout param_layout(int h, int C, int nb) {
  ParamLayout P{};
  P.h = h; P.C = C; P.nb = nb;
  const int64_t K = 2 * h + 1;
  P.conv_w = 0;
  P.conv_b = (int64_t)C * 3 * K * K;
  P.blocks = P.conv_b + C;
  P.block_stride = 2 * (int64_t)C * C + 2 * (int64_t)C;
  P.head_w = P.blocks + (int64_t)nb * P.block_stride;
  P.head_b = P.head_w + (int64_t)NOUT * C;
  P.total = P.head_b + NOUT;
  return P;
}

// live tap t of the masked first kernel (Eq. 3): taps in raster order, h full
// rows of 2h+1 above the pixel, then h to its left
NXHD void tap_of(int h, int t, int& dy, int& dx) {
  const int K = 2 * h + 1;
  if (t < h * K) { dy = t / K; dx = t - K * (t / K); }
  else { dy = h; dx = t - h * K; }
}
// inverse: tap index of kernel position (dy, dx), or -1 where it is masked
NXHD int tap_index(int h, int dy, int dx) {
  const int K = 2 * h + 1;
  if (dy < h) return dy * K + dx;
  if (dy == h && dx < h) return h * K + dx;
  return -1;
}

// Head MFMA row r (0..127) holds slot s = 4 (r/16) + r%4 of lane group
// g = (r%16)/4: parameter s%10 of mixture component g + 4 (s/10), which is
// head output 10 (s%10) + component. Returns -1 for padding rows.
NXHD int head_row_src(int r) {
  const int mt = r / 16, g = (r % 16) / 4, v = r % 4;
  const int s = 4 * mt + v, m = g + 4 * (s / 10), p = s % 10;
  return (s < 30 && m < NMIX) ? 10 * p + m : -1;
}
// inverse of head_row_src
NXHD int head_row_of(int src) {
  const int p = src / 10, m = src % 10;
  const int s = 10 * (m / 4) + p, g = m % 4;
  return 16 * (s / 4) + 4 * g + (s % 4);
}

// Source of weight-image float idx in the parameter vector, or -1 (zero).
// C = model channels, Cp = C rounded up to 16 (the image's channel count).
NXHD int64_t wimg_src(int h, int C, int Cp, int nb, int64_t idx) {
  const WeightLayout L = weight_layout(h, Cp, nb);
  const ParamLayout P = param_layout(h, C, nb);
  const int MT = Cp / 16, K = 2 * h + 1, KQ = conv_quads(h), KC = conv_chunks(h);
  if (idx < 0 || idx >= L.total) return -1;
  if (idx < L.layer0) {
    const int q = (int)(idx % 4), lane = (int)((idx / 4) % 64), kq = (int)((idx / 256) % KQ);
    const int mt = (int)(idx / (256 * (int64_t)KQ));
    const int kc = 4 * kq + q, o = 16 * mt + (lane & 15), k = 4 * kc + (lane >> 4);
    if (kc >= KC || o >= C) return -1;
    int dy, dx;
    tap_of(h, k / 3, dy, dx);
    return P.conv_w + (((int64_t)o * 3 + k % 3) * K + dy) * K + dx;
  }
  if (idx < L.bias_conv) {
    const bool head = idx >= L.head;
    const int64_t rel = head ? idx - L.head : (idx - L.layer0) % L.layer_stride;
    const int q = (int)(rel % 4), lane = (int)((rel / 4) % 64), ct = (int)((rel / 256) % MT);
    const int mt = (int)(rel / (256 * (int64_t)MT));
    const int row = 16 * mt + (lane & 15), col = 16 * ct + 4 * (lane >> 4) + q;
    if (col >= C) return -1;
    if (head) {
      const int src = head_row_src(row);
      return src < 0 ? -1 : P.head_w + (int64_t)src * C + col;
    }
    if (row >= C) return -1;
    const int64_t layer = (idx - L.layer0) / L.layer_stride;
    return P.blocks + (layer / 2) * P.block_stride + (layer % 2) * ((int64_t)C * C + C) + (int64_t)row * C + col;
  }
  if (idx < L.bias_blocks) {
    const int o = (int)(idx - L.bias_conv);
    return o < C ? P.conv_b + o : -1;
  }
  if (idx < L.bias_head) {
    const int64_t rel = idx - L.bias_blocks, layer = rel / Cp;
    const int o = (int)(rel % Cp);
    return o < C ? P.blocks + (layer / 2) * P.block_stride + (layer % 2) * ((int64_t)C * C + C) + (int64_t)C * C + o
                 : -1;
  }
  const int src = head_row_src((int)(idx - L.bias_head));
  return src < 0 ? -1 : P.head_b + src;
}

// Transposed weight image for the backward pass (input gradients of the 1x1
// layers and the head): with the forward's D layout as the B operand, the
// A operand of output tile ct (input channels) and K-chunk (mt, v) is
//   [ct][mt][lane][v] = W[16 mt + 4 (lane/16) + v][16 ct + lane%16]
// per 1x1 layer (2 nb of them), then the head (8 row tiles, permuted rows).
struct WeightTLayout {
  int64_t layer0, layer_stride, head, total;
};
NXHD constexpr WeightTLayout weightT_layout(int Cp, int nb) {
  WeightTLayout T{};
  const int64_t mt = Cp / 16;
  T.layer0 = 0;
  T.layer_stride = mt * mt * 256;
  T.head = 2 * (int64_t)nb * T.layer_stride;
  T.total = T.head + mt * HEAD_TILES * 256;
  return T;
}

NXHD int64_t wimgT_src(int h, int C, int Cp, int nb, int64_t idx) {
  const WeightTLayout T = weightT_layout(Cp, nb);
  const ParamLayout P = param_layout(h, C, nb);
  const int MT = Cp / 16;
  if (idx < 0 || idx >= T.total) return -1;
  const bool head = idx >= T.head;
  const int64_t rel = head ? idx - T.head : idx % T.layer_stride;
  const int KT = head ? HEAD_TILES : MT;  // K-chunk tiles (forward output tiles)
  const int v = (int)(rel % 4), lane = (int)((rel / 4) % 64), mt = (int)((rel / 256) % KT);
  const int ct = (int)(rel / (256 * (int64_t)KT));
  const int row = 16 * mt + 4 * (lane >> 4) + v, col = 16 * ct + (lane & 15);
  if (col >= C) return -1;
  if (head) {
    const int src = head_row_src(row);
    return src < 0 ? -1 : P.head_w + (int64_t)src * C + col;
  }
  if (row >= C) return -1;
  const int64_t layer = idx / T.layer_stride;
  return P.blocks + (layer / 2) * P.block_stride + (layer % 2) * ((int64_t)C * C + C) + (int64_t)row * C + col;
}

}  // namespace nx
