// nx_device.hpp -- the fused per-pixel routine shared by every kernel that
// evaluates the model: causal gather, masked first layer, 1x1 residual blocks,
// head, mixture parameters, quantised CDF point evaluation, channel posterior.
//
// Determinism contract: the encoder's full-image pass and the decoder's
// wavefront/raster passes call exactly these functions, so their CDFs agree
// bit for bit. Everything is FP32 with a fixed operation order: the library is
// built with -ffp-contract=off, FMAs are written out where wanted, sums over
// mixture components use one fixed tree, and the exp/log/sigmoid used here are
// this file's own (hardware exp2/log2/rcp plus explicit range reduction).
//
// Wave layout ("transposed tile"): a wave evaluates 16 pixels at once. Lane
// l = p + 16 g holds pixel p (0..15) and lane group g (0..3). The network runs
// on v_mfma_f32_16x16x4f32 with A = weights (16 output rows x 4 inputs) and
// B = activations (4 inputs x 16 pixels), so the result D (16 output rows x
// 16 pixels) leaves row 16 mt + 4 g + v of pixel p in VGPR v of lane (p, g).
// Read as a B operand, VGPR q of tile ct supplies input channel 16 ct + 4 g + q
// of pixel p: layer outputs feed the next layer without any data movement.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nx_layout.hpp"

namespace nx {

typedef float f4 __attribute__((ext_vector_type(4)));

#define NXD __device__ __forceinline__

// ------------------------------------------------------------------ math
constexpr float kLog2e = 1.44269504088896341f;
constexpr float kLn2 = 0.693147180559945309f;
// exp(x) from the hardware exp2: rounding x log2(e) costs a relative error
// of at most |x| 2^-24 ln 2 (below 5e-6 for the |x| < 100 the model meets);
// exp(-inf) = 0, exp(+big) = +inf
NXD float xexp(float x) { return __builtin_amdgcn_exp2f(x * kLog2e); }

// natural log of x > 0 from the hardware log2
NXD float xlog(float x) { return __builtin_amdgcn_logf(x) * kLn2; }

// log(1 + u) for u >= 0, with the rounding of 1 + u compensated
// (log(v) * u / (v - 1), v = fl(1 + u); Goldberg 1991, Theorem 4), the
// quotient through the hardware reciprocal; no branch
NXD float xlog1p(float u) {
  const float v = 1.0f + u;
  const float d = v - 1.0f;
  const float r = xlog(v) * (u * __builtin_amdgcn_rcpf(d));
  return d == 0.0f ? u : r;
}

// exp(x) - 1: Taylor polynomial through x^9/9! for |x| < ln2/2, else
// exp - 1 (both evaluated, one selected: no branch)
NXD float xexpm1(float x) {
  float q = 2.75573192e-06f;                  // 1/9!
  q = __builtin_fmaf(q, x, 2.48015873e-05f);  // 1/8!
  q = __builtin_fmaf(q, x, 1.98412698e-04f);  // 1/7!
  q = __builtin_fmaf(q, x, 1.38888889e-03f);  // 1/6!
  q = __builtin_fmaf(q, x, 8.33333333e-03f);  // 1/5!
  q = __builtin_fmaf(q, x, 4.16666667e-02f);  // 1/4!
  q = __builtin_fmaf(q, x, 1.66666667e-01f);  // 1/3!
  q = __builtin_fmaf(q, x, 0.5f);             // 1/2!
  const float taylor = __builtin_fmaf(x * x, q, x);
  const float direct = xexp(x) - 1.0f;
  return __builtin_fabsf(x) < 0.34657359f ? taylor : direct;
}

NXD float xtanh(float x) {
  const float e = xexpm1(-2.0f * __builtin_fabsf(x));  // in (-1, 0]
  const float t = -e * __builtin_amdgcn_rcpf(e + 2.0f);
  return __builtin_copysignf(t, x);
}

// ELU with exp(x) - 1 from the hardware exp2 for x <= 0: the rounding of
// x log2(e) costs a relative error of at most |x| 2^-24 ln2 in exp(x), i.e.
// an absolute error below 3e-8 in the activation. For x > 0 the exponent is
// 0 and e = 0; for x <= 0, exp(x) - 1 >= x, so the larger of x and e is the
// activation (x itself where rounding put e below it, |x| < 2^-23)
NXD float xelu(float x) {
  const float e = __builtin_amdgcn_exp2f(fminf(x, 0.0f) * kLog2e) - 1.0f;
  return fmaxf(x, e);
}

// logistic sigmoid: monotone non-decreasing in z because the hardware exp2
// and reciprocal are monotone (nellox_debug_check_monotone scans every finite
// FP32 input of both on the device)
NXD float xsigmoid(float z) {
  float e = __builtin_amdgcn_exp2f(-z * kLog2e);
  return __builtin_amdgcn_rcpf(1.0f + e);
}

// log sigmoid(z) = min(z, 0) - log1p(exp(-|z|))
NXD float xlogsigmoid(float z) {
  return fminf(z, 0.0f) - xlog1p(xexp(-__builtin_fabsf(z)));
}

// normalised pixel value v/127.5 - 1 (exact numerator, rounded reciprocal)
NXD float normalise(int v) { return (float)(2 * v - 255) * (1.0f / 255.0f); }

// lower edge of bin k (1..255): (2k - 256)/255
NXD float bin_edge(int k) { return (float)(2 * k - 256) * (1.0f / 255.0f); }

// ------------------------------------------------------------------ lane group reductions
// A pixel's mixture is spread over its four lanes p + 16 g; these combine one
// value per lane group with a fixed tree (v0 + v1) + (v2 + v3). The exchanges
// use the gfx950 row swaps (VALU, no LDS round trip): permlane16_swap of a
// value with itself leaves every lane holding its own value and that of its
// partner row (0<->1, 2<->3), permlane32_swap that of its partner half (rows
// 0,1 <-> 2,3); the pair is combined in either order, and IEEE addition and
// max are commutative, so every lane of the pixel obtains the same bits.
NXD float grp_sum(float v) {
  const uint32_t u = __float_as_uint(v);
  const auto r = __builtin_amdgcn_permlane16_swap(u, u, false, false);
  const float s = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  const uint32_t w = __float_as_uint(s);
  const auto q = __builtin_amdgcn_permlane32_swap(w, w, false, false);
  return __uint_as_float(q[0]) + __uint_as_float(q[1]);
}
NXD float grp_max(float v) {
  const uint32_t u = __float_as_uint(v);
  const auto r = __builtin_amdgcn_permlane16_swap(u, u, false, false);
  const float s = fmaxf(__uint_as_float(r[0]), __uint_as_float(r[1]));
  const uint32_t w = __float_as_uint(s);
  const auto q = __builtin_amdgcn_permlane32_swap(w, w, false, false);
  return fmaxf(__uint_as_float(q[0]), __uint_as_float(q[1]));
}
// ------------------------------------------------------------------ gather
// Causal context of pixel (i, j) of a lane (a rect of Hl x Wl pixels at (y0, x0)
// of an image with row length W): input index k = 3 tap + ch over the taps in
// raster order (h rows of 2h+1, then h to the left in row i); lane group g
// gathers k = 4 kc + g for K-chunk kc. Outside the lane reads as 0.
// A lane's tap offsets are packed, one byte per K-chunk (dy | dx << 2 | ch << 5),
// into TapCodes once; unpacking them per pixel keeps them out of the register
// budget of the persistent loops.
template <int H_>
struct TapCodes {
  static constexpr int NW = (conv_chunks(H_) + 3) / 4;
  uint32_t w[NW];
  NXD void init(int g) {
    constexpr int K = 2 * H_ + 1;
#pragma unroll
    for (int t = 0; t < NW; ++t) w[t] = 0;
#pragma unroll
    for (int kc = 0; kc < conv_chunks(H_); ++kc) {
      const int k = 4 * kc + g;
      const int tap = k / 3, ch = k - 3 * (k / 3);
      const int dy = tap < H_ * K ? tap / K : H_;
      const int dx = tap < H_ * K ? tap - K * (tap / K) : tap - H_ * K;
      w[kc >> 2] |= (uint32_t)(dy | (dx << 2) | (ch << 5)) << (8 * (kc & 3));
    }
  }
  // an opaque copy per use: the unpacked offsets are not hoisted out of loops
  NXD void refresh() {
#pragma unroll
    for (int t = 0; t < NW; ++t) asm volatile("" : "+v"(w[t]));
  }
};

// global-memory view of a byte pointer (lets the compiler use global loads)
typedef const __attribute__((address_space(1))) uint8_t* gbytes;
NXD gbytes as_global(const uint8_t* p) { return (gbytes)p; }

// Every tap is loaded from a position clamped into the lane (always in
// bounds), then taps outside the lane are replaced by 0: no branch around the
// loads, so all of them are in flight together.
template <int H_>
NXD void gather(float (&ctx)[conv_chunks(H_)], const TapCodes<H_>& tc, const uint8_t* img, int W, int y0, int x0,
                int Hl, int Wl, int i, int j, bool active) {
  const gbytes gimg = as_global(img);
  uint32_t raw[conv_chunks(H_)];
#pragma unroll
  for (int kc = 0; kc < conv_chunks(H_); ++kc) {
    const uint32_t code = (tc.w[kc >> 2] >> (8 * (kc & 3))) & 0xffu;
    const int dy = (int)(code & 3u), dx = (int)((code >> 2) & 7u), ch = (int)(code >> 5);
    const int y = min(max(i - H_ + dy, 0), Hl - 1), x = min(max(j - H_ + dx, 0), Wl - 1);
    raw[kc] = gimg[((int64_t)(y0 + y) * W + (x0 + x)) * 3 + ch];
  }
#pragma unroll
  for (int kc = 0; kc < conv_chunks(H_); ++kc) {
    const uint32_t code = (tc.w[kc >> 2] >> (8 * (kc & 3))) & 0xffu;
    const int dy = (int)(code & 3u), dx = (int)((code >> 2) & 7u);
    const int y = i - H_ + dy, x = j - H_ + dx;
    // inside the lane, as a bit mask (no short-circuit, no branch)
    const int ok = -(int)(((unsigned)y < (unsigned)Hl) & ((unsigned)x < (unsigned)Wl) & (unsigned)active);
    // normalise() of the tap, with the numerator masked: padding is exactly 0
    const int num = (2 * (int)raw[kc] - 255) & ok;
    ctx[kc] = (float)num * (1.0f / 255.0f);
  }
}

// gather() shared by the NW waves of a workgroup that all need the same
// tile's contexts: wave wv loads and normalises the K-chunks kc = wv, wv + NW,
// ... (the same positions, clamps and masks as gather(), tap offsets computed
// from the chunk index), writes them to LDS (cb: 64 lanes x gather_stride
// floats), and after a barrier every wave reads all of them. Every wave of
// the workgroup must call it.
template <int H_>
constexpr int gather_stride() { return (conv_chunks(H_) + 3) / 4 * 4; }
template <int H_, int NW>
NXD void gather_shared(float (&ctx)[conv_chunks(H_)], const uint8_t* img, int W, int y0, int x0, int Hl, int Wl,
                       int i, int j, bool active, int wv, float* cb, int lane) {
  constexpr int KC = conv_chunks(H_), KW = 2 * H_ + 1, CS = gather_stride<H_>();
  const int g = lane >> 4;
  const gbytes gimg = as_global(img);
  float v[(KC + NW - 1) / NW];
#pragma unroll
  for (int k = 0; k < (KC + NW - 1) / NW; ++k) {
    const int kc = min(wv + NW * k, KC - 1);
    const int kk = 4 * kc + g, tap = kk / 3, ch = kk - 3 * tap;
    const int dy = tap < H_ * KW ? tap / KW : H_;
    const int dx = tap < H_ * KW ? tap - KW * dy : tap - H_ * KW;
    const int y = i - H_ + dy, x = j - H_ + dx;
    const int yc = min(max(y, 0), Hl - 1), xc = min(max(x, 0), Wl - 1);
    const uint32_t raw = gimg[((int64_t)(y0 + yc) * W + (x0 + xc)) * 3 + ch];
    const int ok = -(int)(((unsigned)y < (unsigned)Hl) & ((unsigned)x < (unsigned)Wl) & (unsigned)active);
    const int num = (2 * (int)raw - 255) & ok;
    v[k] = (float)num * (1.0f / 255.0f);
  }
#pragma unroll
  for (int k = 0; k < (KC + NW - 1) / NW; ++k)
    if (wv + NW * k < KC) cb[lane * CS + wv + NW * k] = v[k];
  __syncthreads();
#pragma unroll
  for (int kc = 0; kc < KC; ++kc) ctx[kc] = cb[lane * CS + kc];
}

// Context of pixel (i, t) of a lane from its sheared canvas window (Sec. 3.1,
// Algorithm 2): tap (dy, dx) of the causal kernel is row i - h + dy, sheared
// column t - h(h+2) + (h+1) dy + dx, always a column before t. The window
// holds the int16 numerators 2x - 255 with 0 off the lane, so no bounds test
// is needed and the value is the unsheared gather's, bit for bit. i must be
// a row of the lane (callers clamp inactive rows).
template <int H_>
NXD void gather_ring(float (&ctx)[conv_chunks(H_)], const TapCodes<H_>& tc, const int16_t* ring, int rows, int t,
                     int i, bool active) {
  constexpr int o = H_ + 1, Q = H_ * (H_ + 2);
  const __attribute__((address_space(1))) int16_t* g = (const __attribute__((address_space(1))) int16_t*)ring;
  int raw[conv_chunks(H_)];
#pragma unroll
  for (int kc = 0; kc < conv_chunks(H_); ++kc) {
    const uint32_t code = (tc.w[kc >> 2] >> (8 * (kc & 3))) & 0xffu;
    const int dy = (int)(code & 3u), dx = (int)((code >> 2) & 7u), ch = (int)(code >> 5);
    const int col = (t - Q + o * dy + dx) & (RING_COLS - 1);
    raw[kc] = g[(uint32_t)((col * 3 + ch) * rows + i + dy)];
  }
#pragma unroll
  for (int kc = 0; kc < conv_chunks(H_); ++kc) ctx[kc] = (float)(active ? raw[kc] : 0) * (1.0f / 255.0f);
}

// ------------------------------------------------------------------ network
// The weight image is never written after it is staged in LDS, so the
// compiler would hoist every weight read out of the persistent loops and try
// to keep the whole network in registers. An offset it cannot see through
// (always 0) keeps the reads next to their MFMAs.
NXD const float* lds_weights(const float* w) {
  int zero = 0;
  asm volatile("" : "+s"(zero));
  return w + zero;
}

// One 1x1 layer: out[mt] (pre-initialised with the bias) += W in, K-chunks in
// the order (ct, q) = (0,0), (0,1), ..., (C/16-1, 3).
template <int MT_OUT, int CT_IN>
NXD void layer_mm(const float* __restrict__ w, const f4 (&in)[CT_IN], f4 (&out)[MT_OUT], int lane) {
#pragma unroll
  for (int ct = 0; ct < CT_IN; ++ct) {
    f4 wv[MT_OUT];
#pragma unroll
    for (int mt = 0; mt < MT_OUT; ++mt) wv[mt] = *(const f4*)(w + (((int64_t)mt * CT_IN + ct) * 64 + lane) * 4);
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int mt = 0; mt < MT_OUT; ++mt)
        out[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(wv[mt][q], in[ct][q], out[mt], 0, 0, 0);
  }
}

template <int N>
NXD void bias_init(f4 (&a)[N], const float* __restrict__ b, int g) {
#pragma unroll
  for (int mt = 0; mt < N; ++mt)
#pragma unroll
    for (int v = 0; v < 4; ++v) a[mt][v] = b[16 * mt + 4 * g + v];
}

// Receives each post-activation tensor of the network (for the backward
// pass); the default discards them.
struct NoSink {
  template <int N>
  NXD void operator()(int, const f4 (&)[N]) const {}
};

// Network of a 16-pixel tile: head[8] receives the 128 (permuted) head rows.
// w points at the weight image (LDS). ctx is this lane's conv B operand.
// sink(l, u) sees the layer inputs u = elu(.) in order: l = 2b is the input of
// block b's first 1x1 layer, 2b + 1 of its second, 2 nb of the head.
template <int H_, int C_, class Sink = NoSink>
NXD void net_forward(const float* __restrict__ w, int nb, const float (&ctx)[conv_chunks(H_)], f4 (&head)[HEAD_TILES],
                     int lane, const Sink& sink = Sink()) {
  constexpr int MT = C_ / 16;
  constexpr int KC = conv_chunks(H_), KQ = conv_quads(H_);
  const WeightLayout L = weight_layout(H_, C_, 0);
  const int g = lane >> 4;
  const int64_t layer_stride = (int64_t)MT * MT * 256;
  const float* bias_conv = w + L.head + (int64_t)HEAD_TILES * MT * 256 + 2 * (int64_t)nb * layer_stride;
  const float* bias_blk = bias_conv + C_;
  const float* bias_head = bias_blk + 2 * (int64_t)nb * C_;
  const float* w_head = w + L.layer0 + 2 * (int64_t)nb * layer_stride;

  f4 a[MT];
  bias_init(a, bias_conv, g);
#pragma unroll
  for (int kq = 0; kq < KQ; ++kq) {
    f4 wv[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) wv[mt] = *(const f4*)(w + (((int64_t)mt * KQ + kq) * 64 + lane) * 4);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (4 * kq + q < KC) {
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
          a[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(wv[mt][q], ctx[4 * kq + q], a[mt], 0, 0, 0);
      }
    }
  }
  for (int b = 0; b < nb; ++b) {
    f4 u[MT], z[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int v = 0; v < 4; ++v) u[mt][v] = xelu(a[mt][v]);
    sink(2 * b, u);
    bias_init(z, bias_blk + (int64_t)(2 * b) * C_, g);
    layer_mm<MT, MT>(w + L.layer0 + (int64_t)(2 * b) * layer_stride, u, z, lane);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int v = 0; v < 4; ++v) u[mt][v] = xelu(z[mt][v]);
    sink(2 * b + 1, u);
    bias_init(z, bias_blk + (int64_t)(2 * b + 1) * C_, g);
    layer_mm<MT, MT>(w + L.layer0 + (int64_t)(2 * b + 1) * layer_stride, u, z, lane);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) a[mt] = a[mt] + z[mt];
  }
  f4 u[MT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int v = 0; v < 4; ++v) u[mt][v] = xelu(a[mt][v]);
  sink(2 * nb, u);
  bias_init(head, bias_head, g);
  layer_mm<HEAD_TILES, MT>(w_head, u, head, lane);
}

// The network of one 16-pixel tile computed by the NW waves of a workgroup
// together: wave wv computes the output tiles mt with mt % NW == wv of every
// layer and the head tiles likewise, and the activations each 1x1 layer
// reads are exchanged through LDS (xb: two buffers of C/16 tiles x 64 lanes x
// 4 floats, used in turn), so every wave holds all input tiles. Each output
// element is the chain of MFMAs net_forward computes for it, in the same k
// order, so the values are bitwise the same. The head rows go to
// hb[pixel * 128 + row] (the weight image's permuted row order). Every wave
// of the workgroup must call it: it holds barriers, and its last one makes
// hb readable by all.
template <int H_, int C_, int NW>
NXD void net_forward_split(const float* __restrict__ w, int nb, const float (&ctx)[conv_chunks(H_)], float* xb,
                           float* hb, int lane, int wv) {
  constexpr int MT = C_ / 16;
  constexpr int KC = conv_chunks(H_), KQ = conv_quads(H_);
  constexpr int MY = (MT + NW - 1) / NW;  // output tiles per wave (a wave may own none)
  constexpr int HY = HEAD_TILES / NW;
  static_assert(HEAD_TILES % NW == 0, "head tiles are dealt evenly");
  const WeightLayout L = weight_layout(H_, C_, 0);
  const int g = lane >> 4;
  const int64_t layer_stride = (int64_t)MT * MT * 256;
  const float* bias_conv = w + L.head + (int64_t)HEAD_TILES * MT * 256 + 2 * (int64_t)nb * layer_stride;
  const float* bias_blk = bias_conv + C_;
  const float* bias_head = bias_blk + 2 * (int64_t)nb * C_;
  const float* w_head = w + L.layer0 + 2 * (int64_t)nb * layer_stride;

  // out (pre-initialised with the bias) += W in for output tile mt of a
  // layer (or of the head): k-chunks in the order (ct, q), as layer_mm
  // (a wave's tile is one dependent MFMA chain, so the layer's weights are
  // all read from LDS before the chain starts)
  auto tile_mm = [&](const float* wl, const f4(&in)[MT], f4& out, int mt) {
    f4 wq[MT];
#pragma unroll
    for (int ct = 0; ct < MT; ++ct) wq[ct] = *(const f4*)(wl + (((int64_t)mt * MT + ct) * 64 + lane) * 4);
#pragma unroll
    for (int ct = 0; ct < MT; ++ct)
#pragma unroll
      for (int q = 0; q < 4; ++q) out = __builtin_amdgcn_mfma_f32_16x16x4f32(wq[ct][q], in[ct][q], out, 0, 0, 0);
  };
  int par = 0;
  auto share = [&](const f4(&u)[MY], f4(&in)[MT]) {
    float* X = xb + par * (MT * 256);
#pragma unroll
    for (int k = 0; k < MY; ++k) {
      const int mt = wv + NW * k;
      if (mt < MT) *(f4*)(X + ((int64_t)mt * 64 + lane) * 4) = u[k];
    }
    __syncthreads();
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) in[mt] = *(const f4*)(X + ((int64_t)mt * 64 + lane) * 4);
    par ^= 1;
  };

  f4 a[MY];
#pragma unroll
  for (int k = 0; k < MY; ++k) {
    const int mt = wv + NW * k;
    if (mt >= MT) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) a[k][v] = bias_conv[16 * mt + 4 * g + v];
    f4 wq[KQ];
#pragma unroll
    for (int kq = 0; kq < KQ; ++kq) wq[kq] = *(const f4*)(w + (((int64_t)mt * KQ + kq) * 64 + lane) * 4);
#pragma unroll
    for (int kq = 0; kq < KQ; ++kq)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (4 * kq + q < KC) a[k] = __builtin_amdgcn_mfma_f32_16x16x4f32(wq[kq][q], ctx[4 * kq + q], a[k], 0, 0, 0);
  }
  for (int b = 0; b < nb; ++b) {
    f4 u[MY], in[MT], z[MY];
#pragma unroll
    for (int k = 0; k < MY; ++k)
#pragma unroll
      for (int v = 0; v < 4; ++v) u[k][v] = xelu(a[k][v]);
    share(u, in);
#pragma unroll
    for (int k = 0; k < MY; ++k) {
      const int mt = wv + NW * k;
      if (mt >= MT) continue;
      const float* bb = bias_blk + (int64_t)(2 * b) * C_;
#pragma unroll
      for (int v = 0; v < 4; ++v) z[k][v] = bb[16 * mt + 4 * g + v];
      tile_mm(w + L.layer0 + (int64_t)(2 * b) * layer_stride, in, z[k], mt);
    }
#pragma unroll
    for (int k = 0; k < MY; ++k)
#pragma unroll
      for (int v = 0; v < 4; ++v) u[k][v] = xelu(z[k][v]);
    share(u, in);
#pragma unroll
    for (int k = 0; k < MY; ++k) {
      const int mt = wv + NW * k;
      if (mt >= MT) continue;
      const float* bb = bias_blk + (int64_t)(2 * b + 1) * C_;
#pragma unroll
      for (int v = 0; v < 4; ++v) z[k][v] = bb[16 * mt + 4 * g + v];
      tile_mm(w + L.layer0 + (int64_t)(2 * b + 1) * layer_stride, in, z[k], mt);
      a[k] = a[k] + z[k];
    }
  }
  f4 u[MY], in[MT];
#pragma unroll
  for (int k = 0; k < MY; ++k)
#pragma unroll
    for (int v = 0; v < 4; ++v) u[k][v] = xelu(a[k][v]);
  share(u, in);
#pragma unroll
  for (int k = 0; k < HY; ++k) {
    const int hm = wv + NW * k;
    f4 hd;
#pragma unroll
    for (int v = 0; v < 4; ++v) hd[v] = bias_head[16 * hm + 4 * g + v];
    tile_mm(w_head, in, hd, hm);
    *(f4*)(hb + (lane & 15) * 128 + 16 * hm + 4 * g) = hd;
  }
  __syncthreads();
}

// ------------------------------------------------------------------ mixture
// Head slot s = 4 mt + v of lane group g holds parameter s % 10 of component
// m = g + 4 (s / 10) (s < 30, m < 10): 0 logit, 1..3 means R,G,B,
// 4..6 raw log-scales R,G,B, 7..9 pre-tanh coefficients G|R, B|R, B|G.
// Lane groups 0,1 own three components, groups 2,3 own two (slot 2 unused).
struct Mix {
  float logw[3];       // current (posterior) log weights
  float mu[3][3];      // [channel][slot] base means
  float invs[3][3];    // [channel][slot] inverse scales
  float co[3][3];      // [coef][slot] tanh'd coefficients alpha, beta, gamma
};

NXD float head_slot(const f4 (&hd)[HEAD_TILES], int s) { return hd[s >> 2][s & 3]; }

// log-sum-exp over the ten components of one pixel (own slots, fixed tree)
NXD float lse10(const float (&t)[3], bool has2) {
  float m = fmaxf(t[0], t[1]);
  if (has2) m = fmaxf(m, t[2]);
  m = grp_max(m);
  float s = xexp(t[0] - m) + xexp(t[1] - m);
  s = s + (has2 ? xexp(t[2] - m) : 0.0f);
  s = grp_sum(s);
  return m + xlog(s);
}

NXD void mix_prep(const f4 (&hd)[HEAD_TILES], Mix& M, bool has2) {
  float lam[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) lam[j] = head_slot(hd, 10 * j);
  if (!has2) lam[2] = -INFINITY;
  const float lse = lse10(lam, has2);
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    M.logw[j] = lam[j] - lse;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      M.mu[c][j] = head_slot(hd, 10 * j + 1 + c);
      M.invs[c][j] = xexp(-fmaxf(head_slot(hd, 10 * j + 4 + c), -7.0f));
      M.co[c][j] = xtanh(head_slot(hd, 10 * j + 7 + c));
    }
  }
}

// Mixture of channel c given the normalised values of the earlier channels:
// weights, shifted means, inverse scales of this lane's slots, and the
// sigmoid coefficients a = s log2(e), b = mu a used by cdf_eval. (c may be a
// runtime value: the channel rows are selected, not indexed, so the mixture
// stays in registers.)
struct Chan {
  float w[3], mu[3], is[3], a[3], b[3];
};

NXD void chan_params(const Mix& M, int c, float xr, float xg, Chan& K) {
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    K.w[j] = xexp(M.logw[j]);
    const float is = c == 0 ? M.invs[0][j] : (c == 1 ? M.invs[1][j] : M.invs[2][j]);
    float m;
    if (c == 0) {
      m = M.mu[0][j];
    } else if (c == 1) {
      m = M.mu[1][j] + M.co[0][j] * xr;
    } else {
      const float t1 = M.co[1][j] * xr;
      const float t2 = M.co[2][j] * xg;
      m = (M.mu[2][j] + t1) + t2;
    }
    K.mu[j] = m;
    K.is[j] = is;
    K.a[j] = is * kLog2e;
    K.b[j] = m * K.a[j];
  }
}

// Mixture CDF at bin edge k (1..255):
//   F = sum_m w_m / (1 + 2^(b_m - B_k a_m)),  i.e. sum_m w_m sigmoid((B_k - mu_m) s_m),
// the sum taken per lane group over its slots in order, then across groups.
// The exponent is one fused multiply-add, monotone decreasing in k (a >= 0),
// and the hardware exp2 and reciprocal are monotone, so F is monotone in k.
// Every lane of a pixel must call this with the same k (lane-group swaps).
NXD float cdf_eval(int k, const float (&w)[3], const float (&a)[3], const float (&b)[3]) {
  const float e = bin_edge(k);
  float t[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const float x = __builtin_amdgcn_exp2f(__builtin_fmaf(-e, a[j], b[j]));
    t[j] = w[j] * __builtin_amdgcn_rcpf(1.0f + x);
  }
  const float s = (t[0] + t[1]) + t[2];
  return grp_sum(s);
}

// Quantised CDF value: k + floor(clamp(F, 0, 1) * (2^16 - 256)). Monotone in
// k whenever F is, with a step of at least 1 between consecutive symbols.
NXD uint32_t cdf_quant(int k, float F) {
  const float c = __builtin_amdgcn_fmed3f(F, 0.0f, 1.0f);
  return (uint32_t)k + (uint32_t)(c * 65280.0f);
}

// log probability of bin x under this lane's slots (Q: stable difference of
// logistic CDFs: log sig(z_hi) + log sig(-z_lo) + log(1 - exp(-(z_hi - z_lo))),
// with z_hi - z_lo = (2/255) s exactly in real arithmetic).
NXD float log_bin(int x, float mu, float is) {
  // both edge forms and the interior form, then a select (no branch)
  const float zlo = (bin_edge(min(max(x, 1), 255)) - mu) * is;
  const float zhi = (bin_edge(min(max(x + 1, 1), 255)) - mu) * is;
  const float d = is * (2.0f / 255.0f);
  const float lhi = xlogsigmoid(zhi), llo = xlogsigmoid(-zlo);
  const float mid = (lhi + llo) + xlog(-xexpm1(-d));
  return x <= 0 ? lhi : (x >= 255 ? llo : mid);
}

// Condition the weights on the coded value x of channel c (posterior for the
// next channel); returns the channel's natural-log probability.
NXD float posterior(Mix& M, int x, const float (&mu)[3], const float (&is)[3], bool has2) {
  float t[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) t[j] = M.logw[j] + log_bin(x, mu[j], is[j]);
  if (!has2) t[2] = -INFINITY;
  const float lse = lse10(t, has2);
#pragma unroll
  for (int j = 0; j < 3; ++j) M.logw[j] = t[j] - lse;
  return lse;
}

// ------------------------------------------------------------------ mixture, 16 lanes per pixel
// The row decoder's mixture phase gives each pixel a row of 16 lanes: lane m
// holds component m (m < 10; lanes 10..15 hold none and add nothing). The
// arithmetic of a component is the lane-group form's, and sums over the
// components take the same tree: lane g < 4 adds (t_g + t_{g+4}) + t_{g+8},
// then (s_0 + s_1) + (s_2 + s_3), so every value is bitwise the one the
// encoder and the other decoders compute. The tree runs on DPP row shifts
// (lane i reads lane i + n of its row; only lanes 0..3 use the sums), and
// row_newbcast hands lane 0's result to the whole row.
template <int CTRL>
NXD float dpp_row(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, true));
}
constexpr int DPP_SHL1 = 0x101, DPP_SHL2 = 0x102, DPP_SHL4 = 0x104, DPP_SHL8 = 0x108, DPP_BCAST0 = 0x150;
NXD float row_bcast0(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), DPP_BCAST0, 0xf, 0xf, false));
}
NXD float row16_sum(float t) {
  const float s = (t + dpp_row<DPP_SHL4>(t)) + dpp_row<DPP_SHL8>(t);
  const float u = s + dpp_row<DPP_SHL1>(s);
  return row_bcast0(u + dpp_row<DPP_SHL2>(u));
}
NXD float row16_max(float v) {
  v = fmaxf(v, dpp_row<DPP_SHL8>(v));
  v = fmaxf(v, dpp_row<DPP_SHL4>(v));
  v = fmaxf(v, dpp_row<DPP_SHL2>(v));
  v = fmaxf(v, dpp_row<DPP_SHL1>(v));
  return row_bcast0(v);
}
// lse10 over the row's live components (t of a lane without one is ignored)
NXD float lse16(float t, bool live) {
  const float m = row16_max(live ? t : -INFINITY);
  const float e = live ? xexp(t - m) : 0.0f;
  return m + xlog(row16_sum(e));
}

struct Mix16 {
  float logw;                  // posterior log weight of this lane's component
  float mu[3], invs[3], co[3];
};
// the weight image's head row of parameter k (0..9) of component m
NXD int head_row(int m, int k) {
  const int s = 10 * (m >> 2) + k;
  return 16 * (s >> 2) + 4 * (m & 3) + (s & 3);
}
// mix_prep for component m of the pixel whose 128 head rows are at hp
NXD void mix_prep16(const float* hp, int m, Mix16& M) {
  const bool live = m < 10;
  const int mm = live ? m : 0;
  const float lam = live ? hp[head_row(mm, 0)] : -INFINITY;
  M.logw = lam - lse16(lam, live);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    M.mu[c] = hp[head_row(mm, 1 + c)];
    M.invs[c] = xexp(-fmaxf(hp[head_row(mm, 4 + c)], -7.0f));
    M.co[c] = xtanh(hp[head_row(mm, 7 + c)]);
  }
}
struct Chan16 {
  float w, mu, is, a, b;
};
NXD void chan_params16(const Mix16& M, int c, float xr, float xg, Chan16& Q) {
  Q.w = xexp(M.logw);
  Q.is = c == 0 ? M.invs[0] : (c == 1 ? M.invs[1] : M.invs[2]);
  float m;
  if (c == 0) {
    m = M.mu[0];
  } else if (c == 1) {
    m = M.mu[1] + M.co[0] * xr;
  } else {
    const float t1 = M.co[1] * xr;
    const float t2 = M.co[2] * xg;
    m = (M.mu[2] + t1) + t2;
  }
  Q.mu = m;
  Q.a = Q.is * kLog2e;
  Q.b = m * Q.a;
}
NXD float cdf_eval16(int k, const Chan16& Q) {
  const float e = bin_edge(k);
  const float x = __builtin_amdgcn_exp2f(__builtin_fmaf(-e, Q.a, Q.b));
  return row16_sum(Q.w * __builtin_amdgcn_rcpf(1.0f + x));
}
NXD float posterior16(Mix16& M, int x, const Chan16& Q, bool live) {
  const float t = live ? M.logw + log_bin(x, Q.mu, Q.is) : -INFINITY;
  const float lse = lse16(t, live);
  M.logw = t - lse;
  return lse;
}

// ------------------------------------------------------------------ sampling
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): a counter-based
// generator of ten rounds; each round multiplies words 0 and 2 by two odd
// constants (full 128-bit products) and mixes the halves with words 1 and 3
// and the key, which steps by two Weyl increments between rounds. Here the
// counter is (n, 0, 0, 0) and the key (seed, 0).
NXD void philox4x64(uint64_t n, uint64_t seed, uint64_t (&o)[4]) {
  uint64_t x0 = n, x1 = 0, x2 = 0, x3 = 0, k0 = seed, k1 = 0;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t a = 0xD2E7470EE14C6C93ull, b = 0xCA5A826395121157ull;
    const uint64_t hi0 = __umul64hi(a, x0), lo0 = a * x0;
    const uint64_t hi1 = __umul64hi(b, x2), lo1 = b * x2;
    x0 = hi1 ^ x1 ^ k0;
    x1 = lo1;
    x2 = hi0 ^ x3 ^ k1;
    x3 = lo0;
    k0 += 0x9E3779B97F4A7C15ull;
    k1 += 0xBB67AE8584CAA73Bull;
  }
  o[0] = x0; o[1] = x1; o[2] = x2; o[3] = x3;
}

// the 16-bit uniform slots of the three channels of pixel (y, x) of a W-wide
// image: top 16 bits of words 0, 1, 2 of the block with counter y W + x
NXD void sample_slots(uint64_t seed, int W, int y, int x, uint32_t (&sl)[3]) {
  uint64_t o[4];
  philox4x64((uint64_t)y * (uint64_t)W + (uint64_t)x, seed, o);
  sl[0] = (uint32_t)(o[0] >> 48);
  sl[1] = (uint32_t)(o[1] >> 48);
  sl[2] = (uint32_t)(o[2] >> 48);
}

}  // namespace nx
