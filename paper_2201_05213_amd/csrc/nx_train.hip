// nx_train.hip -- the model's code length (Eq. 2 with the local model of
// Eq. 3) as a training objective, and its hand-written gradient, for gfx950.
//
//   k_swizzle      parameter vector -> forward / transposed weight images
//   k_train_fwd    per 16-pixel tile: causal gather, network (the same
//                  net_forward as the coder), joint mixture log-likelihood;
//                  saves the conv inputs, every layer input and the head rows
//   k_train_bwd    per tile: d bits / d head rows (mixture backward), then the
//                  deltas of every layer through the transposed weights
//   k_wgrad        per (layer, pixel chunk), every layer in one launch:
//                  dW = sum_px delta (x) input and db = sum_px delta on
//                  MFMA, one partial per chunk
//   k_grad_reduce  sums the chunk partials in a fixed order into the
//                  parameter vector's layout (deterministic)
//   k_bits_img     per image: sum of per-pixel bits in FP64
//
// Pixel tensors in the workspace are pixel-major: [pixel][channel].
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <atomic>

#include "nx_device.hpp"
#include "nx_kernels.hpp"

namespace nx {

constexpr int TRAIN_WAVES = 16;  // waves per workgroup of the per-tile kernels

// ------------------------------------------------------------------ mixture backward
// log P of bin x (as log_bin) and its partial derivatives in the mean and in
// the inverse scale. Interior bins: log P = log sig(z_hi) + log sig(-z_lo)
// + log(1 - exp(-d)), z = (edge - mu) is, d = (2/255) is, so
//   d/dmu = -is (sig(-z_hi) - sig(z_lo)),
//   d/dis = (e_hi - mu) sig(-z_hi) - (e_lo - mu) sig(z_lo) + (2/255) / expm1(d).
NXD float log_bin_grad(int x, float mu, float is, float& dmu, float& dis) {
  if (x <= 0) {
    const float e = bin_edge(1), z = (e - mu) * is, sg = xsigmoid(-z);
    dmu = -is * sg;
    dis = (e - mu) * sg;
    return xlogsigmoid(z);
  }
  if (x >= 255) {
    const float e = bin_edge(255), z = (e - mu) * is, sg = xsigmoid(z);
    dmu = is * sg;
    dis = -(e - mu) * sg;
    return xlogsigmoid(-z);
  }
  const float elo = bin_edge(x), ehi = bin_edge(x + 1);
  const float zlo = (elo - mu) * is, zhi = (ehi - mu) * is;
  const float d = is * (2.0f / 255.0f);
  const float sh = xsigmoid(-zhi), sl = xsigmoid(zlo);
  dmu = -is * (sh - sl);
  dis = ((ehi - mu) * sh - (elo - mu) * sl) + (2.0f / 255.0f) / xexpm1(d);
  return (xlogsigmoid(zhi) + xlogsigmoid(-zlo)) + xlog(-xexpm1(-d));
}

// Joint log-likelihood of one pixel, log sum_m w_m P_m(r) P_m(g|r) P_m(b|r,g)
// (natural log), over this lane's mixture slots (layout of mix_prep). With
// GRAD it also writes d(scale * bits)/d(head row) in the head
// layout, bits = -log p / ln 2: the responsibilities r_m = w_m prod_c P_cm / p
// give d log p / d logit_m = r_m - w_m and d log p / d log P_cm = r_m.
template <bool GRAD>
NXD float mix_joint(const f4 (&hd)[HEAD_TILES], const int (&xv)[3], bool has2, float scale, f4 (&dh)[HEAD_TILES]) {
  const float xr = normalise(xv[0]), xg = normalise(xv[1]);
  float lam[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) lam[j] = head_slot(hd, 10 * j);
  if (!has2) lam[2] = -INFINITY;
  const float lse = lse10(lam, has2);
  float L[3], gmu[3][3], gis[3][3], is[3][3], co[3][3], rho[3][3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
#pragma unroll
    for (int c = 0; c < 3; ++c) co[c][j] = xtanh(head_slot(hd, 10 * j + 7 + c));
    float mu[3];
    mu[0] = head_slot(hd, 10 * j + 1);
    mu[1] = head_slot(hd, 10 * j + 2) + co[0][j] * xr;
    mu[2] = (head_slot(hd, 10 * j + 3) + co[1][j] * xr) + co[2][j] * xg;
    float lp[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      rho[c][j] = head_slot(hd, 10 * j + 4 + c);
      is[c][j] = xexp(-fmaxf(rho[c][j], -7.0f));
      lp[c] = log_bin_grad(xv[c], mu[c], is[c][j], gmu[c][j], gis[c][j]);
    }
    L[j] = (lam[j] - lse) + ((lp[0] + lp[1]) + lp[2]);
  }
  if (!has2) L[2] = -INFINITY;
  const float logp = lse10(L, has2);
  if (GRAD) {
    const float s2 = -scale * kLog2e;  // d(scale * bits)/d log p
#pragma unroll
    for (int t = 0; t < HEAD_TILES; ++t) dh[t] = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      if (j == 2 && !has2) continue;
      const float r = xexp(L[j] - logp), w = xexp(lam[j] - lse);
      float v[10];
      v[0] = s2 * (r - w);
      float dmu[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        dmu[c] = s2 * r * gmu[c][j];
        const float dis = s2 * r * gis[c][j];
        v[1 + c] = dmu[c];
        v[4 + c] = rho[c][j] >= -7.0f ? -is[c][j] * dis : 0.0f;
      }
      // mu_G += alpha x_R, mu_B += beta x_R + gamma x_G, coefficients = tanh(raw)
      v[7] = dmu[1] * xr * (1.0f - co[0][j] * co[0][j]);
      v[8] = dmu[2] * xr * (1.0f - co[1][j] * co[1][j]);
      v[9] = dmu[2] * xg * (1.0f - co[2][j] * co[2][j]);
#pragma unroll
      for (int q = 0; q < 10; ++q) {
        const int s = 10 * j + q;
        dh[s >> 2][s & 3] = v[q];
      }
    }
  }
  return logp;
}

// ------------------------------------------------------------------ weight images
__global__ void k_swizzle(const float* __restrict__ params, int h, int C, int Cp, int nb, float* wimg, int64_t nw,
                          float* wimgT, int64_t nwT) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nw + nwT; i += stride) {
    if (i < nw) {
      const int64_t s = wimg_src(h, C, Cp, nb, i);
      wimg[i] = s >= 0 ? params[s] : 0.0f;
    } else {
      const int64_t s = wimgT_src(h, C, Cp, nb, i - nw);
      wimgT[i - nw] = s >= 0 ? params[s] : 0.0f;
    }
  }
}

// ------------------------------------------------------------------ per-tile kernels
struct TileCoord {
  int n, y, x;
  bool active;
  int64_t pix;   // global pixel index (clamped into the image row when inactive)
};

NXD TileCoord tile_coord(const TrainArgs& A, int64_t t, int p) {
  TileCoord T;
  const int64_t per_img = (int64_t)A.H * A.ntx;
  T.n = (int)(t / per_img);
  const int64_t r = t - (int64_t)T.n * per_img;
  T.y = (int)(r / A.ntx);
  const int xraw = (int)(r - (int64_t)T.y * A.ntx) * 16 + p;
  T.active = xraw < A.W;
  T.x = T.active ? xraw : A.W - 1;
  T.pix = ((int64_t)T.n * A.H + T.y) * A.W + T.x;
  return T;
}

// stores the layer inputs u (D layout) pixel-major
struct USink {
  float* u;
  int64_t npx, pix;
  int Cp, g;
  bool active;
  template <int N>
  NXD void operator()(int l, const f4 (&a)[N]) const {
    if (!active) return;
    float* dst = u + ((int64_t)l * npx + pix) * Cp + 4 * g;
#pragma unroll
    for (int mt = 0; mt < N; ++mt) *(f4*)(dst + 16 * mt) = a[mt];
  }
};

template <int H_, int C_>
__global__ void __launch_bounds__(TRAIN_WAVES * 64) k_train_fwd(TrainArgs A) {
  extern __shared__ float4 smem_f4[];
  float* w = (float*)smem_f4;
  // the weight image goes to LDS while the first tile's context is gathered;
  // every wave passes the one barrier once, after its first gather or, with
  // no tile, at the end
  const int64_t n4 = A.wfloats >> 2;
  for (int64_t i = threadIdx.x; i < n4; i += TRAIN_WAVES * 64) ((float4*)w)[i] = ((const float4*)A.wimg)[i];
  bool synced = false;
  constexpr int KC = conv_chunks(H_);
  const int lane = threadIdx.x & 63, p = lane & 15, g = lane >> 4;
  const bool has2 = g < 2;
  const int64_t gw = (int64_t)blockIdx.x * TRAIN_WAVES + (threadIdx.x >> 6);
  const int64_t nwv = (int64_t)gridDim.x * TRAIN_WAVES;
  TapCodes<H_> tc;
  tc.init(g);
  for (int64_t t = gw; t < A.n_tiles; t += nwv) {
    tc.refresh();
    const TileCoord T = tile_coord(A, t, p);
    const uint8_t* img = A.imgs + (int64_t)T.n * A.H * A.W * 3;
    float ctx[KC];
    gather<H_>(ctx, tc, img, A.W, 0, 0, A.H, A.W, T.y, T.x, T.active);
    if (!synced) {
      __syncthreads();
      synced = true;
    }
    if (T.active) {
      float* cd = A.ctx + T.pix * A.KP;
#pragma unroll
      for (int kc = 0; kc < KC; ++kc) cd[4 * kc + g] = ctx[kc];
      for (int k = 4 * KC + g; k < A.KP; k += 4) cd[k] = 0.0f;
    }
    f4 head[HEAD_TILES];
    const USink sink{A.u, A.npx, T.pix, A.Cp, g, T.active};
    net_forward<H_, C_>(lds_weights(w), A.nb, ctx, head, lane, sink);
    if (T.active) {
      float* th = A.theta + T.pix * (16 * HEAD_TILES) + 4 * g;
#pragma unroll
      for (int mt = 0; mt < HEAD_TILES; ++mt) *(f4*)(th + 16 * mt) = head[mt];
    }
    const uint8_t* px = img + ((int64_t)T.y * A.W + T.x) * 3;
    const int xv[3] = {px[0], px[1], px[2]};
    f4 unused[HEAD_TILES];
    const float lp = mix_joint<false>(head, xv, has2, 0.0f, unused);
    if (T.active && g == 0) A.bits[T.pix] = -lp * kLog2e;
  }
  if (!synced) __syncthreads();
}

NXD f4 elu_grad(const f4& d, const f4& u) {
  f4 r;
#pragma unroll
  for (int v = 0; v < 4; ++v) r[v] = d[v] * (u[v] > 0.0f ? 1.0f : u[v] + 1.0f);
  return r;
}

template <int MT>
NXD void load_pm(f4 (&a)[MT], const float* base, int64_t pix, int ld, int g) {
  const float* s = base + pix * ld + 4 * g;
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) a[mt] = *(const f4*)(s + 16 * mt);
}

template <int MT>
NXD void store_pm(float* base, int64_t pix, int ld, int g, const f4 (&a)[MT]) {
  float* s = base + pix * ld + 4 * g;
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) *(f4*)(s + 16 * mt) = a[mt];
}

template <int H_, int C_>
__global__ void __launch_bounds__(TRAIN_WAVES * 64) k_train_bwd(TrainArgs A) {
  extern __shared__ float4 smem_f4[];
  float* w = (float*)smem_f4;
  {
    const int64_t n4 = A.wTfloats >> 2;
    for (int64_t i = threadIdx.x; i < n4; i += TRAIN_WAVES * 64) ((float4*)w)[i] = ((const float4*)A.wimgT)[i];
    __syncthreads();
  }
  constexpr int MT = C_ / 16;
  const WeightTLayout TL = weightT_layout(C_, A.nb);
  const int lane = threadIdx.x & 63, p = lane & 15, g = lane >> 4;
  const bool has2 = g < 2;
  const int64_t gw = (int64_t)blockIdx.x * TRAIN_WAVES + (threadIdx.x >> 6);
  const int64_t nwv = (int64_t)gridDim.x * TRAIN_WAVES;
  for (int64_t t = gw; t < A.n_tiles; t += nwv) {
    const TileCoord T = tile_coord(A, t, p);
    const float* wl = lds_weights(w);
    f4 hd[HEAD_TILES];
    load_pm(hd, A.theta, T.pix, 16 * HEAD_TILES, g);
    const uint8_t* px = A.imgs + T.pix * 3;
    const int xv[3] = {px[0], px[1], px[2]};
    f4 dh[HEAD_TILES];
    mix_joint<true>(hd, xv, has2, A.grad_bits[T.n], dh);
    if (!T.active) {
#pragma unroll
      for (int mt = 0; mt < HEAD_TILES; ++mt) dh[mt] = f4{0.0f, 0.0f, 0.0f, 0.0f};
    }
    if (T.active) store_pm(A.dtheta, T.pix, 16 * HEAD_TILES, g, dh);
    // head: d elu(a) = Wh^T dtheta
    f4 d[MT], u[MT], da[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) d[mt] = f4{0.0f, 0.0f, 0.0f, 0.0f};
    layer_mm<MT, HEAD_TILES>(wl + TL.head, dh, d, lane);
    load_pm(u, A.u + (int64_t)(2 * A.nb) * A.npx * C_, T.pix, C_, g);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) da[mt] = elu_grad(d[mt], u[mt]);
    for (int b = A.nb - 1; b >= 0; --b) {
      // a_{b+1} = a_b + W2 elu(z1) + b2,  z1 = W1 elu(a_b) + b1
      if (T.active) store_pm(A.delta + (int64_t)(2 * b + 2) * A.npx * C_, T.pix, C_, g, da);
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) d[mt] = f4{0.0f, 0.0f, 0.0f, 0.0f};
      layer_mm<MT, MT>(wl + TL.layer0 + (int64_t)(2 * b + 1) * TL.layer_stride, da, d, lane);
      load_pm(u, A.u + (int64_t)(2 * b + 1) * A.npx * C_, T.pix, C_, g);
      f4 dz[MT];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) dz[mt] = elu_grad(d[mt], u[mt]);
      if (T.active) store_pm(A.delta + (int64_t)(2 * b + 1) * A.npx * C_, T.pix, C_, g, dz);
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) d[mt] = f4{0.0f, 0.0f, 0.0f, 0.0f};
      layer_mm<MT, MT>(wl + TL.layer0 + (int64_t)(2 * b) * TL.layer_stride, dz, d, lane);
      load_pm(u, A.u + (int64_t)(2 * b) * A.npx * C_, T.pix, C_, g);
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) da[mt] = da[mt] + elu_grad(d[mt], u[mt]);
    }
    if (T.active) store_pm(A.delta, T.pix, C_, g, da);
  }
}

// ------------------------------------------------------------------ weight gradients
// One launch for every layer: one workgroup per (layer, chunk of pixels)
// computes D[row][col] = sum_px delta[px][row] in[px][col] on
// v_mfma_f32_16x16x4f32 with K = 4 pixels per instruction (A[i][k] = delta of
// pixel k, B[k][j] = input of pixel k), and the bias gradient
// sum_px delta[px][row] from the same A values.
//
// Operand rows come in with 16-byte loads: for a width of 16 T channels, lane
// (i, k) loads channels 64 b + 4 i .. 64 b + 4 i + 3 of its pixel for each
// 64-channel block b < T / 4, and they feed tiles 4 b .. 4 b + 3 (tile 4 b + u
// row i is channel 64 b + 4 i + u); the tiles past 4 (T / 4) take channel
// 16 t + i with one 4-byte load. So a wave instruction reads four pixels' 256
// contiguous bytes, and the output is mapped back to channels when stored.
//
// The chunk's K-steps go to the WGRAD_WAVES waves in turn. Each wave streams
// its operands through a ring of WGRAD_DEPTH + 1 K-step slots
// in LDS with direct global-to-LDS loads, WGRAD_DEPTH K-steps ahead of its
// MFMAs, so the loads in flight cost no registers; it waits for a slot with
// an explicit vmcnt (the compiler does not track these loads' LDS writes)
// and refills the slot it read one step earlier, whose LDS reads are known to
// be complete. The waves' sums are added in LDS in wave order, one row tile
// at a time, so the result does not depend on timing.
constexpr int WGRAD_WAVES = 4;
constexpr int WGRAD_DEPTH = 7;  // K-steps (4 pixels each) in flight per wave

// LDS floats of one K-step slot of an MO x KI layer: its delta, then its input
constexpr int wgrad_slot(int MO, int KI) { return (MO + KI) * 64; }

// s_waitcnt immediate that waits until at most n vector memory operations
// are outstanding (expcnt and lgkmcnt left alone)
constexpr int vmcnt_imm(int n) { return (n & 15) | ((n >> 4) << 14) | (7 << 4) | (15 << 8); }

// channel of row r of tile t of a 16 T-wide operand, as the loads place it
NXD int op_channel(int T, int t, int r) {
  return t < 4 * (T / 4) ? 64 * (t >> 2) + 4 * r + (t & 3) : 16 * t + r;
}

// tile and row holding channel c (inverse of op_channel)
NXD void op_tile(int T, int c, int& t, int& r) {
  if (c < 64 * (T / 4)) {
    t = 4 * (c >> 6) + (c & 3);
    r = (c & 63) >> 2;
  } else {
    t = c >> 4;
    r = c & 15;
  }
}

#define NX_LDS(p) ((__attribute__((address_space(3))) void*)(p))

// direct loads of the T operand values of lane l = (i, k) for the pixel row
// at base + row (base wave-uniform, row a 32-bit offset in floats) into the
// LDS block dst (wave-uniform): the 16-byte parts first (lane l's four
// channels of block b at dst + 256 b + 4 l), then the 4-byte parts (tile t
// at dst + 256 (T / 4) + 64 (t - 4 (T / 4)) + l)
template <int T>
NXD void op_issue(const float* __restrict__ base, uint32_t row, int i, float* dst) {
#pragma unroll
  for (int b = 0; b < T / 4; ++b)
    __builtin_amdgcn_global_load_lds(base + (row + 64 * b + 4 * i), NX_LDS(dst + 256 * b), 16, 0, 0);
#pragma unroll
  for (int t = 4 * (T / 4); t < T; ++t)
    __builtin_amdgcn_global_load_lds(base + (row + 16 * t + i), NX_LDS(dst + 256 * (T / 4) + 64 * (t - 4 * (T / 4))),
                                     4, 0, 0);
}

// load instructions per operand block of op_issue
constexpr int op_loads(int T) { return T / 4 + T % 4; }

// lane l's T operand values from an LDS block written by op_issue
template <int T>
NXD void op_read(const float* src, int lane, float (&v)[T]) {
#pragma unroll
  for (int b = 0; b < T / 4; ++b) {
    const f4 x = *reinterpret_cast<const f4*>(src + 256 * b + 4 * lane);
#pragma unroll
    for (int u = 0; u < 4; ++u) v[4 * b + u] = x[u];
  }
#pragma unroll
  for (int t = 4 * (T / 4); t < T; ++t) v[t] = src[256 * (T / 4) + 64 * (t - 4 * (T / 4)) + lane];
}

template <int MO, int KI>
NXD void wgrad_layer(const WgradArgs& A, const WgradLayer& Lr, float* sm) {
  const int64_t c = blockIdx.x;
  const int64_t cl = c * A.chunk;
  const int64_t ch = cl + A.chunk < A.npx ? cl + A.chunk : A.npx;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform: scalar loop bounds
  const int lane = threadIdx.x & 63, i = lane & 15, k = lane >> 4;
  // the chunk's K-steps (4 pixels each) go to the waves in turn: wave w
  // takes K-steps w, w + 4, ..., so the workgroup reads its rows front to
  // back as one stream
  const int nk = (int)((ch - cl + 3) / 4);
  const int nsteps = nk > wv ? (nk - wv + WGRAD_WAVES - 1) / WGRAD_WAVES : 0;
  f4 acc[MO][KI];
  float bacc[MO];
#pragma unroll
  for (int mt = 0; mt < MO; ++mt) {
    bacc[mt] = 0.0f;
#pragma unroll
    for (int kt = 0; kt < KI; ++kt) acc[mt][kt] = f4{0.0f, 0.0f, 0.0f, 0.0f};
  }
  // this wave's step st holds pixels cl + 4 (4 st + w) + k (past the chunk:
  // its first pixel's rows, zeroed once read); addresses are the chunk's
  // first rows (wave-uniform) plus 32-bit offsets
  constexpr int SLOT = wgrad_slot(MO, KI), RING = WGRAD_DEPTH + 1, L = op_loads(MO) + op_loads(KI);
  float* ring = sm + wv * RING * SLOT;
  const float* __restrict__ dbase = Lr.delta + cl * Lr.ld_delta;
  const float* __restrict__ ibase = Lr.in + cl * Lr.ld_in;
  const uint32_t ldd = (uint32_t)Lr.ld_delta, ldi = (uint32_t)Lr.ld_in;
  const int64_t span = ch - cl;
  auto issue = [&](int st) {
    int64_t p = 4 * (WGRAD_WAVES * (int64_t)st + wv) + k;
    if (p >= span) p = 0;
    const uint32_t rp = (uint32_t)p;
    float* slot = ring + (st % RING) * SLOT;
    op_issue<MO>(dbase, rp * ldd, i, slot);
    op_issue<KI>(ibase, rp * ldi, i, slot + MO * 64);
  };
  for (int st = 0; st < nsteps && st < WGRAD_DEPTH; ++st) issue(st);
  for (int st = 0; st < nsteps; ++st) {
    // step st's loads are the oldest outstanding: wait for them, and only
    // them while the ring is full
    if (st + WGRAD_DEPTH <= nsteps)
      __builtin_amdgcn_s_waitcnt(vmcnt_imm(L * (WGRAD_DEPTH - 1)));
    else
      __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");  // the LDS reads stay after the wait
    float fa[MO], fb[KI];
    const float* slot = ring + (st % RING) * SLOT;
    op_read<MO>(slot, lane, fa);
    op_read<KI>(slot + MO * 64, lane, fb);
    const int64_t p0 = 4 * (WGRAD_WAVES * (int64_t)st + wv);
    if (p0 + 4 > span) {
      const bool ok = p0 + k < span;
#pragma unroll
      for (int mt = 0; mt < MO; ++mt) fa[mt] = ok ? fa[mt] : 0.0f;
#pragma unroll
      for (int kt = 0; kt < KI; ++kt) fb[kt] = ok ? fb[kt] : 0.0f;
    }
    // refill the slot read one step ago (its LDS reads have completed: their
    // values fed that step's MFMAs)
    if (st + WGRAD_DEPTH < nsteps) issue(st + WGRAD_DEPTH);
#pragma unroll
    for (int mt = 0; mt < MO; ++mt) {
      bacc[mt] += fa[mt];
#pragma unroll
      for (int kt = 0; kt < KI; ++kt)
        acc[mt][kt] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[mt], fb[kt], acc[mt][kt], 0, 0, 0);
    }
  }
  // the rings are reused below for the waves' sums
  __syncthreads();
  // per row tile mt: every wave parks its values in LDS (value e of lane l at
  // sm[(w E + e) 64 + l], e = 4 kt + v for the MFMA sums, e = 4 KI for the
  // bias), then the workgroup adds the waves in wave order and writes the
  // tile's 16 rows of the partial, a whole row of columns per 16 N threads
  constexpr int E = 4 * KI + 1, N = 16 * KI;
  float* out = A.partial + c * A.ngrad;
#pragma unroll
  for (int mt = 0; mt < MO; ++mt) {
    if (mt > 0) __syncthreads();
    float* dst = sm + (int64_t)wv * E * 64 + lane;
#pragma unroll
    for (int kt = 0; kt < KI; ++kt)
#pragma unroll
      for (int v = 0; v < 4; ++v) dst[(4 * kt + v) * 64] = acc[mt][kt][v];
    dst[4 * KI * 64] = bacc[mt];
    __syncthreads();
    for (int q = threadIdx.x; q < 16 * N + 16; q += WGRAD_WAVES * 64) {
      if (q < 16 * N) {
        // D[r][j] of tile (mt, kt) sits in value r & 3 of lane j + 16 (r >> 2)
        const int r = q / N, col = q - r * N;
        int kt, j;
        op_tile(KI, col, kt, j);
        const int e = 4 * kt + (r & 3), l = j + 16 * (r >> 2);
        float sum = sm[e * 64 + l];
#pragma unroll
        for (int w = 1; w < WGRAD_WAVES; ++w) sum = sum + sm[(w * E + e) * 64 + l];
        out[Lr.w_off + (int64_t)op_channel(MO, mt, r) * N + col] = sum;
      } else {
        // bias of row r: the waves in order, then the four pixel groups
        const int r = q - 16 * N;
        float bs = 0.0f;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          float b = sm[(4 * KI) * 64 + r + 16 * g];
#pragma unroll
          for (int w = 1; w < WGRAD_WAVES; ++w) b = b + sm[(w * E + 4 * KI) * 64 + r + 16 * g];
          bs = g == 0 ? b : bs + b;
        }
        out[Lr.b_off + op_channel(MO, mt, r)] = bs;
      }
    }
  }
}

// CT = C / 16 and KT = KP / 16 tiles; the layer's kind picks its shape:
// (CT, KT) for the first layer, (CT, CT) for the 1x1 layers,
// (HEAD_TILES / WGRAD_HEAD_PARTS, CT) for a part of the head
template <int CT, int KT>
__global__ void __launch_bounds__(WGRAD_WAVES * 64) k_wgrad(WgradArgs A) {
  extern __shared__ float4 wg_smem[];
  float* sm = (float*)wg_smem;
  const WgradLayer Lr = A.layer[blockIdx.y];
  if (Lr.kind == WGRAD_HEAD)
    wgrad_layer<HEAD_TILES / WGRAD_HEAD_PARTS, CT>(A, Lr, sm);
  else if (Lr.kind == WGRAD_FIRST)
    wgrad_layer<CT, KT>(A, Lr, sm);
  else
    wgrad_layer<CT, CT>(A, Lr, sm);
}

// gradient of parameter idx (blob order) = sum over chunks of its partial.
// A workgroup takes GR_PARAMS consecutive parameters; its GR_GROUPS thread
// groups each add one contiguous range of chunks in chunk order (FP64), and
// the ranges' sums are then added in range order, so the result does not
// depend on timing.
constexpr int GR_PARAMS = 64, GR_GROUPS = 4;

NXD int64_t grad_source(const GradReduceArgs& A, const ParamLayout& P, int64_t idx) {
  const int K = 2 * A.h + 1, C = A.C, Cp = A.Cp;
  int64_t src = -1;
  if (idx < P.conv_b) {
    const int64_t o = idx / (3 * K * K), r = idx % (3 * K * K);
    const int ch = (int)(r / (K * K)), dy = (int)((r / K) % K), dx = (int)(r % K);
    const int t = tap_index(A.h, dy, dx);
    if (t >= 0) src = A.off_conv + o * A.KP + 3 * t + ch;
  } else if (idx < P.blocks) {
    src = A.bias_conv + (idx - P.conv_b);
  } else if (idx < P.head_w) {
    const int64_t b = (idx - P.blocks) / P.block_stride, r = (idx - P.blocks) % P.block_stride;
    const int64_t cc = (int64_t)C * C;
    if (r < cc) src = A.off_blocks + (2 * b) * Cp * Cp + (r / C) * Cp + r % C;
    else if (r < cc + C) src = A.bias_blocks + (2 * b) * Cp + (r - cc);
    else if (r < 2 * cc + C) src = A.off_blocks + (2 * b + 1) * Cp * Cp + ((r - cc - C) / C) * Cp + (r - cc - C) % C;
    else src = A.bias_blocks + (2 * b + 1) * Cp + (r - 2 * cc - C);
  } else if (idx < P.head_b) {
    const int64_t r = idx - P.head_w;
    src = A.off_head + (int64_t)head_row_of((int)(r / C)) * Cp + r % C;
  } else {
    src = A.bias_head + head_row_of((int)(idx - P.head_b));
  }
  return src;
}

__global__ void __launch_bounds__(GR_PARAMS * GR_GROUPS) k_grad_reduce(GradReduceArgs A) {
  __shared__ double part[GR_GROUPS][GR_PARAMS];
  const ParamLayout P = param_layout(A.h, A.C, A.nb);
  const int q = threadIdx.x % GR_PARAMS, g = threadIdx.x / GR_PARAMS;
  const int64_t idx = (int64_t)blockIdx.x * GR_PARAMS + q;
  const int64_t src = idx < P.total ? grad_source(A, P, idx) : -1;
  const int64_t per = (A.nchunks + GR_GROUPS - 1) / GR_GROUPS;
  const int64_t c0 = g * per < A.nchunks ? g * per : A.nchunks;
  const int64_t c1 = c0 + per < A.nchunks ? c0 + per : A.nchunks;
  // this group's chunks in order, loaded 8 at a time so that many loads are
  // in flight
  double s = 0.0;
  if (src >= 0) {
    const float* col = A.partial + src;
    int64_t c = c0;
    for (; c + 8 <= c1; c += 8) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = col[(c + u) * A.ngrad];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += (double)v[u];
    }
    for (; c < c1; ++c) s += (double)col[c * A.ngrad];
  }
  part[g][q] = s;
  __syncthreads();
  if (g == 0 && idx < P.total) {
    double t = part[0][q];
#pragma unroll
    for (int r = 1; r < GR_GROUPS; ++r) t += part[r][q];
    A.grad[idx] = (float)t;
  }
}

// per image: sum of per-pixel bits in double, fixed order
__global__ void __launch_bounds__(256) k_bits_img(const float* bits, int64_t per_img, double* out) {
  __shared__ double part[256];
  const float* b = bits + (int64_t)blockIdx.x * per_img;
  double s = 0.0;
  for (int64_t k = threadIdx.x; k < per_img; k += 256) s += (double)b[k];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) part[threadIdx.x] += part[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = part[0];
}

// ------------------------------------------------------------------ launchers
// Raises a kernel's dynamic LDS limit on the current device. The attribute
// call is made again only when a launch needs more than the last call set,
// so once a kernel has run outside a stream capture, launches inside one
// make no such call.
constexpr int MAX_DEVICES = 64;

template <auto Kernel>
static hipError_t allow_lds_t(size_t lds) {
  static std::atomic<size_t> set[MAX_DEVICES];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) dev = -1;
  if (dev >= 0 && lds <= set[dev].load(std::memory_order_relaxed)) return hipSuccess;
  const hipError_t e = hipFuncSetAttribute((const void*)Kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) {
    (void)hipGetLastError();  // reported here, not by the next launch's check
    return e;
  }
  if (dev >= 0) {
    size_t cur = set[dev].load(std::memory_order_relaxed);
    while (cur < lds && !set[dev].compare_exchange_weak(cur, lds, std::memory_order_relaxed)) {
    }
  }
  return hipSuccess;
}

template <int H_, int C_>
static hipError_t train_fwd_t(const TrainArgs& a, int grid, hipStream_t s) {
  const size_t lds = (size_t)a.wfloats * 4;
  hipError_t e = allow_lds_t<k_train_fwd<H_, C_>>(lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_train_fwd<H_, C_>), dim3(grid), dim3(TRAIN_WAVES * 64), lds, s, a);
  return hipGetLastError();
}

template <int H_, int C_>
static hipError_t train_bwd_t(const TrainArgs& a, int grid, hipStream_t s) {
  const size_t lds = (size_t)a.wTfloats * 4;
  hipError_t e = allow_lds_t<k_train_bwd<H_, C_>>(lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_train_bwd<H_, C_>), dim3(grid), dim3(TRAIN_WAVES * 64), lds, s, a);
  return hipGetLastError();
}

#define NX_TRAIN_DISPATCH(FN, h, C, ...)                    \
  do {                                                      \
    if (h == 3 && C == 64) return FN<3, 64>(__VA_ARGS__);   \
    if (h == 3 && C == 32) return FN<3, 32>(__VA_ARGS__);   \
    if (h == 3 && C == 16) return FN<3, 16>(__VA_ARGS__);   \
    if (h == 2 && C == 64) return FN<2, 64>(__VA_ARGS__);   \
    if (h == 2 && C == 32) return FN<2, 32>(__VA_ARGS__);   \
    if (h == 2 && C == 16) return FN<2, 16>(__VA_ARGS__);   \
    if (h == 1 && C == 32) return FN<1, 32>(__VA_ARGS__);   \
    if (h == 1 && C == 16) return FN<1, 16>(__VA_ARGS__);   \
    return hipErrorInvalidValue;                            \
  } while (0)

hipError_t launch_swizzle(const float* params, int h, int C, int Cp, int nb, float* wimg, int64_t nw, float* wimgT,
                          int64_t nwT, hipStream_t s) {
  // one element per thread: the index maps are a few divisions each
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((nw + nwT + 255) / 256, 4096));
  hipLaunchKernelGGL(k_swizzle, dim3((unsigned)blocks), dim3(256), 0, s, params, h, C, Cp, nb, wimg, nw, wimgT, nwT);
  return hipGetLastError();
}

hipError_t launch_train_fwd(int h, int Cp, const TrainArgs& a, int grid, hipStream_t s) {
  NX_TRAIN_DISPATCH(train_fwd_t, h, Cp, a, grid, s);
}

hipError_t launch_train_bwd(int h, int Cp, const TrainArgs& a, int grid, hipStream_t s) {
  NX_TRAIN_DISPATCH(train_bwd_t, h, Cp, a, grid, s);
}

// LDS of the weight-gradient kernel: every wave's ring of K-step slots, or
// one row tile's values of every wave, for the widest layer
static size_t wgrad_lds(int CT, int KT) {
  const int slot = std::max({wgrad_slot(CT, KT), wgrad_slot(CT, CT), wgrad_slot(HEAD_TILES / WGRAD_HEAD_PARTS, CT)});
  const size_t ring = (size_t)WGRAD_WAVES * (WGRAD_DEPTH + 1) * slot;
  const size_t sums = (size_t)WGRAD_WAVES * (4 * std::max(KT, CT) + 1) * 64;
  return std::max(ring, sums) * sizeof(float);
}

// (asked of the runtime once per shape; 0 is not kept, so a query made
// before a device is usable is repeated)
template <int CT, int KT>
static int wgrad_occupancy() {
  static std::atomic<int> known{0};
  int n = known.load(std::memory_order_relaxed);
  if (n > 0) return n;
  if (allow_lds_t<k_wgrad<CT, KT>>(wgrad_lds(CT, KT)) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_wgrad<CT, KT>, WGRAD_WAVES * 64, wgrad_lds(CT, KT)) !=
      hipSuccess)
    return 0;
  if (n > 0) known.store(n, std::memory_order_relaxed);
  return n;
}

int wgrad_blocks_per_cu(int CT, int KT) {
#define NX_WG(ct, kt) if (CT == ct && KT == kt) return wgrad_occupancy<ct, kt>()
  NX_WG(1, 1); NX_WG(1, 3); NX_WG(1, 5);
  NX_WG(2, 1); NX_WG(2, 3); NX_WG(2, 5);
  NX_WG(4, 1); NX_WG(4, 3); NX_WG(4, 5);
#undef NX_WG
  return 0;
}

template <int CT, int KT>
static hipError_t wgrad_t(const WgradArgs& a, int nlayers, hipStream_t s) {
  const size_t lds = wgrad_lds(CT, KT);
  hipError_t e = allow_lds_t<k_wgrad<CT, KT>>(lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_wgrad<CT, KT>), dim3((unsigned)a.nchunks, (unsigned)nlayers), dim3(WGRAD_WAVES * 64), lds, s,
                     a);
  return hipGetLastError();
}

// CT = C / 16 channel tiles, KT = KP / 16 first-layer input tiles
hipError_t launch_wgrad(int CT, int KT, const WgradArgs& a, int nlayers, hipStream_t s) {
  if (nlayers == 0 || a.nchunks == 0) return hipSuccess;
  if (nlayers > WGRAD_MAX_LAYERS) return hipErrorInvalidValue;
#define NX_WG(ct, kt) if (CT == ct && KT == kt) return wgrad_t<ct, kt>(a, nlayers, s)
  NX_WG(1, 1); NX_WG(1, 3); NX_WG(1, 5);
  NX_WG(2, 1); NX_WG(2, 3); NX_WG(2, 5);
  NX_WG(4, 1); NX_WG(4, 3); NX_WG(4, 5);
#undef NX_WG
  return hipErrorInvalidValue;
}

hipError_t launch_grad_reduce(const GradReduceArgs& a, hipStream_t s) {
  const ParamLayout P = param_layout(a.h, a.C, a.nb);
  const int64_t grid = (P.total + GR_PARAMS - 1) / GR_PARAMS;
  hipLaunchKernelGGL(k_grad_reduce, dim3((unsigned)grid), dim3(GR_PARAMS * GR_GROUPS), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_bits_img(const float* bits, int n, int64_t per_img, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_bits_img, dim3(n), dim3(256), 0, s, bits, per_img, out);
  return hipGetLastError();
}

}  // namespace nx
