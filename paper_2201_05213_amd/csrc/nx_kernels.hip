// nx_kernels.hip -- HIP kernels for gfx950 (MI355X):
//   k_pass      full-image pass: every pixel's quantised CDF at its own value
//               (encoder symbols), or its continuous code length (NLL), or a
//               full CDF row (debug), 16 pixels per wave on MFMA
//   k_rans_enc  one thread per lane: rANS-encodes the lane's symbols in
//               reverse decode order into a private slot
//   k_lane_scan / k_img_scan / k_pack   container assembly
//   k_decode    persistent decoder: waves pop lanes from a queue and decode
//               them step by step (wavefront) or pixel by pixel (raster)
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <mutex>

#include "nx_device.hpp"
#include "nx_kernels.hpp"
#include "nx_order.hpp"

namespace nx {

constexpr int NWAVES = 16;      // waves per full-image-pass workgroup (all share the LDS weights)
constexpr int NWAVES_DEC = DECODE_WAVES;  // waves per decoder workgroup
constexpr int PIV_WORDS = 256;            // per decoder wave: 16 pixels x 16 pivot CDF values
constexpr int PRM_STRIDE = 36;            // floats per pixel: (w, a, b) of 12 component slots
constexpr int PRM_WORDS = 16 * PRM_STRIDE;  // per decoder wave: one channel's mixtures of 16 pixels
constexpr int WAVE_LDS_WORDS = PIV_WORDS + PRM_WORDS;
static_assert(DECODE_LDS_EXTRA == NWAVES_DEC * WAVE_LDS_WORDS * 4, "decoder LDS budget");

NXD int find_img(const ImgDesc* __restrict__ d, int n, int64_t key, bool by_lane) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    const int64_t b = by_lane ? d[mid].lane_base : d[mid].tile_base;
    if (b <= key) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// the image holding global stream `key` (by its first stream)
NXD int find_img_stream(const ImgDesc* __restrict__ d, int n, int64_t key) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (d[mid].stream_base <= key) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Where stream e of an image (its stream table entry) lies: its lane (q, and
// the patch row and column ly, lx), the lane's rows and columns, its index
// among the lane's streams (kk, K streams) or its row (r, row streams), the
// pixels of the lanes before it in lane order, and the end of its byte slot
// in the encoder's slot buffer (slots are laid out in entry order: with K
// streams, K slots of 6 B per lane pixel + 8 B per lane; with row streams,
// 6 B per row pixel + 8 B per row).
struct StreamAt {
  int q, ly, lx, Hl, Wl, kk, r;
  int64_t lane_px_off, slot_end;
};
NXD StreamAt stream_at(const ImgDesc& D, int K, int64_t e) {
  StreamAt S;
  if (K == ROW_STREAMS) {
    const int64_t per_prow = (int64_t)D.nlx * D.ph;  // entries of a full patch row
    S.ly = (int)(e / per_prow);
    S.Hl = min(D.ph, D.H - S.ly * D.ph);
    const int64_t rem = e - (int64_t)S.ly * per_prow;
    S.lx = (int)(rem / S.Hl);
    S.r = (int)(rem - (int64_t)S.lx * S.Hl);
    S.kk = 0;
  } else {
    const int q = (int)(e / K);
    S.kk = (int)(e - (int64_t)q * K);
    S.ly = q / D.nlx;
    S.lx = q - S.ly * D.nlx;
    S.Hl = min(D.ph, D.H - S.ly * D.ph);
    S.r = 0;
  }
  S.q = S.ly * D.nlx + S.lx;
  S.Wl = min(D.pw, D.W - S.lx * D.pw);
  S.lane_px_off = (int64_t)S.ly * D.ph * D.W + (int64_t)S.lx * D.pw * S.Hl;
  if (K == ROW_STREAMS)
    S.slot_end = D.slot_base + 6 * (S.lane_px_off + (int64_t)(S.r + 1) * S.Wl) + 8 * (e + 1);
  else
    S.slot_end = D.slot_base + K * (6 * S.lane_px_off + 8 * (int64_t)S.q) +
                 (S.kk + 1) * lane_slot_bytes((int64_t)S.Hl * S.Wl);
  return S;
}


NXD uint32_t rd_u32(const uint8_t* p) {
  return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) | ((uint32_t)p[3] << 24);
}

NXD int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
NXD int64_t uniform64(int64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// the same search with every step wave-uniform (key must be wave-uniform)
NXD int find_img_uniform(const ImgDesc* __restrict__ d, int n, int64_t key, bool by_lane = true) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    const int64_t b = uniform64(by_lane ? d[mid].lane_base : d[mid].tile_base);
    if (b <= key) lo = mid; else hi = mid - 1;
  }
  return uniform(lo);
}

// Descriptor fields as wave-uniform values. Every lane loads the same
// descriptor; saying so (readfirstlane) keeps all control flow that depends
// on it uniform: the compiler then never splits a wave across the exits of the
// persistent loops.
NXD ImgDesc uniform_desc(const ImgDesc* __restrict__ p) {
  ImgDesc D = *p;
  D.px = (uint8_t*)uniform64((int64_t)D.px);
  D.H = uniform(D.H);
  D.W = uniform(D.W);
  D.ph = uniform(D.ph);
  D.pw = uniform(D.pw);
  D.nlx = uniform(D.nlx);
  D.nly = uniform(D.nly);
  D.lane_base = uniform64(D.lane_base);
  D.px_base = uniform64(D.px_base);
  D.tile_base = uniform64(D.tile_base);
  D.ntx = uniform(D.ntx);
  D.slot_base = uniform64(D.slot_base);
  D.seed = (uint64_t)uniform64((int64_t)D.seed);
  return D;
}

NXD uint32_t uniform_u(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }

// the whole workgroup (any block size) copies the weight image into LDS
NXD void load_weights(float* lds, const float* __restrict__ w, int64_t nfloats) {
  const int64_t n4 = nfloats >> 2;
  for (int64_t i = threadIdx.x; i < n4; i += blockDim.x) ((float4*)lds)[i] = ((const float4*)w)[i];
  __syncthreads();
}

// ------------------------------------------------------------------ full-image pass
template <int H_, int C_>
__global__ void __launch_bounds__(NWAVES * 64) k_pass(PassArgs A) {
  extern __shared__ float4 smem_f4[];
  float* w = (float*)smem_f4;
  load_weights(w, A.w, A.wfloats);
  const int lane = threadIdx.x & 63, p = lane & 15, g = lane >> 4;
  const bool has2 = g < 2;
  const int64_t gw = (int64_t)blockIdx.x * NWAVES + (threadIdx.x >> 6);
  const int64_t nwv = (int64_t)gridDim.x * NWAVES;
  TapCodes<H_> tc;
  tc.init(g);
  for (int64_t t = gw; t < A.n_tiles; t += nwv) {
    tc.refresh();
    const int n = find_img_uniform(A.desc, A.n_img, t, false);
    const ImgDesc D = uniform_desc(A.desc + n);
    const int64_t tt = t - D.tile_base;
    const int y = (int)(tt / D.ntx);
    const int xraw = (int)(tt - (int64_t)y * D.ntx) * 16 + p;
    const bool active = xraw < D.W;
    const int x = active ? xraw : D.W - 1;
    const int ly = y / D.ph, lx = x / D.pw;
    const int y0 = ly * D.ph, x0 = lx * D.pw;
    const int Hl = min(D.ph, D.H - y0), Wl = min(D.pw, D.W - x0);
    float ctx[conv_chunks(H_)];
    gather<H_>(ctx, tc, D.px, D.W, y0, x0, Hl, Wl, y - y0, x - x0, active);
    f4 head[HEAD_TILES];
    net_forward<H_, C_>(lds_weights(w), A.nb, ctx, head, lane);
    Mix M;
    mix_prep(head, M, has2);
    const int64_t pix = (int64_t)y * D.W + x;
    int xv[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) xv[c] = D.px[pix * 3 + c];
    const float xr = normalise(xv[0]), xg = normalise(xv[1]);
    float bits = 0.0f;
    const int64_t gpix = D.px_base + pix;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      Chan K;
      chan_params(M, c, xr, xg, K);
      if (A.mode == 0) {
        const float Flo = cdf_eval(max(xv[c], 1), K.w, K.a, K.b);
        const float Fhi = cdf_eval(min(xv[c] + 1, 255), K.w, K.a, K.b);
        const uint32_t lo = xv[c] == 0 ? 0u : cdf_quant(xv[c], Flo);
        const uint32_t hi = xv[c] == 255 ? CDF_TOTAL : cdf_quant(xv[c] + 1, Fhi);
        if (active && g == 0) A.sym[gpix * 3 + c] = lo | ((hi - lo) << 16);
        bits += (float)CDF_BITS - __builtin_amdgcn_logf((float)(hi - lo));
        if (c < 2) posterior(M, xv[c], K.mu, K.is, has2);
      } else if (A.mode == 1) {
        const float lp = posterior(M, xv[c], K.mu, K.is, has2);
        bits += -lp * kLog2e;
      } else {
        for (int k = 1; k < 256; ++k) {
          const uint32_t v = cdf_quant(k, cdf_eval(k, K.w, K.a, K.b));
          if (active && g == 0) A.cdf[(gpix * 3 + c) * 257 + k] = (int32_t)v;
        }
        if (active && g == 0) {
          A.cdf[(gpix * 3 + c) * 257] = 0;
          A.cdf[(gpix * 3 + c) * 257 + 256] = (int32_t)CDF_TOTAL;
        }
        if (c < 2) posterior(M, xv[c], K.mu, K.is, has2);
      }
    }
    if (A.bits && active && g == 0) A.bits[gpix] = bits;
  }
}

// ------------------------------------------------------------------ rANS encoder
// Three kernels. A stream's states are one serial chain, run by one thread,
// and with a few thousand streams a wave has a SIMD to itself: its time per
// symbol is its own instruction count. So the walk over the stream's
// symbols in reverse decode order, and their loads, come out of that chain:
// k_rans_counts and k_rans_scatter lay every stream's symbols out
// contiguously in coding order, reading the symbol buffer in pixel order;
// k_rans_enc then reads them in order and codes.

// lane geometry of stream SL = L K + kk, and where its encoder scratch lies
struct StreamGeom {
  ImgDesc D;
  int kk, q, y0, x0, Hl, Wl;
  int64_t lane_px_off;
  int64_t rev_cap, rev_off;      // words of the stream's coding-order buffer, and its first
  int64_t after_cap, after_off;  // entries of its per-step offsets, and its first
};
NXD StreamGeom stream_geom(const RansEncArgs& A, int64_t SL) {
  StreamGeom G;
  const int64_t L = SL / A.K;
  G.kk = (int)(SL - L * A.K);
  const int n = find_img(A.desc, A.n_img, L, true);
  G.D = A.desc[n];
  G.q = (int)(L - G.D.lane_base);
  const int64_t rel = SL - G.D.lane_base * A.K;  // the stream's index within its image
  G.rev_cap = stream_rev_words(G.D.ph, G.D.pw, A.K);
  G.after_cap = stream_after_entries(G.D.ph, G.D.pw);
  G.rev_off = G.D.rev_base + rel * G.rev_cap;
  G.after_off = G.D.after_base + rel * G.after_cap;
  const int ly = G.q / G.D.nlx, lx = G.q - ly * G.D.nlx;
  G.y0 = ly * G.D.ph;
  G.x0 = lx * G.D.pw;
  G.Hl = min(G.D.ph, G.D.H - G.y0);
  G.Wl = min(G.D.pw, G.D.W - G.x0);
  G.lane_px_off = (int64_t)ly * G.D.ph * G.D.W + (int64_t)lx * G.D.pw * G.Hl;
  return G;
}

// One wave per stream. Each lane counts the stream's symbols in a range of
// wavefront steps (stream_rows_at); a suffix sum across the wave gives the
// symbols after each range; the lane then writes, per step t of its range,
// how many of the stream's symbols come in steps after t (in coding order
// the later steps come first). Lane 0's inclusive sum is the stream's
// length. Raster order: the length only.
template <int O, int K>
__global__ void __launch_bounds__(64) k_rans_counts(RansEncArgs A) {
  const int64_t SL = blockIdx.x;
  const int lane = (int)threadIdx.x;
  const StreamGeom G = stream_geom(A, SL);
  if (A.order == 0) {
    if (lane == 0) A.lane_len[SL] = (uint32_t)min<int64_t>(3LL * G.Hl * G.Wl, G.rev_cap);
    return;
  }
  const int T = G.Wl + O * (G.Hl - 1);
  const int tlo = (int)((int64_t)T * lane / 64), thi = (int)((int64_t)T * (lane + 1) / 64);
  int cnt = 0;
  for (int t = tlo; t < thi; ++t) cnt += 3 * stream_rows_at(t, G.Hl, G.Wl, O, K, G.kk);
  int suf = cnt;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int v = __shfl_down(suf, d, 64);
    if (lane + d < 64) suf += v;
  }
  int32_t* tab = A.after + G.after_off;
  int S = suf - cnt;
  for (int t = thi - 1; t >= tlo; --t) {
    if (t < G.after_cap) tab[t] = S;
    S += 3 * stream_rows_at(t, G.Hl, G.Wl, O, K, G.kk);
  }
  if (lane == 0) A.lane_len[SL] = (uint32_t)min<int64_t>(suf, G.rev_cap);
}

constexpr int SCATTER_PX = 16384;  // pixels of a lane per k_rans_scatter workgroup

// Workgroup (lane, chunk) reads a chunk of the lane's symbols in pixel order
// (coalesced) and puts each at its place in its stream's coding order
// (coding_slot plus the stream's symbols of later steps); raster order
// reverses the raster index. The writes of a workgroup stay within its
// lane's K streams.
template <int O, int K>
__global__ void __launch_bounds__(256) k_rans_scatter(RansEncArgs A) {
  const int64_t L = blockIdx.x;
  const StreamGeom G = stream_geom(A, L * K);
  const int64_t npx = (int64_t)G.Hl * G.Wl;
  const int64_t q0 = (int64_t)blockIdx.y * SCATTER_PX;
  if (q0 >= npx) return;
  const int64_t q1 = min<int64_t>(npx, q0 + SCATTER_PX);
  const uint32_t* sym = A.sym + G.D.px_base * 3;
  for (int64_t q = q0 + threadIdx.x; q < q1; q += 256) {
    const int i = (int)(q / G.Wl), j = (int)(q - (int64_t)i * G.Wl);
    const uint32_t* sp = sym + ((int64_t)(G.y0 + i) * G.D.W + (G.x0 + j)) * 3;
    const uint32_t v[3] = {sp[0], sp[1], sp[2]};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      int kk = 0;
      int64_t p;
      if (A.order == 0) {
        p = 3 * npx - 1 - (3 * q + c);
      } else {
        int t, off;
        coding_slot(i, j, c, G.Hl, G.Wl, O, K, kk, t, off);
        p = (int64_t)A.after[G.after_off + kk * G.after_cap + t] + off;
      }
      if (p >= 0 && p < G.rev_cap) A.rev[G.rev_off + kk * G.rev_cap + p] = v[c];
    }
  }
}

// Spread slots. A push of symbol (s, f) from a state x < f (only near the
// start of a stream) takes the x-th (from 0) slot y of [0, 2^16) whose 16-bit
// reversal lies in [s, s + f): reversal deals the range out about 2^16 / f
// apart, so the state grows by about the symbol's probability, where the
// usual rule would jump to s + x. The decoder recognises such a state (it is
// below 2^16), searches the symbol with the reversed slot and pops by the
// rank of y among the symbol's slots. Both walk the reversal's 16 bits from
// the lowest: the range values with low bits r (j of them) and bit j clear
// number floor((s + f - 1 - r) / 2^(j+1)) - floor((s - 1 - r) / 2^(j+1))
// (the floors are arithmetic shifts).
NXD uint32_t rev16(uint32_t v) { return __builtin_bitreverse32(v) >> 16; }

NXD int32_t spread_count(int32_t lo, int32_t hi, int32_t r, int sh) { return ((hi - r) >> sh) - ((lo - r) >> sh); }

NXD uint32_t spread_select(uint32_t x, uint32_t s, uint32_t f) {
  const int32_t lo = (int32_t)s - 1, hi = (int32_t)(s + f) - 1;
  int32_t r = 0, left = (int32_t)x;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int32_t n0 = spread_count(lo, hi, r, j + 1);
    const bool one = left >= n0;
    left -= one ? n0 : 0;
    r |= one ? (1 << j) : 0;
  }
  return rev16((uint32_t)r);
}

NXD uint32_t spread_rank(uint32_t y, uint32_t s, uint32_t f) {
  const uint32_t v = rev16(y);
  const int32_t lo = (int32_t)s - 1, hi = (int32_t)(s + f) - 1;
  int32_t n = 0;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int32_t r = (int32_t)(v & ((1u << j) - 1u));
    n += ((v >> j) & 1u) ? spread_count(lo, hi, r, j + 1) : 0;
  }
  return (uint32_t)n;
}

// rANS-encodes n symbols (start | freq << 16) into state x, bytes written
// backwards at out. x / f: a float quotient (relative error below 2^-21, so
// within one of the true one, as x / f < 2^15 after renormalisation) fixed
// by one step of the remainder; a state below 2^31 sheds at most two bytes.
// A state below f takes the symbol's spread slot instead.
template <int B>
__device__ __forceinline__ void rans_put(uint32_t& x, uint8_t*& out, const uint32_t (&v)[B], int n) {
#pragma unroll
  for (int k = 0; k < B; ++k) {
    if (k < n) {
      const uint32_t s = v[k] & 0xffffu, f = v[k] >> 16;
      if (x < f) {  // the first pushes of a stream: a spread slot
        x = spread_select(x, s, f);
        continue;
      }
      const float rf = __builtin_amdgcn_rcpf((float)f);
      const uint32_t xmax = ((RANS_L >> CDF_BITS) << 8) * f;
      const uint32_t b1 = x >= xmax ? 1u : 0u;
      const uint32_t b2 = (x >> 8) >= xmax ? 1u : 0u;
      if (b1) out[-1] = (uint8_t)x;
      if (b2) out[-2] = (uint8_t)(x >> 8);
      out -= b1 + b2;
      x >>= 8u * (b1 + b2);
      uint32_t qt = (uint32_t)((float)x * rf);
      int32_t r = (int32_t)(x - qt * f);
      if (r < 0) {
        --qt;
        r += (int32_t)f;
      } else if (r >= (int32_t)f) {
        ++qt;
        r -= (int32_t)f;
      }
      x = (qt << CDF_BITS) + (uint32_t)r + s;
    }
  }
}

// one thread per stream (lane L, stream k): stream index L K + k
__global__ void __launch_bounds__(64) k_rans_enc(RansEncArgs A) {
  const int64_t SL = (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (SL >= A.n_streams) return;
  const StreamGeom G = stream_geom(A, SL);
  const int64_t slot_end = G.D.slot_base + A.K * (6 * G.lane_px_off + 8 * (int64_t)G.q) +
                           (G.kk + 1) * lane_slot_bytes((int64_t)G.Hl * G.Wl);
  uint8_t* out = A.slots + slot_end;
  const uint4* src = (const uint4*)(A.rev + G.rev_off);
  const int64_t n = A.lane_len[SL];
  uint32_t x = RANS_X0;
  constexpr int B = 16;  // symbols per batch; the next batch loads while this one is coded
  uint32_t va[B], vb[B];
  int na = 0;
  for (int64_t p0 = 0;; p0 += B) {
    const int nb = p0 < n ? (int)min<int64_t>(B, n - p0) : 0;
    if (nb > 0) {
#pragma unroll
      for (int k = 0; k < B / 4; ++k) {
        const uint4 w = src[p0 / 4 + k];
        vb[4 * k] = w.x;
        vb[4 * k + 1] = w.y;
        vb[4 * k + 2] = w.z;
        vb[4 * k + 3] = w.w;
      }
    }
    if (na > 0) rans_put(x, out, va, na);
    if (nb == 0) break;
#pragma unroll
    for (int k = 0; k < B; ++k) va[k] = vb[k];
    na = nb;
  }
  // the final state's significant bytes (x >= 1), most significant first
  do {
    *--out = (uint8_t)x;
    x >>= 8;
  } while (x != 0u);
  A.lane_len[SL] = (uint32_t)((A.slots + slot_end) - out);
}

// Row streams: one thread per stream (a lane row). Its symbols in decode
// order are the row's pixels left to right, R, G, B, so in coding order they
// are read in place from the symbol buffer, backwards.
__global__ void __launch_bounds__(64) k_rans_enc_rows(RansEncArgs A) {
  const int64_t SL = (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (SL >= A.n_streams) return;
  const int n = find_img_stream(A.desc, A.n_img, SL);
  const ImgDesc D = A.desc[n];
  const int64_t e = SL - D.stream_base;
  const StreamAt S = stream_at(D, ROW_STREAMS, e);
  uint8_t* out = A.slots + S.slot_end;
  const uint32_t* row = A.sym + (D.px_base + (int64_t)(S.ly * D.ph + S.r) * D.W + (int64_t)S.lx * D.pw) * 3;
  uint32_t x = RANS_X0;
  constexpr int B = 16;
  uint32_t v[B];
  for (int k = 3 * S.Wl - 1; k >= 0; k -= B) {
    const int nb = min(B, k + 1);
#pragma unroll
    for (int m = 0; m < B; ++m) v[m] = m < nb ? row[k - m] : 0u;
    rans_put(x, out, v, nb);
  }
  // the final state's significant bytes (x >= 1), most significant first
  do {
    *--out = (uint8_t)x;
    x >>= 8;
  } while (x != 0u);
  A.lane_len[SL] = (uint32_t)((A.slots + S.slot_end) - out);
}

// ------------------------------------------------------------------ container assembly
// per image: lane_end (inclusive prefix of lane lengths), container bytes
__global__ void __launch_bounds__(256) k_lane_scan(PackArgs A) {
  __shared__ uint32_t part[256];
  __shared__ uint32_t carry;
  const int n = blockIdx.x;
  const ImgDesc D = A.desc[n];
  const int nl = (int)image_streams(A.K, D.H, D.nlx, D.nly);  // streams of this image
  const int64_t sbase = D.stream_base;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int b0 = 0; b0 < nl; b0 += 256) {
    const int q = b0 + threadIdx.x;
    const uint32_t v = q < nl ? A.lane_len[sbase + q] : 0u;
    part[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
      const uint32_t add = threadIdx.x >= off ? part[threadIdx.x - off] : 0u;
      __syncthreads();
      part[threadIdx.x] += add;
      __syncthreads();
    }
    if (q < nl) A.lane_end[sbase + q] = carry + part[threadIdx.x];
    __syncthreads();
    if (threadIdx.x == 255) carry += part[255];
    __syncthreads();
  }
  if (threadIdx.x == 0) A.img_bytes[n] = (uint64_t)HDR_BYTES + 4ull * nl + carry;  // nl = streams
}

__global__ void k_img_scan(PackArgs A) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  uint64_t acc = 0;
  for (int n = 0; n < A.n_img; ++n) {
    A.out_offsets[n] = acc;
    acc += A.img_bytes[n];
  }
  A.out_offsets[A.n_img] = acc;
  *A.overflow = acc > A.out_cap ? 1 : 0;
}

// one 64-thread block per stream: payload copy, stream table entry, header
__global__ void __launch_bounds__(64) k_pack(PackArgs A) {
  if (*A.overflow) return;
  const int64_t SL = blockIdx.x;
  const int n = find_img_stream(A.desc, A.n_img, SL);
  const ImgDesc D = A.desc[n];
  const int64_t entry = SL - D.stream_base;
  const int64_t ns = image_streams(A.K, D.H, D.nlx, D.nly);
  const int nl = D.nlx * D.nly;
  const StreamAt S = stream_at(D, A.K, entry);
  const int64_t slot_end = S.slot_end;
  const uint32_t len = A.lane_len[SL];
  const uint32_t end = A.lane_end[SL];
  uint8_t* C = A.out + A.out_offsets[n];
  uint8_t* dst = C + HDR_BYTES + 4 * ns + (end - len);
  const uint8_t* src = A.slots + slot_end - len;
  for (uint32_t k = threadIdx.x; k < len; k += 64) dst[k] = src[k];
  if (threadIdx.x < 4) C[HDR_BYTES + 4 * entry + threadIdx.x] = (uint8_t)(end >> (8 * threadIdx.x));
  if (entry == 0 && threadIdx.x == 0) {
    uint8_t h[HDR_BYTES];
    for (int k = 0; k < HDR_BYTES; ++k) h[k] = 0;
    h[0] = 'N'; h[1] = 'L'; h[2] = 'X'; h[3] = 'C';
    h[4] = CONTAINER_VERSION;
    h[5] = (uint8_t)A.order;
    h[6] = (uint8_t)A.h;
    h[7] = (uint8_t)A.K;
    for (int k = 0; k < 4; ++k) h[8 + k] = (uint8_t)((uint32_t)D.H >> (8 * k));
    for (int k = 0; k < 4; ++k) h[12 + k] = (uint8_t)((uint32_t)D.W >> (8 * k));
    const uint32_t ph = D.ph == D.H ? 0u : (uint32_t)D.ph, pw = D.pw == D.W ? 0u : (uint32_t)D.pw;
    h[16] = (uint8_t)ph; h[17] = (uint8_t)(ph >> 8);
    h[18] = (uint8_t)pw; h[19] = (uint8_t)(pw >> 8);
    for (int k = 0; k < 8; ++k) h[20 + k] = (uint8_t)(A.model_hash >> (8 * k));
    for (int k = 0; k < 4; ++k) h[28 + k] = (uint8_t)((uint32_t)nl >> (8 * k));
    for (int k = 0; k < HDR_BYTES; ++k) C[k] = h[k];
  }
}

// ------------------------------------------------------------------ decoder
// Bytes of the lane payload, staged 256 at a time: lane l of the wave holds
// bytes base + 4l .. base + 4l + 3; a byte is fetched with a lane read.
struct ByteStage {
  const uint8_t* S;
  uint32_t len, base;
  uint32_t word;
  NXD void fill(uint32_t at, int lane) {
    // clamped, unconditional loads; bytes past the end read as 0
    base = at;
    const gbytes g = as_global(S);
    uint32_t v = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const uint32_t o = at + 4 * (uint32_t)lane + b;
      const uint32_t byte = g[o < len ? o : len - 1];
      v |= (o < len ? byte : 0u) << (8 * b);
    }
    word = v;
  }
  // byte at pos, pos >= base; the caller keeps pos < base + 256 (bytes past
  // the window read as garbage, never as an out-of-range lane)
  NXD uint32_t byte_at(uint32_t pos) const {
    const uint32_t off = pos - base;
    const uint32_t v = (uint32_t)__builtin_amdgcn_readlane((int)word, (int)((off >> 2) & 63u));
    return (v >> (8 * (off & 3u))) & 255u;
  }
  NXD uint32_t get(uint32_t pos, int lane) {
    if (pos - base >= 256u) fill(pos, lane);
    return byte_at(pos);
  }
  // rANS renormalisation after a pop: at most two bytes are read (the popped
  // state is at least 2^7 while bytes remain), each only while x < L and
  // bytes remain; no branch except the rare window refill
  NXD void renorm(uint32_t& x, uint32_t& pos, int lane, bool act = true) {
    if (pos + 2u > base + 256u && pos < len) fill(pos & ~3u, lane);
    const uint32_t b0 = byte_at(pos), b1 = byte_at(pos + 1u);
    const bool r0 = act && x < RANS_L && pos < len;
    x = r0 ? ((x << 8) | b0) : x;
    pos += r0 ? 1u : 0u;
    const bool r1 = x < RANS_L && pos < len;
    x = r1 ? ((x << 8) | b1) : x;
    pos += r1 ? 1u : 0u;
  }
};

// ------------------------------------------------------------------ four-row decoding
// With four streams per lane, the wave's 16-lane rows work independently:
// row g searches the symbol of stream g while every lane evaluates all ten
// mixture components at its own point, so no cross-row reduction is needed.
// A pixel's mixture for the channel is staged in LDS as (w, a, b) of
// component m at floats 3m..3m+2 of the pixel's row of the table.
struct Mix10 {
  float w[10], a[10], b[10];
};

NXD void load_mix10(Mix10& P, const float* prm, int pix) {
  const float4* s = (const float4*)(prm + pix * PRM_STRIDE);
  float v[32];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const float4 t = s[i];
    v[4 * i] = t.x; v[4 * i + 1] = t.y; v[4 * i + 2] = t.z; v[4 * i + 3] = t.w;
  }
#pragma unroll
  for (int m = 0; m < 10; ++m) {
    P.w[m] = v[3 * m];
    P.a[m] = v[3 * m + 1];
    P.b[m] = v[3 * m + 2];
  }
}

// F at bin edge k over all ten components in this lane. The terms and the
// additions are those of cdf_eval: per lane group g the sum
// s_g = (t_g + t_{g+4}) + t_{g+8} (groups 2 and 3 add an exact zero), then
// (s_0 + s_1) + (s_2 + s_3); so the value is bit-identical to the encoder's.
NXD float cdf_eval10(int k, const Mix10& P) {
  const float e = bin_edge(k);
  float t[10];
#pragma unroll
  for (int m = 0; m < 10; ++m) {
    const float x = __builtin_amdgcn_exp2f(__builtin_fmaf(-e, P.a[m], P.b[m]));
    t[m] = P.w[m] * __builtin_amdgcn_rcpf(1.0f + x);
  }
  const float s0 = (t[0] + t[4]) + t[8];
  const float s1 = (t[1] + t[5]) + t[9];
  const float s2 = t[2] + t[6];
  const float s3 = t[3] + t[7];
  return (s0 + s1) + (s2 + s3);
}

// bits of row g in a wave-wide ballot, counted
NXD int row_count(uint64_t bal, int g) {
  const uint32_t half = (g & 2) ? (uint32_t)(bal >> 32) : (uint32_t)bal;
  return __builtin_popcount((half >> ((g & 1) << 4)) & 0xffffu);
}

// One stream per row: state, position and a 64-byte window of its bytes,
// 4 bytes per lane of the row (every value uniform within the row).
struct RowStream {
  const uint8_t* S;
  uint32_t len, base, pos, x, word;
  // lanes of the row load the window [at, at + 64) (clamped, unconditional loads)
  NXD void fill(uint32_t at, int p) {
    base = at;
    const gbytes gs = as_global(S);
    uint32_t v = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const uint32_t o = at + 4 * (uint32_t)p + b;
      const uint32_t byte = gs[o < len ? o : len - 1];
      v |= (o < len ? byte : 0u) << (8 * b);
    }
    word = v;
  }
  // renormalisation after a pop of this row (as ByteStage::renorm): the window
  // is moved first where it would not hold pos + 1
  NXD void renorm(bool act, int p, int g) {
    const bool need = pos + 2u > base + 64u && pos < len;
    if (__ballot(need) != 0ull) {
      if (need) fill(pos & ~3u, p);
    }
    // bytes pos and pos + 1 (off <= 62 here): the two window words from
    // off / 4 on, then the byte pair at off % 4 of their concatenation
    const uint32_t off = pos - base;
    const uint32_t wi = off >> 2;
    const uint32_t w0 = (uint32_t)__shfl((int)word, (g << 4) | (int)(wi & 15u));
    const uint32_t w1 = (uint32_t)__shfl((int)word, (g << 4) | (int)((wi + 1u) & 15u));
    const uint32_t two = __builtin_amdgcn_alignbyte(w1, w0, off & 3u);
    const uint32_t b0 = two & 255u, b1 = (two >> 8) & 255u;
    const bool r0 = act && x < RANS_L && pos < len;
    x = r0 ? ((x << 8) | b0) : x;
    pos += r0 ? 1u : 0u;
    const bool r1 = act && x < RANS_L && pos < len;
    x = r1 ? ((x << 8) | b1) : x;
    pos += r1 ? 1u : 0u;
  }
};

// K >= 8: one stream per pixel row of a 16-row group (K = 16), or one per
// pair of rows p and p + 8 (K = 8); lane (p, g) holds stream p mod K's state,
// the same in every lane of the pixel (and, for K = 8, of both rows)
struct PixStream {
  gbytes S;
  uint32_t len, pos, x;
};

// One symbol of every pixel of a 16-row group, each from the pixel's own
// stream, all pixels at once: eight halvings of [0, 256], each the encoder's
// evaluation of the quantised CDF (cdf_eval, all lanes of a pixel in step),
// keeping the bracket's CDF values, so (start, freq) are bitwise the
// encoder's. Pixels with act pop (state and position updated); the stream's
// next two bytes are loaded before the search (clamped into the stream,
// used only while bytes remain). Every lane must call it (lane-group sums).
NXD int pop_own(const Chan& Q, PixStream& P, bool act, uint32_t& start, uint32_t& freq) {
  const uint32_t lm = P.len - 1u;
  const uint32_t nb0 = P.S[min(P.pos, lm)];
  const uint32_t nb1 = P.S[min(P.pos + 1u, lm)];
  // a state below 2^16 (the end of the stream) holds a spread slot
  const bool small = P.x < CDF_TOTAL;
  const uint32_t slot = small ? rev16(P.x) : (P.x & 0xffffu);
  // the bracket [lo, lo + 2^(8 - it)) halves at every step: its midpoint is
  // lo plus a constant, and only its CDF values need keeping
  int lo = 0;
  uint32_t clo = 0u, chi = CDF_TOTAL;
#pragma unroll
  for (int it = 0; it < 8; ++it) {
    const int mid = lo + (128 >> it);
    const uint32_t v = cdf_quant(mid, cdf_eval(mid, Q.w, Q.a, Q.b));
    const bool le = v <= slot;
    lo = le ? mid : lo;
    clo = le ? v : clo;
    chi = le ? chi : v;
  }
  freq = chi - clo;
  start = clo;
  uint32_t xn = freq * (P.x >> 16) + slot - clo;
  if (__ballot(small && act) != 0ull) {  // rare: a stream's last few pops
    const uint32_t xr = spread_rank(P.x, clo, freq);
    xn = small ? xr : xn;
  }
  uint32_t pn = P.pos;
  const bool r0 = xn < RANS_L && pn < P.len;
  xn = r0 ? ((xn << 8) | nb0) : xn;
  pn += r0 ? 1u : 0u;
  const bool r1 = xn < RANS_L && pn < P.len;
  xn = r1 ? ((xn << 8) | nb1) : xn;
  pn += r1 ? 1u : 0u;
  P.x = act ? xn : P.x;
  P.pos = act ? pn : P.pos;
  return lo;
}

// pop_own for the 16-lanes-per-pixel layout of the row decoder. A wave has
// its SIMD to itself here, so the search trades instructions for a shorter
// dependent chain: four quarterings of [0, 256) instead of eight halvings,
// the three quartile points of a step evaluated together (cdf_eval16,
// bitwise the encoder's CDF values; the CDF is increasing, so the points at
// or below the slot are a prefix). The bracket found, and its CDF values,
// are the bisection's.
NXD int pop16(const Chan16& Q, PixStream& P, bool act, uint32_t& start, uint32_t& freq) {
  const uint32_t lm = P.len - 1u;
  const uint32_t nb0 = P.S[min(P.pos, lm)];
  const uint32_t nb1 = P.S[min(P.pos + 1u, lm)];
  const bool small = P.x < CDF_TOTAL;
  const uint32_t slot = small ? rev16(P.x) : (P.x & 0xffffu);
  int lo = 0;
  uint32_t clo = 0u, chi = CDF_TOTAL;
#pragma unroll
  for (int st = 0; st < 4; ++st) {
    const int d = 64 >> (2 * st);
    const int k1 = lo + d, k2 = lo + 2 * d, k3 = lo + 3 * d;
    const uint32_t v1 = cdf_quant(k1, cdf_eval16(k1, Q));
    const uint32_t v2 = cdf_quant(k2, cdf_eval16(k2, Q));
    const uint32_t v3 = cdf_quant(k3, cdf_eval16(k3, Q));
    const bool l1 = v1 <= slot, l2 = v2 <= slot, l3 = v3 <= slot;
    lo = l3 ? k3 : (l2 ? k2 : (l1 ? k1 : lo));
    clo = l3 ? v3 : (l2 ? v2 : (l1 ? v1 : clo));
    chi = l3 ? chi : (l2 ? v3 : (l1 ? v2 : v1));
  }
  freq = chi - clo;
  start = clo;
  uint32_t xn = freq * (P.x >> 16) + slot - clo;
  if (__ballot(small && act) != 0ull) {
    const uint32_t xr = spread_rank(P.x, clo, freq);
    xn = small ? xr : xn;
  }
  uint32_t pn = P.pos;
  const bool r0 = xn < RANS_L && pn < P.len;
  xn = r0 ? ((xn << 8) | nb0) : xn;
  pn += r0 ? 1u : 0u;
  const bool r1 = xn < RANS_L && pn < P.len;
  xn = r1 ? ((xn << 8) | nb1) : xn;
  pn += r1 ? 1u : 0u;
  P.x = act ? xn : P.x;
  P.pos = act ? pn : P.pos;
  return lo;
}

// a stream's initial state: its first bytes, most significant first, read
// while x < L (at most four; loads clamped into the stream, len >= 1)
NXD void stream_begin(PixStream& P) {
  uint32_t xs = 0u, ps = 0u;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const uint32_t byte = P.S[min((uint32_t)b, P.len - 1u)];
    const bool rd = xs < RANS_L && ps < P.len;
    xs = rd ? ((xs << 8) | byte) : xs;
    ps += rd ? 1u : 0u;
  }
  P.x = xs;
  P.pos = ps;
}

// K: rANS streams of the lane; the chain pops K symbols (rows ts + q0 + k,
// streams k) per iteration, their searches independent of each other;
// K >= 8: every row of a group pops from its own stream at once, found by a
// bisection of the quantised CDF over the whole group.
// SAMPLE: ancestral sampling instead of decoding (no container): each
// symbol is the inverse quantised CDF at its Philox slot, found by bisection
// for all rows of a group at once (their slots do not depend on each other).
// SHEAR: the sheared layout (order 2): contexts from the wave's window of the
// lane's sheared canvas instead of the output image.
template <int H_, int C_, bool TRACE, int K, bool SAMPLE, bool SHEAR>
__device__ void decode_lane(const DecArgs& A, const float* w, uint32_t* piv, int64_t L, int lane) {
  static_assert(!SAMPLE || K == 4, "sampling is instantiated once, as K = 4");
  const int p = lane & 15, g = lane >> 4;
  const bool has2 = g < 2;
  const int n = find_img_uniform(A.desc, A.n_img, L);
  const ImgDesc D = uniform_desc(A.desc + n);
  const int q = (int)(L - D.lane_base);
  const int nl = D.nlx * D.nly;
  const int ly = q / D.nlx, lx = q - ly * D.nlx;
  const int y0 = ly * D.ph, x0 = lx * D.pw;
  const int Hl = min(D.ph, D.H - y0), Wl = min(D.pw, D.W - x0);
  const uint8_t* C = nullptr;
  int64_t clen = 0, pay = 0;
  // header and stream table checks (every lane reads the same bytes; the
  // verdicts are made wave-uniform, and status is stored by every lane)
  bool ok = true;
  bool mismatch = false;
  if constexpr (!SAMPLE) {
  C = A.in + uniform64((int64_t)A.in_off[n]);
  clen = uniform64((int64_t)(A.in_off[n + 1] - A.in_off[n]));
  pay = HDR_BYTES + 4 * (int64_t)nl * K;
  ok = clen >= pay;
  if (ok) {
    const uint32_t ph = D.ph == D.H ? 0u : (uint32_t)D.ph, pw = D.pw == D.W ? 0u : (uint32_t)D.pw;
    ok = C[0] == 'N' && C[1] == 'L' && C[2] == 'X' && C[3] == 'C' && C[4] == CONTAINER_VERSION &&
         C[5] == (uint8_t)(A.order == 0 ? 0 : 1) && C[6] == (uint8_t)H_ && C[7] == (uint8_t)K && rd_u32(C + 8) == (uint32_t)D.H &&
         rd_u32(C + 12) == (uint32_t)D.W && (uint32_t)(C[16] | (C[17] << 8)) == ph &&
         (uint32_t)(C[18] | (C[19] << 8)) == pw && rd_u32(C + 28) == (uint32_t)nl;
    // the streams fill the container exactly: the last end is its payload
    ok = ok && pay + (int64_t)rd_u32(C + HDR_BYTES + 4 * ((int64_t)nl * K - 1)) == clen;
    ok = uniform(ok ? 1 : 0) != 0;
    if (ok) {
      const uint64_t hsh = (uint64_t)rd_u32(C + 20) | ((uint64_t)rd_u32(C + 24) << 32);
      mismatch = uniform(hsh != A.model_hash ? 1 : 0) != 0;
    }
  }
  }  // !SAMPLE
  if (mismatch) {
    A.status[n] = ST_MISMATCH;
    return;
  }
  // K <= 2: the streams' states are scalar (one search after another);
  // K = 4: one stream per 16-lane row, its state held by the row;
  // K >= 8: one stream per pixel (per pair of pixels for K = 8)
  constexpr int KS = K <= 2 ? K : 1;
  ByteStage R[KS];
  uint32_t x[KS], pos[KS];
  RowStream RS;
  PixStream PS;
  if constexpr (SAMPLE) {
  } else if constexpr (K >= 8) {
    const int64_t e = (int64_t)q * K + (p & (K - 1));  // stream table entry of this pixel row
    uint32_t lend = 0, lstart = 0;
    bool okr = ok;
    if (ok) {
      lend = rd_u32(C + HDR_BYTES + 4 * e);
      lstart = e > 0 ? rd_u32(C + HDR_BYTES + 4 * (e - 1)) : 0u;
      okr = lstart <= lend && pay + (int64_t)lend <= clen && lend - lstart >= 1;
    }
    ok = __ballot(okr) == ~0ull;
    PS.S = as_global(C + pay + lstart);
    PS.len = lend - lstart;
  } else if constexpr (K == 4) {
    const int64_t e = (int64_t)q * K + g;  // stream table entry of this row
    uint32_t lend = 0, lstart = 0;
    bool okr = ok;
    if (ok) {
      lend = rd_u32(C + HDR_BYTES + 4 * e);
      lstart = e > 0 ? rd_u32(C + HDR_BYTES + 4 * (e - 1)) : 0u;
      okr = lstart <= lend && pay + (int64_t)lend <= clen && lend - lstart >= 1;
    }
    ok = __ballot(okr) == ~0ull;
    RS.S = C + pay + lstart;
    RS.len = lend - lstart;
  } else {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int64_t e = (int64_t)q * K + k;  // stream table entry
      uint32_t lend = 0, lstart = 0;
      if (ok) {
        lend = (uint32_t)uniform((int)rd_u32(C + HDR_BYTES + 4 * e));
        lstart = e > 0 ? (uint32_t)uniform((int)rd_u32(C + HDR_BYTES + 4 * (e - 1))) : 0u;
        ok = lstart <= lend && pay + (int64_t)lend <= clen && lend - lstart >= 1;
      }
      R[k].S = C + pay + lstart;
      R[k].len = lend - lstart;
    }
  }
  if (!ok) {
    A.status[n] = ST_CORRUPT;
    return;
  }
  if constexpr (SAMPLE) {
  } else if constexpr (K >= 8) {
    stream_begin(PS);
  } else if constexpr (K == 4) {
    // the initial state: the stream's first bytes, most significant first,
    // read while x < L (at most four)
    RS.fill(0, p);
    const uint32_t w0 = (uint32_t)__shfl((int)RS.word, g << 4);  // bytes 0..3
    uint32_t xs = 0u, ps = 0u;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const bool rd = xs < RANS_L && ps < RS.len;
      xs = rd ? ((xs << 8) | ((w0 >> (8 * b)) & 255u)) : xs;
      ps += rd ? 1u : 0u;
    }
    RS.x = xs;
    RS.pos = ps;
  } else {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      R[k].fill(0, lane);
      uint32_t xs = 0u, ps = 0u;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const bool rd = xs < RANS_L && ps < R[k].len;
        xs = rd ? ((xs << 8) | R[k].byte_at((uint32_t)b)) : xs;
        ps += rd ? 1u : 0u;
      }
      x[k] = xs;
      pos[k] = ps;
    }
  }
  float* prm = (float*)(piv + PIV_WORDS);
  uint8_t* img = D.px;
  const int o = H_ + 1;
  const bool raster = A.order == 0;
  // sheared layout: this wave's window of the lane's sheared canvas, cleared
  // (its h top rows stay 0: the padding above the lane)
  constexpr bool shear = SHEAR;
  const int rows = A.ring_rows;
  int16_t* ring = nullptr;
  if constexpr (shear) {
    // workgroups are dealt to the XCDs in turn: the windows of one XCD's
    // waves are kept contiguous, so they spread over its L2 sets
    const int nwv = (int)(blockDim.x >> 6);
    const int xcd_blocks = (int)((gridDim.x + RING_XCDS - 1) / RING_XCDS);
    const int slot = (int)(blockIdx.x % RING_XCDS) * xcd_blocks + (int)(blockIdx.x / RING_XCDS);
    const int wave = uniform(slot * nwv + (int)(threadIdx.x >> 6));
    ring = (int16_t*)(A.ring + (int64_t)wave * ring_wave_bytes(rows));
    uint32_t* r32 = (uint32_t*)ring;
    const int nw = (int)(ring_wave_bytes(rows) >> 2);
    for (int k = lane; k < nw; k += 64) r32[k] = 0u;
    __threadfence_block();
  }
  const int64_t ngroups = raster ? (int64_t)Hl * Wl : (int64_t)Wl + (int64_t)o * (Hl - 1);
  uint32_t* dump = TRACE ? A.sym_dump + D.px_base * 3 : nullptr;
  TapCodes<H_> tc;
  tc.init(g);

  for (int64_t gi = 0; gi < ngroups; ++gi) {
    int ilo, ihi;
    if (raster) {
      ilo = ihi = (int)(gi / Wl);
    } else {
      step_rows((int)gi, Hl, Wl, o, ilo, ihi);
    }
    if constexpr (shear) {
      // column gi of the window: the step's rows [ilo, ihi] are written as
      // they decode; of the other rows (no pixel at this column) only those
      // a later read can reach are cleared: a pixel of step t' in (gi, gi +
      // h(h+2)] reads rows i - h .. i with ilo(gi) <= ilo(t') <= i <=
      // ihi(t') <= ihi(gi) + h + 1, so rows [ilo - h, ihi + h + 1] (at most
      // 2h + 1 of them besides the step's); the rest are never read before
      // the column is rewritten 16 steps later
      int16_t* cb = ring + (int64_t)(gi & (RING_COLS - 1)) * 3 * rows + H_;
      const int r = (ilo <= ihi ? (lane < H_ ? ilo - H_ + lane : ihi + 1 + (lane - H_))
                                : ilo - H_ + lane);
      const int nz = ilo <= ihi ? 2 * H_ + 1 : 2 * H_ + 1 + (ihi + 1 - ilo);
      if (lane < nz && r >= 0 && r < Hl) {
        cb[r] = 0;
        cb[rows + r] = 0;
        cb[2 * rows + r] = 0;
      }
      __threadfence_block();
    }
    for (int ts = ilo; ts <= ihi; ts += 16) {
      const int na = min(16, ihi - ts + 1);
      const int i = ts + p;
      const bool active = p < na;
      const int j = raster ? (int)(gi - (int64_t)ilo * Wl) : (int)gi - o * i;
      float ctx[conv_chunks(H_)];
      tc.refresh();
      if constexpr (shear)
        gather_ring<H_>(ctx, tc, ring, rows, (int)gi, min(i, Hl - 1), active);
      else
        gather<H_>(ctx, tc, img, D.W, y0, x0, Hl, Wl, i, j, active);
      // sampling: the slots of pixel p (every lane group draws the same)
      uint32_t sl[3] = {0u, 0u, 0u};
      if constexpr (SAMPLE) sample_slots(D.seed, D.W, y0 + i, x0 + j, sl);
      f4 head[HEAD_TILES];
      net_forward<H_, C_>(lds_weights(w), A.nb, ctx, head, lane);
      Mix M;
      mix_prep(head, M, has2);
      int xv[3] = {0, 0, 0};
      float xr = 0.0f, xg = 0.0f;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        Chan Q;
        chan_params(M, c, xr, xg, Q);
        if constexpr (SAMPLE) {
          // the v with cdf(v) <= slot < cdf(v + 1): eight halvings of
          // [0, 256] with cdf(0) = 0 <= slot < cdf(256) = 2^16 kept; the
          // evaluations are the encoder's (cdf_eval), so the draw is the
          // inverse of the coder's own row
          int lo = 0;
#pragma unroll
          for (int it = 0; it < 8; ++it) {
            const int mid = lo + (128 >> it);
            const bool le = cdf_quant(mid, cdf_eval(mid, Q.w, Q.a, Q.b)) <= sl[c];
            lo = le ? mid : lo;
          }
          if (c == 0) xv[0] = lo;
          else if (c == 1) xv[1] = lo;
          else xv[2] = lo;
        } else if constexpr (K >= 8) {
          // every pixel's symbol from its own stream (pop_own); K = 8 pops
          // rows 0..7, then rows 8..15
#pragma unroll
          for (int half = 0; half < 16 / K; ++half) {
            const int q0 = half * K;
            if (q0 >= na) break;
            const bool act = p >= q0 && p < q0 + K && p < na;
            uint32_t start, freq;
            const int sy = pop_own(Q, PS, act, start, freq);
            if (act) {
              if (c == 0) xv[0] = sy;
              else if (c == 1) xv[1] = sy;
              else xv[2] = sy;
            }
            if (TRACE && act && g == 0)
              dump[((int64_t)(y0 + i) * D.W + (x0 + j)) * 3 + c] = start | (freq << 16);
            if constexpr (K == 8) {
              // rows p and p + 8 share a stream: the other half takes the new state
              const uint32_t ox = (uint32_t)__shfl_xor((int)PS.x, 8);
              const uint32_t op = (uint32_t)__shfl_xor((int)PS.pos, 8);
              const bool mine = p >= q0 && p < q0 + K;
              PS.x = mine ? PS.x : ox;
              PS.pos = mine ? PS.pos : op;
            }
          }
        } else if constexpr (K == 4) {
          // stage the channel's mixtures: lane (p, g) holds components g + 4 j
          float* mine = prm + p * PRM_STRIDE;
#pragma unroll
          for (int j = 0; j < 3; ++j) {
            const int m = g + 4 * j;
            mine[3 * m] = Q.w[j];
            mine[3 * m + 1] = Q.a[j];
            mine[3 * m + 2] = Q.b[j];
          }
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
          // pops: row g takes row ts + q0 + g of the group (stream g); lane p
          // of the row first evaluates pivot p of that pixel, the cdf at
          // k = 16 (p + 1) (p = 15 stands for k = 256): it does not depend on
          // the coder state, and only the rows that are popped are evaluated
          for (int q0 = 0; q0 < na; q0 += 4) {
            const int pr = q0 + g;
            const bool act = pr < na;
            const int prc = min(pr, 15);
            Mix10 P;
            load_mix10(P, prm, prc);
            const int kp = min(16 * (p + 1), 255);
            const uint32_t pq = cdf_quant(kp, cdf_eval10(kp, P));
            const uint32_t pv = p < 15 ? pq : CDF_TOTAL;
            // a state below 2^16 (the end of the stream) holds a spread slot:
            // the symbol is searched with its reversal
            const bool small = RS.x < CDF_TOTAL;
            const uint32_t slot = small ? rev16(RS.x) : (RS.x & 0xffffu);
            const int b = row_count(__ballot(pv <= slot), g);
            const int k2 = 16 * b + p;
            const uint32_t c2 = cdf_quant(k2, cdf_eval10(max(k2, 1), P));
            const int cnt = row_count(__ballot(c2 <= slot) & 0xfffefffefffefffeull, g);
            const int sy = 16 * b + cnt;
            const int rb = g << 4;
            // start = cdf(16 b + cnt): lane cnt's value, lane 0's being the
            // bucket's lower edge cdf(16 b) (the same evaluation as pivot
            // b - 1), except cdf(0) = 0; end = cdf(16 b + cnt + 1): lane
            // cnt + 1's value, or the bucket's upper edge, pivot b
            const uint32_t st_r = (uint32_t)__shfl((int)c2, rb | cnt);
            const uint32_t nc_r = (uint32_t)__shfl((int)c2, rb | ((cnt + 1) & 15));
            const uint32_t np_r = (uint32_t)__shfl((int)pv, rb | b);
            const uint32_t start = (b == 0 && cnt == 0) ? 0u : st_r;
            const uint32_t freq = (cnt < 15 ? nc_r : np_r) - start;
            uint32_t xn = freq * (RS.x >> 16) + slot - start;
            if (__ballot(small && act) != 0ull) {  // rare: a stream's last few pops
              const uint32_t xr = spread_rank(RS.x, start, freq);
              xn = small ? xr : xn;
            }
            RS.x = act ? xn : RS.x;
            RS.renorm(act, p, g);
            // the symbol of pixel p (decoded by row p - q0) to all its lanes
            const int src = p - q0;
            const int sv = __shfl(sy, (src & 3) << 4);
            if (src >= 0 && src < 4) {
              if (c == 0) xv[0] = sv;
              else if (c == 1) xv[1] = sv;
              else xv[2] = sv;
            }
            if (TRACE && act && p == 0) {
              const int ii = ts + pr;
              const int jj = raster ? (int)(gi - (int64_t)ilo * Wl) : (int)gi - o * ii;
              dump[((int64_t)(y0 + ii) * D.W + (x0 + jj)) * 3 + c] = start | (freq << 16);
            }
          }
        } else {
        // pivot CDF values of every pixel of the group: cdf at k = 16 (j + 1),
        // j = 0..14, and 2^16 for k = 256 (independent evaluations)
#pragma unroll 5
        for (int jp = 0; jp < 15; ++jp) {
          const uint32_t v = cdf_quant(16 * (jp + 1), cdf_eval(16 * (jp + 1), Q.w, Q.a, Q.b));
          if (g == 0) piv[p * 16 + jp] = v;
        }
        if (g == 0) piv[p * 16 + 15] = CDF_TOTAL;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // pops, K per iteration (one per stream); the next iteration's pivot
        // rows and mixtures (which do not depend on the coder states) are
        // fetched one iteration ahead; rows past the group are clamped and
        // their results unused
        float nw[K][3], nA[K][3], nB[K][3];
        uint32_t npv[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const int src = (g << 4) | k;
#pragma unroll
          for (int j = 0; j < 3; ++j) {
            nw[k][j] = __shfl(Q.w[j], src);
            nA[k][j] = __shfl(Q.a[j], src);
            nB[k][j] = __shfl(Q.b[j], src);
          }
          npv[k] = piv[k * 16 + p];
        }
        for (int q0 = 0; q0 < na; q0 += K) {
          float bw[K][3], bA[K][3], bB[K][3];
          uint32_t pv[K];
#pragma unroll
          for (int k = 0; k < K; ++k) {
#pragma unroll
            for (int j = 0; j < 3; ++j) {
              bw[k][j] = nw[k][j];
              bA[k][j] = nA[k][j];
              bB[k][j] = nB[k][j];
            }
            pv[k] = npv[k];
            const int nx = min(q0 + K + k, 15);
            const int src = (g << 4) | nx;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
              nw[k][j] = __shfl(Q.w[j], src);
              nA[k][j] = __shfl(Q.a[j], src);
              nB[k][j] = __shfl(Q.b[j], src);
            }
            npv[k] = piv[nx * 16 + p];
          }
          uint32_t slot[K], start[K], freq[K];
          int sym[K];
#pragma unroll
          for (int k = 0; k < K; ++k) {
            slot[k] = x[k] < CDF_TOTAL ? rev16(x[k]) : (x[k] & 0xffffu);  // spread slot below 2^16
            // bucket: pivots of the pixel at or below the slot (pv of lane p =
            // cdf at 16 (p + 1); lane 15 holds 2^16, so b <= 15)
            const int b = __popcll(__ballot(pv[k] <= slot[k]) & 0xffffull);
            // inside the bucket: cdf at k = 16 b + p for p = 1..15; the
            // bucket's lower bound (p = 0) is cdf at 16 b <= slot
            const int k2 = 16 * b + p;
            const uint32_t c2 = cdf_quant(k2, cdf_eval(max(k2, 1), bw[k], bA[k], bB[k]));
            const int cnt = __popcll(__ballot(c2 <= slot[k]) & 0xfffeull);
            sym[k] = 16 * b + cnt;
            // bounds of the symbol, every read unconditional (no branches)
            const uint32_t lo_r = (uint32_t)__builtin_amdgcn_readlane((int)pv[k], (b + 15) & 15);
            const uint32_t st_r = (uint32_t)__builtin_amdgcn_readlane((int)c2, cnt);
            const uint32_t nc_r = (uint32_t)__builtin_amdgcn_readlane((int)c2, (cnt + 1) & 15);
            const uint32_t np_r = (uint32_t)__builtin_amdgcn_readlane((int)pv[k], b);
            const uint32_t lo = b == 0 ? 0u : lo_r;
            start[k] = cnt == 0 ? lo : st_r;
            freq[k] = (cnt < 15 ? nc_r : np_r) - start[k];
          }
#pragma unroll
          for (int k = 0; k < K; ++k) {
            const bool act = q0 + k < na;
            uint32_t xn = freq[k] * (x[k] >> 16) + slot[k] - start[k];
            if (x[k] < CDF_TOTAL) xn = spread_rank(x[k], start[k], freq[k]);  // wave-uniform
            x[k] = act ? xn : x[k];
            R[k].renorm(x[k], pos[k], lane, act);
            if (p == q0 + k) {
              if (c == 0) xv[0] = sym[k];
              else if (c == 1) xv[1] = sym[k];
              else xv[2] = sym[k];
            }
            if (TRACE && act) {  // every lane stores the same value
              const int ii = ts + q0 + k;
              const int jj = raster ? (int)(gi - (int64_t)ilo * Wl) : (int)gi - o * ii;
              dump[((int64_t)(y0 + ii) * D.W + (x0 + jj)) * 3 + c] = start[k] | (freq[k] << 16);
            }
          }
        }
        }  // K < 4
        if (c == 0) {
          posterior(M, xv[0], Q.mu, Q.is, has2);
          xr = normalise(xv[0]);
        } else if (c == 1) {
          posterior(M, xv[1], Q.mu, Q.is, has2);
          xg = normalise(xv[1]);
        }
      }
      if (active && g == 0) {
        uint8_t* dst = img + ((int64_t)(y0 + i) * D.W + (x0 + j)) * 3;
        dst[0] = (uint8_t)xv[0];
        dst[1] = (uint8_t)xv[1];
        dst[2] = (uint8_t)xv[2];
        if constexpr (shear) {
          int16_t* cb = ring + (int64_t)(gi & (RING_COLS - 1)) * 3 * rows + H_ + i;
          cb[0] = (int16_t)(2 * xv[0] - 255);
          cb[rows] = (int16_t)(2 * xv[1] - 255);
          cb[2 * rows] = (int16_t)(2 * xv[2] - 255);
        }
      }
      // make this group's pixels visible to the wave's later gathers
      __threadfence_block();
    }
  }
  bool clean = true;
  if constexpr (SAMPLE) {
  } else if constexpr (K >= 8) {
    clean = __ballot(PS.x == RANS_X0 && PS.pos == PS.len) == ~0ull;
  } else if constexpr (K == 4) {
    clean = __ballot(RS.x == RANS_X0 && RS.pos == RS.len) == ~0ull;
  } else {
#pragma unroll
    for (int k = 0; k < K; ++k) clean = clean && x[k] == RANS_X0 && pos[k] == R[k].len;
  }
  if (!clean) A.status[n] = ST_CORRUPT;
}

template <int H_, int C_, bool TRACE, int K, bool SAMPLE, bool SHEAR>
__global__ void __launch_bounds__(NWAVES_DEC * 64) k_decode(DecArgs A) {
  extern __shared__ float4 smem_f4[];
  float* w = (float*)smem_f4;
  load_weights(w, A.w, A.wfloats);
  const int lane = threadIdx.x & 63;
  uint32_t* piv = (uint32_t*)(w + A.wfloats) + (threadIdx.x >> 6) * WAVE_LDS_WORDS;
  for (;;) {
    // one queue pop per wave, by its first active lane, broadcast
    const int leader = uniform(lane);
    int L = 0;
    if (lane == leader) L = atomicAdd(A.counter, 1);
    L = uniform(L);
    if ((int64_t)L >= A.n_lanes) break;
    decode_lane<H_, C_, TRACE, K, SAMPLE, SHEAR>(A, w, piv, L, lane);
  }
}

// ------------------------------------------------------------------ row streams
// Row streams (one rANS stream per lane row): a lane is decoded in bands of
// ROW_BAND = 16 rows, one workgroup of ROW_WAVES = 4 waves (one per SIMD) per
// band, so one wavefront step of a band, up to 16 pixels, is shared by a whole
// CU: the network is split by output tiles (net_forward_split, activations
// exchanged through LDS), then each wave decodes four of the band's rows with
// 16 lanes per pixel, one mixture component per lane. Each row pops its own
// stream, so every row of a step decodes at once (the whole step of
// Algorithm 1 in parallel); a row's coder state stays in the registers of
// the lanes that decode it. A band's top rows read the h rows above, decoded
// by the band above it, possibly on another CU: each band publishes how many
// steps it has finished (release), and waits before step t until the band
// above has finished step t - 1 (acquire). Bands are taken from the queue in
// order (by the step they start at, across the images of the batch), so the
// band above is always held by a running or finished workgroup; its skew of
// (h + 1) ROW_BAND steps makes waits rare once a band has started. A wait also
// ends, with the image marked corrupt, if it exceeds band_wait_ticks of the
// 100 MHz clock (20 s unless a test lowers it), so every workgroup reaches
// the end of the kernel whatever happens.
constexpr int32_t BAND_DONE = 0x7fffffff;

NXD int find_img_band(const ImgDesc* __restrict__ d, int n, int64_t key) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    const int64_t b = uniform64(d[mid].band_base);
    if (b <= key) lo = mid; else hi = mid - 1;
  }
  return uniform(lo);
}

NXD void band_publish(int32_t* slot, int32_t v) {
  __hip_atomic_store(slot, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

template <int H_, int C_, bool TRACE>
__device__ void decode_band(const DecArgs& A, const float* w, float* xb, float* hb, float* cb, int32_t* sh,
                            int64_t B) {
  static_assert(ROW_BAND == 16 && ROW_WAVES == 4, "a band is one 16-pixel tile, four rows per wave");
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int p = lane & 15;                 // network phase: the tile's pixel p is band row p
  const int m = lane & 15, pp = 4 * wave + (lane >> 4);  // mixture phase: component m of band row pp
  const int n = find_img_band(A.desc, A.n_img, B);
  const ImgDesc D = uniform_desc(A.desc + n);
  // which lane of the image and which band of it: lanes in order, full patch
  // rows first, each lane cut into bands_of(Hl) bands
  const int64_t bi = B - D.band_base;
  const int64_t per_prow = (int64_t)D.nlx * bands_of(D.ph);
  const int ly = (int)(bi / per_prow);
  const int y0 = ly * D.ph, Hl = min(D.ph, D.H - y0);
  const int64_t rem = bi - (int64_t)ly * per_prow;
  const int lx = (int)(rem / bands_of(Hl)), bb = (int)(rem - (int64_t)lx * bands_of(Hl));
  const int x0 = lx * D.pw, Wl = min(D.pw, D.W - x0);
  const int nl = D.nlx * D.nly;
  const int r0 = bb * ROW_BAND, r1 = min(Hl, r0 + ROW_BAND) - 1, nrows = r1 - r0 + 1;
  int32_t* mine = A.progress + B;
  // header and stream table (every lane reads the same bytes)
  const uint8_t* C = A.in + uniform64((int64_t)A.in_off[n]);
  const int64_t clen = uniform64((int64_t)(A.in_off[n + 1] - A.in_off[n]));
  const int64_t ns = image_streams(ROW_STREAMS, D.H, D.nlx, D.nly);
  const int64_t pay = HDR_BYTES + 4 * ns;
  bool ok = clen >= pay;
  bool mismatch = false;
  if (ok) {
    const uint32_t ph = D.ph == D.H ? 0u : (uint32_t)D.ph, pw = D.pw == D.W ? 0u : (uint32_t)D.pw;
    ok = C[0] == 'N' && C[1] == 'L' && C[2] == 'X' && C[3] == 'C' && C[4] == CONTAINER_VERSION && C[5] == 1 &&
         C[6] == (uint8_t)H_ && C[7] == (uint8_t)ROW_STREAMS && rd_u32(C + 8) == (uint32_t)D.H &&
         rd_u32(C + 12) == (uint32_t)D.W && (uint32_t)(C[16] | (C[17] << 8)) == ph &&
         (uint32_t)(C[18] | (C[19] << 8)) == pw && rd_u32(C + 28) == (uint32_t)nl;
    ok = ok && pay + (int64_t)rd_u32(C + HDR_BYTES + 4 * (ns - 1)) == clen;
    ok = uniform(ok ? 1 : 0) != 0;
    if (ok) {
      const uint64_t hsh = (uint64_t)rd_u32(C + 20) | ((uint64_t)rd_u32(C + 24) << 32);
      mismatch = uniform(hsh != A.model_hash ? 1 : 0) != 0;
    }
  }
  // this lane's row stream (band row pp; rows past the band's last take the
  // last row's and never pop), in every lane of the row's pixel
  const int64_t ebase = row_entry_base(ly, lx, D.nlx, D.ph, Hl) + r0;
  if (threadIdx.x == 0) sh[0] = 1;
  __syncthreads();
  PixStream P;
  P.x = 0u;
  P.pos = 0u;
  P.len = 1u;
  P.S = as_global(C);
  if (ok && !mismatch) {
    const int64_t e = ebase + min(pp, nrows - 1);
    const uint32_t lend = rd_u32(C + HDR_BYTES + 4 * e);
    const uint32_t lstart = e > 0 ? rd_u32(C + HDR_BYTES + 4 * (e - 1)) : 0u;
    const bool okr = lstart <= lend && pay + (int64_t)lend <= clen && lend - lstart >= 1;
    if (okr) {
      P.S = as_global(C + pay + lstart);
      P.len = lend - lstart;
      stream_begin(P);
    } else {
      sh[0] = 0;
    }
  }
  __syncthreads();
  ok = ok && sh[0] != 0;
  if (mismatch || !ok) {
    if (threadIdx.x == 0) {
      A.status[n] = mismatch ? ST_MISMATCH : ST_CORRUPT;
      band_publish(mine, BAND_DONE);  // the band below must not wait for this one
    }
    __syncthreads();
    return;
  }
  uint8_t* img = D.px;
  const int o = H_ + 1;
  const int t_lo = o * r0, t_hi = (Wl - 1) + o * r1;
  uint32_t* dump = TRACE ? A.sym_dump + D.px_base * 3 : nullptr;
  int32_t seen = bb == 0 ? BAND_DONE : 0;  // steps of the band above known to be finished
  for (int t = t_lo; t <= t_hi; ++t) {
    if (seen < t) {
      // wait until the band above has finished step t - 1
      if (threadIdx.x == 0) {
        const int32_t* above = A.progress + (B - 1);
        int32_t v = __hip_atomic_load(above, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        if (v < t) {
          const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
          while (v < t) {
            __builtin_amdgcn_s_sleep(4);
            v = __hip_atomic_load(above, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
            if (v < t && __builtin_amdgcn_s_memrealtime() - t0 > A.band_wait_ticks) {
              A.status[n] = ST_CORRUPT;  // never expected: the image cannot be trusted
              v = BAND_DONE;
            }
          }
        }
        sh[1] = v;
      }
      __syncthreads();
      seen = sh[1];
    }
    // this band's step t - 1 is finished in every wave (its pixels stored)
    __syncthreads();
    if (threadIdx.x == 0) band_publish(mine, t);
    int ilo, ihi;
    step_rows(t, Hl, Wl, o, ilo, ihi);
    const int a = max(ilo, r0), bmax = min(ihi, r1);
    if (a > bmax) continue;  // the same for the whole workgroup
    // network: the waves gather a share of the tile's contexts each, then
    // compute their share of the layers
    {
      const int i = r0 + p;
      const bool active = i >= a && i <= bmax;
      float ctx[conv_chunks(H_)];
      gather_shared<H_, ROW_WAVES>(ctx, img, D.W, y0, x0, Hl, Wl, i, t - o * i, active, wave, cb, lane);
      net_forward_split<H_, C_, ROW_WAVES>(lds_weights(w), A.nb, ctx, xb, hb, lane, wave);
    }
    // mixture and pops: band row pp, component m
    const int i = r0 + pp;
    const bool act = i >= a && i <= bmax;
    const int j = t - o * i;
    const bool live = m < 10;
    Mix16 M;
    mix_prep16(hb + pp * 128, m, M);
    int xv[3] = {0, 0, 0};
    float xr = 0.0f, xg = 0.0f;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      Chan16 Q;
      chan_params16(M, c, xr, xg, Q);
      uint32_t start, freq;
      const int sy = pop16(Q, P, act, start, freq);
      if (c == 0) xv[0] = sy;
      else if (c == 1) xv[1] = sy;
      else xv[2] = sy;
      if (TRACE && act && m == 0)
        dump[((int64_t)(y0 + i) * D.W + (x0 + j)) * 3 + c] = start | (freq << 16);
      if (c == 0) {
        posterior16(M, xv[0], Q, live);
        xr = normalise(xv[0]);
      } else if (c == 1) {
        posterior16(M, xv[1], Q, live);
        xg = normalise(xv[1]);
      }
    }
    if (act && m == 0) {
      uint8_t* dst = img + ((int64_t)(y0 + i) * D.W + (x0 + j)) * 3;
      dst[0] = (uint8_t)xv[0];
      dst[1] = (uint8_t)xv[1];
      dst[2] = (uint8_t)xv[2];
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) band_publish(mine, BAND_DONE);
  // every row's stream must end in the start state with every byte read
  if (pp < nrows && m == 0 && !(P.x == RANS_X0 && P.pos == P.len)) A.status[n] = ST_CORRUPT;
  __syncthreads();
}

// LDS of the row decoder after the weights: two activation exchange buffers
// of C/16 tiles, the band's 16 x 128 head rows, the tile's contexts (64 lanes
// x gather_stride), then a few shared words
template <int H_, int C_>
constexpr size_t rows_lds_extra() {
  return (size_t)(2 * (C_ / 16) * 256 + ROW_BAND * 128 + 64 * gather_stride<H_>()) * sizeof(float) +
         4 * sizeof(int32_t);
}

template <int H_, int C_, bool TRACE>
__global__ void __launch_bounds__(ROW_WAVES * 64) k_decode_rows(DecArgs A) {
  extern __shared__ float4 smem_f4[];
  float* w = (float*)smem_f4;
  load_weights(w, A.w, A.wfloats);
  float* xb = w + A.wfloats;
  float* hb = xb + 2 * (C_ / 16) * 256;
  float* cb = hb + ROW_BAND * 128;
  int32_t* sh = (int32_t*)(cb + 64 * gather_stride<H_>());  // band, wait and flag words shared by the workgroup
  for (;;) {
    if (threadIdx.x == 0) sh[2] = atomicAdd(A.counter, 1);
    __syncthreads();
    const int64_t Q = sh[2];
    __syncthreads();
    if (Q >= A.n_bands) break;
    // the queue's order of the bands (start step, then image and lane), or image order
    const int64_t B = A.band_order ? (int64_t)uniform(A.band_order[Q]) : Q;
    if (B < 0 || B >= A.n_bands) continue;  // only a damaged workspace: never decode out of range
    decode_band<H_, C_, TRACE>(A, w, xb, hb, cb, sh, B);
  }
}

__global__ void k_decode_prep(int32_t* status, int n_img, int32_t* counter, int32_t* progress, int64_t n_bands) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (status && i < n_img) status[i] = ST_OK;
  if (progress && i < n_bands) progress[i] = 0;
  if (i == 0) *counter = 0;
}

// per image: sum of per-pixel bits in double, in a fixed order: block (n, r)
// sums part r of image n (thread-strided partial sums, then a fixed tree),
// then one thread per image adds the REDUCE_PARTS partials in order
__global__ void __launch_bounds__(256) k_reduce_bits(const ImgDesc* desc, const float* bits, double* part_out) {
  __shared__ double part[256];
  const ImgDesc D = desc[blockIdx.x];
  const int64_t npx = (int64_t)D.H * D.W;
  const int64_t per = (npx + REDUCE_PARTS - 1) / REDUCE_PARTS;
  const int64_t lo = (int64_t)blockIdx.y * per, hi = lo + per < npx ? lo + per : npx;
  double s = 0.0;
  for (int64_t k = lo + threadIdx.x; k < hi; k += 256) s += (double)bits[D.px_base + k];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) part[threadIdx.x] += part[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part_out[(int64_t)blockIdx.x * REDUCE_PARTS + blockIdx.y] = part[0];
}

__global__ void k_reduce_final(const double* part, int n_img, double* out) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= n_img) return;
  double s = 0.0;
  for (int r = 0; r < REDUCE_PARTS; ++r) s += part[(int64_t)n * REDUCE_PARTS + r];
  out[n] = s;
}

// ------------------------------------------------------------------ monotonicity check
// The quantised CDF is monotone in k (every frequency >= 1) only if the
// hardware exp2 is non-decreasing and the reciprocal non-increasing on the
// arguments cdf_eval gives them. This scans every finite FP32 value in
// increasing order, a chunk of consecutive values per thread, and counts
// adjacent pairs that break the order: out[0] exp2 on all finite inputs,
// out[1] rcp on [1, FLT_MAX], out[2] rcp(1 + exp2(z)) (non-increasing in z) on
// all finite z, out[3] pairs checked.
constexpr uint32_t MONO_NEG = 0x7F800000u;  // finite negative bit patterns (-FLT_MAX .. -0)
constexpr uint64_t MONO_ALL = 2ull * MONO_NEG;
constexpr uint32_t MONO_CHUNK = 4096;

NXD float mono_value(uint64_t i) {  // i-th finite float in increasing order
  const uint32_t b = i < MONO_NEG ? 0xFF7FFFFFu - (uint32_t)i : (uint32_t)(i - MONO_NEG);
  return __uint_as_float(b);
}

__global__ void __launch_bounds__(256) k_check_monotone(unsigned long long* out) {
  const uint64_t t = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  const uint64_t lo = t * MONO_CHUNK;
  unsigned long long bad_exp = 0, bad_rcp = 0, bad_sig = 0, pairs = 0;
  if (lo < MONO_ALL) {
    const uint64_t hi = lo + MONO_CHUNK < MONO_ALL ? lo + MONO_CHUNK : MONO_ALL;
    const uint64_t first = lo > 0 ? lo - 1 : 0;
    float z = mono_value(first);
    float pe = __builtin_amdgcn_exp2f(z);
    float ps = __builtin_amdgcn_rcpf(1.0f + pe);
    float pr = __builtin_amdgcn_rcpf(z);
    for (uint64_t i = first + 1; i < hi; ++i) {
      z = mono_value(i);
      const float e = __builtin_amdgcn_exp2f(z);
      const float sg = __builtin_amdgcn_rcpf(1.0f + e);
      const float r = __builtin_amdgcn_rcpf(z);
      bad_exp += e < pe ? 1 : 0;
      bad_sig += sg > ps ? 1 : 0;
      // rcp on [1, FLT_MAX]: both values of the pair at or above 1
      bad_rcp += (mono_value(i - 1) >= 1.0f && r > pr) ? 1 : 0;
      ++pairs;
      pe = e;
      ps = sg;
      pr = r;
    }
  }
  if (bad_exp) atomicAdd(out + 0, bad_exp);
  if (bad_rcp) atomicAdd(out + 1, bad_rcp);
  if (bad_sig) atomicAdd(out + 2, bad_sig);
  if (pairs) atomicAdd(out + 3, pairs);
}

__global__ void k_zero4(unsigned long long* out) {
  if (threadIdx.x < 4) out[threadIdx.x] = 0;
}

// ------------------------------------------------------------------ host launchers
bool supported(int h, int C) {
  return (h == 3 && (C == 16 || C == 32 || C == 64)) || (h == 2 && (C == 16 || C == 32 || C == 64)) ||
         (h == 1 && (C == 16 || C == 32));
}

// kernels keep the whole weight image in LDS: allow up to the device limit
template <typename K>
static hipError_t allow_lds(K kernel, size_t lds) {
  const hipError_t e = hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) (void)hipGetLastError();  // reported here, not by the next launch's check
  return e;
}

template <int H_, int C_>
static hipError_t pass_t(const PassArgs& a, int grid, hipStream_t s) {
  const size_t lds = (size_t)a.wfloats * 4;
  hipError_t e = allow_lds(k_pass<H_, C_>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_pass<H_, C_>), dim3(grid), dim3(NWAVES * 64), lds, s, a);
  return hipGetLastError();
}

template <int H_, int C_, bool TRACE, int K, bool SAMPLE = false>
static hipError_t decode_tt(const DecArgs& a, int grid, int waves, hipStream_t s) {
  const size_t lds = (size_t)a.wfloats * 4 + (size_t)waves * WAVE_LDS_WORDS * 4;
  if (a.order == 2)
    hipLaunchKernelGGL((k_decode<H_, C_, TRACE, K, SAMPLE, true>), dim3(grid), dim3(waves * 64), lds, s, a);
  else
    hipLaunchKernelGGL((k_decode<H_, C_, TRACE, K, SAMPLE, false>), dim3(grid), dim3(waves * 64), lds, s, a);
  return hipGetLastError();
}

// the decoder's dynamic LDS limit, raised to the device maximum once per
// kernel before any launch (not a stream operation: kept out of the launch
// path, which a caller may capture)
template <int H_, int C_, int K>
static hipError_t decode_setup_k() {
  int dev = 0, lim = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
  for (int sh = 0; sh < 2 && e == hipSuccess; ++sh) {
    if (e == hipSuccess) e = allow_lds(sh ? k_decode<H_, C_, false, K, false, true> : k_decode<H_, C_, false, K, false, false>, (size_t)lim);
    if (e == hipSuccess) e = allow_lds(sh ? k_decode<H_, C_, true, K, false, true> : k_decode<H_, C_, true, K, false, false>, (size_t)lim);
    if (K == 4 && e == hipSuccess)
      e = allow_lds(sh ? k_decode<H_, C_, false, 4, true, true> : k_decode<H_, C_, false, 4, true, false>, (size_t)lim);
  }
  return e;
}

template <int H_, int C_>
static hipError_t decode_setup(int K) {
  if (K == ROW_STREAMS) {
    int dev = 0, lim = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e == hipSuccess) e = allow_lds(k_decode_rows<H_, C_, false>, (size_t)lim);
    if (e == hipSuccess) e = allow_lds(k_decode_rows<H_, C_, true>, (size_t)lim);
    return e;
  }
  if (K == 2) return decode_setup_k<H_, C_, 2>();
  if (K == 4) return decode_setup_k<H_, C_, 4>();
  if (K == 8) return decode_setup_k<H_, C_, 8>();
  if (K == 16) return decode_setup_k<H_, C_, 16>();
  return decode_setup_k<H_, C_, 1>();
}

template <int H_, int C_, int K>
static hipError_t decode_k(const DecArgs& a, int grid, int waves, hipStream_t s) {
  return a.sym_dump ? decode_tt<H_, C_, true, K>(a, grid, waves, s) : decode_tt<H_, C_, false, K>(a, grid, waves, s);
}

template <int H_, int C_>
static hipError_t sample_t(const DecArgs& a, int grid, int waves, hipStream_t s) {
  return decode_tt<H_, C_, false, 4, true>(a, grid, waves, s);
}

template <int H_, int C_>
static hipError_t decode_t(const DecArgs& a, int grid, int waves, hipStream_t s) {
  if (a.K == 2) return decode_k<H_, C_, 2>(a, grid, waves, s);
  if (a.K == 4) return decode_k<H_, C_, 4>(a, grid, waves, s);
  if (a.K == 8) return decode_k<H_, C_, 8>(a, grid, waves, s);
  if (a.K == 16) return decode_k<H_, C_, 16>(a, grid, waves, s);
  return decode_k<H_, C_, 1>(a, grid, waves, s);
}

#define NX_DISPATCH(FN, h, C, ...)                          \
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

hipError_t launch_pass(int h, int C, const PassArgs& a, int grid, hipStream_t s) {
  if (a.n_tiles == 0) return hipSuccess;
  NX_DISPATCH(pass_t, h, C, a, grid, s);
}

hipError_t prepare_decode(int h, int C, int K) { NX_DISPATCH(decode_setup, h, C, K); }

hipError_t launch_decode(int h, int C, const DecArgs& a, int grid, int waves, hipStream_t s) {
  if (a.n_lanes == 0) return hipSuccess;
  if (waves < 1 || waves > NWAVES_DEC) return hipErrorInvalidValue;
  NX_DISPATCH(decode_t, h, C, a, grid, waves, s);
}

hipError_t launch_sample(int h, int C, const DecArgs& a, int grid, int waves, hipStream_t s) {
  if (a.n_lanes == 0) return hipSuccess;
  if (waves < 1 || waves > NWAVES_DEC) return hipErrorInvalidValue;
  NX_DISPATCH(sample_t, h, C, a, grid, waves, s);
}

template <int O, int K>
static void launch_layout(const RansEncArgs& a, hipStream_t s) {
  hipLaunchKernelGGL((k_rans_counts<O, K>), dim3((unsigned)(a.n_lanes * K)), dim3(64), 0, s, a);
  const unsigned chunks = (unsigned)((a.max_lane_px + SCATTER_PX - 1) / SCATTER_PX);
  hipLaunchKernelGGL((k_rans_scatter<O, K>), dim3((unsigned)a.n_lanes, chunks > 0 ? chunks : 1u), dim3(256), 0, s, a);
}

hipError_t launch_rans_encode(const RansEncArgs& a, hipStream_t s) {
  if (a.n_lanes == 0) return hipSuccess;
  if (a.K == ROW_STREAMS) {
    hipLaunchKernelGGL(k_rans_enc_rows, dim3((unsigned)((a.n_streams + 63) / 64)), dim3(64), 0, s, a);
    return hipGetLastError();
  }
  if (a.h < 1 || a.h > 3 || !valid_interleave(a.K)) return hipErrorInvalidValue;
  const int kx = a.K == 1 ? 0 : a.K == 2 ? 1 : a.K == 4 ? 2 : a.K == 8 ? 3 : 4;
  switch (5 * (a.h - 1) + kx) {
    case 0: launch_layout<2, 1>(a, s); break;
    case 1: launch_layout<2, 2>(a, s); break;
    case 2: launch_layout<2, 4>(a, s); break;
    case 3: launch_layout<2, 8>(a, s); break;
    case 4: launch_layout<2, 16>(a, s); break;
    case 5: launch_layout<3, 1>(a, s); break;
    case 6: launch_layout<3, 2>(a, s); break;
    case 7: launch_layout<3, 4>(a, s); break;
    case 8: launch_layout<3, 8>(a, s); break;
    case 9: launch_layout<3, 16>(a, s); break;
    case 10: launch_layout<4, 1>(a, s); break;
    case 11: launch_layout<4, 2>(a, s); break;
    case 12: launch_layout<4, 4>(a, s); break;
    case 13: launch_layout<4, 8>(a, s); break;
    default: launch_layout<4, 16>(a, s); break;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int grid = (int)((a.n_streams + 63) / 64);
  hipLaunchKernelGGL(k_rans_enc, dim3(grid), dim3(64), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_pack(const PackArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_lane_scan, dim3(a.n_img), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_img_scan, dim3(1), dim3(64), 0, s, a);
  if (a.n_streams > 0) hipLaunchKernelGGL(k_pack, dim3((unsigned)a.n_streams), dim3(64), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_decode_prep(int32_t* status, int n_img, int32_t* counter, hipStream_t s, int32_t* progress,
                              int64_t n_bands) {
  const int64_t items = std::max<int64_t>(std::max<int64_t>(n_img, n_bands), 1);
  hipLaunchKernelGGL(k_decode_prep, dim3((unsigned)((items + 255) / 256)), dim3(256), 0, s, status, n_img, counter,
                     progress, n_bands);
  return hipGetLastError();
}

template <int H_, int C_>
static hipError_t rows_t(const DecArgs& a, int grid, hipStream_t s) {
  const size_t lds = (size_t)a.wfloats * 4 + rows_lds_extra<H_, C_>();
  if (a.sym_dump)
    hipLaunchKernelGGL((k_decode_rows<H_, C_, true>), dim3(grid), dim3(ROW_WAVES * 64), lds, s, a);
  else
    hipLaunchKernelGGL((k_decode_rows<H_, C_, false>), dim3(grid), dim3(ROW_WAVES * 64), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_decode_rows(int h, int C, const DecArgs& a, int grid, hipStream_t s) {
  if (a.n_bands == 0) return hipSuccess;
  NX_DISPATCH(rows_t, h, C, a, grid, s);
}

hipError_t launch_reduce_bits(const ImgDesc* desc, int n_img, const float* bits, double* partials, double* out,
                              hipStream_t s) {
  if (n_img == 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce_bits, dim3(n_img, REDUCE_PARTS), dim3(256), 0, s, desc, bits, partials);
  hipLaunchKernelGGL(k_reduce_final, dim3((n_img + 63) / 64), dim3(64), 0, s, partials, n_img, out);
  return hipGetLastError();
}

}  // namespace nx

namespace nx {
// Scratch of the no-allocation decoder: a file-scope device array that every
// GPU the library runs on holds until the process ends. In host code its name
// is only a stand-in; the device address of each GPU's copy is looked up once
// per device (with that device current) and kept.
static __device__ __align__(256) uint8_t scratch[STATIC_SCRATCH_BYTES];

hipError_t static_scratch(void** ptr) {
  static std::mutex mu;
  static void* addr[64] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = p;
  }
  *ptr = addr[dev];
  return hipSuccess;
}

hipError_t launch_check_monotone(unsigned long long* out, hipStream_t s) {
  hipLaunchKernelGGL(k_zero4, dim3(1), dim3(64), 0, s, out);
  const uint64_t threads = (MONO_ALL + MONO_CHUNK - 1) / MONO_CHUNK;
  hipLaunchKernelGGL(k_check_monotone, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, out);
  return hipGetLastError();
}
}  // namespace nx
