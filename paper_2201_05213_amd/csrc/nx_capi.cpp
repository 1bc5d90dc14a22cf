// nx_capi.cpp -- host runtime behind include/nellox.h: weight-blob parsing and
// device weight image, per-call plans (patch grids, lane and tile counts,
// workspace layout), validation, kernel launches.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "nellox.h"
#include "nx_kernels.hpp"
#include "nx_layout.hpp"

using namespace nx;

namespace {

thread_local std::string g_err;

nellox_status fail(nellox_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

uint32_t rd32(const uint8_t* p) {
  return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) | ((uint32_t)p[3] << 24);
}

uint64_t fnv1a64(const uint8_t* d, size_t n) {
  uint64_t x = 0xcbf29ce484222325ull;
  for (size_t i = 0; i < n; ++i) {
    x ^= d[i];
    x *= 0x100000001b3ull;
  }
  return x;
}

int64_t param_count(int h, int C, int nb) {
  const int64_t K = 2 * h + 1;
  return (int64_t)C * 3 * K * K + C + (int64_t)nb * (2LL * C * C + 2LL * C) + (int64_t)NOUT * C + NOUT;
}

int padded_channels(int C) { return C <= 16 ? 16 : C <= 32 ? 32 : C <= 64 ? 64 : -1; }

int64_t align256(int64_t v) { return (v + 255) & ~(int64_t)255; }

}  // namespace

struct nellox_model {
  int h, C, Cp, nb;
  uint64_t hash;
  float* dw;            // device weight image
  int64_t wfloats;
  int device;
  int num_cu;
  std::mutex mu;        // guards the staging buffer
  void* staging;        // pinned host memory for per-call plans
  size_t staging_bytes;
  hipEvent_t staged;    // recorded after the last plan copy
};

namespace {

// Device weight image in the MFMA operand layout (see nx_layout.hpp).
std::vector<float> weight_image(int h, int C, int Cp, int nb, const float* P) {
  const WeightLayout L = weight_layout(h, Cp, nb);
  std::vector<float> img((size_t)L.total, 0.0f);
  const int K = 2 * h + 1, KC = conv_chunks(h), KQ = conv_quads(h), MT = Cp / 16;
  std::vector<std::pair<int, int>> taps;
  for (int dy = 0; dy <= h; ++dy)
    for (int dx = 0; dx < K; ++dx)
      if (dy < h || dx < h) taps.push_back({dy, dx});
  const float* conv_w = P;
  const float* conv_b = conv_w + (int64_t)C * 3 * K * K;
  const float* blk = conv_b + C;
  const float* head_w = blk + (int64_t)nb * (2LL * C * C + 2LL * C);
  const float* head_b = head_w + (int64_t)NOUT * C;
  // conv: row o, input k = 3 tap + ch
  for (int mt = 0; mt < MT; ++mt)
    for (int kq = 0; kq < KQ; ++kq)
      for (int lane = 0; lane < 64; ++lane)
        for (int q = 0; q < 4; ++q) {
          const int kc = 4 * kq + q;
          if (kc >= KC) continue;
          const int o = 16 * mt + (lane & 15), k = 4 * kc + (lane >> 4);
          float v = 0.0f;
          if (o < C) {
            const int tap = k / 3, ch = k % 3;
            v = conv_w[(((int64_t)o * 3 + ch) * K + taps[tap].first) * K + taps[tap].second];
          }
          img[L.conv + (((int64_t)mt * KQ + kq) * 64 + lane) * 4 + q] = v;
        }
  auto put_1x1 = [&](int64_t base, int mt_out, auto row_src, const float* Wm) {
    for (int mt = 0; mt < mt_out; ++mt)
      for (int ct = 0; ct < MT; ++ct)
        for (int lane = 0; lane < 64; ++lane)
          for (int q = 0; q < 4; ++q) {
            const int r = 16 * mt + (lane & 15), col = 16 * ct + 4 * (lane >> 4) + q;
            const int src = row_src(r);
            img[base + (((int64_t)mt * MT + ct) * 64 + lane) * 4 + q] =
                (src >= 0 && col < C) ? Wm[(int64_t)src * C + col] : 0.0f;
          }
  };
  auto ident = [C](int r) { return r < C ? r : -1; };
  for (int b = 0; b < nb; ++b) {
    const float* w1 = blk + (int64_t)b * (2LL * C * C + 2LL * C);
    const float* b1 = w1 + (int64_t)C * C;
    const float* w2 = b1 + C;
    const float* b2 = w2 + (int64_t)C * C;
    put_1x1(L.layer0 + (2LL * b) * L.layer_stride, MT, ident, w1);
    put_1x1(L.layer0 + (2LL * b + 1) * L.layer_stride, MT, ident, w2);
    for (int o = 0; o < C; ++o) {
      img[L.bias_blocks + (2LL * b) * Cp + o] = b1[o];
      img[L.bias_blocks + (2LL * b + 1) * Cp + o] = b2[o];
    }
  }
  // head rows: MFMA row r = 16 mt + 4 g + v is slot s = 4 mt + v of lane group
  // g, i.e. parameter s % 10 of component g + 4 (s / 10); parameter p of
  // component m is head output 10 p + m
  auto head_src = [](int r) {
    const int mt = r / 16, g = (r % 16) / 4, v = r % 4;
    const int s = 4 * mt + v, m = g + 4 * (s / 10), p = s % 10;
    return (s < 30 && m < NMIX) ? 10 * p + m : -1;
  };
  put_1x1(L.head, HEAD_TILES, head_src, head_w);
  for (int o = 0; o < C; ++o) img[L.bias_conv + o] = conv_b[o];
  for (int r = 0; r < 16 * HEAD_TILES; ++r) {
    const int src = head_src(r);
    img[L.bias_head + r] = src >= 0 ? head_b[src] : 0.0f;
  }
  return img;
}

hipError_t stage_copy(nellox_model* m, void* dst, const void* src, size_t bytes, hipStream_t s) {
  std::lock_guard<std::mutex> lock(m->mu);
  hipError_t e = hipEventSynchronize(m->staged);
  if (e != hipSuccess) return e;
  if (bytes > m->staging_bytes) {
    if (m->staging) (void)hipHostFree(m->staging);
    m->staging = nullptr;
    m->staging_bytes = 0;
    const size_t nb = std::max<size_t>(bytes, 1 << 16);
    e = hipHostMalloc(&m->staging, nb, hipHostMallocDefault);
    if (e != hipSuccess) return e;
    m->staging_bytes = nb;
  }
  memcpy(m->staging, src, bytes);
  e = hipMemcpyAsync(dst, m->staging, bytes, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return e;
  return hipEventRecord(m->staged, s);
}

struct Plan {
  std::vector<ImgDesc> d;
  int64_t n_tiles = 0, n_lanes = 0, n_px = 0, slot_bytes = 0;
};

nellox_status make_plan(int32_t n, const nellox_image* imgs, const nellox_opts* o, Plan& P, bool need_px) {
  if (n < 0) return fail(NELLOX_E_ARG, "n < 0");
  if (n > 0 && !imgs) return fail(NELLOX_E_ARG, "imgs is null");
  if (!o) return fail(NELLOX_E_ARG, "opts is null");
  if (o->order != 0 && o->order != 1) return fail(NELLOX_E_ARG, "order must be 0 (raster) or 1 (wavefront)");
  P.d.resize(n);
  for (int k = 0; k < n; ++k) {
    const nellox_image& im = imgs[k];
    if (im.H < 1 || im.W < 1 || im.H > 65535 || im.W > 65535)
      return fail(NELLOX_E_ARG, "image " + std::to_string(k) + ": H, W must be in 1..65535");
    if (need_px && !im.px) return fail(NELLOX_E_ARG, "image " + std::to_string(k) + ": null pixel pointer");
    ImgDesc& D = P.d[k];
    memset(&D, 0, sizeof(D));
    D.px = im.px;
    D.H = im.H;
    D.W = im.W;
    D.ph = (o->patch_h <= 0 || o->patch_h > im.H) ? im.H : o->patch_h;
    D.pw = (o->patch_w <= 0 || o->patch_w > im.W) ? im.W : o->patch_w;
    D.nlx = (im.W + D.pw - 1) / D.pw;
    D.nly = (im.H + D.ph - 1) / D.ph;
    D.ntx = (im.W + 15) / 16;
    D.lane_base = P.n_lanes;
    D.px_base = P.n_px;
    D.tile_base = P.n_tiles;
    D.slot_base = P.slot_bytes;
    const int64_t npx = (int64_t)im.H * im.W, nl = (int64_t)D.nlx * D.nly;
    P.n_lanes += nl;
    P.n_px += npx;
    P.n_tiles += (int64_t)im.H * D.ntx;
    P.slot_bytes += 6 * npx + 8 * nl;
  }
  return NELLOX_OK;
}

struct WsLayout {
  int64_t desc, sym, slots, lane_len, lane_end, img_bytes, flags, bits, total;
};

WsLayout ws_layout(const Plan& P, int n) {
  WsLayout W{};
  int64_t o = 0;
  W.desc = o; o = align256(o + (int64_t)sizeof(ImgDesc) * std::max(n, 1));
  W.flags = o; o = align256(o + 64);
  W.img_bytes = o; o = align256(o + 8LL * std::max(n, 1));
  W.lane_len = o; o = align256(o + 4 * std::max<int64_t>(P.n_lanes, 1));
  W.lane_end = o; o = align256(o + 4 * std::max<int64_t>(P.n_lanes, 1));
  W.bits = o; o = align256(o + 4 * std::max<int64_t>(P.n_px, 1));
  W.sym = o; o = align256(o + 12 * std::max<int64_t>(P.n_px, 1));
  W.slots = o; o = align256(o + std::max<int64_t>(P.slot_bytes, 1));
  W.total = o;
  return W;
}

nellox_status check_model(const nellox_model* m) {
  if (!m) return fail(NELLOX_E_ARG, "model is null");
  return NELLOX_OK;
}

nellox_status hip_fail(hipError_t e, const char* what) {
  return fail(NELLOX_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

int persistent_grid(const nellox_model* m) { return m->num_cu; }

// upload the plan; fills the PassArgs common fields
nellox_status upload_plan(nellox_model* m, const Plan& P, uint8_t* ws, const WsLayout& W, hipStream_t s) {
  if (P.d.empty()) return NELLOX_OK;
  hipError_t e = stage_copy(m, ws + W.desc, P.d.data(), sizeof(ImgDesc) * P.d.size(), s);
  if (e != hipSuccess) return hip_fail(e, "plan upload");
  return NELLOX_OK;
}

nellox_status run_pass(nellox_model* m, const Plan& P, uint8_t* ws, const WsLayout& W, int mode, uint32_t* sym,
                       float* bits, int32_t* cdf, hipStream_t s) {
  PassArgs a{};
  a.w = m->dw;
  a.wfloats = m->wfloats;
  a.nb = m->nb;
  a.desc = (const ImgDesc*)(ws + W.desc);
  a.n_img = (int)P.d.size();
  a.n_tiles = P.n_tiles;
  a.mode = mode;
  a.sym = sym;
  a.bits = bits;
  a.cdf = cdf;
  const int64_t waves = (P.n_tiles + 0);
  int grid = persistent_grid(m);
  const int64_t need = (waves + 7) / 8;
  if (need < grid) grid = (int)std::max<int64_t>(need, 1);
  hipError_t e = launch_pass(m->h, m->Cp, a, grid, s);
  if (e != hipSuccess) return hip_fail(e, "full-image pass launch");
  return NELLOX_OK;
}

}  // namespace

extern "C" {

const char* nellox_last_error(void) { return g_err.c_str(); }

nellox_status nellox_model_create(const void* blob, size_t nbytes, nellox_model** out) {
  if (!blob || !out) return fail(NELLOX_E_ARG, "blob/out is null");
  *out = nullptr;
  const uint8_t* b = (const uint8_t*)blob;
  if (nbytes < 36 || memcmp(b, "NLXW", 4) != 0) return fail(NELLOX_E_BLOB, "not a weight blob");
  const uint32_t ver = rd32(b + 4), h = rd32(b + 8), C = rd32(b + 12), nb = rd32(b + 16), nmix = rd32(b + 20),
                 flags = rd32(b + 24);
  if (ver != 1) return fail(NELLOX_E_BLOB, "unknown blob version");
  if (nmix != NMIX || flags != 1) return fail(NELLOX_E_BLOB, "blob must have n_mix = 10 and flags = 1");
  if (h < 1 || h > 8 || C < 1 || C > 4096 || nb > 64) return fail(NELLOX_E_BLOB, "dims out of range");
  const int64_t np = param_count((int)h, (int)C, (int)nb);
  if ((int64_t)nbytes != 28 + 4 * np + 8) return fail(NELLOX_E_BLOB, "blob size does not match its dims");
  uint64_t hh = 0;
  for (int k = 0; k < 8; ++k) hh |= (uint64_t)b[nbytes - 8 + k] << (8 * k);
  if (hh != fnv1a64(b, nbytes - 8)) return fail(NELLOX_E_BLOB, "blob hash mismatch");
  const int Cp = padded_channels((int)C);
  if (Cp < 0 || !supported((int)h, Cp)) return fail(NELLOX_E_UNSUPPORTED, "no kernel for these dims");
  std::vector<float> P((size_t)np);
  memcpy(P.data(), b + 28, 4 * (size_t)np);
  std::vector<float> img = weight_image((int)h, (int)C, Cp, (int)nb, P.data());
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
  if (img.size() * 4 + DECODE_LDS_EXTRA > prop.sharedMemPerBlock)
    return fail(NELLOX_E_UNSUPPORTED, "weights exceed the LDS of one workgroup");
  nellox_model* m = new nellox_model();
  m->h = (int)h; m->C = (int)C; m->Cp = Cp; m->nb = (int)nb;
  m->hash = hh;
  m->wfloats = (int64_t)img.size();
  m->device = dev;
  m->num_cu = prop.multiProcessorCount;
  m->staging = nullptr;
  m->staging_bytes = 0;
  e = hipMalloc(&m->dw, img.size() * 4);
  if (e != hipSuccess) { delete m; return hip_fail(e, "hipMalloc(weights)"); }
  e = hipMemcpy(m->dw, img.data(), img.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&m->staged, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventRecord(m->staged, nullptr);
  if (e != hipSuccess) {
    (void)hipFree(m->dw);
    delete m;
    return hip_fail(e, "weight upload");
  }
  // allow the kernels the full LDS of a workgroup
  *out = m;
  return NELLOX_OK;
}

void nellox_model_destroy(nellox_model* m) {
  if (!m) return;
  (void)hipEventSynchronize(m->staged);
  (void)hipEventDestroy(m->staged);
  if (m->staging) (void)hipHostFree(m->staging);
  (void)hipFree(m->dw);
  delete m;
}

nellox_status nellox_model_info(const nellox_model* m, int32_t dims[4], uint64_t* hash) {
  if (!m) return fail(NELLOX_E_ARG, "model is null");
  if (dims) { dims[0] = m->h; dims[1] = m->C; dims[2] = m->nb; dims[3] = NMIX; }
  if (hash) *hash = m->hash;
  return NELLOX_OK;
}

size_t nellox_encode_bound(int32_t H, int32_t W, const nellox_opts* o) {
  if (H < 1 || W < 1) return 0;
  const int ph = (!o || o->patch_h <= 0 || o->patch_h > H) ? H : o->patch_h;
  const int pw = (!o || o->patch_w <= 0 || o->patch_w > W) ? W : o->patch_w;
  const int64_t nl = (int64_t)((H + ph - 1) / ph) * ((W + pw - 1) / pw);
  // header, lane table, per lane 4 flush bytes, at most 2 bytes per symbol
  return (size_t)(HDR_BYTES + 4 * nl + 4 * nl + 6LL * H * W);
}

size_t nellox_workspace_bytes(const nellox_model* m, int32_t n, const nellox_image* imgs, const nellox_opts* o) {
  if (!m) return 0;
  Plan P;
  if (make_plan(n, imgs, o, P, false) != NELLOX_OK) return 0;
  return (size_t)ws_layout(P, n).total;
}

nellox_status nellox_encode(const nellox_model* mc, int32_t n, const nellox_image* imgs, const nellox_opts* o,
                            uint8_t* out, size_t out_cap, uint64_t* out_offsets, void* ws, size_t ws_bytes,
                            void* stream) {
  nellox_model* m = const_cast<nellox_model*>(mc);
  if (check_model(m)) return NELLOX_E_ARG;
  Plan P;
  nellox_status st = make_plan(n, imgs, o, P, true);
  if (st) return st;
  if (!out || !out_offsets || !ws) return fail(NELLOX_E_ARG, "null output/workspace pointer");
  const WsLayout W = ws_layout(P, n);
  if ((int64_t)ws_bytes < W.total) return fail(NELLOX_E_CAPACITY, "workspace too small");
  size_t bound = 0;
  for (int k = 0; k < n; ++k) bound += nellox_encode_bound(imgs[k].H, imgs[k].W, o);
  if (out_cap < bound) return fail(NELLOX_E_CAPACITY, "out_cap below the summed encode bound");
  hipStream_t s = (hipStream_t)stream;
  uint8_t* w8 = (uint8_t*)ws;
  if ((st = upload_plan(m, P, w8, W, s))) return st;
  if ((st = run_pass(m, P, w8, W, 0, (uint32_t*)(w8 + W.sym), nullptr, nullptr, s))) return st;
  RansEncArgs r{};
  r.desc = (const ImgDesc*)(w8 + W.desc);
  r.n_img = n;
  r.n_lanes = P.n_lanes;
  r.order = o->order;
  r.h = m->h;
  r.sym = (const uint32_t*)(w8 + W.sym);
  r.slots = w8 + W.slots;
  r.lane_len = (uint32_t*)(w8 + W.lane_len);
  hipError_t e = launch_rans_encode(r, s);
  if (e != hipSuccess) return hip_fail(e, "rANS encoder launch");
  PackArgs pk{};
  pk.desc = r.desc;
  pk.n_img = n;
  pk.n_lanes = P.n_lanes;
  pk.order = o->order;
  pk.h = m->h;
  pk.model_hash = m->hash;
  pk.slots = w8 + W.slots;
  pk.lane_len = r.lane_len;
  pk.lane_end = (uint32_t*)(w8 + W.lane_end);
  pk.img_bytes = (uint64_t*)(w8 + W.img_bytes);
  pk.out = out;
  pk.out_offsets = out_offsets;
  pk.out_cap = out_cap;
  pk.overflow = (int32_t*)(w8 + W.flags);
  if (n > 0) {
    e = launch_pack(pk, s);
    if (e != hipSuccess) return hip_fail(e, "container packing launch");
  }
  return NELLOX_OK;
}

nellox_status nellox_peek(const uint8_t* c, size_t len, int32_t* H, int32_t* W, nellox_opts* o) {
  if (!c) return fail(NELLOX_E_ARG, "container is null");
  if (len < (size_t)HDR_BYTES || memcmp(c, "NLXC", 4) != 0 || c[4] != CONTAINER_VERSION || c[7] != CODER_RANS8)
    return fail(NELLOX_E_CORRUPT, "not a container of this version");
  const int32_t h = (int32_t)rd32(c + 8), w = (int32_t)rd32(c + 12);
  if (H) *H = h;
  if (W) *W = w;
  if (o) {
    o->order = c[5];
    o->patch_h = c[16] | (c[17] << 8);
    o->patch_w = c[18] | (c[19] << 8);
    o->reserved = 0;
  }
  return NELLOX_OK;
}

static nellox_status decode_impl(const nellox_model* mc, int32_t n, const uint8_t* in, const uint64_t* in_offsets,
                                 const nellox_opts* o, const nellox_image* outs, int32_t* status, uint32_t* dump,
                                 void* ws, size_t ws_bytes, void* stream) {
  nellox_model* m = const_cast<nellox_model*>(mc);
  if (check_model(m)) return NELLOX_E_ARG;
  Plan P;
  nellox_status st = make_plan(n, outs, o, P, true);
  if (st) return st;
  if (n > 0 && (!in || !in_offsets || !status || !ws)) return fail(NELLOX_E_ARG, "null pointer argument");
  const WsLayout W = ws_layout(P, n);
  if ((int64_t)ws_bytes < W.total) return fail(NELLOX_E_CAPACITY, "workspace too small");
  if (n == 0) return NELLOX_OK;
  hipStream_t s = (hipStream_t)stream;
  uint8_t* w8 = (uint8_t*)ws;
  if ((st = upload_plan(m, P, w8, W, s))) return st;
  int32_t* counter = (int32_t*)(w8 + W.flags) + 1;
  hipError_t e = launch_decode_prep(status, n, counter, s);
  if (e != hipSuccess) return hip_fail(e, "decode prep launch");
  DecArgs a{};
  a.w = m->dw;
  a.wfloats = m->wfloats;
  a.nb = m->nb;
  a.desc = (const ImgDesc*)(w8 + W.desc);
  a.n_img = n;
  a.n_lanes = P.n_lanes;
  a.order = o->order;
  a.model_hash = m->hash;
  a.in = in;
  a.in_off = in_offsets;
  a.status = status;
  a.counter = counter;
  a.sym_dump = dump;
  int grid = persistent_grid(m);
  const int64_t need = (P.n_lanes + DECODE_WAVES - 1) / DECODE_WAVES;
  if (need < grid) grid = (int)std::max<int64_t>(need, 1);
  e = launch_decode(m->h, m->Cp, a, grid, s);
  if (e != hipSuccess) return hip_fail(e, "decoder launch");
  return NELLOX_OK;
}

nellox_status nellox_decode(const nellox_model* m, int32_t n, const uint8_t* in, const uint64_t* in_offsets,
                            const nellox_opts* o, const nellox_image* out, int32_t* status, void* ws, size_t ws_bytes,
                            void* stream) {
  return decode_impl(m, n, in, in_offsets, o, out, status, nullptr, ws, ws_bytes, stream);
}

nellox_status nellox_decode_trace(const nellox_model* m, int32_t n, const uint8_t* in, const uint64_t* in_offsets,
                                  const nellox_opts* o, const nellox_image* out, int32_t* status, uint32_t* dump,
                                  void* ws, size_t ws_bytes, void* stream) {
  if (!dump) return fail(NELLOX_E_ARG, "sym_dump is null");
  return decode_impl(m, n, in, in_offsets, o, out, status, dump, ws, ws_bytes, stream);
}

nellox_status nellox_nll(const nellox_model* mc, int32_t n, const nellox_image* imgs, const nellox_opts* o,
                         float* bits_per_px, double* bits_total, void* ws, size_t ws_bytes, void* stream) {
  nellox_model* m = const_cast<nellox_model*>(mc);
  if (check_model(m)) return NELLOX_E_ARG;
  Plan P;
  nellox_status st = make_plan(n, imgs, o, P, true);
  if (st) return st;
  if (n > 0 && (!bits_total || !ws)) return fail(NELLOX_E_ARG, "null pointer argument");
  const WsLayout W = ws_layout(P, n);
  if ((int64_t)ws_bytes < W.total) return fail(NELLOX_E_CAPACITY, "workspace too small");
  if (n == 0) return NELLOX_OK;
  hipStream_t s = (hipStream_t)stream;
  uint8_t* w8 = (uint8_t*)ws;
  if ((st = upload_plan(m, P, w8, W, s))) return st;
  float* bits = bits_per_px ? bits_per_px : (float*)(w8 + W.bits);
  if ((st = run_pass(m, P, w8, W, 1, nullptr, bits, nullptr, s))) return st;
  hipError_t e = launch_reduce_bits((const ImgDesc*)(w8 + W.desc), n, bits, bits_total, s);
  if (e != hipSuccess) return hip_fail(e, "reduction launch");
  return NELLOX_OK;
}

nellox_status nellox_debug_symbols(const nellox_model* mc, int32_t n, const nellox_image* imgs,
                                   const nellox_opts* o, uint32_t* sym, double* ideal, void* ws, size_t ws_bytes,
                                   void* stream) {
  nellox_model* m = const_cast<nellox_model*>(mc);
  if (check_model(m)) return NELLOX_E_ARG;
  Plan P;
  nellox_status st = make_plan(n, imgs, o, P, true);
  if (st) return st;
  if (n > 0 && (!sym || !ws)) return fail(NELLOX_E_ARG, "null pointer argument");
  const WsLayout W = ws_layout(P, n);
  if ((int64_t)ws_bytes < W.total) return fail(NELLOX_E_CAPACITY, "workspace too small");
  if (n == 0) return NELLOX_OK;
  hipStream_t s = (hipStream_t)stream;
  uint8_t* w8 = (uint8_t*)ws;
  if ((st = upload_plan(m, P, w8, W, s))) return st;
  float* bits = (float*)(w8 + W.bits);
  if ((st = run_pass(m, P, w8, W, 0, sym, bits, nullptr, s))) return st;
  if (ideal) {
    hipError_t e = launch_reduce_bits((const ImgDesc*)(w8 + W.desc), n, bits, ideal, s);
    if (e != hipSuccess) return hip_fail(e, "reduction launch");
  }
  return NELLOX_OK;
}

nellox_status nellox_debug_cdf(const nellox_model* mc, const nellox_image* img, const nellox_opts* o, int32_t* cdf,
                               void* ws, size_t ws_bytes, void* stream) {
  nellox_model* m = const_cast<nellox_model*>(mc);
  if (check_model(m)) return NELLOX_E_ARG;
  Plan P;
  nellox_status st = make_plan(1, img, o, P, true);
  if (st) return st;
  if (!cdf || !ws) return fail(NELLOX_E_ARG, "null pointer argument");
  const WsLayout W = ws_layout(P, 1);
  if ((int64_t)ws_bytes < W.total) return fail(NELLOX_E_CAPACITY, "workspace too small");
  hipStream_t s = (hipStream_t)stream;
  uint8_t* w8 = (uint8_t*)ws;
  if ((st = upload_plan(m, P, w8, W, s))) return st;
  return run_pass(m, P, w8, W, 2, nullptr, nullptr, cdf, s);
}

}  // extern "C"
