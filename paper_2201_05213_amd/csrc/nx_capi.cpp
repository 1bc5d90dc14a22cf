// nx_capi.cpp -- host runtime behind include/nellox.h: weight-blob parsing and
// device weight image, per-call plans (patch grids, lane and tile counts,
// workspace layout), validation, kernel launches.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <atomic>
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

// pinned plan staging allocated with the model, so that the no-allocation
// decoder never has to grow it: descriptors of up to 2,730 images
constexpr size_t STAGING_BYTES = (size_t)256 << 10;
// the row decoder's wait limit for launches from now on (nellox_debug_band_wait)
std::atomic<uint64_t> g_band_wait{BAND_WAIT_TICKS};

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
// Weight image of a parameter vector (layout and index map in nx_layout.hpp;
// the training kernels build the same image on the device from the same map).
std::vector<float> weight_image(int h, int C, int Cp, int nb, const float* P) {
  const WeightLayout L = weight_layout(h, Cp, nb);
  std::vector<float> img((size_t)L.total, 0.0f);
  for (int64_t i = 0; i < L.total; ++i) {
    const int64_t src = wimg_src(h, C, Cp, nb, i);
    if (src >= 0) img[(size_t)i] = P[src];
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
  int64_t n_streams = 0, n_bands = 0;  // rANS streams of the batch; row streams: decoding bands
  int K = 1;       // rANS streams per lane (ROW_STREAMS: one per lane row)
  int order = 0;   // 0 raster, 1 wavefront, 2 wavefront decoded in the sheared layout
  int ph_max = 0;  // tallest lane of the batch
  int64_t ring_waves = 0, ring_rows = 0;  // sheared context rings (set by plan_ring)
  int64_t rev_words = 0;    // encoder: coding-order symbol words of all streams
  int64_t after_words = 0;  // encoder: per-step offset entries of all streams
  int64_t max_lane_px = 0;
  // row streams, decoding: the queue order of the bands (band_queue), kept
  // only if it fits the staging buffer beside the descriptors
  std::vector<int32_t> band_order;
};

// the coded order of a request: the sheared layout codes the wavefront order
int coded_order(int order) { return order == 0 ? 0 : 1; }

nellox_status make_plan(int32_t n, const nellox_image* imgs, const nellox_opts* o, Plan& P, bool need_px) {
  if (n < 0) return fail(NELLOX_E_ARG, "n < 0");
  if (n > 0 && !imgs) return fail(NELLOX_E_ARG, "imgs is null");
  if (!o) return fail(NELLOX_E_ARG, "opts is null");
  if (o->order < 0 || o->order > 2)
    return fail(NELLOX_E_ARG, "order must be 0 (raster), 1 (wavefront) or 2 (wavefront, sheared layout)");
  P.order = o->order;
  P.K = o->interleave == -1 ? ROW_STREAMS : o->interleave <= 1 ? 1 : o->interleave;
  if (P.K != ROW_STREAMS && !valid_interleave(P.K))
    return fail(NELLOX_E_ARG, "interleave must be 0, 1, 2, 4, 8, 16, or -1 (a stream per row)");
  if (P.K != 1 && o->order == 0) return fail(NELLOX_E_ARG, "interleaved streams need the wavefront order");
  if (P.K == ROW_STREAMS && o->order == 2)
    return fail(NELLOX_E_ARG, "row streams are decoded in the wavefront order (1), not the sheared layout");
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
    P.ph_max = std::max(P.ph_max, D.ph);
    const int64_t ns = image_streams(P.K, im.H, D.nlx, D.nly);
    D.stream_base = P.n_streams;
    P.n_streams += ns;
    D.rev_base = P.rev_words;
    D.after_base = P.after_words;
    if (P.K == ROW_STREAMS) {
      // a slot of 6 B per pixel and 8 B per row stream; the symbols are read in place
      P.slot_bytes += 6 * npx + 8 * ns;
      D.band_base = P.n_bands;
      P.n_bands += image_bands(im.H, D.ph, D.nlx, D.nly);
    } else {
      P.slot_bytes += P.K * (6 * npx + 8 * nl);
      P.rev_words += nl * P.K * stream_rev_words(D.ph, D.pw, P.K);
      P.after_words += nl * P.K * stream_after_entries(D.ph, D.pw);
    }
    P.max_lane_px = std::max(P.max_lane_px, (int64_t)D.ph * D.pw);
  }
  return NELLOX_OK;
}

// Row streams: the bands of a batch in the order of the wavefront step they
// start at (band bb of a lane starts at step (h + 1) ROW_BAND bb): the bb-th
// band of every lane before any (bb + 1)-th, lanes in image and lane order.
// Each entry is the band's index in image order (band_base, then lanes in
// order, a lane's bands in order), which is what the kernel decomposes. A
// band's upper neighbour comes earlier, so it is always held by a running
// or finished workgroup; and the bands that may run at a time are taken
// together, so an image that comes late in the batch does not wait for the
// CUs of the images before it.
std::vector<int32_t> band_queue(const Plan& P) {
  std::vector<int32_t> q;
  q.reserve((size_t)P.n_bands);
  int max_b = 0;
  for (const ImgDesc& D : P.d) max_b = std::max(max_b, bands_of(D.ph));
  for (int bb = 0; bb < max_b; ++bb)
    for (const ImgDesc& D : P.d)
      for (int ly = 0; ly < D.nly; ++ly) {
        const int Hl = std::min(D.ph, D.H - ly * D.ph), nb = bands_of(Hl);
        if (nb <= bb) continue;
        for (int lx = 0; lx < D.nlx; ++lx)
          q.push_back((int32_t)(D.band_base + (int64_t)ly * D.nlx * bands_of(D.ph) + (int64_t)lx * nb + bb));
      }
  return q;
}

// descriptors, then (row streams) the band order, in one upload
int64_t desc_bytes(const Plan& P, int n) {
  const int64_t d = ((int64_t)sizeof(ImgDesc) * std::max(n, 1) + 15) & ~(int64_t)15;
  return d + (P.K == ROW_STREAMS ? 4 * P.n_bands : 0);
}

// Workspace segments: first those of decoding, sampling, the NLL and the
// debug calls (descriptors, queue counter, sheared windows, per-pixel bits,
// partial sums, row-stream band progress; `small` bytes), then the
// encoder's alone (per-image sizes, stream lengths, symbols, stream slots,
// coding-order buffers).
struct WsLayout {
  int64_t desc, flags, ring, bits, partials, progress, small;
  int64_t img_bytes, lane_len, lane_end, sym, slots, rev, after, total;
};

WsLayout ws_layout(const Plan& P, int n) {
  WsLayout W{};
  int64_t o = 0;
  W.desc = o; o = align256(o + desc_bytes(P, n));
  W.flags = o; o = align256(o + 64);
  W.ring = o; o = align256(o + P.ring_waves * ring_wave_bytes(P.ring_rows));
  W.bits = o; o = align256(o + 4 * std::max<int64_t>(P.n_px, 1));
  W.partials = o; o = align256(o + 8LL * REDUCE_PARTS * std::max(n, 1));
  W.progress = o; o = align256(o + 4 * std::max<int64_t>(P.n_bands, 1));
  W.small = o;
  W.img_bytes = o; o = align256(o + 8LL * std::max(n, 1));
  W.lane_len = o; o = align256(o + 4 * std::max<int64_t>(P.n_streams, 1));
  W.lane_end = o; o = align256(o + 4 * std::max<int64_t>(P.n_streams, 1));
  W.sym = o; o = align256(o + 12 * std::max<int64_t>(P.n_px, 1));
  W.slots = o; o = align256(o + std::max<int64_t>(P.slot_bytes, 1));
  W.rev = o; o = align256(o + 4 * std::max<int64_t>(P.rev_words, 1));
  W.after = o; o = align256(o + 4 * std::max<int64_t>(P.after_words, 1));
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

// the persistent decoder's launch shape: waves per workgroup = lanes per CU
// (at most DECODE_WAVES), one workgroup per CU while lanes remain; the waves
// of a CU share its LDS (weights, pivot tables, cross-lane traffic)
void decode_shape(int64_t n_lanes, int cus, int& grid, int& waves) {
  waves = (int)std::min<int64_t>(DECODE_WAVES, std::max<int64_t>(1, (n_lanes + cus - 1) / cus));
  grid = (int)std::min<int64_t>(cus, (n_lanes + waves - 1) / waves);
}

// sheared layout: one context ring per wave of the launch, RING_COLS columns
// of the tallest lane plus h zero rows on top
void plan_ring(const nellox_model* m, Plan& P) {
  if (P.order != 2 || P.n_lanes == 0) return;
  int grid = 0, waves = 0;
  decode_shape(P.n_lanes, m->num_cu, grid, waves);
  P.ring_waves = ring_windows(grid, waves);
  P.ring_rows = ring_rows_for(P.ph_max, m->h);
}

// upload the plan; fills the PassArgs common fields
nellox_status upload_plan(nellox_model* m, const Plan& P, uint8_t* ws, const WsLayout& W, hipStream_t s) {
  if (P.d.empty()) return NELLOX_OK;
  hipError_t e;
  if (P.band_order.empty()) {
    e = stage_copy(m, ws + W.desc, P.d.data(), sizeof(ImgDesc) * P.d.size(), s);
  } else {
    const int64_t off = desc_bytes(P, (int)P.d.size()) - 4 * P.n_bands;
    std::vector<uint8_t> buf((size_t)desc_bytes(P, (int)P.d.size()), 0);
    memcpy(buf.data(), P.d.data(), sizeof(ImgDesc) * P.d.size());
    memcpy(buf.data() + off, P.band_order.data(), 4 * P.band_order.size());
    e = stage_copy(m, ws + W.desc, buf.data(), buf.size(), s);
  }
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

namespace {
// ------------------------------------------------------------------ training plan
struct TrainPlan {
  int h, C, Cp, nb, KP;
  int n, H, W, ntx;
  int64_t npx, ntiles, chunk, nchunks, ngrad;
  int64_t wfloats, wTfloats;
  // workspace byte offsets
  int64_t wimg, wimgT, bits, ctx, u, theta, delta, dtheta, partial, total;
  // float offsets inside one gradient partial
  int64_t off_conv, off_blocks, off_head, bias_conv, bias_blocks, bias_head;
};

constexpr int TRAIN_MAX_BLOCKS = 4;      // the head's parts, the first layer and 2 n_blocks 1x1 layers in one gradient launch
static_assert(2 * TRAIN_MAX_BLOCKS + 1 + WGRAD_HEAD_PARTS <= WGRAD_MAX_LAYERS, "gradient launch layer table too small");
constexpr int64_t WGRAD_CHUNK_ALIGN = 16;   // weight-gradient chunks: whole 4-pixel K-steps of each of 4 waves

int device_lds_limit() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return 0;
  return v;
}

int device_cus() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 1;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 1;
  return v > 0 ? v : 1;
}

nellox_status train_plan(const int32_t* dims, int32_t n, int32_t H, int32_t W, TrainPlan& T, bool check_lds) {
  if (!dims) return fail(NELLOX_E_ARG, "dims is null");
  const int h = dims[0], C = dims[1], nb = dims[2];
  if (dims[3] != NMIX) return fail(NELLOX_E_ARG, "n_mix must be 10");
  if (h < 1 || h > 3 || C < 1 || C > 64 || nb < 0 || nb > TRAIN_MAX_BLOCKS)
    return fail(NELLOX_E_ARG, "dims out of range (h 1..3, C 1..64, n_blocks 0..4)");
  const int Cp = (C + 15) / 16 * 16;
  if (!supported(h, Cp)) return fail(NELLOX_E_UNSUPPORTED, "no kernel for these dims");
  if (n < 1 || H < 1 || W < 1 || H > 65535 || W > 65535) return fail(NELLOX_E_ARG, "n, H, W out of range");
  T.h = h; T.C = C; T.Cp = Cp; T.nb = nb;
  T.KP = (3 * n_taps(h) + 15) / 16 * 16;
  T.n = n; T.H = H; T.W = W; T.ntx = (W + 15) / 16;
  T.npx = (int64_t)n * H * W;
  T.ntiles = (int64_t)n * H * T.ntx;
  // pixels per weight-gradient partial: as many chunks per layer as make
  // the launch (layer entries x chunks workgroups) fill the device's
  // resident workgroup slots once, so that every workgroup runs at the same
  // time and none is left over to run alone on a mostly idle device
  {
    const int64_t layers = 2LL * nb + 1 + WGRAD_HEAD_PARTS;
    const int64_t slots = std::max(1, wgrad_blocks_per_cu(Cp / 16, T.KP / 16)) * (int64_t)device_cus();
    const int64_t per_layer = std::max<int64_t>(1, slots / layers);
    const int64_t chunk = (T.npx + per_layer - 1) / per_layer;
    T.chunk = std::max(WGRAD_CHUNK_ALIGN, (chunk + WGRAD_CHUNK_ALIGN - 1) / WGRAD_CHUNK_ALIGN * WGRAD_CHUNK_ALIGN);
    T.nchunks = (T.npx + T.chunk - 1) / T.chunk;
  }
  T.wfloats = weight_layout(h, Cp, nb).total;
  T.wTfloats = weightT_layout(Cp, nb).total;
  if (check_lds) {
    const int64_t lim = device_lds_limit();
    if (T.wfloats * 4 > lim || T.wTfloats * 4 > lim)
      return fail(NELLOX_E_UNSUPPORTED, "weights exceed the LDS of one workgroup");
  }
  T.off_conv = 0;
  T.off_blocks = (int64_t)Cp * T.KP;
  T.off_head = T.off_blocks + 2LL * nb * Cp * Cp;
  T.bias_conv = T.off_head + 16LL * HEAD_TILES * Cp;
  T.bias_blocks = T.bias_conv + Cp;
  T.bias_head = T.bias_blocks + 2LL * nb * Cp;
  T.ngrad = T.bias_head + 16 * HEAD_TILES;
  int64_t o = 0;
  auto seg = [&o](int64_t bytes) { const int64_t at = o; o = align256(o + std::max<int64_t>(bytes, 1)); return at; };
  T.wimg = seg(4 * T.wfloats);
  T.wimgT = seg(4 * T.wTfloats);
  T.bits = seg(4 * T.npx);
  T.ctx = seg(4 * T.npx * T.KP);
  T.u = seg(4 * (2LL * nb + 1) * T.npx * Cp);
  T.theta = seg(4 * T.npx * 16 * HEAD_TILES);
  T.delta = seg(4 * (2LL * nb + 1) * T.npx * Cp);
  T.dtheta = seg(4 * T.npx * 16 * HEAD_TILES);
  T.partial = seg(4 * T.nchunks * T.ngrad);
  T.total = o;
  return NELLOX_OK;
}

TrainArgs train_args(const TrainPlan& T, const uint8_t* imgs, uint8_t* ws, const float* grad_bits) {
  TrainArgs a{};
  a.imgs = imgs;
  a.n = T.n; a.H = T.H; a.W = T.W; a.ntx = T.ntx;
  a.npx = T.npx; a.n_tiles = T.ntiles;
  a.nb = T.nb; a.Cp = T.Cp; a.KP = T.KP;
  a.wimg = (const float*)(ws + T.wimg);
  a.wimgT = (const float*)(ws + T.wimgT);
  a.wfloats = T.wfloats; a.wTfloats = T.wTfloats;
  a.bits = (float*)(ws + T.bits);
  a.ctx = (float*)(ws + T.ctx);
  a.u = (float*)(ws + T.u);
  a.theta = (float*)(ws + T.theta);
  a.delta = (float*)(ws + T.delta);
  a.dtheta = (float*)(ws + T.dtheta);
  a.grad_bits = grad_bits;
  return a;
}

int train_grid(const TrainPlan& T) {
  const int64_t need = (T.ntiles + 15) / 16;
  return (int)std::max<int64_t>(1, std::min<int64_t>(need, device_cus()));
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
  e = hipHostMalloc(&m->staging, STAGING_BYTES, hipHostMallocDefault);
  if (e != hipSuccess) {
    (void)hipFree(m->dw);
    delete m;
    return hip_fail(e, "hipHostMalloc(plan staging)");
  }
  m->staging_bytes = STAGING_BYTES;
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
  const int64_t K = !o ? 1 : o->interleave == -1 ? ROW_STREAMS : o->interleave <= 1 ? 1 : o->interleave;
  if (K != ROW_STREAMS && !valid_interleave((int)K)) return 0;
  const int nlx = (W + pw - 1) / pw, nly = (H + ph - 1) / ph;
  const int64_t ns = image_streams((int)K, H, nlx, nly);
  // header, stream table, per stream at most 4 flush bytes, at most 2 bytes per symbol
  return (size_t)(HDR_BYTES + 4 * ns + 4 * ns + 6LL * H * W);
}

size_t nellox_workspace_bytes(const nellox_model* m, int32_t n, const nellox_image* imgs, const nellox_opts* o) {
  if (!m) return 0;
  Plan P;
  if (make_plan(n, imgs, o, P, false) != NELLOX_OK) return 0;
  plan_ring(m, P);
  return (size_t)ws_layout(P, n).total;
}

size_t nellox_decode_workspace_bytes(const nellox_model* m, int32_t n, const nellox_image* imgs,
                                     const nellox_opts* o) {
  if (!m) return 0;
  Plan P;
  if (make_plan(n, imgs, o, P, false) != NELLOX_OK) return 0;
  plan_ring(m, P);
  return (size_t)ws_layout(P, n).small;
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
  r.n_streams = P.n_streams;
  r.order = coded_order(o->order);
  r.h = m->h;
  r.K = P.K;
  r.sym = (const uint32_t*)(w8 + W.sym);
  r.slots = w8 + W.slots;
  r.lane_len = (uint32_t*)(w8 + W.lane_len);
  r.rev = (uint32_t*)(w8 + W.rev);
  r.after = (int32_t*)(w8 + W.after);
  r.max_lane_px = P.max_lane_px;
  hipError_t e = launch_rans_encode(r, s);
  if (e != hipSuccess) return hip_fail(e, "rANS encoder launch");
  PackArgs pk{};
  pk.desc = r.desc;
  pk.n_img = n;
  pk.n_lanes = P.n_lanes;
  pk.n_streams = P.n_streams;
  pk.order = coded_order(o->order);
  pk.h = m->h;
  pk.K = P.K;
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
  if (len < (size_t)HDR_BYTES || memcmp(c, "NLXC", 4) != 0 || c[4] != CONTAINER_VERSION || !valid_stream_code(c[7]))
    return fail(NELLOX_E_CORRUPT, "not a container of this version");
  const int32_t h = (int32_t)rd32(c + 8), w = (int32_t)rd32(c + 12);
  if (H) *H = h;
  if (W) *W = w;
  if (o) {
    o->order = c[5];
    o->patch_h = c[16] | (c[17] << 8);
    o->patch_w = c[18] | (c[19] << 8);
    o->interleave = c[7] == ROW_STREAMS ? -1 : c[7];
  }
  return NELLOX_OK;
}

static nellox_status prepare_impl(nellox_model* m, int32_t n, const nellox_image* outs, const nellox_opts* o,
                                  void* ws, size_t ws_bytes, nellox_decode_plan* plan, void* stream) {
  if (check_model(m)) return NELLOX_E_ARG;
  if (!plan) return fail(NELLOX_E_ARG, "plan is null");
  Plan P;
  nellox_status st = make_plan(n, outs, o, P, true);
  if (st) return st;
  plan_ring(m, P);
  if (n > 0 && !ws) return fail(NELLOX_E_ARG, "null workspace");
  const WsLayout W = ws_layout(P, n);
  if ((int64_t)ws_bytes < W.small) return fail(NELLOX_E_CAPACITY, "workspace too small");
  // row streams: the bands in start-step order, if they fit one upload with
  // the descriptors (else the bands are taken in image order)
  if (P.K == ROW_STREAMS && n > 0 && desc_bytes(P, n) <= (int64_t)STAGING_BYTES) P.band_order = band_queue(P);
  hipStream_t s = (hipStream_t)stream;
  if (n > 0 && (st = upload_plan(m, P, (uint8_t*)ws, W, s))) return st;
  int grid = 0, waves = 0;
  if (P.K == ROW_STREAMS) {
    // row streams: a workgroup per band, every band of the batch in flight if the CUs allow
    waves = ROW_WAVES;
    grid = (int)std::max<int64_t>(1, std::min<int64_t>(persistent_grid(m), P.n_bands));
  } else {
    decode_shape(P.n_lanes, persistent_grid(m), grid, waves);
  }
  memset(plan, 0, sizeof(*plan));
  plan->n = n;
  plan->order = o->order;
  plan->interleave = P.K == ROW_STREAMS ? -1 : P.K;
  plan->n_bands = P.n_bands;
  plan->progress_offset = W.progress;
  plan->band_order_offset = P.band_order.empty() ? 0 : W.desc + desc_bytes(P, n) - 4 * P.n_bands;
  plan->waves = std::max(waves, 1);
  plan->grid = grid;
  plan->ring_offset = W.ring;
  plan->ring_rows = P.ring_rows;
  plan->n_lanes = P.n_lanes;
  plan->model_hash = m->hash;
  plan->ws_bytes = W.small;
  plan->desc_offset = W.desc;
  plan->counter_offset = W.flags + 4;
  hipError_t e = prepare_decode(m->h, m->Cp, P.K);
  if (e != hipSuccess) return hip_fail(e, "decoder set-up");
  return NELLOX_OK;
}

static nellox_status run_impl(nellox_model* m, const nellox_decode_plan* plan, const uint8_t* in,
                              const uint64_t* in_offsets, int32_t* status, uint32_t* dump, void* ws, void* stream) {
  if (check_model(m)) return NELLOX_E_ARG;
  const bool rows = plan && plan->interleave == -1;
  if (!plan || plan->model_hash != m->hash || plan->n < 0 || plan->waves < 1 || plan->waves > DECODE_WAVES ||
      (!rows && !valid_interleave(plan->interleave)) || plan->order < 0 || plan->order > 2 ||
      (rows && (plan->order != 1 || plan->waves != ROW_WAVES || plan->n_bands < 0 ||
                plan->progress_offset + 4 * plan->n_bands > plan->ws_bytes ||
                (plan->band_order_offset != 0 && (plan->band_order_offset < plan->desc_offset ||
                                                  plan->band_order_offset + 4 * plan->n_bands > plan->ws_bytes)))) ||
      (plan->order == 2 && plan->n_lanes > 0 &&
       (ring_windows(plan->grid, plan->waves) * ring_wave_bytes(plan->ring_rows) > plan->ws_bytes ||
        plan->ring_rows < 4)))
    return fail(NELLOX_E_ARG, "plan does not belong to this model");
  const int n = plan->n;
  if (n == 0) return NELLOX_OK;
  if (!in || !in_offsets || !status || !ws) return fail(NELLOX_E_ARG, "null pointer argument");
  hipStream_t s = (hipStream_t)stream;
  uint8_t* w8 = (uint8_t*)ws;
  int32_t* counter = (int32_t*)(w8 + plan->counter_offset);
  int32_t* progress = rows ? (int32_t*)(w8 + plan->progress_offset) : nullptr;
  hipError_t e = launch_decode_prep(status, n, counter, s, progress, rows ? plan->n_bands : 0);
  if (e != hipSuccess) return hip_fail(e, "decode prep launch");
  DecArgs a{};
  a.w = m->dw;
  a.wfloats = m->wfloats;
  a.nb = m->nb;
  a.desc = (const ImgDesc*)(w8 + plan->desc_offset);
  a.n_img = n;
  a.n_lanes = plan->n_lanes;
  a.order = plan->order;
  a.K = plan->interleave;
  a.model_hash = m->hash;
  a.in = in;
  a.in_off = in_offsets;
  a.status = status;
  a.counter = counter;
  a.sym_dump = dump;
  a.ring = plan->order == 2 ? w8 + plan->ring_offset : nullptr;
  a.ring_rows = (int)plan->ring_rows;
  a.progress = progress;
  a.n_bands = plan->n_bands;
  a.band_order = rows && plan->band_order_offset ? (const int32_t*)(w8 + plan->band_order_offset) : nullptr;
  a.band_wait_ticks = g_band_wait.load();
  if (rows) {
    a.K = ROW_STREAMS;
    e = launch_decode_rows(m->h, m->Cp, a, plan->grid, s);
  } else {
    e = launch_decode(m->h, m->Cp, a, plan->grid, plan->waves, s);
  }
  if (e != hipSuccess) return hip_fail(e, "decoder launch");
  return NELLOX_OK;
}

static nellox_status decode_impl(const nellox_model* mc, int32_t n, const uint8_t* in, const uint64_t* in_offsets,
                                 const nellox_opts* o, const nellox_image* outs, int32_t* status, uint32_t* dump,
                                 void* ws, size_t ws_bytes, void* stream) {
  nellox_model* m = const_cast<nellox_model*>(mc);
  if (n > 0 && (!in || !in_offsets || !status || !ws)) return fail(NELLOX_E_ARG, "null pointer argument");
  nellox_decode_plan plan;
  nellox_status st = prepare_impl(m, n, outs, o, ws, ws_bytes, &plan, stream);
  if (st) return st;
  return run_impl(m, &plan, in, in_offsets, status, dump, ws, stream);
}

nellox_status nellox_decode(const nellox_model* m, int32_t n, const uint8_t* in, const uint64_t* in_offsets,
                            const nellox_opts* o, const nellox_image* out, int32_t* status, void* ws, size_t ws_bytes,
                            void* stream) {
  return decode_impl(m, n, in, in_offsets, o, out, status, nullptr, ws, ws_bytes, stream);
}

nellox_status nellox_decode_prepare(const nellox_model* m, int32_t n, const nellox_image* out, const nellox_opts* opts,
                                    void* ws, size_t ws_bytes, nellox_decode_plan* plan, void* stream) {
  return prepare_impl(const_cast<nellox_model*>(m), n, out, opts, ws, ws_bytes, plan, stream);
}

nellox_status nellox_decode_run(const nellox_model* m, const nellox_decode_plan* plan, const uint8_t* in,
                                const uint64_t* in_offsets, int32_t* status, void* ws, void* stream) {
  return run_impl(const_cast<nellox_model*>(m), plan, in, in_offsets, status, nullptr, ws, stream);
}

nellox_status nellox_decode_static(const nellox_model* mc, int32_t n, const uint8_t* in, const uint64_t* in_offsets,
                                   const nellox_opts* o, const nellox_image* out, int32_t* status, void* stream) {
  nellox_model* m = const_cast<nellox_model*>(mc);
  if (check_model(m)) return NELLOX_E_ARG;
  if (n > 0 && (!in || !in_offsets || !status)) return fail(NELLOX_E_ARG, "null pointer argument");
  Plan P;
  nellox_status st = make_plan(n, out, o, P, true);
  if (st) return st;
  plan_ring(m, P);
  const WsLayout W = ws_layout(P, n);
  if (W.small > (int64_t)STATIC_SCRATCH_BYTES)
    return fail(NELLOX_E_CAPACITY, "this batch needs " + std::to_string(W.small) +
                                       " bytes of decoder scratch, more than the " +
                                       std::to_string(STATIC_SCRATCH_BYTES) +
                                       " the no-allocation decoder has (use nellox_decode with a workspace)");
  if (sizeof(ImgDesc) * (size_t)n > STAGING_BYTES)
    return fail(NELLOX_E_CAPACITY, "the no-allocation decoder takes at most " +
                                       std::to_string(STAGING_BYTES / sizeof(ImgDesc)) + " images per call");
  void* ws = nullptr;
  hipError_t e = static_scratch(&ws);
  if (e != hipSuccess) return hip_fail(e, "scratch address (hipGetSymbolAddress)");
  return decode_impl(m, n, in, in_offsets, o, out, status, nullptr, ws, STATIC_SCRATCH_BYTES, stream);
}

nellox_status nellox_decode_trace(const nellox_model* m, int32_t n, const uint8_t* in, const uint64_t* in_offsets,
                                  const nellox_opts* o, const nellox_image* out, int32_t* status, uint32_t* dump,
                                  void* ws, size_t ws_bytes, void* stream) {
  if (!dump) return fail(NELLOX_E_ARG, "sym_dump is null");
  return decode_impl(m, n, in, in_offsets, o, out, status, dump, ws, ws_bytes, stream);
}

nellox_status nellox_sample(const nellox_model* mc, int32_t n, const uint64_t* seeds, const nellox_opts* o,
                            const nellox_image* out, void* ws, size_t ws_bytes, void* stream) {
  nellox_model* m = const_cast<nellox_model*>(mc);
  if (check_model(m)) return NELLOX_E_ARG;
  if (n > 0 && !seeds) return fail(NELLOX_E_ARG, "seeds is null");
  if (!o) return fail(NELLOX_E_ARG, "opts is null");
  nellox_opts so = *o;
  so.interleave = 1;  // no streams when sampling
  Plan P;
  nellox_status st = make_plan(n, out, &so, P, true);
  if (st) return st;
  plan_ring(m, P);
  if (n == 0) return NELLOX_OK;
  if (!ws) return fail(NELLOX_E_ARG, "null workspace");
  const WsLayout W = ws_layout(P, n);
  if ((int64_t)ws_bytes < W.small) return fail(NELLOX_E_CAPACITY, "workspace too small");
  for (int k = 0; k < n; ++k) P.d[k].seed = seeds[k];
  hipStream_t s = (hipStream_t)stream;
  uint8_t* w8 = (uint8_t*)ws;
  hipError_t e = prepare_decode(m->h, m->Cp, 4);
  if (e != hipSuccess) return hip_fail(e, "sampler set-up");
  if ((st = upload_plan(m, P, w8, W, s))) return st;
  int32_t* counter = (int32_t*)(w8 + W.flags + 4);
  e = launch_decode_prep(nullptr, 0, counter, s);
  if (e != hipSuccess) return hip_fail(e, "sampler prep launch");
  DecArgs a{};
  a.w = m->dw;
  a.wfloats = m->wfloats;
  a.nb = m->nb;
  a.desc = (const ImgDesc*)(w8 + W.desc);
  a.n_img = n;
  a.n_lanes = P.n_lanes;
  a.order = o->order;
  a.K = 4;
  a.model_hash = m->hash;
  a.counter = counter;
  a.ring = o->order == 2 ? w8 + W.ring : nullptr;
  a.ring_rows = (int)P.ring_rows;
  int grid = 0, waves = 0;
  decode_shape(P.n_lanes, persistent_grid(m), grid, waves);
  e = launch_sample(m->h, m->Cp, a, grid, waves, s);
  if (e != hipSuccess) return hip_fail(e, "sampler launch");
  return NELLOX_OK;
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
  if ((int64_t)ws_bytes < W.small) return fail(NELLOX_E_CAPACITY, "workspace too small");
  if (n == 0) return NELLOX_OK;
  hipStream_t s = (hipStream_t)stream;
  uint8_t* w8 = (uint8_t*)ws;
  if ((st = upload_plan(m, P, w8, W, s))) return st;
  float* bits = bits_per_px ? bits_per_px : (float*)(w8 + W.bits);
  if ((st = run_pass(m, P, w8, W, 1, nullptr, bits, nullptr, s))) return st;
  hipError_t e = launch_reduce_bits((const ImgDesc*)(w8 + W.desc), n, bits, (double*)(w8 + W.partials), bits_total, s);
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
  if ((int64_t)ws_bytes < W.small) return fail(NELLOX_E_CAPACITY, "workspace too small");
  if (n == 0) return NELLOX_OK;
  hipStream_t s = (hipStream_t)stream;
  uint8_t* w8 = (uint8_t*)ws;
  if ((st = upload_plan(m, P, w8, W, s))) return st;
  float* bits = ideal ? (float*)(w8 + W.bits) : nullptr;  // the pass alone when no sum is asked for
  if ((st = run_pass(m, P, w8, W, 0, sym, bits, nullptr, s))) return st;
  if (ideal) {
    hipError_t e = launch_reduce_bits((const ImgDesc*)(w8 + W.desc), n, bits, (double*)(w8 + W.partials), ideal, s);
    if (e != hipSuccess) return hip_fail(e, "reduction launch");
  }
  return NELLOX_OK;
}

uint64_t nellox_debug_band_wait(uint64_t ticks) { return g_band_wait.exchange(ticks ? ticks : BAND_WAIT_TICKS); }

nellox_status nellox_debug_check_monotone(uint64_t* counts, void* stream) {
  if (!counts) return fail(NELLOX_E_ARG, "counts is null");
  hipError_t e = launch_check_monotone((unsigned long long*)counts, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "monotonicity check launch");
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
  if ((int64_t)ws_bytes < W.small) return fail(NELLOX_E_CAPACITY, "workspace too small");
  hipStream_t s = (hipStream_t)stream;
  uint8_t* w8 = (uint8_t*)ws;
  if ((st = upload_plan(m, P, w8, W, s))) return st;
  return run_pass(m, P, w8, W, 2, nullptr, nullptr, cdf, s);
}

int64_t nellox_param_count(const int32_t dims[4]) {
  if (!dims || dims[0] < 1 || dims[0] > 3 || dims[1] < 1 || dims[2] < 0 || dims[3] != NMIX) return -1;
  return param_layout(dims[0], dims[1], dims[2]).total;
}

size_t nellox_train_workspace_bytes(const int32_t dims[4], int32_t n, int32_t H, int32_t W) {
  TrainPlan T;
  if (train_plan(dims, n, H, W, T, false) != NELLOX_OK) return 0;
  return (size_t)T.total;
}

nellox_status nellox_nll_fwd_train(const float* params, const int32_t dims[4], const uint8_t* imgs, int32_t n,
                                   int32_t H, int32_t W, double* bits_per_img, float* bits_per_px, void* ws,
                                   size_t ws_bytes, void* stream) {
  TrainPlan T;
  nellox_status st = train_plan(dims, n, H, W, T, true);
  if (st) return st;
  if (!params || !imgs || !bits_per_img || !ws) return fail(NELLOX_E_ARG, "null pointer argument");
  if ((int64_t)ws_bytes < T.total) return fail(NELLOX_E_CAPACITY, "workspace too small");
  hipStream_t s = (hipStream_t)stream;
  uint8_t* w8 = (uint8_t*)ws;
  hipError_t e = launch_swizzle(params, T.h, T.C, T.Cp, T.nb, (float*)(w8 + T.wimg), T.wfloats,
                                (float*)(w8 + T.wimgT), T.wTfloats, s);
  if (e != hipSuccess) return hip_fail(e, "weight image launch");
  const TrainArgs a = train_args(T, imgs, w8, nullptr);
  e = launch_train_fwd(T.h, T.Cp, a, train_grid(T), s);
  if (e != hipSuccess) return hip_fail(e, "training forward launch");
  e = launch_bits_img(a.bits, T.n, (int64_t)T.H * T.W, bits_per_img, s);
  if (e != hipSuccess) return hip_fail(e, "bits reduction launch");
  if (bits_per_px) {
    e = hipMemcpyAsync(bits_per_px, a.bits, 4 * (size_t)T.npx, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "per-pixel bits copy");
  }
  return NELLOX_OK;
}

nellox_status nellox_nll_bwd(const float* params, const int32_t dims[4], const uint8_t* imgs, int32_t n, int32_t H,
                             int32_t W, const float* grad_bits, float* grad_params, void* ws, size_t ws_bytes,
                             void* stream) {
  TrainPlan T;
  nellox_status st = train_plan(dims, n, H, W, T, true);
  if (st) return st;
  if (!params || !imgs || !grad_bits || !grad_params || !ws) return fail(NELLOX_E_ARG, "null pointer argument");
  if ((int64_t)ws_bytes < T.total) return fail(NELLOX_E_CAPACITY, "workspace too small");
  hipStream_t s = (hipStream_t)stream;
  uint8_t* w8 = (uint8_t*)ws;
  // the transposed weight image is the one the forward built from the same
  // params (the workspace holds the forward's state)
  const TrainArgs a = train_args(T, imgs, w8, grad_bits);
  hipError_t e = launch_train_bwd(T.h, T.Cp, a, train_grid(T), s);
  if (e != hipSuccess) return hip_fail(e, "training backward launch");
  WgradArgs g{};
  g.npx = T.npx; g.chunk = T.chunk; g.nchunks = T.nchunks; g.ngrad = T.ngrad;
  g.partial = (float*)(w8 + T.partial);
  const int64_t pc = T.npx * T.Cp;
  // one launch for every layer, the head's row parts first: their deltas
  // are the head rows', their input the last block's output; the first
  // layer's deltas are those of a_0, its inputs the causal taps; 1x1 layer l
  // (W1 of block l / 2 or W2) has delta l + 1 and input u_l
  int nl = 0;
  constexpr int head_rows = 16 * HEAD_TILES / WGRAD_HEAD_PARTS;
  for (int q = 0; q < WGRAD_HEAD_PARTS; ++q)
    g.layer[nl++] = WgradLayer{a.dtheta + q * head_rows, a.u + 2LL * T.nb * pc, 16 * HEAD_TILES, T.Cp,
                               T.off_head + (int64_t)q * head_rows * T.Cp, T.bias_head + q * head_rows, WGRAD_HEAD};
  g.layer[nl++] = WgradLayer{a.delta, a.ctx, T.Cp, T.KP, T.off_conv, T.bias_conv, WGRAD_FIRST};
  for (int l = 0; l < 2 * T.nb; ++l)
    g.layer[nl++] = WgradLayer{a.delta + (l + 1) * pc, a.u + l * pc, T.Cp, T.Cp,
                               T.off_blocks + (int64_t)l * T.Cp * T.Cp, T.bias_blocks + (int64_t)l * T.Cp,
                               WGRAD_BLOCK};
  e = launch_wgrad(T.Cp / 16, T.KP / 16, g, nl, s);
  if (e != hipSuccess) return hip_fail(e, "weight gradient launch");
  GradReduceArgs r{};
  r.h = T.h; r.C = T.C; r.Cp = T.Cp; r.nb = T.nb; r.KP = T.KP;
  r.off_conv = T.off_conv; r.off_blocks = T.off_blocks; r.off_head = T.off_head;
  r.bias_conv = T.bias_conv; r.bias_blocks = T.bias_blocks; r.bias_head = T.bias_head;
  r.nchunks = T.nchunks; r.ngrad = T.ngrad;
  r.partial = g.partial;
  r.grad = grad_params;
  e = launch_grad_reduce(r, s);
  if (e != hipSuccess) return hip_fail(e, "gradient reduction launch");
  return NELLOX_OK;
}

}  // extern "C"
