// nx_order.hpp -- the coding order of a lane's symbols, shared by the host
// (tests) and the kernels: which rows a wavefront step holds, and the
// encoder's reverse walk over one rANS stream.
#pragma once
#include "nx_layout.hpp"

namespace nx {

NXHD int nx_min(int a, int b) { return a < b ? a : b; }

// rows active at wavefront step t of an Hl x Wl lane, step offset o = h + 1
NXHD void step_rows(int t, int Hl, int Wl, int o, int& ilo, int& ihi) {
  const int a = t - (Wl - 1);
  ilo = a <= 0 ? 0 : (a + o - 1) / o;
  ihi = nx_min(Hl - 1, t / o);
}

// rows of stream kk (of K, K dividing 16) at wavefront step t: a full group
// of 16 rows gives each stream 16 / K of them, a partial group of r rows the
// offsets kk, kk + K, ... below r
NXHD int stream_rows_at(int t, int Hl, int Wl, int o, int K, int kk) {
  int ilo, ihi;
  step_rows(t, Hl, Wl, o, ilo, ihi);
  if (ilo > ihi) return 0;
  const int n = ihi - ilo + 1, full = n / 16, rem = n - 16 * full;
  return full * (16 / K) + (rem > kk ? (rem - kk + K - 1) / K : 0);
}

// The place of symbol (row i, column j, channel c) of an Hl x Wl lane in its
// stream's coding order (the reverse decode order below), wavefront order:
// its stream kk, its step t = j + o i, and its offset among the stream's
// symbols of step t. The stream's symbols of later steps come first (their
// count is added by the caller); within step t, those of the groups above
// (visited first), then of the channels after c (B, G, R), then the
// stream's rows above row i in the group (rows descending).
NXHD void coding_slot(int i, int j, int c, int Hl, int Wl, int o, int K, int& kk, int& t, int& off) {
  t = j + o * i;
  int ilo, ihi;
  step_rows(t, Hl, Wl, o, ilo, ihi);
  const int n = ihi - ilo + 1, nfull = n / 16, rem = n - 16 * nfull;
  const int g = (i - ilo) / 16, ts = ilo + 16 * g, r = i - ts;
  kk = r % K;
  const int len_g = nx_min(16, ihi - ts + 1);
  const int rows_g = (len_g - kk + K - 1) / K;
  const int rows_part = rem > kk ? (rem - kk + K - 1) / K : 0;
  const int above = g < nfull ? (nfull - 1 - g) * (16 / K) + rows_part : 0;
  off = 3 * above + (2 - c) * rows_g + (rows_g - 1 - (r - kk) / K);
}

// Symbols of a lane in decode order:
//   wavefront: steps t ascending; within a step the active rows are cut into
//   groups of 16 consecutive rows; per group channels R, G, B; per channel
//   rows ascending. With K streams, row ts + r of a group (ts = first row of
//   the group, a multiple of 16 rows after the step's first row) belongs to
//   stream r mod K; each stream codes its own rows in this order.
//   raster: rows, columns, channels (one stream).
// The encoder walks one stream's symbols backwards.
struct RevOrder {
  int Hl, Wl, o, raster, K, kk;
  int t, ilo, ihi, ts, te, c, i;
  bool done;

  // highest row of stream kk in rows [ts, te], or ts - 1 if it has none
  NXHD int top_row() const {
    const int span = te - ts;
    return span < kk ? ts - 1 : ts + kk + ((span - kk) / K) * K;
  }
  // the top group of step t, or of the closest earlier non-empty step: a lane
  // narrower than h + 1 columns has steps without any pixel
  NXHD void enter_step() {
    for (;;) {
      step_rows(t, Hl, Wl, o, ilo, ihi);
      if (ilo <= ihi) break;
      if (--t < 0) { done = true; return; }
    }
    ts = ilo + ((ihi - ilo) / 16) * 16;
    te = nx_min(ts + 15, ihi);
    c = 2;
    i = top_row();
  }
  // move back until row i belongs to the current (step, group, channel)
  NXHD void settle() {
    while (!done && i < ts) {
      if (--c >= 0) { i = top_row(); continue; }
      ts -= 16;
      if (ts >= ilo) { te = ts + 15; c = 2; i = top_row(); continue; }
      if (--t < 0) { done = true; return; }
      enter_step();
    }
  }
  NXHD void init(int Hl_, int Wl_, int o_, int raster_, int K_, int kk_) {
    Hl = Hl_; Wl = Wl_; o = o_; raster = raster_; K = K_; kk = kk_; done = false;
    if (raster) { i = Hl - 1; j = Wl - 1; c = 2; return; }
    t = Wl + o * (Hl - 1) - 1;
    enter_step();
    settle();
  }
  int j;
  // current symbol: row i, column col(), channel c
  NXHD int col() const { return raster ? j : t - o * i; }
  NXHD void advance() {
    if (raster) {
      if (--c >= 0) return;
      c = 2;
      if (--j >= 0) return;
      j = Wl - 1;
      if (--i >= 0) return;
      done = true;
      return;
    }
    i -= K;
    settle();
  }
};

}  // namespace nx
