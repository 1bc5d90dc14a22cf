// nx_order.hpp -- the coding order of a lane's symbols, shared by the host
// (tests) and the kernels: which rows a wavefront step holds, how many of
// them each rANS stream has, and a symbol's place in its stream's coding
// order.
//
// Symbols of a lane in decode order (wavefront): steps t ascending; within a
// step the active rows are cut into groups of 16 consecutive rows; per group
// channels R, G, B; per channel rows ascending. With K streams, row ts + r of
// a group (ts = first row of the group, a multiple of 16 rows after the
// step's first row) belongs to stream r mod K; each stream codes its own
// rows in this order, and its encoder codes them backwards. Raster order:
// rows, columns, channels (one stream).
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
// stream's coding order (the decode order above, reversed), wavefront order:
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

}  // namespace nx
