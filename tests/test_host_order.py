"""CPU check of the coding order shared by the encoder and the decoder.

The wavefront decoder (Sec. 3, Algorithm 1) pops a lane's symbols in this
order: steps t ascending; the active rows of a step cut into groups of 16
consecutive rows; per group the channels R, G, B; per channel the rows
ascending, dealt to K interleaved rANS streams (row ts + r of a group goes
to stream r mod K, K rows popped per round). The test restates the
decoder's loop, checks that the streams together cover every symbol of the
lane once, and that the encoder's layout (stream_rows_at, coding_slot in
nx_order.hpp, compiled here for the host) puts every symbol at its index in
its stream's coding order, the decode order reversed; for K = 1, 2, 4, 8,
16, lanes narrower than h + 1 columns, single rows and columns, and ragged
group sizes.
"""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2201_05213_amd", "csrc")

DRIVER = r"""
#include <cstdio>
#include <vector>
#include <tuple>
#include <algorithm>
#include "nx_order.hpp"
using namespace nx;
typedef std::tuple<int, int, int> Sym;  // row, column, channel

// the decoder's pop order, stream by stream
static std::vector<std::vector<Sym>> decoder_order(int Hl, int Wl, int h, int K) {
  const int o = h + 1;
  std::vector<std::vector<Sym>> dec(K);
  for (int t = 0; t < Wl + o * (Hl - 1); ++t) {
    int ilo, ihi;
    step_rows(t, Hl, Wl, o, ilo, ihi);
    for (int ts = ilo; ts <= ihi; ts += 16) {
      const int na = std::min(16, ihi - ts + 1);
      for (int c = 0; c < 3; ++c)
        for (int q0 = 0; q0 < na; q0 += K)
          for (int k = 0; k < K; ++k)
            if (q0 + k < na) dec[k].push_back(Sym(ts + q0 + k, t - o * (ts + q0 + k), c));
    }
  }
  return dec;
}

int main() {
  int cases = 0, bad = 0;
  for (int h = 1; h <= 3; ++h)
    for (int K : {1, 2, 4, 8, 16})
      for (int Hl = 1; Hl <= 90; Hl += (Hl < 6 ? 1 : 13))
        for (int Wl = 1; Wl <= 70; Wl += (Wl < 8 ? 1 : 13)) {
          ++cases;
          const int o = h + 1, T = Wl + o * (Hl - 1);
          const auto dec = decoder_order(Hl, Wl, h, K);
          // every symbol of the lane in exactly one stream
          std::vector<Sym> all;
          for (int k = 0; k < K; ++k) all.insert(all.end(), dec[k].begin(), dec[k].end());
          std::sort(all.begin(), all.end());
          bool cover = all.size() == (size_t)Hl * Wl * 3;
          for (size_t n = 0; cover && n < all.size(); ++n) {
            const int i = (int)(n / (3 * Wl)), j = (int)(n / 3 % Wl), c = (int)(n % 3);
            cover = all[n] == Sym(i, j, c);
          }
          if (!cover) {
            if (bad < 5) printf("coverage h=%d K=%d %dx%d\n", h, K, Hl, Wl);
            ++bad;
          }
          // coding order = decode order reversed; per step the stream's
          // symbols of later steps from stream_rows_at
          std::vector<std::vector<long>> after(K, std::vector<long>(T, 0));
          for (int kk = 0; kk < K; ++kk) {
            long S = 0;
            for (int t = T - 1; t >= 0; --t) { after[kk][t] = S; S += 3 * stream_rows_at(t, Hl, Wl, o, K, kk); }
            if (S != (long)dec[kk].size()) { ++bad; if (bad < 5) printf("length h%d K%d %dx%d kk%d\n", h, K, Hl, Wl, kk); }
          }
          for (int i = 0; i < Hl; ++i)
            for (int j = 0; j < Wl; ++j)
              for (int c = 0; c < 3; ++c) {
                int kk, t, off;
                coding_slot(i, j, c, Hl, Wl, o, K, kk, t, off);
                const long p = after[kk][t] + off;
                const long n = (long)dec[kk].size();
                if (kk < 0 || kk >= K || p < 0 || p >= n || dec[kk][n - 1 - p] != Sym(i, j, c)) {
                  ++bad;
                  if (bad < 5) printf("slot h%d K%d %dx%d (%d,%d,%d)\n", h, K, Hl, Wl, i, j, c);
                }
              }
        }
  printf("%d cases %d bad\n", cases, bad);
  return bad != 0;
}
"""


def build_and_run(tmp_path, driver, name):
    src = tmp_path / f"{name}.cpp"
    exe = tmp_path / name
    src.write_text(driver)
    cmd = ["g++", "-std=c++17", "-O1", "-D__HIP_PLATFORM_AMD__", "-I", CSRC, "-I", "/opt/rocm/include",
           str(src), "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        pytest.fail("host build of nx_order.hpp failed:\n" + r.stderr[-2000:])
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout
    assert " 0 bad" in r.stdout


def test_streams_cover_the_lane_and_slots_reverse_the_decode_order(tmp_path):
    build_and_run(tmp_path, DRIVER, "order")
