// Host check of the column order the pivoted QR uses (qr_order.h), built and
// run by tests/test_qr_order.py: for norm arrays with ties, NaN, +-Inf,
// signed zeros and denormals,
//  - the ranks counted as the panel selection counts them (rank of q = number
//    of columns ordered before it) are a permutation of 0..n-1, the columns of
//    rank < w are the w first in a sorted order, and the key of rank w is the
//    largest key left outside the panel;
//  - the in-panel pivot reduced over a 64-lane wavefront in the order the
//    kernel's butterfly uses (xor 1, xor 2, mirror within 8, mirror within 16,
//    xor 16, xor 32) gives every lane the first column of largest key, the
//    same as a linear scan.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <limits>
#include <random>
#include <vector>

#include "qr_order.h"

using bss::rank_key;
using bss::ranks_before;

static int fails = 0;
#define CHECK(c, ...) do { if (!(c)) { ++fails; std::printf(__VA_ARGS__); std::printf("\n"); } } while (0)

static void check_ranks(const std::vector<double> &norm, int c0, int w) {
  const int n = (int)norm.size();
  std::vector<int> rank(n, -1), seen(n - c0, 0), src(w, -1);
  for (int q = c0; q < n; ++q) {
    int r = 0;
    for (int p = c0; p < n; ++p) r += ranks_before(rank_key(norm[p]), p, rank_key(norm[q]), q);
    rank[q] = r;
    CHECK(r >= 0 && r < n - c0, "rank out of range");
    if (r >= 0 && r < n - c0) seen[r]++;
    if (r < w) src[r] = q;
  }
  for (int r = 0; r < n - c0; ++r) CHECK(seen[r] == 1, "rank %d taken %d times (c0=%d)", r, seen[r], c0);
  std::vector<int> idx;
  for (int q = c0; q < n; ++q) idx.push_back(q);
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return rank_key(norm[a]) > rank_key(norm[b]); });
  for (int r = 0; r < w && r < n - c0; ++r) CHECK(src[r] == idx[r], "rank %d: %d, sorted %d", r, src[r], idx[r]);
  if (n - c0 > w) {
    double outside = -2.0;
    for (int q = c0; q < n; ++q)
      if (rank[q] >= w) outside = std::max(outside, rank_key(norm[q]));
    CHECK(rank_key(norm[idx[w]]) == outside, "key of rank w is not the largest outside");
  }
}

static int partner(int lane, int step) {
  switch (step) {
    case 0: return lane ^ 1;
    case 1: return lane ^ 2;
    case 2: return (lane & ~7) | (7 - (lane & 7));
    case 3: return (lane & ~15) | (15 - (lane & 15));
    case 4: return lane ^ 16;
    default: return lane ^ 32;
  }
}

static void check_pivot(const std::vector<double> &pn, int j, int w) {
  double best[64];
  int p[64];
  for (int l = 0; l < 64; ++l) {
    best[l] = (j + l < w) ? rank_key(pn[j + l]) : -1.0;
    p[l] = j + l;
  }
  for (int step = 0; step < 6; ++step) {
    double nb[64];
    int np_[64];
    for (int l = 0; l < 64; ++l) {
      const int o = partner(l, step);
      nb[l] = best[l];
      np_[l] = p[l];
      if (ranks_before(best[o], p[o], nb[l], np_[l])) { nb[l] = best[o]; np_[l] = p[o]; }
    }
    for (int l = 0; l < 64; ++l) { best[l] = nb[l]; p[l] = np_[l]; }
  }
  int lin = j;
  for (int q = j + 1; q < w; ++q)
    if (ranks_before(rank_key(pn[q]), q, rank_key(pn[lin]), lin)) lin = q;
  for (int l = 0; l < 64; ++l) CHECK(p[l] == lin, "lane %d pivot %d, scan %d (j=%d w=%d)", l, p[l], lin, j, w);
}

int main() {
  const double nan = std::numeric_limits<double>::quiet_NaN(), inf = std::numeric_limits<double>::infinity();
  const double den = std::numeric_limits<double>::denorm_min();
  std::mt19937_64 g(7);
  const double pool[] = {0.0, -0.0, 1.0, 1.0, 2.5, inf, nan, den, 2 * den, 1e300, 3.0, 3.0};
  std::vector<std::vector<double>> cases = {
      {nan, nan, nan, nan}, {inf, inf, 1.0, nan, inf}, {0.0, -0.0, 0.0, -0.0}, {1, 1, 1, 1, 1, 1, 1, 1, 1}};
  for (int t = 0; t < 200; ++t) {
    const int n = 1 + (int)(g() % 300);
    std::vector<double> v(n);
    for (auto &x : v) x = (t % 2) ? pool[g() % 12] : std::ldexp((double)(g() % 5), (int)(g() % 7) - 3);
    cases.push_back(v);
  }
  for (const auto &v : cases) {
    const int n = (int)v.size();
    for (int c0 : {0, n / 3, n - 1}) {
      if (c0 < 0 || c0 >= n) continue;
      for (int w : {1, 16, 32}) check_ranks(v, c0, std::min(w, n - c0));
    }
    for (int w : {1, std::min(n, 16), std::min(n, 32)})
      for (int j = 0; j < w; ++j) check_pivot(v, j, w);
  }
  std::printf(fails ? "FAILED %d\n" : "ok\n", fails);
  return fails ? 1 : 0;
}
