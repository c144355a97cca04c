// Host check of the grouped sliced-ELL packing (one, two or four entries per
// lane and step)
// against an independent walk of the addresses the device mat-vec reads.
// Random row lengths (empty rows, ragged slices, a partial last slice) for
// every lane count G = 1..16, every step width.  For each row, the entries
// reached by the walk of its G lanes, in the order each lane accumulates
// them, must be the row's entries in storage order followed by padding
// (value 0, the row's last column); every stored position must be reached
// by exactly one row (or be a zero past the last row); the block-diagonal
// check and the 16-bit column compression must accept the layout and decode
// to the same columns.  Exit status 0 when every case passes.
#include <cstdio>
#include <random>

#include "../../paper_1906_10575_amd/csrc/setup.cpp"

using namespace amgdd;

// Positions lane `sub` of row r reads, in its accumulation order, following
// the device address map: with widest steps of W = 2^vlg entries per lane, a
// slice of u = size/64 unpaired-step equivalents holds floor(u/W) steps at
// sptr + 64W k + W p + {0..W-1}, then one step of width 2^v at the next
// 64 * 2^v entries for every bit v < vlg set in u, narrowest last
// (p = (r mod 64/G) G + sub).
static std::vector<size_t> lane_walk(const Sell &S, int r, int sub) {
  const int rs = 64 >> S.lg, s = r / rs, u = (S.sptr[s + 1] - S.sptr[s]) / 64;
  const int p = (r % rs) * (1 << S.lg) + sub;
  std::vector<size_t> out;
  size_t base = S.sptr[s];
  for (int v = S.vlg; v >= 0; --v) {
    const int steps = v == S.vlg ? u >> v : (u >> v) & 1, W = 1 << v;
    for (int k = 0; k < steps; ++k)
      for (int e = 0; e < W; ++e) out.push_back(base + 64 * W * k + W * p + e);
    base += (size_t)64 * W * steps;
  }
  return out;
}

// Entries of its row lane j adds, in order: region by region (widest first),
// step k of width W holds entries K + (k G + j) W + {0..W-1}, where K counts
// the row's entries in the earlier regions.
static std::vector<int> lane_entries(const Sell &S, int r, int j) {
  const int rs = 64 >> S.lg, s = r / rs, u = (S.sptr[s + 1] - S.sptr[s]) / 64, G = 1 << S.lg;
  std::vector<int> ks;
  int K = 0;
  for (int v = S.vlg; v >= 0; --v) {
    const int steps = v == S.vlg ? u >> v : (u >> v) & 1, W = 1 << v;
    for (int k = 0; k < steps; ++k)
      for (int e = 0; e < W; ++e) ks.push_back(K + (k * G + j) * W + e);
    K += steps * G * W;
  }
  return ks;
}

static int check(int nrows, int lg, int vlg, int maxlen, unsigned seed) {
  std::mt19937 rng(seed);
  const int G = 1 << lg;
  SellBuilder b;
  b.init(nrows, lg, vlg);
  std::vector<std::vector<std::pair<int, double>>> rows(nrows);
  for (int r = 0; r < nrows; ++r) {
    const int len = (rng() % 7 == 0) ? 0 : (int)(rng() % (maxlen + 1));
    std::vector<int> cols;
    for (int k = 0; k < len; ++k) cols.push_back((int)(rng() % 1000));
    std::sort(cols.begin(), cols.end());
    for (int c : cols) rows[r].push_back({c, 1.0 + (double)(rng() % 1000)});
    b.len[r] = len;
  }
  b.shape();
  for (int r = 0; r < nrows; ++r) {
    for (int k = 0; k < (int)rows[r].size(); ++k) b.put(r, k, rows[r][k].first, rows[r][k].second);
    b.pad(r, 7);
  }
  const Sell S = b.S;  // b keeps its copy for at()
  if (!sell_in_bounds(S, nrows, 1000)) return 1;
  // 1. the walk of each row's lanes meets its entries in storage order, then padding
  std::vector<int> hits(S.val.size(), 0);
  for (int r = 0; r < nrows; ++r) {
    std::vector<std::vector<size_t>> walks;
    for (int j = 0; j < G; ++j) walks.push_back(lane_walk(S, r, j));
    const int per_lane = (int)walks[0].size();
    std::vector<size_t> seen;
    for (int j = 0; j < G; ++j)
      for (size_t a : walks[j]) {
        if (a >= S.val.size()) return 2;
        hits[a]++;
        seen.push_back(a);
      }
    const int kmax = per_lane * G;
    const int last_col = rows[r].empty() ? 7 : rows[r].back().first;
    for (int k = 0; k < kmax; ++k) {
      const size_t a = b.at(r, k);
      if (std::find(seen.begin(), seen.end(), a) == seen.end()) return 3;
      if (k < (int)rows[r].size()) {
        if (S.col[a] != rows[r][k].first || S.val[a] != rows[r][k].second) return 4;
      } else if (S.col[a] != last_col || S.val[a] != 0.0) {
        return 5;
      }
    }
    // lane j adds the entries the layout assigns it, in storage order
    for (int j = 0; j < G; ++j) {
      const std::vector<int> ks = lane_entries(S, r, j);
      if ((int)ks.size() != per_lane) return 6;
      for (int q = 0; q < per_lane; ++q)
        if (b.at(r, ks[q]) != walks[j][q]) return 6;
    }
    for (size_t a : seen)
      if (sell_slice_row(S, S.sptr[r / (64 >> lg) + 1] - S.sptr[r / (64 >> lg)], (int)(a - S.sptr[r / (64 >> lg)])) != r % (64 >> lg)) return 7;
  }
  // 2. every position belongs to one row, or is a zero past the last row
  const int rs = 64 >> lg, ns = (nrows + rs - 1) / rs;
  for (int s = 0; s < ns; ++s)
    for (int a = S.sptr[s]; a < S.sptr[s + 1]; ++a) {
      const int r = s * rs + sell_slice_row(S, S.sptr[s + 1] - S.sptr[s], a - S.sptr[s]);
      if (r < nrows ? hits[a] != 1 : (hits[a] != 0 || S.val[a] != 0.0)) return 8;
    }
  // 3. block-diagonal check and 16-bit compression on the packed layout
  std::vector<int> owner_r(nrows, 0), owner_c(1000, 0);
  if (!sell_block_diagonal(S, owner_r, owner_c)) return 9;
  Sell C = S;
  if (!compress_columns(C, owner_r, owner_c)) return 10;
  for (int s = 0; s < ns; ++s)
    for (int a = S.sptr[s]; a < S.sptr[s + 1]; ++a) {
      const int c = ((C.col16[a] & 0x8000) ? C.base[2 * s + 1] : C.base[2 * s]) + (C.col16[a] & 0x7fff);
      const int r = s * rs + sell_slice_row(S, S.sptr[s + 1] - S.sptr[s], a - S.sptr[s]);
      if (r < nrows && S.val[a] != 0.0 && c != S.col[a]) return 11;
    }
  return 0;
}

int main() {
  int fails = 0, runs = 0;
  const int sizes[] = {1, 63, 64, 65, 200, 1000};
  for (int lg = 0; lg <= 4; ++lg)
    for (int vlg = 0; vlg <= 2; ++vlg)
      for (int n : sizes)
        for (int maxlen : {1, 3, 7, 20, 70}) {
          const int rc = check(n, lg, vlg, maxlen, 1000u * lg + 100u * vlg + (unsigned)n + 7u * maxlen);
          ++runs;
          if (rc) {
            ++fails;
            std::printf("FAIL lg %d vlg %d rows %d maxlen %d: code %d\n", lg, vlg, n, maxlen, rc);
          }
        }
  std::printf("%d layouts, %d failed\n", runs, fails);
  return fails ? 1 : 0;
}
