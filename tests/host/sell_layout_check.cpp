// Host check of the grouped sliced-ELL packing (unpaired and paired steps)
// against an independent walk of the addresses the device mat-vec reads.
// Random row lengths (empty rows, ragged slices, a partial last slice) for
// every lane count G = 1..16, both step kinds.  For each row, the entries
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
// the device address map: unpaired steps at sptr + 64k + p; paired steps at
// sptr + 128k + 2p + {0, 1} for the first floor(u/2) steps, then one
// unpaired step at sptr + 128 floor(u/2) + p when u is odd
// (p = (r mod 64/G) G + sub, u = slice size / 64).
static std::vector<size_t> lane_walk(const Sell &S, int r, int sub) {
  const int rs = 64 >> S.lg, s = r / rs, beg = S.sptr[s], u = (S.sptr[s + 1] - beg) / 64;
  const int p = (r % rs) * (1 << S.lg) + sub;
  std::vector<size_t> out;
  if (!S.vlg) {
    for (int k = 0; k < u; ++k) out.push_back((size_t)beg + 64 * k + p);
    return out;
  }
  for (int k = 0; k < u / 2; ++k) {
    out.push_back((size_t)beg + 128 * k + 2 * p);
    out.push_back((size_t)beg + 128 * k + 2 * p + 1);
  }
  if (u % 2) out.push_back((size_t)beg + 128 * (u / 2) + p);
  return out;
}

static int check(int nrows, int lg, int vlg, int maxlen, unsigned seed) {
  std::mt19937 rng(seed);
  const int G = 1 << lg;
  SellBuilder b;
  b.init(nrows, lg, vlg != 0);
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
    // lane j accumulates entries kG + j (unpaired steps), or 2(mG + j),
    // 2(mG + j) + 1 for paired steps m, then 2G floor(u/2) + j
    for (int j = 0; j < G; ++j) {
      std::vector<int> ks;
      if (!S.vlg) {
        for (int k = 0; k < per_lane; ++k) ks.push_back(k * G + j);
      } else {
        const int np = per_lane / 2;
        for (int m = 0; m < np; ++m) {
          ks.push_back(2 * (m * G + j));
          ks.push_back(2 * (m * G + j) + 1);
        }
        if (per_lane % 2) ks.push_back(2 * G * np + j);
      }
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
    for (int vlg = 0; vlg <= 1; ++vlg)
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
