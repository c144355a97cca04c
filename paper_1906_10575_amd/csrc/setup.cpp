// Host setup of the AMG-DD solve phase: classical AMG hierarchy, composite
// grids of every subdomain, and the block-diagonal batched layouts that the
// device kernels consume.
//
// Paper references (Mitchell, Strzodka, Falgout, AMG-DD):
//   Section 2   C/F splitting from strength of connection, interpolation P,
//               R = P^T, Galerkin coarse operators, direct coarsest solve.
//   Section 3   composite grids: padding eta_l through the graph of A_l on
//               every level, C-points carried to the next level, coarsest
//               level stored whole (Figure 1).
//   Section 4.1 ghost extension Dbar_l = D_l plus the row stencils of D_l.
//   Section 4.2 interpolation columns outside Dbar_{l+1} are dropped
//               (connectivity assumption); the count is reported.
// The paper runs its setup on the CPU as well and names global-to-local
// reindexing as its dominant cost; here reindexing uses per-thread stamp
// arrays and all composite grids are built in parallel.
//
// Readings where the paper defers to its host AMG library:
//   strength: j in S_i iff j != i, m_i = max_{k!=i}(-a_ik) > 0 and
//             -a_ij >= theta m_i (1 - 1e-12)
//   RS first pass only; largest measure first, smallest index on ties
//   direct interpolation with positive off-diagonals lumped into the diagonal
//   Galerkin product on the symbolic pattern, values from R (A P)
// Floating-point row sums run sequentially in ascending column order and the
// file is compiled without FMA contraction, so the hierarchy is reproducible.

#include "amgdd_internal.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <functional>
#include <limits>
#include <mutex>
#include <queue>
#include <stdexcept>
#include <thread>

namespace amgdd {

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

bool verbose() {
  static int v = std::getenv("AMGDD_VERBOSE") ? 1 : 0;
  return v != 0;
}

void vlog(const char *what, double t0) {
  if (verbose()) std::fprintf(stderr, "[amgdd setup] %-28s %8.3f s\n", what, now_s() - t0);
}

int n_threads() {
  const char *e = std::getenv("AMGDD_THREADS");
  int n = e ? std::atoi(e) : (int)std::thread::hardware_concurrency();
  if (n < 1) n = 1;
  if (n > 64) n = 64;
  return n;
}

// Static chunking: f(begin, end, thread_id).
void parallel_for(long long n, const std::function<void(long long, long long, int)> &f, long long grain = 4096) {
  int nt = n_threads();
  long long maxt = (n + grain - 1) / grain;
  if (maxt < nt) nt = (int)std::max(1LL, maxt);
  if (nt <= 1) {
    f(0, n, 0);
    return;
  }
  std::vector<std::thread> th;
  for (int t = 0; t < nt; ++t) {
    long long b = n * t / nt, e = n * (t + 1) / nt;
    th.emplace_back([&f, b, e, t] { f(b, e, t); });
  }
  for (auto &x : th) x.join();
}

// Dynamic work queue over items: f(item, thread_id).
void parallel_items(int n, const std::function<void(int, int)> &f) {
  int nt = std::min(n_threads(), std::max(1, n));
  if (nt <= 1) {
    for (int i = 0; i < n; ++i) f(i, 0);
    return;
  }
  std::atomic<int> next(0);
  std::vector<std::thread> th;
  for (int t = 0; t < nt; ++t)
    th.emplace_back([&, t] {
      for (;;) {
        int i = next.fetch_add(1);
        if (i >= n) break;
        f(i, t);
      }
    });
  for (auto &x : th) x.join();
}

std::vector<double> l1_rowsum(const Csr &A) {
  std::vector<double> d(A.nrows);
  for (int i = 0; i < A.nrows; ++i) {
    double s = 0.0;
    for (int jj = A.ptr[i]; jj < A.ptr[i + 1]; ++jj) s += std::fabs(A.val[jj]);
    d[i] = s;
  }
  return d;
}

Csr pattern_transpose(const Csr &A) {
  Csr T;
  T.nrows = A.ncols;
  T.ncols = A.nrows;
  T.ptr.assign(T.nrows + 1, 0);
  for (int jj = 0; jj < (int)A.nnz(); ++jj) T.ptr[A.col[jj] + 1]++;
  for (int i = 0; i < T.nrows; ++i) T.ptr[i + 1] += T.ptr[i];
  T.col.resize(A.nnz());
  std::vector<int> pos(T.ptr.begin(), T.ptr.end() - 1);
  for (int i = 0; i < A.nrows; ++i)
    for (int jj = A.ptr[i]; jj < A.ptr[i + 1]; ++jj) T.col[pos[A.col[jj]]++] = i;
  return T;
}

// Undirected graph of the stored pattern without the diagonal.
Csr adjacency(const Csr &A) {
  Csr T = pattern_transpose(A);
  Csr G;
  G.nrows = G.ncols = A.nrows;
  G.ptr.assign(A.nrows + 1, 0);
  std::vector<int> buf;
  std::vector<std::vector<int>> rows(A.nrows);
  for (int i = 0; i < A.nrows; ++i) {
    int a = A.ptr[i], ae = A.ptr[i + 1], t = T.ptr[i], te = T.ptr[i + 1];
    buf.clear();
    while (a < ae || t < te) {
      int c;
      if (t >= te || (a < ae && A.col[a] < T.col[t])) c = A.col[a++];
      else if (a >= ae || T.col[t] < A.col[a]) c = T.col[t++];
      else { c = A.col[a]; ++a; ++t; }
      if (c != i) buf.push_back(c);
    }
    G.ptr[i + 1] = G.ptr[i] + (int)buf.size();
    G.col.insert(G.col.end(), buf.begin(), buf.end());
  }
  return G;
}

// Dense inverse by Gauss-Jordan elimination with partial pivoting.
bool dense_inverse(int n, const std::vector<double> &A, std::vector<double> &inv) {
  std::vector<double> M(A);
  inv.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) inv[(size_t)i * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    double best = std::fabs(M[(size_t)c * n + c]);
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(M[(size_t)r * n + c]) > best) { best = std::fabs(M[(size_t)r * n + c]); piv = r; }
    if (!(best > 0.0)) return false;
    if (piv != c)
      for (int k = 0; k < n; ++k) {
        std::swap(M[(size_t)c * n + k], M[(size_t)piv * n + k]);
        std::swap(inv[(size_t)c * n + k], inv[(size_t)piv * n + k]);
      }
    double p = M[(size_t)c * n + c];
    for (int k = 0; k < n; ++k) { M[(size_t)c * n + k] /= p; inv[(size_t)c * n + k] /= p; }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      double f = M[(size_t)r * n + c];
      if (f == 0.0) continue;
      for (int k = 0; k < n; ++k) {
        M[(size_t)r * n + k] -= f * M[(size_t)c * n + k];
        inv[(size_t)r * n + k] -= f * inv[(size_t)c * n + k];
      }
    }
  }
  return true;
}

void free_csr(Csr &M) {
  Csr e;
  std::swap(M, e);
}

// Every stored column of a batched matrix must index its source vector and
// the slice table must cover exactly nrows rows (checked before any upload).
bool sell_in_bounds(const Sell &S, int nrows, int ncols) {
  if (S.nrows != nrows) return false;
  const int rs = 64 >> S.lg;
  const int ns = (nrows + rs - 1) / rs;
  if (nrows == 0) return S.sptr.empty() || S.sptr.back() == 0;
  if ((int)S.sptr.size() != ns + 1 || (size_t)S.sptr.back() != S.col.size() || S.col.size() != S.val.size()) return false;
  std::atomic<bool> ok(true);
  parallel_for((long long)S.col.size(), [&](long long b, long long e, int) {
    for (long long k = b; k < e; ++k)
      if (S.col[k] < 0 || S.col[k] >= ncols) { ok = false; return; }
  }, 1 << 20);
  return ok;
}

// Step structure of a slice of `size` = 64u entries with widest steps of
// V = 2^vlg entries per lane: floor(u/V) steps of 64V entries, then at most
// one step of each narrower width (64 * 2^v entries for v = vlg-1 .. 0, when
// bit v of u is set), so slice sizes equal those of the unpaired layout.
// Step of width 2^v holds, for lane p = (r mod 64/G) G + j, the 2^v
// consecutive entries of row r at offset p 2^v within the step.
inline int sell_region_steps(int u, int vlg, int v) { return v == vlg ? (u >> v) : ((u >> v) & 1); }

// Row (within its slice) of the entry stored at position `pos` of the slice.
inline int sell_slice_row(const Sell &S, int size, int pos) {
  const int u = size >> 6;
  int base = 0;
  for (int v = S.vlg; v > 0; --v) {
    const int span = sell_region_steps(u, S.vlg, v) << (6 + v);
    if (pos < base + span) return ((pos - base) & ((64 << v) - 1)) >> (S.lg + v);
    base += span;
  }
  return ((pos - base) & 63) >> S.lg;
}

// Block-diagonal check: every stored entry of row r (padding included) must
// point at a column owned by the same composite grid / problem as r.  The
// per-grid schedule runs grids concurrently, so any cross-grid load would race.
bool sell_block_diagonal(const Sell &S, const std::vector<int> &row_owner, const std::vector<int> &col_owner) {
  const int rs = 64 >> S.lg;
  const int ns = (S.nrows + rs - 1) / rs;
  std::atomic<bool> ok(true);
  parallel_for(ns, [&](long long b, long long e, int) {
    for (long long sl = b; sl < e && ok; ++sl) {
      const int base = S.sptr[sl], size = S.sptr[sl + 1] - base;
      for (int pos = 0; pos < size; ++pos) {
        const int r = (int)sl * rs + sell_slice_row(S, size, pos);
        if (r >= S.nrows) continue;
        const size_t a = (size_t)base + pos;
        // rows of no grid (alignment gaps) hold zeros only
        if (row_owner[r] < 0 ? S.val[a] != 0.0 : col_owner[S.col[a]] != row_owner[r]) { ok = false; return; }
      }
    }
  }, 256);
  return ok;
}

// Sliced-ELL layout filled row by row (rows may be written concurrently by
// different threads): set len[] for every row, call shape(), then put() every
// entry of a row and pad() it; rows never written keep padding from shape().
struct SellBuilder {
  Sell S;
  std::vector<int> len;
  int rs = 64;  // rows per slice
  void init(int nrows, int lg, int step_log2) {
    S.nrows = nrows;
    S.lg = lg;
    S.vlg = step_log2;
    rs = 64 >> lg;
    len.assign(nrows, 0);
  }
  void shape() {
    const int G = 1 << S.lg;
    const int ns = (S.nrows + rs - 1) / rs;
    std::vector<int> width(ns, 0);
    parallel_for(ns, [&](long long b, long long e, int) {
      for (long long s = b; s < e; ++s) {
        int w = 0;
        for (int r = (int)s * rs; r < std::min(S.nrows, (int)s * rs + rs); ++r) w = std::max(w, (len[r] + G - 1) / G);
        width[s] = w;
      }
    }, 1024);
    S.sptr.assign(ns + 1, 0);
    long long tot = 0;
    for (int s = 0; s < ns; ++s) {
      tot += 64LL * width[s];
      if (tot > std::numeric_limits<int>::max()) throw std::length_error("sliced-ELL layout exceeds 2^31 entries");
      S.sptr[s + 1] = (int)tot;
    }
    S.col.resize(tot);
    S.val.resize(tot);
    // rows past the last row of the final slice (never computed)
    if (ns > 0)
      for (int r = S.nrows; r < ns * rs; ++r)
        for (int k = 0; k < width[ns - 1] * G; ++k) {
          S.col[at(r, k)] = 0;
          S.val[at(r, k)] = 0.0;
        }
  }
  // entry k of row r (see sell_region_steps for the step structure)
  inline size_t at(int r, int k) const {
    const int lg = S.lg, s = r / rs, u = (S.sptr[s + 1] - S.sptr[s]) >> 6;
    size_t b = (size_t)S.sptr[s];
    for (int v = S.vlg; v >= 0; --v) {
      const int steps = sell_region_steps(u, S.vlg, v), gv = lg + v;
      const int per_row = steps << gv;  // entries of the row in this region
      if (k < per_row || v == 0)
        return b + ((size_t)(k >> gv) << (6 + v)) + ((size_t)(r % rs) << gv) + (k & ((1 << gv) - 1));
      k -= per_row;
      b += (size_t)steps << (6 + v);
    }
    return b;
  }
  inline void put(int r, int k, int c, double v) {
    const size_t a = at(r, k);
    S.col[a] = c;
    S.val[a] = v;
  }
  // padding entries of row r: value 0, column = the row's last column, or
  // `own` (a column of the same composite grid / problem) for an empty row,
  // so a padded load never touches another grid's data
  inline void pad(int r, int own) {
    const int s = r / rs;
    const int kmax = ((S.sptr[s + 1] - S.sptr[s]) >> 6) << S.lg;
    const int c = len[r] > 0 ? S.col[at(r, len[r] - 1)] : own;
    for (int k = len[r]; k < kmax; ++k) {
      S.col[at(r, k)] = c;
      S.val[at(r, k)] = 0.0;
    }
  }
  long long nnz_rows(int r0, int r1) const {
    long long n = 0;
    for (int r = r0; r < r1; ++r) n += len[r];
    return n;
  }
  Sell take() {
    std::vector<int>().swap(len);
    return std::move(S);
  }
};

// Copy of rows [0, nrows) of a filled layout into a layout of their own in
// which the rows are reordered: inside consecutive windows of `win` rows,
// by decreasing length (stable), so a slice holds rows of similar length.
// perm[k] = row held by position k.  own[r]: a column of row r's grid for its
// padding (rows of no grid: any, they hold zeros).
Sell permuted_layout(const SellBuilder &src, int nrows, int lg, int step_log2, int win, const std::vector<int> &own,
                     std::vector<int> &perm) {
  perm.resize(nrows);
  for (int r = 0; r < nrows; ++r) perm[r] = r;
  if (win > 0)
    parallel_for((nrows + win - 1) / win, [&](long long b, long long e, int) {
      for (long long w = b; w < e; ++w) {
        const int r0 = (int)w * win, r1 = std::min(nrows, r0 + win);
        std::stable_sort(perm.begin() + r0, perm.begin() + r1, [&](int x, int y) { return src.len[x] > src.len[y]; });
      }
    }, 64);
  SellBuilder dst;
  dst.init(nrows, lg, step_log2);
  for (int k = 0; k < nrows; ++k) dst.len[k] = src.len[perm[k]];
  dst.shape();
  parallel_for(nrows, [&](long long b, long long e, int) {
    for (long long k = b; k < e; ++k) {
      const int r = perm[k];
      for (int j = 0; j < src.len[r]; ++j) {
        const size_t a = src.at(r, j);
        dst.put((int)k, j, src.S.col[a], src.S.val[a]);
      }
      dst.pad((int)k, own[r]);
    }
  }, 4096);
  return dst.take();
}

// LDS bands of a composite operator, for its level-synchronous passes run in
// 1024-thread workgroups that stage the gathered vector in LDS.  Tile t is
// the ts slices from ts t on (one workgroup).  Its band is
// the set of columns of its nonzero entries, covered by at most kBandWindows
// windows: the span split at its kBandWindows - 1 largest gaps.  With
// W = kBandWindows, tiles[2W t .. 2W t + W-1] are the window starts and
// tiles[2W t + W .. 2W t + 2W-1] the cumulative window lengths (the last one
// is the band size, 0 for a tile without nonzero entries).  A tile whose
// windows would exceed `cap` values (rows that touch many scattered columns,
// e.g. ghost rows along a grid's boundary) lists its distinct columns
// instead: its first start is -1 - (offset of the list in bidx) and its
// band is the list.  colL[a] is the position of entry a's column in its
// tile's band (0 for zero entries).  Returns the largest band, or 0 with no
// bands kept when some tile's list still exceeds `cap` (the layout's passes
// then gather from memory).
int build_bands(Sell &S, int cap, int ts) {
  constexpr int W = kBandWindows;
  const int ns = (int)S.sptr.size() - 1;
  S.colL.clear();
  S.tiles.clear();
  S.bidx.clear();
  S.ts = 0;
  if (ns <= 0) return 0;
  const int nt = (ns + ts - 1) / ts;
  S.colL.assign(S.col.size(), 0);
  S.tiles.assign(2 * W * (size_t)nt, 0);
  std::vector<int> bmax(n_threads(), 0);
  std::atomic<bool> over{false};
  // listed tiles: (tile, its distinct columns), per thread, placed in bidx
  // in tile order afterwards
  std::vector<std::vector<std::pair<long long, std::vector<int>>>> lists(n_threads());
  parallel_for(nt, [&](long long b, long long e, int tid) {
    std::vector<int> cs;
    std::vector<std::pair<int, int>> gaps;
    for (long long t = b; t < e && !over.load(std::memory_order_relaxed); ++t) {
      const int e0 = S.sptr[(long long)ts * t], e1 = S.sptr[std::min<long long>(ns, (long long)ts * t + ts)];
      cs.clear();
      for (int a = e0; a < e1; ++a)
        if (S.val[a] != 0.0) cs.push_back(S.col[a]);
      if (cs.empty()) continue;
      std::sort(cs.begin(), cs.end());
      cs.erase(std::unique(cs.begin(), cs.end()), cs.end());
      gaps.clear();
      for (size_t k = 1; k < cs.size(); ++k)
        if (cs[k] - cs[k - 1] > 1) gaps.push_back({cs[k] - cs[k - 1], (int)k});
      const size_t ng = std::min<size_t>(W - 1, gaps.size());
      std::partial_sort(gaps.begin(), gaps.begin() + ng, gaps.end(),
                        [](const std::pair<int, int> &x, const std::pair<int, int> &y) {
                          return x.first > y.first || (x.first == y.first && x.second < y.second);
                        });
      std::vector<int> cut;  // first index in cs of windows 1..
      for (size_t k = 0; k < ng; ++k) cut.push_back(gaps[k].second);
      std::sort(cut.begin(), cut.end());
      int lo[W] = {}, end[W] = {};
      int first = 0, acc = 0;
      for (size_t w = 0; w <= cut.size(); ++w) {
        const int last = (w < cut.size() ? cut[w] : (int)cs.size()) - 1;
        lo[w] = cs[first];
        acc += cs[last] - cs[first] + 1;
        end[w] = acc;
        first = last + 1;
      }
      for (size_t w = cut.size() + 1; w < (size_t)W; ++w) end[w] = acc;
      int *d = &S.tiles[2 * W * (size_t)t];
      if (acc > cap) {
        const int n = (int)cs.size();
        if (n > cap) {
          over = true;
          return;
        }
        for (int w = 0; w < W; ++w) d[W + w] = n;
        bmax[tid] = std::max(bmax[tid], n);
        for (int a = e0; a < e1; ++a)
          if (S.val[a] != 0.0) S.colL[a] = (uint16_t)(std::lower_bound(cs.begin(), cs.end(), S.col[a]) - cs.begin());
        lists[tid].push_back({t, cs});
        continue;
      }
      for (int w = 0; w < W; ++w) {
        d[w] = lo[w];
        d[W + w] = end[w];
      }
      bmax[tid] = std::max(bmax[tid], acc);
      for (int a = e0; a < e1; ++a) {
        if (S.val[a] == 0.0) continue;
        const int c = S.col[a];
        int w = W - 1;
        while (w > 0 && (end[w - 1] == end[w] || c < lo[w])) --w;
        S.colL[a] = (uint16_t)((w ? end[w - 1] : 0) + c - lo[w]);
      }
    }
  }, 1);
  if (over) {
    std::vector<uint16_t>().swap(S.colL);
    std::vector<int>().swap(S.tiles);
    return 0;
  }
  std::vector<std::pair<long long, std::vector<int>>> all;
  for (auto &v : lists)
    for (auto &x : v) all.push_back(std::move(x));
  std::sort(all.begin(), all.end(), [](const auto &x, const auto &y) { return x.first < y.first; });
  for (auto &x : all) {
    S.tiles[2 * W * (size_t)x.first] = -1 - (int)S.bidx.size();
    S.bidx.insert(S.bidx.end(), x.second.begin(), x.second.end());
  }
  S.ts = ts;
  return *std::max_element(bmax.begin(), bmax.end());
}

// Check of build_bands: every nonzero entry of a banded tile decodes back to
// its column through its window, and every entry's position lies in the band.
bool bands_valid(const Sell &S, int cap, int ts) {
  constexpr int W = kBandWindows;
  const int ns = (int)S.sptr.size() - 1;
  if (S.tiles.empty()) return S.colL.empty();
  const int nt = (ns + ts - 1) / ts;
  if (ns <= 0) return true;
  if (S.colL.size() != S.col.size() || S.tiles.size() != 2 * W * (size_t)nt) return false;
  std::atomic<bool> ok{true};
  parallel_for(nt, [&](long long b, long long e, int) {
    for (long long t = b; t < e; ++t) {
      const int *d = &S.tiles[2 * W * (size_t)t];
      const int n = d[2 * W - 1];
      if (n == 0) continue;
      if (n > cap || d[W] < 0) { ok = false; return; }
      for (int w = 1; w < W; ++w)
        if (d[W + w - 1] > d[W + w]) { ok = false; return; }
      const bool listed = d[0] < 0;
      const long long off = listed ? -1LL - d[0] : 0;
      if (listed && (off + n > (long long)S.bidx.size() || d[W] != n)) { ok = false; return; }
      const int e0 = S.sptr[(long long)ts * t], e1 = S.sptr[std::min<long long>(ns, (long long)ts * t + ts)];
      for (int a = e0; a < e1; ++a) {
        const int q = S.colL[a];
        if (q >= n) { ok = false; return; }
        if (S.val[a] == 0.0) continue;
        if (listed) {
          if (S.bidx[off + q] != S.col[a]) { ok = false; return; }
          continue;
        }
        int w = 0;
        while (q >= d[W + w]) ++w;
        if (d[w] + q - (w ? d[W + w - 1] : 0) != S.col[a]) { ok = false; return; }
      }
    }
  }, 1);
  return ok;
}

// 16-bit column compression of a checked block-diagonal layout (see Sell).
// Per slice, the columns of its nonzero entries are split at their largest gap
// into two windows of at most 32768 columns (one window of 65536 when they
// span no more).  Zero-valued entries (padding, explicit symbolic zeros)
// contribute nothing and may take any column of their row's own grid /
// problem: one outside the windows is moved to a column of the same owner
// inside them; rows past the last row take the first window's base.  Returns
// false (layout left as is) when some slice does not fit.
bool compress_columns(Sell &S, const std::vector<int> &row_owner, const std::vector<int> &col_owner) {
  const int rs = 64 >> S.lg;
  const int ns = (int)S.sptr.size() - 1;
  if (ns <= 0) return false;
  std::vector<uint16_t> c16(S.col.size());
  std::vector<int> base(2 * (size_t)ns);
  std::atomic<bool> ok{true};
  parallel_for(ns, [&](long long b, long long e, int) {
    std::vector<int> cs, owners;
    for (long long s = b; s < e && ok.load(std::memory_order_relaxed); ++s) {
      const int e0 = S.sptr[s], e1 = S.sptr[s + 1];
      const int r0 = (int)s * rs;
      auto row_of = [&](int a) { return r0 + sell_slice_row(S, e1 - e0, a - e0); };
      cs.clear();
      owners.clear();
      for (int a = e0; a < e1; ++a) {
        const int r = row_of(a);
        if (S.val[a] != 0.0 && r < S.nrows) {
          cs.push_back(S.col[a]);
          if (std::find(owners.begin(), owners.end(), row_owner[r]) == owners.end()) owners.push_back(row_owner[r]);
        }
      }
      // an owner whose rows in this slice hold zeros only keeps one of its
      // own columns in the windows
      for (int a = e0; a < e1; ++a) {
        const int r = row_of(a);
        if (r < S.nrows && row_owner[r] >= 0 && std::find(owners.begin(), owners.end(), row_owner[r]) == owners.end()) {
          owners.push_back(row_owner[r]);
          cs.push_back(S.col[a]);
        }
      }
      std::sort(cs.begin(), cs.end());
      cs.erase(std::unique(cs.begin(), cs.end()), cs.end());
      int b0 = cs.empty() ? 0 : cs.front(), b1 = b0 + 32768;
      if (!cs.empty() && cs.back() - cs.front() > 65535) {
        size_t gi = 0;
        int gap = -1;
        for (size_t k = 1; k < cs.size(); ++k)
          if (cs[k] - cs[k - 1] > gap) { gap = cs[k] - cs[k - 1]; gi = k; }
        b1 = cs[gi];
        if (cs[gi - 1] - b0 > 32767 || cs.back() - b1 > 32767) { ok = false; return; }
      }
      auto enc = [&](int c, uint16_t &out) {
        if (c >= b0 && c - b0 <= 32767) { out = (uint16_t)(c - b0); return true; }
        if (c >= b1 && c - b1 <= 32767) { out = (uint16_t)(0x8000 | (c - b1)); return true; }
        return false;
      };
      for (int a = e0; a < e1; ++a) {
        const int r = row_of(a);
        if (r >= S.nrows || (row_owner[r] < 0 && S.val[a] == 0.0)) { S.col[a] = b0; c16[a] = 0; continue; }
        if (!enc(S.col[a], c16[a])) {
          if (S.val[a] != 0.0) { ok = false; return; }
          // a zero entry outside the windows: any in-window column of the same owner
          bool moved = false;
          for (int c : cs)
            if (col_owner[c] == row_owner[r]) { S.col[a] = c; enc(c, c16[a]); moved = true; break; }
          for (int a2 = e0; a2 < e1 && !moved; ++a2) {
            uint16_t q;
            if (row_of(a2) < S.nrows && col_owner[S.col[a2]] == row_owner[r] && enc(S.col[a2], q)) {
              S.col[a] = S.col[a2];
              c16[a] = q;
              moved = true;
            }
          }
          if (!moved) { ok = false; return; }
        }
        const int dec = ((c16[a] & 0x8000) ? b1 : b0) + (c16[a] & 0x7fff);
        if (dec != S.col[a]) { ok = false; return; }
      }
      base[2 * s] = b0;
      base[2 * s + 1] = b1;
    }
  }, 64);
  if (!ok) return false;
  S.col16 = std::move(c16);
  S.base = std::move(base);
  std::vector<int>().swap(S.col);
  return true;
}

// Lanes per row for rows averaging `avg` entries: one lane up to 20 entries,
// otherwise the smallest power of two G <= 16 with at most `target` entries
// per lane (Setup::comp_lane_target on composite levels, 12 on the global
// levels of the V-cycle).
#ifndef AMGDD_LANE_ONE
#define AMGDD_LANE_ONE 20.0
#endif
#ifndef AMGDD_GLANE_TARGET
#define AMGDD_GLANE_TARGET 12.0
#endif
int lanes_log2(double avg, double target) {
  if (avg <= AMGDD_LANE_ONE) return 0;
  int lg = 1;
  while (lg < 4 && avg / (1 << lg) > target) ++lg;
  return lg;
}

}  // namespace

// ---------------------------------------------------------------------------
// AMG components (Section 2)

Csr strength(const Csr &A, double theta) {
  const int n = A.nrows;
  Csr S;
  S.nrows = S.ncols = n;
  S.ptr.assign(n + 1, 0);
  for (int i = 0; i < n; ++i) {
    double m = -std::numeric_limits<double>::infinity();
    for (int jj = A.ptr[i]; jj < A.ptr[i + 1]; ++jj)
      if (A.col[jj] != i) m = std::max(m, -A.val[jj]);
    if (m > 0.0) {
      double thr = theta * m * (1.0 - 1e-12);
      for (int jj = A.ptr[i]; jj < A.ptr[i + 1]; ++jj)
        if (A.col[jj] != i && -A.val[jj] >= thr) S.col.push_back(A.col[jj]);
    }
    S.ptr[i + 1] = (int)S.col.size();
  }
  return S;
}

std::vector<int8_t> rs_first_pass(const Csr &S) {
  const int n = S.nrows;
  Csr T = pattern_transpose(S);  // row i: points that i strongly influences
  std::vector<long long> lam(n);
  std::vector<int8_t> st(n, 0);
  // Tournament tree over the undecided points, key = (lambda, smallest index
  // first); decided points have key 0.  The root is the next C-point.
  int size = 1;
  while (size < n) size <<= 1;
  std::vector<unsigned long long> tree(2 * (size_t)size, 0ull);
  auto key = [](long long l, int i) -> unsigned long long {
    return ((unsigned long long)(l + 1) << 32) | (unsigned long long)(0xFFFFFFFFu - (unsigned)i);
  };
  auto update = [&](int i, unsigned long long k) {
    size_t pos = (size_t)size + i;
    tree[pos] = k;
    for (pos >>= 1; pos >= 1; pos >>= 1) {
      unsigned long long m = std::max(tree[2 * pos], tree[2 * pos + 1]);
      if (tree[pos] == m) break;
      tree[pos] = m;
    }
  };
  for (int i = 0; i < n; ++i) {
    lam[i] = T.ptr[i + 1] - T.ptr[i];
    if (S.ptr[i + 1] == S.ptr[i] && lam[i] == 0) st[i] = -1;
    else tree[(size_t)size + i] = key(lam[i], i);
  }
  for (size_t pos = (size_t)size - 1; pos >= 1; --pos) tree[pos] = std::max(tree[2 * pos], tree[2 * pos + 1]);
  std::vector<int> newf;
  while (tree[1] != 0ull) {
    const unsigned long long k = tree[1];
    const int i = (int)(0xFFFFFFFFu - (unsigned)(k & 0xFFFFFFFFull));
    if (lam[i] == 0) {
      for (int u = 0; u < n; ++u) {
        if (st[u] != 0) continue;
        bool has_c = false;
        for (int jj = S.ptr[u]; jj < S.ptr[u + 1]; ++jj)
          if (st[S.col[jj]] == 1) { has_c = true; break; }
        st[u] = has_c ? -1 : 1;
      }
      break;
    }
    st[i] = 1;
    update(i, 0ull);
    newf.clear();
    for (int jj = T.ptr[i]; jj < T.ptr[i + 1]; ++jj)
      if (st[T.col[jj]] == 0) newf.push_back(T.col[jj]);
    for (int j : newf) { st[j] = -1; update(j, 0ull); }
    for (int j : newf)
      for (int kk = S.ptr[j]; kk < S.ptr[j + 1]; ++kk) {
        int q = S.col[kk];
        if (st[q] == 0) { lam[q] += 1; update(q, key(lam[q], q)); }
      }
    for (int jj = S.ptr[i]; jj < S.ptr[i + 1]; ++jj) {
      int q = S.col[jj];
      if (st[q] == 0) { lam[q] -= 1; update(q, key(lam[q], q)); }
    }
  }
  return st;
}

Csr direct_interpolation(const Csr &A, const Csr &S, const std::vector<int8_t> &cf) {
  const int n = A.nrows;
  std::vector<int> cidx(n, -1);
  int nc = 0;
  for (int i = 0; i < n; ++i)
    if (cf[i] == 1) cidx[i] = nc++;
  Csr P;
  P.nrows = n;
  P.ncols = nc;
  P.ptr.assign(n + 1, 0);
  std::vector<char> inp;
  for (int i = 0; i < n; ++i) {
    if (cf[i] == 1) {
      P.col.push_back(cidx[i]);
      P.val.push_back(1.0);
    } else {
      const int a0 = A.ptr[i], a1 = A.ptr[i + 1];
      inp.assign(a1 - a0, 0);
      // membership in S_i by a merge of two sorted rows
      int s = S.ptr[i];
      for (int jj = a0; jj < a1; ++jj) {
        int c = A.col[jj];
        while (s < S.ptr[i + 1] && S.col[s] < c) ++s;
        bool strong = s < S.ptr[i + 1] && S.col[s] == c;
        inp[jj - a0] = strong && cf[c] == 1;
      }
      double neg = 0.0, pos = 0.0, den = 0.0, diag = 0.0;
      bool any = false;
      for (int jj = a0; jj < a1; ++jj) {
        int c = A.col[jj];
        double v = A.val[jj];
        neg += (c != i) ? std::min(v, 0.0) : 0.0;
        pos += (c != i) ? std::max(v, 0.0) : 0.0;
        den += inp[jj - a0] ? v : 0.0;
        if (c == i) diag = v;
        any = any || inp[jj - a0];
      }
      if (any) {
        double at = diag + pos;
        double alpha = neg / den;
        for (int jj = a0; jj < a1; ++jj)
          if (inp[jj - a0]) {
            P.col.push_back(cidx[A.col[jj]]);
            P.val.push_back((-alpha * A.val[jj]) / at);
          }
      }
    }
    P.ptr[i + 1] = (int)P.col.size();
  }
  return P;
}

// ---- "best practices" components (PMIS / HMIS coarsening, extended+i
// interpolation) from their published definitions: De Sterck, Yang, Heys
// (2006) and De Sterck, Falgout, Nolting, Yang (2008).

// SplitMix64 (Steele, Lea, Flood 2014), all arithmetic mod 2^64.
uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Tie-break values of PMIS on `level`: r_i = (SplitMix64(2^32 level + i) >> 11) / 2^53.
std::vector<double> pmis_random(int level, int n) {
  std::vector<double> r(n);
  for (int i = 0; i < n; ++i)
    r[i] = (double)(splitmix64(((uint64_t)level << 32) + (uint64_t)i) >> 11) * 0x1.0p-53;
  return r;
}

// PMIS: lambda_i = |S^T_i| + r_i; points influencing nobody are F; each round
// every undecided point whose lambda exceeds that of all its undecided strong
// neighbours (either direction; equal lambda: smaller index wins) becomes C,
// and the undecided points strongly depending on a new C-point become F.
// c_init (optional): C-points fixed before the first round (their dependents F).
std::vector<int8_t> pmis(const Csr &S, const std::vector<double> &rand, const std::vector<char> *c_init) {
  const int n = S.nrows;
  Csr T = pattern_transpose(S);
  std::vector<double> lam(n);
  std::vector<int8_t> st(n, 0);
  for (int i = 0; i < n; ++i) lam[i] = (double)(T.ptr[i + 1] - T.ptr[i]) + rand[i];
  if (c_init)
    for (int i = 0; i < n; ++i)
      if ((*c_init)[i]) st[i] = 1;
  for (int i = 0; i < n; ++i)
    if (st[i] == 0 && T.ptr[i + 1] == T.ptr[i]) st[i] = -1;
  auto mark = [&](const std::vector<int> &cs) {
    for (int i : cs)
      for (int jj = T.ptr[i]; jj < T.ptr[i + 1]; ++jj)
        if (st[T.col[jj]] == 0) st[T.col[jj]] = -1;
  };
  if (c_init) {
    std::vector<int> c0;
    for (int i = 0; i < n; ++i)
      if ((*c_init)[i]) c0.push_back(i);
    mark(c0);
  }
  std::vector<int> und, nc;
  for (;;) {
    und.clear();
    for (int i = 0; i < n; ++i)
      if (st[i] == 0) und.push_back(i);
    if (und.empty()) break;
    nc.clear();
    for (int i : und) {
      bool win = true;
      auto beats = [&](int j) { return st[j] == 0 && j != i && (lam[j] > lam[i] || (lam[j] == lam[i] && j < i)); };
      for (int jj = S.ptr[i]; jj < S.ptr[i + 1] && win; ++jj)
        if (beats(S.col[jj])) win = false;
      for (int jj = T.ptr[i]; jj < T.ptr[i + 1] && win; ++jj)
        if (beats(T.col[jj])) win = false;
      if (win) nc.push_back(i);
    }
    for (int i : nc) st[i] = 1;
    mark(nc);
  }
  return st;
}

// HMIS: one RS first pass inside every subdomain (strong connections between
// points of the same subdomain only); its C-points without a strong connection
// to another subdomain start PMIS.
std::vector<int8_t> hmis(const Csr &S, const std::vector<int> &part, const std::vector<double> &rand) {
  const int n = S.nrows;
  Csr L;
  L.nrows = L.ncols = n;
  L.ptr.assign(n + 1, 0);
  std::vector<char> bnd(n, 0);
  for (int i = 0; i < n; ++i) {
    for (int jj = S.ptr[i]; jj < S.ptr[i + 1]; ++jj) {
      const int j = S.col[jj];
      if (part[j] == part[i]) L.col.push_back(j);
      else bnd[i] = bnd[j] = 1;
    }
    L.ptr[i + 1] = (int)L.col.size();
  }
  std::vector<int8_t> cf = rs_first_pass(L);
  std::vector<char> c0(n, 0);
  for (int i = 0; i < n; ++i) c0[i] = cf[i] == 1 && !bnd[i];
  return pmis(S, rand, &c0);
}

// Extended+i interpolation, no truncation.  F-point i: strong C-neighbours
// C_i, strong F-neighbours F_i, weak neighbours W_i (all other off-diagonal
// entries); Chat_i = C_i plus the strong C-neighbours of every k in F_i;
// abar_kl = a_kl when a_kl a_kk < 0, else 0; d_k = sum of abar_kl over
// l in Chat_i + {i};
//   w_ij = -num_ij / at_ii,  num_ij = a_ij + sum_k a_ik abar_kj / d_k,
//   at_ii = a_ii + sum_{n in W_i \ Chat_i} a_in + sum_k a_ik abar_ki / d_k,
// a k with d_k = 0 lumped into at_ii like a weak neighbour.  Sums in ascending
// index order (W terms, then k terms, into at_ii).  C-points inject; F-points
// with empty Chat_i get an empty row.
// Truncation of one interpolation row: keep the pmax entries of largest
// magnitude (smaller column first on ties), scaled by (sum of all entries) /
// (sum of the kept ones), both summed in ascending column order; pmax <= 0 or
// a row of at most pmax entries is left as is.
void truncate_row(std::vector<int> &cols, std::vector<double> &vals, int pmax) {
  const int m = (int)vals.size();
  if (pmax <= 0 || m <= pmax) return;
  std::vector<int> order(m);
  for (int q = 0; q < m; ++q) order[q] = q;
  std::sort(order.begin(), order.end(), [&](int a, int b) {
    const double fa = std::fabs(vals[a]), fb = std::fabs(vals[b]);
    return fa != fb ? fa > fb : cols[a] < cols[b];
  });
  std::vector<int> keep(order.begin(), order.begin() + pmax);
  std::sort(keep.begin(), keep.end(), [&](int a, int b) { return cols[a] < cols[b]; });
  double total = 0.0, kept = 0.0;
  for (double v : vals) total += v;
  for (int q : keep) kept += vals[q];
  std::vector<int> c2;
  std::vector<double> v2;
  for (int q : keep) {
    c2.push_back(cols[q]);
    v2.push_back(kept == 0.0 ? vals[q] : vals[q] * (total / kept));
  }
  cols.swap(c2);
  vals.swap(v2);
}

Csr ext_i_interpolation(const Csr &A, const Csr &S, const std::vector<int8_t> &cf, int pmax) {
  const int n = A.nrows;
  std::vector<int> cidx(n, -1);
  int nc = 0;
  for (int i = 0; i < n; ++i)
    if (cf[i] == 1) cidx[i] = nc++;
  Csr P;
  P.nrows = n;
  P.ncols = nc;
  P.ptr.assign(n + 1, 0);
  std::vector<int> mark_s(n, -1), mark_c(n, -1), posk(n, -1), posi(n, -1);
  std::vector<double> vk(n, 0.0), vi(n, 0.0), num;
  std::vector<int> chat, Fi;
  for (int i = 0; i < n; ++i) {
    if (cf[i] == 1) {
      P.col.push_back(cidx[i]);
      P.val.push_back(1.0);
      P.ptr[i + 1] = (int)P.col.size();
      continue;
    }
    chat.clear();
    Fi.clear();
    for (int jj = S.ptr[i]; jj < S.ptr[i + 1]; ++jj) {
      const int j = S.col[jj];
      mark_s[j] = i;
      if (cf[j] == 1) {
        if (mark_c[j] != i) { mark_c[j] = i; chat.push_back(j); }
      } else {
        Fi.push_back(j);
      }
    }
    for (int k : Fi)
      for (int jj = S.ptr[k]; jj < S.ptr[k + 1]; ++jj) {
        const int l = S.col[jj];
        if (cf[l] == 1 && mark_c[l] != i) { mark_c[l] = i; chat.push_back(l); }
      }
    if (chat.empty()) {
      P.ptr[i + 1] = (int)P.col.size();
      continue;
    }
    std::sort(chat.begin(), chat.end());
    std::sort(Fi.begin(), Fi.end());
    // row i scattered
    double aii = 0.0;
    for (int jj = A.ptr[i]; jj < A.ptr[i + 1]; ++jj) {
      posi[A.col[jj]] = i;
      vi[A.col[jj]] = A.val[jj];
      if (A.col[jj] == i) aii = A.val[jj];
    }
    double at = aii;
    for (int jj = A.ptr[i]; jj < A.ptr[i + 1]; ++jj) {
      const int c = A.col[jj];
      if (c != i && mark_s[c] != i && mark_c[c] != i) at += A.val[jj];
    }
    num.assign(chat.size(), 0.0);
    for (size_t q = 0; q < chat.size(); ++q) num[q] = posi[chat[q]] == i ? vi[chat[q]] : 0.0;
    for (int k : Fi) {
      double akk = 0.0;
      for (int jj = A.ptr[k]; jj < A.ptr[k + 1]; ++jj) {
        posk[A.col[jj]] = k;
        vk[A.col[jj]] = A.val[jj];
        if (A.col[jj] == k) akk = A.val[jj];
      }
      double d = 0.0;
      for (int jj = A.ptr[k]; jj < A.ptr[k + 1]; ++jj) {
        const int l = A.col[jj];
        if ((mark_c[l] == i || l == i) && A.val[jj] * akk < 0) d += A.val[jj];
      }
      const double aik = vi[k];
      if (d == 0.0) {
        at += aik;
        continue;
      }
      for (size_t q = 0; q < chat.size(); ++q) {
        const int j = chat[q];
        const double abar = posk[j] == k ? vk[j] : 0.0;
        if (abar * akk < 0) num[q] += aik * abar / d;
      }
      const double abar_ki = posk[i] == k ? vk[i] : 0.0;
      if (abar_ki * akk < 0) at += aik * abar_ki / d;
    }
    std::vector<int> rc(chat.size());
    std::vector<double> rv(chat.size());
    for (size_t q = 0; q < chat.size(); ++q) {
      rc[q] = cidx[chat[q]];
      rv[q] = -(num[q] / at);
    }
    truncate_row(rc, rv, pmax);
    P.col.insert(P.col.end(), rc.begin(), rc.end());
    P.val.insert(P.val.end(), rv.begin(), rv.end());
    P.ptr[i + 1] = (int)P.col.size();
  }
  return P;
}

Csr transpose(const Csr &A) {
  Csr T;
  T.nrows = A.ncols;
  T.ncols = A.nrows;
  T.ptr.assign(T.nrows + 1, 0);
  for (long long jj = 0; jj < A.nnz(); ++jj) T.ptr[A.col[jj] + 1]++;
  for (int i = 0; i < T.nrows; ++i) T.ptr[i + 1] += T.ptr[i];
  T.col.resize(A.nnz());
  T.val.resize(A.nnz());
  std::vector<int> pos(T.ptr.begin(), T.ptr.end() - 1);
  for (int i = 0; i < A.nrows; ++i)
    for (int jj = A.ptr[i]; jj < A.ptr[i + 1]; ++jj) {
      int p = pos[A.col[jj]]++;
      T.col[p] = i;
      T.val[p] = A.val[jj];
    }
  return T;
}

// Row-by-row product; every product term creates an entry (symbolic
// pattern), accumulated in the order of A's row then B's row.
Csr spgemm(const Csr &A, const Csr &B) {
  const int n = A.nrows, m = B.ncols;
  int nt = n_threads();
  long long chunks = std::max(1LL, std::min<long long>(4LL * nt, (n + 1023) / 1024));
  std::vector<std::vector<int>> ccol(chunks), clen(chunks);
  std::vector<std::vector<double>> cval(chunks);
  std::atomic<long long> next(0);
  auto work = [&] {
    std::vector<double> acc(m, 0.0);
    std::vector<int> mark(m, -1), list;
    for (;;) {
      long long c = next.fetch_add(1);
      if (c >= chunks) break;
      int r0 = (int)(n * c / chunks), r1 = (int)(n * (c + 1) / chunks);
      auto &oc = ccol[c];
      auto &ov = cval[c];
      auto &ol = clen[c];
      for (int i = r0; i < r1; ++i) {
        list.clear();
        for (int jj = A.ptr[i]; jj < A.ptr[i + 1]; ++jj) {
          int k = A.col[jj];
          double a = A.val[jj];
          for (int kk = B.ptr[k]; kk < B.ptr[k + 1]; ++kk) {
            int j = B.col[kk];
            if (mark[j] != i) { mark[j] = i; acc[j] = 0.0; list.push_back(j); }
            acc[j] += a * B.val[kk];
          }
        }
        std::sort(list.begin(), list.end());
        for (int j : list) { oc.push_back(j); ov.push_back(acc[j]); }
        ol.push_back((int)list.size());
      }
    }
  };
  int nth = (int)std::min<long long>(nt, chunks);
  std::vector<std::thread> th;
  for (int t = 1; t < nth; ++t) th.emplace_back(work);
  work();
  for (auto &x : th) x.join();
  Csr C;
  C.nrows = n;
  C.ncols = m;
  C.ptr.assign(n + 1, 0);
  long long tot = 0;
  int row = 0;
  for (long long c = 0; c < chunks; ++c)
    for (int len : clen[c]) { tot += len; C.ptr[++row] = (int)tot; }
  if (tot > std::numeric_limits<int>::max()) throw std::length_error("product exceeds 2^31 nonzeros");
  C.col.reserve(tot);
  C.val.reserve(tot);
  for (long long c = 0; c < chunks; ++c) {
    C.col.insert(C.col.end(), ccol[c].begin(), ccol[c].end());
    C.val.insert(C.val.end(), cval[c].begin(), cval[c].end());
  }
  return C;
}

// ---------------------------------------------------------------------------

namespace {

int validate(const ProblemInput &in, int max_coarse, std::string &err) {
  if (in.n <= 0 || !in.rowptr || !in.colind || !in.val || !in.part) { err = "null array or n <= 0"; return ST_EINVAL; }
  if (in.nparts <= 0 || in.nparts > in.n) { err = "nparts out of range"; return ST_EINVAL; }
  if (in.eta < 0) { err = "negative padding"; return ST_EINVAL; }
  if (in.n_etas < 0 || in.n_etas > 1024 || (in.n_etas > 0 && !in.etas)) { err = "bad per-level padding array"; return ST_EINVAL; }
  for (int l = 0; l < in.n_etas; ++l)
    if (in.etas[l] < 0) { err = "negative padding on level " + std::to_string(l); return ST_EINVAL; }
  if (in.rowptr[0] != 0) { err = "rowptr[0] != 0"; return ST_EINVAL; }
  for (int i = 0; i < in.n; ++i) {
    int a = in.rowptr[i], b = in.rowptr[i + 1];
    if (b < a) { err = "rowptr not monotone at row " + std::to_string(i); return ST_EINVAL; }
    bool diag = false;
    for (int jj = a; jj < b; ++jj) {
      int c = in.colind[jj];
      if (c < 0 || c >= in.n) { err = "column out of range in row " + std::to_string(i); return ST_EINVAL; }
      if (jj > a && c <= in.colind[jj - 1]) { err = "columns not sorted/unique in row " + std::to_string(i); return ST_EINVAL; }
      if (!std::isfinite(in.val[jj])) { err = "non-finite value in row " + std::to_string(i); return ST_EINVAL; }
      if (c == i) {
        diag = true;
        if (!(in.val[jj] > 0.0)) { err = "non-positive diagonal in row " + std::to_string(i); return ST_EINVAL; }
      }
    }
    if (!diag) { err = "missing diagonal in row " + std::to_string(i); return ST_EINVAL; }
  }
  std::vector<int> cnt(in.nparts, 0);
  for (int i = 0; i < in.n; ++i) {
    if (in.part[i] < 0 || in.part[i] >= in.nparts) { err = "part value out of range"; return ST_EINVAL; }
    cnt[in.part[i]]++;
  }
  for (int p = 0; p < in.nparts; ++p)
    if (cnt[p] == 0) { err = "empty subdomain " + std::to_string(p); return ST_EINVAL; }
  if (in.n <= max_coarse) { err = "problem not larger than max_coarse: no multigrid levels"; return ST_EUNSUP; }
  return ST_OK;
}

int build_hierarchy(ProblemHost &P, double theta, int max_coarse, int max_levels, int coarsen, int interp, int pmax,
                    std::string &err) {
  Hierarchy &H = P.H;
  H.A.push_back(P.A0);
  std::vector<int> part = P.part;  // subdomains of the current level (HMIS)
  while (H.A.back().nrows > max_coarse && (int)H.A.size() < max_levels) {
    const Csr &A = H.A.back();
    double th = now_s();
    Csr S = strength(A, theta);
    vlog("hier: strength", th);
    th = now_s();
    std::vector<int8_t> cf = coarsen == 1 ? hmis(S, part, pmis_random((int)H.A.size() - 1, A.nrows)) : rs_first_pass(S);
    vlog("hier: coarsening", th);
    th = now_s();
    int nc = 0;
    for (auto c : cf) nc += c == 1;
    if (nc == 0 || nc == A.nrows) break;
    Csr Pm = interp == 1 ? ext_i_interpolation(A, S, cf, pmax) : direct_interpolation(A, S, cf);
    {
      std::vector<int> next;
      next.reserve(nc);
      for (int i = 0; i < A.nrows; ++i)
        if (cf[i] == 1) next.push_back(part[i]);
      part = std::move(next);
    }
    vlog("hier: interp", th);
    th = now_s();
    Csr R = transpose(Pm);
    Csr AP = spgemm(A, Pm);
    vlog("hier: AP", th);
    th = now_s();
    Csr Ac = spgemm(R, AP);
    vlog("hier: RAP", th);
    H.cf.push_back(std::move(cf));
    H.P.push_back(std::move(Pm));
    H.R.push_back(std::move(R));
    H.A.push_back(std::move(Ac));
  }
  if (H.L() < 1) { err = "coarsening produced no coarse level"; return ST_EUNSUP; }
  for (auto &A : H.A) H.l1.push_back(l1_rowsum(A));
  const Csr &Ac = H.A.back();
  int nl = Ac.nrows;
  if (nl > 1024) { err = "coarsest level has " + std::to_string(nl) + " > 1024 points"; return ST_EUNSUP; }
  H.Ac.assign((size_t)nl * nl, 0.0);
  for (int i = 0; i < nl; ++i)
    for (int jj = Ac.ptr[i]; jj < Ac.ptr[i + 1]; ++jj) H.Ac[(size_t)i * nl + Ac.col[jj]] = Ac.val[jj];
  if (!dense_inverse(nl, H.Ac, H.Ac_inv)) { err = "singular coarsest operator"; return ST_EINVAL; }
  return ST_OK;
}

struct Stamp {
  std::vector<int> mark, idx;
  int epoch = 0;
  void size(int n) {
    if ((int)mark.size() < n) { mark.assign(n, 0); idx.assign(n, 0); epoch = 0; }
  }
  int next() {
    if (++epoch == std::numeric_limits<int>::max()) { std::fill(mark.begin(), mark.end(), 0); epoch = 1; }
    return epoch;
  }
};

struct Scratch {
  Stamp a, b, c;
  std::vector<int> front, nxt, list;
};

// Composite sets of one subdomain (Section 3, Section 4.1).
void build_sets(const ProblemHost &P, const std::vector<Csr> &G, const std::vector<std::vector<int>> &cmap, int p,
                CompGrid &cg, Scratch &sc) {
  const Hierarchy &H = P.H;
  const int L = H.L();
  cg.lv.assign(L + 1, CompLevel());
  std::vector<int> seeds;
  for (int i = 0; i < P.n; ++i)
    if (P.part[i] == p) seeds.push_back(i);
  cg.owned_gid = seeds;
  for (int l = 0; l <= L; ++l) {
    const int nl = H.A[l].nrows;
    sc.a.size(nl);
    CompLevel &lv = cg.lv[l];
    std::vector<int> D;
    if (l == L) {
      D.resize(nl);
      for (int i = 0; i < nl; ++i) D[i] = i;
    } else {
      int e = sc.a.next();
      D = seeds;
      for (int s : seeds) sc.a.mark[s] = e;
      sc.front = seeds;
      const int eta = P.eta_of(l);
      for (int r = 0; r < eta && !sc.front.empty(); ++r) {
        sc.nxt.clear();
        for (int v : sc.front)
          for (int jj = G[l].ptr[v]; jj < G[l].ptr[v + 1]; ++jj) {
            int u = G[l].col[jj];
            if (sc.a.mark[u] != e) { sc.a.mark[u] = e; sc.nxt.push_back(u); D.push_back(u); }
          }
        std::swap(sc.front, sc.nxt);
      }
      std::sort(D.begin(), D.end());
    }
    int e = sc.a.next();
    for (int v : D) sc.a.mark[v] = e;
    std::vector<int> ghost;
    for (int v : D)
      for (int jj = G[l].ptr[v]; jj < G[l].ptr[v + 1]; ++jj) {
        int u = G[l].col[jj];
        if (sc.a.mark[u] != e) { sc.a.mark[u] = e; ghost.push_back(u); }
      }
    std::sort(ghost.begin(), ghost.end());
    lv.nreal = (int)D.size();
    lv.gid = std::move(D);
    lv.gid.insert(lv.gid.end(), ghost.begin(), ghost.end());
    if (l < L) {
      seeds.clear();
      for (int i = 0; i < lv.nreal; ++i) {
        int g = lv.gid[i];
        if (H.cf[l][g] == 1) seeds.push_back(cmap[l][g]);
      }
    }
  }
}

// Local operators of one composite grid (Sections 4.1, 4.2).
void build_local_ops(const ProblemHost &P, CompGrid &cg, Scratch &sc) {
  const Hierarchy &H = P.H;
  const int L = H.L();
  Stamp *cur = &sc.a, *nxt = &sc.b;
  auto map_level = [&](Stamp &st, int l) {
    st.size(H.A[l].nrows);
    int e = st.next();
    const auto &g = cg.lv[l].gid;
    for (int i = 0; i < (int)g.size(); ++i) { st.mark[g[i]] = e; st.idx[g[i]] = i; }
    return e;
  };
  int ecur = map_level(*cur, 0);
  for (int l = 0; l <= L; ++l) {
    CompLevel &lv = cg.lv[l];
    const Csr &A = H.A[l];
    const int nb = lv.nbar();
    lv.A.nrows = lv.A.ncols = nb;
    lv.A.ptr.assign(nb + 1, 0);
    for (int i = 0; i < nb; ++i) {
      int g = lv.gid[i];
      for (int jj = A.ptr[g]; jj < A.ptr[g + 1]; ++jj) {
        int c = A.col[jj];
        if (cur->mark[c] != ecur) continue;  // only ghost rows can reach outside Dbar
        int li = cur->idx[c];
        if (i < lv.nreal || li < lv.nreal) { lv.A.col.push_back(li); lv.A.val.push_back(A.val[jj]); }
      }
      lv.A.ptr[i + 1] = (int)lv.A.col.size();
    }
    lv.dinv.resize(lv.nreal);
    for (int i = 0; i < lv.nreal; ++i) lv.dinv[i] = 1.0 / H.l1[l][lv.gid[i]];
    if (l < L) {
      int enxt = map_level(*nxt, l + 1);
      const Csr &Pg = H.P[l];
      lv.P.nrows = nb;
      lv.P.ncols = cg.lv[l + 1].nbar();
      lv.P.ptr.assign(nb + 1, 0);
      for (int i = 0; i < nb; ++i) {
        int g = lv.gid[i];
        for (int jj = Pg.ptr[g]; jj < Pg.ptr[g + 1]; ++jj) {
          int c = Pg.col[jj];
          if (nxt->mark[c] == enxt) { lv.P.col.push_back(nxt->idx[c]); lv.P.val.push_back(Pg.val[jj]); }
          else lv.omissions++;
        }
        lv.P.ptr[i + 1] = (int)lv.P.col.size();
      }
      std::swap(cur, nxt);
      ecur = enxt;
    }
  }
  // owned points are real level-0 points; local index = position in the sorted real list
  const auto &g0 = cg.lv[0].gid;
  cg.owned_local.resize(cg.owned_gid.size());
  for (size_t k = 0; k < cg.owned_gid.size(); ++k)
    cg.owned_local[k] = (int)(std::lower_bound(g0.begin(), g0.begin() + cg.lv[0].nreal, cg.owned_gid[k]) - g0.begin());
}

}  // namespace

namespace {

// Copies and validates every input problem and builds its AMG hierarchy.
int setup_hierarchies(const std::vector<ProblemInput> &in, double theta, int max_coarse, int max_levels, Setup &S,
                      std::string &err) {
  S.theta = theta;
  S.max_coarse = max_coarse;
  S.max_levels = max_levels;
  const int nprob = (int)in.size();
  if (nprob <= 0) { err = "no problems"; return ST_EINVAL; }
  if (!(theta > 0.0 && theta <= 1.0) || max_coarse < 1 || max_levels < 2) { err = "bad AMG parameters"; return ST_EINVAL; }
  for (int q = 0; q < nprob; ++q) {
    int st = validate(in[q], max_coarse, err);
    if (st) { err = "problem " + std::to_string(q) + ": " + err; return st; }
  }
  double t0 = now_s();
  S.probs.resize(nprob);
  std::vector<int> status(nprob, ST_OK);
  std::vector<std::string> errs(nprob);
  for (int q = 0; q < nprob; ++q) {
    ProblemHost &P = S.probs[q];
    P.n = in[q].n;
    P.nparts = in[q].nparts;
    P.eta = in[q].eta;
    if (in[q].n_etas > 0) P.etas.assign(in[q].etas, in[q].etas + in[q].n_etas);
    P.A0.nrows = P.A0.ncols = P.n;
    P.A0.ptr.assign(in[q].rowptr, in[q].rowptr + P.n + 1);
    long long nnz = P.A0.ptr[P.n];
    P.A0.col.assign(in[q].colind, in[q].colind + nnz);
    P.A0.val.assign(in[q].val, in[q].val + nnz);
    P.part.assign(in[q].part, in[q].part + P.n);
    // exact numerical symmetry (the adjoint then reuses the forward operators)
    Csr T = transpose(P.A0);
    P.symmetric = (T.col == P.A0.col && T.val == P.A0.val);
  }
  // problems are independent: build the hierarchies in parallel when batched
  parallel_items(nprob, [&](int q, int) {
    status[q] = build_hierarchy(S.probs[q], theta, max_coarse, max_levels, S.coarsen, S.interp, S.interp_max, errs[q]);
  });
  for (int q = 0; q < nprob; ++q)
    if (status[q]) { err = "problem " + std::to_string(q) + ": " + errs[q]; return status[q]; }
  S.times.hierarchy = now_s() - t0;
  return ST_OK;
}

// Composite grids of every subdomain (when `composite`) and the batched
// layouts of every level, from the problems' hierarchies.  Without composite
// grids only the global layouts (V-cycle) are filled.
int setup_layouts(Setup &S, bool composite, std::string &err) {
  const int nprob = (int)S.probs.size();
  // ---- composite grids
  double t0 = now_s();
  int maxL = 0;
  for (auto &P : S.probs) maxL = std::max(maxL, P.H.L());
  for (int q = 0; q < nprob && composite; ++q)
    for (int p = 0; p < S.probs[q].nparts; ++p) {
      S.probs[q].grids.push_back((int)S.grids.size());
      CompGrid cg;
      cg.prob = q;
      cg.p = p;
      S.grids.push_back(std::move(cg));
    }
  std::vector<std::vector<Csr>> graphs(nprob);
  std::vector<std::vector<std::vector<int>>> cmaps(nprob);
  parallel_items(nprob, [&](int q, int) {
    const Hierarchy &H = S.probs[q].H;
    for (int l = 0; l <= H.L(); ++l) graphs[q].push_back(adjacency(H.A[l]));
    for (int l = 0; l < H.L(); ++l) {
      std::vector<int> cm(H.A[l].nrows, -1);
      int c = 0;
      for (int i = 0; i < H.A[l].nrows; ++i)
        if (H.cf[l][i] == 1) cm[i] = c++;
      cmaps[q].push_back(std::move(cm));
    }
  });
  int nt = n_threads();
  std::vector<Scratch> scratch(nt);
  parallel_items((int)S.grids.size(), [&](int g, int t) {
    CompGrid &cg = S.grids[g];
    const ProblemHost &P = S.probs[cg.prob];
    build_sets(P, graphs[cg.prob], cmaps[cg.prob], cg.p, cg, scratch[t]);
    build_local_ops(P, cg, scratch[t]);
  });
  graphs.clear();
  cmaps.clear();
  S.omissions = 0;
  S.composite_real_nnz = S.global_nnz = S.composite_rows = S.composite_real_rows = 0;
  for (auto &P : S.probs)
    for (auto &A : P.H.A) S.global_nnz += A.nnz();
  for (auto &cg : S.grids) {
    const Hierarchy &H = S.probs[cg.prob].H;
    for (int l = 0; l <= H.L(); ++l) {
      const CompLevel &lv = cg.lv[l];
      S.omissions += lv.omissions;
      S.composite_rows += lv.nbar();
      S.composite_real_rows += lv.nreal;
      for (int i = 0; i < lv.nreal; ++i) S.composite_real_nnz += H.A[l].ptr[lv.gid[i] + 1] - H.A[l].ptr[lv.gid[i]];
    }
  }
  S.times.composite = now_s() - t0;

  // ---- batched layouts
  t0 = now_s();
  S.dense_off.assign(nprob, 0);
  int doff = 0;
  for (int q = 0; q < nprob; ++q) {
    S.dense_off[q] = doff;
    doff += (int)S.probs[q].H.Ac.size();
    S.dense_A.insert(S.dense_A.end(), S.probs[q].H.Ac.begin(), S.probs[q].H.Ac.end());
    S.dense_inv.insert(S.dense_inv.end(), S.probs[q].H.Ac_inv.begin(), S.probs[q].H.Ac_inv.end());
  }
  const int ng = (int)S.grids.size();
  S.lv.assign(maxL + 1, BatchLevel());
  // composite offsets per level: off[g] for normal real, ghost, or coarse rows
  std::vector<std::vector<int>> roff(maxL + 1, std::vector<int>(ng, -1)), goff = roff, coff = roff;
  std::vector<std::vector<int>> gro(maxL + 1, std::vector<int>(nprob, -1)), gco = gro;
  for (int l = 0; l <= maxL; ++l) {
    BatchLevel &B = S.lv[l];
    int r = 0, gh = 0, c = 0;
    for (int g = 0; g < ng; ++g) {
      int L = S.probs[S.grids[g].prob].H.L();
      const CompLevel *lv = l <= L ? &S.grids[g].lv[l] : nullptr;
      if (!lv) continue;
      // a grid with no points on a level above its coarsest (possible with
      // small paddings: D_l empty, hence every deeper level but the coarsest)
      // keeps one empty ghost row there, so the padding entries of its rows
      // on the neighbouring levels have a column of their own grid
      if (L > l) { roff[l][g] = r; r += lv->nreal; goff[l][g] = gh; gh += std::max(1, lv->nbar()) - lv->nreal; }
      else { coff[l][g] = c; c += lv->nbar(); }
    }
    B.NRn = r;
    // ghost rows start on a 64-row boundary: no slice mixes real and ghost rows
    // (rows [NRn, NRa) belong to no grid and hold no entries)
    B.NRa = (r + 63) / 64 * 64;
    B.NBn = B.NRa + gh;
    B.NB = B.NBn + c;
    int gn = 0, gc = 0;
    for (int q = 0; q < nprob; ++q) {
      int L = S.probs[q].H.L();
      if (l > L) continue;
      if (L > l) { gro[l][q] = gn; gn += S.probs[q].H.A[l].nrows; }
      else { gco[l][q] = gc; gc += S.probs[q].H.A[l].nrows; }
    }
    B.GNn = gn;
    B.GN = gn + gc;
    if ((long long)B.NB >= std::numeric_limits<int>::max() / 2) throw std::length_error("level too large");
  }
  // Row order within each grid's real and ghost ranges.  Real rows: CF
  // ordering puts C-points first (each class in local order).  On levels
  // with grouped rows (mean composite row length above one lane's share) and
  // a sort window > 0, rows are then sorted by decreasing length within
  // consecutive windows of that many rows (never across the C/F boundary),
  // so sliced-ELL slices hold rows of similar length; ghost rows likewise.
  // Jacobi sweeps and mat-vecs do not depend on row order (up to the
  // rounding of grouped rows: with wide steps, which lane adds which entry
  // depends on the step count of the row's slice).
  const int sortw = S.sort_window;
  std::vector<char> sort_lv(maxL + 1, 0);
  for (int l = 0; l <= maxL && sortw > 0; ++l) {
    long long nz = 0;
    for (int g = 0; g < ng; ++g)
      if (roff[l][g] >= 0) nz += S.grids[g].lv[l].A.nnz();
    sort_lv[l] = S.lv[l].NBn > 0 && (double)nz / S.lv[l].NBn > AMGDD_LANE_ONE;
  }
  std::vector<std::vector<std::vector<int>>> rpos(maxL + 1), gpos(maxL + 1);
  if (S.cf || sortw > 0) {
    for (int l = 0; l <= maxL; ++l) {
      rpos[l].resize(ng);
      gpos[l].resize(ng);
    }
    parallel_items(ng, [&](int g, int) {
      const Hierarchy &H = S.probs[S.grids[g].prob].H;
      for (int l = 0; l < H.L(); ++l) {
        const CompLevel &lv = S.grids[g].lv[l];
        auto len = [&](int i) { return lv.A.ptr[i + 1] - lv.A.ptr[i]; };
        // windows of `ord` positions [b, e) sorted by decreasing row length
        auto sort_windows = [&](std::vector<int> &ord, int b, int e) {
          if (sortw <= 0 || !sort_lv[l]) return;
          for (int w = b; w < e; w += sortw)
            std::stable_sort(ord.begin() + w, ord.begin() + std::min(e, w + sortw),
                             [&](int x, int y) { return len(x) > len(y); });
        };
        std::vector<int> ord;
        ord.reserve(lv.nreal);
        int nc = lv.nreal;
        if (S.cf) {
          for (int pass = 0; pass < 2; ++pass) {
            for (int i = 0; i < lv.nreal; ++i)
              if ((H.cf[l][lv.gid[i]] == 1) == (pass == 0)) ord.push_back(i);
            if (pass == 0) nc = (int)ord.size();
          }
        } else {
          for (int i = 0; i < lv.nreal; ++i) ord.push_back(i);
        }
        sort_windows(ord, 0, nc);
        sort_windows(ord, nc, lv.nreal);
        std::vector<int> &pos = rpos[l][g];
        pos.resize(lv.nreal);
        for (int k = 0; k < lv.nreal; ++k) pos[ord[k]] = k;
        if (sortw > 0 && sort_lv[l]) {
          const int ngh = lv.nbar() - lv.nreal;
          std::vector<int> go(ngh);
          for (int k = 0; k < ngh; ++k) go[k] = lv.nreal + k;
          sort_windows(go, 0, ngh);
          std::vector<int> &gp = gpos[l][g];
          gp.resize(ngh);
          for (int k = 0; k < ngh; ++k) gp[go[k] - lv.nreal] = k;
        }
      }
    });
  }
  auto bidx = [&](int g, int l, int i) -> int {
    const CompLevel &lv = S.grids[g].lv[l];
    if (roff[l][g] >= 0) {
      if (i < lv.nreal) return roff[l][g] + (rpos[l].empty() ? i : rpos[l][g][i]);
      return S.lv[l].NRa + goff[l][g] + (gpos[l].empty() || gpos[l][g].empty() ? i - lv.nreal : gpos[l][g][i - lv.nreal]);
    }
    return S.lv[l].NBn + coff[l][g] + i;
  };
  auto gbidx = [&](int q, int l, int i) -> int {
    if (gro[l][q] >= 0) return gro[l][q] + i;
    return S.lv[l].GNn + gco[l][q] + i;
  };
  vlog("pack: offsets", t0);
  // lanes per row of every level, from the mean row length of A_l (of the
  // restriction rows on a level that only holds coarsest grids); the fine
  // global level keeps one lane per row
  // Interpolation rows (a few entries) get their own lane count.
  for (int l = 0; l <= maxL; ++l) {
    long long nzA = 0, nzR = 0, nzP = 0;
    for (int g = 0; g < ng; ++g) {
      if (roff[l][g] >= 0) {
        nzA += S.grids[g].lv[l].A.nnz();
        nzP += S.grids[g].lv[l].P.nnz();
      }
      if (l > 0 && (roff[l][g] >= 0 || coff[l][g] >= 0)) nzR += S.grids[g].lv[l - 1].P.nnz();
    }
    BatchLevel &B = S.lv[l];
    const double tgt = S.comp_lane_target;
    B.lg = B.NBn > 0 ? lanes_log2((double)nzA / B.NBn, tgt) : (B.NB > 0 ? lanes_log2((double)nzR / B.NB, tgt) : 0);
    B.plg = B.NBn > 0 ? lanes_log2((double)nzP / B.NBn, tgt) : 0;
    long long nzG = 0, nzGP = 0;
    for (int q = 0; q < nprob; ++q) {
      if (l <= S.probs[q].H.L()) nzG += S.probs[q].H.A[l].nnz();
      if (l < S.probs[q].H.L()) nzGP += S.probs[q].H.P[l].nnz();
    }
    B.glg = (l == 0 || B.GN == 0) ? 0 : lanes_log2((double)nzG / B.GN, AMGDD_GLANE_TARGET);
    B.gplg = B.GNn > 0 ? lanes_log2((double)nzGP / B.GNn, AMGDD_GLANE_TARGET) : 0;
  }
  for (int l = 0; l <= maxL; ++l) {
    BatchLevel &B = S.lv[l];
    double tp = now_s();
    std::vector<int> normal;
    for (int g = 0; g < ng; ++g) {
      if (roff[l][g] >= 0) normal.push_back(g);
      else if (coff[l][g] >= 0) {
        const CompLevel &lv = S.grids[g].lv[l];
        B.cg_row0.push_back(B.NBn + coff[l][g]);
        B.cg_n.push_back(lv.nbar());
        B.cg_dense.push_back(S.dense_off[S.grids[g].prob]);
      }
    }
    const int nn = (int)normal.size();
    // ---- composite A and P rows of normal grids, dinv, gather sources
    SellBuilder bA, bP;
    bA.init(B.NBn, B.lg, S.comp_step_log2);
    bP.init(B.NBn, B.plg, S.comp_step_log2);
    B.dinv.assign(B.NRn, 0.0);
    B.gsrc.assign(B.NB, -1);
    parallel_items(ng, [&](int g, int) {
      const int q = S.grids[g].prob;
      if (roff[l][g] >= 0) {
        const CompLevel &lv = S.grids[g].lv[l];
        for (int i = 0; i < lv.nbar(); ++i) {
          int row = bidx(g, l, i);
          bA.len[row] = lv.A.ptr[i + 1] - lv.A.ptr[i];
          bP.len[row] = lv.P.ptr[i + 1] - lv.P.ptr[i];
          if (i < lv.nreal) { B.dinv[row] = lv.dinv[i]; B.gsrc[row] = gbidx(q, l, lv.gid[i]); }
        }
      } else if (coff[l][g] >= 0) {
        const CompLevel &lv = S.grids[g].lv[l];
        for (int i = 0; i < lv.nbar(); ++i) B.gsrc[B.NBn + coff[l][g] + i] = gbidx(q, l, lv.gid[i]);
      }
    });
    bA.shape();
    bP.shape();
    parallel_items(nn, [&](int k, int) {
      int g = normal[k];
      const CompLevel &lv = S.grids[g].lv[l];
      for (int i = 0; i < lv.nbar(); ++i) {
        int row = bidx(g, l, i);
        int kk = 0;
        for (int jj = lv.A.ptr[i]; jj < lv.A.ptr[i + 1]; ++jj) bA.put(row, kk++, bidx(g, l, lv.A.col[jj]), lv.A.val[jj]);
        bA.pad(row, bidx(g, l, 0));
        kk = 0;
        for (int jj = lv.P.ptr[i]; jj < lv.P.ptr[i + 1]; ++jj) bP.put(row, kk++, bidx(g, l + 1, lv.P.col[jj]), lv.P.val[jj]);
        bP.pad(row, bidx(g, l + 1, 0));
      }
      if (lv.nbar() == 0) {
        // the empty ghost row of a grid without points on this level
        const int row = bidx(g, l, 0);
        bA.pad(row, row);
        bP.pad(row, bidx(g, l + 1, 0));
      }
    });
    B.nnzA_r = bA.nnz_rows(0, B.NRn);
    B.nnzA = bA.nnz_rows(0, B.NBn);
    if (S.cf) {
      B.cls.assign(B.NRn, 0);
      for (int g : normal) {
        const CompLevel &lv = S.grids[g].lv[l];
        const Hierarchy &H = S.probs[S.grids[g].prob].H;
        for (int i = 0; i < lv.nreal; ++i) {
          const int8_t c = H.cf[l][lv.gid[i]];
          B.cls[bidx(g, l, i)] = c;
          if (c == 1) {
            B.NRc++;
            B.nnzA_c += lv.A.ptr[i + 1] - lv.A.ptr[i];
          }
        }
      }
    }
    B.nnzP = bP.nnz_rows(0, B.NBn);
    if (S.tight && B.NBn > 0) {
      // interpolation rows in an order of their own for the level-synchronous
      // pass (C rows inject one value, F rows interpolate from several)
      std::vector<int> own(B.NBn, 0);
      parallel_items(nn, [&](int k, int) {
        const int g = normal[k];
        for (int i = 0; i < std::max(1, S.grids[g].lv[l].nbar()); ++i) own[bidx(g, l, i)] = bidx(g, l + 1, 0);
      });
      B.Pt = permuted_layout(bP, B.NBn, B.plg, S.comp_step_log2, S.tight_window, own, B.pperm);
    }
    B.A = bA.take();
    B.P = bP.take();
    vlog("pack: composite A, P", tp);
    // ---- R_l = P_l^T (block-diagonal: one transpose per grid), rows of level l+1
    if (l < maxL) {
      BatchLevel &Bn = S.lv[l + 1];
      SellBuilder bR;
      bR.init(Bn.NB, Bn.lg, S.comp_step_log2);
      std::vector<Csr> Rl(nn);
      parallel_items(nn, [&](int k, int) {
        int g = normal[k];
        const CompLevel &lv = S.grids[g].lv[l];
        Rl[k] = transpose(lv.P);
        Rl[k].nrows = S.grids[g].lv[l + 1].nbar();
        Rl[k].ptr.resize(Rl[k].nrows + 1, Rl[k].ptr.back());
        for (int J = 0; J < Rl[k].nrows; ++J) bR.len[bidx(g, l + 1, J)] = Rl[k].ptr[J + 1] - Rl[k].ptr[J];
      });
      bR.shape();
      parallel_items(nn, [&](int k, int) {
        int g = normal[k];
        const Csr &R = Rl[k];
        for (int J = 0; J < R.nrows; ++J) {
          int row = bidx(g, l + 1, J);
          int kk = 0;
          for (int jj = R.ptr[J]; jj < R.ptr[J + 1]; ++jj) bR.put(row, kk++, bidx(g, l, R.col[jj]), R.val[jj]);
          bR.pad(row, bidx(g, l, 0));
        }
        if (R.nrows == 0) bR.pad(bidx(g, l + 1, 0), bidx(g, l, 0));
      });
      Bn.nnzR_n = bR.nnz_rows(0, Bn.NBn);
      Bn.nnzR = bR.nnz_rows(0, Bn.NB);
      if (S.tight && Bn.NBn > 0) {
        // restriction rows of the normal grids in an order and a lane count
        // of their own, for a restriction pass of its own (the operator's
        // rows are several times longer and differently distributed)
        std::vector<int> own(Bn.NBn, 0);
        parallel_items(nn, [&](int k, int) {
          const int g = normal[k];
          if (roff[l + 1][g] < 0) return;
          for (int J = 0; J < std::max(1, S.grids[g].lv[l + 1].nbar()); ++J) own[bidx(g, l + 1, J)] = bidx(g, l, 0);
        });
        Bn.rlg = lanes_log2((double)Bn.nnzR_n / Bn.NBn, S.comp_lane_target);
        Bn.Rt = permuted_layout(bR, Bn.NBn, Bn.rlg, S.comp_step_log2, S.tight_window_r, own, Bn.rperm);
      }
      Bn.R = bR.take();
    }
    // local operators of this level are no longer needed
    parallel_items(nn, [&](int k, int) {
      CompLevel &lv = S.grids[normal[k]].lv[l];
      free_csr(lv.A);
      free_csr(lv.P);
    });
    vlog("pack: composite R", tp);
    tp = now_s();
    // ---- global level l over problems
    SellBuilder bGA, bGP;
    bGA.init(B.GN, B.glg, S.step_log2);
    bGP.init(B.GNn, B.gplg, S.step_log2);
    B.gdinv.assign(B.GNn, 0.0);
    B.prob_row0.assign(nprob, -1);
    for (int q = 0; q < nprob; ++q) {
      const Hierarchy &H = S.probs[q].H;
      if (l > H.L()) continue;
      B.prob_row0[q] = gbidx(q, l, 0);
      if (l == H.L()) {
        B.gc_row0.push_back(gbidx(q, l, 0));
        B.gc_n.push_back(H.A[l].nrows);
        B.gc_dense.push_back(S.dense_off[q]);
      }
    }
    parallel_items(nprob, [&](int q, int) {
      const Hierarchy &H = S.probs[q].H;
      if (l > H.L()) return;
      int base = gbidx(q, l, 0);
      const Csr &Al = H.A[l];
      for (int i = 0; i < Al.nrows; ++i) bGA.len[base + i] = Al.ptr[i + 1] - Al.ptr[i];
      if (l < H.L())
        for (int i = 0; i < Al.nrows; ++i) {
          bGP.len[base + i] = H.P[l].ptr[i + 1] - H.P[l].ptr[i];
          B.gdinv[base + i] = 1.0 / H.l1[l][i];
        }
    });
    bGA.shape();
    bGP.shape();
    parallel_items(nprob, [&](int q, int) {
      const Hierarchy &H = S.probs[q].H;
      if (l > H.L()) return;
      int base = gbidx(q, l, 0);
      const Csr &Al = H.A[l];
      for (int i = 0; i < Al.nrows; ++i) {
        int kk = 0;
        for (int jj = Al.ptr[i]; jj < Al.ptr[i + 1]; ++jj) bGA.put(base + i, kk++, base + Al.col[jj], Al.val[jj]);
        bGA.pad(base + i, base);
      }
      if (l < H.L()) {
        int cbase = gbidx(q, l + 1, 0);
        const Csr &Pl = H.P[l];
        for (int i = 0; i < Al.nrows; ++i) {
          int kk = 0;
          for (int jj = Pl.ptr[i]; jj < Pl.ptr[i + 1]; ++jj) bGP.put(base + i, kk++, cbase + Pl.col[jj], Pl.val[jj]);
          bGP.pad(base + i, cbase);
        }
      }
    });
    B.nnzGA_n = bGA.nnz_rows(0, B.GNn);
    B.nnzGA = bGA.nnz_rows(0, B.GN);
    if (S.cf) {
      B.gcls.assign(B.GNn, 0);
      for (int q = 0; q < nprob; ++q) {
        const Hierarchy &H = S.probs[q].H;
        if (l >= H.L()) continue;
        const int base = gbidx(q, l, 0);
        for (int i = 0; i < H.A[l].nrows; ++i) {
          B.gcls[base + i] = H.cf[l][i];
          if (H.cf[l][i] == 1) {
            B.GNc++;
            B.nnzGA_c += H.A[l].ptr[i + 1] - H.A[l].ptr[i];
          }
        }
      }
    }
    B.nnzGP = bGP.nnz_rows(0, B.GNn);
    B.GA = bGA.take();
    B.GP = bGP.take();
    if (l < maxL) {
      // R_l = P_l^T is stored in the hierarchy; rows = level l+1
      BatchLevel &Bn = S.lv[l + 1];
      SellBuilder bGR;
      bGR.init(Bn.GN, Bn.glg, S.step_log2);
      parallel_items(nprob, [&](int q, int) {
        const Hierarchy &H = S.probs[q].H;
        if (l >= H.L()) return;
        int cbase = gbidx(q, l + 1, 0);
        for (int J = 0; J < H.R[l].nrows; ++J) bGR.len[cbase + J] = H.R[l].ptr[J + 1] - H.R[l].ptr[J];
      });
      bGR.shape();
      parallel_items(nprob, [&](int q, int) {
        const Hierarchy &H = S.probs[q].H;
        if (l >= H.L()) return;
        int base = gbidx(q, l, 0), cbase = gbidx(q, l + 1, 0);
        const Csr &R = H.R[l];
        for (int J = 0; J < R.nrows; ++J) {
          int kk = 0;
          for (int jj = R.ptr[J]; jj < R.ptr[J + 1]; ++jj) bGR.put(cbase + J, kk++, base + R.col[jj], R.val[jj]);
          bGR.pad(cbase + J, base);
        }
      });
      Bn.nnzGR_n = bGR.nnz_rows(0, Bn.GNn);
      Bn.nnzGR = bGR.nnz_rows(0, Bn.GN);
      Bn.GR = bGR.take();
    }
    vlog("pack: global", tp);
  }
  vlog("pack: levels", t0);
  if (verbose())
    for (int l = 0; l <= maxL; ++l) {
      const BatchLevel &B = S.lv[l];
      std::fprintf(stderr,
                   "[amgdd setup] level %d rows %d/%d/%d G %d/%d  A %lld/%lld  P %lld/%lld (reordered %lld, G %d)  R "
                   "%lld/%lld (normal rows %lld/%lld, reordered %lld, G %d)\n",
                   l, B.NRn, B.NBn, B.NB, 1 << B.lg, 1 << B.glg, B.nnzA, B.A.entries(), B.nnzP, B.P.entries(),
                   B.Pt.entries(), 1 << B.plg, B.nnzR, B.R.entries(), B.nnzR_n,
                   B.R.sptr.empty() ? 0LL : (long long)B.R.sptr[(size_t)B.NBn >> (6 - B.R.lg)], B.Rt.entries(),
                   1 << B.rlg);
    }
  for (int l = 0; l <= maxL; ++l) {
    const BatchLevel &B = S.lv[l];
    const int nbn = l < maxL ? S.lv[l + 1].NB : 0, nbp = l > 0 ? S.lv[l - 1].NB : 0;
    const int gnn = l < maxL ? S.lv[l + 1].GN : 0, gnp = l > 0 ? S.lv[l - 1].GN : 0;
    bool ok = sell_in_bounds(B.A, B.NBn, B.NB) && sell_in_bounds(B.P, B.NBn, std::max(nbn, 1)) &&
              sell_in_bounds(B.GA, B.GN, B.GN) && sell_in_bounds(B.GP, B.GNn, std::max(gnn, 1));
    if (l > 0) ok = ok && sell_in_bounds(B.R, B.NB, nbp) && sell_in_bounds(B.GR, B.GN, gnp);
    if (!B.pperm.empty()) ok = ok && sell_in_bounds(B.Pt, B.NBn, std::max(nbn, 1));
    if (!B.rperm.empty()) ok = ok && sell_in_bounds(B.Rt, B.NBn, nbp);
    if (!ok) { err = "internal: batched layout check failed on level " + std::to_string(l); return ST_EINVAL; }
  }
  {
    // owners of every composite / global row, per level
    std::vector<std::vector<int>> cown(maxL + 1), gown(maxL + 1);
    for (int l = 0; l <= maxL; ++l) {
      cown[l].assign(S.lv[l].NB, -1);
      gown[l].assign(S.lv[l].GN, -1);
    }
    for (int g = 0; g < ng; ++g)
      for (int l = 0; l <= S.probs[S.grids[g].prob].H.L(); ++l)
        for (int i = 0; i < std::max(1, S.grids[g].lv[l].nbar()); ++i) cown[l][bidx(g, l, i)] = g;
    for (int q = 0; q < nprob; ++q)
      for (int l = 0; l <= S.probs[q].H.L(); ++l)
        for (int i = 0; i < S.probs[q].H.A[l].nrows; ++i) gown[l][gbidx(q, l, i)] = q;
    for (int l = 0; l <= maxL; ++l) {
      const BatchLevel &B = S.lv[l];
      bool ok = sell_block_diagonal(B.A, cown[l], cown[l]) && sell_block_diagonal(B.GA, gown[l], gown[l]);
      if (l < maxL) ok = ok && sell_block_diagonal(B.P, cown[l], cown[l + 1]) && sell_block_diagonal(B.GP, gown[l], gown[l + 1]);
      if (l > 0) ok = ok && sell_block_diagonal(B.R, cown[l], cown[l - 1]) && sell_block_diagonal(B.GR, gown[l], gown[l - 1]);
      // the reordered layouts: owner of position k = owner of the row it holds
      if (!B.pperm.empty() || !B.rperm.empty()) {
        std::vector<int> po(B.pperm.size()), ro(B.rperm.size());
        for (size_t k = 0; k < po.size(); ++k) po[k] = cown[l][B.pperm[k]];
        for (size_t k = 0; k < ro.size(); ++k) ro[k] = cown[l][B.rperm[k]];
        if (!B.pperm.empty()) ok = ok && sell_block_diagonal(B.Pt, po, cown[l + 1]);
        if (!B.rperm.empty()) ok = ok && sell_block_diagonal(B.Rt, ro, cown[l - 1]);
      }
      if (!ok) { err = "internal: batched layout is not block-diagonal on level " + std::to_string(l); return ST_EINVAL; }
    }
    // LDS bands of the composite operators (level-synchronous passes)
    const double tb = now_s();
    if (S.bands)
      for (int l = 0; l <= maxL; ++l) {
        BatchLevel &B = S.lv[l];
        if (B.Rt.entries() > 0) {
          // the reordered restriction gathers from the finer level
          B.rband_max = build_bands(B.Rt, S.band_cap, kTileSlicesR);
          if (!bands_valid(B.Rt, S.band_cap, kTileSlicesR)) { err = "internal: LDS band check failed on level " + std::to_string(l); return ST_EINVAL; }
        }
        if (B.A.entries() == 0) continue;
        // the largest tile (tile_slices_max halved down to kTileSlicesS
        // slices) that leaves the level wide_tiles_min tiles, or a smaller one
        // when some tile's band would not fit the cap
        const long long nsl = (long long)B.A.sptr.size() - 1;
        int ts = kTileSlicesS;
        for (int c = S.tile_slices_max; c > kTileSlicesS; c >>= 1)
          if (nsl >= (long long)c * S.wide_tiles_min) {
            ts = c;
            break;
          }
        B.band_max = build_bands(B.A, S.band_cap, ts);
        while (B.A.tiles.empty() && ts > kTileSlicesS) {
          ts >>= 1;
          B.band_max = build_bands(B.A, S.band_cap, ts);
        }
        if (!bands_valid(B.A, S.band_cap, ts)) { err = "internal: LDS band check failed on level " + std::to_string(l); return ST_EINVAL; }
        if (verbose()) {
          long long nb = 0, sum = 0;
          const int nt = (int)B.A.tiles.size() / (2 * kBandWindows);
          for (int t = 0; t < nt; ++t)
            if (const int n = B.A.tiles[2 * kBandWindows * t + 2 * kBandWindows - 1]) { ++nb; sum += n; }
          std::fprintf(stderr, "[amgdd setup] level %d LDS bands: %lld of %d tiles of %d slices, %.2f values per row, largest %d (R: %d)\n",
                       l, nb, nt, ts, nb ? (double)sum / nb / ((64 * ts) >> B.A.lg) : 0.0, B.band_max, B.rband_max);
        }
      }
    vlog("pack: LDS bands", tb);
    // 16-bit column indices where every slice fits (checked by decoding)
    if (S.compress) {
      std::vector<char> done(6 * (maxL + 1), 0);
      for (int k = 0; k < 6 * (maxL + 1); ++k) {
        const int l = k / 6, m = k % 6;
        BatchLevel &B = S.lv[l];
        if (m == 0) done[k] = compress_columns(B.A, cown[l], cown[l]);
        if (m == 1 && l < maxL) done[k] = compress_columns(B.P, cown[l], cown[l + 1]);
        if (m == 2 && l > 0) done[k] = compress_columns(B.R, cown[l], cown[l - 1]);
        if (m == 3) done[k] = compress_columns(B.GA, gown[l], gown[l]);
        if (m == 4 && l < maxL) done[k] = compress_columns(B.GP, gown[l], gown[l + 1]);
        if (m == 5 && l > 0) done[k] = compress_columns(B.GR, gown[l], gown[l - 1]);
      }
      for (int l = 0; l <= maxL; ++l) {
        BatchLevel &B = S.lv[l];
        if (!B.pperm.empty()) {
          std::vector<int> po(B.pperm.size());
          for (size_t k = 0; k < po.size(); ++k) po[k] = cown[l][B.pperm[k]];
          const bool okp = compress_columns(B.Pt, po, cown[l + 1]);
          if (verbose()) std::fprintf(stderr, "[amgdd setup] level %d reordered P 16-bit columns %d\n", l, (int)okp);
        }
        if (!B.rperm.empty()) {
          std::vector<int> ro(B.rperm.size());
          for (size_t k = 0; k < ro.size(); ++k) ro[k] = cown[l][B.rperm[k]];
          const bool okr = compress_columns(B.Rt, ro, cown[l - 1]);
          if (verbose()) std::fprintf(stderr, "[amgdd setup] level %d reordered R 16-bit columns %d\n", l, (int)okr);
        }
      }
      if (verbose())
        for (int l = 0; l <= maxL; ++l)
          std::fprintf(stderr, "[amgdd setup] level %d 16-bit columns A %d P %d R %d GA %d GP %d GR %d\n", l, done[6 * l],
                       done[6 * l + 1], done[6 * l + 2], done[6 * l + 3], done[6 * l + 4], done[6 * l + 5]);
    }
  }
  // fine-vector offsets (every problem is normal on level 0, so problem order)
  S.prob_off.assign(nprob + 1, 0);
  for (int q = 0; q < nprob; ++q) S.prob_off[q + 1] = S.prob_off[q] + S.probs[q].n;
  if (composite) {
    S.owner.assign(S.prob_off[nprob], -1);
    for (int g = 0; g < ng; ++g) {
      const CompGrid &cg = S.grids[g];
      int base = S.prob_off[cg.prob];
      for (size_t k = 0; k < cg.owned_gid.size(); ++k) S.owner[base + cg.owned_gid[k]] = bidx(g, 0, cg.owned_local[k]);
    }
    for (int v : S.owner)
      if (v < 0) { err = "internal: fine point without owner"; return ST_EINVAL; }
  }
  // residual blocks of 256 rows that never straddle two problems
  S.prob_blk0.assign(nprob + 1, 0);
  for (int q = 0; q < nprob; ++q) {
    S.prob_blk0[q] = (int)S.blk_row0.size();
    for (int r = S.prob_off[q]; r < S.prob_off[q + 1]; r += 256) {
      S.blk_row0.push_back(r);
      S.blk_row1.push_back(std::min(r + 256, S.prob_off[q + 1]));
      S.blk_prob.push_back(q);
    }
  }
  S.prob_blk0[nprob] = (int)S.blk_row0.size();
  // per-grid row ranges for the per-grid (persistent) schedule
  const int nlv = maxL + 1;
  S.gl_rbeg.assign((size_t)ng * nlv, 0);
  S.gl_nreal.assign((size_t)ng * nlv, 0);
  S.gl_gbeg.assign((size_t)ng * nlv, 0);
  S.gl_nghost.assign((size_t)ng * nlv, 0);
  S.grid_L.assign(ng, 0);
  for (int g = 0; g < ng; ++g) {
    int L = S.probs[S.grids[g].prob].H.L();
    S.grid_L[g] = L;
    for (int l = 0; l <= L; ++l) {
      const CompLevel &lv = S.grids[g].lv[l];
      size_t k = (size_t)g * nlv + l;
      if (l < L) {
        S.gl_rbeg[k] = roff[l][g];
        S.gl_nreal[k] = lv.nreal;
        S.gl_gbeg[k] = S.lv[l].NRa + goff[l][g];
        S.gl_nghost[k] = std::max(1, lv.nbar()) - lv.nreal;
      } else {
        S.gl_rbeg[k] = S.lv[l].NBn + coff[l][g];
        S.gl_nreal[k] = lv.nbar();
      }
    }
  }
  S.times.pack = now_s() - t0;
  return ST_OK;
}

template <typename F>
int guarded(std::string &err, F &&f) {
  try {
    return f();
  } catch (const std::bad_alloc &) {
    err = "host allocation failed during setup";
    return ST_ENOMEM;
  } catch (const std::length_error &e) {
    err = std::string("layout too large: ") + e.what();
    return ST_EUNSUP;
  } catch (const std::logic_error &e) {
    err = std::string("internal: ") + e.what();
    return ST_EINVAL;
  }
}

}  // namespace

int build_setup(const std::vector<ProblemInput> &in, double theta, int max_coarse, int max_levels, Setup &S,
                std::string &err) {
  return guarded(err, [&]() {
    int st = setup_hierarchies(in, theta, max_coarse, max_levels, S, err);
    return st ? st : setup_layouts(S, true, err);
  });
}

// Hybrid AMG-DD (Algorithm 3, Section 3.1).  The level-lt problem of every
// problem that coarsens below lt is A_lt with levels lt..L of its hierarchy
// (classical coarsening depends on the matrix alone, so setting A_lt up from
// scratch would give the same levels) and the subdomains inherited along the
// C-points: a coarse point stays in the subdomain of the fine point it was
// chosen from (the per-level subdomains of Section 5).  Subdomains left without
// points on level lt are dropped: they would patch nothing.
int build_setup_hybrid(const std::vector<ProblemInput> &in, double theta, int max_coarse, int max_levels, int lt,
                       Setup &outer, Setup &inner, std::vector<int> &inner_of, std::vector<std::vector<int>> &part_map,
                       std::string &err) {
  return guarded(err, [&]() {
    if (lt < 1) { err = "hybrid level must be >= 1"; return (int)ST_EINVAL; }
    int st = setup_hierarchies(in, theta, max_coarse, max_levels, outer, err);
    if (st) return st;
    if ((st = setup_layouts(outer, false, err))) return st;
    const int nprob = (int)outer.probs.size();
    const bool cf = outer.cf;
    inner = Setup();
    inner.cf = cf;
    inner.coarsen = outer.coarsen;
    inner.interp = outer.interp;
    inner.interp_max = outer.interp_max;
    inner.compress = outer.compress;
    inner.step_log2 = outer.step_log2;
    inner.comp_step_log2 = outer.comp_step_log2;
    inner.sort_window = outer.sort_window;
    inner.comp_lane_target = outer.comp_lane_target;
    inner.theta = theta;
    inner.max_coarse = max_coarse;
    inner.max_levels = max_levels;
    inner_of.assign(nprob, -1);
    part_map.assign(nprob, std::vector<int>());
    double t0 = now_s();
    for (int q = 0; q < nprob; ++q) {
      const ProblemHost &O = outer.probs[q];
      part_map[q].assign(O.nparts, -1);
      if (O.H.L() <= lt) continue;
      std::vector<int> part = O.part;
      for (int l = 0; l < lt; ++l) {
        std::vector<int> next;
        next.reserve(O.H.A[l + 1].nrows);
        for (int i = 0; i < O.H.A[l].nrows; ++i)
          if (O.H.cf[l][i] == 1) next.push_back(part[i]);
        part = std::move(next);
      }
      std::vector<int> count(O.nparts, 0);
      for (int v : part) count[v]++;
      int np = 0;
      for (int p = 0; p < O.nparts; ++p)
        if (count[p] > 0) part_map[q][p] = np++;
      for (int &v : part) v = part_map[q][v];
      inner_of[q] = (int)inner.probs.size();
      inner.probs.emplace_back();
      ProblemHost &P = inner.probs.back();
      P.n = O.H.A[lt].nrows;
      P.nparts = np;
      P.eta = O.eta;
      if ((int)O.etas.size() > lt) P.etas.assign(O.etas.begin() + lt, O.etas.end());
      P.part = std::move(part);
      P.symmetric = O.symmetric;
      P.H.A.assign(O.H.A.begin() + lt, O.H.A.end());
      P.H.P.assign(O.H.P.begin() + lt, O.H.P.end());
      P.H.R.assign(O.H.R.begin() + lt, O.H.R.end());
      P.H.cf.assign(O.H.cf.begin() + lt, O.H.cf.end());
      P.H.l1.assign(O.H.l1.begin() + lt, O.H.l1.end());
      P.H.Ac = O.H.Ac;
      P.H.Ac_inv = O.H.Ac_inv;
    }
    inner.times.hierarchy = now_s() - t0;
    if (inner.probs.empty()) return (int)ST_OK;
    return setup_layouts(inner, true, err);
  });
}

// Transposed hierarchy for the adjoint A^T lambda = g.  With R_l = P_l^T and
// A_{l+1} = R_l A_l P_l (Section 2), A_{l+1}^T = R_l A_l^T P_l: the same C/F
// splittings, P_l and R_l form a Galerkin hierarchy for A^T whose operators are
// the transposes A_l^T; its l1-Jacobi diagonals are the row sums of |A_l^T|
// and its coarsest solve uses the inverse of A_L^T.  Composite sets depend on
// the undirected graph of A_l only, which A_l^T shares, so every composite
// grid has the forward one's points; its local operators are rows of A_l^T.
int build_setup_transposed(const Setup &F, bool composite, Setup &T, std::string &err) {
  return guarded(err, [&]() {
    double t0 = now_s();
    T = Setup();
    T.theta = F.theta;
    T.max_coarse = F.max_coarse;
    T.max_levels = F.max_levels;
    T.cf = F.cf;
    T.compress = F.compress;
    T.step_log2 = F.step_log2;
    T.comp_step_log2 = F.comp_step_log2;
    T.sort_window = F.sort_window;
    T.comp_lane_target = F.comp_lane_target;
    T.coarsen = F.coarsen;
    T.interp = F.interp;
    T.interp_max = F.interp_max;
    const int nprob = (int)F.probs.size();
    T.probs.resize(nprob);
    std::vector<int> status(nprob, ST_OK);
    parallel_items(nprob, [&](int q, int) {
      const ProblemHost &O = F.probs[q];
      ProblemHost &P = T.probs[q];
      P.n = O.n;
      P.nparts = O.nparts;
      P.eta = O.eta;
      P.etas = O.etas;
      P.part = O.part;
      P.symmetric = O.symmetric;
      P.A0 = transpose(O.A0);
      Hierarchy &H = P.H;
      H.P = O.H.P;
      H.R = O.H.R;
      H.cf = O.H.cf;
      for (const Csr &A : O.H.A) H.A.push_back(transpose(A));
      for (const Csr &A : H.A) H.l1.push_back(l1_rowsum(A));
      const Csr &Ac = H.A.back();
      const int nl = Ac.nrows;
      H.Ac.assign((size_t)nl * nl, 0.0);
      for (int i = 0; i < nl; ++i)
        for (int jj = Ac.ptr[i]; jj < Ac.ptr[i + 1]; ++jj) H.Ac[(size_t)i * nl + Ac.col[jj]] = Ac.val[jj];
      if (!dense_inverse(nl, H.Ac, H.Ac_inv)) status[q] = ST_EINVAL;
    });
    for (int q = 0; q < nprob; ++q)
      if (status[q]) { err = "problem " + std::to_string(q) + ": singular transposed coarsest operator"; return status[q]; }
    T.times.hierarchy = now_s() - t0;
    return setup_layouts(T, composite, err);
  });
}

}  // namespace amgdd
