// CDNA4 (gfx950) kernels of the AMG-DD solve phase.
//
// Every matrix is a block-diagonal batch over all composite grids (or over
// all problems for the global hierarchy) stored as *grouped sliced ELL* (with
// 16-bit column indices where each slice's columns fit two 32K windows): each
// row is served by G = 2^lg lanes (G = 1 on levels with short rows, up to 16
// on coarse levels whose Galerkin rows hold ~100 entries); one 64-lane
// wavefront owns one slice of 64/G rows, and step k of the slice stores, for
// every row r of the slice and every lane j of its group, entry k*G + j of row
// r at
//     sptr[slice] + 64*k + (r mod 64/G)*G + j
// so every load instruction of a wavefront is one contiguous 128-byte (16-bit
// index) / 512-byte (FP64) segment.  Wide-step matrices (see sell_dotw) store
// two or four consecutive entries of a row per lane and step instead, cutting
// the index and value load instructions per entry (the slices keep the same
// size: the last steps narrow down to what is left).  Each lane accumulates its entries in order; the
// G partial sums are combined by an xor-shuffle tree (fixed order, so results
// do not depend on the launch schedule).  Padding entries carry value 0 and a
// column of the row's own grid.
//
// The AlgFAC cycle (Algorithm 4 of the paper) is split into passes, each
// fusing the vector updates of one algorithm step with the mat-vec it needs:
//   relax        delta = (f - A u) / d at real rows, u += delta, t (+)= delta
//   w            w = s + A t                       (restrict update, part 1)
//   down         s = R w_{l-1}; f <- f - A u - s;  (restrict update part 2,
//                u <- 0; first relaxation from 0    recalculation, initialise)
//   coarse       f <- f - A u - s; u = A_L^{-1} f   (dense, one workgroup/grid)
//   interp       u += P u_{l+1}
// Relaxation never reads and writes the same u buffer (Jacobi): it reads
// buffer `u_in` and writes `u_out` for every row of the level (copies where it
// does not relax).
//
// CF-ordered relaxation (the smoother of the paper's experiments): a sweep is
// two Jacobi half-sweeps, C-points then F-points on the way down and F then C
// on the way up, each over the points of one class and seeing the update of
// the other.  The relaxing passes then take the class of every real row
// (cls, +1 C / -1 F) and the class `want` they relax; cls == nullptr is the
// natural order (every real row relaxes).  Rows of the other class are copied
// (and keep or clear their t entry as the pass's t mode says).
//
// No MFMA: every step is a sparse mat-vec or a vector update (HBM bound).
#pragma once

#include <hip/hip_runtime.h>

namespace amgdd {
namespace dev {

constexpr int BLOCK = 256;
constexpr int NXCD = 8;
constexpr int BAND_WINDOWS = 8;  // windows of an LDS band (see SellD)

#ifndef AMGDD_UNROLL
#define AMGDD_UNROLL 4
#endif
// 16-bit-index mat-vecs issue the next group's index / value loads before the
// current group's gathers (measured: 1-3% faster on every workload)
#ifndef AMGDD_PIPE
#define AMGDD_PIPE 1
#endif

// Column indices are int32 (col) or, when every slice allows it, 16-bit
// (col16) relative to one of two per-slice bases:
//   column = (c16 & 0x8000 ? base[2s+1] : base[2s]) + (c16 & 0x7fff).
template <typename T>
struct SellD {
  const int *sptr;
  const int *col;
  const T *val;
  int lg;  // lanes per row G = 1 << lg
  const unsigned short *col16;
  const int *base;
  int vlg;  // log2 entries per lane in the widest steps (see sell_dotw)
  // LDS bands (composite operators): tile t = the ts slices from ts t on,
  // one 1024-thread workgroup; with W = BAND_WINDOWS, tiles[2Wt .. 2Wt+W-1]
  // window starts, [2Wt+W .. 2Wt+2W-1] cumulative window lengths (the last
  // one is the band size); a first start -1 - o < 0 marks a listed tile
  // whose band is bidx[o .. o + size); colL = each entry's position in its
  // tile's band
  const unsigned short *colL;
  const int *tiles;
  const int *bidx;
  int ntiles;
  int nslices;
  int ts;  // slices per LDS tile
};

// Workgroups are dispatched round-robin over the 8 XCDs; remap so that each
// XCD processes one contiguous range of row blocks (neighbouring rows share
// vector entries, which then stay in that XCD's L2).
__device__ __forceinline__ int xcd_block() {
  const int b = blockIdx.x, n = gridDim.x;
  const int q = n / NXCD, r = n % NXCD;
  const int x = b % NXCD, i = b / NXCD;
  return x * q + (x < r ? x : r) + i;
}

__device__ __forceinline__ int thread_id() { return xcd_block() * BLOCK + (int)threadIdx.x; }
template <int WG>
__device__ __forceinline__ int thread_id_wg() { return xcd_block() * WG + (int)threadIdx.x; }

// Sum over the G = 2^lg lanes of each row group (xor butterfly, fixed order).
template <typename V>
__device__ __forceinline__ V group_sum(V acc, int lg) {
  for (int o = (1 << lg) >> 1; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  return acc;
}

// Wide load steps: a slice of 64u entries (u unpaired steps of 64 lanes)
// whose widest steps carry W = 2^VL entries per lane holds floor(u/W) steps
// of 64W entries first, then one step of 64 * 2^v entries for each narrower
// width 2^v whose bit is set in u (v = VL-1 .. 0), so slices keep the size
// of the unpaired layout.  A step of width 2^v stores, for lane
// p = (r mod 64/G)*G + j, 2^v consecutive entries of row r at offset p 2^v
// (the first step of the widest region holds entries 0 .. W-1 of lane j's
// share, i.e. entries jW .. jW + W-1 of the row): one W-wide value load
// (16 bytes for two FP64 or four FP32 values) and one W-wide load of 16-bit
// indices per lane and step.  Each lane accumulates in storage order.
template <typename T, typename V, int VL>
__device__ __forceinline__ V sell_dotw(const SellD<T> &M, int s, int beg, int r, int sub, const V *__restrict__ x) {
  constexpr int W = 1 << VL;
  typedef T TW __attribute__((ext_vector_type(W)));
  typedef T T2 __attribute__((ext_vector_type(2)));
  typedef unsigned short CW __attribute__((ext_vector_type(W)));
  typedef unsigned short C2 __attribute__((ext_vector_type(2)));
  typedef int IW __attribute__((ext_vector_type(W)));
  typedef int I2 __attribute__((ext_vector_type(2)));
  const int lg = M.lg;
  const int u = (M.sptr[s + 1] - beg) >> 6, w = u >> VL;
  const int p = ((r & ((64 >> lg) - 1)) << lg) + sub;
  const TW *__restrict__ v = (const TW *)(M.val + beg + W * p);
  // narrower steps after the widest region
  const int off2 = beg + (w << (6 + VL));                          // width 2 (VL == 2 only)
  const int has2 = VL == 2 ? (u >> 1) & 1 : 0;
  const int off1 = off2 + (has2 << 7);                             // width 1
  constexpr int U = AMGDD_UNROLL / W > 0 ? AMGDD_UNROLL / W : 1;  // steps in flight
  V acc = V(0);
  int k = 0;
  if (M.col16) {
    const CW *__restrict__ c = (const CW *)(M.col16 + beg + W * p);
    const int b0 = M.base[2 * s], b1 = M.base[2 * s + 1];
    auto dec = [&](unsigned short q) { return ((q & 0x8000) ? b1 : b0) + (int)(q & 0x7fff); };
    // The slice's last pieces (the widest steps after the last group of U,
    // the two-wide step, the odd entry) are loaded first, so their loads
    // overlap the groups' instead of following them.
    const int rem = w % U, kr = w - rem;
    CW cr[U];
    TW vr[U];
    C2 c2 = {0, 0};
    T2 v2 = {T(0), T(0)};
    unsigned short c1 = 0;
    T v1 = T(0);
#pragma unroll
    for (int j = 0; j < U - 1; ++j)
      if (j < rem) {
        cr[j] = __builtin_nontemporal_load(c + 64 * (kr + j));
        vr[j] = __builtin_nontemporal_load(v + 64 * (kr + j));
      }
    if (has2) {
      c2 = __builtin_nontemporal_load((const C2 *)(M.col16 + off2 + 2 * p));
      v2 = __builtin_nontemporal_load((const T2 *)(M.val + off2 + 2 * p));
    }
    if (u & 1) {
      c1 = __builtin_nontemporal_load(M.col16 + off1 + p);
      v1 = __builtin_nontemporal_load(M.val + off1 + p);
    }
    if (k + U <= w) {
      CW cn[U];
      TW vn[U];
#pragma unroll
      for (int j = 0; j < U; ++j) {
        cn[j] = __builtin_nontemporal_load(c + 64 * (k + j));
        vn[j] = __builtin_nontemporal_load(v + 64 * (k + j));
      }
      for (; k + U <= w; k += U) {
        int cc[W * U];
        V vv[W * U], xx[W * U];
#pragma unroll
        for (int j = 0; j < U; ++j)
#pragma unroll
          for (int e = 0; e < W; ++e) {
            cc[W * j + e] = dec(cn[j][e]);
            vv[W * j + e] = (V)vn[j][e];
          }
#pragma unroll
        for (int j = 0; j < W * U; ++j) xx[j] = x[cc[j]];
        if (k + 2 * U <= w) {
#pragma unroll
          for (int j = 0; j < U; ++j) {
            cn[j] = __builtin_nontemporal_load(c + 64 * (k + U + j));
            vn[j] = __builtin_nontemporal_load(v + 64 * (k + U + j));
          }
        }
#pragma unroll
        for (int j = 0; j < W * U; ++j) acc = fma(vv[j], xx[j], acc);
      }
    }
    // the pieces' gathers, then their products in storage order
    V xr[W * U], x2[2], x1 = V(0);
#pragma unroll
    for (int j = 0; j < U - 1; ++j)
      if (j < rem)
#pragma unroll
        for (int e = 0; e < W; ++e) xr[W * j + e] = x[dec(cr[j][e])];
    if (has2) {
      x2[0] = x[dec(c2.x)];
      x2[1] = x[dec(c2.y)];
    }
    if (u & 1) x1 = x[dec(c1)];
#pragma unroll
    for (int j = 0; j < U - 1; ++j)
      if (j < rem)
#pragma unroll
        for (int e = 0; e < W; ++e) acc = fma((V)vr[j][e], xr[W * j + e], acc);
    if (has2) {
      acc = fma((V)v2.x, x2[0], acc);
      acc = fma((V)v2.y, x2[1], acc);
    }
    if (u & 1) acc = fma((V)v1, x1, acc);
  } else {
    const IW *__restrict__ c = (const IW *)(M.col + beg + W * p);
    for (; k + U <= w; k += U) {
      IW cq[U];
      TW vq[U];
      V xx[W * U];
#pragma unroll
      for (int j = 0; j < U; ++j) {
        cq[j] = __builtin_nontemporal_load(c + 64 * (k + j));
        vq[j] = __builtin_nontemporal_load(v + 64 * (k + j));
      }
#pragma unroll
      for (int j = 0; j < U; ++j)
#pragma unroll
        for (int e = 0; e < W; ++e) xx[W * j + e] = x[cq[j][e]];
#pragma unroll
      for (int j = 0; j < U; ++j)
#pragma unroll
        for (int e = 0; e < W; ++e) acc = fma((V)vq[j][e], xx[W * j + e], acc);
    }
    for (; k < w; ++k) {
      const IW cq = __builtin_nontemporal_load(c + 64 * k);
      const TW vq = __builtin_nontemporal_load(v + 64 * k);
      V xx[W];
#pragma unroll
      for (int e = 0; e < W; ++e) xx[e] = x[cq[e]];
#pragma unroll
      for (int e = 0; e < W; ++e) acc = fma((V)vq[e], xx[e], acc);
    }
    if (has2) {
      const I2 cq = __builtin_nontemporal_load((const I2 *)(M.col + off2 + 2 * p));
      const T2 vq = __builtin_nontemporal_load((const T2 *)(M.val + off2 + 2 * p));
      const V x0 = x[cq.x], x1 = x[cq.y];
      acc = fma((V)vq.x, x0, acc);
      acc = fma((V)vq.y, x1, acc);
    }
    if (u & 1) acc = fma((V)__builtin_nontemporal_load(M.val + off1 + p), x[__builtin_nontemporal_load(M.col + off1 + p)], acc);
  }
  return group_sum(acc, lg);
}

// Row r of a grouped sliced-ELL matrix times x; `sub` is the calling lane's
// position in the row's group.  The group's first lane (sub == 0) returns the
// full sum.
// ALIGNED: the wavefront lies in one slice (threads assigned 64-aligned), so
// the slice bounds are wave-uniform scalars.
template <typename T, typename V, bool ALIGNED = true>
__device__ __forceinline__ V sell_dot(const SellD<T> &M, int r, int sub, const V *__restrict__ x) {
  const int lg = M.lg;
  int s = r >> (6 - lg);
  if (ALIGNED) s = __builtin_amdgcn_readfirstlane(s);
  const int beg = M.sptr[s];
  if (M.vlg == 1) return sell_dotw<T, V, 1>(M, s, beg, r, sub, x);
  if (M.vlg == 2) return sell_dotw<T, V, 2>(M, s, beg, r, sub, x);
  const int w = (M.sptr[s + 1] - beg) >> 6;
  const int off = beg + ((r & ((64 >> lg) - 1)) << lg) + sub;
  const T *__restrict__ v = M.val + off;
  // The matrix streams are read once per pass: non-temporal loads keep them
  // from evicting the gathered vector from L2 / MALL.
  V acc = V(0);
  int k = 0;
  // U entries in flight per lane: all index and value loads of a group are
  // issued before its gathers; the sum stays in storage order.
  constexpr int U = AMGDD_UNROLL;
  if (M.col16) {
    const unsigned short *__restrict__ c = M.col16 + off;
    const int b0 = M.base[2 * s], b1 = M.base[2 * s + 1];
    auto dec = [&](unsigned short q) { return ((q & 0x8000) ? b1 : b0) + (int)(q & 0x7fff); };
#if AMGDD_PIPE
    // software pipelined: the next group's index / value loads are issued
    // before this group's gathers
    if (k + U <= w) {
      unsigned short cn[U];
      V vn[U];
#pragma unroll
      for (int j = 0; j < U; ++j) {
        cn[j] = __builtin_nontemporal_load(c + 64 * (k + j));
        vn[j] = (V)__builtin_nontemporal_load(v + 64 * (k + j));
      }
      for (; k + U <= w; k += U) {
        int cc[U];
        V vv[U], xx[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
          cc[j] = dec(cn[j]);
          vv[j] = vn[j];
        }
#pragma unroll
        for (int j = 0; j < U; ++j) xx[j] = x[cc[j]];
        if (k + 2 * U <= w) {
#pragma unroll
          for (int j = 0; j < U; ++j) {
            cn[j] = __builtin_nontemporal_load(c + 64 * (k + U + j));
            vn[j] = (V)__builtin_nontemporal_load(v + 64 * (k + U + j));
          }
        }
#pragma unroll
        for (int j = 0; j < U; ++j) acc = fma(vv[j], xx[j], acc);
      }
    }
#endif
    for (; k + U <= w; k += U) {
      int cc[U];
      V vv[U], xx[U];
#pragma unroll
      for (int j = 0; j < U; ++j) {
        cc[j] = dec(__builtin_nontemporal_load(c + 64 * (k + j)));
        vv[j] = (V)__builtin_nontemporal_load(v + 64 * (k + j));
      }
#pragma unroll
      for (int j = 0; j < U; ++j) xx[j] = x[cc[j]];
#pragma unroll
      for (int j = 0; j < U; ++j) acc = fma(vv[j], xx[j], acc);
    }
    for (; k < w; ++k)
      acc = fma((V)__builtin_nontemporal_load(v + 64 * k), x[dec(__builtin_nontemporal_load(c + 64 * k))], acc);
  } else {
    const int *__restrict__ c = M.col + off;
    for (; k + U <= w; k += U) {
      int cc[U];
      V vv[U], xx[U];
#pragma unroll
      for (int j = 0; j < U; ++j) {
        cc[j] = __builtin_nontemporal_load(c + 64 * (k + j));
        vv[j] = (V)__builtin_nontemporal_load(v + 64 * (k + j));
      }
#pragma unroll
      for (int j = 0; j < U; ++j) xx[j] = x[cc[j]];
#pragma unroll
      for (int j = 0; j < U; ++j) acc = fma(vv[j], xx[j], acc);
    }
    for (; k < w; ++k) acc = fma((V)__builtin_nontemporal_load(v + 64 * k), x[__builtin_nontemporal_load(c + 64 * k)], acc);
  }
  return group_sum(acc, lg);
}

__device__ __forceinline__ bool relaxes(const signed char *__restrict__ cls, int want, int i) {
  return cls == nullptr || cls[i] == want;
}

extern __shared__ double lds_band[];

// LDS variants (template argument LV = the operator's step width, >= 0):
// 1024-thread workgroups (16 waves), one tile (16 or 32 slices, a property of
// the layout) each,
// compiled for two workgroups per CU (8 waves per SIMD, at most 64 VGPRs) so
// that one workgroup's staging phase overlaps the other's mat-vecs.  The
// workgroup copies its tile's band into LDS once, then each wave takes the
// tile's slices one after another from a counter in LDS: slices of one tile
// differ in length (rows are sorted by length in windows), and a wave that
// finishes a short slice takes the next one instead of idling until the
// longest is done.  They are used only on levels every tile of which has a
// band.
constexpr int LDS_WAVES = 8;
constexpr int LDS_WG = 1024;

// H consecutive load steps of W entries per lane (64 lanes apart) times the
// band: all loads first, then the gathers and the lane's fused multiply-adds
// in storage order.
template <typename T, int W, int H>
__device__ __forceinline__ void lds_steps(const unsigned short *c, const T *v, const T *band, T &acc) {
  typedef T TW __attribute__((ext_vector_type(W)));
  typedef unsigned short CW __attribute__((ext_vector_type(W)));
  CW cn[H];
  TW vn[H];
#pragma unroll
  for (int j = 0; j < H; ++j) {
    cn[j] = __builtin_nontemporal_load((const CW *)c + 64 * j);
    vn[j] = __builtin_nontemporal_load((const TW *)v + 64 * j);
  }
#pragma unroll
  for (int j = 0; j < H; ++j) {
    T xx[W];
#pragma unroll
    for (int e = 0; e < W; ++e) xx[e] = band[cn[j][e]];
#pragma unroll
    for (int e = 0; e < W; ++e) acc = fma(vn[j][e], xx[e], acc);
  }
}

// Slice s of M (the calling wave's 64 lanes) times the band: row r, lane
// `sub` of its group; entries gathered from LDS through their band
// positions (colL).  Same accumulation order as sell_dot / sell_dotw: each
// lane adds its entries in storage order, then the group's xor tree.
template <typename T, int VL>
__device__ __forceinline__ T lds_row_dot(const SellD<T> &M, int s, int r, int sub, const T *band) {
  constexpr int W = 1 << VL;
  typedef T T2 __attribute__((ext_vector_type(2)));
  typedef unsigned short C2 __attribute__((ext_vector_type(2)));
  // The widest steps go in batches of B (eight entries per lane), then the
  // rest in batches of B/2, B/4, ... steps: every load of a batch is issued
  // before its first gather, so a wave keeps a batch of matrix data in flight.
  constexpr int B = 8 / W > 0 ? 8 / W : 1;
  const int lg = M.lg;
  const int beg = M.sptr[s];
  const int u = (M.sptr[s + 1] - beg) >> 6, w = u >> VL;
  const int p = ((r & ((64 >> lg) - 1)) << lg) + sub;
  const unsigned short *__restrict__ c = M.colL + beg + W * p;
  const T *__restrict__ v = M.val + beg + W * p;
  const int off2 = beg + (w << (6 + VL));
  const int has2 = VL == 2 ? (u >> 1) & 1 : 0;
  const int off1 = off2 + (has2 << 7);
  T acc = T(0);
  int k = 0;
  for (; k + B <= w; k += B) lds_steps<T, W, B>(c + 64 * W * k, v + 64 * W * k, band, acc);
  if constexpr (B >= 8)
    if ((w - k) & 4) {
      lds_steps<T, W, 4>(c + 64 * W * k, v + 64 * W * k, band, acc);
      k += 4;
    }
  if constexpr (B >= 4)
    if ((w - k) & 2) {
      lds_steps<T, W, 2>(c + 64 * W * k, v + 64 * W * k, band, acc);
      k += 2;
    }
  if constexpr (B >= 2)
    if ((w - k) & 1) lds_steps<T, W, 1>(c + 64 * W * k, v + 64 * W * k, band, acc);
  if (VL == 2 && has2) {
    const C2 cq = __builtin_nontemporal_load((const C2 *)(M.colL + off2 + 2 * p));
    const T2 vq = __builtin_nontemporal_load((const T2 *)(M.val + off2 + 2 * p));
    const T x0 = band[cq.x], x1 = band[cq.y];
    acc = fma(vq.x, x0, acc);
    acc = fma(vq.y, x1, acc);
  }
  if (VL >= 1 && (u & 1))
    acc = fma(__builtin_nontemporal_load(M.val + off1 + p), band[__builtin_nontemporal_load(M.colL + off1 + p)], acc);
  return group_sum(acc, lg);
}

// One LDS tile of M.ts slices (every thread of the workgroup calls it; it holds
// the workgroup barrier): when `stage`, the tile's band of x is copied into LDS
// (coalesced loads of its windows, or of its listed columns); then the waves
// take the tile's slices from a counter and, for each lane's row r (group lane
// `sub`), call pre(r, sub, q) (it loads the operands of the row's update into
// q, so that their loads overlap the mat-vec's) and op(r, sub, dot, q), dot =
// row r of M times x (0 when the tile is not staged or the slice lies beyond
// M).  q lives across the slices (a field that pre leaves alone keeps its
// earlier value): resetting it per slice would overwrite the registers of the
// previous slice's loads and make the wave wait for all its memory operations,
// stores included, first.
template <typename T, int VL, typename Q, typename Pre, typename Op>
__device__ __forceinline__ void lds_tile(const SellD<T> &M, const T *__restrict__ x, bool stage, Pre pre, Op op) {
  constexpr int NW = BAND_WINDOWS;
  __shared__ int next_slice;
  const int tile = xcd_block(), lane = threadIdx.x & 63, lg = M.lg;
  const int *__restrict__ d = M.tiles + 2 * NW * tile;
  const int n = stage && tile < M.ntiles ? d[2 * NW - 1] : 0;
  T *band = (T *)lds_band;
  if (threadIdx.x == 0) next_slice = 0;
  Q q{};
  if (n > 0) {
    int lo[NW], end[NW];
#pragma unroll
    for (int k = 0; k < NW; ++k) {
      lo[k] = d[k];
      end[k] = d[NW + k];
    }
    // SB values per thread in flight: the loads of a batch go out before its
    // stores (positions past the band load and store its last value again)
    constexpr int SB = 4;
    if (lo[0] < 0) {
      const int *__restrict__ ix = M.bidx + (-1 - lo[0]);
      for (int k0 = threadIdx.x; k0 < n; k0 += SB * LDS_WG) {
        int c[SB];
        T t[SB];
#pragma unroll
        for (int j = 0; j < SB; ++j) c[j] = ix[min(k0 + j * LDS_WG, n - 1)];
#pragma unroll
        for (int j = 0; j < SB; ++j) t[j] = x[c[j]];
#pragma unroll
        for (int j = 0; j < SB; ++j) band[min(k0 + j * LDS_WG, n - 1)] = t[j];
      }
    } else {
      for (int k0 = threadIdx.x; k0 < n; k0 += SB * LDS_WG) {
        T t[SB];
#pragma unroll
        for (int j = 0; j < SB; ++j) {
          const int k = min(k0 + j * LDS_WG, n - 1);
          int base = lo[0] + k;
#pragma unroll
          for (int q = 1; q < NW; ++q)
            if (k >= end[q - 1]) base = lo[q] + (k - end[q - 1]);
          t[j] = x[base];
        }
#pragma unroll
        for (int j = 0; j < SB; ++j) band[min(k0 + j * LDS_WG, n - 1)] = t[j];
      }
    }
  }
  __syncthreads();
  for (;;) {
    int sl = 0;
    if (lane == 0) sl = atomicAdd(&next_slice, 1);
    sl = __builtin_amdgcn_readfirstlane(__shfl(sl, 0));
    if (sl >= M.ts) break;
    const int s = tile * M.ts + sl;
    const int r = s * (64 >> lg) + (lane >> lg), sub = lane & ((1 << lg) - 1);
    pre(r, sub, q);
    T dot = T(0);
    // a tile without nonzero entries: every product is +0 (as the sum of
    // zero terms from +0 is)
    if (n > 0 && s < M.nslices) dot = lds_row_dot<T, VL>(M, s, r, sub, band);
    op(r, sub, dot, q);
  }
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Block-wide sum in a fixed order (deterministic).
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double part[BLOCK / 64];
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) part[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < BLOCK / 64; ++i) s += part[i];
  return s;  // valid in thread 0
}

// ---------------------------------------------------------------- outer loop

// r = b - A x on the fine level of every problem (FP64; fine operators use one
// lane per row), plus per-block partial sums of r^2.  Blocks never straddle two
// problems (block table).  VC: also the V-cycle's first relaxation from zero,
// e = r / d (CF order: at C-points only, e = 0 at F-points).
template <typename TR, bool VC>
__global__ __launch_bounds__(BLOCK) void k_resid(SellD<double> A, const double *__restrict__ b,
                                                  const double *__restrict__ x, TR *__restrict__ r_out,
                                                  double *__restrict__ partial, const int *__restrict__ blk_row0,
                                                  const int *__restrict__ blk_row1, const double *__restrict__ dinv,
                                                  double *__restrict__ e_out, const signed char *__restrict__ cls) {
  const int blk = xcd_block();
  const int row = blk_row0[blk] + (int)threadIdx.x;
  double sq = 0.0;
  if (row < blk_row1[blk]) {
    const double r = b[row] - sell_dot<double, double, false>(A, row, 0, x);
    r_out[row] = (TR)r;
    if (VC) e_out[row] = relaxes(cls, 1, row) ? r * dinv[row] : 0.0;
    sq = r * r;
  }
  const double s = block_sum(sq);
  if (threadIdx.x == 0) partial[blk] = s;
}

// ||r||^2 of every problem from its blocks' partial sums (one workgroup per
// problem, fixed summation order).
__global__ __launch_bounds__(BLOCK) void k_norm_final(const double *__restrict__ partial,
                                                       const int *__restrict__ prob_blk0, double *__restrict__ out) {
  const int q = blockIdx.x;
  const int b0 = prob_blk0[q], b1 = prob_blk0[q + 1];
  double s = 0.0;
  for (int b = b0 + (int)threadIdx.x; b < b1; b += BLOCK) s += partial[b];
  s = block_sum(s);
  if (threadIdx.x == 0) out[q] = s;
}

// y = M x over rows [0, n) (restriction chain r_{l+1} = R_l r_l), computed in
// T and stored as TO.
template <typename T, typename TO = T>
__global__ __launch_bounds__(BLOCK) void k_spmv(SellD<T> M, int n, const T *__restrict__ x, TO *__restrict__ y) {
  const int t = thread_id(), i = t >> M.lg, sub = t & ((1 << M.lg) - 1);
  if (i < n) {
    const T v = sell_dot<T, T>(M, i, sub, x);
    if (sub == 0) y[i] = (TO)v;
  }
}

// Composite right-hand sides of every level at once: f[k] = r[src[k]] where
// src[k] >= 0 (real points); ghost entries are left untouched.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_gather(int n, const int *__restrict__ src, const T *__restrict__ r,
                                                   T *__restrict__ f) {
  const int i = thread_id();
  if (i < n) {
    const int s = src[i];
    if (s >= 0) f[i] = r[s];
  }
}

// Correction patched on each owned subdomain: x[g] += u0[owner[g]]
// (ASSIGN: x[g] = u0[owner[g]], the iterate of a cycle started from zero).
template <typename T, bool ASSIGN = false>
__global__ __launch_bounds__(BLOCK) void k_patch(int n, double *__restrict__ x, const int *__restrict__ owner,
                                                  const T *__restrict__ u0) {
  const int i = thread_id();
  if (i < n) {
    if (ASSIGN) x[i] = (double)u0[owner[i]];
    else x[i] += (double)u0[owner[i]];
  }
}

// ---------------------------------------------------------------- AlgFAC

// Level 0, first cycle (u = 0): delta = f / d at real rows (CF order: at C
// rows, 0 at F rows); ghosts set to 0.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_relax_zero(int nr, int nb, const T *__restrict__ f,
                                                       const T *__restrict__ dinv, T *__restrict__ u_out,
                                                       T *__restrict__ t, const signed char *__restrict__ cls) {
  const int i = thread_id();
  if (i < nr) {
    const T d = relaxes(cls, 1, i) ? f[i] * dinv[i] : T(0);
    u_out[i] = d;
    t[i] = d;
  } else if (i < nb) {
    u_out[i] = T(0);
  }
}

// l1-Jacobi sweep at rows [0, nr) of class `want` (all of them when cls is
// null); other rows of [0, nb) are copied.
// tmode: 0 t = delta (t = 0 at real rows of the other class), 1 t += delta,
// 2 no t.
// LV >= 0: LDS variant (see lds_tile).
template <typename T, int WG = BLOCK, int LV = -1>
__global__ __launch_bounds__(WG, LV >= 0 ? LDS_WAVES : 1) void k_relax(SellD<T> A, int nr, int nb,
                                                                        const T *__restrict__ f,
                                                                        const T *__restrict__ dinv,
                                                                        const T *__restrict__ u_in,
                                                                        T *__restrict__ u_out, T *__restrict__ t,
                                                                        int tmode,
                                                                        const signed char *__restrict__ cls,
                                                                        int want) {
  auto row = [&](int i, int sub, bool act, T au) {
    if (act) {
      const T d = (f[i] - au) * dinv[i];
      if (sub == 0) {
        u_out[i] = u_in[i] + d;
        if (tmode == 0) t[i] = d;
        else if (tmode == 1) t[i] += d;
      }
    } else if (i < nb && sub == 0) {
      u_out[i] = u_in[i];
      if (i < nr && tmode == 0) t[i] = T(0);
    }
  };
  if constexpr (LV >= 0) {
    // tiles of rows >= nr relax nothing: no staging
    const bool stage = xcd_block() * ((64 * A.ts) >> A.lg) < nr;
    struct Q {
      bool act;
      T f, d, u, t;
    };
    lds_tile<T, LV, Q>(
        A, u_in, stage,
        [&](int i, int sub, Q &q) {
          q.act = false;
          if (i < nb && sub == 0) {
            q.u = u_in[i];
            q.act = i < nr && relaxes(cls, want, i);
            if (q.act) {
              q.f = f[i];
              q.d = dinv[i];
              if (tmode == 1) q.t = t[i];
            }
          }
        },
        [&](int i, int sub, T au, const Q &q) {
          // row() with the operands loaded beforehand (q.act only in the
          // group's first lane, the one that stores)
          if (q.act) {
            const T d = (q.f - au) * q.d;
            u_out[i] = q.u + d;
            if (tmode == 0) t[i] = d;
            else if (tmode == 1) t[i] = q.t + d;
          } else if (i < nb && sub == 0) {
            u_out[i] = q.u;
            if (i < nr && tmode == 0) t[i] = T(0);
          }
        });
  } else {
    const int th = thread_id_wg<WG>(), i = th >> A.lg, sub = th & ((1 << A.lg) - 1);
    const bool act = i < nr && relaxes(cls, want, i);
    row(i, sub, act, act ? sell_dot<T, T>(A, i, sub, u_in) : T(0));
  }
}

// w = s + A t over rows [0, nb), in place in the s buffer (s is absent on
// level 0).  t is zero at ghost points, so ghost rows store real columns only.
template <typename T, int WG = BLOCK, int LV = -1>
__global__ __launch_bounds__(WG, LV >= 0 ? LDS_WAVES : 1) void k_w(SellD<T> A, int nb, T *__restrict__ sw,
                                                                    const T *__restrict__ t, int has_s) {
  auto row = [&](int i, int sub, T at) {
    if (i < nb && sub == 0) sw[i] = has_s ? sw[i] + at : at;
  };
  if constexpr (LV >= 0) {
    lds_tile<T, LV, T>(
        A, t, true,
        [&](int i, int sub, T &s0) {
          if (has_s && i < nb && sub == 0) s0 = sw[i];
        },
        [&](int i, int sub, T at, T s0) {
          if (i < nb && sub == 0) sw[i] = has_s ? s0 + at : at;
        });
  } else {
    const int th = thread_id_wg<WG>(), i = th >> A.lg, sub = th & ((1 << A.lg) - 1);
    if (i < nb) row(i, sub, sell_dot<T, T>(A, i, sub, t));
  }
}

// Level l >= 1, normal rows [0, nb): s = R_{l-1} w_{l-1} (stored for the next
// w pass); at real rows [0, nr) the coarse residual recalculation
// f <- (f - A u) - s (skipped in the first cycle, where u = 0), then u <- 0
// and the first relaxation from zero delta = f / d (CF order: the C half,
// delta = 0 at F rows); ghost rows get u = 0.  R and A of one level share the
// lane grouping.
template <typename T, int WG = BLOCK>
__global__ __launch_bounds__(WG) void k_down(SellD<T> R, SellD<T> A, int nr, int nb, const T *__restrict__ w_prev,
                                                 T *__restrict__ sw, T *__restrict__ f, const T *__restrict__ dinv,
                                                 const T *__restrict__ u_in, T *__restrict__ u_out, T *__restrict__ t,
                                                 int first, const signed char *__restrict__ cls) {
  const int th = thread_id_wg<WG>(), i = th >> A.lg, sub = th & ((1 << A.lg) - 1);
  if (i >= nb) return;
  const T s = sell_dot<T, T>(R, i, sub, w_prev);
  if (i < nr) {
    T fi = f[i];
    if (!first) fi -= sell_dot<T, T>(A, i, sub, u_in);
    fi -= s;
    if (sub == 0) {
      sw[i] = s;
      f[i] = fi;
      const T d = relaxes(cls, 1, i) ? fi * dinv[i] : T(0);
      u_out[i] = d;
      t[i] = first ? d : t[i] + d;
    }
  } else if (sub == 0) {
    sw[i] = s;
    u_out[i] = T(0);
  }
}

// Restriction of the level-synchronous down pass on its own, for level l >= 1
// with R_{l-1} stored in a row order of its own (position k holds row
// perm[k]): s = R w_prev at every normal row (stored for the down and w
// passes), and u = 0 at ghost rows [nr, nb) (the down pass then covers the
// real rows only).
// LV >= 0: LDS variant (see lds_tile).
template <typename T, int WG = BLOCK, int LV = -1>
__global__ __launch_bounds__(WG, LV >= 0 ? LDS_WAVES : 1) void k_restrict_rows(SellD<T> Rt,
                                                                                const int *__restrict__ perm, int nb,
                                                                                int nr, const T *__restrict__ w_prev,
                                                                                T *__restrict__ sw,
                                                                                T *__restrict__ u_out) {
  auto row = [&](int k, int sub, T s) {
    if (k < nb && sub == 0) {
      const int i = perm[k];
      sw[i] = s;
      if (i >= nr) u_out[i] = T(0);
    }
  };
  if constexpr (LV >= 0) {
    lds_tile<T, LV, int>(
        Rt, w_prev, true,
        [&](int k, int sub, int &i) {
          if (k < nb && sub == 0) i = perm[k];
        },
        [&](int k, int sub, T s, int i) {
          if (k < nb && sub == 0) {
            sw[i] = s;
            if (i >= nr) u_out[i] = T(0);
          }
        });
  } else {
    const int th = thread_id_wg<WG>(), k = th >> Rt.lg, sub = th & ((1 << Rt.lg) - 1);
    if (k < nb) {
      const int i = perm[k];  // loaded before the mat-vec
      const T s = sell_dot<T, T>(Rt, k, sub, w_prev);
      if (sub == 0) {
        sw[i] = s;
        if (i >= nr) u_out[i] = T(0);
      }
    }
  }
}

// Down pass of level l >= 1 at real rows [0, nr) once s = R w_prev is in sw
// (k_restrict_rows): f <- (f - A u) - s (A u skipped in the first cycle),
// u <- 0 and the first relaxation from zero (CF order: the C half).  Same
// per-row arithmetic as k_down.
template <typename T, int WG = BLOCK, int LV = -1>
__global__ __launch_bounds__(WG, LV >= 0 ? LDS_WAVES : 1) void k_down_real(SellD<T> A, int nr,
                                                                            const T *__restrict__ sw,
                                                                            T *__restrict__ f,
                                                                            const T *__restrict__ dinv,
                                                                            const T *__restrict__ u_in,
                                                                            T *__restrict__ u_out,
                                                                            T *__restrict__ t, int first,
                                                                            const signed char *__restrict__ cls) {
  auto row = [&](int i, int sub, T au) {
    if (i < nr) {
      T fi = f[i];
      if (!first) fi -= au;
      fi -= sw[i];
      if (sub == 0) {
        f[i] = fi;
        const T d = relaxes(cls, 1, i) ? fi * dinv[i] : T(0);
        u_out[i] = d;
        t[i] = first ? d : t[i] + d;
      }
    }
  };
  if constexpr (LV >= 0) {
    struct Q {
      bool rel;
      T f, s, d, t;
    };
    lds_tile<T, LV, Q>(
        A, u_in, !first,
        [&](int i, int sub, Q &q) {
          if (i < nr && sub == 0) {
            q.f = f[i];
            q.s = sw[i];
            q.rel = relaxes(cls, 1, i);
            if (q.rel) q.d = dinv[i];
            if (!first) q.t = t[i];
          }
        },
        [&](int i, int sub, T au, const Q &q) {
          // row() with the operands loaded beforehand
          if (i < nr && sub == 0) {
            T fi = q.f;
            if (!first) fi -= au;
            fi -= q.s;
            f[i] = fi;
            const T d = q.rel ? fi * q.d : T(0);
            u_out[i] = d;
            t[i] = first ? d : q.t + d;
          }
        });
  } else {
    const int th = thread_id_wg<WG>(), i = th >> A.lg, sub = th & ((1 << A.lg) - 1);
    if (i < nr) row(i, sub, first ? T(0) : sell_dot<T, T>(A, i, sub, u_in));
  }
}

// u += P u_c with P in a row order of its own (position k holds row perm[k]).
template <typename T, int WG = BLOCK>
__global__ __launch_bounds__(WG) void k_interp_rows(SellD<T> Pt, const int *__restrict__ perm, int nb,
                                                        T *__restrict__ u, const T *__restrict__ uc) {
  const int th = thread_id_wg<WG>(), k = th >> Pt.lg, sub = th & ((1 << Pt.lg) - 1);
  if (k < nb) {
    // the row's target and old value are loaded before the mat-vec
    const int i = perm[k];
    const T ui = u[i];
    const T v = sell_dot<T, T>(Pt, k, sub, uc);
    if (sub == 0) u[i] = ui + v;
  }
}

// Coarsest level, one workgroup per grid (or per problem):
//   mode 0 (AlgFAC): f <- (f - A_L u) - R w_prev  (A_L u skipped when first),
//                    u_out = A_L^{-1} f
//   mode 1 (V-cycle): f = R w_prev, u_out = A_L^{-1} f
// Arithmetic in FP64 (the coarsest solve stays FP64 in the mixed form).
// u_both, if given, receives u as well (the coarsest level keeps its value in
// both buffers).
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_coarse(SellD<T> R, int has_r, const T *__restrict__ w_prev,
                                                   T *__restrict__ f, const T *__restrict__ u_in,
                                                   T *__restrict__ u_out, const double *__restrict__ Ad,
                                                   const double *__restrict__ Ainv, const int *__restrict__ row0,
                                                   const int *__restrict__ nn, const int *__restrict__ doff, int mode,
                                                   int first, T *u_both) {
  extern __shared__ double sh[];
  const int g = blockIdx.x;
  const int r0 = row0[g], n = nn[g];
  const double *Ag = Ad + doff[g];
  const double *Ig = Ainv + doff[g];
  const int lg = R.lg, sub = threadIdx.x & ((1 << lg) - 1);
  double *fs = sh;       // n
  double *us = sh + n;   // n
  for (int i = threadIdx.x; i < n; i += BLOCK) us[i] = (mode == 0 && !first) ? (double)u_in[r0 + i] : 0.0;
  __syncthreads();
  for (int i = threadIdx.x >> lg; i < n; i += BLOCK >> lg) {
    double s = 0.0;
    if (has_r) s = (double)sell_dot<T, T, false>(R, r0 + i, sub, w_prev);
    if (sub == 0) {
      double fi;
      if (mode == 0) {
        fi = (double)f[r0 + i];
        if (!first) {
          double au = 0.0;
          for (int j = 0; j < n; ++j) au = fma(Ag[(size_t)i * n + j], us[j], au);
          fi -= au;
        }
        fi -= s;
      } else {
        fi = s;
      }
      fs[i] = fi;
      f[r0 + i] = (T)fi;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += BLOCK) {
    double u = 0.0;
    for (int j = 0; j < n; ++j) u = fma(Ig[(size_t)i * n + j], fs[j], u);
    u_out[r0 + i] = (T)u;
    if (u_both) u_both[r0 + i] = (T)u;
  }
}

// u += P u_c over rows [0, nb).
template <typename T, int WG = BLOCK>
__global__ __launch_bounds__(WG) void k_interp(SellD<T> P, int nb, T *__restrict__ u, const T *__restrict__ uc) {
  const int th = thread_id_wg<WG>(), i = th >> P.lg, sub = th & ((1 << P.lg) - 1);
  if (i < nb) {
    const T v = sell_dot<T, T>(P, i, sub, uc);
    if (sub == 0) u[i] += v;
  }
}

// ---------------------------------------------------------------- per-grid schedule

// Pointers of one batched composite level (A and R share the lane grouping;
// P has its own).  Pt / Rt (when Pt.sptr / Rt.sptr are set): P and R of the
// normal rows in row orders of their own, row i at position ppos[i] /
// rpos[i]; R is then applied in a step of its own before the rest of the
// down pass, and the coarse-grid rows of R keep using R.
template <typename T>
struct LevelDev {
  SellD<T> A, P, R;
  const T *dinv;
  T *u0, *u1, *t, *sw, *f;
  const signed char *cls;  // C/F class of the real rows (CF order), or null
  SellD<T> Pt, Rt;
  const int *ppos, *rpos;
};

// Row ranges of one grid on one level (see the batched layout).
struct GridLevel {
  int rbeg, nreal, gbeg, nghost;
};

__device__ __forceinline__ int grid_row(const GridLevel &d, int j) {
  return j < d.nreal ? d.rbeg + j : d.gbeg + (j - d.nreal);
}

// Persistent per-grid AlgFAC: one workgroup owns one composite grid and runs
// every level from `lt` down to the grid's coarsest level and back up, for
// `ncycles` cycles, with workgroup barriers between passes.  The composite
// operators are block-diagonal over grids (checked at setup, padding
// included), so no pass of one grid touches another grid.  Each pass is the
// same per-row arithmetic as the level-synchronous kernels (k_relax_zero /
// k_relax, k_down, k_w, k_coarse, k_interp), so both schedules give identical
// results.  Buffer convention (kept by the level-synchronous path too): at
// the start and end of every cycle a level's u lives in u0; the down pass
// writes u1, interpolation updates u1, post-relaxation writes u0; the
// coarsest solve writes both.  CF order adds one half-sweep on each side: the
// down pass writes u1 and its F half u0, interpolation updates u0, the up F
// half writes u1 and the C half u0.
template <typename T>
__global__ __launch_bounds__(1024) void k_fac_tail(const LevelDev<T> *__restrict__ lv, const GridLevel *__restrict__ gl,
                                                    int nlev, const int *__restrict__ grids,
                                                    const int *__restrict__ gridL, const int *__restrict__ gdense,
                                                    const double *__restrict__ Ad, const double *__restrict__ Ainv,
                                                    int lt, int ncycles, int first_cycle) {
  extern __shared__ double sh[];
  const int g = grids[blockIdx.x];
  const int L = gridL[g];
  const GridLevel *G = gl + (size_t)g * nlev;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int c = 0; c < ncycles; ++c) {
    const int first = first_cycle && c == 0;
    for (int l = lt; l < L; ++l) {
      const LevelDev<T> B = lv[l];
      const GridLevel d = G[l];
      const int nb = d.nreal + d.nghost;
      const int lg = B.A.lg, sub = tid & ((1 << lg) - 1), j0 = tid >> lg, js = nt >> lg;
      if (l == 0) {
        for (int j = j0; j < nb; j += js) {
          const int i = grid_row(d, j);
          const bool rc = j < d.nreal && relaxes(B.cls, 1, i);
          if (j < d.nreal && first) {
            if (sub == 0) {
              const T dl = rc ? B.f[i] * B.dinv[i] : T(0);
              B.u1[i] = dl;
              B.t[i] = dl;
            }
          } else if (rc) {
            const T dl = (B.f[i] - sell_dot<T, T, false>(B.A, i, sub, B.u0)) * B.dinv[i];
            if (sub == 0) {
              B.u1[i] = B.u0[i] + dl;
              B.t[i] += dl;
            }
          } else if (sub == 0) {
            B.u1[i] = first ? T(0) : B.u0[i];
          }
        }
      } else if (B.Rt.sptr) {
        // as k_restrict_rows then k_down_real
        const T *wprev = lv[l - 1].sw;
        const int rg = B.Rt.lg, rsub = tid & ((1 << rg) - 1);
        for (int j = tid >> rg; j < nb; j += nt >> rg) {
          const int i = grid_row(d, j);
          const T s = sell_dot<T, T, false>(B.Rt, B.rpos[i], rsub, wprev);
          if (rsub == 0) {
            B.sw[i] = s;
            if (j >= d.nreal) B.u1[i] = T(0);
          }
        }
        __syncthreads();
        for (int j = j0; j < d.nreal; j += js) {
          const int i = grid_row(d, j);
          T fi = B.f[i];
          if (!first) fi -= sell_dot<T, T, false>(B.A, i, sub, B.u0);
          fi -= B.sw[i];
          if (sub == 0) {
            B.f[i] = fi;
            const T dl = relaxes(B.cls, 1, i) ? fi * B.dinv[i] : T(0);
            B.u1[i] = dl;
            B.t[i] = first ? dl : B.t[i] + dl;
          }
        }
      } else {
        const T *wprev = lv[l - 1].sw;
        for (int j = j0; j < nb; j += js) {
          const int i = grid_row(d, j);
          const T s = sell_dot<T, T, false>(B.R, i, sub, wprev);
          if (j < d.nreal) {
            T fi = B.f[i];
            if (!first) fi -= sell_dot<T, T, false>(B.A, i, sub, B.u0);
            fi -= s;
            if (sub == 0) {
              B.sw[i] = s;
              B.f[i] = fi;
              const T dl = relaxes(B.cls, 1, i) ? fi * B.dinv[i] : T(0);
              B.u1[i] = dl;
              B.t[i] = first ? dl : B.t[i] + dl;
            }
          } else if (sub == 0) {
            B.sw[i] = s;
            B.u1[i] = T(0);
          }
        }
      }
      __syncthreads();
      if (B.cls) {
        // F half of the CF sweep: u1 -> u0
        for (int j = j0; j < nb; j += js) {
          const int i = grid_row(d, j);
          if (j < d.nreal && B.cls[i] == -1) {
            const T dl = (B.f[i] - sell_dot<T, T, false>(B.A, i, sub, B.u1)) * B.dinv[i];
            if (sub == 0) {
              B.u0[i] = B.u1[i] + dl;
              B.t[i] += dl;
            }
          } else if (sub == 0) {
            B.u0[i] = B.u1[i];
          }
        }
        __syncthreads();
      }
      for (int j = j0; j < nb; j += js) {
        const int i = grid_row(d, j);
        const T at = sell_dot<T, T, false>(B.A, i, sub, B.t);
        if (sub == 0) B.sw[i] = l > 0 ? B.sw[i] + at : at;
      }
      __syncthreads();
    }
    {
      const LevelDev<T> B = lv[L];
      const GridLevel d = G[L];
      const int n = d.nreal, r0 = d.rbeg;
      const int lg = B.R.lg, sub = tid & ((1 << lg) - 1);
      const double *Ag = Ad + gdense[g];
      const double *Ig = Ainv + gdense[g];
      double *fs = sh, *us = sh + n;
      for (int j = tid; j < n; j += nt) us[j] = first ? 0.0 : (double)B.u0[r0 + j];
      __syncthreads();
      const T *wprev = lv[L - 1].sw;
      for (int j = tid >> lg; j < n; j += nt >> lg) {
        const double s = (double)sell_dot<T, T, false>(B.R, r0 + j, sub, wprev);
        if (sub == 0) {
          double fi = (double)B.f[r0 + j];
          if (!first) {
            double au = 0.0;
            for (int k = 0; k < n; ++k) au = fma(Ag[(size_t)j * n + k], us[k], au);
            fi -= au;
          }
          fi -= s;
          fs[j] = fi;
          B.f[r0 + j] = (T)fi;
        }
      }
      __syncthreads();
      for (int j = tid; j < n; j += nt) {
        double u = 0.0;
        for (int k = 0; k < n; ++k) u = fma(Ig[(size_t)j * n + k], fs[k], u);
        B.u0[r0 + j] = (T)u;
        B.u1[r0 + j] = (T)u;
      }
      __syncthreads();
    }
    for (int l = L - 1; l >= lt; --l) {
      const LevelDev<T> B = lv[l];
      const GridLevel d = G[l];
      const int nb = d.nreal + d.nghost;
      const int lg = B.A.lg, sub = tid & ((1 << lg) - 1), j0 = tid >> lg, js = nt >> lg;
      const T *uc = lv[l + 1].u0;
      T *ucur = B.cls ? B.u0 : B.u1;
      if (B.Pt.sptr) {
        // as k_interp_rows
        const int pg = B.Pt.lg, psub = tid & ((1 << pg) - 1);
        for (int j = tid >> pg; j < nb; j += nt >> pg) {
          const int i = grid_row(d, j);
          const T v = sell_dot<T, T, false>(B.Pt, B.ppos[i], psub, uc);
          if (psub == 0) ucur[i] += v;
        }
      } else {
        // interpolation rows have their own lane count
        const int pg = B.P.lg, psub = tid & ((1 << pg) - 1);
        for (int j = tid >> pg; j < nb; j += nt >> pg) {
          const int i = grid_row(d, j);
          const T v = sell_dot<T, T, false>(B.P, i, psub, uc);
          if (psub == 0) ucur[i] += v;
        }
      }
      __syncthreads();
      if (B.cls) {
        // F half (t = delta, cleared at C rows) u0 -> u1, then the C half below
        for (int j = j0; j < nb; j += js) {
          const int i = grid_row(d, j);
          if (j < d.nreal && B.cls[i] == -1) {
            const T dl = (B.f[i] - sell_dot<T, T, false>(B.A, i, sub, B.u0)) * B.dinv[i];
            if (sub == 0) {
              B.u1[i] = B.u0[i] + dl;
              B.t[i] = dl;
            }
          } else if (sub == 0) {
            B.u1[i] = B.u0[i];
            if (j < d.nreal) B.t[i] = T(0);
          }
        }
        __syncthreads();
      }
      for (int j = j0; j < nb; j += js) {
        const int i = grid_row(d, j);
        if (j < d.nreal && relaxes(B.cls, 1, i)) {
          const T dl = (B.f[i] - sell_dot<T, T, false>(B.A, i, sub, B.u1)) * B.dinv[i];
          if (sub == 0) {
            B.u0[i] = B.u1[i] + dl;
            if (B.cls) B.t[i] += dl;
            else B.t[i] = dl;
          }
        } else if (sub == 0) {
          B.u0[i] = B.u1[i];
        }
      }
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------- V-cycle

// q = f - A e over rows [0, n).
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_vresid(SellD<T> A, int n, const T *__restrict__ f, const T *__restrict__ e,
                                                   T *__restrict__ q) {
  const int th = thread_id(), i = th >> A.lg, sub = th & ((1 << A.lg) - 1);
  if (i < n) {
    const T v = sell_dot<T, T>(A, i, sub, e);
    if (sub == 0) q[i] = f[i] - v;
  }
}

// f = R q_prev, e = f / d (relaxation from zero; CF order: the C half, e = 0
// at F rows) over rows [0, n).
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_vdown(SellD<T> R, int n, const T *__restrict__ q_prev, T *__restrict__ f,
                                                  const T *__restrict__ dinv, T *__restrict__ e,
                                                  const signed char *__restrict__ cls) {
  const int th = thread_id(), i = th >> R.lg, sub = th & ((1 << R.lg) - 1);
  if (i < n) {
    const T fi = sell_dot<T, T>(R, i, sub, q_prev);
    if (sub == 0) {
      f[i] = fi;
      e[i] = relaxes(cls, 1, i) ? fi * dinv[i] : T(0);
    }
  }
}

// Level-0 post-relaxation fused with the iterate update:
// x += e + (f - A e) / d  (fine operators use one lane per row; CF order: the
// closing C half, x += e at F rows).
__global__ __launch_bounds__(BLOCK) void k_vfinal(SellD<double> A, int n, const double *__restrict__ f,
                                                   const double *__restrict__ dinv, const double *__restrict__ e,
                                                   double *__restrict__ x, const signed char *__restrict__ cls) {
  const int i = thread_id();
  if (i < n) {
    if (relaxes(cls, 1, i)) x[i] += e[i] + (f[i] - sell_dot<double, double>(A, i, 0, e)) * dinv[i];
    else x[i] += e[i];
  }
}

// ---------------------------------------------------------------- adjoint

// dL/dc_f = -(lam_i - lam_j)(u_i - u_j) (interior), -lam_i u_i (j < 0).
__global__ __launch_bounds__(BLOCK) void k_face_grad(int nf, const int *__restrict__ fi, const int *__restrict__ fj,
                                                      const double *__restrict__ u, const double *__restrict__ lam,
                                                      double *__restrict__ out) {
  const int k = thread_id();
  if (k < nf) {
    const int i = fi[k], j = fj[k];
    out[k] = j >= 0 ? -(lam[i] - lam[j]) * (u[i] - u[j]) : -lam[i] * u[i];
  }
}

}  // namespace dev
}  // namespace amgdd
