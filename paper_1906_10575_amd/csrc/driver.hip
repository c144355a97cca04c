// Device driver and C ABI of the AMG-DD solve phase (see include/amgdd.h).
//
// One outer AMG-DD iteration (Algorithm 2 of the paper) is enqueued as:
//   restriction chain r_{l+1} = R_l r_l (global batched operators)
//   one gather of the composite right-hand sides of every level
//   n_fac AlgFAC cycles (Algorithm 4) over all composite grids at once,
//     level-synchronous: relax/down + w on the way down, coarse solve,
//     interp + relax on the way up
//   patch x += u_0 on owned points
//   fine residual r = b - A x and its norm (for the next iteration)
// and is captured once into a HIP graph that is replayed every iteration; the
// host reads the per-problem residual norms (8 bytes each) after each replay.
// The V(1,1) cycle (Algorithm 1) is enqueued the same way on the global
// batched hierarchy, in correction form e = V(r), x += e.  The hybrid cycle
// (Algorithm 3) runs the V-cycle's passes above its transition level and a
// second handle's AMG-DD passes (the level-L~ problems) below it, captured
// into the same graph.

#include <dlfcn.h>
#include <hip/hip_runtime.h>

#include <sys/stat.h>
#include <unistd.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/amgdd.h"
#include "amgdd_internal.h"
#include "kernels.hpp"

using namespace amgdd;

namespace {

thread_local std::string g_last_error;

amgdd_status fail(int st, const std::string &msg) {
  g_last_error = msg;
  return (amgdd_status)st;
}

#define HIP_TRY(expr)                                                                           \
  do {                                                                                          \
    hipError_t _e = (expr);                                                                     \
    if (_e != hipSuccess) {                                                                     \
      return fail(_e == hipErrorOutOfMemory ? ST_ENOMEM : ST_EDEVICE,                           \
                  std::string(#expr) + ": " + hipGetErrorString(_e));                           \
    }                                                                                           \
  } while (0)

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Named ranges for timeline tools (rocprofv3 --marker-trace) when the
// environment sets AMGDD_TRACE=1: setup, upload, autotuning, graph capture,
// every solve and every outer iteration.  The roctx library is opened only
// then (dlopen), so an ordinary process loads no profiling library through
// this one: the HIP runtime in use may be another ROCm release's (the one
// torch ships).
struct Roctx {
  int (*push)(const char *) = nullptr;
  int (*pop)() = nullptr;
};
const Roctx &roctx() {
  static const Roctx r = [] {
    Roctx x;
    const char *e = std::getenv("AMGDD_TRACE");
    if (!(e && e[0] == '1')) return x;
    void *lib = dlopen("librocprofiler-sdk-roctx.so.1", RTLD_NOW | RTLD_GLOBAL);
    if (!lib) lib = dlopen("/opt/rocm/lib/librocprofiler-sdk-roctx.so.1", RTLD_NOW | RTLD_GLOBAL);
    if (!lib) return x;
    x.push = (int (*)(const char *))dlsym(lib, "roctxRangePushA");
    x.pop = (int (*)())dlsym(lib, "roctxRangePop");
    if (!x.push || !x.pop) x.push = nullptr, x.pop = nullptr;
    return x;
  }();
  return r;
}
bool tracing() { return roctx().push != nullptr; }
struct TraceRange {
  bool on;
  explicit TraceRange(const char *name) : on(tracing()) {
    if (on) roctx().push(name);
  }
  TraceRange(const std::string &name) : TraceRange(name.c_str()) {}
  ~TraceRange() {
    if (on) roctx().pop();
  }
};

struct DSell {
  int *sptr = nullptr;
  int *col = nullptr;
  void *val = nullptr;  // double or float
  unsigned short *col16 = nullptr;  // 16-bit columns (then col is null)
  int *base = nullptr;              // two bases per slice
  int nrows = 0;
  int lg = 0;           // lanes per row (log2)
  int vlg = 0;          // log2 entries per lane in the widest steps
  long long entries = 0;
  unsigned short *colL = nullptr;  // LDS bands (composite operators)
  int *tiles = nullptr;
  int *bidx = nullptr;
  int ntiles = 0, nslices = 0;
  int ts = 0;  // slices per LDS tile
  template <typename T>
  dev::SellD<T> as() const {
    return dev::SellD<T>{sptr, col, (const T *)val, lg, col16, base, vlg, colL, tiles, bidx, ntiles, nslices, ts};
  }
};

struct DLevel {
  // composite
  int NRn = 0, NBn = 0, NB = 0;
  int lg = 0, glg = 0;  // lanes per row (log2) of composite / global rows
  int wg = dev::BLOCK;  // workgroup size of the level's composite passes (256, 512 or 1024)
  // the passes with the composite operator run in 1024-thread workgroups that
  // stage the gathered vector's band in LDS (band_max values at most)
  bool lds = false;
  int band_max = 0;
  bool rlds = false;  // same for the reordered restriction pass (w_{l-1}'s band)
  int rband_max = 0;
  DSell A, P, R;
  // reordered P / R_{l-1} of the normal rows (Setup::tight): position k holds
  // row pperm[k] / rperm[k]; ppos / rpos are the inverse maps (per-grid tail)
  DSell Pt, Rt;
  int *pperm = nullptr, *rperm = nullptr, *ppos = nullptr, *rpos = nullptr;
  void *dinv = nullptr;
  void *u[2] = {nullptr, nullptr};
  void *t = nullptr, *sw = nullptr, *f = nullptr;  // f points into the level-f arena
  int ncg = 0;
  int *cg_row0 = nullptr, *cg_n = nullptr, *cg_dense = nullptr;
  int cg_maxn = 0;
  // global
  int GNn = 0, GN = 0;
  DSell GA, GP, GRd, GRt;  // GRd: FP64 (V-cycle); GRt: composite precision (restriction chain)
  double *gdinv = nullptr;
  double *ve[2] = {nullptr, nullptr};
  double *vq = nullptr, *vf = nullptr;
  void *rt = nullptr;  // restricted residual r_l (composite precision), points into r arena
  int ngc = 0;
  int *gc_row0 = nullptr, *gc_n = nullptr, *gc_dense = nullptr;
  int gc_maxn = 0;
  // stored nonzeros (algorithmic-bytes model of the profiler)
  long long nnzA_r = 0, nnzA = 0, nnzP = 0, nnzR_n = 0, nnzR = 0;
  long long nnzGA_n = 0, nnzGA = 0, nnzGP = 0, nnzGR_n = 0, nnzGR = 0;
  // CF-ordered relaxation: classes of the composite real rows and of the
  // normal global rows (null in natural order)
  signed char *cls = nullptr, *gcls = nullptr;
  int NRc = 0, GNc = 0;
  long long nnzA_c = 0, nnzGA_c = 0;
};

// Per-launch event timing (amgdd_profile): one event pair per launch site.
struct Prof {
  struct Site {
    std::string name;
    int level;
    double bytes;
    hipEvent_t e0, e1;
    int grid, block;
    int rep;
  };
  std::vector<Site> sites;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  int rep = 0;  // iteration being recorded
  hipEvent_t get() {
    if (used == pool.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      pool.push_back(e);
    }
    return pool[used++];
  }
  int begin(const char *name, int level, double bytes, hipStream_t s, int grid, int block) {
    Site st{name, level, bytes, get(), get(), grid, block, rep};
    (void)hipEventRecord(st.e0, s);
    sites.push_back(st);
    return (int)sites.size() - 1;
  }
  void end(int k, hipStream_t s) { (void)hipEventRecord(sites[k].e1, s); }
  ~Prof() {
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

}  // namespace

struct amgdd_ctx {
  Setup S;
  amgdd_params prm{};
  bool host_only = true;
  bool symmetric = true;
  double setup_s = 0.0;
  int device = 0;
  hipStream_t stream = nullptr;      // caller's stream
  hipStream_t cap_stream = nullptr;  // private stream used for graph capture
  // second branch of an AMG-DD iteration (restriction chain and coarse
  // right-hand sides, beside the first cycle's level-0 passes); off when
  // AMGDD_SERIAL is set
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  bool overlap = true;
  long long f_off1 = 0;  // composite right-hand sides of level 0: arena entries [0, f_off1)
  std::vector<void *> allocs;
  long long dev_bytes = 0;
  long long max_bytes = 0;  // > 0: device-memory cap (AMGDD_TEST_MAX_BYTES, failure-path tests)
  std::vector<DLevel> L;
  // outer vectors
  double *b = nullptr, *x = nullptr;
  double *partial = nullptr, *norm2 = nullptr;
  // residual partial sums / norms in use: the handle's own, or the library's
  // static scratch during amgdd_solve_noalloc
  double *rs_partial = nullptr, *rs_norm2 = nullptr;
  double *partial_buf() const { return rs_partial ? rs_partial : partial; }
  double *norm2_buf() const { return rs_norm2 ? rs_norm2 : norm2; }
  double *h_norm2 = nullptr;  // pinned
  int *blk_row0 = nullptr, *blk_row1 = nullptr, *prob_blk0 = nullptr;
  int nblk = 0, nprob = 0, N0 = 0;
  int *owner = nullptr;
  double *dense_A = nullptr, *dense_inv = nullptr;
  void *f_arena = nullptr;
  int *gather_src = nullptr;
  long long f_total = 0;
  void *r_arena = nullptr;
  // per-grid persistent schedule
  void *lvdev = nullptr;                 // LevelDev<T>[nlev]
  dev::GridLevel *gl = nullptr;          // [ngrids * nlev]
  int *gridL = nullptr, *gdense = nullptr;
  int *tail_lists = nullptr;             // grids with L >= lt, largest first, for every lt
  std::vector<int> tail_off, tail_cnt;   // per lt
  int tail_maxn = 0;                     // largest coarsest level (shared memory of the tail)
  int sched_level = -2, sched_block = 256;
  int sched_cached = 0;  // schedule taken from the schedule cache
  bool wg_fixed = false;  // composite-pass workgroup sizes set by the environment (not tuned)
  bool lds_fixed = false; // LDS staging set by the environment (not tuned)
  double autotune_s = 0.0;
  hipGraphExec_t g_dd = nullptr, g_v = nullptr;
  hipGraph_t gr_dd = nullptr, gr_v = nullptr;
  std::vector<std::vector<double>> hist;  // per problem
  Prof *prof = nullptr;
  int lbase = 0;  // level of this handle's fine level in the profiling sites
  // hybrid AMG-DD: the level-L~ AMG-DD problems live in a handle of their own
  amgdd_ctx *inner = nullptr;
  int hybrid_lt = 0;                       // transition level L~ (0: not hybrid)
  std::vector<int> inner_of;               // problem -> its level-L~ problem (-1: none)
  std::vector<std::vector<int>> part_map;  // subdomain -> level-L~ subdomain (-1: empty)
  // adjoint of a non-symmetric operator: a handle of its own on the transposed
  // hierarchy (built at the first adjoint solve)
  amgdd_ctx *adj = nullptr;

  bool mixed() const { return prm.precision == AMGDD_MIXED; }
  bool cf() const { return S.cf; }

  amgdd_status alloc(void **p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) return AMGDD_OK;
    if (max_bytes > 0 && dev_bytes + (long long)bytes > max_bytes)
      return fail(ST_ENOMEM, "device memory cap reached (" + std::to_string(max_bytes) + " bytes)");
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) return fail(e == hipErrorOutOfMemory ? ST_ENOMEM : ST_EDEVICE, std::string("hipMalloc: ") + hipGetErrorString(e));
    allocs.push_back(*p);
    dev_bytes += (long long)bytes;
    return AMGDD_OK;
  }
  template <typename V>
  amgdd_status upload(V **dst, const V *src, size_t n) {
    amgdd_status st = alloc((void **)dst, n * sizeof(V));
    if (st) return st;
    if (n) HIP_TRY(hipMemcpy(*dst, src, n * sizeof(V), hipMemcpyHostToDevice));
    return AMGDD_OK;
  }
  amgdd_status upload_vals(void **dst, const std::vector<double> &v, bool as_float) {
    if (!as_float) return upload((double **)dst, v.data(), v.size());
    std::vector<float> f(v.begin(), v.end());
    return upload((float **)dst, f.data(), f.size());
  }
  amgdd_status upload_sell(DSell &d, const Sell &s, bool as_float) {
    d.nrows = s.nrows;
    d.lg = s.lg;
    d.vlg = s.vlg;
    d.entries = s.entries();
    d.nslices = s.sptr.empty() ? 0 : (int)s.sptr.size() - 1;
    amgdd_status st = upload(&d.sptr, s.sptr.data(), s.sptr.size());
    if (st) return st;
    if (s.compressed()) {
      if ((st = upload(&d.col16, (const unsigned short *)s.col16.data(), s.col16.size()))) return st;
      if ((st = upload(&d.base, s.base.data(), s.base.size()))) return st;
    } else if ((st = upload(&d.col, s.col.data(), s.col.size()))) {
      return st;
    }
    if (!s.tiles.empty()) {
      if ((st = upload(&d.colL, (const unsigned short *)s.colL.data(), s.colL.size()))) return st;
      if ((st = upload(&d.tiles, s.tiles.data(), s.tiles.size()))) return st;
      if (!s.bidx.empty() && (st = upload(&d.bidx, s.bidx.data(), s.bidx.size()))) return st;
      static_assert(kBandWindows == dev::BAND_WINDOWS, "tile descriptor layout");
      d.ntiles = (int)(s.tiles.size() / (2 * kBandWindows));
      d.ts = s.ts;
    }
    return upload_vals(&d.val, s.val, as_float);
  }

  void drop_graphs() {
    if (g_dd) (void)hipGraphExecDestroy(g_dd);
    if (g_v) (void)hipGraphExecDestroy(g_v);
    if (gr_dd) (void)hipGraphDestroy(gr_dd);
    if (gr_v) (void)hipGraphDestroy(gr_v);
    g_dd = g_v = nullptr;
    gr_dd = gr_v = nullptr;
  }

  ~amgdd_ctx() {
    delete adj;
    delete inner;
    if (!host_only) {
      (void)hipSetDevice(device);
      // nothing of this handle may still run when its resources go
      (void)hipStreamSynchronize(stream);
      if (cap_stream) (void)hipStreamSynchronize(cap_stream);
      if (side) (void)hipStreamSynchronize(side);
      drop_graphs();
      for (void *p : allocs) (void)hipFree(p);
      if (h_norm2) (void)hipHostFree(h_norm2);
      if (cap_stream) (void)hipStreamDestroy(cap_stream);
      if (side) (void)hipStreamDestroy(side);
      if (ev_fork) (void)hipEventDestroy(ev_fork);
      if (ev_join) (void)hipEventDestroy(ev_join);
    }
  }
};

namespace {

inline int nblocks(long long n) { return (int)((n + dev::BLOCK - 1) / dev::BLOCK); }
inline int nblocks_wg(long long n, int wg) { return (int)((n + wg - 1) / wg); }
// instantiation of a composite pass for a level's workgroup size
#define WGK(K, T, wg) ((wg) == 1024 ? K<T, 1024> : (wg) == 512 ? K<T, 512> : K<T, 256>)
// passes with the level's composite operator: 1024-thread workgroups staging
// the gathered vector's LDS band when the level uses bands
#define LK(K, T, vl) ((vl) == 2 ? K<T, dev::LDS_WG, 2> : (vl) == 1 ? K<T, dev::LDS_WG, 1> : K<T, dev::LDS_WG, 0>)
#define AK(K, T, B) ((B).lds ? LK(K, T, (B).A.vlg) : WGK(K, T, (B).wg))
inline int a_wg(const DLevel &B) { return B.lds ? dev::LDS_WG : B.wg; }
// workgroups of a pass over `rows` rows with lg lanes each: one per LDS tile
// of ts slices, or one per wg threads
inline int a_blocks(long long rows, int lg, bool lds, int wg, int ts) {
  return lds ? nblocks_wg(rows << lg, 64 * ts) : nblocks_wg(rows << lg, wg);
}
template <typename T>
size_t a_lds(const DLevel &B) { return B.lds ? (size_t)B.band_max * sizeof(T) : 0; }

// Algorithmic bytes of one stored matrix entry: its value (w bytes) and its
// column index (2 bytes when the layout holds 16-bit columns, else 4).
inline double ent(const DSell &M, double w) { return w + (M.col16 ? 2.0 : 4.0); }

// ---------------------------------------------------------------- upload

amgdd_status upload_all(amgdd_ctx *h) {
  Setup &S = h->S;
  // the outer handle of a hybrid pair runs only FP64 V-cycle passes
  const bool fl = h->mixed() && h->hybrid_lt == 0;
  const size_t tsz = fl ? sizeof(float) : sizeof(double);
  amgdd_status st;
  const int nl = S.maxL() + 1;
  h->L.assign(nl, DLevel());
  h->nprob = (int)S.probs.size();
  h->N0 = S.prob_off.back();
  // f arena and gather map over all composite levels; r arena over all global levels
  std::vector<long long> foff(nl + 1, 0), roff(nl + 1, 0);
  for (int l = 0; l < nl; ++l) {
    foff[l + 1] = foff[l] + S.lv[l].NB;
    roff[l + 1] = roff[l] + S.lv[l].GN;
  }
  h->f_total = foff[nl];
  h->f_off1 = nl > 1 ? foff[1] : foff[nl];
  if ((st = h->alloc(&h->f_arena, foff[nl] * tsz))) return st;
  if (!S.grids.empty())
    if ((st = h->alloc(&h->r_arena, roff[nl] * tsz))) return st;
  {
    std::vector<int> src(foff[nl], -1);
    for (int l = 0; l < nl; ++l)
      for (int i = 0; i < S.lv[l].NB; ++i)
        if (S.lv[l].gsrc[i] >= 0) src[foff[l] + i] = (int)(roff[l] + S.lv[l].gsrc[i]);
    if ((st = h->upload(&h->gather_src, src.data(), src.size()))) return st;
  }
  for (int l = 0; l < nl; ++l) {
    BatchLevel &B = S.lv[l];
    DLevel &D = h->L[l];
    D.NRn = B.NRn;
    D.NBn = B.NBn;
    {
      // measurement: AMGDD_WG=256|512|1024 fixes the composite passes'
      // workgroup size on every level (otherwise the autotuner picks 256 or
      // 512 per level)
      const char *e = std::getenv("AMGDD_WG");
      const int v = e ? std::atoi(e) : dev::BLOCK;
      D.wg = (v == 512 || v == 1024) ? v : dev::BLOCK;
      if (e) h->wg_fixed = true;
    }
    D.band_max = B.band_max;
    D.rband_max = B.rband_max;
    {
      int lim = 0;
      const bool ok = hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, h->device) == hipSuccess;
      // bands that do not fit one workgroup's LDS: not used; nor with
      // four-wide FP64 steps (their LDS variant exceeds the register budget
      // of two workgroups per CU)
      if (!ok || (long long)D.band_max * (h->mixed() ? 4 : 8) > lim || (!h->mixed() && B.A.vlg == 2)) D.band_max = 0;
      if (!ok || (long long)D.rband_max * (h->mixed() ? 4 : 8) > lim || (!h->mixed() && B.Rt.vlg == 2))
        D.rband_max = 0;
    }
    {
      // measurement: AMGDD_LDS=1|0 stages the bands on every level that has
      // them / on none (otherwise the autotuner decides per level)
      const char *e = std::getenv("AMGDD_LDS");
      D.lds = e && std::atoi(e) == 1 && D.band_max > 0;
      D.rlds = e && std::atoi(e) == 1 && D.rband_max > 0;
      if (e) h->lds_fixed = true;
    }
    D.NB = B.NB;
    D.lg = B.lg;
    D.glg = B.glg;
    D.nnzA_r = B.nnzA_r;
    D.nnzA = B.nnzA;
    D.nnzP = B.nnzP;
    D.nnzR_n = B.nnzR_n;
    D.nnzR = B.nnzR;
    D.nnzGA_n = B.nnzGA_n;
    D.nnzGA = B.nnzGA;
    D.nnzGP = B.nnzGP;
    D.nnzGR_n = B.nnzGR_n;
    D.nnzGR = B.nnzGR;
    D.NRc = B.NRc;
    D.GNc = B.GNc;
    D.nnzA_c = B.nnzA_c;
    D.nnzGA_c = B.nnzGA_c;
    if (S.cf) {
      if ((st = h->upload((int8_t **)&D.cls, B.cls.data(), B.cls.size()))) return st;
      if ((st = h->upload((int8_t **)&D.gcls, B.gcls.data(), B.gcls.size()))) return st;
    }
    if ((st = h->upload_sell(D.A, B.A, fl))) return st;
    // with a reordered P every pass uses it (the original is not uploaded)
    if (B.pperm.empty()) {
      if ((st = h->upload_sell(D.P, B.P, fl))) return st;
    } else {
      if ((st = h->upload_sell(D.Pt, B.Pt, fl))) return st;
      std::vector<int> pos(B.pperm.size());
      for (size_t k = 0; k < pos.size(); ++k) pos[B.pperm[k]] = (int)k;
      if ((st = h->upload(&D.pperm, B.pperm.data(), B.pperm.size()))) return st;
      if ((st = h->upload(&D.ppos, pos.data(), pos.size()))) return st;
    }
    if ((st = h->upload_sell(D.R, B.R, fl))) return st;
    if (!B.rperm.empty()) {
      if ((st = h->upload_sell(D.Rt, B.Rt, fl))) return st;
      std::vector<int> pos(B.rperm.size());
      for (size_t k = 0; k < pos.size(); ++k) pos[B.rperm[k]] = (int)k;
      if ((st = h->upload(&D.rperm, B.rperm.data(), B.rperm.size()))) return st;
      if ((st = h->upload(&D.rpos, pos.data(), pos.size()))) return st;
    }
    if ((st = h->upload_vals(&D.dinv, B.dinv, fl))) return st;
    for (int k = 0; k < 2; ++k)
      if ((st = h->alloc(&D.u[k], (size_t)B.NB * tsz))) return st;
    if ((st = h->alloc(&D.t, (size_t)B.NB * tsz))) return st;
    if ((st = h->alloc(&D.sw, (size_t)B.NB * tsz))) return st;
    if (B.NB) {
      // t must be zero at ghost rows (never written); sw/u are always written before read
      HIP_TRY(hipMemset(D.t, 0, (size_t)B.NB * tsz));
      HIP_TRY(hipMemset(D.sw, 0, (size_t)B.NB * tsz));
      HIP_TRY(hipMemset(D.u[0], 0, (size_t)B.NB * tsz));
      HIP_TRY(hipMemset(D.u[1], 0, (size_t)B.NB * tsz));
    }
    D.f = (char *)h->f_arena + foff[l] * tsz;
    D.ncg = (int)B.cg_row0.size();
    if ((st = h->upload(&D.cg_row0, B.cg_row0.data(), B.cg_row0.size()))) return st;
    if ((st = h->upload(&D.cg_n, B.cg_n.data(), B.cg_n.size()))) return st;
    if ((st = h->upload(&D.cg_dense, B.cg_dense.data(), B.cg_dense.size()))) return st;
    for (int v : B.cg_n) D.cg_maxn = std::max(D.cg_maxn, v);
    // global
    D.GNn = B.GNn;
    D.GN = B.GN;
    if ((st = h->upload_sell(D.GA, B.GA, false))) return st;
    if ((st = h->upload_sell(D.GP, B.GP, false))) return st;
    if ((st = h->upload_sell(D.GRd, B.GR, false))) return st;
    if (fl) {
      if ((st = h->upload_sell(D.GRt, B.GR, true))) return st;
    } else {
      D.GRt = D.GRd;
    }
    if ((st = h->upload(&D.gdinv, B.gdinv.data(), B.gdinv.size()))) return st;
    for (int k = 0; k < 2; ++k)
      if ((st = h->alloc((void **)&D.ve[k], (size_t)B.GN * sizeof(double)))) return st;
    if ((st = h->alloc((void **)&D.vq, (size_t)B.GN * sizeof(double)))) return st;
    if ((st = h->alloc((void **)&D.vf, (size_t)B.GN * sizeof(double)))) return st;
    D.rt = h->r_arena ? (char *)h->r_arena + roff[l] * tsz : nullptr;
    D.ngc = (int)B.gc_row0.size();
    if ((st = h->upload(&D.gc_row0, B.gc_row0.data(), B.gc_row0.size()))) return st;
    if ((st = h->upload(&D.gc_n, B.gc_n.data(), B.gc_n.size()))) return st;
    if ((st = h->upload(&D.gc_dense, B.gc_dense.data(), B.gc_dense.size()))) return st;
    for (int v : B.gc_n) D.gc_maxn = std::max(D.gc_maxn, v);
  }
  if ((st = h->alloc((void **)&h->b, (size_t)h->N0 * sizeof(double)))) return st;
  if ((st = h->alloc((void **)&h->x, (size_t)h->N0 * sizeof(double)))) return st;
  HIP_TRY(hipMemset(h->b, 0, (size_t)h->N0 * sizeof(double)));
  HIP_TRY(hipMemset(h->x, 0, (size_t)h->N0 * sizeof(double)));
  h->nblk = (int)S.blk_row0.size();
  if ((st = h->upload(&h->blk_row0, S.blk_row0.data(), S.blk_row0.size()))) return st;
  if ((st = h->upload(&h->blk_row1, S.blk_row1.data(), S.blk_row1.size()))) return st;
  if ((st = h->upload(&h->prob_blk0, S.prob_blk0.data(), S.prob_blk0.size()))) return st;
  if ((st = h->alloc((void **)&h->partial, (size_t)h->nblk * sizeof(double)))) return st;
  if ((st = h->alloc((void **)&h->norm2, (size_t)h->nprob * sizeof(double)))) return st;
  HIP_TRY(hipHostMalloc((void **)&h->h_norm2, (size_t)h->nprob * sizeof(double), hipHostMallocDefault));
  if ((st = h->upload(&h->owner, S.owner.data(), S.owner.size()))) return st;
  if ((st = h->upload(&h->dense_A, S.dense_A.data(), S.dense_A.size()))) return st;
  if ((st = h->upload(&h->dense_inv, S.dense_inv.data(), S.dense_inv.size()))) return st;
  {
    const int nlev = nl, ng = (int)S.grids.size();
    std::vector<dev::GridLevel> glh((size_t)ng * nlev);
    for (size_t k = 0; k < glh.size(); ++k)
      glh[k] = dev::GridLevel{S.gl_rbeg[k], S.gl_nreal[k], S.gl_gbeg[k], S.gl_nghost[k]};
    if ((st = h->upload(&h->gl, glh.data(), glh.size()))) return st;
    if ((st = h->upload(&h->gridL, S.grid_L.data(), S.grid_L.size()))) return st;
    std::vector<int> gd(ng);
    for (int g = 0; g < ng; ++g) gd[g] = S.dense_off[S.grids[g].prob];
    if ((st = h->upload(&h->gdense, gd.data(), gd.size()))) return st;
    // tail grid lists, largest composite grid first (longest work starts first)
    std::vector<long long> work(ng, 0);
    for (int g = 0; g < ng; ++g)
      for (int l = 0; l < nlev; ++l) work[g] += S.gl_nreal[(size_t)g * nlev + l] + S.gl_nghost[(size_t)g * nlev + l];
    std::vector<int> order(ng);
    for (int g = 0; g < ng; ++g) order[g] = g;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work[a] > work[b]; });
    std::vector<int> lists;
    h->tail_off.assign(nlev, 0);
    h->tail_cnt.assign(nlev, 0);
    for (int lt = 0; lt < nlev; ++lt) {
      h->tail_off[lt] = (int)lists.size();
      for (int g : order)
        if (S.grid_L[g] >= lt) lists.push_back(g);
      h->tail_cnt[lt] = (int)lists.size() - h->tail_off[lt];
    }
    if ((st = h->upload(&h->tail_lists, lists.data(), lists.size()))) return st;
    for (auto &P : S.probs) h->tail_maxn = std::max(h->tail_maxn, P.H.A.back().nrows);
    // level pointer table in the composite precision
    auto fill = [&](auto tag) -> amgdd_status {
      using T = decltype(tag);
      std::vector<dev::LevelDev<T>> v(nlev);
      for (int l = 0; l < nlev; ++l) {
        DLevel &D = h->L[l];
        v[l] = dev::LevelDev<T>{D.A.as<T>(), D.P.as<T>(), D.R.as<T>(), (const T *)D.dinv, (T *)D.u[0], (T *)D.u[1],
                                (T *)D.t, (T *)D.sw, (T *)D.f, D.cls, D.Pt.as<T>(), D.Rt.as<T>(), D.ppos, D.rpos};
      }
      dev::LevelDev<T> *d = nullptr;
      amgdd_status s2 = h->upload(&d, v.data(), v.size());
      h->lvdev = d;
      return s2;
    };
    if ((st = fl ? fill(float()) : fill(double()))) return st;
  }
  HIP_TRY(hipDeviceSynchronize());
  return AMGDD_OK;
}

// ---------------------------------------------------------------- enqueue

#define LAUNCH(kernel, grid, block, shmem, stream, ...)                         \
  do {                                                                          \
    if ((grid) > 0) hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), shmem, stream, __VA_ARGS__); \
  } while (0)

// Launch with a profiling site: name, level and algorithmic bytes (the bytes
// expression is evaluated only while profiling).
#define PLAUNCH(h, name, level, bytes, kernel, grid, block, shmem, stream, ...)                     \
  do {                                                                                              \
    if ((grid) > 0) {                                                                               \
      Prof *_p = (h)->prof;                                                                         \
      int _k = _p ? _p->begin(name, (level) + (h)->lbase, (double)(bytes), stream, (int)(grid), (int)(block)) : -1; \
      hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), shmem, stream, __VA_ARGS__);              \
      if (_p) _p->end(_k, stream);                                                                  \
    }                                                                                               \
  } while (0)

// Fine residual and its per-problem squared norm.  vc: also e0 = r / d for the V-cycle.
template <typename T>
void enqueue_residual(amgdd_ctx *h, hipStream_t s, bool vc) {
  DLevel &D0 = h->L[0];
  if (vc)
    PLAUNCH(h, "resid_v", 0, D0.nnzGA * ent(D0.GA, 8.0) + h->N0 * 40.0, (dev::k_resid<double, true>), h->nblk, dev::BLOCK, 0, s, D0.GA.as<double>(), h->b, h->x, D0.vf, h->partial_buf(),
           h->blk_row0, h->blk_row1, D0.gdinv, D0.ve[0], (const signed char *)D0.gcls);
  else
    PLAUNCH(h, "resid", 0, D0.nnzGA * ent(D0.GA, 8.0) + h->N0 * (16.0 + sizeof(T)), (dev::k_resid<T, false>), h->nblk, dev::BLOCK, 0, s, D0.GA.as<double>(), h->b, h->x, (T *)D0.rt,
           h->partial_buf(), h->blk_row0, h->blk_row1, (const double *)nullptr, (double *)nullptr, (const signed char *)nullptr);
  PLAUNCH(h, "norm", 0, h->nblk * 8.0, dev::k_norm_final, h->nprob, dev::BLOCK, 0, s, h->partial_buf(), h->prob_blk0, h->norm2_buf());
  (void)hipMemcpyAsync(h->h_norm2, h->norm2_buf(), (size_t)h->nprob * sizeof(double), hipMemcpyDeviceToHost, s);
}

// Level-synchronous downsweep pass of level l (all grids normal at l, plus the
// coarsest solve of grids whose coarsest level is l) and its w pass.
template <typename T>
void enqueue_fac_down(amgdd_ctx *h, hipStream_t s, int *cur, int l, int first) {
  const int maxL = (int)h->L.size() - 1;
  const double w = sizeof(T);
  DLevel &B = h->L[l];
  T *uin = (T *)B.u[cur[l]], *uout = (T *)B.u[cur[l] ^ 1];
  const bool cf = B.cls != nullptr;
  const double nzc = cf ? (double)B.nnzA_c : (double)B.nnzA_r, nrc = cf ? B.NRc : B.NRn;
  if (l == 0) {
    if (first)
      PLAUNCH(h, "relax0", 0, nrc * 4.0 * w + (B.NBn - nrc) * w + (cf ? B.NRn : 0), dev::k_relax_zero<T>, nblocks(B.NBn), dev::BLOCK, 0, s, B.NRn, B.NBn, (const T *)B.f,
             (const T *)B.dinv, uout, (T *)B.t, (const signed char *)B.cls);
    else
      PLAUNCH(h, "relax_pre", 0, nzc * ent(B.A, w) + nrc * 4.0 * w + B.NBn * 2.0 * w + (cf ? B.NRn : 0), AK(dev::k_relax, T, B), a_blocks(B.NBn, B.lg, B.lds, a_wg(B), B.A.ts), a_wg(B), a_lds<T>(B), s, B.A.as<T>(), B.NRn, B.NBn, (const T *)B.f,
             (const T *)B.dinv, (const T *)uin, uout, (T *)B.t, 1, (const signed char *)B.cls, 1);
  } else {
    DLevel &Bp = h->L[l - 1];
    if (B.rperm) {
      // restriction in R's own row order, then the rest of the down pass at real rows
      const int rwg = B.rlds ? dev::LDS_WG : B.wg;
      PLAUNCH(h, "restrict_s", l, B.nnzR_n * ent(B.Rt, w) + Bp.NBn * w + B.NBn * (w + 4.0) + (B.NBn - B.NRn) * w,
              (B.rlds ? LK(dev::k_restrict_rows, T, B.Rt.vlg) : WGK(dev::k_restrict_rows, T, B.wg)),
              a_blocks(B.NBn, B.Rt.lg, B.rlds, rwg, B.Rt.ts), rwg, B.rlds ? (size_t)B.rband_max * sizeof(T) : 0, s,
              B.Rt.as<T>(), B.rperm, B.NBn, B.NRn, (const T *)Bp.sw, (T *)B.sw, uout);
      PLAUNCH(h, "down", l, (first ? 0.0 : B.nnzA_r * ent(B.A, w) + B.NBn * w) + B.NRn * ((first ? 4.0 : 5.0) + 2.0) * w + (cf ? B.NRn : 0),
              AK(dev::k_down_real, T, B), a_blocks(B.NRn, B.lg, B.lds, a_wg(B), B.A.ts), a_wg(B), a_lds<T>(B), s, B.A.as<T>(), B.NRn,
              (const T *)B.sw, (T *)B.f, (const T *)B.dinv, (const T *)uin, uout, (T *)B.t, first, (const signed char *)B.cls);
    } else
    PLAUNCH(h, "down", l, B.nnzR_n * ent(B.R, w) + Bp.NBn * w + B.NBn * 2.0 * w + (first ? 0.0 : B.nnzA_r * ent(B.A, w) + B.NBn * w) + B.NRn * (first ? 4.0 : 5.0) * w + (cf ? B.NRn : 0), WGK(dev::k_down, T, B.wg), nblocks_wg((long long)B.NBn << B.lg, B.wg), B.wg, 0, s, B.R.as<T>(), B.A.as<T>(), B.NRn, B.NBn,
           (const T *)Bp.sw, (T *)B.sw, (T *)B.f, (const T *)B.dinv, (const T *)uin, uout, (T *)B.t, first, (const signed char *)B.cls);
    PLAUNCH(h, "coarse", l, (B.nnzR - B.nnzR_n) * ent(B.R, w) + (B.NB - B.NBn) * 3.0 * w, dev::k_coarse<T>, B.ncg, dev::BLOCK, 2 * B.cg_maxn * sizeof(double), s, B.R.as<T>(), 1,
           (const T *)Bp.sw, (T *)B.f, (const T *)uin, uout, h->dense_A, h->dense_inv, B.cg_row0, B.cg_n,
           B.cg_dense, 0, first, uin);
  }
  cur[l] ^= 1;
  if (cf && B.NBn > 0 && l < maxL) {
    // F half of the CF sweep (normal grids only; the coarse grids' rows of
    // this level keep their solve, copied along)
    const int nrf = B.NRn - B.NRc;
    T *ui = (T *)B.u[cur[l]], *uo = (T *)B.u[cur[l] ^ 1];
    PLAUNCH(h, "relax_f", l, (B.nnzA_r - B.nnzA_c) * ent(B.A, w) + nrf * 4.0 * w + B.NB * 2.0 * w + B.NRn, AK(dev::k_relax, T, B), a_blocks(B.NB, B.lg, B.lds, a_wg(B), B.A.ts), a_wg(B), a_lds<T>(B), s, B.A.as<T>(), B.NRn, B.NB, (const T *)B.f,
            (const T *)B.dinv, (const T *)ui, uo, (T *)B.t, 1, (const signed char *)B.cls, -1);
    cur[l] ^= 1;
  }
  if (B.NBn > 0 && l < maxL)
    PLAUNCH(h, "w", l, B.nnzA * ent(B.A, w) + B.NBn * (l > 0 ? 3.0 : 2.0) * w, AK(dev::k_w, T, B), a_blocks(B.NBn, B.lg, B.lds, a_wg(B), B.A.ts), a_wg(B), a_lds<T>(B), s, B.A.as<T>(), B.NBn, (T *)B.sw, (const T *)B.t, l > 0);
}

template <typename T>
void enqueue_fac_up(amgdd_ctx *h, hipStream_t s, int *cur, int l) {
  const double w = sizeof(T);
  DLevel &B = h->L[l];
  if (B.NBn == 0) return;
  DLevel &Bc = h->L[l + 1];
  if (B.pperm)
    PLAUNCH(h, "interp", l, B.nnzP * ent(B.Pt, w) + B.NBn * (2.0 * w + 4.0) + Bc.NB * w,
            WGK(dev::k_interp_rows, T, B.wg), nblocks_wg((long long)B.NBn << B.Pt.lg, B.wg), B.wg, 0, s, B.Pt.as<T>(),
            B.pperm, B.NBn, (T *)B.u[cur[l]], (const T *)Bc.u[cur[l + 1]]);
  else
  PLAUNCH(h, "interp", l, B.nnzP * ent(B.P, w) + B.NBn * 2.0 * w + Bc.NB * w, WGK(dev::k_interp, T, B.wg), nblocks_wg((long long)B.NBn << B.P.lg, B.wg), B.wg, 0, s, B.P.as<T>(), B.NBn, (T *)B.u[cur[l]],
         (const T *)Bc.u[cur[l + 1]]);
  if (B.cls) {
    const int nrf = B.NRn - B.NRc;
    PLAUNCH(h, "relax_post_f", l, (B.nnzA_r - B.nnzA_c) * ent(B.A, w) + nrf * 3.0 * w + B.NRc * w + B.NB * 2.0 * w + B.NRn, AK(dev::k_relax, T, B), a_blocks(B.NB, B.lg, B.lds, a_wg(B), B.A.ts), a_wg(B), a_lds<T>(B), s, B.A.as<T>(), B.NRn, B.NB, (const T *)B.f,
            (const T *)B.dinv, (const T *)B.u[cur[l]], (T *)B.u[cur[l] ^ 1], (T *)B.t, 0, (const signed char *)B.cls, -1);
    cur[l] ^= 1;
    PLAUNCH(h, "relax_post_c", l, B.nnzA_c * ent(B.A, w) + B.NRc * 4.0 * w + B.NB * 2.0 * w + B.NRn, AK(dev::k_relax, T, B), a_blocks(B.NB, B.lg, B.lds, a_wg(B), B.A.ts), a_wg(B), a_lds<T>(B), s, B.A.as<T>(), B.NRn, B.NB, (const T *)B.f,
            (const T *)B.dinv, (const T *)B.u[cur[l]], (T *)B.u[cur[l] ^ 1], (T *)B.t, 1, (const signed char *)B.cls, 1);
  } else {
    PLAUNCH(h, "relax_post", l, B.nnzA_r * ent(B.A, w) + B.NRn * 3.0 * w + B.NB * 2.0 * w, AK(dev::k_relax, T, B), a_blocks(B.NB, B.lg, B.lds, a_wg(B), B.A.ts), a_wg(B), a_lds<T>(B), s, B.A.as<T>(), B.NRn, B.NB, (const T *)B.f,
           (const T *)B.dinv, (const T *)B.u[cur[l]], (T *)B.u[cur[l] ^ 1], (T *)B.t, 0, (const signed char *)nullptr, 1);
  }
  cur[l] ^= 1;
}

// Algorithmic bytes of the persistent tail over levels >= lt (one cycle).
template <typename T>
double tail_bytes(amgdd_ctx *h, int lt, int first) {
  const double w = sizeof(T);
  double b = 0;
  const int maxL = (int)h->L.size() - 1;
  for (int l = lt; l <= maxL; ++l) {
    DLevel &B = h->L[l];
    if (l == 0) b += first ? B.NRn * 4.0 * w + (B.NBn - B.NRn) * w : B.nnzA_r * ent(B.A, w) + B.NRn * 4.0 * w + B.NBn * 2.0 * w;
    else b += (B.rperm ? B.nnzR_n * ent(B.Rt, w) + (B.nnzR - B.nnzR_n) * ent(B.R, w) : B.nnzR * ent(B.R, w)) + h->L[l - 1].NBn * w + B.NBn * 2.0 * w + (first ? 0.0 : B.nnzA_r * ent(B.A, w) + B.NBn * w) + B.NRn * (first ? 4.0 : 5.0) * w;
    if (l < maxL) {
      b += B.nnzA * ent(B.A, w) + B.NBn * (l > 0 ? 3.0 : 2.0) * w;
      b += B.nnzP * ent(B.pperm ? B.Pt : B.P, w) + B.NBn * 2.0 * w + h->L[l + 1].NB * w;
      b += B.nnzA_r * ent(B.A, w) + B.NRn * 3.0 * w + B.NB * 2.0 * w;
      // CF order: the extra half-sweeps re-read and re-write the vectors
      if (B.cls) b += 2.0 * (B.NBn * 2.0 * w + B.NRn) + (B.nnzA_r - B.nnzA_c) * ent(B.A, w);
    }
  }
  return b;
}

template <typename T>
void enqueue_tail(amgdd_ctx *h, hipStream_t s, int lt, int ncycles, int first) {
  const int ngr = h->tail_cnt[lt];
  const int nlev = (int)h->L.size();
  PLAUNCH(h, "fac_tail", lt, ncycles * tail_bytes<T>(h, lt, first), dev::k_fac_tail<T>, ngr, h->sched_block,
          2 * h->tail_maxn * sizeof(double), s, (const dev::LevelDev<T> *)h->lvdev, h->gl, nlev,
          h->tail_lists + h->tail_off[lt], h->gridL, h->gdense, h->dense_A, h->dense_inv, lt, ncycles, first);
}

// n_fac AlgFAC cycles over every composite grid.  Levels below the schedule's
// cut level run one launch per pass over all grids; levels from the cut down
// run in one persistent launch per cycle (the whole AlgFAC in one launch when
// the cut is level 0).  At the start and end of each cycle every level's u is
// in buffer 0 (cur[l] == 0).
template <typename T>
// skip0: the first cycle's level-0 down passes are already enqueued.
void enqueue_fac(amgdd_ctx *h, hipStream_t s, int *cur, bool skip0 = false) {
  const int maxL = (int)h->L.size() - 1;
  const int nfac = h->prm.n_fac;
  const int lt = h->sched_level < 0 ? maxL + 1 : h->sched_level;
  if (lt == 0) {
    enqueue_tail<T>(h, s, 0, nfac, 1);
    return;
  }
  for (int c = 0; c < nfac; ++c) {
    const int first = c == 0;
    for (int l = first && skip0 ? 1 : 0; l < std::min(lt, maxL + 1); ++l) enqueue_fac_down<T>(h, s, cur, l, first);
    if (lt <= maxL) enqueue_tail<T>(h, s, lt, 1, first);
    for (int l = std::min(lt, maxL) - 1; l >= 0; --l) enqueue_fac_up<T>(h, s, cur, l);
  }
}

// One AMG-DD cycle from a current residual r_0 (already in L[0].rt): the
// restriction chain, composite right-hand sides, n_fac AlgFAC cycles and the
// patch of u_0 into x (x += u_0; assign: x = u_0, a cycle started from zero).
template <typename T>
void enqueue_dd_core(amgdd_ctx *h, hipStream_t s, double *x, bool assign) {
  const int maxL = (int)h->L.size() - 1;
  const int lt = h->sched_level < 0 ? maxL + 1 : h->sched_level;
  std::vector<int> cur(maxL + 1, 0);
  // Two branches when the first cycle starts with level-synchronous level-0
  // passes: those need only the level-0 right-hand sides, so the restriction
  // chain and the coarser right-hand sides run beside them on the side stream
  // and join before level 1 (a fork/join in a captured graph).  Profiling
  // keeps one stream so every launch is timed alone.
  const bool fork = h->side && h->overlap && !h->prof && maxL >= 1 && lt > 0;
  hipStream_t sr = s;
  if (fork) {
    (void)hipEventRecord(h->ev_fork, s);
    (void)hipStreamWaitEvent(h->side, h->ev_fork, 0);
    sr = h->side;
  }
  for (int l = 1; l <= maxL; ++l) {
    DLevel &B = h->L[l];
    PLAUNCH(h, "restrict", l, B.nnzGR * ent(B.GRt, sizeof(T)) + (h->L[l - 1].GN + B.GN) * (double)sizeof(T), dev::k_spmv<T>, nblocks((long long)B.GN << B.glg), dev::BLOCK, 0, sr, B.GRt.as<T>(), B.GN, (const T *)h->L[l - 1].rt, (T *)B.rt);
  }
  if (fork) {
    const long long n1 = h->f_total - h->f_off1;
    PLAUNCH(h, "gather", 1, n1 * 4.0 + n1 * 2.0 * sizeof(T), dev::k_gather<T>, nblocks(n1), dev::BLOCK, 0, sr, (int)n1, h->gather_src + h->f_off1,
           (const T *)h->r_arena, (T *)h->f_arena + h->f_off1);
    (void)hipEventRecord(h->ev_join, sr);
    PLAUNCH(h, "gather", 0, h->f_off1 * (4.0 + 2.0 * sizeof(T)), dev::k_gather<T>, nblocks(h->f_off1), dev::BLOCK, 0, s, (int)h->f_off1, h->gather_src,
           (const T *)h->r_arena, (T *)h->f_arena);
    enqueue_fac_down<T>(h, s, cur.data(), 0, 1);
    (void)hipStreamWaitEvent(s, h->ev_join, 0);
    enqueue_fac<T>(h, s, cur.data(), true);
  } else {
    PLAUNCH(h, "gather", 0, h->f_total * 4.0 + h->S.composite_real_rows * 2.0 * sizeof(T), dev::k_gather<T>, nblocks(h->f_total), dev::BLOCK, 0, s, (int)h->f_total, h->gather_src,
           (const T *)h->r_arena, (T *)h->f_arena);
    enqueue_fac<T>(h, s, cur.data());
  }
  if (assign)
    PLAUNCH(h, "patch", 0, h->N0 * (12.0 + sizeof(T)), (dev::k_patch<T, true>), nblocks(h->N0), dev::BLOCK, 0, s, h->N0, x, h->owner, (const T *)h->L[0].u[cur[0]]);
  else
    PLAUNCH(h, "patch", 0, h->N0 * (20.0 + sizeof(T)), dev::k_patch<T>, nblocks(h->N0), dev::BLOCK, 0, s, h->N0, x, h->owner, (const T *)h->L[0].u[cur[0]]);
}

// One AMG-DD iteration (Algorithm 2) from r_0 in L[0].rt, then the new
// residual and its norms.
template <typename T>
void enqueue_dd_iteration(amgdd_ctx *h, hipStream_t s) {
  enqueue_dd_core<T>(h, s, h->x, false);
  enqueue_residual<T>(h, s, false);
}

// V-cycle downsweep passes of levels 0..lv-1 in correction form: residual
// q_l = f_l - A_l e_l, then f_{l+1} = R_l q_l with the first relaxation from
// zero e_{l+1} = f_{l+1} / d (problems continuing below l+1) or the direct
// solve (problems whose coarsest level is l+1).  hyb (lv = L~ of a hybrid
// handle): on the last level, the restricted residual of the problems that
// continue goes, in the level-L~ handle's precision, into that handle's fine
// residual instead.  CF order: the first relaxation from zero is the C half;
// an F half-sweep follows on every relaxed level (level 0 included).
void enqueue_v_relax(amgdd_ctx *h, hipStream_t s, int *cur, int l, int want, const char *name) {
  DLevel &B = h->L[l];
  const double nz = want == 1 ? (double)B.nnzGA_c : (double)(B.nnzGA_n - B.nnzGA_c);
  const double nr = want == 1 ? B.GNc : B.GNn - B.GNc;
  PLAUNCH(h, name, l, nz * ent(B.GA, 8.0) + nr * 16.0 + B.GN * 16.0 + B.GNn, dev::k_relax<double>, nblocks((long long)B.GN << B.glg), dev::BLOCK, 0, s, B.GA.as<double>(), B.GNn, B.GN, B.vf, B.gdinv,
          B.ve[cur[l]], B.ve[cur[l] ^ 1], (double *)nullptr, 2, (const signed char *)B.gcls, want);
  cur[l] ^= 1;
}

template <typename T>
void enqueue_v_down(amgdd_ctx *h, hipStream_t s, int *cur, int lv, bool hyb) {
  const bool cf = h->cf();
  if (cf && lv > 0) enqueue_v_relax(h, s, cur, 0, -1, "vrelax_f");
  for (int l = 0; l < lv; ++l) {
    DLevel &B = h->L[l];
    DLevel &Bc = h->L[l + 1];
    if (B.GNn == 0) continue;
    PLAUNCH(h, "vresid", l, B.nnzGA_n * ent(B.GA, 8.0) + B.GN * 8.0 + B.GNn * 16.0, dev::k_vresid<double>, nblocks((long long)B.GNn << B.glg), dev::BLOCK, 0, s, B.GA.as<double>(), B.GNn, B.vf, B.ve[cur[l]], B.vq);
    if (hyb && l + 1 == lv)
      PLAUNCH(h, "hrestrict", l + 1, Bc.nnzGR_n * ent(Bc.GRd, 8.0) + B.GNn * 8.0 + Bc.GNn * (double)sizeof(T), (dev::k_spmv<double, T>), nblocks((long long)Bc.GNn << Bc.glg), dev::BLOCK, 0, s, Bc.GRd.as<double>(), Bc.GNn,
              (const double *)B.vq, (T *)h->inner->L[0].rt);
    else
      PLAUNCH(h, "vdown", l + 1, Bc.nnzGR_n * ent(Bc.GRd, 8.0) + B.GNn * 8.0 + Bc.GNn * 24.0 + (cf ? Bc.GNn : 0), dev::k_vdown<double>, nblocks((long long)Bc.GNn << Bc.glg), dev::BLOCK, 0, s, Bc.GRd.as<double>(), Bc.GNn, B.vq, Bc.vf,
             Bc.gdinv, Bc.ve[cur[l + 1]], (const signed char *)Bc.gcls);
    PLAUNCH(h, "vcoarse", l + 1, (Bc.nnzGR - Bc.nnzGR_n) * ent(Bc.GRd, 8.0) + (Bc.GN - Bc.GNn) * 16.0, dev::k_coarse<double>, Bc.ngc, dev::BLOCK, 2 * Bc.gc_maxn * sizeof(double), s, Bc.GRd.as<double>(), 1, B.vq,
           Bc.vf, Bc.ve[cur[l + 1]], Bc.ve[cur[l + 1]], h->dense_A, h->dense_inv, Bc.gc_row0, Bc.gc_n, Bc.gc_dense, 1,
           1, (double *)nullptr);
    if (cf && !(hyb && l + 1 == lv) && Bc.GNn > 0) enqueue_v_relax(h, s, cur, l + 1, -1, "vrelax_f");
  }
}

// V-cycle upsweep passes of levels lv-1..0: e_l += P_l e_{l+1}, relaxation;
// on level 0 the final relaxation is fused with x += e_0.
void enqueue_v_up(amgdd_ctx *h, hipStream_t s, int *cur, int lv) {
  for (int l = lv - 1; l >= 0; --l) {
    DLevel &B = h->L[l];
    DLevel &Bc = h->L[l + 1];
    if (B.GNn == 0) continue;
    PLAUNCH(h, "vinterp", l, B.nnzGP * ent(B.GP, 8.0) + B.GNn * 16.0 + Bc.GN * 8.0, dev::k_interp<double>, nblocks((long long)B.GNn << B.GP.lg), dev::BLOCK, 0, s, B.GP.as<double>(), B.GNn, B.ve[cur[l]],
           Bc.ve[cur[l + 1]]);
    const bool cf = B.gcls != nullptr;
    if (cf) enqueue_v_relax(h, s, cur, l, -1, "vrelax_fu");
    if (l > 0) {
      if (cf) {
        enqueue_v_relax(h, s, cur, l, 1, "vrelax_cu");
      } else {
        PLAUNCH(h, "vrelax", l, B.nnzGA_n * ent(B.GA, 8.0) + B.GNn * 16.0 + B.GN * 16.0, dev::k_relax<double>, nblocks((long long)B.GN << B.glg), dev::BLOCK, 0, s, B.GA.as<double>(), B.GNn, B.GN, B.vf, B.gdinv,
               B.ve[cur[l]], B.ve[cur[l] ^ 1], (double *)nullptr, 2, (const signed char *)nullptr, 1);
        cur[l] ^= 1;
      }
    } else {
      PLAUNCH(h, "vfinal", 0, (cf ? B.nnzGA_c : B.nnzGA_n) * ent(B.GA, 8.0) + B.GNn * 40.0 + (cf ? B.GNn : 0), dev::k_vfinal, nblocks(B.GNn), dev::BLOCK, 0, s, B.GA.as<double>(), B.GNn, B.vf, B.gdinv, B.ve[cur[0]],
             h->x, (const signed char *)B.gcls);
    }
  }
}

// One V(1,1) cycle in correction form from r_0 (L[0].vf) and e_0 = r_0 / d (L[0].ve[0]).
void enqueue_v_iteration(amgdd_ctx *h, hipStream_t s) {
  const int maxL = (int)h->L.size() - 1;
  std::vector<int> cur(maxL + 1, 0);
  enqueue_v_down<double>(h, s, cur.data(), maxL, false);
  enqueue_v_up(h, s, cur.data(), maxL);
  enqueue_residual<double>(h, s, true);
}

// One hybrid AMG-DD V(1,1) cycle (Algorithm 3) in correction form, same start
// as the V-cycle: downsweep to L~; one AMG-DD cycle from zero on the level-L~
// problems (their fine residual is the restricted one) whose iterate becomes
// e_L~ of those problems (the others took the direct solve on L~); upsweep.
template <typename T>
void enqueue_hybrid_iteration(amgdd_ctx *h, hipStream_t s) {
  const int lt = h->hybrid_lt;
  std::vector<int> cur(lt + 1, 0);
  enqueue_v_down<T>(h, s, cur.data(), lt, true);
  enqueue_dd_core<T>(h->inner, s, h->L[lt].ve[cur[lt]], true);
  enqueue_v_up(h, s, cur.data(), lt);
  enqueue_residual<double>(h, s, true);
}

void enqueue_hybrid(amgdd_ctx *h, hipStream_t s) {
  if (h->inner->mixed()) enqueue_hybrid_iteration<float>(h, s);
  else enqueue_hybrid_iteration<double>(h, s);
}

amgdd_status capture(amgdd_ctx *h, bool dd, hipGraph_t *gr, hipGraphExec_t *ex) {
  TraceRange tr(dd ? "amgdd: capture AMG-DD iteration" : "amgdd: capture V-cycle");
  HIP_TRY(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
  if (dd && h->inner) {
    enqueue_hybrid(h, h->cap_stream);
  } else if (dd) {
    if (h->mixed()) enqueue_dd_iteration<float>(h, h->cap_stream);
    else enqueue_dd_iteration<double>(h, h->cap_stream);
  } else {
    enqueue_v_iteration(h, h->cap_stream);
  }
  HIP_TRY(hipStreamEndCapture(h->cap_stream, gr));
  HIP_TRY(hipGraphInstantiate(ex, *gr, nullptr, nullptr, 0));
  return AMGDD_OK;
}

// ---------------------------------------------------------------- schedule cache
//
// The autotuner's choice depends only on the layout (levels, rows, stored
// entries and lane groupings of every batched matrix, grids, precision, cycles,
// relaxation order), on the device and on the kernels, so it is cached under a
// 64-bit FNV-1a hash of those: in memory for the process, and in a JSON file
// (one entry per line) that later processes read.  The file is
// $AMGDD_TUNE_CACHE, or $HOME/.cache/amgdd/schedules.json when that is unset;
// AMGDD_TUNE_CACHE=off disables the file.  The kernels enter the key through
// the library's build time, so a rebuilt library tunes again.

struct SchedKey {
  uint64_t h = 1469598103934665603ull;
  void add(const void *p, size_t n) {
    const unsigned char *c = (const unsigned char *)p;
    for (size_t i = 0; i < n; ++i) { h ^= c[i]; h *= 1099511628211ull; }
  }
  template <typename V>
  void add(V v) { add(&v, sizeof(v)); }
  void add_str(const char *s) { add(s, std::strlen(s)); }
};

uint64_t schedule_key(amgdd_ctx *h) {
  SchedKey k;
  k.add_str(__DATE__ " " __TIME__);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, h->device) == hipSuccess) {
    k.add_str(prop.gcnArchName);
    k.add(prop.multiProcessorCount);
  }
  k.add(h->prm.precision);
  k.add(h->prm.n_fac);
  k.add(h->prm.tail_level);
  k.add(h->prm.tail_block);
  k.add((int)h->S.cf);
  k.add((int)h->S.grids.size());
  k.add(h->tail_maxn);
  k.add((int)h->wg_fixed);
  k.add((int)h->lds_fixed);
  for (const DLevel &D : h->L) {
    k.add(D.NRn); k.add(D.NBn); k.add(D.NB); k.add(D.lg); k.add(D.ncg); k.add(D.cg_maxn);
    for (const DSell *M : {&D.A, &D.P, &D.R, &D.Pt, &D.Rt}) { k.add(M->entries); k.add(M->lg); k.add(M->vlg); k.add((int)(M->col16 != nullptr)); }
    k.add(D.nnzA); k.add(D.nnzP); k.add(D.nnzR); k.add(D.band_max); k.add(D.A.ntiles); k.add(D.rband_max);
  }
  for (int c : h->tail_cnt) k.add(c);
  return k.h;
}

struct SchedEntry {
  int level, block;
  double ms;
  unsigned wide = 0;  // levels whose composite passes use 512-thread workgroups (bit l)
  unsigned lds = 0;   // levels whose operator passes stage LDS bands (bit l)
  unsigned rlds = 0;  // levels whose restriction pass stages LDS bands (bit l)
};

std::string sched_cache_path() {
  const char *e = std::getenv("AMGDD_TUNE_CACHE");
  if (e && std::strcmp(e, "off") == 0) return std::string();
  if (e && e[0]) return e;
  const char *home = std::getenv("HOME");
  if (!home || !home[0]) return std::string();
  return std::string(home) + "/.cache/amgdd/schedules.json";
}

// Entries of the cache file (lines of the form  "key": [level, block, ms],).
std::vector<std::pair<uint64_t, SchedEntry>> read_sched_file(const std::string &path) {
  std::vector<std::pair<uint64_t, SchedEntry>> out;
  FILE *f = path.empty() ? nullptr : std::fopen(path.c_str(), "r");
  if (!f) return out;
  char line[512];
  while (std::fgets(line, sizeof line, f)) {
    unsigned long long key;
    SchedEntry e;
    const int k = std::sscanf(line, " \"%16llx\": [%d, %d, %lf, %u, %u, %u]", &key, &e.level, &e.block, &e.ms,
                              &e.wide, &e.lds, &e.rlds);
    if (k >= 4) {
      if (k == 4) e.wide = 0;
      if (k <= 5) e.lds = 0;
      if (k <= 6) e.rlds = 0;
      out.push_back({(uint64_t)key, e});
    }
  }
  std::fclose(f);
  return out;
}

// Adds or replaces one entry; written to a temporary file and renamed over the
// old one, so readers never see a partial file.  Failures are silent (the
// cache is an optimisation).
void write_sched_file(const std::string &path, uint64_t key, const SchedEntry &e) {
  if (path.empty()) return;
  auto ent = read_sched_file(path);
  bool found = false;
  for (auto &x : ent)
    if (x.first == key) { x.second = e; found = true; }
  if (!found) ent.push_back({key, e});
  const size_t slash = path.rfind('/');
  if (slash != std::string::npos && slash > 0) {
    // create the directory chain
    for (size_t pos = 1; pos <= slash; ++pos)
      if (pos == slash || path[pos] == '/') (void)mkdir(path.substr(0, pos).c_str(), 0755);
  }
  const std::string tmp = path + ".tmp" + std::to_string((long long)getpid());
  FILE *f = std::fopen(tmp.c_str(), "w");
  if (!f) return;
  std::fprintf(f, "{\n");
  for (size_t i = 0; i < ent.size(); ++i)
    std::fprintf(f, "\"%016llx\": [%d, %d, %.6f, %u, %u, %u]%s\n", (unsigned long long)ent[i].first,
                 ent[i].second.level, ent[i].second.block, ent[i].second.ms, ent[i].second.wide, ent[i].second.lds,
                 ent[i].second.rlds, i + 1 < ent.size() ? "," : "");
  std::fprintf(f, "}\n");
  const bool ok = std::fclose(f) == 0;
  if (!ok || std::rename(tmp.c_str(), path.c_str()) != 0) (void)std::remove(tmp.c_str());
}

std::mutex g_sched_mu;
std::vector<std::pair<uint64_t, SchedEntry>> g_sched_mem;

bool sched_lookup(uint64_t key, SchedEntry &e) {
  std::lock_guard<std::mutex> lk(g_sched_mu);
  for (auto &x : g_sched_mem)
    if (x.first == key) { e = x.second; return true; }
  for (auto &x : read_sched_file(sched_cache_path()))
    if (x.first == key) {
      e = x.second;
      g_sched_mem.push_back(x);
      return true;
    }
  return false;
}

void sched_store(uint64_t key, const SchedEntry &e) {
  std::lock_guard<std::mutex> lk(g_sched_mu);
  bool found = false;
  for (auto &x : g_sched_mem)
    if (x.first == key) { x.second = e; found = true; }
  if (!found) g_sched_mem.push_back({key, e});
  write_sched_file(sched_cache_path(), key, e);
}

// Project autotuner: time one graph-replayed AMG-DD iteration for every
// schedule candidate (cut level x workgroup size) on the caller's data and keep
// the fastest.  Every candidate computes identical results, so the choice only
// affects time.  The iterate is restored afterwards.
amgdd_status autotune(amgdd_ctx *h) {
  TraceRange tr("amgdd: autotune");
  const double t0 = now_s();
  const int nlev = (int)h->L.size();
  const uint64_t key = schedule_key(h);
  // per-level modes of the level-synchronous passes: 512-thread workgroups
  // (bit l of m.w), LDS bands for the operator passes (bit l of m.a) and for
  // the restriction pass (bit l of m.r)
  struct Modes {
    unsigned w = 0, a = 0, r = 0;
  };
  auto set_modes = [&](Modes m) {
    for (int l = 0; l < nlev; ++l) {
      if (!h->wg_fixed) h->L[l].wg = l < 32 && (m.w >> l) & 1u ? 512 : dev::BLOCK;
      if (!h->lds_fixed) {
        h->L[l].lds = l < 32 && (m.a >> l) & 1u && h->L[l].band_max > 0;
        h->L[l].rlds = l < 32 && (m.r >> l) & 1u && h->L[l].rband_max > 0;
      }
    }
  };
  {
    SchedEntry e;
    if (sched_lookup(key, e) && e.level >= -1 && e.level < nlev && (e.block == 256 || e.block == 512 || e.block == 1024)) {
      h->sched_level = e.level;
      h->sched_block = e.block;
      set_modes(Modes{e.wide, e.lds, e.rlds});
      h->sched_cached = 1;
      h->autotune_s = now_s() - t0;
      return AMGDD_OK;
    }
  }
  hipStream_t s = h->stream;
  std::vector<int> levels, blocks;
  if (h->prm.tail_level >= -1) levels.push_back(h->prm.tail_level >= nlev ? -1 : h->prm.tail_level);
  else {
    levels.push_back(-1);
    for (int l = nlev - 1; l >= 0; --l) levels.push_back(l);
  }
  if (h->prm.tail_block > 0) blocks.push_back(h->prm.tail_block);
  else blocks = {256, 512, 1024};
  double *xsave = nullptr;
  amgdd_status st = h->alloc((void **)&xsave, (size_t)h->N0 * sizeof(double));
  if (st) return st;
  HIP_TRY(hipMemcpyAsync(xsave, h->x, (size_t)h->N0 * sizeof(double), hipMemcpyDeviceToDevice, s));
  if (h->mixed()) enqueue_residual<float>(h, s, false);
  else enqueue_residual<double>(h, s, false);
  // host-clock time of three replays of one captured iteration (after one
  // warm replay) with the handle's current schedule
  // one captured iteration of the handle's current schedule, and the host-clock
  // time of three replays of it (after one warm replay)
  struct Captured {
    hipGraph_t g = nullptr;
    hipGraphExec_t e = nullptr;
    void drop() {
      if (e) (void)hipGraphExecDestroy(e);
      if (g) (void)hipGraphDestroy(g);
      e = nullptr;
      g = nullptr;
    }
  };
  auto time_exec = [&](hipGraphExec_t ex, double &ms) -> amgdd_status {
    HIP_TRY(hipGraphLaunch(ex, s));
    HIP_TRY(hipStreamSynchronize(s));
    const double tc = now_s();
    for (int r = 0; r < 3; ++r) HIP_TRY(hipGraphLaunch(ex, s));
    HIP_TRY(hipStreamSynchronize(s));
    ms = (now_s() - tc) * 1e3;
    return AMGDD_OK;
  };
  // levels of fewer rows than this take a few microseconds per pass whichever
  // mode they run in: not tuned, left in the default modes
  constexpr int kTuneMinRows = 32768;
  // first the cut level and the tail's workgroup size, with LDS bands on the
  // larger levels that have them (the modes that usually win there: cuts are
  // compared against level-synchronous passes as the second phase is likely
  // to leave them, not against their slowest form)
  Modes base;
  for (int l = 0; l < nlev && l < 32; ++l) {
    if (h->lds_fixed || h->L[l].NBn < kTuneMinRows) continue;
    if (h->L[l].band_max > 0) base.a |= 1u << l;
    if (h->L[l].rband_max > 0 && h->L[l].rperm) base.r |= 1u << l;
  }
  double best = 1e300;
  int best_l = -1, best_b = 256;
  set_modes(base);
  for (int lt : levels)
    for (int bs : blocks) {
      if (lt < 0 && bs != blocks[0]) continue;
      h->sched_level = lt;
      h->sched_block = bs;
      Captured c;
      double ms = 0;
      st = capture(h, true, &c.g, &c.e);
      if (!st) st = time_exec(c.e, ms);
      c.drop();
      if (st) return st;
      if (ms < best) { best = ms; best_l = lt; best_b = bs; }
    }
  h->sched_level = best_l;
  h->sched_block = best_b;
  {
    // levels from the cut on run in the per-grid tail kernel: no modes
    const int cut = best_l < 0 ? nlev : best_l;
    const unsigned keep = cut >= 32 ? ~0u : (1u << cut) - 1u;
    base.a &= keep;
    base.r &= keep;
    set_modes(base);
  }
  // then, level by level above the cut, the modes of its level-synchronous
  // passes: the current modes, and each of them with one mode switched —
  // 512-thread workgroups (more rows per workgroup share the L1 cache's
  // gathered vector lines), LDS bands for the operator passes, LDS bands for
  // the restriction.  Each candidate is captured once; the captures are timed
  // alternately, twice each, and a candidate is kept when its faster time
  // beats the current one's by more than 0.1%.  Every mode computes the same
  // sums in the same order.
  Modes cur = base;
  if (!h->wg_fixed || !h->lds_fixed) {
    const int cut = best_l < 0 ? nlev : best_l;
    for (int l = 0; l < std::min(cut, nlev) && l < 32; ++l) {
      if (h->L[l].NBn < kTuneMinRows) continue;
      const unsigned bit = 1u << l;
      std::vector<Modes> cand = {cur};
      if (!h->wg_fixed) cand.push_back(Modes{cur.w ^ bit, cur.a, cur.r});
      if (!h->lds_fixed && h->L[l].band_max > 0) cand.push_back(Modes{cur.w, cur.a ^ bit, cur.r});
      if (!h->lds_fixed && h->L[l].rband_max > 0 && h->L[l].rperm) cand.push_back(Modes{cur.w, cur.a, cur.r ^ bit});
      if (cand.size() == 1) continue;
      std::vector<Captured> cap(cand.size());
      std::vector<double> t(cand.size(), 1e300);
      auto time_all = [&](size_t from) -> amgdd_status {
        for (size_t c = from; c < cand.size(); ++c) {
          set_modes(cand[c]);
          amgdd_status cs = capture(h, true, &cap[c].g, &cap[c].e);
          if (cs) return cs;
        }
        for (int rep = 0; rep < 2; ++rep)
          for (size_t c = 0; c < cand.size(); ++c) {
            double ms = 0;
            amgdd_status ts = time_exec(cap[c].e, ms);
            if (ts) return ts;
            t[c] = std::min(t[c], ms);
          }
        return AMGDD_OK;
      };
      st = time_all(0);
      size_t bi = 0;
      if (!st) {
        for (size_t c = 1; c < cand.size(); ++c)
          if (t[c] < t[bi] && t[c] < t[0] * 0.999) bi = c;
        // one more candidate: the switches that beat the current modes, together
        Modes both = cand[bi];
        for (size_t c = 1; bi && c < cand.size(); ++c)
          if (c != bi && t[c] < t[0] * 0.999)
            both = Modes{both.w ^ (cand[c].w ^ cur.w), both.a ^ (cand[c].a ^ cur.a), both.r ^ (cand[c].r ^ cur.r)};
        if (bi && (both.w != cand[bi].w || both.a != cand[bi].a || both.r != cand[bi].r)) {
          cand.push_back(both);
          cap.emplace_back();
          t.push_back(1e300);
          for (double &x : t) x = 1e300;
          st = time_all(cand.size() - 1);
          if (!st && t.back() < t[bi] * 0.999 && t.back() < t[0] * 0.999) bi = cand.size() - 1;
        }
      }
      for (auto &c : cap) c.drop();
      if (st) return st;
      cur = cand[bi];
      if (bi) best = t[bi];
      set_modes(cur);
    }
  }
  h->sched_cached = 0;
  HIP_TRY(hipMemcpyAsync(h->x, xsave, (size_t)h->N0 * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  h->drop_graphs();
  SchedEntry e{best_l, best_b, best / 3.0};
  e.wide = cur.w;
  e.lds = cur.a;
  e.rlds = cur.r;
  sched_store(key, e);
  h->autotune_s = now_s() - t0;
  return AMGDD_OK;
}

enum SolveKind { SOLVE_DD = 0, SOLVE_V = 1 };

// noalloc: no tuning runs (an untuned handle runs the level-synchronous
// schedule, which gives the same iterates), no graph capture (kernels are
// enqueued one by one), residual scratch as set in h->rs_partial / rs_norm2.
amgdd_status run_solve(amgdd_ctx *h, SolveKind kind, const double *b_dev, double *x_dev, double rtol, int maxit,
                       amgdd_info *info, bool noalloc = false) {
  TraceRange tr(kind == SOLVE_V ? "amgdd: V-cycle solve" : "amgdd: AMG-DD solve");
  if (!h) return fail(ST_EINVAL, "null handle");
  if (h->host_only) return fail(ST_EDEVICE, "host-only handle (device = -1): no device solve");
  if (!b_dev || !x_dev) return fail(ST_EINVAL, "null device vector");
  if (maxit < 0) return fail(ST_EINVAL, "maxit < 0");
  HIP_TRY(hipSetDevice(h->device));
  hipStream_t s = h->stream;
  const size_t nbytes = (size_t)h->N0 * sizeof(double);
  // a hybrid handle none of whose problems reaches its transition level runs
  // V-cycles (the level-L~ AMG-DD of a one-level problem is the direct solve)
  if (kind == SOLVE_DD && h->hybrid_lt > 0 && !h->inner) kind = SOLVE_V;
  const bool hybrid = kind == SOLVE_DD && h->inner;
  HIP_TRY(hipMemcpyAsync(h->b, b_dev, nbytes, hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipMemcpyAsync(h->x, x_dev, nbytes, hipMemcpyDeviceToDevice, s));
  // an untuned schedule during a no-allocation solve: level-synchronous for
  // this call only
  struct SchedRestore {
    amgdd_ctx *t = nullptr;
    ~SchedRestore() {
      if (t) t->sched_level = -2;
    }
  } sched_restore;
  if (kind == SOLVE_DD) {
    amgdd_ctx *t = hybrid ? h->inner : h;
    if (t->sched_level == -2) {
      if (noalloc) {
        t->sched_level = -1;
        sched_restore.t = t;
      } else {
        amgdd_status st = autotune(t);
        if (st) return st;
      }
    }
  }
  bool use_graph = h->prm.use_graph != 0 && !noalloc;
  if (use_graph) {
    if (kind == SOLVE_DD && !h->g_dd) {
      amgdd_status st = capture(h, true, &h->gr_dd, &h->g_dd);
      if (st) return st;
    }
    if (kind == SOLVE_V && !h->g_v) {
      amgdd_status st = capture(h, false, &h->gr_v, &h->g_v);
      if (st) return st;
    }
  }
  auto enqueue_res = [&](hipStream_t st) {
    if (kind == SOLVE_V || hybrid) enqueue_residual<double>(h, st, true);
    else if (h->mixed()) enqueue_residual<float>(h, st, false);
    else enqueue_residual<double>(h, st, false);
  };
  auto enqueue_iter = [&](hipStream_t st) -> hipError_t {
    if (use_graph) return hipGraphLaunch(kind == SOLVE_DD ? h->g_dd : h->g_v, st);
    if (kind == SOLVE_V) enqueue_v_iteration(h, st);
    else if (hybrid) enqueue_hybrid(h, st);
    else if (h->mixed()) enqueue_dd_iteration<float>(h, st);
    else enqueue_dd_iteration<double>(h, st);
    return hipGetLastError();
  };
  const double t_start = now_s();
  enqueue_res(s);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(s));
  const int np = h->nprob;
  h->hist.assign(np, std::vector<double>());
  std::vector<double> r0(np);
  for (int q = 0; q < np; ++q) {
    r0[q] = std::sqrt(h->h_norm2[q]);
    h->hist[q].push_back(r0[q]);
  }
  auto converged = [&]() {
    if (rtol <= 0) return false;
    for (int q = 0; q < np; ++q)
      if (!(h->hist[q].back() <= rtol * r0[q])) return false;
    return true;
  };
  auto finite = [&]() {
    for (int q = 0; q < np; ++q)
      if (!std::isfinite(h->hist[q].back())) return false;
    return true;
  };
  int it = 0;
  amgdd_status result = AMGDD_OK;
  if (!finite()) result = fail(ST_EBREAKDOWN, "non-finite initial residual");
  while (result == AMGDD_OK && !converged() && it < maxit) {
    TraceRange ti(tracing() ? "amgdd: iteration " + std::to_string(it + 1) : std::string());
    HIP_TRY(enqueue_iter(s));
    HIP_TRY(hipStreamSynchronize(s));
    ++it;
    for (int q = 0; q < np; ++q) h->hist[q].push_back(std::sqrt(h->h_norm2[q]));
    if (!finite()) result = fail(ST_EBREAKDOWN, "non-finite residual norm at iteration " + std::to_string(it));
  }
  const double solve_s = now_s() - t_start;  // every iteration ended in a stream synchronisation
  HIP_TRY(hipMemcpyAsync(x_dev, h->x, nbytes, hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (result == AMGDD_OK && rtol > 0 && !converged())
    result = fail(ST_ENOCONV, "maxit reached before rtol");
  if (info) {
    info->iters = it;
    info->solve_s = solve_s;
    info->setup_s = h->setup_s;
    double rel = 0.0, rho = 0.0;
    for (int q = 0; q < np; ++q) {
      const auto &hq = h->hist[q];
      double rq = r0[q] > 0 ? hq.back() / r0[q] : 0.0;
      rel = std::max(rel, rq);
      int k = std::min<int>(5, (int)hq.size() - 1);
      if (k > 0 && hq[hq.size() - 1 - k] > 0) rho = std::max(rho, std::pow(hq.back() / hq[hq.size() - 1 - k], 1.0 / k));
    }
    info->relres = rel;
    info->rho_asym = rho;
  }
  return result;
}

// ---------------------------------------------------------------- no-allocation solve
//
// amgdd_solve_noalloc keeps the only device memory a solve needs beyond the
// handle's own arrays -- the residual partial sums (one per 256-row block) and
// the per-problem squared norms -- in this static array, so the call itself
// allocates nothing.  Each device holds its own copy; its address is taken once
// per device when a handle is first set up there.  Calls that overlap on one
// device share the array and race.
constexpr long long NOALLOC_SCRATCH = 1LL << 17;  // doubles (1 MiB): blocks + problems
static __device__ __align__(256) double scratch[NOALLOC_SCRATCH];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[MAX_DEVICES] = {};

// Device address of `scratch` on the current device (recorded once per device).
amgdd_status resolve_scratch(int device) {
  if (device < 0 || device >= MAX_DEVICES) return fail(ST_EUNSUP, "device ordinal beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return AMGDD_OK;
  void *p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    return fail(ST_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  g_scratch_ptr[device] = (double *)p;
  return AMGDD_OK;
}

// Streams, events and device layouts of a handle and of its level-L~ handle.
amgdd_status init_device(amgdd_ctx *h, int device, hipStream_t stream) {
  HIP_TRY(hipSetDevice(device));
  {
    amgdd_status ss = resolve_scratch(device);
    if (ss) return ss;
  }
  long long cap = 0;
  if (const char *e2 = std::getenv("AMGDD_TEST_MAX_BYTES")) cap = std::atoll(e2);
  for (amgdd_ctx *c : {h, h->inner}) {
    if (!c) continue;
    c->host_only = false;
    c->max_bytes = cap;
    c->device = device;
    c->stream = stream;
    c->overlap = std::getenv("AMGDD_SERIAL") == nullptr;
    if (hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess)
      return fail(ST_EDEVICE, "stream/event creation failed");
    TraceRange tru("amgdd: upload");
    amgdd_status us = upload_all(c);
    if (us) return us;
  }
  return AMGDD_OK;
}

// The handle of the transposed hierarchy (A_l^T with the same P_l, R_l and
// composite grids; see build_setup_transposed) for adjoint solves of a
// non-symmetric operator, and of its level-L~ problems on a hybrid handle.
amgdd_status make_adjoint(amgdd_ctx *h) {
  TraceRange tr("amgdd: setup of the transposed hierarchy");
  const double t0 = now_s();
  amgdd_ctx *a = new (std::nothrow) amgdd_ctx();
  if (!a) return fail(ST_ENOMEM, "handle allocation");
  auto copy_cfg = [](amgdd_ctx *dst, const amgdd_ctx *src) {
    dst->prm = src->prm;
    dst->symmetric = src->symmetric;
    dst->sched_level = src->prm.tail_level >= -1 && src->prm.tail_block != 0 ? src->sched_level : -2;
    dst->sched_block = src->prm.tail_block ? src->prm.tail_block : 256;
    dst->lbase = src->lbase;
    dst->hybrid_lt = src->hybrid_lt;
    dst->inner_of = src->inner_of;
    dst->part_map = src->part_map;
  };
  copy_cfg(a, h);
  std::string err;
  int st = build_setup_transposed(h->S, !h->S.grids.empty(), a->S, err);
  if (!st && h->inner) {
    a->inner = new (std::nothrow) amgdd_ctx();
    if (!a->inner) st = ST_ENOMEM, err = "handle allocation";
    else {
      copy_cfg(a->inner, h->inner);
      st = build_setup_transposed(h->inner->S, true, a->inner->S, err);
    }
  }
  if (st) {
    delete a;
    return fail(st, err);
  }
  amgdd_status us = init_device(a, h->device, h->stream);
  if (us) {
    std::string msg = g_last_error;
    delete a;
    return fail(us, msg);
  }
  a->setup_s = now_s() - t0;
  h->adj = a;
  return AMGDD_OK;
}

amgdd_status make_handle(const std::vector<ProblemInput> &in, const amgdd_params *prm, void *stream, amgdd_handle *out) {
  TraceRange tr("amgdd: setup");
  if (!out) return fail(ST_EINVAL, "null output handle");
  *out = nullptr;
  double t0 = now_s();
  amgdd_ctx *h = new (std::nothrow) amgdd_ctx();
  if (!h) return fail(ST_ENOMEM, "handle allocation");
  amgdd_params_default(&h->prm);
  if (prm) h->prm = *prm;
  const amgdd_params &p = h->prm;
  if (p.tail_block != 0 && p.tail_block != 256 && p.tail_block != 512 && p.tail_block != 1024) {
    delete h;
    return fail(ST_EINVAL, "tail_block must be 0, 256, 512 or 1024");
  }
  if (p.tail_level < -2) {
    delete h;
    return fail(ST_EINVAL, "tail_level must be >= -2");
  }
  h->sched_level = -2;
  h->sched_block = p.tail_block ? p.tail_block : 256;
  if (p.tail_level >= -1 && p.tail_block != 0) h->sched_level = p.tail_level;
  if (p.n_fac < 1 || (p.precision != AMGDD_FP64 && p.precision != AMGDD_MIXED)) {
    delete h;
    return fail(ST_EINVAL, "bad n_fac or precision");
  }
  if (p.hybrid_level < 0) {
    delete h;
    return fail(ST_EINVAL, "hybrid_level must be >= 0");
  }
  if (p.relax_order != 0 && p.relax_order != 1) {
    delete h;
    return fail(ST_EINVAL, "relax_order must be 0 (natural) or 1 (CF)");
  }
  if (p.coarsen != 0 && p.coarsen != 1) {
    delete h;
    return fail(ST_EINVAL, "coarsen must be 0 (RS) or 1 (HMIS)");
  }
  if (p.interp != 0 && p.interp != 1) {
    delete h;
    return fail(ST_EINVAL, "interp must be 0 (direct) or 1 (extended+i)");
  }
  if (p.interp_max < 0) {
    delete h;
    return fail(ST_EINVAL, "interp_max must be >= 0");
  }
  h->S.coarsen = p.coarsen;
  h->S.interp = p.interp;
  h->S.interp_max = p.interp_max;
  h->S.cf = p.relax_order == 1;
  // measurement / testing: int32 column indices everywhere, one or four
  // entries per lane and step everywhere, the row-sorting window
  h->S.compress = std::getenv("AMGDD_INDEX32") == nullptr;
  // composite operators stored in FP32 load four entries per lane and step
  if (p.precision == AMGDD_MIXED) h->S.comp_step_log2 = 2;
  if (std::getenv("AMGDD_QUAD")) h->S.step_log2 = h->S.comp_step_log2 = 2;
  if (std::getenv("AMGDD_UNPAIRED")) h->S.step_log2 = h->S.comp_step_log2 = 0;
  if (const char *e = std::getenv("AMGDD_SORT_WINDOW")) h->S.sort_window = std::max(0, std::atoi(e));
  if (const char *e = std::getenv("AMGDD_LANE_TARGET")) h->S.comp_lane_target = std::max(1.0, std::atof(e));
  if (std::getenv("AMGDD_FUSED_R")) h->S.tight = false;
  if (const char *e = std::getenv("AMGDD_TIGHT_WINDOW")) h->S.tight_window = h->S.tight_window_r = std::max(0, std::atoi(e));
  if (const char *e = std::getenv("AMGDD_TIGHT_WINDOW_R")) h->S.tight_window_r = std::max(0, std::atoi(e));
  if (const char *e = std::getenv("AMGDD_WIDE_TILES_MIN")) h->S.wide_tiles_min = std::max(0, std::atoi(e));
  if (const char *e = std::getenv("AMGDD_TILE_SLICES_MAX")) {
    const int v = std::atoi(e);
    h->S.tile_slices_max = v >= 128 ? 128 : v >= 64 ? 64 : v >= 32 ? 32 : 16;
  }
  std::string err;
  Setup inner_S;
  int st;
  {
    TraceRange trh("amgdd: host setup (hierarchy, composite grids, layouts)");
    st = p.hybrid_level > 0 ? build_setup_hybrid(in, p.theta, p.max_coarse, p.max_levels, p.hybrid_level, h->S, inner_S,
                                                 h->inner_of, h->part_map, err)
                            : build_setup(in, p.theta, p.max_coarse, p.max_levels, h->S, err);
  }
  if (st) {
    delete h;
    return fail(st, err);
  }
  h->symmetric = true;
  for (auto &P : h->S.probs) h->symmetric = h->symmetric && P.symmetric;
  h->hybrid_lt = p.hybrid_level;
  if (!inner_S.probs.empty()) {
    // the level-L~ problems: an AMG-DD handle of their own whose fine vectors
    // are the leading rows of the outer global level L~ (problems that
    // continue below L~, in problem order)
    const int lt = h->hybrid_lt;
    long long n = 0;
    for (auto &P : inner_S.probs) n += P.n;
    if (lt > h->S.maxL() || n != h->S.lv[lt].GNn) {
      delete h;
      return fail(ST_EINVAL, "internal: hybrid level layout mismatch");
    }
    amgdd_ctx *in2 = new (std::nothrow) amgdd_ctx();
    if (!in2) {
      delete h;
      return fail(ST_ENOMEM, "handle allocation");
    }
    h->inner = in2;
    in2->prm = h->prm;
    in2->prm.hybrid_level = 0;
    in2->S = std::move(inner_S);
    in2->symmetric = h->symmetric;
    in2->sched_level = h->sched_level;
    in2->sched_block = h->sched_block;
    in2->lbase = lt;
    if (in2->sched_level > in2->S.maxL()) in2->sched_level = -1;
  }
  if (h->sched_level > h->S.maxL()) h->sched_level = -1;
  h->host_only = p.device < 0;
  if (h->inner) h->inner->host_only = h->host_only;
  if (!h->host_only) {
    double tu = now_s();
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || p.device >= ndev) {
      h->host_only = true;
      if (h->inner) h->inner->host_only = true;
      delete h;
      return fail(ST_EDEVICE, "no HIP device " + std::to_string(p.device));
    }
    amgdd_status us = init_device(h, p.device, (hipStream_t)stream);
    if (us) {
      std::string msg = g_last_error;
      delete h;
      return fail(us, msg);
    }
    h->S.times.upload = now_s() - tu;
  }
  h->setup_s = now_s() - t0;
  *out = h;
  return AMGDD_OK;
}

}  // namespace

// ======================================================================= C ABI

extern "C" {

void amgdd_params_default(amgdd_params *prm) {
  if (!prm) return;
  prm->theta = 0.25;
  prm->max_coarse = 16;
  prm->max_levels = 25;
  prm->padding = 1;
  prm->n_fac = 2;
  prm->precision = AMGDD_FP64;
  prm->device = 0;
  prm->use_graph = 1;
  prm->tail_level = -2;
  prm->tail_block = 0;
  prm->hybrid_level = 0;
  prm->relax_order = 0;
  prm->coarsen = 0;
  prm->interp = 0;
  prm->interp_max = 4;
  prm->n_padding_levels = 0;
  prm->padding_per_level = nullptr;
}

amgdd_status amgdd_setup_composite(int n, const int *rowptr, const int *colind, const double *val, const int *part,
                                   int nparts, const amgdd_params *prm, void *hip_stream, amgdd_handle *out) {
  amgdd_params p;
  amgdd_params_default(&p);
  if (prm) p = *prm;
  std::vector<ProblemInput> in{ProblemInput{n, rowptr, colind, val, part, nparts, p.padding, p.padding_per_level, p.n_padding_levels}};
  return make_handle(in, &p, hip_stream, out);
}

amgdd_status amgdd_setup_composite_batch(int nprob, const int *n, const int *const *rowptr, const int *const *colind,
                                         const double *const *val, const int *const *part, const int *nparts,
                                         const amgdd_params *prm, void *hip_stream, amgdd_handle *out) {
  if (nprob <= 0 || !n || !rowptr || !colind || !val || !part || !nparts || !prm)
    return fail(ST_EINVAL, "null batch argument");
  std::vector<ProblemInput> in;
  for (int q = 0; q < nprob; ++q)
    in.push_back(ProblemInput{n[q], rowptr[q], colind[q], val[q], part[q], nparts[q], prm[q].padding,
                              prm[q].padding_per_level, prm[q].n_padding_levels});
  return make_handle(in, &prm[0], hip_stream, out);
}

amgdd_status amgdd_solve(amgdd_handle h, const double *b_dev, double *x_dev, double rtol, int maxit, amgdd_info *info) {
  return run_solve(h, SOLVE_DD, b_dev, x_dev, rtol, maxit, info);
}

amgdd_status amgv_solve(amgdd_handle h, const double *b_dev, double *x_dev, double rtol, int maxit, amgdd_info *info) {
  return run_solve(h, SOLVE_V, b_dev, x_dev, rtol, maxit, info);
}

amgdd_status amgdd_solve_noalloc(amgdd_handle h, const double *b_dev, double *x_dev, double rtol, int maxit,
                                 amgdd_info *info) {
  if (!h) return fail(ST_EINVAL, "null handle");
  if (h->host_only) return fail(ST_EDEVICE, "host-only handle (device = -1): no device solve");
  long long cap = NOALLOC_SCRATCH;
  if (const char *e = std::getenv("AMGDD_TEST_NOALLOC_CAP")) cap = std::min(cap, std::atoll(e));
  const long long need = (long long)h->nblk + h->nprob;
  if (need > cap)
    return fail(ST_EUNSUP, "amgdd_solve_noalloc: the handle needs " + std::to_string(need) +
                               " doubles of residual scratch (one per 256 fine rows plus one per problem); the "
                               "library's static scratch holds " + std::to_string(cap));
  double *p = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (h->device >= 0 && h->device < MAX_DEVICES) p = g_scratch_ptr[h->device];
  }
  if (!p) return fail(ST_EDEVICE, "amgdd_solve_noalloc: no scratch address for this device");
  struct Restore {
    amgdd_ctx *h;
    ~Restore() { h->rs_partial = h->rs_norm2 = nullptr; }
  } restore{h};
  h->rs_partial = p;
  h->rs_norm2 = p + h->nblk;
  return run_solve(h, SOLVE_DD, b_dev, x_dev, rtol, maxit, info, true);
}

amgdd_status amgdd_solve_adjoint(amgdd_handle h, const double *g_dev, double *lambda_dev, double rtol, int maxit,
                                 amgdd_info *info) {
  if (!h) return fail(ST_EINVAL, "null handle");
  if (h->symmetric || h->host_only) return run_solve(h, SOLVE_DD, g_dev, lambda_dev, rtol, maxit, info);
  if (!h->adj) {
    HIP_TRY(hipSetDevice(h->device));
    amgdd_status st = make_adjoint(h);
    if (st) return st;
  }
  amgdd_status st = run_solve(h->adj, SOLVE_DD, g_dev, lambda_dev, rtol, maxit, info);
  h->hist = h->adj->hist;  // amgdd_get_history reports the last solve
  return st;
}

amgdd_status amgdd_face_gradient(amgdd_handle h, const double *u_dev, const double *lambda_dev, const int *face_i_dev,
                                 const int *face_j_dev, int nfaces, double *dLdc_dev) {
  if (!h) return fail(ST_EINVAL, "null handle");
  if (h->host_only) return fail(ST_EDEVICE, "host-only handle");
  if (nfaces < 0 || (nfaces > 0 && (!u_dev || !lambda_dev || !face_i_dev || !face_j_dev || !dLdc_dev)))
    return fail(ST_EINVAL, "bad face-gradient arguments");
  HIP_TRY(hipSetDevice(h->device));
  LAUNCH(dev::k_face_grad, nblocks(nfaces), dev::BLOCK, 0, h->stream, nfaces, face_i_dev, face_j_dev, u_dev, lambda_dev,
         dLdc_dev);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(h->stream));
  return AMGDD_OK;
}

amgdd_status amgdd_get_stats(amgdd_handle h, amgdd_stats *st) {
  if (!h || !st) return fail(ST_EINVAL, "null argument");
  const Setup &S = h->S;
  std::memset(st, 0, sizeof(*st));
  st->n_problems = (int)S.probs.size();
  st->n_grids = (int)S.grids.size();
  st->max_levels = S.maxL() + 1;
  st->fine_rows = S.prob_off.back();
  st->global_nnz = S.global_nnz;
  st->composite_real_nnz = S.composite_real_nnz;
  st->composite_rows = S.composite_rows;
  st->composite_real_rows = S.composite_real_rows;
  // entries stored on the device, padding included (a reordered P replaces P)
  auto stored = [](const BatchLevel &B) {
    return B.A.entries() + (B.pperm.empty() ? B.P.entries() : B.Pt.entries()) + B.R.entries() + B.Rt.entries();
  };
  long long e = 0;
  for (auto &B : S.lv) e += stored(B);
  st->composite_stored_nnz = e;
  long long u = 0;
  for (auto &B : S.lv) u += B.nnzA + B.nnzP + B.nnzR;
  st->composite_nnz = u;
  st->omissions = S.omissions;
  st->composite_overhead = S.global_nnz ? (double)S.composite_real_nnz / (double)S.global_nnz : 0.0;
  st->setup_hierarchy_s = S.times.hierarchy;
  st->setup_composite_s = S.times.composite;
  st->setup_pack_s = S.times.pack;
  st->setup_upload_s = S.times.upload;
  st->device_bytes = h->dev_bytes + (h->adj ? h->adj->dev_bytes + (h->adj->inner ? h->adj->inner->dev_bytes : 0) : 0);
  st->tail_level = h->sched_level;
  st->tail_block = h->sched_block;
  st->autotune_s = h->autotune_s;
  st->schedule_cached = h->sched_cached;
  for (int l = 0; l < (int)h->L.size() && l < 32; ++l) {
    if (h->L[l].wg == 512) st->wide_levels |= 1 << l;
    if (h->L[l].lds) st->lds_levels |= 1 << l;
    if (h->L[l].rlds) st->restrict_lds_levels |= 1 << l;
  }
  if (h->hybrid_lt > 0) {
    // composite figures of the level-L~ problems; levels above L~ (and whole
    // hierarchies that end at or above L~) are cycled on the global grids
    const int lt = h->hybrid_lt;
    st->hybrid_level = lt;
    long long upper = 0;
    for (size_t q = 0; q < S.probs.size(); ++q) {
      const Hierarchy &H = S.probs[q].H;
      const int top = h->inner_of[q] >= 0 ? lt : H.L() + 1;
      for (int l = 0; l < top; ++l) upper += H.A[l].nnz();
    }
    st->n_grids = 0;
    st->composite_real_nnz = st->composite_rows = st->composite_real_rows = 0;
    st->composite_stored_nnz = st->composite_nnz = st->omissions = 0;
    st->setup_composite_s = 0.0;
    st->tail_level = -1;
    if (const amgdd_ctx *in = h->inner) {
      const Setup &I = in->S;
      st->n_grids = (int)I.grids.size();
      st->composite_real_nnz = I.composite_real_nnz;
      st->composite_rows = I.composite_rows;
      st->composite_real_rows = I.composite_real_rows;
      st->omissions = I.omissions;
      long long e2 = 0, u2 = 0;
      for (auto &B : I.lv) {
        e2 += stored(B);
        u2 += B.nnzA + B.nnzP + B.nnzR;
      }
      st->composite_stored_nnz = e2;
      st->composite_nnz = u2;
      st->setup_composite_s = I.times.composite;
      st->setup_pack_s += I.times.pack;
      st->device_bytes += in->dev_bytes;
      st->tail_level = in->sched_level;
      st->tail_block = in->sched_block;
      st->autotune_s = in->autotune_s;
      st->schedule_cached = in->sched_cached;
      st->wide_levels = st->lds_levels = st->restrict_lds_levels = 0;
      for (int l = 0; l < (int)in->L.size() && l + h->hybrid_lt < 32; ++l) {
        if (in->L[l].wg == 512) st->wide_levels |= 1 << (l + h->hybrid_lt);
        if (in->L[l].lds) st->lds_levels |= 1 << (l + h->hybrid_lt);
        if (in->L[l].rlds) st->restrict_lds_levels |= 1 << (l + h->hybrid_lt);
      }
    }
    st->composite_overhead = S.global_nnz ? (double)(upper + st->composite_real_nnz) / (double)S.global_nnz : 0.0;
  }
  return AMGDD_OK;
}

amgdd_status amgdd_get_levels(amgdd_handle h, int prob, int *nlevels, int *n_per_level, long long *nnz_per_level) {
  if (!h || !nlevels || prob < 0 || prob >= (int)h->S.probs.size()) return fail(ST_EINVAL, "bad argument");
  const Hierarchy &H = h->S.probs[prob].H;
  *nlevels = H.L() + 1;
  for (int l = 0; l <= H.L(); ++l) {
    if (n_per_level) n_per_level[l] = H.A[l].nrows;
    if (nnz_per_level) nnz_per_level[l] = H.A[l].nnz();
  }
  return AMGDD_OK;
}

amgdd_status amgdd_get_cf(amgdd_handle h, int prob, int level, signed char *cf) {
  if (!h || !cf || prob < 0 || prob >= (int)h->S.probs.size()) return fail(ST_EINVAL, "bad argument");
  const Hierarchy &H = h->S.probs[prob].H;
  if (level < 0 || level >= H.L()) return fail(ST_EINVAL, "level has no C/F splitting");
  std::memcpy(cf, H.cf[level].data(), H.cf[level].size());
  return AMGDD_OK;
}

amgdd_status amgdd_get_operator(amgdd_handle h, int prob, int level, int which, int *nrows, int *nnz, int *rowptr,
                                int *col, double *val) {
  if (!h || !nrows || !nnz || prob < 0 || prob >= (int)h->S.probs.size()) return fail(ST_EINVAL, "bad argument");
  const Hierarchy &H = h->S.probs[prob].H;
  const Csr *M = nullptr;
  if (which == 0 && level >= 0 && level <= H.L()) M = &H.A[level];
  if (which == 1 && level >= 0 && level < H.L()) M = &H.P[level];
  if (!M) return fail(ST_EINVAL, "no such operator");
  *nrows = M->nrows;
  *nnz = (int)M->nnz();
  if (rowptr) std::memcpy(rowptr, M->ptr.data(), M->ptr.size() * sizeof(int));
  if (col) std::memcpy(col, M->col.data(), M->col.size() * sizeof(int));
  if (val) std::memcpy(val, M->val.data(), M->val.size() * sizeof(double));
  return AMGDD_OK;
}

amgdd_status amgdd_get_composite(amgdd_handle h, int prob, int p, int level, int *n_real, int *n_bar, int *gids,
                                 int *omissions) {
  if (!h || prob < 0 || prob >= (int)h->S.probs.size()) return fail(ST_EINVAL, "bad problem");
  const ProblemHost &P = h->S.probs[prob];
  if (p < 0 || p >= P.nparts || level < 0 || level > P.H.L()) return fail(ST_EINVAL, "bad subdomain or level");
  const Setup *S = &h->S;
  int q = prob;
  if (h->hybrid_lt > 0) {
    q = h->inner_of[prob];
    if (q < 0 || !h->inner) return fail(ST_EINVAL, "problem has no level-L~ AMG-DD problem (hierarchy ends at or above L~)");
    if (level < h->hybrid_lt) return fail(ST_EINVAL, "hybrid handle: composite grids exist on levels >= hybrid_level only");
    p = h->part_map[prob][p];
    if (p < 0) return fail(ST_EINVAL, "subdomain has no points on the hybrid level");
    level -= h->hybrid_lt;
    S = &h->inner->S;
  }
  const CompLevel &lv = S->grids[S->probs[q].grids[p]].lv[level];
  if (n_real) *n_real = lv.nreal;
  if (n_bar) *n_bar = lv.nbar();
  if (gids) std::memcpy(gids, lv.gid.data(), lv.gid.size() * sizeof(int));
  if (omissions) *omissions = lv.omissions;
  return AMGDD_OK;
}

amgdd_status amgdd_get_history(amgdd_handle h, int prob, double *hist, int cap, int *len) {
  if (!h || !len || prob < 0 || prob >= (int)h->S.probs.size()) return fail(ST_EINVAL, "bad argument");
  if (prob >= (int)h->hist.size()) { *len = 0; return AMGDD_OK; }
  const auto &v = h->hist[prob];
  *len = (int)v.size();
  if (hist)
    for (int i = 0; i < std::min(cap, (int)v.size()); ++i) hist[i] = v[i];
  return AMGDD_OK;
}

amgdd_status amgdd_profile(amgdd_handle h, int kind, int reps, amgdd_kernel_time *out, int cap, int *n) {
  if (!h || !n || reps < 1 || (kind != 0 && kind != 1)) return fail(ST_EINVAL, "bad profile arguments");
  if (h->host_only) return fail(ST_EDEVICE, "host-only handle");
  HIP_TRY(hipSetDevice(h->device));
  Prof prof;
  struct Reset {
    amgdd_ctx *h;
    ~Reset() {
      h->prof = nullptr;
      if (h->inner) h->inner->prof = nullptr;
    }
  } reset{h};
  hipStream_t s = h->stream;
  if (kind == 0 && h->hybrid_lt > 0 && !h->inner) kind = 1;
  const bool hybrid = kind == 0 && h->inner;
  if (kind == 0) {
    amgdd_ctx *t = hybrid ? h->inner : h;
    if (t->sched_level == -2) {
      amgdd_status ts = autotune(t);
      if (ts) return ts;
    }
  }
  if (kind == 1 || hybrid) enqueue_residual<double>(h, s, true);
  else if (h->mixed()) enqueue_residual<float>(h, s, false);
  else enqueue_residual<double>(h, s, false);
  h->prof = &prof;
  if (h->inner) h->inner->prof = &prof;
  for (int r = 0; r < reps; ++r) {
    prof.rep = r;
    if (kind == 1) enqueue_v_iteration(h, s);
    else if (hybrid) enqueue_hybrid(h, s);
    else if (h->mixed()) enqueue_dd_iteration<float>(h, s);
    else enqueue_dd_iteration<double>(h, s);
  }
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(s));
  h->prof = nullptr;
  if (h->inner) h->inner->prof = nullptr;
  struct Agg {
    std::string name;
    int level, launches;
    std::vector<double> ms;  // per rep
    double bytes;
    int grid, block;
  };
  std::vector<Agg> agg;
  for (auto &site : prof.sites) {
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, site.e0, site.e1));
    Agg *a = nullptr;
    for (auto &x : agg)
      if (x.name == site.name && x.level == site.level) a = &x;
    if (!a) {
      agg.push_back(Agg{site.name, site.level, 0, std::vector<double>(reps, 0.0), 0.0, site.grid, site.block});
      a = &agg.back();
    }
    a->launches++;
    a->ms[site.rep] += ms;
    a->bytes += site.bytes;
  }
  auto median = [](std::vector<double> v) {
    std::sort(v.begin(), v.end());
    const size_t m = v.size() / 2;
    return v.size() % 2 ? v[m] : 0.5 * (v[m - 1] + v[m]);
  };
  *n = (int)agg.size();
  for (int i = 0; i < (int)agg.size() && out && i < cap; ++i) {
    std::memset(&out[i], 0, sizeof(out[i]));
    std::strncpy(out[i].name, agg[i].name.c_str(), sizeof(out[i].name) - 1);
    out[i].level = agg[i].level;
    out[i].launches = agg[i].launches / reps;
    out[i].ms = median(agg[i].ms);
    out[i].bytes = agg[i].bytes / reps;
    out[i].workgroups = agg[i].grid;
    out[i].block = agg[i].block;
  }
  return AMGDD_OK;
}

amgdd_status amgdd_set_stream(amgdd_handle h, void *hip_stream) {
  if (!h) return fail(ST_EINVAL, "null handle");
  for (amgdd_ctx *c : {h, h->inner, h->adj, h->adj ? h->adj->inner : nullptr})
    if (c) c->stream = (hipStream_t)hip_stream;
  return AMGDD_OK;
}

const char *amgdd_last_error(void) { return g_last_error.c_str(); }

void amgdd_destroy(amgdd_handle h) { delete h; }

}  // extern "C"
