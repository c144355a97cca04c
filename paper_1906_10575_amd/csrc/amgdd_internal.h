// Internal host-side data structures shared by the host setup (setup.cpp)
// and the device driver (driver.hip).  Not part of the public ABI.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace amgdd {

// Compressed sparse rows, 0-based, int32 indices, FP64 values.
struct Csr {
  int nrows = 0, ncols = 0;
  std::vector<int> ptr, col;
  std::vector<double> val;
  long long nnz() const { return ptr.empty() ? 0 : ptr[nrows]; }
};

// Global AMG hierarchy of one problem (Section 2 of the paper).
struct Hierarchy {
  std::vector<Csr> A;                    // levels 0..L
  std::vector<Csr> P;                    // levels 0..L-1, N_l x N_{l+1}
  std::vector<Csr> R;                    // levels 0..L-1, R_l = P_l^T
  std::vector<std::vector<int8_t>> cf;   // levels 0..L-1, +1 C / -1 F
  std::vector<std::vector<double>> l1;   // levels 0..L, d_i = sum_j |a_ij|
  std::vector<double> Ac;                // coarsest A_L, dense row-major
  std::vector<double> Ac_inv;            // its inverse (Gauss-Jordan, partial pivoting)
  int L() const { return (int)A.size() - 1; }
};

// One level of one composite grid, local numbering: real points D_l first
// (increasing global id), then ghost points Dbar_l \ D_l (increasing id).
struct CompLevel {
  std::vector<int> gid;
  int nreal = 0;
  int omissions = 0;
  Csr A;                      // rows Dbar_l; real rows full, ghost rows real columns only
  Csr P;                      // rows Dbar_l, columns Dbar_{l+1} (local), dropped outside
  std::vector<double> dinv;   // 1 / d_i at real rows
  int nbar() const { return (int)gid.size(); }
};

struct CompGrid {
  int prob = 0, p = 0;
  std::vector<CompLevel> lv;        // levels 0..L of its problem
  std::vector<int> owned_local;     // level-0 local index of each owned point
  std::vector<int> owned_gid;       // its global id
};

struct ProblemHost {
  int n = 0, nparts = 0, eta = 1;
  std::vector<int> etas;            // per-level padding override (levels < etas.size())
  int eta_of(int l) const { return l < (int)etas.size() ? etas[l] : eta; }
  Csr A0;
  std::vector<int> part;
  Hierarchy H;
  std::vector<int> grids;           // indices into Setup::grids
  bool symmetric = false;
};

// Grouped sliced ELL: G = 2^lg lanes per row, 64/G rows per slice (one
// wavefront); entry k of row r is stored at
//   sptr[r / (64/G)] + 64*(k / G) + (r % (64/G))*G + k % G;
// a slice has (sptr[s+1]-sptr[s]) / 64 steps; rows shorter than the slice are
// padded with value 0 and a column of the same grid.
//
// Compressed column indices (used when every slice fits): per slice two int32
// bases b0 = base[2s], b1 = base[2s+1] and one 16-bit word per entry,
//   column = (c16 & 0x8000 ? b1 : b0) + (c16 & 0x7fff),
// i.e. each slice's columns lie in at most two windows of 32768 (a grid's
// real rows and its ghost rows sit in different regions of the level).  col
// is then emptied.
// windows of an LDS band and slices of an LDS tile (the kernels read the
// same tile descriptors)
constexpr int kBandWindows = 8;
constexpr int kTileSlices = 32;   // operators: default largest tile
constexpr int kTileSlicesS = 16;  // operators: smallest tile
constexpr int kTileSlicesR = 16;  // reordered restriction

struct Sell {
  int nrows = 0;
  int lg = 0;
  int vlg = 0;  // log2 entries per lane in the widest load steps (0, 1 or 2)
  std::vector<int> sptr;
  std::vector<int> col;
  std::vector<double> val;
  std::vector<uint16_t> col16;
  std::vector<int> base;
  // LDS bands (composite operators; see build_bands): 2 kBandWindows ints per
  // tile of ts slices, and each entry's position in its tile's band
  int ts = 0;
  std::vector<int> tiles;
  std::vector<uint16_t> colL;
  std::vector<int> bidx;  // column lists of listed tiles
  long long entries() const { return sptr.empty() ? 0 : sptr.back(); }
  bool compressed() const { return !col16.empty(); }
};

// Block-diagonal batched layout of one level, over every composite grid
// (and, for the G* members, over every problem's global level).
//   composite rows: [normal-grid real rows | gap to a multiple of 64 | normal-grid ghost rows | coarse-grid rows]
//   (with CF ordering, each grid's real rows are C rows then F rows)
//   "normal" grids are those whose problem has L > l; "coarse" grids have L == l.
//   global rows:    [normal problems | coarse problems]
struct BatchLevel {
  int NRn = 0, NBn = 0, NB = 0;
  int NRa = 0;                     // first ghost row: NRn rounded up to 64 (rows between belong to no grid)
  int lg = 0, glg = 0;             // lanes per row (log2) of composite / global rows of this level
  int plg = 0, gplg = 0;           // lanes per row (log2) of composite / global P rows
  Sell A;                          // rows [0, NBn)
  Sell P;                          // rows [0, NBn) -> level l+1 composite rows
  Sell R;                          // R_{l-1}: rows [0, NB) -> level l-1 composite rows
  // level-synchronous passes (Setup::tight): P and R_{l-1} of the normal rows
  // [0, NBn) again, each in a row order of its own (rows sorted by their own
  // length in sort_window windows; position k holds row pperm[k] / rperm[k])
  // and, for R, a lane count of its own (rlg)
  Sell Pt, Rt;
  std::vector<int> pperm, rperm;
  int rlg = 0;
  int band_max = 0;                // largest LDS band of A's tiles (values)
  int rband_max = 0;               // ... of Rt's tiles
  std::vector<double> dinv;        // [NRn]
  std::vector<int> gsrc;           // [NB] global row (this level) of each real row, -1 for ghosts
  std::vector<int> cg_row0, cg_n, cg_dense;  // coarse grids: first row, size, dense offset
  int GNn = 0, GN = 0;
  Sell GA;                         // rows [0, GN)
  Sell GP;                         // rows [0, GNn) -> level l+1 global rows
  Sell GR;                         // R_{l-1}: rows [0, GN) -> level l-1 global rows
  std::vector<double> gdinv;       // [GNn]
  std::vector<int> gc_row0, gc_n, gc_dense;  // coarse problems
  std::vector<int> prob_row0;      // per problem, first global row at this level (-1 absent)
  // stored (unpadded) nonzeros of row ranges, for the algorithmic-bytes model
  long long nnzA_r = 0, nnzA = 0, nnzP = 0, nnzR_n = 0, nnzR = 0;
  long long nnzGA_n = 0, nnzGA = 0, nnzGP = 0, nnzGR_n = 0, nnzGR = 0;
  // CF-ordered relaxation only: C/F class (+1 / -1) of the normal real rows
  // and of the normal global rows; C rows / their nonzeros
  std::vector<int8_t> cls;         // [NRn]
  std::vector<int8_t> gcls;        // [GNn]
  int NRc = 0, GNc = 0;
  long long nnzA_c = 0, nnzGA_c = 0;
};

struct SetupTimes {
  double hierarchy = 0, composite = 0, pack = 0, upload = 0;
};

struct Setup {
  double theta = 0.25;
  int max_coarse = 16, max_levels = 25;
  // CF-ordered relaxation: class arrays are filled and each grid's real rows
  // of a level are stored C-points first (Jacobi within a class does not
  // depend on row order, so results agree up to the rounding of grouped rows,
  // whose lanes' shares follow their slice; the half-sweeps then read
  // contiguous row ranges)
  bool cf = false;
  // 16-bit column indices for every matrix whose slices allow them
  bool compress = true;
  // log2 of the entries of its row each lane loads per sliced-ELL step in
  // the widest steps (the device mat-vec gives the address map): 0 one,
  // 1 two (paired), 2 four; for the global operators and for the composite
  // operators (four when those are stored in FP32: one 16-byte value load)
  int step_log2 = 1;
  int comp_step_log2 = 1;
  // on levels with grouped rows, each grid's real and ghost rows are sorted
  // by decreasing length within windows of this many rows (0: local order)
  int sort_window = 512;
  // grouped composite rows: lanes per row = smallest power of two with at
  // most this many entries per lane (rows of up to 20 entries keep one lane)
  double comp_lane_target = 16.0;
  // separate reordered layouts of P and R for the level-synchronous passes
  // (see BatchLevel::Pt / Rt); the per-grid schedule keeps P and R
  bool tight = true;
  int tight_window = 512;     // their sort windows (rows): P
  int tight_window_r = 1024;  // R
  // LDS bands of the composite operators (at most band_cap values per tile)
  bool bands = true;
  int band_cap = 8192;
  // operator tiles hold the largest power of two of slices from
  // tile_slices_max down that leaves the level at least wide_tiles_min tiles
  // (default: every level), and kTileSlicesS slices on levels of fewer; a
  // level whose bands overflow the cap at that size takes smaller tiles
  int tile_slices_max = kTileSlices;
  int wide_tiles_min = 0;
  // AMG components: coarsen 0 = RS first pass, 1 = HMIS; interp 0 = direct,
  // 1 = extended+i
  int coarsen = 0, interp = 0;
  int interp_max = 4;  // extended+i: at most this many entries per row (0: no truncation)
  std::vector<ProblemHost> probs;
  std::vector<CompGrid> grids;
  std::vector<BatchLevel> lv;      // 0..maxL
  std::vector<double> dense_A, dense_inv;  // coarsest operators of all problems
  std::vector<int> dense_off;      // per problem offset into dense_*
  std::vector<int> owner;          // [sum N_0] composite level-0 row patched into each fine point
  std::vector<int> prob_off;       // [nprob+1] fine-vector offsets
  // residual blocks: rows [blk_row0[b], blk_row1[b]) of problem blk_prob[b]
  std::vector<int> blk_row0, blk_row1, blk_prob;
  std::vector<int> prob_blk0;      // [nprob+1] first residual block of each problem
  // per (grid, level) row ranges of the batched layout, [ngrids * (maxL+1)]:
  // normal level: real rows [rbeg, rbeg+nreal), ghost rows [gbeg, gbeg+nghost);
  // the grid's coarsest level: rows [rbeg, rbeg+nreal), nghost = 0; absent: all 0
  std::vector<int> gl_rbeg, gl_nreal, gl_gbeg, gl_nghost;
  std::vector<int> grid_L;         // [ngrids] coarsest level of each grid
  SetupTimes times;
  long long omissions = 0;
  long long composite_real_nnz = 0, global_nnz = 0, composite_rows = 0, composite_real_rows = 0;
  int maxL() const { return (int)lv.size() - 1; }
};

// Status codes mirror amgdd_status.
enum { ST_OK = 0, ST_EINVAL = 1, ST_ENOMEM = 2, ST_EDEVICE = 3, ST_ENOCONV = 4, ST_EBREAKDOWN = 5, ST_EUNSUP = 6 };

struct ProblemInput {
  int n;
  const int *rowptr, *colind;
  const double *val;
  const int *part;
  int nparts;
  int eta;
  const int *etas;  // per-level padding (levels < n_etas), may be null
  int n_etas;
};

// Host setup: hierarchy, composite grids and batched layouts.  Returns a
// status and fills `err` on failure.
int build_setup(const std::vector<ProblemInput> &in, double theta, int max_coarse, int max_levels,
                Setup &S, std::string &err);

// Hybrid AMG-DD setup (Algorithm 3): `outer` holds every input problem's
// global hierarchy and layouts without composite grids; `inner` holds the
// level-lt problem (A_lt, levels lt..L, inherited partition with empty
// subdomains dropped) of every problem with L > lt, with composite grids.
// inner_of[q]: index of problem q in `inner` (-1: the problem's hierarchy ends
// at or above lt and its cycle is a plain V-cycle); part_map[q][p]: index of
// subdomain p in that inner problem (-1: empty on level lt).
int build_setup_hybrid(const std::vector<ProblemInput> &in, double theta, int max_coarse, int max_levels, int lt,
                       Setup &outer, Setup &inner, std::vector<int> &inner_of, std::vector<std::vector<int>> &part_map,
                       std::string &err);

// Hierarchy of A^T from the forward setup F (same C/F splittings, P_l, R_l
// and composite sets; operators A_l^T and their l1 diagonals and coarsest
// inverse), with composite grids and layouts when `composite` (F has grids).
int build_setup_transposed(const Setup &F, bool composite, Setup &T, std::string &err);

// Individual steps, exposed for the driver's introspection.
uint64_t splitmix64(uint64_t x);
std::vector<double> pmis_random(int level, int n);
std::vector<int8_t> pmis(const Csr &S, const std::vector<double> &rand, const std::vector<char> *c_init);
std::vector<int8_t> hmis(const Csr &S, const std::vector<int> &part, const std::vector<double> &rand);
Csr ext_i_interpolation(const Csr &A, const Csr &S, const std::vector<int8_t> &cf, int pmax);
Csr strength(const Csr &A, double theta);
std::vector<int8_t> rs_first_pass(const Csr &S);
Csr direct_interpolation(const Csr &A, const Csr &S, const std::vector<int8_t> &cf);
Csr transpose(const Csr &A);
Csr spgemm(const Csr &A, const Csr &B);

}  // namespace amgdd
