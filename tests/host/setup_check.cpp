// Host-only driver of the setup code for sanitizer builds: assembles 2D and
// 3D Laplacians with block partitions and runs every setup variant (RS /
// HMIS, direct / extended+i, natural / CF row order, hybrid levels, batches;
// one / two / four entries per lane and step, sorted / local row order,
// 16-bit / int32 indices).
// Exit status 0 when every setup returns OK and its layout checks pass.
#include <cstdio>
#include <string>
#include <vector>

#include "../../paper_1906_10575_amd/csrc/amgdd_internal.h"

using namespace amgdd;

struct Prob {
  int n = 0;
  std::vector<int> ptr, col, part;
  std::vector<double> val;
};

static Prob laplace(int nx, int ny, int nz, int px, int py, int pz, double upwind = 0.0) {
  Prob P;
  P.n = nx * ny * nz;
  P.ptr.push_back(0);
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        const int i = x + nx * (y + ny * z);
        std::vector<std::pair<int, double>> row;
        if (z > 0) row.push_back({i - nx * ny, -1.0});
        if (y > 0) row.push_back({i - nx, -1.0});
        // upwind > 0: convection in +x (non-symmetric values, same pattern)
        if (x > 0) row.push_back({i - 1, -1.0 - upwind});
        row.push_back({i, (nz > 1 ? 6.0 : 4.0) + upwind});
        if (x < nx - 1) row.push_back({i + 1, -1.0});
        if (y < ny - 1) row.push_back({i + nx, -1.0});
        if (z < nz - 1) row.push_back({i + nx * ny, -1.0});
        for (auto &e : row) {
          P.col.push_back(e.first);
          P.val.push_back(e.second);
        }
        P.ptr.push_back((int)P.col.size());
        P.part.push_back((x * px) / nx + px * ((y * py) / ny + py * ((z * pz) / nz)));
      }
  return P;
}

int main() {
  std::vector<Prob> probs = {laplace(40, 36, 1, 3, 2, 1), laplace(14, 12, 10, 2, 2, 2), laplace(9, 9, 1, 3, 3, 1)};
  const int nparts[] = {6, 8, 9};
  static const int per_level_eta[] = {2, 0, 1};
  int fails = 0, runs = 0;
  for (int coarsen = 0; coarsen < 2; ++coarsen)
    for (int interp = 0; interp < 2; ++interp)
      for (int cf = 0; cf < 2; ++cf)
        for (int hybrid = 0; hybrid < 3; ++hybrid) {
          std::vector<ProblemInput> in;
          for (size_t q = 0; q < probs.size(); ++q)
            in.push_back(ProblemInput{probs[q].n, probs[q].ptr.data(), probs[q].col.data(), probs[q].val.data(),
                                      probs[q].part.data(), nparts[q], 1 + (int)q % 2,
                                      q == 2 ? per_level_eta : nullptr, q == 2 ? 3 : 0});
          Setup S, I;
          S.coarsen = coarsen;
          S.interp = interp;
          S.cf = cf;
          // the other layouts (unpaired steps, local row order, int32
          // indices) on a rotating subset of the variants
          const int k = runs % 4;
          S.step_log2 = k == 1 ? 0 : (k == 2 ? 2 : 1);
          S.comp_step_log2 = k == 3 ? 2 : S.step_log2;
          S.sort_window = k == 2 ? 0 : (k == 1 ? 512 : 128);
          S.compress = k != 3;
          // LDS tiles of 16 to 128 slices on every level (bands that
          // overflow the cap at the larger sizes fall back to smaller tiles)
          S.tile_slices_max = 16 << (runs % 4);
          S.wide_tiles_min = runs % 2 ? 0 : 2048;
          std::string err;
          int st;
          if (hybrid == 0) {
            st = build_setup(in, 0.25, 16, 25, S, err);
          } else {
            std::vector<int> inner_of;
            std::vector<std::vector<int>> pm;
            st = build_setup_hybrid(in, 0.25, 16, 25, hybrid, S, I, inner_of, pm, err);
          }
          ++runs;
          if (st) {
            ++fails;
            std::fprintf(stderr, "setup coarsen %d interp %d cf %d hybrid %d: status %d %s\n", coarsen, interp, cf,
                         hybrid, st, err.c_str());
          }
        }
  // padding 0 with subdomains that have no points on some level above their
  // coarsest (30^2 in 5 x 5, 24 x 22 x 20 in 3 x 3 x 3), every layout variant
  {
    std::vector<Prob> p0 = {laplace(30, 30, 1, 5, 5, 1), laplace(24, 22, 20, 3, 3, 3)};
    const int np0[] = {25, 27};
    for (int v = 0; v < 8; ++v) {
      std::vector<ProblemInput> in;
      for (size_t q = 0; q < p0.size(); ++q)
        in.push_back(ProblemInput{p0[q].n, p0[q].ptr.data(), p0[q].col.data(), p0[q].val.data(), p0[q].part.data(),
                                  np0[q], 0, nullptr, 0});
      Setup S, I;
      S.cf = v & 1;
      S.step_log2 = (v >> 1) & 1 ? 0 : 1;
      S.comp_step_log2 = v == 6 ? 2 : S.step_log2;
      S.sort_window = v & 2 ? 0 : 128;
      S.compress = v < 4;
      std::string err;
      int st = (v & 4) ? [&] {
        std::vector<int> inner_of;
        std::vector<std::vector<int>> pm;
        return build_setup_hybrid(in, 0.25, 16, 25, 1, S, I, inner_of, pm, err);
      }() : build_setup(in, 0.25, 16, 25, S, err);
      ++runs;
      if (st) {
        ++fails;
        std::fprintf(stderr, "padding-0 setup variant %d: status %d %s\n", v, st, err.c_str());
      }
    }
  }
  // transposed hierarchies (adjoint of a non-symmetric operator), plain and hybrid
  {
    std::vector<Prob> pc = {laplace(40, 36, 1, 3, 2, 1, 0.5), laplace(14, 12, 10, 2, 2, 2, 0.7)};
    const int npc[] = {6, 8};
    for (int v = 0; v < 4; ++v) {
      std::vector<ProblemInput> in;
      for (size_t q = 0; q < pc.size(); ++q)
        in.push_back(ProblemInput{pc[q].n, pc[q].ptr.data(), pc[q].col.data(), pc[q].val.data(), pc[q].part.data(),
                                  npc[q], 1 + (int)q % 2, nullptr, 0});
      Setup S, I, T, TI;
      S.cf = v & 1;
      std::string err;
      int st;
      if (v < 2) {
        st = build_setup(in, 0.25, 16, 25, S, err);
        if (!st) st = build_setup_transposed(S, true, T, err);
      } else {
        std::vector<int> inner_of;
        std::vector<std::vector<int>> pm;
        st = build_setup_hybrid(in, 0.25, 16, 25, 2, S, I, inner_of, pm, err);
        if (!st) st = build_setup_transposed(S, false, T, err);
        if (!st && !I.probs.empty()) st = build_setup_transposed(I, true, TI, err);
      }
      ++runs;
      if (!st && S.probs[0].symmetric) {
        st = 1;
        err = "non-symmetric input reported symmetric";
      }
      if (st) {
        ++fails;
        std::fprintf(stderr, "transposed setup variant %d: status %d %s\n", v, st, err.c_str());
      }
    }
  }
  std::printf("%d setups, %d failed\n", runs, fails);
  return fails ? 1 : 0;
}
