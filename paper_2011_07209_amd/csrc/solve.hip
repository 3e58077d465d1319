// Launchers of the persistent CG solve (the instances live in solve_n*.hip).
#include <cstring>

#include "solve_impl.h"

namespace exx {

hipError_t solve_dispatch_n1(const SolveKArgs& a, bool mixed, int max_cols, int threads, int depth, int groups,
                             size_t lds, hipStream_t s, int* occ);
hipError_t solve_dispatch_n2(const SolveKArgs& a, bool mixed, int max_cols, int threads, int depth, int groups,
                             size_t lds, hipStream_t s, int* occ);
hipError_t solve_dispatch_n3(const SolveKArgs& a, bool mixed, int max_cols, int threads, int depth, int groups,
                             size_t lds, hipStream_t s, int* occ);

// Two plane buffers, then the plane offsets of the class, with room for the
// sweeps' look-ahead reads a few planes past the last one (their values are
// discarded).
size_t solve_lds_bytes(const Geo& g, int max_zmax) {
  return (size_t)2 * kLdsWX * g.lds_wy * sizeof(double) + (size_t)(2 * max_zmax + 2 + 8) * sizeof(int);
}

long long solve_slot_bytes(bool mixed, long long sstride) {
  const long long b = mixed ? 24 * sstride : 16 * sstride;
  return (b + 255) & ~255LL;
}

static hipError_t solve_dispatch(const SolveArgs& in, int max_cols, int max_zmax, int groups, hipStream_t s,
                                 int* occ) {
  SolveKArgs a;
  a.cls = in.cls;
  a.pairs = in.pairs;
  a.order = in.order;
  a.p0 = in.p0;
  a.npair = in.npair;
  a.n_eff = in.n_eff;
  a.warm_store = in.warm_store;
  a.warm_cap = in.warm_cap;
  a.warm_state = in.warm_state;
  a.warm_map = in.warm_map;
  a.prev_pairs = in.prev_pairs;
  a.n = in.g.n;
  for (int ax = 0; ax < 3; ++ax) a.N[ax] = in.g.N[ax];
  a.cls_id = in.cls_id;
  a.class_cnt = in.class_cnt;
  a.ncls = in.ncls;
  a.queue = in.queue;
  a.bx_ws = in.bx_ws;
  a.rstride = in.rstride;
  a.slot_ws = in.slot_ws;
  a.sstride = in.sstride;
  a.slot_bytes = solve_slot_bytes(in.mixed, in.sstride);
  a.outIt = in.outIt;
  a.outRes = in.outRes;
  a.outUpd = in.outUpd;
  a.outSav = in.outSav;
  a.outExit = in.outExit;
  a.tol = in.tol;
  a.max_iter = in.max_iter;
  a.delta = in.delta;
  for (int q = 0; q < 4; ++q) a.S.w[q] = in.g.w2[q];
  for (int al = 0; al < 3; ++al) a.S.c[al] = in.g.inv_d2[al];
  a.S.diag = in.g.w2[0] * (a.S.c[0] + a.S.c[1] + a.S.c[2]);
  a.S.cd = 0.0;
  a.S.sd = 0;
  if (in.g.gen && in.quads) {
    // a general cell in the quad layout: its arms in the CG frame are the x',
    // y' and z' axes and at most one diagonal of the sweep plane
    double c[3] = {0.0, 0.0, 0.0}, sum = 0.0;
    for (int m = 0; m < in.g.n_arms; ++m) {
      const int ux = in.g.arm_u[m][in.g.perm[0]], uy = in.g.arm_u[m][in.g.perm[1]], uz = in.g.arm_u[m][in.g.perm[2]];
      const double cf = in.g.arm_coef[m];
      sum += cf;
      if (uz != 0) {
        if (ux != 0 || uy != 0) return hipErrorInvalidValue;
        c[2] += cf;
      } else if (ux != 0 && uy != 0) {
        if (a.S.sd != 0 || (ux != 1 && ux != -1) || (uy != 1 && uy != -1)) return hipErrorInvalidValue;
        a.S.cd = cf;
        a.S.sd = ux * uy;   // oriented so that one step raises x' by one
      } else if (ux != 0) {
        c[0] += cf;
      } else {
        c[1] += cf;
      }
    }
    for (int al = 0; al < 3; ++al) a.S.c[al] = c[al];
    a.S.diag = in.g.w2[0] * sum;
  }
  // general cell: the NK arms in the CG frame (x', y', z') = o[perm]
  a.gen = in.g.gen;
  a.quads = in.quads ? 1 : 0;
  std::memset(&a.G, 0, sizeof(a.G));
  if (a.gen) {
    for (int q = 0; q < 4; ++q) a.G.w[q] = in.g.w2[q];
    double sum = 0.0;
    for (int m = 0; m < in.g.n_arms; ++m) {
      const int ux = in.g.arm_u[m][in.g.perm[0]], uy = in.g.arm_u[m][in.g.perm[1]], uz = in.g.arm_u[m][in.g.perm[2]];
      const double cf = in.g.arm_coef[m];
      sum += cf;
      if (ux == 0 && uy == 0) {
        a.G.cz += cf;
      } else if (uz == 0) {
        if (a.G.n_in == 3) return hipErrorInvalidValue;
        a.G.in_off[a.G.n_in] = ux + kLdsWX * uy;
        a.G.in_coef[a.G.n_in++] = cf;
      } else {
        if (a.G.n_tl == 3 || (uz != 1 && uz != -1)) return hipErrorInvalidValue;
        a.G.tl_off[a.G.n_tl] = uz * (ux + kLdsWX * uy);   // oriented so that a step raises z' by one
        a.G.tl_coef[a.G.n_tl++] = cf;
      }
    }
    a.G.diag = in.g.w2[0] * sum;
  }
  for (int q = 0; q < 4; ++q) {
    a.G.czw[q] = a.G.cz * a.G.w[q];
    for (int k = 0; k < 3; ++k) a.G.tl_cw[k][q] = a.G.tl_coef[k] * a.G.w[q];
  }
  for (int q = 0; q < 4; ++q) {
    a.G32.czw[q] = (float)a.G.czw[q];
    for (int k = 0; k < 3; ++k) a.G32.tl_cw[k][q] = (float)a.G.tl_cw[k][q];
  }
  for (int q = 0; q < 4; ++q) a.G32.w[q] = (float)a.G.w[q];
  a.G32.cz = (float)a.G.cz;
  a.G32.diag = (float)a.G.diag;
  a.G32.n_in = a.G.n_in;
  a.G32.n_tl = a.G.n_tl;
  for (int k = 0; k < 3; ++k) {
    a.G32.in_off[k] = a.G.in_off[k];
    a.G32.in_coef[k] = (float)a.G.in_coef[k];
    a.G32.tl_off[k] = a.G.tl_off[k];
    a.G32.tl_coef[k] = (float)a.G.tl_coef[k];
  }
  a.lds_cx = in.g.lds_cx;
  a.lds_cy = in.g.lds_cy;
  a.lds_wx = in.g.lds_wx;
  a.lds_wy = in.g.lds_wy;
  const size_t lds = solve_lds_bytes(in.g, max_zmax);
  switch (in.g.n) {
    case 1: return solve_dispatch_n1(a, in.mixed, max_cols, in.threads, in.depth, groups, lds, s, occ);
    case 2: return solve_dispatch_n2(a, in.mixed, max_cols, in.threads, in.depth, groups, lds, s, occ);
    case 3: return solve_dispatch_n3(a, in.mixed, max_cols, in.threads, in.depth, groups, lds, s, occ);
    default: return hipErrorInvalidValue;
  }
}

bool solve_supported(int max_cols, int threads) {
  if (threads == 1024) return max_cols <= 4 * 1024;
  if (threads == 768) return max_cols <= 4 * 768;   // quad layout only
  if (threads == 512) return max_cols <= 8 * 512;
  return false;
}

int solve_groups_per_cu(const Geo& g, int max_cols, int max_zmax, bool mixed, bool quads, int threads, int depth) {
  if (!solve_supported(max_cols, threads)) return 0;
  SolveArgs a;
  a.g = g;
  a.mixed = mixed;
  a.quads = quads;
  a.threads = threads;
  a.depth = depth;
  int occ = 0;
  if (solve_dispatch(a, max_cols, max_zmax, 1, nullptr, &occ) != hipSuccess) return 0;
  return occ;
}

hipError_t launch_solve(const SolveArgs& a, int max_cols, int max_zmax, int groups, hipStream_t s) {
  if (a.npair <= 0) return hipSuccess;
  return solve_dispatch(a, max_cols, max_zmax, groups, s, nullptr);
}

}  // namespace exx
