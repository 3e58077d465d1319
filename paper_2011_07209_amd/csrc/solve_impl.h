// The persistent CG solve of the pair Poisson problems (eq. pe discretised with
// the axis stencil of eq. d2_1), FP64 and mixed precision.  Included by one
// translation unit per stencil half-width.
//
// Data layout: a PE vector is stored plane by plane (z ascending); within a
// plane the sphere's (x,y) columns appear in one fixed order sorted by column
// half-height, so plane z holds a prefix of that order.  Thread t of a
// workgroup owns columns t, t + NT, ... for the whole solve and marches z:
// the z neighbours of its points live in a register window of 2n+1 values per
// column, the x/y neighbours come from the current plane staged in LDS
// (double-buffered: one barrier per plane).  Global loads run PD planes ahead
// of their use, so a CU keeps several planes of loads in flight.
#pragma once

#include <type_traits>

#include "device_common.h"
#include "exx_launch.h"

namespace exx {

// Exit reasons of a pair's CG (low byte of SolveKArgs::outExit; the mixed
// solve keeps its restarts above it).
constexpr int kCgConverged = EXX_CG_CONVERGED;
constexpr int kCgCap = EXX_CG_CAP;
constexpr int kCgBreakdown = EXX_CG_BREAKDOWN;
constexpr int kCgNonFinite = EXX_CG_NONFINITE;
// Restarts the mixed solve allows from its last FP64 solution after a
// breakdown or a non-finite norm of its FP32 recursion.
constexpr int kCgMaxRestarts = 3;

template <typename T>
struct StencilT {
  T w[4];      // second-derivative weights w_0..w_3
  T c[3];      // 1 / d_al^2 (general cells in the quad layout: the coefficients of the x', y', z' arms)
  T cd;        // quad layout of a general cell: coefficient of its diagonal arm in the sweep plane (else 0)
  int sd;      // that arm's step along y' for one step along +x' (+-1)
  T diag;      // w_0 times the sum of the arm coefficients
};

template <typename T>
__device__ __forceinline__ StencilT<T> stencil_cast(const StencilT<double>& s) {
  StencilT<T> o;
  for (int q = 0; q < 4; ++q) o.w[q] = (T)s.w[q];
  for (int a = 0; a < 3; ++a) o.c[a] = (T)s.c[a];
  o.cd = (T)s.cd;
  o.sd = s.sd;
  o.diag = (T)s.diag;
  return o;
}

// The solution update of a pass B: x = x + ap p + ar r_in, with r_in the
// residual before the pass's own update.  With `zero` the old x is taken as
// zero; with `skip` x is neither read nor written, and the update is deferred
// to the next pass B: p_k = (p_k+1 - r_k+1) / beta_k, so the two steps
// alpha_k p_k + alpha_k+1 p_k+1 make ap = alpha_k+1 + alpha_k / beta_k and
// ar = -alpha_k / beta_k.  x is then read and written every other iteration
// (seven vector accesses per point and iteration in place of eight).
template <typename T>
struct XStep {
  T ap, ar;
  bool zero, skip;
};

// A value that is the same in every lane (the CG's step lengths, from block
// sums), moved to scalar registers so that the plane loops keep their vector
// registers for the vectors.
__device__ __forceinline__ float uniform(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ double uniform(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffLL));
  const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
  return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}
template <typename T>
__device__ __forceinline__ XStep<T> uniform(XStep<T> s) {
  return XStep<T>{uniform(s.ap), uniform(s.ar), s.zero, s.skip};
}

// The NK Laplacian of a general cell in the CG frame (x', y' in the LDS plane,
// z' the sweep axis).  Arms inside the sweep plane read the staged plane at
// one LDS step off per grid step; arms that leave it (oriented so that one
// step raises z' by one) are gathered plane by plane into a window of partial
// sums; the z' axis arm uses the register window of the point's own column.
template <typename T>
struct GenStencilT {
  T w[4];         // second-derivative weights w_0..w_3
  T cz;           // coefficient of the z' axis arm (0 when it has none)
  T diag;         // w_0 * (sum of all arm coefficients)
  int n_in, n_tl;
  int in_off[3];  // in-plane arms: LDS offset of one step, coefficient
  T in_coef[3];
  int tl_off[3];  // arms leaving the plane: LDS offset of one step (with z' + 1)
  T tl_coef[3];
  T tl_cw[3][4];  // tl_coef[k] * w[q], and cz * w[q] (made on the host, rounded once)
  T czw[4];
};

// Loads and stores of the CG vectors (global memory) at a 32-bit element
// index from the workgroup's uniform base: the address is one 32-bit offset
// register on top of the base held in scalar registers.
#define EXX_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ T gload(const T* base, unsigned idx) {
  return *(const EXX_GLOBAL T*)((const EXX_GLOBAL char*)base + idx * (unsigned)sizeof(T));
}
template <typename T>
__device__ __forceinline__ void gstore(T* base, unsigned idx, T v) {
  *(EXX_GLOBAL T*)((EXX_GLOBAL char*)base + idx * (unsigned)sizeof(T)) = v;
}
// plane start of plane index k (the same for every thread)
__device__ __forceinline__ unsigned plane_base(const int* pst, int k) {
  return (unsigned)__builtin_amdgcn_readfirstlane(pst[k]);
}

struct SolveKArgs {
  const ClassDev* cls;
  const PairDev* pairs;
  const int* order;
  long long p0, npair;    // batch start and capacity; the batch holds min(npair, *n_eff - p0) pairs
  const int* n_eff;       // device pair count of the processing order
  int cls_id;             // >= 0: only the rows of this sphere class (class_cnt, ncls give the ranges)
  const int* class_cnt;
  int ncls;
  int* queue;
  double* bx_ws;          // per pair: right-hand side in, solution out
  long long rstride;
  void* slot_ws;          // per workgroup: CG vectors
  long long sstride;      // elements per vector
  long long slot_bytes;   // bytes per workgroup slot
  int* outIt;
  double* outRes;
  int* outUpd;            // mixed: reliable updates per pair
  int* outSav;            // sweeps that saved two vector accesses per point, per pair (a fused
                          // sweep, or a pass B that left x alone; both in one sweep count twice)
  int* outExit;           // per pair: exit reason (kCg*) | restarts << 8
  double tol;
  int max_iter;
  double delta;           // mixed: update when ||r|| < delta * (residual at the last update)
  StencilT<double> S;
  int gen;                 // general cell: padded columns and the NK arms in G
  int quads;               // orthorhombic cell in the quad layout (one run of four columns per thread)
  GenStencilT<double> G;
  // G in FP32 for the mixed passes, made on the host: the passes index the
  // arms with a runtime index, which reads kernel arguments with scalar
  // loads, where a local copy would live in scratch memory
  GenStencilT<float> G32;
  int lds_cx, lds_cy, lds_wx, lds_wy;
  // warm start (warm_store null: every solve starts from zero)
  const float* warm_store;   // [2][warm_cap][rstride]; the previous solutions are half warm_state[0]
  long long warm_cap;
  const int* warm_state;
  const int* warm_map;       // row of each pair in the previous list, or -1
  const PairDev* prev_pairs;
  int n;                     // stencil half-width (origin of the class lookup maps)
  int N[3];                  // grid, for the periodic change of a pair's grid centre
};

// Packed PE index of local offset (ox, oy, oz) in class C, or -1 off the sphere.
__device__ __forceinline__ int pe_index(const ClassDev& C, int n, int ox, int oy, int oz) {
  const int mx = ox + C.Rg[0] + n, my = oy + C.Rg[1] + n;
  if (mx < 0 || my < 0 || mx >= C.Wm[0] || my >= C.Wm[1]) return -1;
  if (C.pe_map) {   // general cell
    const int mz = oz + C.Rg[2] + n;
    if (mz < 0 || mz >= C.Wm[2]) return -1;
    return C.pe_map[mx + C.Wm[0] * (my + C.Wm[1] * mz)];
  }
  const int m2 = mx + C.Wm[0] * my;
  const int zr = C.zr_map[m2];
  if (zr < 0 || abs(oz) > zr) return -1;
  return C.plane_start[oz + C.Zmax] + C.col_map[m2];
}

// Initial guess of a warm-started solve: the previous solution of the same
// pair, moved by the change of its grid centre (at most one point per axis;
// points that come from outside the previous sphere start at zero), into x
// for the pair's points.  Returns false when the pair starts from zero.
template <typename TX>
__device__ bool warm_gather(const SolveKArgs& a, const ClassDev& C, int pid, TX* x) {
  if (!a.warm_store) return false;
  const int q = a.warm_map[pid];
  if (q < 0) return false;
  const PairDev P = a.pairs[pid], Q = a.prev_pairs[q];
  int d[3];
  for (int ax = 0; ax < 3; ++ax) {
    d[ax] = P.c[ax] - Q.c[ax];
    if (d[ax] > a.N[ax] / 2) d[ax] -= a.N[ax];
    if (d[ax] < -a.N[ax] / 2) d[ax] += a.N[ax];
  }
  const float* prev = a.warm_store + (long long)a.warm_state[0] * a.warm_cap * a.rstride + (long long)q * a.rstride;
  for (long long k = threadIdx.x; k < C.n_pe; k += blockDim.x) {
    const short4 o = C.me_off[k];
    const int idx = o.w ? -1 : pe_index(C, a.n, o.x + d[0], o.y + d[1], o.z + d[2]);
    x[k] = idx >= 0 ? (TX)prev[idx] : (TX)0;
  }
  return true;
}

// This pair's solution, for the next evaluation's warm start.
__device__ __forceinline__ void warm_store_solution(const SolveKArgs& a, long long npe, int pid, const double* x) {
  if (!a.warm_store) return;
  float* cur = const_cast<float*>(a.warm_store) + (long long)(1 - a.warm_state[0]) * a.warm_cap * a.rstride +
               (long long)pid * a.rstride;
  for (long long k = threadIdx.x; k < npe; k += blockDim.x) cur[k] = (float)x[k];
}

// -(stencil Laplacian) at one point in the arithmetic of T: ctr is the centre
// value, pl the LDS plane (values of the current plane, zero off the PE
// sphere), wz the z window
template <int NS, typename T>
__device__ __forceinline__ T apply_point(const StencilT<T>& S, T ctr, const T* pl, int pos, const T* wz) {
  T sx = 0, sy = 0, sz = 0;
#pragma unroll
  for (int q = 1; q <= NS; ++q) {
    sx += S.w[q] * (pl[pos + q] + pl[pos - q]);
    sy += S.w[q] * (pl[pos + q * kLdsWX] + pl[pos - q * kLdsWX]);
    sz += S.w[q] * (wz[NS + q] + wz[NS - q]);
  }
  return -(S.diag * ctr + S.c[0] * sx + S.c[1] * sy + S.c[2] * sz);
}

template <int CPT>
struct Cols {
  int zr[CPT];    // half-height, -1 for no column
  int pos[CPT];   // LDS plane position
  int col[CPT];   // column index (valid only when zr >= 0)
};

template <int CPT, int NT>
__device__ __forceinline__ void load_cols(const ClassDev& C, const SolveKArgs& a, Cols<CPT>& cl) {
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    const int col = threadIdx.x + c * NT;
    cl.zr[c] = -1;
    cl.col[c] = 0;
    cl.pos[c] = 0;
    if (col < C.n_cols) {
      const int4 cc = C.cols[col];
      cl.zr[c] = cc.z;
      cl.col[c] = col;
      cl.pos[c] = (cc.x + a.lds_cx) + kLdsWX * (cc.y + a.lds_cy);
    }
  }
}

// Rows [lo, hi) of the processing order this launch solves: the batch, cut
// to the stored pairs and, for a per-class launch, to the class's rows
// (classes are laid out in descending class index).
__device__ __forceinline__ void solve_range(const SolveKArgs& a, long long* lo, long long* hi) {
  long long l = a.p0, h = a.p0 + a.npair;
  const long long ne = *a.n_eff;
  if (h > ne) h = ne;
  if (a.cls_id >= 0) {
    long long start = 0;
    for (int k = a.ncls - 1; k > a.cls_id; --k) start += a.class_cnt[k];
    const long long end = start + a.class_cnt[a.cls_id];
    if (l < start) l = start;
    if (h > end) h = end;
  }
  *lo = l;
  *hi = h;
}

#define EXX_VALID(c, zz) (abs(zz) <= cl.zr[c])
#define EXX_IDX(c, zz) (plane_base(pst, (zz) + Zmax) + (unsigned)cl.col[c])

// Pass A of a CG iteration: p = r + beta p (p = r on the first iteration) is
// stored, q = A p is formed on the fly; accumulates p.q and r.r in FP64.
template <int NS, int CPT, int PD, typename T>
__device__ void cg_pass_a(const StencilT<T>& S, const Cols<CPT>& cl, const int* pst, int Zmax, const T* __restrict__ r,
                          T* __restrict__ p, T beta, bool first, T* pl0, T* pl1, double& pq, double& rr) {
  T win[CPT][2 * NS + 1];
  T qr[PD][CPT], qp[PD][CPT];   // raw r, p of planes z+NS+1 .. z+NS+PD
  pq = 0.0;
  rr = 0.0;
#pragma unroll
  for (int k = 0; k < 2 * NS + 1; ++k) {
    const int zz = -Zmax - NS + k;
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      T v = 0;
      if (EXX_VALID(c, zz)) {
        const unsigned idx = EXX_IDX(c, zz);
        const T rv = gload(r, idx);
        v = first ? rv : rv + beta * gload(p, idx);
        gstore(p, idx, v);
        rr += (double)rv * (double)rv;
      }
      win[c][k] = v;
    }
  }
#pragma unroll
  for (int d = 0; d < PD; ++d) {
    const int zz = -Zmax + NS + 1 + d;
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      qr[d][c] = 0;
      qp[d][c] = 0;
      if (EXX_VALID(c, zz)) {
        const unsigned idx = EXX_IDX(c, zz);
        qr[d][c] = gload(r, idx);
        if (!first) qp[d][c] = gload(p, idx);
      }
    }
  }
  for (int z = -Zmax; z <= Zmax; ++z) {
    const int zl = z + NS + PD + 1;   // plane whose loads are issued now
    T nr[CPT], np[CPT];
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      nr[c] = 0;
      np[c] = 0;
      if (EXX_VALID(c, zl)) {
        const unsigned idx = EXX_IDX(c, zl);
        nr[c] = gload(r, idx);
        if (!first) np[c] = gload(p, idx);
      }
    }
    T* pl = (z & 1) ? pl1 : pl0;
#pragma unroll
    for (int c = 0; c < CPT; ++c)
      if (cl.zr[c] >= 0) pl[cl.pos[c]] = win[c][NS];
    __syncthreads();
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      if (EXX_VALID(c, z))
        pq += (double)win[c][NS] * (double)apply_point<NS, T>(S, win[c][NS], pl, cl.pos[c], win[c]);
    }
    const int zc = z + NS + 1;        // plane entering the window
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
#pragma unroll
      for (int k = 0; k < 2 * NS; ++k) win[c][k] = win[c][k + 1];
      T v = 0;
      if (EXX_VALID(c, zc)) {
        v = first ? qr[0][c] : qr[0][c] + beta * qp[0][c];
        gstore(p, EXX_IDX(c, zc), v);
        rr += (double)qr[0][c] * (double)qr[0][c];
      }
      win[c][2 * NS] = v;
#pragma unroll
      for (int d = 0; d + 1 < PD; ++d) {
        qr[d][c] = qr[d + 1][c];
        qp[d][c] = qp[d + 1][c];
      }
      qr[PD - 1][c] = nr[c];
      qp[PD - 1][c] = np[c];
    }
  }
}

// Pass B: q = A p again (same arithmetic as pass A), x += alpha p,
// r -= alpha q; returns this thread's FP64 sum of r^2 after the update.  The
// residual is read from r_in and written to r (they may alias); x is updated
// as xs says (see XStep); with xs.zero the old x is taken as zero (and x may
// alias r_in: each point is read before it is written, by the same thread).
template <int NS, int CPT, int PD, bool SKIP, typename T>
__device__ double cg_pass_b_x(const StencilT<T>& S, const Cols<CPT>& cl, const int* pst, int Zmax, T* x,
                            const T* r_in, T* r, const T* __restrict__ p, T alpha, XStep<T> xs, T* pl0, T* pl1) {
  T win[CPT][2 * NS + 1];
  T qp[PD][CPT];           // p of planes z+NS+1 .. z+NS+PD
  T cx[CPT], cr[CPT];      // x, r of plane z
#pragma unroll
  for (int k = 0; k < 2 * NS + 1; ++k) {
    const int zz = -Zmax - NS + k;
#pragma unroll
    for (int c = 0; c < CPT; ++c) win[c][k] = EXX_VALID(c, zz) ? gload(p, EXX_IDX(c, zz)) : (T)0;
  }
#pragma unroll
  for (int d = 0; d < PD; ++d) {
    const int zz = -Zmax + NS + 1 + d;
#pragma unroll
    for (int c = 0; c < CPT; ++c) qp[d][c] = EXX_VALID(c, zz) ? gload(p, EXX_IDX(c, zz)) : (T)0;
  }
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    cx[c] = 0;
    cr[c] = 0;
    if (EXX_VALID(c, -Zmax)) {
      const unsigned idx = EXX_IDX(c, -Zmax);
      cr[c] = gload(r_in, idx);
      if (!SKIP && !xs.zero) cx[c] = gload(x, idx);
    }
  }
  double acc = 0.0;
  for (int z = -Zmax; z <= Zmax; ++z) {
    const int zl = z + NS + PD + 1;
    T np[CPT], nx[CPT], nr[CPT];
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      np[c] = EXX_VALID(c, zl) ? gload(p, EXX_IDX(c, zl)) : (T)0;
      nx[c] = 0;
      nr[c] = 0;
      if (EXX_VALID(c, z + 1)) {
        const unsigned idx = EXX_IDX(c, z + 1);
        nr[c] = gload(r_in, idx);
        if (!SKIP && !xs.zero) nx[c] = gload(x, idx);
      }
    }
    T* pl = (z & 1) ? pl1 : pl0;
#pragma unroll
    for (int c = 0; c < CPT; ++c)
      if (cl.zr[c] >= 0) pl[cl.pos[c]] = win[c][NS];
    __syncthreads();
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      if (EXX_VALID(c, z)) {
        const unsigned idx = EXX_IDX(c, z);
        const T q = apply_point<NS, T>(S, win[c][NS], pl, cl.pos[c], win[c]);
        const T rn = cr[c] - alpha * q;
        if constexpr (!SKIP) gstore(x, idx, cx[c] + xs.ap * win[c][NS] + xs.ar * cr[c]);
        gstore(r, idx, rn);
        acc += (double)rn * (double)rn;
      }
    }
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
#pragma unroll
      for (int k = 0; k < 2 * NS; ++k) win[c][k] = win[c][k + 1];
      win[c][2 * NS] = qp[0][c];
#pragma unroll
      for (int d = 0; d + 1 < PD; ++d) qp[d][c] = qp[d + 1][c];
      qp[PD - 1][c] = np[c];
      cx[c] = nx[c];
      cr[c] = nr[c];
    }
  }
  return acc;
}

// The two forms of pass B as separate loops (as on the quad layout): one
// that leaves x alone keeps no x values live across the plane loop.
template <int NS, int CPT, int PD, typename T>
__device__ __forceinline__ double cg_pass_b(const StencilT<T>& S, const Cols<CPT>& cl, const int* pst, int Zmax,
                                            T* x, const T* r_in, T* r, const T* __restrict__ p, T alpha, XStep<T> xs,
                                            T* pl0, T* pl1) {
  if (xs.skip) return cg_pass_b_x<NS, CPT, PD, true, T>(S, cl, pst, Zmax, x, r_in, r, p, alpha, xs, pl0, pl1);
  return cg_pass_b_x<NS, CPT, PD, false, T>(S, cl, pst, Zmax, x, r_in, r, p, alpha, xs, pl0, pl1);
}

// Reliable update of the mixed-precision solve, in FP64, second half: with the
// accumulated FP32 correction already folded into the FP64 solution x (see
// k_solve_mixed), the true residual b - A x is recomputed and stored, times rs
// and rounded to FP32, as the new working residual.  Returns this thread's
// FP64 sum of the (unscaled) true residual^2.  One plane of loads ahead: the
// pass runs a few times per solve, and its registers bound the whole kernel's.
template <int NS, int CPT, typename TR>
__device__ double cg_true_residual(const StencilT<double>& S, const Cols<CPT>& cl, const int* pst, int Zmax,
                                   const double* __restrict__ x, const double* __restrict__ b,
                                   TR* __restrict__ r, double rs, double* pl0, double* pl1) {
  double win[CPT][2 * NS + 1];
#pragma unroll
  for (int k = 0; k < 2 * NS + 1; ++k) {
    const int zz = -Zmax - NS + k;
#pragma unroll
    for (int c = 0; c < CPT; ++c) win[c][k] = EXX_VALID(c, zz) ? gload(x, EXX_IDX(c, zz)) : 0.0;
  }
  double acc = 0.0;
  for (int z = -Zmax; z <= Zmax; ++z) {
    const int zc = z + NS + 1;        // plane entering the window
    double nx[CPT], cb[CPT];
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      nx[c] = EXX_VALID(c, zc) ? gload(x, EXX_IDX(c, zc)) : 0.0;
      cb[c] = EXX_VALID(c, z) ? gload(b, EXX_IDX(c, z)) : 0.0;
    }
    double* pl = (z & 1) ? pl1 : pl0;
#pragma unroll
    for (int c = 0; c < CPT; ++c)
      if (cl.zr[c] >= 0) pl[cl.pos[c]] = win[c][NS];
    __syncthreads();
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      if (EXX_VALID(c, z)) {
        const double rt = cb[c] - apply_point<NS, double>(S, win[c][NS], pl, cl.pos[c], win[c]);
        gstore(r, EXX_IDX(c, z), (TR)(rt * rs));
        acc += rt * rt;
      }
    }
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
#pragma unroll
      for (int k = 0; k < 2 * NS; ++k) win[c][k] = win[c][k + 1];
      win[c][2 * NS] = nx[c];
    }
  }
  return acc;
}

#undef EXX_VALID
#undef EXX_IDX

// ---------------------------------------------------------------------------
// General cells.  Columns are padded to a symmetric z' range, so plane z' is
// still a prefix of the column order and the index is pst[z' + Zmax] + col;
// a slot holds a point only for lo <= z' <= hi (dead slots are never read or
// written here, and read as zero through the LDS plane).

template <int CPT>
struct ColsG {
  int lo[CPT], hi[CPT];   // z' interval of the column (lo > hi: no column)
  int pos[CPT];           // LDS plane position
  int col[CPT];
};

template <int CPT, int NT>
__device__ __forceinline__ void load_cols_gen(const ClassDev& C, const SolveKArgs& a, ColsG<CPT>& cl) {
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    const int col = threadIdx.x + c * NT;
    cl.lo[c] = 1;
    cl.hi[c] = 0;
    cl.col[c] = 0;
    cl.pos[c] = 0;
    if (col < C.n_cols) {
      const int4 cc = C.cols[col];
      cl.lo[c] = cc.z;
      cl.hi[c] = cc.w;
      cl.col[c] = col;
      cl.pos[c] = (cc.x + a.lds_cx) + kLdsWX * (cc.y + a.lds_cy);
    }
  }
}

#define EXX_GVALID(c, zz) ((zz) >= cl.lo[c] && (zz) <= cl.hi[c])
#define EXX_GHAS(c) (cl.lo[c] <= cl.hi[c])
#define EXX_GIDX(c, zz) (plane_base(pst, (zz) + Zmax) + (unsigned)cl.col[c])

// Laplacian sum at a point from its own column (z' arm, centre) and the
// in-plane arms (staged plane pl)
template <int NS, typename T>
__device__ __forceinline__ T gen_inplane(const GenStencilT<T>& S, T ctr, const T* pl, int pos, const T* wz) {
  T sz = 0;
#pragma unroll
  for (int q = 1; q <= NS; ++q) sz += S.w[q] * (wz[NS + q] + wz[NS - q]);
  T s = S.diag * ctr + S.cz * sz;
  for (int k = 0; k < S.n_in; ++k) {
    const int off = S.in_off[k];
    T t = 0;
#pragma unroll
    for (int q = 1; q <= NS; ++q) t += S.w[q] * (pl[pos + q * off] + pl[pos - q * off]);
    s += S.in_coef[k] * t;
  }
  return s;
}

// Arms leaving the plane: plane z' is the +q neighbour of the column's point
// at z' - q and the -q neighbour of its point at z' + q.  acc[k] holds the
// partial sum of the point at z' - DL + k (DL = n).
template <int NS, int DL, typename T>
__device__ __forceinline__ void gen_tilted(const GenStencilT<T>& S, const T* pl, int pos, T* acc) {
  if constexpr (DL > 0) {
    const T* bp = pl + pos;   // the point's slot: each neighbour is one add of a uniform offset
    // at most three arms leave the plane: the loop unrolls, with a uniform
    // test per arm slot (measured on tri64: the mixed CG 9% faster; unrolling
    // the in-plane arm loop as well made it slower again)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      if (k >= S.n_tl) break;
      const int off = S.tl_off[k];
#pragma unroll
      for (int q = 1; q <= NS; ++q) {
        acc[DL - q] += S.tl_cw[k][q] * bp[q * off];
        acc[DL + q] += S.tl_cw[k][q] * bp[-q * off];
      }
    }
  }
}

// Pass A (general cell, every arm inside the sweep plane or along z'): as
// cg_pass_a, with the in-plane arms at runtime LDS offsets.
template <int NS, int CPT, int PD, typename T>
__device__ void cg_pass_a_gen(const GenStencilT<T>& S, const ColsG<CPT>& cl, const int* pst, int Zmax,
                              const T* __restrict__ r, T* __restrict__ p, T beta, bool first, T* pl0, T* pl1,
                              double& pq, double& rr) {
  T win[CPT][2 * NS + 1];
  T qr[PD][CPT], qp[PD][CPT];
  pq = 0.0;
  rr = 0.0;
#pragma unroll
  for (int k = 0; k < 2 * NS + 1; ++k) {
    const int zz = -Zmax - NS + k;
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      T v = 0;
      if (EXX_GVALID(c, zz)) {
        const unsigned idx = EXX_GIDX(c, zz);
        const T rv = gload(r, idx);
        v = first ? rv : rv + beta * gload(p, idx);
        gstore(p, idx, v);
        rr += (double)rv * (double)rv;
      }
      win[c][k] = v;
    }
  }
#pragma unroll
  for (int d = 0; d < PD; ++d) {
    const int zz = -Zmax + NS + 1 + d;
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      qr[d][c] = 0;
      qp[d][c] = 0;
      if (EXX_GVALID(c, zz)) {
        const unsigned idx = EXX_GIDX(c, zz);
        qr[d][c] = gload(r, idx);
        if (!first) qp[d][c] = gload(p, idx);
      }
    }
  }
  for (int z = -Zmax; z <= Zmax; ++z) {
    const int zl = z + NS + PD + 1;
    T nr[CPT], np[CPT];
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      nr[c] = 0;
      np[c] = 0;
      if (EXX_GVALID(c, zl)) {
        const unsigned idx = EXX_GIDX(c, zl);
        nr[c] = gload(r, idx);
        if (!first) np[c] = gload(p, idx);
      }
    }
    T* pl = (z & 1) ? pl1 : pl0;
#pragma unroll
    for (int c = 0; c < CPT; ++c)
      if (EXX_GHAS(c)) pl[cl.pos[c]] = win[c][NS];
    __syncthreads();
#pragma unroll
    for (int c = 0; c < CPT; ++c)
      if (EXX_GVALID(c, z))
        pq -= (double)win[c][NS] * (double)gen_inplane<NS, T>(S, win[c][NS], pl, cl.pos[c], win[c]);
    const int zc = z + NS + 1;
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
#pragma unroll
      for (int k = 0; k < 2 * NS; ++k) win[c][k] = win[c][k + 1];
      T v = 0;
      if (EXX_GVALID(c, zc)) {
        v = first ? qr[0][c] : qr[0][c] + beta * qp[0][c];
        gstore(p, EXX_GIDX(c, zc), v);
        rr += (double)qr[0][c] * (double)qr[0][c];
      }
      win[c][2 * NS] = v;
#pragma unroll
      for (int d = 0; d + 1 < PD; ++d) {
        qr[d][c] = qr[d + 1][c];
        qp[d][c] = qp[d + 1][c];
      }
      qr[PD - 1][c] = nr[c];
      qp[PD - 1][c] = np[c];
    }
  }
}

// Pass B (general cell, in-plane arms): as cg_pass_b; the plane's x and r
// are loaded in the step that updates them (ahead of the barrier), which
// keeps two fewer values per column live across steps.  Each point's r_in and
// x are read before the same thread writes them.
template <int NS, int CPT, int PD, typename T>
__device__ double cg_pass_b_gen(const GenStencilT<T>& S, const ColsG<CPT>& cl, const int* pst, int Zmax, T* x,
                                const T* r_in, T* r, const T* __restrict__ p, T alpha, XStep<T> xs, T* pl0, T* pl1) {
  T win[CPT][2 * NS + 1];
  T qp[PD][CPT];
#pragma unroll
  for (int k = 0; k < 2 * NS + 1; ++k) {
    const int zz = -Zmax - NS + k;
#pragma unroll
    for (int c = 0; c < CPT; ++c) win[c][k] = EXX_GVALID(c, zz) ? gload(p, EXX_GIDX(c, zz)) : (T)0;
  }
#pragma unroll
  for (int d = 0; d < PD; ++d) {
    const int zz = -Zmax + NS + 1 + d;
#pragma unroll
    for (int c = 0; c < CPT; ++c) qp[d][c] = EXX_GVALID(c, zz) ? gload(p, EXX_GIDX(c, zz)) : (T)0;
  }
  double sum = 0.0;
  for (int z = -Zmax; z <= Zmax; ++z) {
    const int zl = z + NS + PD + 1;
    T np[CPT], ox[CPT], orr[CPT];
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      np[c] = EXX_GVALID(c, zl) ? gload(p, EXX_GIDX(c, zl)) : (T)0;
      ox[c] = 0;
      orr[c] = 0;
      if (EXX_GVALID(c, z)) {
        const unsigned idx = EXX_GIDX(c, z);
        orr[c] = gload(r_in, idx);
        if (!xs.zero && !xs.skip) ox[c] = gload(x, idx);
      }
    }
    T* pl = (z & 1) ? pl1 : pl0;
#pragma unroll
    for (int c = 0; c < CPT; ++c)
      if (EXX_GHAS(c)) pl[cl.pos[c]] = win[c][NS];
    __syncthreads();
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      if (EXX_GVALID(c, z)) {
        const unsigned idx = EXX_GIDX(c, z);
        const T lap = gen_inplane<NS, T>(S, win[c][NS], pl, cl.pos[c], win[c]);
        const T rn = orr[c] + alpha * lap;   // r - alpha A p, A p = -lap
        if (!xs.skip) gstore(x, idx, ox[c] + xs.ap * win[c][NS] + xs.ar * orr[c]);
        gstore(r, idx, rn);
        sum += (double)rn * (double)rn;
      }
    }
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
#pragma unroll
      for (int k = 0; k < 2 * NS; ++k) win[c][k] = win[c][k + 1];
      win[c][2 * NS] = qp[0][c];
#pragma unroll
      for (int d = 0; d + 1 < PD; ++d) qp[d][c] = qp[d + 1][c];
      qp[PD - 1][c] = np[c];
    }
  }
  return sum;
}

// FP64 true residual b - A x of a general cell with in-plane arms (see
// cg_true_residual).
template <int NS, int CPT, typename TR>
__device__ double cg_true_residual_gen(const GenStencilT<double>& S, const ColsG<CPT>& cl, const int* pst, int Zmax,
                                       const double* __restrict__ x, const double* __restrict__ b,
                                       TR* __restrict__ r, double rs, double* pl0, double* pl1) {
  double win[CPT][2 * NS + 1];
#pragma unroll
  for (int k = 0; k < 2 * NS + 1; ++k) {
    const int zz = -Zmax - NS + k;
#pragma unroll
    for (int c = 0; c < CPT; ++c) win[c][k] = EXX_GVALID(c, zz) ? gload(x, EXX_GIDX(c, zz)) : 0.0;
  }
  double sum = 0.0;
  for (int z = -Zmax; z <= Zmax; ++z) {
    const int zc = z + NS + 1;
    double nx[CPT], cb[CPT];
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      nx[c] = EXX_GVALID(c, zc) ? gload(x, EXX_GIDX(c, zc)) : 0.0;
      cb[c] = EXX_GVALID(c, z) ? gload(b, EXX_GIDX(c, z)) : 0.0;
    }
    double* pl = (z & 1) ? pl1 : pl0;
#pragma unroll
    for (int c = 0; c < CPT; ++c)
      if (EXX_GHAS(c)) pl[cl.pos[c]] = win[c][NS];
    __syncthreads();
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      if (EXX_GVALID(c, z)) {
        const double rt = cb[c] + gen_inplane<NS, double>(S, win[c][NS], pl, cl.pos[c], win[c]);
        gstore(r, EXX_GIDX(c, z), (TR)(rt * rs));
        sum += rt * rt;
      }
    }
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
#pragma unroll
      for (int k = 0; k < 2 * NS; ++k) win[c][k] = win[c][k + 1];
      win[c][2 * NS] = nx[c];
    }
  }
  return sum;
}

// ---------------------------------------------------------------------------
// General cells with arms leaving the sweep plane.  Every arm, the z' axis
// included, is applied by scattering the staged plane z' into acc[k], the
// Laplacian partial sums of the column's points at z' - n + k; the point at
// z' - n is complete after plane z'.  Besides acc, a column keeps p of its last
// n + 1 planes and loads one plane ahead, so a thread holds about 2.5 (2n + 1)
// values per column instead of the 2n + 1 window plus the 2n + 1 sums.

template <int NS, typename T>
__device__ __forceinline__ void tl_scatter(const GenStencilT<T>& S, T v, bool point, const T* pl, int pos, T* acc) {
  if (point) {   // the point (column, z') exists: centre and in-plane arms
    T s = S.diag * v;
    const T* bp = pl + pos;
    for (int k = 0; k < S.n_in; ++k) {
      const int off = S.in_off[k];
      T t = 0;
#pragma unroll
      for (int q = 1; q <= NS; ++q) t += S.w[q] * (bp[q * off] + bp[-q * off]);
      s += S.in_coef[k] * t;
    }
    acc[NS] += s;
  }
  // z' arm: v is the +q neighbour of the point q planes down, the -q
  // neighbour of the point q planes up
#pragma unroll
  for (int q = 1; q <= NS; ++q) {
    const T t = S.czw[q] * v;
    acc[NS - q] += t;
    acc[NS + q] += t;
  }
  gen_tilted<NS, NS, T>(S, pl, pos, acc);
}

// With QS (the fused sweeps below), pass A also stores Ap in q and forms
// r.Ap and |Ap|^2 (r of the completed point kept in a window like p).
template <int NS, int CPT, typename T, bool QS = false>
__device__ void cg_pass_a_tl(const GenStencilT<T>& S, const ColsG<CPT>& cl, const int* pst, int Zmax,
                             const T* __restrict__ r, T* __restrict__ p, T beta, bool first, T* pl0, T* pl1,
                             double& pq, double& rr, T* __restrict__ q = nullptr, double* ra = nullptr,
                             double* aa = nullptr) {
  T pd[CPT][NS + 1];       // p of planes z - n .. z
  T rd[CPT][QS ? NS + 1 : 1];   // (QS) r of planes z - n .. z
  T acc[CPT][2 * NS + 1];
  T cr[CPT], cp[CPT];      // r and the previous p of plane z
  double sra = 0.0, saa = 0.0;
  pq = 0.0;
  rr = 0.0;
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
#pragma unroll
    for (int k = 0; k < 2 * NS + 1; ++k) acc[c][k] = 0;
#pragma unroll
    for (int k = 0; k < NS + 1; ++k) pd[c][k] = 0;
#pragma unroll
    for (int k = 0; k < (QS ? NS + 1 : 1); ++k) rd[c][k] = 0;
    cr[c] = 0;
    cp[c] = 0;
    if (EXX_GVALID(c, -Zmax)) {
      const unsigned idx = EXX_GIDX(c, -Zmax);
      cr[c] = gload(r, idx);
      if (!first) cp[c] = gload(p, idx);
    }
  }
  for (int z = -Zmax; z <= Zmax + NS; ++z) {
    T nr[CPT], np[CPT];
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      nr[c] = 0;
      np[c] = 0;
      if (EXX_GVALID(c, z + 1)) {
        const unsigned idx = EXX_GIDX(c, z + 1);
        nr[c] = gload(r, idx);
        if (!first) np[c] = gload(p, idx);
      }
    }
    T* pl = (z & 1) ? pl1 : pl0;
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      T v = 0;
      if (EXX_GVALID(c, z)) {
        v = first ? cr[c] : cr[c] + beta * cp[c];
        gstore(p, EXX_GIDX(c, z), v);
        rr += (double)cr[c] * (double)cr[c];
      }
      pd[c][NS] = v;
      if constexpr (QS) rd[c][NS] = EXX_GVALID(c, z) ? cr[c] : (T)0;
      if (EXX_GHAS(c)) pl[cl.pos[c]] = v;
    }
    __syncthreads();
    const int zo = z - NS;
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      if (EXX_GHAS(c)) tl_scatter<NS, T>(S, pd[c][NS], EXX_GVALID(c, z), pl, cl.pos[c], acc[c]);
      if (EXX_GVALID(c, zo)) {
        pq -= (double)pd[c][0] * (double)acc[c][0];
        if constexpr (QS) {
          const T ap = -acc[c][0];
          gstore(q, EXX_GIDX(c, zo), ap);
          sra += (double)rd[c][0] * (double)ap;
          saa += (double)ap * (double)ap;
        }
      }
#pragma unroll
      for (int k = 0; k < 2 * NS; ++k) acc[c][k] = acc[c][k + 1];
      acc[c][2 * NS] = 0;
#pragma unroll
      for (int k = 0; k < NS; ++k) pd[c][k] = pd[c][k + 1];
      if constexpr (QS) {
#pragma unroll
        for (int k = 0; k < NS; ++k) rd[c][k] = rd[c][k + 1];
      }
      cr[c] = nr[c];
      cp[c] = np[c];
    }
  }
  if constexpr (QS) {
    *ra = sra;
    *aa = saa;
  }
}

template <int NS, int CPT, typename T>
__device__ double cg_pass_b_tl(const GenStencilT<T>& S, const ColsG<CPT>& cl, const int* pst, int Zmax, T* x,
                               const T* r_in, T* r, const T* __restrict__ p, T alpha, XStep<T> xs, T* pl0, T* pl1) {
  T pd[CPT][NS + 1];
  T acc[CPT][2 * NS + 1];
  T cp[CPT];               // p of plane z
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
#pragma unroll
    for (int k = 0; k < 2 * NS + 1; ++k) acc[c][k] = 0;
#pragma unroll
    for (int k = 0; k < NS + 1; ++k) pd[c][k] = 0;
    cp[c] = EXX_GVALID(c, -Zmax) ? gload(p, EXX_GIDX(c, -Zmax)) : (T)0;
  }
  double sum = 0.0;
  for (int z = -Zmax; z <= Zmax + NS; ++z) {
    const int zo = z - NS;
    T np[CPT], ox[CPT], orr[CPT];
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      np[c] = EXX_GVALID(c, z + 1) ? gload(p, EXX_GIDX(c, z + 1)) : (T)0;
      ox[c] = 0;
      orr[c] = 0;
      if (EXX_GVALID(c, zo)) {   // read before the same thread writes them below
        const unsigned idx = EXX_GIDX(c, zo);
        orr[c] = gload(r_in, idx);
        if (!xs.zero && !xs.skip) ox[c] = gload(x, idx);
      }
    }
    T* pl = (z & 1) ? pl1 : pl0;
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      pd[c][NS] = cp[c];
      if (EXX_GHAS(c)) pl[cl.pos[c]] = cp[c];
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      if (EXX_GHAS(c)) tl_scatter<NS, T>(S, pd[c][NS], EXX_GVALID(c, z), pl, cl.pos[c], acc[c]);
      if (EXX_GVALID(c, zo)) {
        const unsigned idx = EXX_GIDX(c, zo);
        const T rn = orr[c] + alpha * acc[c][0];   // r - alpha A p, A p = -acc
        if (!xs.skip) gstore(x, idx, ox[c] + xs.ap * pd[c][0] + xs.ar * orr[c]);
        gstore(r, idx, rn);
        sum += (double)rn * (double)rn;
      }
#pragma unroll
      for (int k = 0; k < 2 * NS; ++k) acc[c][k] = acc[c][k + 1];
      acc[c][2 * NS] = 0;
#pragma unroll
      for (int k = 0; k < NS; ++k) pd[c][k] = pd[c][k + 1];
      cp[c] = np[c];
    }
  }
  return sum;
}

// Pass B of iteration k and pass A of k+1 in one sweep, for the tilted-arm
// form, with Ap kept in q between sweeps: the scatter form completes a point's
// Ap only n planes after the point, so (unlike the quad sweep, which forms
// Ap_k again from a window of p_k) the sweep cannot recompute Ap_k in time for
// r_k+1 = r_k - alpha Ap_k at the plane it reaches.  Storing it instead keeps
// one stencil per iteration and as many vector accesses as the two passes
// (r, p, q in and out; x every other iteration, see XStep).  Along the sweep,
// plane z: r_k+1 = r_k - alpha q_k, p_k+1 = r_k+1 + beta p_k (beta from
// |r_k - alpha Ap_k|^2, known before the sweep), x += ap p_k + ar r_k; then
// p_k+1 enters the plane's scatter, and the point n planes behind completes
// Ap_k+1 for q, p_k+1.Ap_k+1, r_k+1.Ap_k+1 and |Ap_k+1|^2.  Returns |r_k+1|^2
// and writes the three products of iteration k+1 to out3.
template <int NS, int CPT, typename T>
__device__ double cg_pass_fused_tl(const GenStencilT<T>& S, const ColsG<CPT>& cl, const int* pst, int Zmax, T* x,
                                   T* r, T* p, T* q, T alpha, T beta, XStep<T> xs, T* pl0, T* pl1,
                                   double (&out3)[3]) {
  T pd[CPT][NS + 1];       // p_k+1 of planes z - n .. z
  T rd[CPT][NS + 1];       // r_k+1 of planes z - n .. z
  T acc[CPT][2 * NS + 1];
  T cr[CPT], cp[CPT], cq[CPT];   // r_k, p_k, Ap_k of plane z
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
#pragma unroll
    for (int k = 0; k < 2 * NS + 1; ++k) acc[c][k] = 0;
#pragma unroll
    for (int k = 0; k < NS + 1; ++k) {
      pd[c][k] = 0;
      rd[c][k] = 0;
    }
    cr[c] = 0;
    cp[c] = 0;
    cq[c] = 0;
    if (EXX_GVALID(c, -Zmax)) {
      const unsigned idx = EXX_GIDX(c, -Zmax);
      cr[c] = gload(r, idx);
      cp[c] = gload(p, idx);
      cq[c] = gload(q, idx);
    }
  }
  double rn = 0.0, pq = 0.0, ra = 0.0, aa = 0.0;
  for (int z = -Zmax; z <= Zmax + NS; ++z) {
    T nr[CPT], np[CPT], nq[CPT], ox[CPT];
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      nr[c] = 0;
      np[c] = 0;
      nq[c] = 0;
      ox[c] = 0;
      if (EXX_GVALID(c, z + 1)) {
        const unsigned idx = EXX_GIDX(c, z + 1);
        nr[c] = gload(r, idx);
        np[c] = gload(p, idx);
        nq[c] = gload(q, idx);
      }
      if (!xs.zero && !xs.skip && EXX_GVALID(c, z)) ox[c] = gload(x, EXX_GIDX(c, z));
    }
    T* pl = (z & 1) ? pl1 : pl0;
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      T rv = 0, pv = 0;
      if (EXX_GVALID(c, z)) {
        const unsigned idx = EXX_GIDX(c, z);
        rv = cr[c] - alpha * cq[c];
        pv = rv + beta * cp[c];
        gstore(r, idx, rv);
        gstore(p, idx, pv);
        rn += (double)rv * (double)rv;
      }
      rd[c][NS] = rv;
      pd[c][NS] = pv;
      if (EXX_GHAS(c)) pl[cl.pos[c]] = pv;
    }
    __syncthreads();
    const int zo = z - NS;
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      if (!xs.skip && EXX_GVALID(c, z)) gstore(x, EXX_GIDX(c, z), ox[c] + xs.ap * cp[c] + xs.ar * cr[c]);
      if (EXX_GHAS(c)) tl_scatter<NS, T>(S, pd[c][NS], EXX_GVALID(c, z), pl, cl.pos[c], acc[c]);
      if (EXX_GVALID(c, zo)) {
        const T ap = -acc[c][0];
        gstore(q, EXX_GIDX(c, zo), ap);
        pq += (double)pd[c][0] * (double)ap;
        ra += (double)rd[c][0] * (double)ap;
        aa += (double)ap * (double)ap;
      }
#pragma unroll
      for (int k = 0; k < 2 * NS; ++k) acc[c][k] = acc[c][k + 1];
      acc[c][2 * NS] = 0;
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        pd[c][k] = pd[c][k + 1];
        rd[c][k] = rd[c][k + 1];
      }
      cr[c] = nr[c];
      cp[c] = np[c];
      cq[c] = nq[c];
    }
  }
  out3[0] = pq;
  out3[1] = ra;
  out3[2] = aa;
  return rn;
}

template <int NS, int CPT, typename TR>
__device__ double cg_true_residual_tl(const GenStencilT<double>& S, const ColsG<CPT>& cl, const int* pst, int Zmax,
                                      const double* __restrict__ x, const double* __restrict__ b,
                                      TR* __restrict__ r, double rs, double* pl0, double* pl1) {
  double acc[CPT][2 * NS + 1];
  double cx[CPT];
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
#pragma unroll
    for (int k = 0; k < 2 * NS + 1; ++k) acc[c][k] = 0.0;
    cx[c] = EXX_GVALID(c, -Zmax) ? gload(x, EXX_GIDX(c, -Zmax)) : 0.0;
  }
  double sum = 0.0;
  for (int z = -Zmax; z <= Zmax + NS; ++z) {
    const int zo = z - NS;
    double nx[CPT], ob[CPT];
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      nx[c] = EXX_GVALID(c, z + 1) ? gload(x, EXX_GIDX(c, z + 1)) : 0.0;
      ob[c] = EXX_GVALID(c, zo) ? gload(b, EXX_GIDX(c, zo)) : 0.0;
    }
    double* pl = (z & 1) ? pl1 : pl0;
#pragma unroll
    for (int c = 0; c < CPT; ++c)
      if (EXX_GHAS(c)) pl[cl.pos[c]] = cx[c];
    __syncthreads();
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      if (EXX_GHAS(c)) tl_scatter<NS, double>(S, cx[c], EXX_GVALID(c, z), pl, cl.pos[c], acc[c]);
      if (EXX_GVALID(c, zo)) {
        const double rt = ob[c] + acc[c][0];   // b - A x, A x = -acc
        gstore(r, EXX_GIDX(c, zo), (TR)(rt * rs));
        sum += rt * rt;
      }
#pragma unroll
      for (int k = 0; k < 2 * NS; ++k) acc[c][k] = acc[c][k + 1];
      acc[c][2 * NS] = 0.0;
      cx[c] = nx[c];
    }
  }
  return sum;
}

#undef EXX_GVALID
#undef EXX_GHAS
#undef EXX_GIDX


// ---------------------------------------------------------------------------
// Quad layout (orthorhombic cells, and general cells whose arms stay in the
// sweep plane with at most one diagonal among them and whose columns are
// symmetric about it; coordinates in the CG frame).  The sphere's columns are
// grouped into runs of four x-adjacent columns of one row (starting at x = 4k on even rows,
// 4k + 2 on odd rows, so a run starts at an even LDS position), padded to the
// run's tallest column: plane z holds the runs whose tallest column reaches
// it, as a prefix of the runs sorted by that height, four slots per run; a
// slot whose own column is shorter (or lies outside the sphere) is dead and
// stays zero.  Thread t owns runs t, t + NT, ... (RQ of them; one in
// workgroups of 768 or 1024 threads, two in workgroups of 512).  A run's four
// points of a plane are one 16-byte (FP32) vector in global memory and two
// 8-byte halves in the LDS plane; the in-plane stencil reads the run's left
// and right neighbours along x (n <= 3 points each) and the rows y +- q as
// such halves.  The x neighbours inside the run are the thread's own
// registers.

template <int RQ>
struct ColsQ {
  int zr[RQ][4];   // half-height of each column, -1 outside the sphere
  int zq[RQ];      // half-height of the run (max zr), -1 for no run
  int pos[RQ];     // LDS plane position of the run's first column (even)
  int base[RQ];    // offset of the run's slots within a plane (4 run)
};

template <int NT, int RQ>
__device__ __forceinline__ void load_cols_quad(const ClassDev& C, const SolveKArgs& a, ColsQ<RQ>& cl) {
#pragma unroll
  for (int u = 0; u < RQ; ++u) {
    const int run = threadIdx.x + u * NT;
    cl.zq[u] = -1;
    cl.pos[u] = 0;
    cl.base[u] = 4 * run;
#pragma unroll
    for (int j = 0; j < 4; ++j) cl.zr[u][j] = -1;
    if (4 * run < C.n_cols) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int4 cc = C.cols[4 * run + j];
        cl.zr[u][j] = cc.z;
        cl.zq[u] = max(cl.zq[u], cc.z);
      }
      const int4 c0 = C.cols[4 * run];
      cl.pos[u] = (c0.x + a.lds_cx) + kLdsWX * (c0.y + a.lds_cy);
    }
  }
}

// A run's four values of one plane.  The passes work on these 4-point vectors
// throughout, so that global accesses stay whole 16-byte (FP32) or 32-byte
// (FP64) accesses and the z window is one register tuple per plane.
template <typename T>
using V4 = T __attribute__((ext_vector_type(4)));

// Global-memory vectors: element idx (a multiple of 4) of the plane-major
// vector at base, which is aligned to the vector size.  The accesses name the
// global address space and take a 32-bit byte offset from the workgroup's
// uniform base.
template <typename T>
__device__ __forceinline__ V4<T> ld_quad(const T* base, int idx) {
  return *(const EXX_GLOBAL V4<T>*)((const EXX_GLOBAL char*)base + (unsigned)idx * (unsigned)sizeof(T));
}
template <typename T>
__device__ __forceinline__ void st_quad(T* base, int idx, V4<T> v) {
  *(EXX_GLOBAL V4<T>*)((EXX_GLOBAL char*)base + (unsigned)idx * (unsigned)sizeof(T)) = v;
}

template <typename T>
__device__ __forceinline__ double dot4(V4<T> a, V4<T> b) {
  return (double)a.x * (double)b.x + (double)a.y * (double)b.y + (double)a.z * (double)b.z +
         (double)a.w * (double)b.w;
}

// plane values K points right (xr) and left (xl) of the run's four columns,
// from the run's own values c and its neighbour vectors lf (x - 4 .. x - 1)
// and rt (x + 4 .. x + 7)
template <int K, typename T>
__device__ __forceinline__ V4<T> shift_right(V4<T> c, V4<T> rt) {
  return __builtin_shufflevector(c, rt, K, K + 1, K + 2, K + 3);
}
template <int K, typename T>
__device__ __forceinline__ V4<T> shift_left(V4<T> lf, V4<T> c) {
  return __builtin_shufflevector(lf, c, 4 - K, 5 - K, 6 - K, 7 - K);
}

// A run's vector in the LDS plane (p even: 8-byte aligned for FP32) as two
// halves of two points.  The compiler barrier keeps the halves separate
// accesses: on gfx950 one 16-byte LDS access per thread occupies the LDS
// longer than two 8-byte ones (measured on the CG).
template <typename T>
__device__ __forceinline__ V4<T> lds_quad(const T* p) {
  using V2 = T __attribute__((ext_vector_type(2)));
  const V2 a = *reinterpret_cast<const V2*>(p);
  __asm__ volatile("" ::: "memory");
  const V2 b = *reinterpret_cast<const V2*>(p + 2);
  return V4<T>{a.x, a.y, b.x, b.y};
}
template <typename T>
__device__ __forceinline__ void lds_quad_store(T* p, V4<T> v) {
  using V2 = T __attribute__((ext_vector_type(2)));
  *reinterpret_cast<V2*>(p) = V2{v.x, v.y};
  __asm__ volatile("" ::: "memory");
  *reinterpret_cast<V2*>(p + 2) = V2{v.z, v.w};
}

// Terms of one step K of the stencil.  With DG, the cell's diagonal arm in the
// sweep plane: step +K reaches (x + K, y + s K), read from the run's vector of
// row y + s K and the one right of it; step -K reaches (x - K, y - s K), from
// row y - s K and the vector left of it.
template <int K, int NS, bool DG, typename T>
__device__ __forceinline__ void quad_terms(const StencilT<T>& S, const V4<T> (&win)[2 * NS + 1], const T* pl,
                                           int pos, V4<T> lf, V4<T> rt, V4<T>& sx, V4<T>& sy, V4<T>& sz,
                                           V4<T>& sdg) {
  if constexpr (K <= NS) {
    const V4<T> up = lds_quad(pl + pos + K * kLdsWX);
    const V4<T> dn = lds_quad(pl + pos - K * kLdsWX);
    sx += S.w[K] * (shift_right<K, T>(win[NS], rt) + shift_left<K, T>(lf, win[NS]));
    sy += S.w[K] * (up + dn);
    sz += S.w[K] * (win[NS + K] + win[NS - K]);
    if constexpr (DG) {
      const int row = S.sd * K * kLdsWX;
      const V4<T> fwd = S.sd > 0 ? up : dn;    // row y + s K
      const V4<T> bwd = S.sd > 0 ? dn : up;    // row y - s K
      const V4<T> fr = lds_quad(pl + pos + row + 4);
      const V4<T> bl = lds_quad(pl + pos - row - 4);
      sdg += S.w[K] * (shift_right<K, T>(fwd, fr) + shift_left<K, T>(bl, bwd));
    }
    quad_terms<K + 1, NS, DG, T>(S, win, pl, pos, lf, rt, sx, sy, sz, sdg);
  }
}

// -(stencil Laplacian) at the run's four points of the staged plane pl, with
// the z window of the run; per point the arithmetic is that of apply_point
// (of the general passes' arm sum, with DG).
template <int NS, bool DG, typename T>
__device__ __forceinline__ V4<T> apply_quad(const StencilT<T>& S, const V4<T> (&win)[2 * NS + 1], const T* pl,
                                            int pos) {
  const V4<T> lf = lds_quad(pl + pos - 4);
  const V4<T> rt = lds_quad(pl + pos + 4);
  V4<T> sx = {0, 0, 0, 0}, sy = {0, 0, 0, 0}, sz = {0, 0, 0, 0}, sdg = {0, 0, 0, 0};
  quad_terms<1, NS, DG, T>(S, win, pl, pos, lf, rt, sx, sy, sz, sdg);
  if constexpr (DG) return -(S.diag * win[NS] + S.c[0] * sx + S.c[1] * sy + S.c[2] * sz + S.cd * sdg);
  return -(S.diag * win[NS] + S.c[0] * sx + S.c[1] * sy + S.c[2] * sz);
}

// v at the live slots of run u in plane z, 0 at its dead ones
template <typename T, int RQ>
__device__ __forceinline__ V4<T> live_only(const ColsQ<RQ>& cl, int u, int z, V4<T> v) {
  const int az = abs(z);
  v.x = az <= cl.zr[u][0] ? v.x : (T)0;
  v.y = az <= cl.zr[u][1] ? v.y : (T)0;
  v.z = az <= cl.zr[u][2] ? v.z : (T)0;
  v.w = az <= cl.zr[u][3] ? v.w : (T)0;
  return v;
}

#define EXX_QVALID(u, zz) (abs(zz) <= cl.zq[u])
#define EXX_QIDX(u, zz) (pst[(zz) + Zmax] + cl.base[u])

// Pass A (cg_pass_a_quad below) for one run per thread (768 and 1024
// threads), in a loop of its own: the loop written for RQ runs compiles at
// RQ = 1 to code that spills registers in the plane loops of the 1024-thread
// kernels.
template <int NS, int PD, bool DG, bool RA, typename T>
__device__ void cg_pass_a_quad_one(const StencilT<T>& S, const ColsQ<1>& cl, const int* pst, int Zmax,
                                   const T* __restrict__ r, T* __restrict__ p, T beta, bool first, T* pl0, T* pl1,
                                   double& pq, double& rr, double& ra, double& aa) {
  const V4<T> zero = {0, 0, 0, 0};
  V4<T> win[2 * NS + 1];
  V4<T> qr[PD], qp[PD];   // raw r, p of planes z+NS+1 .. z+NS+PD
  V4<T> rw[RA ? NS + 1 : 1];   // with RA: r of planes z .. z+NS
  pq = 0.0;
  rr = 0.0;
  ra = 0.0;
  aa = 0.0;
#pragma unroll
  for (int k = 0; k < 2 * NS + 1; ++k) {
    const int zz = -Zmax - NS + k;
    V4<T> v = zero, rv = zero;
    if (EXX_QVALID(0, zz)) {
      const int idx = EXX_QIDX(0, zz);
      rv = ld_quad(r, idx);
      v = first ? rv : rv + beta * ld_quad(p, idx);
      rr += dot4(rv, rv);
      st_quad(p, idx, v);
    }
    win[k] = v;
    if constexpr (RA) {
      if (k >= NS) rw[k - NS] = rv;
    }
  }
#pragma unroll
  for (int d = 0; d < PD; ++d) {
    const int zz = -Zmax + NS + 1 + d;
    qr[d] = zero;
    qp[d] = zero;
    if (EXX_QVALID(0, zz)) {
      qr[d] = ld_quad(r, EXX_QIDX(0, zz));
      if (!first) qp[d] = ld_quad(p, EXX_QIDX(0, zz));
    }
  }
  for (int z = -Zmax; z <= Zmax; ++z) {
    const int zl = z + NS + PD + 1;   // plane whose loads are issued now
    V4<T> nr = zero, np = zero;
    if (EXX_QVALID(0, zl)) {
      nr = ld_quad(r, EXX_QIDX(0, zl));
      if (!first) np = ld_quad(p, EXX_QIDX(0, zl));
    }
    T* pl = (z & 1) ? pl1 : pl0;
    if (cl.zq[0] >= 0) lds_quad_store(pl + cl.pos[0], win[NS]);
    __syncthreads();
    if (EXX_QVALID(0, z)) {
      const V4<T> ap = apply_quad<NS, DG, T>(S, win, pl, cl.pos[0]);
      pq += dot4(win[NS], ap);
      if constexpr (RA) {
        const V4<T> al = live_only(cl, 0, z, ap);
        ra += dot4(rw[0], al);
        aa += dot4(al, al);
      }
    }
    const int zc = z + NS + 1;        // plane entering the window
    V4<T> v = zero;
    if (EXX_QVALID(0, zc)) {
      v = first ? qr[0] : qr[0] + beta * qp[0];
      rr += dot4(qr[0], qr[0]);
      st_quad(p, EXX_QIDX(0, zc), v);
    }
#pragma unroll
    for (int k = 0; k < 2 * NS; ++k) win[k] = win[k + 1];
    win[2 * NS] = v;
    if constexpr (RA) {
#pragma unroll
      for (int k = 0; k < NS; ++k) rw[k] = rw[k + 1];
      rw[NS] = EXX_QVALID(0, zc) ? qr[0] : zero;
    }
#pragma unroll
    for (int d = 0; d + 1 < PD; ++d) {
      qr[d] = qr[d + 1];
      qp[d] = qp[d + 1];
    }
    qr[PD - 1] = nr;
    qp[PD - 1] = np;
  }
}

// Pass A (as cg_pass_a) on the quad layout.  Dead slots hold r = p = 0, so p
// stays zero there and adds nothing to the dot products.  With RA it also
// returns r.Ap and |Ap|^2 (Ap kept to the live slots), from which the next
// residual norm |r - alpha Ap|^2 follows before r is updated; r of the planes
// z .. z+NS is then kept in registers for the product with Ap of plane z.
template <int NS, int PD, bool DG, bool RA, typename T, int RQ>
__device__ void cg_pass_a_quad(const StencilT<T>& S, const ColsQ<RQ>& cl, const int* pst, int Zmax,
                               const T* __restrict__ r, T* __restrict__ p, T beta, bool first, T* pl0, T* pl1,
                               double& pq, double& rr, double& ra, double& aa) {
  if constexpr (RQ == 1) {
    cg_pass_a_quad_one<NS, PD, DG, RA, T>(S, cl, pst, Zmax, r, p, beta, first, pl0, pl1, pq, rr, ra, aa);
    return;
  }
  const V4<T> zero = {0, 0, 0, 0};
  V4<T> win[RQ][2 * NS + 1];
  V4<T> qr[RQ][PD], qp[RQ][PD];   // raw r, p of planes z+NS+1 .. z+NS+PD
  V4<T> rw[RQ][RA ? NS + 1 : 1];   // with RA: r of planes z .. z+NS
  pq = 0.0;
  rr = 0.0;
  ra = 0.0;
  aa = 0.0;
#pragma unroll
  for (int u = 0; u < RQ; ++u) {
#pragma unroll
    for (int k = 0; k < 2 * NS + 1; ++k) {
      const int zz = -Zmax - NS + k;
      V4<T> v = zero, rv = zero;
      if (EXX_QVALID(u, zz)) {
        const int idx = EXX_QIDX(u, zz);
        rv = ld_quad(r, idx);
        v = first ? rv : rv + beta * ld_quad(p, idx);
        rr += dot4(rv, rv);
        st_quad(p, idx, v);
      }
      win[u][k] = v;
      if constexpr (RA) {
        if (k >= NS) rw[u][k - NS] = rv;
      }
    }
#pragma unroll
    for (int d = 0; d < PD; ++d) {
      const int zz = -Zmax + NS + 1 + d;
      qr[u][d] = zero;
      qp[u][d] = zero;
      if (EXX_QVALID(u, zz)) {
        qr[u][d] = ld_quad(r, EXX_QIDX(u, zz));
        if (!first) qp[u][d] = ld_quad(p, EXX_QIDX(u, zz));
      }
    }
  }
  for (int z = -Zmax; z <= Zmax; ++z) {
    const int zl = z + NS + PD + 1;   // plane whose loads are issued now
    V4<T> nr[RQ], np[RQ];
#pragma unroll
    for (int u = 0; u < RQ; ++u) {
      nr[u] = zero;
      np[u] = zero;
      if (EXX_QVALID(u, zl)) {
        nr[u] = ld_quad(r, EXX_QIDX(u, zl));
        if (!first) np[u] = ld_quad(p, EXX_QIDX(u, zl));
      }
    }
    T* pl = (z & 1) ? pl1 : pl0;
#pragma unroll
    for (int u = 0; u < RQ; ++u)
      if (cl.zq[u] >= 0) lds_quad_store(pl + cl.pos[u], win[u][NS]);
    __syncthreads();
#pragma unroll
    for (int u = 0; u < RQ; ++u) {
      if (EXX_QVALID(u, z)) {
        const V4<T> ap = apply_quad<NS, DG, T>(S, win[u], pl, cl.pos[u]);
        pq += dot4(win[u][NS], ap);
        if constexpr (RA) {
          const V4<T> al = live_only(cl, u, z, ap);
          ra += dot4(rw[u][0], al);
          aa += dot4(al, al);
        }
      }
    }
    const int zc = z + NS + 1;        // plane entering the window
#pragma unroll
    for (int u = 0; u < RQ; ++u) {
      V4<T> v = zero;
      if (EXX_QVALID(u, zc)) {
        v = first ? qr[u][0] : qr[u][0] + beta * qp[u][0];
        rr += dot4(qr[u][0], qr[u][0]);
        st_quad(p, EXX_QIDX(u, zc), v);
      }
#pragma unroll
      for (int k = 0; k < 2 * NS; ++k) win[u][k] = win[u][k + 1];
      win[u][2 * NS] = v;
      if constexpr (RA) {
#pragma unroll
        for (int k = 0; k < NS; ++k) rw[u][k] = rw[u][k + 1];
        rw[u][NS] = EXX_QVALID(u, zc) ? qr[u][0] : zero;
      }
#pragma unroll
      for (int d = 0; d + 1 < PD; ++d) {
        qr[u][d] = qr[u][d + 1];
        qp[u][d] = qp[u][d + 1];
      }
      qr[u][PD - 1] = nr[u];
      qp[u][PD - 1] = np[u];
    }
  }
}

// Pass B (as cg_pass_b) on the quad layout; the new r is kept to the run's
// live slots, so dead slots keep r = 0 (and x = 0, since p is zero there).
template <int NS, int PD, bool DG, bool SKIP, typename T, int RQ>
__device__ double cg_pass_b_quad_x(const StencilT<T>& S, const ColsQ<RQ>& cl, const int* pst, int Zmax, T* x,
                                 const T* r_in, T* r, const T* __restrict__ p, T alpha, XStep<T> xs, T* pl0, T* pl1) {
  const V4<T> zero = {0, 0, 0, 0};
  V4<T> win[RQ][2 * NS + 1];
  V4<T> qp[RQ][PD];              // p of planes z+NS+1 .. z+NS+PD
  V4<T> cx[RQ], cr[RQ];          // x, r of plane z
#pragma unroll
  for (int u = 0; u < RQ; ++u) {
#pragma unroll
    for (int k = 0; k < 2 * NS + 1; ++k) {
      const int zz = -Zmax - NS + k;
      win[u][k] = EXX_QVALID(u, zz) ? ld_quad(p, EXX_QIDX(u, zz)) : zero;
    }
#pragma unroll
    for (int d = 0; d < PD; ++d) {
      const int zz = -Zmax + NS + 1 + d;
      qp[u][d] = EXX_QVALID(u, zz) ? ld_quad(p, EXX_QIDX(u, zz)) : zero;
    }
    cx[u] = zero;
    cr[u] = zero;
    if (EXX_QVALID(u, -Zmax)) {
      const int idx = EXX_QIDX(u, -Zmax);
      cr[u] = ld_quad(r_in, idx);
      if (!SKIP && !xs.zero) cx[u] = ld_quad(x, idx);
    }
  }
  double acc = 0.0;
  for (int z = -Zmax; z <= Zmax; ++z) {
    const int zl = z + NS + PD + 1;
    V4<T> np[RQ], nx[RQ], nr[RQ];
#pragma unroll
    for (int u = 0; u < RQ; ++u) {
      np[u] = zero;
      nx[u] = zero;
      nr[u] = zero;
      if (EXX_QVALID(u, zl)) np[u] = ld_quad(p, EXX_QIDX(u, zl));
      if (EXX_QVALID(u, z + 1)) {
        const int idx = EXX_QIDX(u, z + 1);
        nr[u] = ld_quad(r_in, idx);
        if (!SKIP && !xs.zero) nx[u] = ld_quad(x, idx);
      }
    }
    T* pl = (z & 1) ? pl1 : pl0;
#pragma unroll
    for (int u = 0; u < RQ; ++u)
      if (cl.zq[u] >= 0) lds_quad_store(pl + cl.pos[u], win[u][NS]);
    __syncthreads();
#pragma unroll
    for (int u = 0; u < RQ; ++u) {
      if (EXX_QVALID(u, z)) {
        const int idx = EXX_QIDX(u, z);
        const V4<T> rn = live_only(cl, u, z, cr[u] - alpha * apply_quad<NS, DG, T>(S, win[u], pl, cl.pos[u]));
        if constexpr (!SKIP) st_quad(x, idx, cx[u] + xs.ap * win[u][NS] + xs.ar * cr[u]);
        st_quad(r, idx, rn);
        acc += dot4(rn, rn);
      }
#pragma unroll
      for (int k = 0; k < 2 * NS; ++k) win[u][k] = win[u][k + 1];
      win[u][2 * NS] = qp[u][0];
#pragma unroll
      for (int d = 0; d + 1 < PD; ++d) qp[u][d] = qp[u][d + 1];
      qp[u][PD - 1] = np[u];
      cx[u] = nx[u];
      cr[u] = nr[u];
    }
  }
  return acc;
}

// The two forms of pass B as separate loops: one that leaves x alone keeps no
// x vectors live across the plane loop.
template <int NS, int PD, bool DG, typename T, int RQ>
__device__ __forceinline__ double cg_pass_b_quad(const StencilT<T>& S, const ColsQ<RQ>& cl, const int* pst, int Zmax,
                                                 T* x, const T* r_in, T* r, const T* __restrict__ p, T alpha,
                                                 XStep<T> xs, T* pl0, T* pl1) {
  if (xs.skip) return cg_pass_b_quad_x<NS, PD, DG, true, T>(S, cl, pst, Zmax, x, r_in, r, p, alpha, xs, pl0, pl1);
  return cg_pass_b_quad_x<NS, PD, DG, false, T>(S, cl, pst, Zmax, x, r_in, r, p, alpha, xs, pl0, pl1);
}

// Pass B of one iteration and pass A of the next in one sweep on the quad
// layout.  With the step alpha of p (= p_k) and the next beta (which the
// caller takes from |r - alpha Ap|^2, known before r is updated): along the
// sweep, Ap_k of plane c is recomputed from the z window of p_k, then
// x is updated as xs says (with p_k), r -= alpha Ap_k and p_k+1 = r + beta p_k
// are written over the same slots; NS planes behind, Ap_k+1 is taken from the z window of the
// new p, for p_k+1.Ap_k+1, r_k+1.Ap_k+1 and |Ap_k+1|^2 (r_k+1 restated as
// p_k+1 - beta p_k from the two windows).  Each plane is read and written once
// per iteration (p, r, x in; p, r, x out; x only every other iteration when
// its updates are paired, see XStep) instead of twice for p.  Each step
// stages the planes of both stencils (la*, lb*) behind one barrier.
// The two z windows take 56 registers per thread (FP32, n = 3), which fit
// beside the rest only with at most three waves per SIMD (768 threads).
// Returns |r_k+1|^2 and writes the products of iteration k+1 to out3.
template <int NS, int PD, bool DG, typename T, int RQ>
__device__ double cg_pass_fused_quad(const StencilT<T>& S, const ColsQ<RQ>& cl, const int* pst, int Zmax, T* x,
                                     T* r, T* p, T alpha, T beta, XStep<T> xs, T* la0, T* la1, T* lb0, T* lb1,
                                     double (&out3)[3]) {
  const V4<T> zero = {0, 0, 0, 0};
  V4<T> wk[RQ][2 * NS + 1];      // p_k of planes c - NS .. c + NS
  V4<T> wn[RQ][2 * NS + 1];      // p_k+1 of planes c - 2 NS .. c (the top one formed in the step)
  V4<T> qp[RQ][PD];              // p_k of planes c+NS+1 .. c+NS+PD
  V4<T> cx[RQ], cr[RQ];          // x, r of plane c
#pragma unroll
  for (int u = 0; u < RQ; ++u) {
#pragma unroll
    for (int k = 0; k < 2 * NS + 1; ++k) {
      const int zz = -Zmax - NS + k;
      wk[u][k] = EXX_QVALID(u, zz) ? ld_quad(p, EXX_QIDX(u, zz)) : zero;
      wn[u][k] = zero;
    }
#pragma unroll
    for (int d = 0; d < PD; ++d) {
      const int zz = -Zmax + NS + 1 + d;
      qp[u][d] = EXX_QVALID(u, zz) ? ld_quad(p, EXX_QIDX(u, zz)) : zero;
    }
    cx[u] = zero;
    cr[u] = zero;
    if (EXX_QVALID(u, -Zmax)) {
      const int idx = EXX_QIDX(u, -Zmax);
      cr[u] = ld_quad(r, idx);
      if (!xs.zero && !xs.skip) cx[u] = ld_quad(x, idx);
    }
  }
  double rn = 0.0, pq = 0.0, ra = 0.0, aa = 0.0;
  for (int c = -Zmax; c <= Zmax + NS; ++c) {
    const int zl = c + NS + PD + 1;
    V4<T> np[RQ], nx[RQ], nr[RQ];
#pragma unroll
    for (int u = 0; u < RQ; ++u) {
      np[u] = zero;
      nx[u] = zero;
      nr[u] = zero;
      if (EXX_QVALID(u, zl)) np[u] = ld_quad(p, EXX_QIDX(u, zl));
      if (EXX_QVALID(u, c + 1)) {
        const int idx = EXX_QIDX(u, c + 1);
        nr[u] = ld_quad(r, idx);
        if (!xs.zero && !xs.skip) nx[u] = ld_quad(x, idx);
      }
    }
    T* la = (c & 1) ? la1 : la0;
    T* lb = (c & 1) ? lb1 : lb0;
#pragma unroll
    for (int u = 0; u < RQ; ++u) {
      if (cl.zq[u] >= 0) {
        lds_quad_store(la + cl.pos[u], wk[u][NS]);
        lds_quad_store(lb + cl.pos[u], wn[u][NS]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < RQ; ++u) {
      V4<T> pn = zero;
      if (EXX_QVALID(u, c)) {
        const int idx = EXX_QIDX(u, c);
        const V4<T> rn1 = live_only(cl, u, c, cr[u] - alpha * apply_quad<NS, DG, T>(S, wk[u], la, cl.pos[u]));
        pn = rn1 + beta * wk[u][NS];
        if (!xs.skip) st_quad(x, idx, cx[u] + xs.ap * wk[u][NS] + xs.ar * cr[u]);
        st_quad(r, idx, rn1);
        st_quad(p, idx, pn);
        rn += dot4(rn1, rn1);
      }
      wn[u][2 * NS] = pn;
      const int c2 = c - NS;
      if (EXX_QVALID(u, c2)) {
        const V4<T> ap = live_only(cl, u, c2, apply_quad<NS, DG, T>(S, wn[u], lb, cl.pos[u]));
        pq += dot4(wn[u][NS], ap);
        ra += dot4(wn[u][NS] - beta * wk[u][0], ap);
        aa += dot4(ap, ap);
      }
#pragma unroll
      for (int k = 0; k < 2 * NS; ++k) {
        wk[u][k] = wk[u][k + 1];
        wn[u][k] = wn[u][k + 1];
      }
      wk[u][2 * NS] = qp[u][0];
#pragma unroll
      for (int d = 0; d + 1 < PD; ++d) qp[u][d] = qp[u][d + 1];
      qp[u][PD - 1] = np[u];
      cx[u] = nx[u];
      cr[u] = nr[u];
    }
  }
  out3[0] = pq;
  out3[1] = ra;
  out3[2] = aa;
  return rn;
}

// FP64 true residual (as cg_true_residual) on the quad layout, zero at dead
// slots.  It sweeps twice, once per half of the run (columns 2h, 2h+1), with
// a z window of 2-point FP64 vectors: a window of whole runs in FP64 does not
// fit the registers of a 1024-thread workgroup (its plane loop spilled to
// scratch memory).  Each plane still stages the run's four values in LDS.
template <int NS, bool DG, typename TR, int RQ>
__device__ double cg_true_residual_quad(const StencilT<double>& S, const ColsQ<RQ>& cl, const int* pst, int Zmax,
                                        const double* __restrict__ x, const double* __restrict__ b,
                                        TR* __restrict__ r, double rs, double* pl0, double* pl1) {
  using V2d = double __attribute__((ext_vector_type(2)));
  using V2r = TR __attribute__((ext_vector_type(2)));
  const V2d zero2 = {0, 0};
  const V4<double> zero4 = {0, 0, 0, 0};
  auto ld_half = [](const double* base, int idx) {
    return *(const EXX_GLOBAL V2d*)((const EXX_GLOBAL char*)base + (unsigned)idx * 8u);
  };
  double acc = 0.0;
  for (int h = 0; h < 2; ++h) {
    const int off = 2 * h;   // the half's first column within the run
    V2d win[RQ][2 * NS + 1];
#pragma unroll
    for (int u = 0; u < RQ; ++u)
#pragma unroll
      for (int k = 0; k < 2 * NS + 1; ++k) {
        const int zz = -Zmax - NS + k;
        win[u][k] = EXX_QVALID(u, zz) ? ld_half(x, EXX_QIDX(u, zz) + off) : zero2;
      }
    for (int z = -Zmax; z <= Zmax; ++z) {
      const int zc = z + NS + 1;        // plane entering the window
      V2d nx[RQ], cb[RQ];
      double* pl = (z & 1) ? pl1 : pl0;
#pragma unroll
      for (int u = 0; u < RQ; ++u) {
        nx[u] = EXX_QVALID(u, zc) ? ld_half(x, EXX_QIDX(u, zc) + off) : zero2;
        const V4<double> xq = EXX_QVALID(u, z) ? ld_quad(x, EXX_QIDX(u, z)) : zero4;
        cb[u] = EXX_QVALID(u, z) ? ld_half(b, EXX_QIDX(u, z) + off) : zero2;
        if (cl.zq[u] >= 0) lds_quad_store(pl + cl.pos[u], xq);
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < RQ; ++u) {
        if (EXX_QVALID(u, z)) {
          // plane values at x offsets -4 .. 5 from the half's first column
          const int p = cl.pos[u] + off;
          const V2d l2 = *reinterpret_cast<const V2d*>(pl + p - 4), l1 = *reinterpret_cast<const V2d*>(pl + p - 2);
          const V2d r1 = *reinterpret_cast<const V2d*>(pl + p + 2), r2 = *reinterpret_cast<const V2d*>(pl + p + 4);
          const V2d c = win[u][NS];
          const double row[10] = {l2.x, l2.y, l1.x, l1.y, c.x, c.y, r1.x, r1.y, r2.x, r2.y};
          V2d sx = zero2, sy = zero2, sz = zero2, sdg = zero2;
#pragma unroll
          for (int k = 1; k <= NS; ++k) {
            const V2d up = *reinterpret_cast<const V2d*>(pl + p + k * kLdsWX);
            const V2d dn = *reinterpret_cast<const V2d*>(pl + p - k * kLdsWX);
            const V2d xr = {row[4 + k], row[5 + k]}, xl = {row[4 - k], row[5 - k]};
            sx += S.w[k] * (xr + xl);
            sy += S.w[k] * (up + dn);
            sz += S.w[k] * (win[u][NS + k] + win[u][NS - k]);
            if constexpr (DG) {   // the diagonal arm: (x + k, y + s k) and (x - k, y - s k)
              const int rs_k = S.sd * k * kLdsWX;
              const V2d f = {pl[p + k + rs_k], pl[p + 1 + k + rs_k]};
              const V2d bk = {pl[p - k - rs_k], pl[p + 1 - k - rs_k]};
              sdg += S.w[k] * (f + bk);
            }
          }
          V2d aq = S.diag * c + S.c[0] * sx + S.c[1] * sy + S.c[2] * sz;
          if constexpr (DG) aq += S.cd * sdg;
          V2d rt = cb[u] - (-aq);
          const int az = abs(z);
          rt.x = az <= cl.zr[u][off] ? rt.x : 0.0;
          rt.y = az <= cl.zr[u][off + 1] ? rt.y : 0.0;
          const V2d ro = rt * rs;
          *(EXX_GLOBAL V2r*)((EXX_GLOBAL char*)r + (unsigned)(EXX_QIDX(u, z) + off) * (unsigned)sizeof(TR)) =
              V2r{(TR)ro.x, (TR)ro.y};
          acc += rt.x * rt.x + rt.y * rt.y;
        }
#pragma unroll
        for (int k = 0; k < 2 * NS; ++k) win[u][k] = win[u][k + 1];
        win[u][2 * NS] = nx[u];
      }
    }
    __syncthreads();   // the next half's first plane reuses the buffer of this half's last one
  }
  return acc;
}

#undef EXX_QVALID
#undef EXX_QIDX

// Orthorhombic (axis stencil, column or quad layout) or general-cell (NK
// arms) form of the passes.
// (quad layout: CPT counts the columns of a thread's runs, 4 per run)
template <bool GEN, bool QD, int CPT>
using ColsOf = std::conditional_t<QD, ColsQ<(CPT + 3) / 4>, std::conditional_t<GEN, ColsG<CPT>, Cols<CPT>>>;

template <bool GEN, bool QD, int CPT, int NT>
__device__ __forceinline__ void cols_load(const ClassDev& C, const SolveKArgs& a, ColsOf<GEN, QD, CPT>& cl) {
  if constexpr (QD)
    load_cols_quad<NT, (CPT + 3) / 4>(C, a, cl);
  else if constexpr (GEN)
    load_cols_gen<CPT, NT>(C, a, cl);
  else
    load_cols<CPT, NT>(C, a, cl);
}

template <int NS, int CPT, int PD, bool GEN, bool TL, bool QD, typename T>
__device__ __forceinline__ void pass_a(const StencilT<T>& S, const GenStencilT<T>& G,
                                       const ColsOf<GEN, QD, CPT>& cl, const int* pst, int Zmax, const T* r, T* p,
                                       T beta, bool first, T* pl0, T* pl1, double& pq, double& rr) {
  beta = uniform(beta);
  if constexpr (QD) {
    double ra, aa;
    cg_pass_a_quad<NS, PD, GEN, false, T>(S, cl, pst, Zmax, r, p, beta, first, pl0, pl1, pq, rr, ra, aa);
  }
  else if constexpr (GEN && TL)
    cg_pass_a_tl<NS, CPT, T>(G, cl, pst, Zmax, r, p, beta, first, pl0, pl1, pq, rr);
  else if constexpr (GEN)
    cg_pass_a_gen<NS, CPT, PD, T>(G, cl, pst, Zmax, r, p, beta, first, pl0, pl1, pq, rr);
  else
    cg_pass_a<NS, CPT, PD, T>(S, cl, pst, Zmax, r, p, beta, first, pl0, pl1, pq, rr);
}

template <int NS, int CPT, int PD, bool GEN, bool TL, bool QD, typename T>
__device__ __forceinline__ double pass_b(const StencilT<T>& S, const GenStencilT<T>& G,
                                         const ColsOf<GEN, QD, CPT>& cl, const int* pst, int Zmax, T* x,
                                         const T* r_in, T* r, const T* p, T alpha, XStep<T> xs, T* pl0, T* pl1) {
  alpha = uniform(alpha);
  xs = uniform(xs);
  if constexpr (QD)
    return cg_pass_b_quad<NS, PD, GEN, T>(S, cl, pst, Zmax, x, r_in, r, p, alpha, xs, pl0, pl1);
  else if constexpr (GEN && TL)
    return cg_pass_b_tl<NS, CPT, T>(G, cl, pst, Zmax, x, r_in, r, p, alpha, xs, pl0, pl1);
  else if constexpr (GEN)
    return cg_pass_b_gen<NS, CPT, PD, T>(G, cl, pst, Zmax, x, r_in, r, p, alpha, xs, pl0, pl1);
  else
    return cg_pass_b<NS, CPT, PD, T>(S, cl, pst, Zmax, x, r_in, r, p, alpha, xs, pl0, pl1);
}

template <int NS, int CPT, bool GEN, bool TL, bool QD, typename TR>
__device__ __forceinline__ double true_residual(const SolveKArgs& a, const ColsOf<GEN, QD, CPT>& cl, const int* pst,
                                                int Zmax, const double* x, const double* b, TR* r, double rs,
                                                double* pl0, double* pl1) {
  if constexpr (QD)
    return cg_true_residual_quad<NS, GEN, TR>(a.S, cl, pst, Zmax, x, b, r, rs, pl0, pl1);
  else if constexpr (GEN && TL)
    return cg_true_residual_tl<NS, CPT, TR>(a.G, cl, pst, Zmax, x, b, r, rs, pl0, pl1);
  else if constexpr (GEN)
    return cg_true_residual_gen<NS, CPT, TR>(a.G, cl, pst, Zmax, x, b, r, rs, pl0, pl1);
  else
    return cg_true_residual<NS, CPT, TR>(a.S, cl, pst, Zmax, x, b, r, rs, pl0, pl1);
}

// block_sum of four values at once (two barriers for the four); red must hold
// 4 blockDim/64 doubles.
__device__ __forceinline__ void block_sum4(double (&v)[4], double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int i = 0; i < 4; ++i) v[i] = wave_sum(v[i]);
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) red[4 * wave + i] = v[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    double t = 0.0;
    for (int w = 0; w < nw; ++w) t += red[4 * w + i];
    v[i] = t;
  }
  __syncthreads();
}

// One workgroup solves one pair at a time, taking pairs from a device queue
// until the batch is exhausted (every workgroup exits when the counter passes
// the batch size).  Unpreconditioned CG from x = 0, stop at ||r|| <= tol ||b||.
template <int NS, int CPT, int NT, int PD, bool GEN, bool TL, bool QD>
__global__ __launch_bounds__(NT) void k_solve(SolveKArgs a) {
  extern __shared__ double lds[];
  __shared__ double red[NT / 64];
  __shared__ int s_item;
  const int tid = threadIdx.x;
  const int plane = kLdsWX * a.lds_wy;
  double* pl0 = lds;
  double* pl1 = lds + plane;
  int* pst = reinterpret_cast<int*>(lds + 2 * plane);
  double* r = (double*)((char*)a.slot_ws + (long long)blockIdx.x * a.slot_bytes);
  double* p = r + a.sstride;

  long long lo, hi;
  solve_range(a, &lo, &hi);
  for (;;) {
    if (tid == 0) s_item = atomicAdd(a.queue, 1);
    __syncthreads();
    const long long row = lo + s_item;   // row of the processing order
    __syncthreads();
    if (row >= hi) break;
    const long long item = row - a.p0;   // row of the batch workspace
    const int pid = a.order[row];
    const ClassDev& C = a.cls[a.pairs[pid].cls];
    const int Zmax = C.Zmax;
    const long long npe = C.n_pe;
    double* x = a.bx_ws + item * a.rstride;

    for (int k = tid; k < 2 * plane; k += NT) lds[k] = 0.0;
    for (int k = tid; k < 2 * Zmax + 2; k += NT) pst[k] = C.plane_start[k];
    ColsOf<GEN, QD, CPT> cl;
    cols_load<GEN, QD, CPT, NT>(C, a, cl);
    __syncthreads();

    int it = 0, code = kCgConverged;
    double rr = 0.0, bnorm = 0.0, beta = 0.0;
    bool first = true;
    // Warm start: with x0 gathered into p, a first half-iteration runs pass B
    // alone with alpha = 1, x = 0 and r_in = b, which leaves r = b - A x0 in
    // the slot and x = x0 in place of b.  The CG proper then starts from that
    // residual.  (One pass-B call site serves both, to keep the kernel's
    // register allocation that of the cold solve.)
    bool init = false;
    if (a.warm_store && a.warm_map[pid] >= 0) {
      double bb = 0.0;
      for (long long k = tid; k < npe; k += NT) bb += x[k] * x[k];
      bnorm = sqrt(block_sum(bb, red));
      init = warm_gather<double>(a, C, pid, p);
      __syncthreads();
    }
    const bool from_b = !init;   // cold: the first pass reads b from x, and x starts at zero
    bool conv = false;
    // a pass B that left x alone (its step alpha_k p_k deferred, see XStep)
    bool pend = false;
    double a_pend = 0.0, b_pend = 1.0;
    int nsav = 0;
    while (it < a.max_iter) {
      double alpha = 1.0;
      if (!init) {
        double pq_t, rr_t;
        pass_a<NS, CPT, PD, GEN, TL, QD, double>(a.S, a.G, cl, pst, Zmax, (first && from_b) ? x : r, p, beta, first,
                                             pl0, pl1, pq_t, rr_t);
        const double pq = block_sum(pq_t, red);
        if (first && from_b) {
          rr = block_sum(rr_t, red);
          bnorm = sqrt(rr);
          if (bnorm == 0.0) {   // b == 0: x = b = 0 already
            conv = true;
            break;
          }
          if (!(bnorm < INFINITY)) {   // b holds a NaN or an infinity
            code = kCgNonFinite;
            break;
          }
        }
        // breakdown: A is SPD, so in FP64 only non-finite input gets here;
        // the solution is left as it stands (b is no longer held)
        if (!(pq > 0.0) || !(pq < INFINITY)) {
          code = kCgBreakdown;
          break;
        }
        alpha = rr / pq;
      }
      const bool from_b_now = init || (first && from_b);
      XStep<double> xs{alpha, 0.0, from_b_now, false};
      if (pend) {   // this pass also takes the deferred step
        xs.ap = alpha + a_pend / b_pend;
        xs.ar = -a_pend / b_pend;
        pend = false;
      } else if (!from_b_now) {   // x holds the solution: defer this step to the next pass B
        xs.skip = true;
        pend = true;
        a_pend = alpha;
        ++nsav;
      }
      const double rn = block_sum(pass_b<NS, CPT, PD, GEN, TL, QD, double>(a.S, a.G, cl, pst, Zmax, x,
                                                                       from_b_now ? x : r, r, p, alpha, xs, pl0, pl1),
                                  red);
      if (init) {   // the warm start's residual
        init = false;
        rr = rn;
        if (!(bnorm > 0.0) || sqrt(rn) <= a.tol * bnorm) {
          conv = true;
          break;
        }
        continue;
      }
      ++it;
      first = false;
      if (sqrt(rn) <= a.tol * bnorm) {
        rr = rn;
        conv = true;
        break;
      }
      if (!(rn == rn)) {
        rr = NAN;
        code = kCgNonFinite;
        break;
      }
      beta = rn / rr;
      rr = rn;
      b_pend = beta;
    }
    if (pend) {   // the last pass B deferred its step; p still holds its p
      for (long long k = tid; k < npe; k += NT) x[k] += a_pend * p[k];
      __syncthreads();
    }
    if (!conv && code == kCgConverged) code = kCgCap;
    warm_store_solution(a, npe, pid, x);
    if (tid == 0) {
      a.outIt[pid] = it;
      a.outRes[pid] = bnorm > 0.0 ? sqrt(rr) / bnorm : 0.0;
      a.outUpd[pid] = 0;
      a.outSav[pid] = nsav;
      a.outExit[pid] = code;
    }
    __syncthreads();
  }
}

// Mixed precision: FP32 CG (stencil, vectors and updates in FP32, dot products
// and norms in FP64) with reliable updates in FP64 (residual replacement:
// van der Vorst and Ye 2000; Clark et al. 2010).  The solution accumulates in
// FP64 and the stop test is on the FP64 true residual, ||b - A x|| <= tol ||b||,
// the same criterion as the FP64 path.
template <int NS, int CPT, int NT, int PD, bool GEN, bool TL, bool QD>
__global__ __launch_bounds__(NT) void k_solve_mixed(SolveKArgs a) {
  extern __shared__ double lds[];
  __shared__ double red[NT / 64];
  // Tilted arms: the fused sweep with Ap kept in q (cg_pass_fused_tl),
  // except with four columns per thread in 1024 threads, where its windows
  // spill the plane loop's registers.
  constexpr bool FUSE_TL = GEN && TL && !QD && (NT < 1024 || CPT <= 3);
  __shared__ double red4[(QD || FUSE_TL) ? 4 * (NT / 64) : 1];
  __shared__ int s_item;
  const int tid = threadIdx.x;
  const int plane = kLdsWX * a.lds_wy;
  double* pl0 = lds;
  double* pl1 = lds + plane;
  float* fl0 = reinterpret_cast<float*>(lds);   // four FP32 planes in the space of two FP64 ones
  float* fl1 = fl0 + plane;
  float* fl2 = fl1 + plane;
  float* fl3 = fl2 + plane;
  int* pst = reinterpret_cast<int*>(lds + 2 * plane);
  // slot: x (FP64), then r, p, y, q (FP32; q holds Ap between fused sweeps)
  double* x = (double*)((char*)a.slot_ws + (long long)blockIdx.x * a.slot_bytes);
  float* r = reinterpret_cast<float*>(x + a.sstride);
  float* p = r + a.sstride;
  float* y = p + a.sstride;
  float* q = y + a.sstride;
  const StencilT<float> S32 = stencil_cast<float>(a.S);
  // Quad layout: pass B and the next pass A share a sweep (cg_pass_fused_quad)
  // in workgroups of up to 768 threads (one run per thread with 768, two with
  // 512).  Its two z windows need the registers of at most three waves per
  // SIMD; with four (1024 threads) the sweep spills to scratch memory and runs
  // slower than the two passes.
  constexpr bool FUSE = QD && NT <= 768;

  long long lo, hi;
  solve_range(a, &lo, &hi);
  for (;;) {
    if (tid == 0) s_item = atomicAdd(a.queue, 1);
    __syncthreads();
    const long long row = lo + s_item;   // row of the processing order
    __syncthreads();
    if (row >= hi) break;
    const long long item = row - a.p0;   // row of the batch workspace
    const int pid = a.order[row];
    const ClassDev& C = a.cls[a.pairs[pid].cls];
    const int Zmax = C.Zmax;
    const long long npe = C.n_pe;
    double* bx = a.bx_ws + item * a.rstride;

    for (int k = tid; k < 2 * plane; k += NT) lds[k] = 0.0;
    for (int k = tid; k < 2 * Zmax + 2; k += NT) pst[k] = C.plane_start[k];
    ColsOf<GEN, QD, CPT> cl;
    cols_load<GEN, QD, CPT, NT>(C, a, cl);
    // ||b|| in FP64; the FP32 recursion runs in units of ||b|| (r = b / ||b||),
    // so its values stay far from the FP32 range limits whatever the pair's
    // overlap, and the solution is x = ||b|| sum y
    double bb = 0.0;
    for (long long k = tid; k < npe; k += NT) {
      const double bv = bx[k];
      bb += bv * bv;
    }
    bb = block_sum(bb, red);   // also orders the plane zeroing before the first pass
    const double bnorm = sqrt(bb);
    const double inv_b = bnorm > 0.0 ? 1.0 / bnorm : 0.0;
    for (long long k = tid; k < npe; k += NT) r[k] = (float)(bx[k] * inv_b);
    __syncthreads();

    int it = 0, upd = 0, nsav = 0, rst = 0, code = kCgConverged;
    double rr = 1.0, rr_true = bb, rmax = 1.0, beta = 0.0;
    bool first = true, x_zero = true, y_zero = true;
    bool conv = bnorm == 0.0;
    if (!conv && !(bnorm < INFINITY)) code = kCgNonFinite;   // b holds a NaN or an infinity
    // warm start: x = x0 (FP64) and the working residual (b - A x0) / ||b||
    if (!conv && code == kCgConverged && warm_gather<double>(a, C, pid, x)) {
      for (int k = tid; k < 2 * plane; k += NT) lds[k] = 0.0;
      __syncthreads();
      rr_true = block_sum(true_residual<NS, CPT, GEN, TL, QD, float>(a, cl, pst, Zmax, x, bx, r, inv_b, pl0, pl1), red);
      for (int k = tid; k < 2 * plane; k += NT) lds[k] = 0.0;
      __syncthreads();
      x_zero = false;
      rr = rr_true * inv_b * inv_b;
      rmax = sqrt(rr);
      conv = sqrt(rr_true) <= a.tol * bnorm;
    }
    // quad layout: p of the iteration and its products already formed by a
    // fused sweep (cg_pass_fused_quad)
    bool have_p = false;
    double pq = 0.0, ra = 0.0, aa = 0.0;
    // the correction y is updated by every other pass B (see XStep): pend
    // marks a pass that deferred its step a_pend p; b_pend is the FP32 beta
    // that formed the next p from it
    bool pend = false;
    double a_pend = 0.0, b_pend = 1.0;
    while (!conv && code == kCgConverged && it < a.max_iter) {
      // bad: the FP32 recursion broke down (p.Ap not positive and finite) or
      // produced a non-finite norm; the CG then restarts from the last FP64
      // solution (its FP32 correction y is dropped), up to kCgMaxRestarts times
      int bad = kCgConverged;
      double rn = 0.0;
      if (!have_p) {
        if constexpr (QD) {
          double t[4], rr_t;
          cg_pass_a_quad<NS, PD, GEN, FUSE, float>(S32, cl, pst, Zmax, r, p, uniform((float)beta), first, fl0, fl1,
                                                   t[0], rr_t, t[1], t[2]);
          t[3] = 0.0;
          block_sum4(t, red4);
          pq = t[0];
          ra = t[1];
          aa = t[2];
        } else if constexpr (FUSE_TL) {
          double t[4], rr_t;
          cg_pass_a_tl<NS, CPT, float, true>(a.G32, cl, pst, Zmax, r, p, uniform((float)beta), first, fl0, fl1, t[0],
                                             rr_t, q, &t[1], &t[2]);
          t[3] = 0.0;
          block_sum4(t, red4);
          pq = t[0];
          ra = t[1];
          aa = t[2];
        } else {
          double pq_t, rr_t;
          pass_a<NS, CPT, PD, GEN, TL, QD, float>(S32, a.G32, cl, pst, Zmax, r, p, (float)beta, first, fl0, fl1, pq_t,
                                                  rr_t);
          pq = block_sum(pq_t, red);
        }
      }
      if (!(pq > 0.0) || !(pq < INFINITY)) bad = kCgBreakdown;
      if (bad == kCgConverged) {
        const double alpha = rr / pq;
        XStep<float> xs{(float)alpha, 0.0f, y_zero, false};
        if (pend) {   // this pass also takes the deferred step
          xs.ap = (float)(alpha + a_pend / b_pend);
          xs.ar = (float)(-a_pend / b_pend);
        } else {
          xs.skip = true;
        }
        bool fused = false;
        if constexpr (FUSE || FUSE_TL) {
          // |r - alpha Ap|^2 before r is updated; the sweep is fused only where
          // this next norm stays clear of the reliable-update and stop thresholds
          // (2% margin), so that every update and stop test follows a pass B
          const double rn_next = rr - 2.0 * alpha * ra + alpha * alpha * aa;
          const double thr = 1.02 * fmax(a.delta * rmax, a.tol);
          if (rn_next > thr * thr && it + 1 < a.max_iter) {
            double o3[3], t[4];
            const float bnext = (float)(rn_next / rr);
            if constexpr (FUSE)
              t[0] = cg_pass_fused_quad<NS, PD, GEN, float>(S32, cl, pst, Zmax, y, r, p, uniform((float)alpha),
                                                            uniform(bnext), uniform(xs), fl0, fl1, fl2, fl3, o3);
            else
              t[0] = cg_pass_fused_tl<NS, CPT, float>(a.G32, cl, pst, Zmax, y, r, p, q, uniform((float)alpha),
                                                      uniform(bnext), uniform(xs), fl0, fl1, o3);
            t[1] = o3[0];
            t[2] = o3[1];
            t[3] = o3[2];
            block_sum4(t, red4);
            ++it;
            // (the tilted-arm sweep reads and writes q in place of a second
            // pass over p: it saves no accesses beyond a deferred x step)
            nsav += FUSE ? (xs.skip ? 2 : 1) : (xs.skip ? 1 : 0);
            first = false;
            if (!xs.skip) y_zero = false;
            pend = xs.skip;
            a_pend = alpha;
            b_pend = (double)bnext;
            fused = true;
            if (!(t[0] == t[0]) || !(t[0] < INFINITY)) {
              bad = kCgNonFinite;
            } else {
              rr = t[0];
              pq = t[1];
              ra = t[2];
              aa = t[3];
              have_p = true;
              continue;
            }
          }
          have_p = false;
        }
        if (!fused) {
          rn = block_sum(pass_b<NS, CPT, PD, GEN, TL, QD, float>(S32, a.G32, cl, pst, Zmax, y, r, r, p, (float)alpha,
                                                                 xs, fl0, fl1),
                         red);
          ++it;
          nsav += xs.skip ? 1 : 0;
          first = false;
          if (!xs.skip) y_zero = false;
          pend = xs.skip;
          a_pend = alpha;
          if (!(rn == rn) || !(rn < INFINITY)) bad = kCgNonFinite;
        }
      }
      const double rnorm = sqrt(rn);
      const bool restart = bad != kCgConverged;
      if (restart && rst >= kCgMaxRestarts) {
        code = bad;
        break;
      }
      if (restart || rnorm < a.delta * rmax || rnorm <= a.tol || it >= a.max_iter) {
        // A reliable update folds the FP32 correction into the FP64 solution,
        // x = x + ||b|| y (a flat pass over the points); a restart drops it.
        // Then the FP64 true residual replaces the working one (or, with no
        // FP64 solution yet, b / ||b|| does).  The FP64 and FP32 plane views
        // share LDS, so it is cleared around the FP64 pass (the barrier also
        // orders the fold before the sweep).
        if (!restart) {
          // (with a deferred step, p still holds that pass's p: a reliable
          // update always follows a plain pass B, which leaves p alone)
          const double ap = pend ? a_pend : 0.0;
          for (long long k = tid; k < npe; k += NT)
            x[k] = (x_zero ? 0.0 : x[k]) + bnorm * ((y_zero ? 0.0 : (double)y[k]) + ap * (double)p[k]);
          x_zero = false;
          ++upd;
        } else {
          ++rst;
          have_p = false;
        }
        pend = false;
        if (x_zero) {
          for (long long k = tid; k < npe; k += NT) r[k] = (float)(bx[k] * inv_b);
          __syncthreads();
          rr_true = bb;
        } else {
          for (int k = tid; k < 2 * plane; k += NT) lds[k] = 0.0;
          __syncthreads();
          rr_true =
              block_sum(true_residual<NS, CPT, GEN, TL, QD, float>(a, cl, pst, Zmax, x, bx, r, inv_b, pl0, pl1), red);
          for (int k = tid; k < 2 * plane; k += NT) lds[k] = 0.0;
          __syncthreads();
        }
        y_zero = true;
        rn = rr_true * inv_b * inv_b;
        rmax = sqrt(rn);
        if (sqrt(rr_true) <= a.tol * bnorm) conv = true;
        if (!(rn < INFINITY)) code = kCgNonFinite;   // the FP64 solution itself is not finite
        if (restart) first = true;   // steepest descent from the refreshed residual
      }
      beta = rn / rr;
      rr = rn;
      if (pend) b_pend = (double)(float)beta;   // the FP32 beta of the next pass A
    }
    if (!conv && code == kCgConverged) code = kCgCap;
    // the FP64 solution replaces the right-hand side
    if (!x_zero) {
      for (long long k = tid; k < npe; k += NT) bx[k] = x[k];
    } else if (bnorm > 0.0) {
      for (long long k = tid; k < npe; k += NT) bx[k] = 0.0;
    }
    __syncthreads();
    warm_store_solution(a, npe, pid, bx);
    if (tid == 0) {
      a.outIt[pid] = it;
      a.outRes[pid] = bnorm > 0.0 ? sqrt(rr_true) / bnorm : 0.0;
      a.outUpd[pid] = upd;
      a.outSav[pid] = nsav;
      a.outExit[pid] = code | (rst << 8);
    }
    __syncthreads();
  }
}

// Launch (or occupancy query, when occ is not NULL) of one instance.
template <int NS, int CPT, int NT, int PD, bool GEN, bool TL, bool QD = false>
hipError_t solve_instance_g(const SolveKArgs& a, bool mixed, int groups, size_t lds, hipStream_t s, int* occ) {
  const void* fn = mixed ? (const void*)k_solve_mixed<NS, CPT, NT, PD, GEN, TL, QD>
                         : (const void*)k_solve<NS, CPT, NT, PD, GEN, TL, QD>;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  if (occ) {
    return mixed
               ? hipOccupancyMaxActiveBlocksPerMultiprocessor(occ, k_solve_mixed<NS, CPT, NT, PD, GEN, TL, QD>, NT, lds)
               : hipOccupancyMaxActiveBlocksPerMultiprocessor(occ, k_solve<NS, CPT, NT, PD, GEN, TL, QD>, NT, lds);
  }
  if (mixed)
    k_solve_mixed<NS, CPT, NT, PD, GEN, TL, QD><<<groups, NT, lds, s>>>(a);
  else
    k_solve<NS, CPT, NT, PD, GEN, TL, QD><<<groups, NT, lds, s>>>(a);
  return hipGetLastError();
}

// Orthorhombic cells and general cells whose arms stay in the sweep plane
// take every load depth; with arms leaving the plane the passes load one
// plane ahead whatever the depth asked.
template <int NS, int CPT, int NT, int PD>
hipError_t solve_instance(const SolveKArgs& a, bool mixed, int groups, size_t lds, hipStream_t s, int* occ) {
  if (!a.gen) return solve_instance_g<NS, CPT, NT, PD, false, false>(a, mixed, groups, lds, s, occ);
  if (a.G.n_tl > 0) return solve_instance_g<NS, CPT, NT, 1, true, true>(a, mixed, groups, lds, s, occ);
  return solve_instance_g<NS, CPT, NT, PD, true, false>(a, mixed, groups, lds, s, occ);
}

// Columns per thread available for each workgroup size: 1024 threads take up
// to 4 columns each, 512 threads up to 8.
template <int NS, int NT, int PD>
hipError_t solve_cpt(const SolveKArgs& a, bool mixed, int cpt, int groups, size_t lds, hipStream_t s, int* occ) {
  if constexpr (NT == 1024) {
    switch (cpt) {
      case 1: return solve_instance<NS, 1, NT, PD>(a, mixed, groups, lds, s, occ);
      case 2: return solve_instance<NS, 2, NT, PD>(a, mixed, groups, lds, s, occ);
      case 3: return solve_instance<NS, 3, NT, PD>(a, mixed, groups, lds, s, occ);
      case 4: return solve_instance<NS, 4, NT, PD>(a, mixed, groups, lds, s, occ);
      default: return hipErrorInvalidValue;
    }
  } else {
  switch (cpt) {
    case 1:
    case 2: return solve_instance<NS, 2, NT, PD>(a, mixed, groups, lds, s, occ);
    case 3:
    case 4: return solve_instance<NS, 4, NT, PD>(a, mixed, groups, lds, s, occ);
    case 5:
    case 6: return solve_instance<NS, 6, NT, PD>(a, mixed, groups, lds, s, occ);
    case 7:
    case 8: return solve_instance<NS, 8, NT, PD>(a, mixed, groups, lds, s, occ);
    default: return hipErrorInvalidValue;
  }
  }
}

template <int NS>
hipError_t solve_ns_dispatch(const SolveKArgs& a, bool mixed, int max_cols, int threads, int depth, int groups,
                             size_t lds, hipStream_t s, int* occ) {
  if (a.quads) {   // runs of four columns: one per thread with 768 or 1024 threads, two with 512 (GEN: with a
                   // diagonal arm)
    if ((threads != 512 && threads != 768 && threads != 1024) || max_cols > 4 * (threads == 512 ? 2 : 1) * threads)
      return hipErrorInvalidValue;
    if (threads == 512) {
      if (a.gen) {
        if (depth <= 1) return solve_instance_g<NS, 8, 512, 1, true, false, true>(a, mixed, groups, lds, s, occ);
        return solve_instance_g<NS, 8, 512, 2, true, false, true>(a, mixed, groups, lds, s, occ);
      }
      if (depth <= 1) return solve_instance_g<NS, 8, 512, 1, false, false, true>(a, mixed, groups, lds, s, occ);
      return solve_instance_g<NS, 8, 512, 2, false, false, true>(a, mixed, groups, lds, s, occ);
    }
    if (threads == 768) {
      if (a.gen) {
        if (depth <= 1) return solve_instance_g<NS, 4, 768, 1, true, false, true>(a, mixed, groups, lds, s, occ);
        return solve_instance_g<NS, 4, 768, 2, true, false, true>(a, mixed, groups, lds, s, occ);
      }
      if (depth <= 1) return solve_instance_g<NS, 4, 768, 1, false, false, true>(a, mixed, groups, lds, s, occ);
      return solve_instance_g<NS, 4, 768, 2, false, false, true>(a, mixed, groups, lds, s, occ);
    }
    if (a.gen) {
      if (depth <= 1) return solve_instance_g<NS, 4, 1024, 1, true, false, true>(a, mixed, groups, lds, s, occ);
      return solve_instance_g<NS, 4, 1024, 2, true, false, true>(a, mixed, groups, lds, s, occ);
    }
    if (depth <= 1) return solve_instance_g<NS, 4, 1024, 1, false, false, true>(a, mixed, groups, lds, s, occ);
    return solve_instance_g<NS, 4, 1024, 2, false, false, true>(a, mixed, groups, lds, s, occ);
  }
  const int cpt = (max_cols + threads - 1) / threads;
  if (threads == 1024) {
    if (depth <= 1) return solve_cpt<NS, 1024, 1>(a, mixed, cpt, groups, lds, s, occ);
    return solve_cpt<NS, 1024, 2>(a, mixed, cpt, groups, lds, s, occ);
  }
  if (threads == 512) {
    if (depth <= 1) return solve_cpt<NS, 512, 1>(a, mixed, cpt, groups, lds, s, occ);
    return solve_cpt<NS, 512, 2>(a, mixed, cpt, groups, lds, s, occ);
  }
  return hipErrorInvalidValue;
}

}  // namespace exx
