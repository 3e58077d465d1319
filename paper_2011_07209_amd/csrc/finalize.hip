// E_xx and sigma_xx of each pair as one plane sweep over its PE sphere
// (orthorhombic cells, column or quad layout of the CG vectors):
//   E = -w dV sum rho v                                   (eq. exxGen_mlwf)
//   sigma^{a al} = -2 w dV sum_b (h^-1)_{al b} sum rbar_b rho dv/dr_a
//                                                          (eq. sxx_working)
// with dv/dr_a from the first-derivative stencil of eq. d1_1 along each axis
// (the Jacobian of eq. jacb is the identity for an orthorhombic cell).
//
// One workgroup per pair.  Thread t owns the sphere's columns t, t + 1024,
// ... and marches z with the column's potential in a register window of
// 2n+1 planes; a column's points beyond its PE extent take the far-field
// (Dirichlet) values there.  Each plane is staged in LDS together with the
// plane's Dirichlet points, so the x and y neighbours of every PE point come
// from one LDS plane: the PE points and the Dirichlet points of a plane are
// disjoint, so one barrier per plane orders both.  Every value is read from
// HBM once (the potential, the density and the far-field values).
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "exx_launch.h"

namespace exx {

namespace {

constexpr int kFinThreads = 1024;

template <int NS, int CPT>
__global__ __launch_bounds__(kFinThreads) void k_finalize_sweep(Geo g, const ClassDev* __restrict__ cls,
                                                                const PairDev* __restrict__ pairs,
                                                                const int* __restrict__ order, long long p0,
                                                                const int* __restrict__ n_eff,
                                                                const double* __restrict__ rho_ws,
                                                                const double* __restrict__ v_ws, long long rstride,
                                                                const double* __restrict__ halo_ws, long long hstride,
                                                                double* __restrict__ outE, double* __restrict__ outS) {
  extern __shared__ double lds[];
  __shared__ double red[kFinThreads / 64];
  const int bq = blockIdx.x;
  if (p0 + bq >= *n_eff) return;
  const int pid = order[p0 + bq];
  const PairDev P = pairs[pid];
  const ClassDev& C = cls[P.cls];
  const int plane = kLdsWX * g.lds_wy;
  double* pl0 = lds;
  double* pl1 = lds + plane;
  const double* rho = rho_ws + (long long)bq * rstride;
  const double* x = v_ws + (long long)bq * rstride;
  const double* halo = halo_ws + (long long)bq * hstride;
  const int Zmax = C.Zmax, Zh = C.Zh;
  const int W01 = C.Wm[0] * C.Wm[1];

  // this thread's columns (the sphere's columns without the quad layout's
  // padding): slot in the layout, PE half-height zr (-1: none) and the x and
  // y offsets packed in one register (16 bits each); the LDS position and the
  // far-field map index follow from them where needed
  int slot[CPT], zr[CPT], oxy[CPT];
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    const int col = threadIdx.x + c * kFinThreads;
    slot[c] = 0;
    zr[c] = -1;
    oxy[c] = 0;
    if (col < C.n_fin) {
      const int4 cc = C.fin_cols[col];
      slot[c] = cc.x;
      zr[c] = cc.y;
      oxy[c] = (cc.z & 0xffff) | (cc.w << 16);
    }
  }
  auto ox_of = [&](int c) { return (int)(short)(oxy[c] & 0xffff); };
  auto oy_of = [&](int c) { return oxy[c] >> 16; };
  auto pos_of = [&](int c) { return (ox_of(c) + g.lds_cx) + kLdsWX * (oy_of(c) + g.lds_cy); };
  // the potential at (column c, plane zz): the solution inside PE, the
  // far-field value at the n points beyond each end of the column
  auto value = [&](int c, int zz) -> double {
    const int az = abs(zz);
    if (az <= zr[c]) return x[C.plane_start[zz + Zmax] + slot[c]];
    if (zr[c] >= 0 && az <= zr[c] + NS) {
      const int m = (ox_of(c) + C.Rg[0] + g.n) + C.Wm[0] * (oy_of(c) + C.Rg[1] + g.n) + W01 * (zz + C.Rg[2] + g.n);
      const int h = C.halo_map[m];
      return h >= 0 ? halo[h] : 0.0;
    }
    return 0.0;
  };

  double win[CPT][2 * NS + 1];
#pragma unroll
  for (int k = 0; k < 2 * NS + 1; ++k)
#pragma unroll
    for (int c = 0; c < CPT; ++c) win[c][k] = value(c, -Zmax - NS + k);
  double e = 0.0, T[9];
#pragma unroll
  for (int t = 0; t < 9; ++t) T[t] = 0.0;
  double w1[NS + 1];
#pragma unroll
  for (int q = 0; q <= NS; ++q) w1[q] = g.w1[q];

  for (int z = -Zmax; z <= Zmax; ++z) {
    // loads for the plane entering the window, and this plane's density
    double nv[CPT], rh[CPT];
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      nv[c] = value(c, z + NS + 1);
      rh[c] = abs(z) <= zr[c] ? rho[C.plane_start[z + Zmax] + slot[c]] : 0.0;
    }
    double* pl = (z & 1) ? pl1 : pl0;
#pragma unroll
    for (int c = 0; c < CPT; ++c)
      if (abs(z) <= zr[c]) pl[pos_of(c)] = win[c][NS];
    for (int k = C.halo_zstart[z + Zh] + (int)threadIdx.x; k < C.halo_zstart[z + Zh + 1]; k += kFinThreads) {
      const int h = C.halo_zidx[k];
      const short4 o = C.halo_off[h];
      pl[(o.x + g.lds_cx) + kLdsWX * (o.y + g.lds_cy)] = halo[h];
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      if (abs(z) <= zr[c]) {
        const int pos = pos_of(c);
        const double v = win[c][NS];
        double d0 = 0.0, d1 = 0.0, d2 = 0.0;
#pragma unroll
        for (int q = 1; q <= NS; ++q) {
          d0 += w1[q] * (pl[pos + q] - pl[pos - q]);
          d1 += w1[q] * (pl[pos + q * kLdsWX] - pl[pos - q * kLdsWX]);
          d2 += w1[q] * (win[c][NS + q] - win[c][NS - q]);
        }
        const double ga[3] = {d0 * g.inv_d[0], d1 * g.inv_d[1], d2 * g.inv_d[2]};
        const double rb[3] = {ox_of(c) * g.d[0], oy_of(c) * g.d[1], z * g.d[2]};
        e += rh[c] * v;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int b = 0; b < 3; ++b) T[a + 3 * b] += rb[b] * rh[c] * ga[a];
      }
#pragma unroll
      for (int k = 0; k < 2 * NS; ++k) win[c][k] = win[c][k + 1];
      win[c][2 * NS] = nv[c];
    }
  }
  e = block_sum(e, red);
#pragma unroll
  for (int t = 0; t < 9; ++t) T[t] = block_sum(T[t], red);
  if (threadIdx.x == 0) {
    const double w = (P.i == P.j) ? 1.0 : 2.0;
    outE[pid] = -w * g.dV * e;
    for (int a = 0; a < 3; ++a)
      for (int al = 0; al < 3; ++al) {
        double s = 0.0;
        for (int b = 0; b < 3; ++b) s += g.hinv[al + 3 * b] * T[a + 3 * b];
        outS[9 * (long long)pid + a + 3 * al] = -2.0 * w * g.dV * s;
      }
  }
}

template <int NS>
hipError_t finalize_sweep_cpt(int cpt, const Geo& g, const Batch& B, const double* rho_ws, const double* v_ws,
                              long long rstride, const double* halo_ws, long long hstride, double* outE, double* outS,
                              size_t lds, hipStream_t s) {
  const void* fn = nullptr;
  switch (cpt) {
    case 1: fn = (const void*)k_finalize_sweep<NS, 1>; break;
    case 2: fn = (const void*)k_finalize_sweep<NS, 2>; break;
    case 3: fn = (const void*)k_finalize_sweep<NS, 3>; break;
    case 4: fn = (const void*)k_finalize_sweep<NS, 4>; break;
    default: return hipErrorInvalidValue;
  }
  if (lds > 64 * 1024) {
    const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  const dim3 grid((unsigned)B.nb);
#define EXX_FIN_ARGS g, B.cls, B.pairs, B.order, B.p0, B.n_eff, rho_ws, v_ws, rstride, halo_ws, hstride, outE, outS
  switch (cpt) {
    case 1: k_finalize_sweep<NS, 1><<<grid, kFinThreads, lds, s>>>(EXX_FIN_ARGS); break;
    case 2: k_finalize_sweep<NS, 2><<<grid, kFinThreads, lds, s>>>(EXX_FIN_ARGS); break;
    case 3: k_finalize_sweep<NS, 3><<<grid, kFinThreads, lds, s>>>(EXX_FIN_ARGS); break;
    default: k_finalize_sweep<NS, 4><<<grid, kFinThreads, lds, s>>>(EXX_FIN_ARGS); break;
  }
#undef EXX_FIN_ARGS
  return hipGetLastError();
}

}  // namespace

bool finalize_sweep_supported(const Geo& g, long long max_cols) {
  return !g.gen && max_cols > 0 && max_cols <= 4LL * kFinThreads && (size_t)2 * kLdsWX * g.lds_wy * sizeof(double) <= 160 * 1024;
}

hipError_t launch_finalize_sweep(const Geo& g, const Batch& B, long long max_cols, const double* rho_ws,
                                 const double* v_ws, long long rstride, const double* halo_ws, long long hstride,
                                 double* outE, double* outS, hipStream_t s) {
  if (B.nb <= 0) return hipSuccess;
  if (!finalize_sweep_supported(g, max_cols)) return hipErrorInvalidValue;
  const int cpt = (int)((max_cols + kFinThreads - 1) / kFinThreads);
  const size_t lds = (size_t)2 * kLdsWX * g.lds_wy * sizeof(double);
  switch (g.n) {
    case 1: return finalize_sweep_cpt<1>(cpt, g, B, rho_ws, v_ws, rstride, halo_ws, hstride, outE, outS, lds, s);
    case 2: return finalize_sweep_cpt<2>(cpt, g, B, rho_ws, v_ws, rstride, halo_ws, hstride, outE, outS, lds, s);
    case 3: return finalize_sweep_cpt<3>(cpt, g, B, rho_ws, v_ws, rstride, halo_ws, hstride, outE, outS, lds, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace exx
