// E_xx and sigma_xx of each pair as one plane sweep over its PE sphere
// (column or quad layout of the CG vectors):
//   E = -w dV sum rho v                                   (eq. exxGen_mlwf)
//   sigma^{a al} = -2 w dV sum_b (h^-1)_{al b} sum rbar_b rho dv/dr_a
//                                                          (eq. sxx_working)
// with dv/dr_a = sum_al J_{a al} dv/dxi_al (eq. jacb) and dv/dxi_al from the
// first-derivative stencil of eq. d1_1 along lattice axis al (J is the
// identity for an orthorhombic cell).  General cells sweep in their CG frame
// (x', y', z') = (o[perm[0]], o[perm[1]], o[perm[2]]): lattice axes too, so
// every derivative still reads the staged plane or the column's window.
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

template <int NS, int CPT, bool GEN>
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
  // padding): slot in the layout, PE extent [lo, hi] along z (lo > hi: none)
  // and the x and y offsets packed in one register (16 bits each); the LDS
  // position and the far-field map index follow from them where needed.
  // Orthorhombic columns are (slot, half-height, x, y), general ones (slot,
  // lo, hi, x | y << 16), x, y, z in the CG frame.
  int slot[CPT], lo[CPT], hi[CPT], oxy[CPT];
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    const int col = threadIdx.x + c * kFinThreads;
    slot[c] = 0;
    lo[c] = 1;    // no column: empty for both forms (lo > hi, hi < 0)
    hi[c] = -1;
    oxy[c] = 0;
    if (col < C.n_fin) {
      const int4 cc = C.fin_cols[col];
      slot[c] = cc.x;
      if constexpr (GEN) {
        lo[c] = cc.y;
        hi[c] = cc.z;
        oxy[c] = cc.w;
      } else {   // (lo = -hi: only hi is read)
        hi[c] = cc.y;
        oxy[c] = (cc.z & 0xffff) | (cc.w << 16);
      }
    }
  }
  auto ox_of = [&](int c) { return (int)(short)(oxy[c] & 0xffff); };
  auto oy_of = [&](int c) { return oxy[c] >> 16; };
  auto pos_of = [&](int c) { return (ox_of(c) + g.lds_cx) + kLdsWX * (oy_of(c) + g.lds_cy); };
  auto inside = [&](int c, int zz) {
    if constexpr (GEN)
      return zz >= lo[c] && zz <= hi[c];
    else
      return abs(zz) <= hi[c];
  };
  // the far-field map index of CG-frame point (x, y, z): the maps are over the
  // lattice offsets, centred at (Wm - 1) / 2 = Rg + n
  auto map_index = [&](int px, int py, int pz) {
    if constexpr (GEN) {
      int o[3];
      o[g.perm[0]] = px;
      o[g.perm[1]] = py;
      o[g.perm[2]] = pz;
      return (o[0] + (C.Wm[0] - 1) / 2) + C.Wm[0] * (o[1] + (C.Wm[1] - 1) / 2) + W01 * (o[2] + (C.Wm[2] - 1) / 2);
    } else {
      return (px + C.Rg[0] + g.n) + C.Wm[0] * (py + C.Rg[1] + g.n) + W01 * (pz + C.Rg[2] + g.n);
    }
  };
  // the potential at (column c, plane zz): the solution inside PE, the
  // far-field value at the n points beyond each end of the column
  auto value = [&](int c, int zz) -> double {
    if (inside(c, zz)) return x[C.plane_start[zz + Zmax] + slot[c]];
    const bool reach = GEN ? lo[c] <= hi[c] && zz >= lo[c] - NS && zz <= hi[c] + NS
                           : hi[c] >= 0 && abs(zz) <= hi[c] + NS;
    if (reach) {
      const int h = C.halo_map[map_index(ox_of(c), oy_of(c), zz)];
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
      rh[c] = inside(c, z) ? rho[C.plane_start[z + Zmax] + slot[c]] : 0.0;
    }
    double* pl = (z & 1) ? pl1 : pl0;
#pragma unroll
    for (int c = 0; c < CPT; ++c)
      if (inside(c, z)) pl[pos_of(c)] = win[c][NS];
    for (int k = C.halo_zstart[z + Zh] + (int)threadIdx.x; k < C.halo_zstart[z + Zh + 1]; k += kFinThreads) {
      const int h = C.halo_zidx[k];
      const short4 o = C.halo_off[h];
      int px = o.x, py = o.y;
      if constexpr (GEN) {
        const int oo[3] = {o.x, o.y, o.z};
        px = oo[g.perm[0]];
        py = oo[g.perm[1]];
      }
      pl[(px + g.lds_cx) + kLdsWX * (py + g.lds_cy)] = halo[h];
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      if (inside(c, z)) {
        const int pos = pos_of(c);
        const double v = win[c][NS];
        double d0 = 0.0, d1 = 0.0, d2 = 0.0;
#pragma unroll
        for (int q = 1; q <= NS; ++q) {
          d0 += w1[q] * (pl[pos + q] - pl[pos - q]);
          d1 += w1[q] * (pl[pos + q * kLdsWX] - pl[pos - q * kLdsWX]);
          d2 += w1[q] * (win[c][NS + q] - win[c][NS - q]);
        }
        double ga[3], rb[3];
        if constexpr (GEN) {
          // dv/dxi along the lattice axes, then dv/dr = J dv/dxi; rbar = A o
          double dxi[3];
          dxi[g.perm[0]] = d0;
          dxi[g.perm[1]] = d1;
          dxi[g.perm[2]] = d2;
#pragma unroll
          for (int al = 0; al < 3; ++al) dxi[al] *= g.inv_d[al];
#pragma unroll
          for (int a = 0; a < 3; ++a) ga[a] = g.J[a] * dxi[0] + g.J[a + 3] * dxi[1] + g.J[a + 6] * dxi[2];
          int o[3];
          o[g.perm[0]] = ox_of(c);
          o[g.perm[1]] = oy_of(c);
          o[g.perm[2]] = z;
#pragma unroll
          for (int a = 0; a < 3; ++a) rb[a] = g.A[a] * o[0] + g.A[a + 3] * o[1] + g.A[a + 6] * o[2];
        } else {
          ga[0] = d0 * g.inv_d[0];
          ga[1] = d1 * g.inv_d[1];
          ga[2] = d2 * g.inv_d[2];
          rb[0] = ox_of(c) * g.d[0];
          rb[1] = oy_of(c) * g.d[1];
          rb[2] = z * g.d[2];
        }
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

template <int NS, bool GEN>
hipError_t finalize_sweep_cpt(int cpt, const Geo& g, const Batch& B, const double* rho_ws, const double* v_ws,
                              long long rstride, const double* halo_ws, long long hstride, double* outE, double* outS,
                              size_t lds, hipStream_t s) {
  const void* fn = nullptr;
  switch (cpt) {
    case 1: fn = (const void*)k_finalize_sweep<NS, 1, GEN>; break;
    case 2: fn = (const void*)k_finalize_sweep<NS, 2, GEN>; break;
    case 3: fn = (const void*)k_finalize_sweep<NS, 3, GEN>; break;
    case 4: fn = (const void*)k_finalize_sweep<NS, 4, GEN>; break;
    default: return hipErrorInvalidValue;
  }
  if (lds > 64 * 1024) {
    const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  const dim3 grid((unsigned)B.nb);
#define EXX_FIN_ARGS g, B.cls, B.pairs, B.order, B.p0, B.n_eff, rho_ws, v_ws, rstride, halo_ws, hstride, outE, outS
  switch (cpt) {
    case 1: k_finalize_sweep<NS, 1, GEN><<<grid, kFinThreads, lds, s>>>(EXX_FIN_ARGS); break;
    case 2: k_finalize_sweep<NS, 2, GEN><<<grid, kFinThreads, lds, s>>>(EXX_FIN_ARGS); break;
    case 3: k_finalize_sweep<NS, 3, GEN><<<grid, kFinThreads, lds, s>>>(EXX_FIN_ARGS); break;
    default: k_finalize_sweep<NS, 4, GEN><<<grid, kFinThreads, lds, s>>>(EXX_FIN_ARGS); break;
  }
#undef EXX_FIN_ARGS
  return hipGetLastError();
}

}  // namespace

bool finalize_sweep_supported(const Geo& g, long long max_cols) {
  return max_cols > 0 && max_cols <= 4LL * kFinThreads && (size_t)2 * kLdsWX * g.lds_wy * sizeof(double) <= 160 * 1024;
}

hipError_t launch_finalize_sweep(const Geo& g, const Batch& B, long long max_cols, const double* rho_ws,
                                 const double* v_ws, long long rstride, const double* halo_ws, long long hstride,
                                 double* outE, double* outS, hipStream_t s) {
  if (B.nb <= 0) return hipSuccess;
  if (!finalize_sweep_supported(g, max_cols)) return hipErrorInvalidValue;
  const int cpt = (int)((max_cols + kFinThreads - 1) / kFinThreads);
  const size_t lds = (size_t)2 * kLdsWX * g.lds_wy * sizeof(double);
#define EXX_FIN_CALL(NS, GEN) \
  finalize_sweep_cpt<NS, GEN>(cpt, g, B, rho_ws, v_ws, rstride, halo_ws, hstride, outE, outS, lds, s)
  switch (g.n) {
    case 1: return g.gen ? EXX_FIN_CALL(1, true) : EXX_FIN_CALL(1, false);
    case 2: return g.gen ? EXX_FIN_CALL(2, true) : EXX_FIN_CALL(2, false);
    case 3: return g.gen ? EXX_FIN_CALL(3, true) : EXX_FIN_CALL(3, false);
    default: return hipErrorInvalidValue;
  }
#undef EXX_FIN_CALL
}

}  // namespace exx
