// gfx950 kernels of the EXX pair path (the CG itself is in solve_impl.h, the
// moment and boundary contractions in moments.hip).
//
//   k_pair_count / k_pair_scan / k_pair_fill   unique pair list (Sec. III A Step II)
//   k_pair_order                                processing order, largest spheres first
//   k_gather                                    pair density on PE (Step III)
//   k_rhs                                       CG right-hand side 4 pi rho plus the
//                                               Dirichlet terms of eq. d2_1
//   k_finalize                                  the pair's E_xx and sigma_xx (eq. exxGen_mlwf,
//                                               eq. sxx_working with eq. d1_1)
//   k_dscatter                                  D^i += v phi_j, D^j += v phi_i on the ME
//                                               sphere (Sec. II B 2, eq. Dxx)
//   k_reduce                                    E_xx, sigma_xx over pairs in a fixed order
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_common.h"
#include "exx_launch.h"
#include "harmonics.h"

namespace exx {

namespace {

// ---------------------------------------------------------------------------
// pair list

__device__ __forceinline__ unsigned long long splitmix64_once(unsigned long long state) {
  unsigned long long z = state + 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

// Cartesian local coordinate of offset o (Sec. III B 1: r = h (o / N))
__device__ __forceinline__ void rbar_of(const Geo& g, const short4& o, double* x, double* y, double* z) {
  if (g.gen) {
    *x = g.A[0] * o.x + g.A[3] * o.y + g.A[6] * o.z;
    *y = g.A[1] * o.x + g.A[4] * o.y + g.A[7] * o.z;
    *z = g.A[2] * o.x + g.A[5] * o.y + g.A[8] * o.z;
  } else {
    *x = o.x * g.d[0];
    *y = o.y * g.d[1];
    *z = o.z * g.d[2];
  }
}

// minimum-image separation d = C_j - C_i; returns whether (i, j) is a kept pair
__device__ __forceinline__ bool pair_keep(const Geo& g, const PairParams& pp, const double* C, int i, int j,
                                          double* dm) {
  double d[3], s[3];
  for (int a = 0; a < 3; ++a) d[a] = C[3 * j + a] - C[3 * i + a];
  for (int al = 0; al < 3; ++al)
    s[al] = g.hinv[al + 0] * d[0] + g.hinv[al + 3] * d[1] + g.hinv[al + 6] * d[2];
  for (int al = 0; al < 3; ++al) s[al] -= round(s[al]);
  for (int a = 0; a < 3; ++a) dm[a] = g.h[a + 0] * s[0] + g.h[a + 3] * s[1] + g.h[a + 6] * s[2];
  if (i != j && dm[0] * dm[0] + dm[1] * dm[1] + dm[2] * dm[2] > pp.R_pair2) return false;
  if (pp.frac < 1.0) {
    unsigned long long u =
        splitmix64_once(pp.seed ^ ((unsigned long long)(unsigned)i << 32) ^ (unsigned long long)(unsigned)j);
    double f = (double)(u >> 11) * (1.0 / 9007199254740992.0);
    if (!(f < pp.frac)) return false;
  }
  return true;
}

__global__ void k_pair_count(Geo g, PairParams pp, const double* __restrict__ C, int n_orb, int* __restrict__ cnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_orb) return;
  int c = 0;
  double dm[3];
  for (int j = i; j < n_orb; ++j) c += pair_keep(g, pp, C, i, j, dm) ? 1 : 0;
  cnt[i] = c;
}

// exclusive scan of the counts (one workgroup): off[i] at cnt[n_orb + i], total at cnt[2 n_orb]
__global__ void k_pair_scan(int* cnt, int n_orb) {
  __shared__ long long part[1024];
  const int t = threadIdx.x, nt = blockDim.x;
  const int per = (n_orb + nt - 1) / nt;
  const int lo = t * per, hi = min(n_orb, lo + per);
  long long s = 0;
  for (int i = lo; i < hi; ++i) s += cnt[i];
  part[t] = s;
  __syncthreads();
  if (t == 0) {
    long long a = 0;
    for (int k = 0; k < nt; ++k) {
      long long v = part[k];
      part[k] = a;
      a += v;
    }
    cnt[2 * n_orb] = (int)min(a, (long long)0x7fffffff);
  }
  __syncthreads();
  long long a = part[t];
  for (int i = lo; i < hi; ++i) {
    cnt[n_orb + i] = (int)a;
    a += cnt[i];
  }
}

__global__ void k_pair_fill(Geo g, PairParams pp, const double* __restrict__ C, const double* __restrict__ R_orb,
                            int n_orb, const int* __restrict__ cnt, PairDev* __restrict__ pairs, long long cap) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_orb) return;
  long long k = cnt[n_orb + i];
  double dm[3];
  for (int j = i; j < n_orb; ++j) {
    if (!pair_keep(g, pp, C, i, j, dm)) continue;
    if (k < cap) {
      PairDev P;
      P.i = i;
      P.j = j;
      double Cij[3], s[3];
      for (int a = 0; a < 3; ++a) Cij[a] = C[3 * i + a] + 0.5 * dm[a];
      for (int al = 0; al < 3; ++al)
        s[al] = g.hinv[al + 0] * Cij[0] + g.hinv[al + 3] * Cij[1] + g.hinv[al + 6] * Cij[2];
      for (int al = 0; al < 3; ++al) {
        const double f = s[al] - floor(s[al]);
        P.c[al] = wrapi((int)round(g.N[al] * f), g.N[al]);
      }
      int cls = 0;
      if (pp.n_class > 0 && R_orb) {
        double r = 0.5 * (R_orb[i] + R_orb[j]);
        double kk = round((r - pp.R_min) / pp.R_step);
        kk = fmax(0.0, fmin((double)(pp.n_class - 1), kk));
        cls = (int)kk;
      }
      if (i == j && pp.self_class >= 0) cls = pp.self_class;
      P.cls = cls;
      pairs[k] = P;
    }
    ++k;
  }
}

// Stable counting sort of the pairs by class, largest class index (radius)
// first.  One workgroup: each thread takes a contiguous chunk of pairs.
__global__ __launch_bounds__(1024) void k_pair_order(const PairDev* __restrict__ pairs, const int* __restrict__ cnt,
                                                     int n_orb, int n_class, int* __restrict__ order,
                                                     int* __restrict__ class_cnt, long long cap,
                                                     int* __restrict__ n_eff) {
  __shared__ int tcount[kMaxClasses][1024];
  const int t = threadIdx.x, nt = blockDim.x;
  const long long np = min((long long)cnt[2 * n_orb], cap);   // pairs beyond the capacity were not stored
  if (t == 0) *n_eff = (int)np;
  const long long per = (np + nt - 1) / nt;
  const long long lo = t * per, hi = min(np, lo + per);
  int c[kMaxClasses];
  for (int k = 0; k < kMaxClasses; ++k) c[k] = 0;
  for (long long p = lo; p < hi; ++p) c[pairs[p].cls]++;
  for (int k = 0; k < kMaxClasses; ++k) tcount[k][t] = c[k];
  __syncthreads();
  if (t == 0) {
    long long a = 0;
    for (int k = n_class - 1; k >= 0; --k) {
      long long tot = 0;
      for (int u = 0; u < nt; ++u) {
        int v = tcount[k][u];
        tcount[k][u] = (int)a;
        a += v;
        tot += v;
      }
      class_cnt[k] = (int)tot;
    }
  }
  __syncthreads();
  for (int k = 0; k < kMaxClasses; ++k) c[k] = tcount[k][t];
  for (long long p = lo; p < hi; ++p) order[c[pairs[p].cls]++] = (int)p;
}

// ---------------------------------------------------------------------------
// pair density and moments

template <typename TO>
__device__ __forceinline__ double ldv(const TO* p, long long i) { return (double)p[i]; }

// One workgroup per pair: rho on the PE points in packed order, and the
// power of two 2^e with max |rho| in [2^(e-1), 2^e) (1 for a zero density),
// by which the mixed moment path divides rho before rounding it to BF16.
template <typename TO>
__global__ __launch_bounds__(256) void k_gather(Geo g, const ClassDev* __restrict__ cls,
                                                const PairDev* __restrict__ pairs, const int* __restrict__ order,
                                                long long p0, const int* __restrict__ n_eff,
                                                const TO* __restrict__ orb, double* __restrict__ rho_ws,
                                                long long rstride, double* __restrict__ rho_scale) {
  __shared__ double red[4];
  const int b = blockIdx.x;
  if (p0 + b >= *n_eff) return;
  const PairDev P = pairs[order[p0 + b]];
  const ClassDev& C = cls[P.cls];
  const TO* phi_i = orb + (long long)P.i * g.ngrid;
  const TO* phi_j = orb + (long long)P.j * g.ngrid;
  double* rho = rho_ws + (long long)b * rstride;
  const long long npe = C.n_pe;
  double amax = 0.0;
  for (long long k = threadIdx.x; k < npe; k += blockDim.x) {
    const short4 o = C.me_off[k];
    if (o.w) {   // dead slot of a general cell's padded column
      rho[k] = 0.0;
      continue;
    }
    const int gx = wrapi(P.c[0] + o.x, g.N[0]);
    const int gy = wrapi(P.c[1] + o.y, g.N[1]);
    const int gz = wrapi(P.c[2] + o.z, g.N[2]);
    const long long gi = gx + (long long)g.N[0] * (gy + (long long)g.N[1] * gz);
    const double r = ldv(phi_i, gi) * ldv(phi_j, gi);
    rho[k] = r;
    amax = fmax(amax, fabs(r));
  }
  const long long npad = (npe + 31) / 32 * 32;   // zeros up to the moment kernels' 32-point steps
  for (long long k = npe + threadIdx.x; k < npad; k += blockDim.x) rho[k] = 0.0;
  amax = block_max(amax, red);
  if (threadIdx.x == 0) {
    int e = 0;
    if (amax > 0.0) (void)frexp(amax, &e);
    rho_scale[b] = ldexp(1.0, e);
  }
}

// ---------------------------------------------------------------------------
// the right-hand side, the persistent CG solve, and the per-pair E / sigma

// value of the pair potential at offset o: the CG vector inside PE (or 0 when
// pe_zero), the far field at a Dirichlet point
__device__ __forceinline__ double point_value(const ClassDev& C, int n, const double* xv, const double* halo, int ox,
                                              int oy, int oz, bool pe_zero) {
  const int mx = ox + C.Rg[0] + n, my = oy + C.Rg[1] + n, mz = oz + C.Rg[2] + n;
  if (C.pe_map) {   // general cell: 3D maps of the PE slots and the Dirichlet points
    const long long m = mx + (long long)C.Wm[0] * (my + (long long)C.Wm[1] * mz);
    const int s = C.pe_map[m];
    if (s >= 0) return pe_zero ? 0.0 : xv[s];
    const int h = C.halo_map[m];
    return h >= 0 ? halo[h] : 0.0;
  }
  const int m2 = mx + C.Wm[0] * my;
  const int zr = C.zr_map[m2];
  if (abs(oz) <= zr) return pe_zero ? 0.0 : xv[C.plane_start[oz + C.Zmax] + C.col_map[m2]];
  const int h = C.halo_map[m2 + C.Wm[0] * C.Wm[1] * mz];
  return h >= 0 ? halo[h] : 0.0;
}

// b = 4 pi rho + the stencil reach into the Dirichlet points, where v takes its
// far-field values (eq. pe discretised with eq. d2_1)
__global__ __launch_bounds__(256) void k_rhs(Geo g, const ClassDev* __restrict__ cls, const PairDev* __restrict__ pairs,
                                             const int* __restrict__ order, long long p0,
                                             const int* __restrict__ n_eff, const double* __restrict__ rho_ws,
                                             double* __restrict__ b_ws, long long rstride,
                                             const double* __restrict__ halo_ws, long long hstride) {
  const int bq = blockIdx.y;
  if (p0 + bq >= *n_eff) return;
  const PairDev P = pairs[order[p0 + bq]];
  const ClassDev& C = cls[P.cls];
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= C.n_pe) return;
  const double* halo = halo_ws + (long long)bq * hstride;
  double acc = 4.0 * kPi * rho_ws[(long long)bq * rstride + k];
  if (C.rhs_ptr) {
    // orthorhombic tables: the slot's Dirichlet terms from the plan's CSR
    // table (dead slots have none, and their density is zero)
    for (int e = C.rhs_ptr[k]; e < C.rhs_ptr[k + 1]; ++e) {
      const int2 t = C.rhs_ent[e];
      acc += g.inv_d2[t.y >> 2] * g.w2[t.y & 3] * halo[t.x];
    }
    b_ws[(long long)bq * rstride + k] = acc;
    return;
  }
  const short4 o = C.me_off[k];
  if (g.gen) {
    // every arm of the NK Laplacian (eq. lapG_mod_nk3d), eq. d2_1 along it, at
    // the slots near the Dirichlet points (elsewhere every arm stays in PE)
    if (!o.w && (!C.rhs_edge || ((C.rhs_edge[k >> 5] >> (k & 31)) & 1u))) {
      for (int m = 0; m < g.n_arms; ++m) {
        const int ux = g.arm_u[m][0], uy = g.arm_u[m][1], uz = g.arm_u[m][2];
        for (int q = 1; q <= g.n; ++q)
          acc += g.arm_coef[m] * g.w2[q] *
                 (point_value(C, g.n, nullptr, halo, o.x + q * ux, o.y + q * uy, o.z + q * uz, true) +
                  point_value(C, g.n, nullptr, halo, o.x - q * ux, o.y - q * uy, o.z - q * uz, true));
      }
    }
    b_ws[(long long)bq * rstride + k] = o.w ? 0.0 : acc;
    return;
  }
  if (o.w) {   // dead slot of a padded run
    b_ws[(long long)bq * rstride + k] = 0.0;
    return;
  }
  for (int q = 1; q <= g.n; ++q) {
    acc += g.inv_d2[0] * g.w2[q] *
           (point_value(C, g.n, nullptr, halo, o.x + q, o.y, o.z, true) +
            point_value(C, g.n, nullptr, halo, o.x - q, o.y, o.z, true));
    acc += g.inv_d2[1] * g.w2[q] *
           (point_value(C, g.n, nullptr, halo, o.x, o.y + q, o.z, true) +
            point_value(C, g.n, nullptr, halo, o.x, o.y - q, o.z, true));
    acc += g.inv_d2[2] * g.w2[q] *
           (point_value(C, g.n, nullptr, halo, o.x, o.y, o.z + q, true) +
            point_value(C, g.n, nullptr, halo, o.x, o.y, o.z - q, true));
  }
  b_ws[(long long)bq * rstride + k] = acc;
}

// E_xx and sigma_xx of one pair from its density and potential (one workgroup
// per pair): E = -w dV sum rho v (eq. exxGen_mlwf); sigma^{a al} = -2 w dV
// sum_b (h^-1)_{al b} sum rbar_b rho dv/dr_a (eq. sxx_working), with dv/dr_a =
// sum_al J_{a al} dv/dxi_al from the first-derivative stencil (eq. d1_1).
__global__ __launch_bounds__(256) void k_finalize(Geo g, const ClassDev* __restrict__ cls,
                                                  const PairDev* __restrict__ pairs, const int* __restrict__ order,
                                                  long long p0, const int* __restrict__ n_eff,
                                                  const double* __restrict__ rho_ws,
                                                  const double* __restrict__ v_ws, long long rstride,
                                                  const double* __restrict__ halo_ws, long long hstride,
                                                  double* __restrict__ outE, double* __restrict__ outS) {
  __shared__ double red[4];
  const int bq = blockIdx.x;
  if (p0 + bq >= *n_eff) return;
  const int pid = order[p0 + bq];
  const PairDev P = pairs[pid];
  const ClassDev& C = cls[P.cls];
  const double* rho = rho_ws + (long long)bq * rstride;
  const double* x = v_ws + (long long)bq * rstride;
  const double* halo = halo_ws + (long long)bq * hstride;
  double e = 0.0;
  double T[9];
  for (int t = 0; t < 9; ++t) T[t] = 0.0;
  for (long long k = threadIdx.x; k < C.n_pe; k += blockDim.x) {
    const short4 o = C.me_off[k];
    if (o.w) continue;   // dead slot
    const double rh = rho[k];
    e += rh * x[k];
    double dxi[3] = {0.0, 0.0, 0.0};
    if (!C.pe_map) {
      // orthorhombic tables: the point's own column and plane serve its z and
      // its x/y neighbours (the same lookups as point_value, fewer of them)
      const int mx = o.x + C.Rg[0] + g.n, my = o.y + C.Rg[1] + g.n, mz = o.z + C.Rg[2] + g.n;
      const int m2 = mx + C.Wm[0] * my;
      const int plane = C.Wm[0] * C.Wm[1];
      const int col = C.col_map[m2], zr = C.zr_map[m2];
      const int ps = C.plane_start[o.z + C.Zmax];
      auto in_plane = [&](int dm) -> double {
        const int m = m2 + dm;
        if (abs(o.z) <= C.zr_map[m]) return x[ps + C.col_map[m]];
        const int hh = C.halo_map[m + plane * mz];
        return hh >= 0 ? halo[hh] : 0.0;
      };
      auto along_z = [&](int oz) -> double {
        if (abs(oz) <= zr) return x[C.plane_start[oz + C.Zmax] + col];
        const int hh = C.halo_map[m2 + plane * (oz + C.Rg[2] + g.n)];
        return hh >= 0 ? halo[hh] : 0.0;
      };
      for (int q = 1; q <= g.n; ++q) {
        dxi[0] += g.w1[q] * (in_plane(q) - in_plane(-q));
        dxi[1] += g.w1[q] * (in_plane(q * C.Wm[0]) - in_plane(-q * C.Wm[0]));
        dxi[2] += g.w1[q] * (along_z(o.z + q) - along_z(o.z - q));
      }
    } else {
      for (int q = 1; q <= g.n; ++q) {
        dxi[0] += g.w1[q] * (point_value(C, g.n, x, halo, o.x + q, o.y, o.z, false) -
                             point_value(C, g.n, x, halo, o.x - q, o.y, o.z, false));
        dxi[1] += g.w1[q] * (point_value(C, g.n, x, halo, o.x, o.y + q, o.z, false) -
                             point_value(C, g.n, x, halo, o.x, o.y - q, o.z, false));
        dxi[2] += g.w1[q] * (point_value(C, g.n, x, halo, o.x, o.y, o.z + q, false) -
                             point_value(C, g.n, x, halo, o.x, o.y, o.z - q, false));
      }
    }
    for (int al = 0; al < 3; ++al) dxi[al] *= g.inv_d[al];
    double rb[3];
    rbar_of(g, o, &rb[0], &rb[1], &rb[2]);
    for (int aa = 0; aa < 3; ++aa) {
      const double ga = g.J[aa] * dxi[0] + g.J[aa + 3] * dxi[1] + g.J[aa + 6] * dxi[2];
      for (int b = 0; b < 3; ++b) T[aa + 3 * b] += rb[b] * rh * ga;
    }
  }
  e = block_sum(e, red);
  for (int t = 0; t < 9; ++t) T[t] = block_sum(T[t], red);
  if (threadIdx.x == 0) {
    const double w = (P.i == P.j) ? 1.0 : 2.0;
    outE[pid] = -w * g.dV * e;
    for (int aa = 0; aa < 3; ++aa)
      for (int al = 0; al < 3; ++al) {
        double s = 0.0;
        for (int b = 0; b < 3; ++b) s += g.hinv[al + 3 * b] * T[aa + 3 * b];
        outS[9 * (long long)pid + aa + 3 * al] = -2.0 * w * g.dV * s;
      }
  }
}

// ---------------------------------------------------------------------------
// wavefunction forces

template <int L, typename TO>
__global__ __launch_bounds__(256) void k_dscatter(Geo g, const ClassDev* __restrict__ cls,
                                                  const PairDev* __restrict__ pairs, const int* __restrict__ order,
                                                  long long p0, const int* __restrict__ n_eff,
                                                  const TO* __restrict__ orb, TO* __restrict__ D,
                                                  const int* __restrict__ d_slot,
                                                  const double* __restrict__ v_ws, long long rstride,
                                                  const double* __restrict__ Q_ws) {
  constexpr int NLM = (L + 1) * (L + 1);
  __shared__ double Q[NLM];
  const int b = blockIdx.y;
  if (p0 + b >= *n_eff) return;
  const PairDev P = pairs[order[p0 + b]];
  const ClassDev& C = cls[P.cls];
  if (threadIdx.x < NLM) Q[threadIdx.x] = Q_ws[(long long)b * kMaxLM + threadIdx.x];
  __syncthreads();
  // the ME points in grid raster order, so that a wavefront's orbital reads
  // and D updates fall on consecutive addresses along x
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= C.n_scan) return;
  const int e = C.me_scan[k];
  const short4 o = C.scan_off[k];
  double rx, ry, rz;
  rbar_of(g, o, &rx, &ry, &rz);
  const double v = (e < C.n_pe) ? v_ws[(long long)b * rstride + e] : far_field<L>(rx, ry, rz, g.ylm_norm, Q);
  const int gx = wrapi(P.c[0] + o.x, g.N[0]);
  const int gy = wrapi(P.c[1] + o.y, g.N[1]);
  const int gz = wrapi(P.c[2] + o.z, g.N[2]);
  const long long gi = gx + (long long)g.N[0] * (gy + (long long)g.N[1] * gz);
  const double fi = (double)orb[(long long)P.i * g.ngrid + gi];
  const double fj = (double)orb[(long long)P.j * g.ngrid + gi];
  // output rows: the orbital itself, or its slot in the requested subset (-1: not written)
  const int si = d_slot ? d_slot[P.i] : P.i;
  const int sj = d_slot ? d_slot[P.j] : P.j;
  if (si >= 0) unsafeAtomicAdd(&D[(long long)si * g.ngrid + gi], (TO)(v * fj));
  if (P.i != P.j && sj >= 0) unsafeAtomicAdd(&D[(long long)sj * g.ngrid + gi], (TO)(v * fi));
}

// ---------------------------------------------------------------------------
// warm start: the previous evaluation's pair list and solutions

// warm_map[p] = row of pair p in the previous list (same i, j and class, grid
// centre moved by at most one point per axis), else -1.  Both lists are in
// canonical order (i ascending, then j), so the previous pairs of orbital i
// are a sorted range found from the previous per-orbital offsets.
__global__ void k_warm_match(Geo g, const PairDev* __restrict__ pairs, const int* __restrict__ n_eff,
                             const PairDev* __restrict__ prev_pairs, const int* __restrict__ prev_offs,
                             const int* __restrict__ state, int* __restrict__ warm_map) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= *n_eff) return;
  int q = -1;
  const PairDev P = pairs[p];
  const int prev_valid = state[1], prev_orb = state[2], prev_stored = state[3];
  if (prev_valid && P.i < prev_orb) {
    int lo = prev_offs[P.i], hi = prev_offs[P.i + 1];
    if (hi > prev_stored) hi = prev_stored;
    while (lo < hi) {   // first previous pair of orbital i with j >= P.j
      const int mid = (lo + hi) >> 1;
      if (prev_pairs[mid].j < P.j) lo = mid + 1; else hi = mid;
    }
    const int end = min(prev_offs[P.i + 1], prev_stored);
    if (lo < end && prev_pairs[lo].j == P.j && prev_pairs[lo].cls == P.cls) {
      bool near = true;
      for (int a = 0; a < 3; ++a) {
        int d = P.c[a] - prev_pairs[lo].c[a];
        if (d > g.N[a] / 2) d -= g.N[a];
        if (d < -g.N[a] / 2) d += g.N[a];
        near = near && d >= -1 && d <= 1;
      }
      if (near) q = lo;
    }
  }
  warm_map[p] = q;
}

// After an evaluation: its pair list becomes the previous one, and the store
// its solutions were written to becomes the one the next evaluation reads.
// One thread per element of the larger of the two copies.
__global__ void k_warm_commit(const PairDev* __restrict__ pairs, const int* __restrict__ counts, int n_orb,
                              const int* __restrict__ n_eff, long long cap, PairDev* __restrict__ prev_pairs,
                              int* __restrict__ prev_offs, int* __restrict__ state) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long stored = *n_eff;
  if (t < stored && t < cap) prev_pairs[t] = pairs[t];
  if (t <= n_orb) prev_offs[t] = counts[n_orb + t];
  if (t == 0) {
    state[0] = 1 - state[0];
    state[1] = 1;
    state[2] = n_orb;
    state[3] = (int)stored;
  }
}

template <typename T>
__global__ void k_zero(T* p, long long n) {
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (long long)gridDim.x * blockDim.x)
    p[k] = (T)0;
}

__global__ void k_set_int(int* p, int v) { *p = v; }

// slot[i] = position of orbital i in the D subset, or -1 (entries outside
// [0, n_orb) are skipped; the caller guarantees distinct entries)
__global__ void k_dslot_clear(int* slot, int n_orb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_orb) slot[i] = -1;
}
__global__ void k_dslot_fill(int* slot, int n_orb, const int* __restrict__ subset, int n_subset) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < n_subset && subset[s] >= 0 && subset[s] < n_orb) slot[subset[s]] = s;
}

__global__ __launch_bounds__(256) void k_reduce(const double* __restrict__ pE, const double* __restrict__ pS,
                                                const int* __restrict__ pIt, const double* __restrict__ pRes,
                                                const int* __restrict__ pUpd, const int* __restrict__ pSav,
                                                const int* __restrict__ pExit,
                                                const PairDev* __restrict__ pairs, const ClassDev* __restrict__ cls,
                                                const int* __restrict__ cnt, int n_orb, const int* __restrict__ n_eff,
                                                const int* __restrict__ warm_map,
                                                double* __restrict__ E, double* __restrict__ sigma,
                                                double* __restrict__ stats) {
  __shared__ double red[4];
  const long long np = *n_eff;
  double e = 0.0, s[9], isum = 0.0, imax = 0.0, nunc = 0.0, rmax = 0.0, work = 0.0, pts = 0.0, umax = 0.0,
         warm = 0.0, ncap = 0.0, nbrk = 0.0, nnan = 0.0, nrst = 0.0;
  for (int t = 0; t < 9; ++t) s[t] = 0.0;
  for (long long k = threadIdx.x; k < np; k += blockDim.x) {
    e += pE[k];
    for (int t = 0; t < 9; ++t) s[t] += pS[9 * k + t];
    isum += pIt[k];
    imax = fmax(imax, (double)pIt[k]);
    umax = fmax(umax, (double)pUpd[k]);
    // the solve's own exit reason, not the iteration count, says whether a
    // pair converged (a pair may converge on its last permitted iteration)
    const int ex = pExit[k] & 0xff;
    nunc += ex != EXX_CG_CONVERGED ? 1.0 : 0.0;
    ncap += ex == EXX_CG_CAP ? 1.0 : 0.0;
    nbrk += ex == EXX_CG_BREAKDOWN ? 1.0 : 0.0;
    nnan += ex == EXX_CG_NONFINITE ? 1.0 : 0.0;
    nrst += (double)(pExit[k] >> 8);
    rmax = fmax(rmax, pRes[k]);
    const double npe = (double)cls[pairs[k].cls].n_real;
    // 8 vector accesses per point and iteration, two fewer for each fused
    // sweep and each pass B that left x alone
    work += (pIt[k] - 0.25 * pSav[k]) * npe;
    pts += npe;
    if (warm_map && warm_map[k] >= 0) warm += 1.0;
  }
  e = block_sum(e, red);
  for (int t = 0; t < 9; ++t) s[t] = block_sum(s[t], red);
  isum = block_sum(isum, red);
  nunc = block_sum(nunc, red);
  work = block_sum(work, red);
  pts = block_sum(pts, red);
  warm = block_sum(warm, red);
  ncap = block_sum(ncap, red);
  nbrk = block_sum(nbrk, red);
  nnan = block_sum(nnan, red);
  nrst = block_sum(nrst, red);
  // max via shuffles
  for (int o = 32; o > 0; o >>= 1) {
    imax = fmax(imax, __shfl_xor(imax, o, 64));
    rmax = fmax(rmax, __shfl_xor(rmax, o, 64));
    umax = fmax(umax, __shfl_xor(umax, o, 64));
  }
  __shared__ double mx[3][4];
  if ((threadIdx.x & 63) == 0) {
    mx[0][threadIdx.x >> 6] = imax;
    mx[1][threadIdx.x >> 6] = rmax;
    mx[2][threadIdx.x >> 6] = umax;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) {
      imax = fmax(imax, mx[0][w]);
      rmax = fmax(rmax, mx[1][w]);
      umax = fmax(umax, mx[2][w]);
    }
    if (E) *E = e;
    if (sigma)
      for (int t = 0; t < 9; ++t) sigma[t] = s[t];
    stats[0] = isum;
    stats[1] = imax;
    stats[2] = nunc;
    stats[3] = rmax;
    stats[4] = (double)cnt[2 * n_orb];   // every kept pair, also those beyond the capacity
    stats[5] = work;
    stats[6] = umax;
    stats[7] = pts;
    stats[8] = warm;
    stats[9] = ncap;
    stats[10] = nbrk;
    stats[11] = nnan;
    stats[12] = nrst;
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers

hipError_t launch_pairlist(const Geo& g, const PairParams& pp, const double* centres, const double* R_orb, int n_orb,
                           int* counts, PairDev* pairs, long long cap, hipStream_t s) {
  const int nb = (n_orb + 127) / 128;
  k_pair_count<<<nb, 128, 0, s>>>(g, pp, centres, n_orb, counts);
  k_pair_scan<<<1, 1024, 0, s>>>(counts, n_orb);
  if (cap > 0) k_pair_fill<<<nb, 128, 0, s>>>(g, pp, centres, R_orb, n_orb, counts, pairs, cap);
  return hipGetLastError();
}

hipError_t launch_order(const PairDev* pairs, const int* counts, int n_orb, int n_class, int* order, long long cap,
                        int* n_eff, hipStream_t s) {
  int* class_cnt = const_cast<int*>(counts) + 2 * n_orb + 1;
  k_pair_order<<<1, 1024, 0, s>>>(pairs, counts, n_orb, n_class, order, class_cnt, cap, n_eff);
  return hipGetLastError();
}

hipError_t launch_dslot(int* slot, int n_orb, const int* subset, int n_subset, hipStream_t s) {
  k_dslot_clear<<<(n_orb + 255) / 256, 256, 0, s>>>(slot, n_orb);
  if (n_subset > 0) k_dslot_fill<<<(n_subset + 255) / 256, 256, 0, s>>>(slot, n_orb, subset, n_subset);
  return hipGetLastError();
}

#define EXX_L_DISPATCH(L, ...)                       \
  switch (L) {                                       \
    case 0: { constexpr int LL = 0; __VA_ARGS__; } break; \
    case 1: { constexpr int LL = 1; __VA_ARGS__; } break; \
    case 2: { constexpr int LL = 2; __VA_ARGS__; } break; \
    case 3: { constexpr int LL = 3; __VA_ARGS__; } break; \
    case 4: { constexpr int LL = 4; __VA_ARGS__; } break; \
    case 5: { constexpr int LL = 5; __VA_ARGS__; } break; \
    case 6: { constexpr int LL = 6; __VA_ARGS__; } break; \
    case 7: { constexpr int LL = 7; __VA_ARGS__; } break; \
    case 8: { constexpr int LL = 8; __VA_ARGS__; } break; \
    default: return hipErrorInvalidValue;            \
  }

hipError_t launch_gather(const Geo& g, const Batch& B, const void* orb, int dt, double* rho_ws, long long rstride,
                         double* rho_scale, hipStream_t s) {
  if (B.nb <= 0) return hipSuccess;
  if (dt == EXX_F64)
    k_gather<double><<<(unsigned)B.nb, 256, 0, s>>>(g, B.cls, B.pairs, B.order, B.p0, B.n_eff, (const double*)orb,
                                                    rho_ws, rstride, rho_scale);
  else
    k_gather<float><<<(unsigned)B.nb, 256, 0, s>>>(g, B.cls, B.pairs, B.order, B.p0, B.n_eff, (const float*)orb,
                                                   rho_ws, rstride, rho_scale);
  return hipGetLastError();
}

hipError_t launch_rhs(const Geo& g, const Batch& B, long long max_pe, const double* rho_ws, double* b_ws,
                      long long rstride, const double* halo_ws, long long hstride, hipStream_t s) {
  if (B.nb <= 0) return hipSuccess;
  dim3 grid((unsigned)((max_pe + 255) / 256), (unsigned)B.nb);
  k_rhs<<<grid, 256, 0, s>>>(g, B.cls, B.pairs, B.order, B.p0, B.n_eff, rho_ws, b_ws, rstride, halo_ws, hstride);
  return hipGetLastError();
}

hipError_t launch_finalize(const Geo& g, const Batch& B, const double* rho_ws, const double* v_ws, long long rstride,
                           const double* halo_ws, long long hstride, double* outE, double* outS, hipStream_t s) {
  if (B.nb <= 0) return hipSuccess;
  k_finalize<<<(unsigned)B.nb, 256, 0, s>>>(g, B.cls, B.pairs, B.order, B.p0, B.n_eff, rho_ws, v_ws, rstride,
                                            halo_ws, hstride, outE, outS);
  return hipGetLastError();
}

hipError_t launch_dscatter(const Geo& g, const Batch& B, long long max_me, const void* orb, void* D,
                           const int* d_slot, int dt, const double* v_ws, long long rstride, const double* Q_ws,
                           hipStream_t s) {
  if (B.nb <= 0) return hipSuccess;
  dim3 grid((unsigned)((max_me + 255) / 256), (unsigned)B.nb);
  if (dt == EXX_F64) {
    EXX_L_DISPATCH(g.l_max, (k_dscatter<LL, double><<<grid, 256, 0, s>>>(g, B.cls, B.pairs, B.order, B.p0, B.n_eff,
                                                                         (const double*)orb, (double*)D, d_slot,
                                                                         v_ws, rstride, Q_ws)));
  } else {
    EXX_L_DISPATCH(g.l_max, (k_dscatter<LL, float><<<grid, 256, 0, s>>>(g, B.cls, B.pairs, B.order, B.p0, B.n_eff,
                                                                        (const float*)orb, (float*)D, d_slot,
                                                                        v_ws, rstride, Q_ws)));
  }
  return hipGetLastError();
}

hipError_t launch_warm_match(const Geo& g, const PairDev* pairs, const int* n_eff, long long cap,
                             const PairDev* prev_pairs, const int* prev_offs, const int* state, int* warm_map,
                             hipStream_t s) {
  if (cap <= 0) return hipSuccess;
  k_warm_match<<<(unsigned)((cap + 255) / 256), 256, 0, s>>>(g, pairs, n_eff, prev_pairs, prev_offs, state,
                                                             warm_map);
  return hipGetLastError();
}

hipError_t launch_warm_commit(const PairDev* pairs, const int* counts, int n_orb, const int* n_eff, long long cap,
                              PairDev* prev_pairs, int* prev_offs, int* state, hipStream_t s) {
  const long long n = std::max<long long>(cap, (long long)n_orb + 1);
  k_warm_commit<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(pairs, counts, n_orb, n_eff, cap, prev_pairs, prev_offs,
                                                            state);
  return hipGetLastError();
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s) {
  if (bytes == 0) return hipSuccess;
  if (bytes % 8 == 0) {
    long long n = (long long)(bytes / 8);
    unsigned nb = (unsigned)std::min<long long>((n + 255) / 256, 65536);
    k_zero<double><<<nb, 256, 0, s>>>((double*)p, n);
  } else {
    long long n = (long long)(bytes / 4);
    unsigned nb = (unsigned)std::min<long long>((n + 255) / 256, 65536);
    k_zero<float><<<nb, 256, 0, s>>>((float*)p, n);
  }
  return hipGetLastError();
}

hipError_t launch_set_int(int* p, int v, hipStream_t s) {
  k_set_int<<<1, 1, 0, s>>>(p, v);
  return hipGetLastError();
}

hipError_t launch_reduce(const double* pE, const double* pS, const int* pIt, const double* pRes, const int* pUpd,
                         const int* pSav, const int* pExit, const PairDev* pairs, const ClassDev* cls,
                         const int* counts, int n_orb, const int* n_eff, const int* warm_map, double* E, double* sigma,
                         double* stats, hipStream_t s) {
  k_reduce<<<1, 256, 0, s>>>(pE, pS, pIt, pRes, pUpd, pSav, pExit, pairs, cls, counts, n_orb, n_eff, warm_map, E, sigma,
                             stats);
  return hipGetLastError();
}

}  // namespace exx
