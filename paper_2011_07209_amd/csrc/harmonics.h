// Real solid harmonics shared by the host plan (moment tables) and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace exx {

// Regular solid harmonics R_lm(r) = |r|^l S_lm(rhat) with real orthonormal S
// (no Condon-Shortley phase), generated as polynomials in x, y, z:
//   (x + i y)^m gives the azimuthal factor,
//   P_mm = (2m-1)!!,  P_{m+1,m} = (2m+1) z P_mm,
//   (l-m) P_lm = (2l-1) z P_{l-1,m} - (l+m-1) |r|^2 P_{l-2,m},
// so that R_lm = norm_lm P_lm Re/Im (x + i y)^m.  sink(l, index, value) receives
// each of the (L+1)^2 values once.
template <int L, typename F>
__host__ __device__ __forceinline__ void solid_harmonics(double x, double y, double z, const double* norm, F&& sink) {
  const double r2 = x * x + y * y + z * z;
  double cm = 1.0, sm = 0.0, pmm = 1.0;
#pragma unroll
  for (int m = 0; m <= L; ++m) {
    double p0 = pmm, p1 = 0.0;
    if (m == 0) {
      sink(0, 0, norm[0] * p0);
    } else {
      sink(m, m * m + 2 * m, norm[m * m + 2 * m] * p0 * cm);
      sink(m, m * m, norm[m * m] * p0 * sm);
    }
    if (m < L) {
      p1 = (2.0 * m + 1.0) * z * pmm;
      const int l = m + 1;
      if (m == 0) {
        sink(l, l * l + l, norm[l * l + l] * p1);
      } else {
        sink(l, l * l + l + m, norm[l * l + l + m] * p1 * cm);
        sink(l, l * l + l - m, norm[l * l + l - m] * p1 * sm);
      }
    }
#pragma unroll
    for (int l = m + 2; l <= L; ++l) {
      const double p2 = ((2.0 * l - 1.0) * z * p1 - (l + m - 1.0) * r2 * p0) * (1.0 / (double)(l - m));
      if (m == 0) {
        sink(l, l * l + l, norm[l * l + l] * p2);
      } else {
        sink(l, l * l + l + m, norm[l * l + l + m] * p2 * cm);
        sink(l, l * l + l - m, norm[l * l + l - m] * p2 * sm);
      }
      p0 = p1;
      p1 = p2;
    }
    const double cn = x * cm - y * sm;
    sm = x * sm + y * cm;
    cm = cn;
    pmm *= (2.0 * m + 1.0);
  }
}

// Far-field potential 4 pi sum_lm Q_lm R_lm(r) / ((2l+1) |r|^(2l+1))
template <int L>
__host__ __device__ __forceinline__ double far_field(double x, double y, double z, const double* norm, const double* Q) {
  double s[L + 1];
#pragma unroll
  for (int l = 0; l <= L; ++l) s[l] = 0.0;
  solid_harmonics<L>(x, y, z, norm, [&](int l, int idx, double v) { s[l] += Q[idx] * v; });
  const double r2 = x * x + y * y + z * z;
  const double rinv = 1.0 / std::sqrt(r2);
  const double rinv2 = rinv * rinv;
  double rp = rinv, v = 0.0;
#pragma unroll
  for (int l = 0; l <= L; ++l) {
    v += s[l] * rp * (4.0 * 3.14159265358979323846 / (2.0 * l + 1.0));
    rp *= rinv2;
  }
  return v;
}

// Runtime-L entry for host code: R_lm(r) for all (l, m), l <= L, into out[l*l + l + m].
inline void solid_harmonics_host(int L, double x, double y, double z, const double* norm, double* out) {
  auto put = [&](int, int idx, double v) { out[idx] = v; };
  switch (L) {
    case 0: solid_harmonics<0>(x, y, z, norm, put); break;
    case 1: solid_harmonics<1>(x, y, z, norm, put); break;
    case 2: solid_harmonics<2>(x, y, z, norm, put); break;
    case 3: solid_harmonics<3>(x, y, z, norm, put); break;
    case 4: solid_harmonics<4>(x, y, z, norm, put); break;
    case 5: solid_harmonics<5>(x, y, z, norm, put); break;
    case 6: solid_harmonics<6>(x, y, z, norm, put); break;
    case 7: solid_harmonics<7>(x, y, z, norm, put); break;
    default: solid_harmonics<8>(x, y, z, norm, put); break;
  }
}

}  // namespace exx
