// Multipole moments of the pair densities (Sec. I, eq. mepole) on the matrix
// cores.  For the pairs of one sphere class the moments are one dense
// contraction,
//   Q[pair][lm] = dV N_lm sum_k P_lm(rbar_k) rho[pair][k],
// with P_lm the unnormalised solid harmonics of the PE offsets, a per-class
// table built at plan time (rows padded to 16, points padded to 16, zeros).
// The normalisation N_lm and dV are applied in FP64 after the sum, so that the
// constant l = 0 row is exactly 1 in every table precision.
//
// Workgroup: 4 wavefronts, 64 pairs of one class; wavefront w takes pairs
// 16w..16w+15 as the 16 columns of its MFMA tiles and every 16-row tile of
// the table.  Table layout [k/4][row][4]: lane l reads row (l mod 16) at points
// 4 (l / 16) .. +3 of each block of 16, and the same points of its own pair's
// density, so one MFMA k-slot pairs table and density entries of the same
// point.
//   FP64 plans:  v_mfma_f64_16x16x4_f64, FP64 table, FP64 accumulation.
//   Mixed plans: split BF16 (x = hi + lo) for table and density,
//                hi*hi + hi*lo + lo*hi on v_mfma_f32_16x16x16_bf16 with FP32
//                accumulation, folded into FP64 every 512 points.  The
//                density is first divided by its pair's power-of-two scale
//                (max |rho| <= scale < 2 max |rho|), which is exact and keeps
//                vanishing densities inside the FP32/BF16 normal range.
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "exx_launch.h"

namespace exx {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef short v4s __attribute__((ext_vector_type(4)));

constexpr int kTilePairs = 64;
constexpr int kFoldSteps = 32;   // 16-point blocks between FP32 -> FP64 folds

__device__ __forceinline__ unsigned short f2bf(float f) {   // round to nearest even (finite inputs)
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

// The tile of this workgroup: classes are laid out in processing order
// (descending class index) with class_cnt[k] pairs each; the tiles of one
// class never straddle a class boundary.  Returns false for surplus groups.
__device__ __forceinline__ bool locate_tile(const int* __restrict__ class_cnt, int ncls, long long pbeg,
                                            long long pend, int* cls, long long* tb, long long* te) {
  long long t = blockIdx.x, start = 0;
  for (int k = ncls - 1; k >= 0; --k) {
    const long long cnt = class_cnt[k];
    const long long lo = start > pbeg ? start : pbeg;
    const long long hi = start + cnt < pend ? start + cnt : pend;
    start += cnt;
    if (hi <= lo) continue;
    const long long nt = (hi - lo + kTilePairs - 1) / kTilePairs;
    if (t < nt) {
      *cls = k;
      *tb = lo + t * kTilePairs;
      *te = *tb + kTilePairs < hi ? *tb + kTilePairs : hi;
      return true;
    }
    t -= nt;
  }
  return false;
}

template <int RT>
__global__ __launch_bounds__(256) void k_moments_f64(Geo g, const ClassDev* __restrict__ cls_tab,
                                                     const int* __restrict__ class_cnt, int ncls, long long pbeg,
                                                     long long pend, const double* __restrict__ rho_ws,
                                                     long long rstride, const double* __restrict__ rho_scale,
                                                     double* __restrict__ Q_ws) {
  int cls;
  long long tb, te;
  if (!locate_tile(class_cnt, ncls, pbeg, pend, &cls, &tb, &te)) return;
  const ClassDev& C = cls_tab[cls];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, kq = lane >> 4;
  const long long p = tb + 16 * wave + col;
  const bool valid = p < te;
  const double* rho = rho_ws + (valid ? (p - pbeg) * rstride : 0);
  const long long npe = C.n_pe;
  const double* tab = C.mom_f64 + (long long)col * 4;
  constexpr int ROWS = 16 * RT;
  v4d acc[RT];
#pragma unroll
  for (int r = 0; r < RT; ++r) acc[r] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll 2
  for (long long k0 = 0; k0 < npe; k0 += 16) {
    const long long kb = k0 + 4 * kq;
    double b[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) b[j] = (valid && kb + j < npe) ? rho[kb + j] : 0.0;
    const double* tk = tab + (kb >> 2) * (ROWS * 4);
#pragma unroll
    for (int r = 0; r < RT; ++r) {
      const v4d a = *reinterpret_cast<const v4d*>(tk + r * 64);
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[r] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[j], b[j], acc[r], 0, 0, 0);
    }
  }
  if (!valid) return;
  // v_mfma_f64_16x16x4_f64 leaves D[i][j] in lane j + 16 (i mod 4), item i / 4
  double* Q = Q_ws + (p - pbeg) * kMaxLM;
#pragma unroll
  for (int r = 0; r < RT; ++r)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int lm = 16 * r + kq + 4 * i;
      if (lm < g.n_lm) Q[lm] = g.dV * g.ylm_norm[lm] * acc[r][i];
    }
}

template <int RT>
__global__ __launch_bounds__(256) void k_moments_bf16(Geo g, const ClassDev* __restrict__ cls_tab,
                                                      const int* __restrict__ class_cnt, int ncls, long long pbeg,
                                                      long long pend, const double* __restrict__ rho_ws,
                                                      long long rstride, const double* __restrict__ rho_scale,
                                                      double* __restrict__ Q_ws) {
  int cls;
  long long tb, te;
  if (!locate_tile(class_cnt, ncls, pbeg, pend, &cls, &tb, &te)) return;
  const ClassDev& C = cls_tab[cls];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, kq = lane >> 4;
  const long long p = tb + 16 * wave + col;
  const bool valid = p < te;
  const double* rho = rho_ws + (valid ? (p - pbeg) * rstride : 0);
  const long long npe = C.n_pe;
  const double scale = valid ? rho_scale[p - pbeg] : 1.0;
  const double inv_scale = 1.0 / scale;   // exact: a power of two
  const unsigned short* th = C.mom_hi + (long long)col * 4;
  const unsigned short* tl = C.mom_lo + (long long)col * 4;
  constexpr int ROWS = 16 * RT;
  v4f acc[RT];
  double accd[RT][4];
#pragma unroll
  for (int r = 0; r < RT; ++r) {
    acc[r] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int i = 0; i < 4; ++i) accd[r][i] = 0.0;
  }
  int steps = 0;
  for (long long k0 = 0; k0 < npe; k0 += 16) {
    const long long kb = k0 + 4 * kq;
    v4s bh, bl;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float x = (valid && kb + j < npe) ? (float)(rho[kb + j] * inv_scale) : 0.0f;
      const unsigned short h = f2bf(x);
      bh[j] = (short)h;
      bl[j] = (short)f2bf(x - bf2f(h));
    }
    const long long off = (kb >> 2) * (ROWS * 4);
#pragma unroll
    for (int r = 0; r < RT; ++r) {
      const v4s ah = *reinterpret_cast<const v4s*>(th + off + r * 64);
      const v4s al = *reinterpret_cast<const v4s*>(tl + off + r * 64);
      acc[r] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, acc[r], 0, 0, 0);
      acc[r] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, acc[r], 0, 0, 0);
      acc[r] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, acc[r], 0, 0, 0);
    }
    if (++steps == kFoldSteps) {
      steps = 0;
#pragma unroll
      for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          accd[r][i] += (double)acc[r][i];
          acc[r][i] = 0.f;
        }
    }
  }
  if (!valid) return;
  // v_mfma_f32_16x16x16_bf16 leaves D[i][j] in lane j + 16 (i / 4), item i mod 4
  double* Q = Q_ws + (p - pbeg) * kMaxLM;
#pragma unroll
  for (int r = 0; r < RT; ++r)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int lm = 16 * r + 4 * kq + i;
      if (lm < g.n_lm) Q[lm] = g.dV * g.ylm_norm[lm] * scale * (accd[r][i] + (double)acc[r][i]);
    }
}

}  // namespace

int moment_rows(int l_max) { return ((l_max + 1) * (l_max + 1) + 15) / 16 * 16; }

long long moment_tiles(long long nb, int ncls) { return (nb + kTilePairs - 1) / kTilePairs + ncls - 1; }

hipError_t launch_moments(const Geo& g, const ClassDev* cls, const int* class_cnt, int ncls, bool mixed,
                          long long pbeg, long long nb, const double* rho_ws, long long rstride,
                          const double* rho_scale, double* Q_ws, hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  const unsigned tiles = (unsigned)moment_tiles(nb, ncls);
  const long long pend = pbeg + nb;
#define EXX_MOM(RT)                                                                                             \
  case RT:                                                                                                      \
    if (mixed)                                                                                                  \
      k_moments_bf16<RT><<<tiles, 256, 0, s>>>(g, cls, class_cnt, ncls, pbeg, pend, rho_ws, rstride, rho_scale, Q_ws);     \
    else                                                                                                        \
      k_moments_f64<RT><<<tiles, 256, 0, s>>>(g, cls, class_cnt, ncls, pbeg, pend, rho_ws, rstride, rho_scale, Q_ws);      \
    break;
  switch (moment_rows(g.l_max) / 16) {
    EXX_MOM(1) EXX_MOM(2) EXX_MOM(3) EXX_MOM(4) EXX_MOM(5) EXX_MOM(6)
    default: return hipErrorInvalidValue;
  }
#undef EXX_MOM
  return hipGetLastError();
}

}  // namespace exx
