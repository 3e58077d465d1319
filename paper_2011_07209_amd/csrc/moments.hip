// Multipole moments of the pair densities (Sec. I, eq. mepole) on the matrix
// cores.  For the pairs of one sphere class the moments are one dense
// contraction,
//   Q[pair][lm] = dV N_lm sum_k P_lm(rbar_k) rho[pair][k],
// with P_lm the unnormalised solid harmonics of the PE offsets, a per-class
// table built at plan time (rows padded to 16, points padded to 32, zeros).
// The normalisation N_lm and dV are applied in FP64 after the sum, so that the
// constant l = 0 row is exactly 1 in every table precision.
//
// Work decomposition: a workgroup takes a tile of 64 pairs of one class and
// one chunk of the points (the grid's y index), so that a batch of a few
// thousand pairs still fills the chip.  Each wavefront takes CT 16-pair MFMA
// column tiles (FP64: 2 wavefronts of 2 tiles; mixed: 4 wavefronts of 1 tile,
// which keeps its FP64 fold registers within occupancy 4) and every 16-row
// tile of the table.
// Each chunk writes FP64 partial sums; k_moment_sum adds them in chunk order,
// so the result does not depend on scheduling.
//
//   FP64 plans:  v_mfma_f64_16x16x4_f64 on an FP64 table, layout [k/4][row][4]
//                (lane l: row l mod 16, points 4 (l/16) .. +3 of a 16-point step).
//   Mixed plans: split BF16 (x = hi + lo) for table and density,
//                hi*hi + hi*lo + lo*hi on v_mfma_f32_16x16x32_bf16, FP32
//                accumulation folded into FP64 every 512 points; table layout
//                [k/8][row][8] (lane l: row l mod 16, points 8 (l/16) .. +7 of
//                a 32-point step).  The density is first divided by its pair's
//                power-of-two scale (max |rho| <= scale < 2 max |rho|), which is
//                exact and keeps vanishing densities inside the BF16 normal range.
//
// The density rows are zero from n_pe up to the next multiple of 32 (written
// by the gather), so the point loop needs no bounds test.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_common.h"
#include "exx_launch.h"

namespace exx {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8b __attribute__((ext_vector_type(8)));

constexpr int kTilePairs = 64;
constexpr int kColTilesF64 = 2;                           // 16-pair MFMA column tiles per wavefront
constexpr int kColTilesBF16 = 1;
constexpr int kFoldSteps = 16;                            // 32-point steps between FP32 -> FP64 folds

// The tile of this workgroup: classes are laid out in processing order
// (descending class index) with class_cnt[k] pairs each; the tiles of one
// class never straddle a class boundary.  Returns false for surplus groups.
__device__ __forceinline__ bool locate_tile(const int* __restrict__ class_cnt, int ncls, long long pbeg,
                                            long long pend, const int* __restrict__ n_eff, int* cls, long long* tb,
                                            long long* te) {
  if (pend > *n_eff) pend = *n_eff;
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

// Steps [s0, s1) of chunk blockIdx.y when a class's `steps` steps are cut into
// gridDim.y nearly equal chunks (possibly empty ones at the end).
__device__ __forceinline__ void chunk_range(long long steps, long long* s0, long long* s1) {
  const long long per = (steps + gridDim.y - 1) / gridDim.y;
  const long long a = (long long)blockIdx.y * per;
  *s0 = a < steps ? a : steps;
  *s1 = a + per < steps ? a + per : steps;
}

template <int RT, int REM, int kColTiles = kColTilesF64>
__global__ __launch_bounds__(kTilePairs / kColTiles * 4) void k_moments_f64(const ClassDev* __restrict__ cls_tab,
                                                             const int* __restrict__ class_cnt, int ncls,
                                                             long long pbeg, long long pend,
                                                             const int* __restrict__ n_eff,
                                                             const double* __restrict__ rho_ws, long long rstride,
                                                             double* __restrict__ Qp, long long nb) {
  int cls;
  long long tb, te;
  if (!locate_tile(class_cnt, ncls, pbeg, pend, n_eff, &cls, &tb, &te)) return;
  const ClassDev& C = cls_tab[cls];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, kq = lane >> 4;
  constexpr int ROWS = 16 * RT + REM;   // MFMA row tiles, then REM rows on the vector ALU
  long long p[kColTiles];
  bool valid[kColTiles];
  const double* rho[kColTiles];
#pragma unroll
  for (int c = 0; c < kColTiles; ++c) {
    p[c] = tb + 16 * (kColTiles * wave + c) + col;
    valid[c] = p[c] < te;
    rho[c] = rho_ws + (valid[c] ? (p[c] - pbeg) * rstride : 0) + 4 * kq;
  }
  long long s0, s1;
  chunk_range((C.n_pe + 15) / 16, &s0, &s1);
  const double* tab = C.mom_f64 + (long long)kq * (ROWS * 4) + s0 * (ROWS * 16);
  v4d acc[kColTiles][RT];
  double vrow[kColTiles][REM > 0 ? REM : 1];
#pragma unroll
  for (int c = 0; c < kColTiles; ++c) {
#pragma unroll
    for (int r = 0; r < RT; ++r) acc[c][r] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int e = 0; e < REM; ++e) vrow[c][e] = 0.0;
  }
  for (long long st = s0; st < s1; ++st, tab += ROWS * 16) {
    const long long k0 = st * 16;
    v4d b[kColTiles];
#pragma unroll
    for (int c = 0; c < kColTiles; ++c)
      b[c] = valid[c] ? *reinterpret_cast<const v4d*>(rho[c] + k0) : v4d{0.0, 0.0, 0.0, 0.0};
    v4d a[RT];
#pragma unroll
    for (int r = 0; r < RT; ++r) a[r] = *reinterpret_cast<const v4d*>(tab + col * 4 + r * 64);
    // independent accumulators innermost, so consecutive MFMAs do not wait on each other
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int c = 0; c < kColTiles; ++c)
          acc[c][r] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[r][j], b[c][j], acc[c][r], 0, 0, 0);
#pragma unroll
    for (int e = 0; e < REM; ++e) {
      const v4d t = *reinterpret_cast<const v4d*>(tab + (16 * RT + e) * 4);
#pragma unroll
      for (int c = 0; c < kColTiles; ++c)
#pragma unroll
        for (int j = 0; j < 4; ++j) vrow[c][e] = fma(t[j], b[c][j], vrow[c][e]);
    }
  }
  // the vector-ALU rows: sum the four lane groups' points
#pragma unroll
  for (int c = 0; c < kColTiles; ++c)
#pragma unroll
    for (int e = 0; e < REM; ++e) {
      vrow[c][e] += __shfl_xor(vrow[c][e], 16, 64);
      vrow[c][e] += __shfl_xor(vrow[c][e], 32, 64);
    }
  // v_mfma_f64_16x16x4_f64 leaves D[i][j] in lane j + 16 (i mod 4), item i / 4
#pragma unroll
  for (int c = 0; c < kColTiles; ++c) {
    if (!valid[c]) continue;
    double* Q = Qp + ((long long)blockIdx.y * nb + (p[c] - pbeg)) * kMaxLM;
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int lm = 16 * r + kq + 4 * i;
        if (lm < kMaxLM) Q[lm] = acc[c][r][i];
      }
    if (kq == 0)
#pragma unroll
      for (int e = 0; e < REM; ++e) Q[16 * RT + e] = vrow[c][e];
  }
}

template <int RT, int kColTiles = kColTilesBF16>
__global__ __launch_bounds__(kTilePairs / kColTiles * 4) void k_moments_bf16(const ClassDev* __restrict__ cls_tab,
                                                              const int* __restrict__ class_cnt, int ncls,
                                                              long long pbeg, long long pend,
                                                              const int* __restrict__ n_eff,
                                                              const double* __restrict__ rho_ws, long long rstride,
                                                              const double* __restrict__ rho_scale,
                                                              double* __restrict__ Qp, long long nb) {
  int cls;
  long long tb, te;
  if (!locate_tile(class_cnt, ncls, pbeg, pend, n_eff, &cls, &tb, &te)) return;
  const ClassDev& C = cls_tab[cls];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, kq = lane >> 4;
  constexpr int ROWS = 16 * RT;
  long long p[kColTiles];
  bool valid[kColTiles];
  const double* rho[kColTiles];
  double inv_scale[kColTiles];
#pragma unroll
  for (int c = 0; c < kColTiles; ++c) {
    p[c] = tb + 16 * (kColTiles * wave + c) + col;
    valid[c] = p[c] < te;
    rho[c] = rho_ws + (valid[c] ? (p[c] - pbeg) * rstride : 0) + 8 * kq;
    inv_scale[c] = valid[c] ? 1.0 / rho_scale[p[c] - pbeg] : 0.0;   // exact: a power of two
  }
  long long s0, s1;
  chunk_range((C.n_pe + 31) / 32, &s0, &s1);
  const long long toff = (long long)col * 8 + (long long)kq * (ROWS * 8) + s0 * (ROWS * 32);
  const __bf16* th = reinterpret_cast<const __bf16*>(C.mom_hi) + toff;
  const __bf16* tl = reinterpret_cast<const __bf16*>(C.mom_lo) + toff;
  v4f acc[kColTiles][RT];
  double accd[kColTiles][RT][4];
#pragma unroll
  for (int c = 0; c < kColTiles; ++c)
#pragma unroll
    for (int r = 0; r < RT; ++r) {
      acc[c][r] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int i = 0; i < 4; ++i) accd[c][r][i] = 0.0;
    }
  int steps = 0;
  for (long long st = s0; st < s1; ++st, th += ROWS * 32, tl += ROWS * 32) {
    const long long k0 = st * 32;
    v8b bh[kColTiles], bl[kColTiles];
#pragma unroll
    for (int c = 0; c < kColTiles; ++c) {
      v4d x0 = v4d{0.0, 0.0, 0.0, 0.0}, x1 = v4d{0.0, 0.0, 0.0, 0.0};
      if (valid[c]) {
        x0 = *reinterpret_cast<const v4d*>(rho[c] + k0);
        x1 = *reinterpret_cast<const v4d*>(rho[c] + k0 + 4);
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const float x = (float)((j < 4 ? x0[j & 3] : x1[j & 3]) * inv_scale[c]);
        const __bf16 h = (__bf16)x;
        bh[c][j] = h;
        bl[c][j] = (__bf16)(x - (float)h);
      }
    }
#pragma unroll
    for (int r = 0; r < RT; ++r) {
      const v8b ah = *reinterpret_cast<const v8b*>(th + r * 128);
      const v8b al = *reinterpret_cast<const v8b*>(tl + r * 128);
#pragma unroll
      for (int c = 0; c < kColTiles; ++c) {
        acc[c][r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[c], acc[c][r], 0, 0, 0);
        acc[c][r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[c], acc[c][r], 0, 0, 0);
        acc[c][r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[c], acc[c][r], 0, 0, 0);
      }
    }
    if (++steps == kFoldSteps) {
      steps = 0;
#pragma unroll
      for (int c = 0; c < kColTiles; ++c)
#pragma unroll
        for (int r = 0; r < RT; ++r)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            accd[c][r][i] += (double)acc[c][r][i];
            acc[c][r][i] = 0.f;
          }
    }
  }
  // v_mfma_f32_16x16x32_bf16 leaves D[i][j] in lane j + 16 (i / 4), item i mod 4
#pragma unroll
  for (int c = 0; c < kColTiles; ++c) {
    if (!valid[c]) continue;
    double* Q = Qp + ((long long)blockIdx.y * nb + (p[c] - pbeg)) * kMaxLM;
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int lm = 16 * r + 4 * kq + i;
        if (lm < kMaxLM) Q[lm] = accd[c][r][i] + (double)acc[c][r][i];
      }
  }
}

// Q[b][lm] = dV N_lm scale_b sum_s Qp[s][b][lm], chunks added in order.
__global__ __launch_bounds__(256) void k_moment_sum(Geo g, const double* __restrict__ Qp, int splits, long long nb,
                                                    long long p0, const int* __restrict__ n_eff,
                                                    const double* __restrict__ rho_scale, double* __restrict__ Q_ws) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nb * g.n_lm) return;
  const long long b = t / g.n_lm;
  if (p0 + b >= *n_eff) return;
  const int lm = (int)(t - b * g.n_lm);
  double s = 0.0;
  for (int c = 0; c < splits; ++c) s += Qp[((long long)c * nb + b) * kMaxLM + lm];
  const double sc = rho_scale ? rho_scale[b] : 1.0;
  Q_ws[b * kMaxLM + lm] = g.dV * g.ylm_norm[lm] * sc * s;
}

// The far field at the Dirichlet points (Sec. I, eq. me) as a contraction on
// the matrix cores: V[pair][h] = sum_lm Q[pair][lm] T[lm][h], with T the
// class's boundary table.  A workgroup takes a 64-pair tile of one class (16
// pairs per wavefront, the A operand: Q of pair (lane mod 16) at
// lm = 4 s + lane / 16, kept in registers) and a chunk of the class's 16-point
// tiles of Dirichlet points (the B operand: one coalesced 64-value row of
// the table per k step).  v_mfma_f64_16x16x4_f64 leaves V[pair 4 u + lane / 16]
// [point lane mod 16] in item u.
template <int L>
__global__ __launch_bounds__(256) void k_boundary_f64(const ClassDev* __restrict__ cls_tab,
                                                      const int* __restrict__ class_cnt, int ncls, long long pbeg,
                                                      long long pend, const int* __restrict__ n_eff,
                                                      const double* __restrict__ Q_ws, double* __restrict__ halo_ws,
                                                      long long hstride) {
  constexpr int NLM = (L + 1) * (L + 1), S = (NLM + 3) / 4;
  int cls;
  long long tb, te;
  if (!locate_tile(class_cnt, ncls, pbeg, pend, n_eff, &cls, &tb, &te)) return;
  const ClassDev& C = cls_tab[cls];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, kq = lane >> 4;
  const long long pa = tb + 16 * wave + col;   // this lane's pair of the A operand
  double q[S];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int lm = 4 * s + kq;
    q[s] = (pa < te && lm < NLM) ? Q_ws[(pa - pbeg) * kMaxLM + lm] : 0.0;
  }
  long long t0, t1;
  chunk_range((C.n_halo + 15) / 16, &t0, &t1);
  for (long long t = t0; t < t1; ++t) {
    const double* tab = C.bnd_tab + t * (S * 64) + lane;
    v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < S; ++s) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(q[s], tab[s * 64], acc, 0, 0, 0);
    const long long h = 16 * t + col;
    if (h < C.n_halo) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const long long p = tb + 16 * wave + 4 * u + kq;
        if (p < te) halo_ws[(p - pbeg) * hstride + h] = acc[u];
      }
    }
  }
}

}  // namespace

void moment_layout(int l_max, bool mixed, int* rows, int* mfma_rows) {
  const int nlm = (l_max + 1) * (l_max + 1);
  const int padded = (nlm + 15) / 16 * 16;
  // FP64: up to 4 rows past the last full 16-row tile go to the vector ALU
  const int rem = nlm % 16;
  if (!mixed && nlm >= 16 && rem <= 4) {
    *rows = nlm;
    *mfma_rows = nlm - rem;
  } else {
    *rows = padded;
    *mfma_rows = padded;
  }
}

int moment_splits(long long nb, int ncls, long long max_pe) {
  const long long tiles = (nb + kTilePairs - 1) / kTilePairs + ncls - 1;
  long long s = (2048 + tiles - 1) / tiles;                              // about 2048 workgroups
  const long long max_chunks = std::max<long long>(1, max_pe / 2048);   // at least 2048 points per chunk
  s = std::min(s, std::min<long long>(max_chunks, 32));
  return (int)std::max<long long>(s, 1);
}

hipError_t launch_boundary(const Geo& g, const Batch& B, const int* class_cnt, int ncls, long long max_halo,
                           const double* Q_ws, double* halo_ws, long long hstride, hipStream_t s) {
  const long long nb = B.nb, pbeg = B.p0;
  if (nb <= 0 || max_halo <= 0) return hipSuccess;
  const long long tiles = (nb + kTilePairs - 1) / kTilePairs + ncls - 1;
  // chunks of Dirichlet-point tiles: about 2048 workgroups in all
  const long long htiles = (max_halo + 15) / 16;
  const long long splits = std::max<long long>(1, std::min<long long>(htiles, (2048 + tiles - 1) / tiles));
  const dim3 grid((unsigned)tiles, (unsigned)splits);
  const long long pend = pbeg + nb;
  switch (g.l_max) {
#define EXX_BND(LL)                                                                                              \
  case LL:                                                                                                       \
    k_boundary_f64<LL><<<grid, 256, 0, s>>>(B.cls, class_cnt, ncls, pbeg, pend, B.n_eff, Q_ws, halo_ws, hstride); \
    break;
    EXX_BND(0) EXX_BND(1) EXX_BND(2) EXX_BND(3) EXX_BND(4) EXX_BND(5) EXX_BND(6) EXX_BND(7) EXX_BND(8)
#undef EXX_BND
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_moments(const Geo& g, const Batch& B, const int* class_cnt, int ncls, bool mixed,
                          const double* rho_ws, long long rstride, const double* rho_scale, double* Qp, int splits,
                          double* Q_ws, hipStream_t s) {
  const long long nb = B.nb, pbeg = B.p0;
  const ClassDev* cls = B.cls;
  const int* n_eff = B.n_eff;
  if (nb <= 0) return hipSuccess;
  const long long tiles = (nb + kTilePairs - 1) / kTilePairs + ncls - 1;
  const dim3 grid((unsigned)tiles, (unsigned)splits);
  const long long pend = pbeg + nb;
  constexpr int tb16 = kTilePairs / kColTilesBF16 * 4, tb64 = kTilePairs / kColTilesF64 * 4;
  int rows = 0, mrows = 0;
  moment_layout(g.l_max, mixed, &rows, &mrows);
  if (mixed) {
    switch (rows / 16) {
#define EXX_MOM16(RT)                                                                                        \
  case RT:                                                                                                   \
    k_moments_bf16<RT><<<grid, tb16, 0, s>>>(cls, class_cnt, ncls, pbeg, pend, n_eff, rho_ws, rstride, rho_scale, Qp, \
                                             nb);                                                                  \
    break;
      EXX_MOM16(1) EXX_MOM16(2) EXX_MOM16(3) EXX_MOM16(4) EXX_MOM16(5) EXX_MOM16(6)
#undef EXX_MOM16
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (8 * (mrows / 16) + (rows - mrows)) {
#define EXX_MOM64(RT, REM)                                                                              \
  case 8 * RT + REM:                                                                                    \
    k_moments_f64<RT, REM><<<grid, tb64, 0, s>>>(cls, class_cnt, ncls, pbeg, pend, n_eff, rho_ws, rstride, Qp, \
                                                 nb);                                                            \
    break;
      EXX_MOM64(1, 0) EXX_MOM64(2, 0) EXX_MOM64(2, 4) EXX_MOM64(3, 0) EXX_MOM64(3, 1) EXX_MOM64(4, 0)
      EXX_MOM64(5, 0) EXX_MOM64(5, 1) EXX_MOM64(6, 0)
#undef EXX_MOM64
      default: return hipErrorInvalidValue;
    }
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const long long n = nb * g.n_lm;
  k_moment_sum<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(g, Qp, splits, nb, pbeg, n_eff,
                                                            mixed ? rho_scale : nullptr, Q_ws);
  return hipGetLastError();
}

}  // namespace exx
