// The Natan-Kronik (NK) Laplacian of a general cell (Sec. III C 1-2): pure
// second derivatives along the three lattice directions and along up to three
// auxiliary grid directions, eq. lapG_mod_nk3d, with the auxiliary directions
// chosen by Algorithm 1.  Plan-time host code.
//
// In grid-index coordinates every term is a second difference along an integer
// step u (eq. d2_1 with the step |sum_al u_al L_al / N_al|), so the operator is
// a list of arms (u, beta / step^2).
#include <algorithm>
#include <array>
#include <cmath>
#include <vector>

#include "exx_internal.h"

namespace exx {

namespace {

using Vec3 = std::array<double, 3>;

// Cartesian step of grid direction u: sum_al u_al L_al / N_al
Vec3 grid_step(const double h[9], const int N[3], const int u[3]) {
  Vec3 v{0.0, 0.0, 0.0};
  for (int al = 0; al < 3; ++al)
    for (int a = 0; a < 3; ++a) v[a] += u[al] * h[a + 3 * al] / N[al];
  return v;
}

double norm3(const Vec3& v) { return std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]); }

double det3(const double m[9]) {   // column-major
  return m[0] * (m[4] * m[8] - m[7] * m[5]) - m[3] * (m[1] * m[8] - m[7] * m[2]) + m[6] * (m[1] * m[5] - m[4] * m[2]);
}

struct Candidate {
  int u[3];
  double step;
};

// Relative tolerance of equal steps and of the parallel / singular tests, and
// the weight below which (relative to max F_al,al) an arm is dropped.
constexpr double kTie = 1e-10;
constexpr double kZeroWeight = 1e-12;
constexpr int kCandidates = 15;   // N_q
constexpr int kMaxShell = 8;

}  // namespace

std::string build_nk_arms(const double h[9], const int N[3], std::vector<NkArm>* arms) {
  arms->clear();
  const double dh = det3(h);
  if (!(std::fabs(dh) > 0.0)) return "singular cell";
  // h^-1 by cofactors: hinv[al + 3 a] = (h^-1)_{al a}
  double hinv[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      const int r1 = (c + 1) % 3, r2 = (c + 2) % 3, c1 = (r + 1) % 3, c2 = (r + 2) % 3;
      // (h^-1)_{r c} = cofactor_{c r} / det
      hinv[r + 3 * c] = (h[r1 + 3 * c1] * h[r2 + 3 * c2] - h[r1 + 3 * c2] * h[r2 + 3 * c1]) / dh;
    }
  double len[3], dxi[3];
  for (int al = 0; al < 3; ++al) {
    len[al] = std::sqrt(h[0 + 3 * al] * h[0 + 3 * al] + h[1 + 3 * al] * h[1 + 3 * al] + h[2 + 3 * al] * h[2 + 3 * al]);
    dxi[al] = len[al] / N[al];
  }
  // F = J^T J with J_{a al} = |L_al| (h^-1)_{al a} (eq. jacb, eq. lapG_)
  double F[3][3];
  for (int al = 0; al < 3; ++al)
    for (int be = 0; be < 3; ++be) {
      double s = 0.0;
      for (int a = 0; a < 3; ++a) s += (len[al] * hinv[al + 3 * a]) * (len[be] * hinv[be + 3 * a]);
      F[al][be] = s;
    }

  // Candidate auxiliary directions: non-axial grid directions (one of each
  // +-u pair, leading non-zero component positive), shell by shell
  // (max_al |u_al| = S; within a shell u_3, then u_2, then u_1 ascending).  The
  // sweep ends with the first shell S >= 2 whose every point is farther than
  // the longest step of the first shell, once N_q candidates are in hand.
  std::vector<Candidate> cand;
  double first_shell_max = 0.0;
  for (int S = 1; S <= kMaxShell; ++S) {
    double shell_min = INFINITY;
    for (int u3 = -S; u3 <= S; ++u3)
      for (int u2 = -S; u2 <= S; ++u2)
        for (int u1 = -S; u1 <= S; ++u1) {
          if (std::max(std::abs(u1), std::max(std::abs(u2), std::abs(u3))) != S) continue;
          const int u[3] = {u1, u2, u3};
          const double st = norm3(grid_step(h, N, u));
          shell_min = std::min(shell_min, st);
          if (S == 1) first_shell_max = std::max(first_shell_max, st);
          const int nonzero = (u1 != 0) + (u2 != 0) + (u3 != 0);
          const int lead = u1 != 0 ? u1 : (u2 != 0 ? u2 : u3);
          if (nonzero < 2 || lead < 0) continue;
          cand.push_back({{u1, u2, u3}, st});
        }
    if (S >= 2 && shell_min > first_shell_max && (int)cand.size() >= kCandidates) break;
  }
  // ascending step; equal steps keep the sweep order
  std::stable_sort(cand.begin(), cand.end(), [](const Candidate& x, const Candidate& y) {
    return x.step < y.step - kTie * std::max(x.step, y.step);
  });
  if ((int)cand.size() > kCandidates) cand.resize(kCandidates);

  // Algorithm 1.  Unit direction of u in the unit lattice vectors:
  // a_al = u_al dxi_al / step; M's column for it is (a1 a2, a1 a3, a2 a3).
  std::array<Vec3, 3> acc_a{};
  std::array<Vec3, 3> col{};
  std::array<int, 3> pick{};
  int p = 0;
  for (int q = 0; q < (int)cand.size() && p < 3; ++q) {
    Vec3 a;
    for (int al = 0; al < 3; ++al) a[al] = cand[q].u[al] * dxi[al] / cand[q].step;
    const Vec3 m{a[0] * a[1], a[0] * a[2], a[1] * a[2]};
    bool accept = true;
    if (p == 1) {
      const double dot = m[0] * col[0][0] + m[1] * col[0][1] + m[2] * col[0][2];
      accept = std::fabs(dot) < (1.0 - kTie) * norm3(m) * norm3(col[0]);   // not parallel (Cauchy-Schwarz)
    } else if (p == 2) {
      const double Mt[9] = {col[0][0], col[0][1], col[0][2], col[1][0], col[1][1], col[1][2], m[0], m[1], m[2]};
      accept = std::fabs(det3(Mt)) > kTie * norm3(col[0]) * norm3(col[1]) * norm3(m);   // M non-singular
    }
    if (!accept) continue;
    acc_a[p] = a;
    col[p] = m;
    pick[p] = q;
    ++p;
  }
  if (p < 3) return "Algorithm 1 found no three admissible auxiliary grid directions";

  // M b = (F12, F13, F23) (eq. nk3d_Mb_f), by elimination with partial pivoting
  double Mb[3][4];
  for (int r = 0; r < 3; ++r) {
    for (int k = 0; k < 3; ++k) Mb[r][k] = col[k][r];
  }
  Mb[0][3] = F[0][1];
  Mb[1][3] = F[0][2];
  Mb[2][3] = F[1][2];
  for (int c = 0; c < 3; ++c) {
    int piv = c;
    for (int r = c + 1; r < 3; ++r)
      if (std::fabs(Mb[r][c]) > std::fabs(Mb[piv][c])) piv = r;
    for (int k = 0; k < 4; ++k) std::swap(Mb[c][k], Mb[piv][k]);
    for (int r = c + 1; r < 3; ++r) {
      const double f = Mb[r][c] / Mb[c][c];
      for (int k = c; k < 4; ++k) Mb[r][k] -= f * Mb[c][k];
    }
  }
  double b[3];
  for (int r = 2; r >= 0; --r) {
    double s = Mb[r][3];
    for (int k = r + 1; k < 3; ++k) s -= Mb[r][k] * b[k];
    b[r] = s / Mb[r][r];
  }

  // eq. lapG_mod_nk3d
  const double fmax = std::max(F[0][0], std::max(F[1][1], F[2][2]));
  for (int al = 0; al < 3; ++al) {
    double beta = F[al][al];
    for (int k = 0; k < 3; ++k) beta -= b[k] * acc_a[k][al] * acc_a[k][al];
    if (std::fabs(beta) <= kZeroWeight * fmax) continue;
    NkArm A;
    A.u[0] = A.u[1] = A.u[2] = 0;
    A.u[al] = 1;
    A.beta = beta;
    A.step = dxi[al];
    arms->push_back(A);
  }
  for (int k = 0; k < 3; ++k) {
    if (std::fabs(b[k]) <= kZeroWeight * fmax) continue;
    NkArm A;
    for (int al = 0; al < 3; ++al) A.u[al] = cand[pick[k]].u[al];
    A.beta = b[k];
    A.step = cand[pick[k]].step;
    arms->push_back(A);
  }
  for (const NkArm& A : *arms)
    if (!(A.beta > 0.0)) return "the NK Laplacian of this cell has a non-positive weight (the CG needs a positive operator)";
  return std::string();
}

}  // namespace exx
