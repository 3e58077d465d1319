// Host-side construction of the proto-subdomain tables of one sphere class
// (Sec. III A Step II and Sec. III B 1): the PE sphere of radius R_PE about the
// grid origin, the Dirichlet points its stencil reaches, and the ME shell out
// to R_ME.  Each pair's subdomain is this set translated to the pair's grid
// centre (eq. l2g), so the tables are shared by every pair of the class.
//
// Layout of a PE vector ("column-major planes"): the (x,y) columns of the
// sphere are sorted by half-height zr descending (ties by angle about the z
// axis, then y, then x).  At plane z the columns with zr >= |z| are therefore
// a prefix of that order, and the plane is stored as that prefix, planes in
// ascending z.  A workgroup that assigns column c to a fixed thread then reads
// every plane with consecutive addresses from one per-plane base offset.
#include <algorithm>
#include <cmath>
#include <cstdio>

#include "exx_internal.h"
#include "harmonics.h"

namespace exx {

namespace {

inline double r2_of(const double L[3], const int N[3], int ox, int oy, int oz) {
  // same arithmetic as r = h (o / N) for a diagonal h
  double x = L[0] * ((double)ox / N[0]);
  double y = L[1] * ((double)oy / N[1]);
  double z = L[2] * ((double)oz / N[2]);
  return x * x + y * y + z * z;
}

}  // namespace

std::string build_class(const double L[3], const int N[3], double R_PE, double R_ME, int n, ClassHost* out) {
  ClassHost& C = *out;
  C = ClassHost();
  C.R_PE = R_PE;
  const double pe2 = R_PE * R_PE * (1.0 + kSlack);
  const double me2 = R_ME * R_ME * (1.0 + kSlack);
  int K[3];   // bounding half-widths of the ME sphere
  for (int a = 0; a < 3; ++a) {
    double d = L[a] / N[a];
    K[a] = (int)std::ceil(R_ME / d) + 1;
    C.Rg[a] = 0;
  }
  // PE extents
  for (int a = 0; a < 3; ++a) {
    int k = 0;
    while (true) {
      int o[3] = {0, 0, 0};
      o[a] = k + 1;
      if (r2_of(L, N, o[0], o[1], o[2]) <= pe2) ++k; else break;
    }
    C.Rg[a] = k;
  }
  for (int a = 0; a < 3; ++a) {
    if (2 * (C.Rg[a] + n) + 1 > 32000) return "sphere too large for 16-bit offsets";
  }
  C.Zmax = C.Rg[2];
  for (int a = 0; a < 3; ++a) C.Wm[a] = 2 * (C.Rg[a] + n) + 1;

  // columns, sorted by half-height descending (ties by angle about the z
  // axis, then y, then x): at plane z the columns that reach it are a prefix
  // of this order
  struct Col { int ox, oy, zr; double ang; };
  std::vector<Col> cols;
  for (int oy = -C.Rg[1]; oy <= C.Rg[1]; ++oy)
    for (int ox = -C.Rg[0]; ox <= C.Rg[0]; ++ox) {
      int zr = -1;
      for (int oz = 0; oz <= C.Rg[2]; ++oz)
        if (r2_of(L, N, ox, oy, oz) <= pe2) zr = oz; else break;
      if (zr >= 0) cols.push_back({ox, oy, zr, std::atan2((double)oy, (double)ox)});
    }
  std::stable_sort(cols.begin(), cols.end(), [](const Col& a, const Col& b) {
    if (a.zr != b.zr) return a.zr > b.zr;
    if (a.ang != b.ang) return a.ang < b.ang;
    if (a.oy != b.oy) return a.oy < b.oy;
    return a.ox < b.ox;
  });
  C.n_cols = (int)cols.size();
  C.cols.resize(cols.size());
  for (size_t c = 0; c < cols.size(); ++c) C.cols[c] = make_int4(cols[c].ox, cols[c].oy, cols[c].zr, 0);

  // planes: plane z holds the prefix of columns that reach it
  C.plane_start.assign(2 * C.Zmax + 2, 0);
  long long acc = 0;
  for (int z = -C.Zmax; z <= C.Zmax; ++z) {
    C.plane_start[z + C.Zmax] = (int)acc;
    int nz = 0;
    while (nz < C.n_cols && cols[nz].zr >= std::abs(z)) ++nz;
    acc += nz;
  }
  C.plane_start[2 * C.Zmax + 1] = (int)acc;
  C.n_pe = acc;
  if (acc > 0x7fffffffLL) return "PE sphere too large";

  // lookup maps
  const int W0 = C.Wm[0], W1 = C.Wm[1], W2 = C.Wm[2];
  const int cx = C.Rg[0] + n, cy = C.Rg[1] + n, cz = C.Rg[2] + n;
  C.zr_map.assign((size_t)W0 * W1, -1);
  C.col_map.assign((size_t)W0 * W1, -1);
  for (int c = 0; c < C.n_cols; ++c) {
    size_t m = (size_t)(cols[c].ox + cx) + (size_t)W0 * (cols[c].oy + cy);
    C.zr_map[m] = cols[c].zr;
    C.col_map[m] = c;
  }
  auto in_pe = [&](int ox, int oy, int oz) {
    if (std::abs(ox) > C.Rg[0] || std::abs(oy) > C.Rg[1]) return false;
    int zr = C.zr_map[(size_t)(ox + cx) + (size_t)W0 * (oy + cy)];
    return std::abs(oz) <= zr;
  };

  // Dirichlet (halo) points: outside PE, reached from a PE point by q <= n steps along an axis
  C.halo_map.assign((size_t)W0 * W1 * W2, -1);
  for (int oz = -cz; oz <= cz; ++oz)
    for (int oy = -cy; oy <= cy; ++oy)
      for (int ox = -cx; ox <= cx; ++ox) {
        if (in_pe(ox, oy, oz)) continue;
        bool reach = false;
        for (int q = 1; q <= n && !reach; ++q) {
          reach = in_pe(ox + q, oy, oz) || in_pe(ox - q, oy, oz) || in_pe(ox, oy + q, oz) ||
                  in_pe(ox, oy - q, oz) || in_pe(ox, oy, oz + q) || in_pe(ox, oy, oz - q);
        }
        if (!reach) continue;
        if (r2_of(L, N, ox, oy, oz) > me2) return "R_ME does not cover the stencil reach of the PE sphere";
        C.halo_map[(size_t)(ox + cx) + (size_t)W0 * ((oy + cy) + (size_t)W1 * (oz + cz))] = (int)C.halo_off.size();
        C.halo_off.push_back(make_short4((short)ox, (short)oy, (short)oz, 0));
      }
  C.n_halo = (long long)C.halo_off.size();

  // ME list: PE points in packed order, then the shell
  C.me_off.reserve((size_t)C.n_pe);
  for (int z = -C.Zmax; z <= C.Zmax; ++z) {
    const int nz = C.plane_start[z + C.Zmax + 1] - C.plane_start[z + C.Zmax];
    for (int c = 0; c < nz; ++c) C.me_off.push_back(make_short4((short)cols[c].ox, (short)cols[c].oy, (short)z, 0));
  }
  for (int oz = -K[2]; oz <= K[2]; ++oz)
    for (int oy = -K[1]; oy <= K[1]; ++oy)
      for (int ox = -K[0]; ox <= K[0]; ++ox) {
        if (r2_of(L, N, ox, oy, oz) > me2) continue;
        if (in_pe(ox, oy, oz)) continue;
        if (std::abs(ox) > 32000 || std::abs(oy) > 32000 || std::abs(oz) > 32000) return "ME sphere too large";
        C.me_off.push_back(make_short4((short)ox, (short)oy, (short)oz, 0));
      }
  C.n_me = (long long)C.me_off.size();
  return std::string();
}

void build_moment_table(const ClassHost& C, const double d[3], int l_max, int rows, int group,
                        std::vector<double>* out) {
  const long long kpad = (C.n_pe + 31) / 32 * 32;
  out->assign((size_t)(kpad * rows), 0.0);
  std::vector<double> ones(kMaxLM, 1.0), v(kMaxLM, 0.0);
  const int nlm = (l_max + 1) * (l_max + 1);
  for (long long k = 0; k < C.n_pe; ++k) {
    const short4 o = C.me_off[(size_t)k];
    solid_harmonics_host(l_max, o.x * d[0], o.y * d[1], o.z * d[2], ones.data(), v.data());
    double* dst = out->data() + (size_t)((k / group) * rows * group + (k % group));
    for (int lm = 0; lm < nlm; ++lm) dst[(size_t)lm * group] = v[lm];
  }
}

}  // namespace exx
