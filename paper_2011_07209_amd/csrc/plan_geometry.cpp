// Host-side construction of the proto-subdomain tables of one sphere class
// (Sec. III A Step II and Sec. III B 1): the PE sphere of radius R_PE about the
// grid origin, the Dirichlet points its stencil reaches, and the ME shell out
// to R_ME.  Each pair's subdomain is this set translated to the pair's grid
// centre (eq. l2g), so the tables are shared by every pair of the class.
//
// Layout of a PE vector ("column-major planes"): the (x,y) columns of the
// sphere are sorted by half-height zr descending; columns of equal half-height
// are ordered so that the LDS words a wavefront stages spread over the banks.
// At plane z the columns with zr >= |z| are therefore a prefix of that order,
// and the plane is stored as that prefix, planes in ascending z.  A workgroup that assigns column c to a fixed thread then reads
// every plane with consecutive addresses from one per-plane base offset.
//
// Quad layout (orthorhombic cells, one CG thread per run): the columns are
// grouped into runs of four x-adjacent columns of a row (x = 4k + s .. 4k + s
// + 3, s = 0 on even rows and 2 on odd rows), each run padded to its tallest
// column; the runs are sorted by that height (descending), and plane z holds
// the runs that reach it, four slots each.  A slot whose own column does not reach plane z, or lies
// outside the sphere, is dead (me_off.w = 1): it holds no point, stays zero in
// every vector, and every kernel skips it.
#include <algorithm>
#include <array>
#include <climits>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <functional>

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

// One column of a vector layout: (x, y) in the CG frame, the column's own
// half-height zr (-1 outside the sphere) and the half-height zq of the unit
// (column or run) that the plane prefixes are taken over.
struct LayCol {
  int ox, oy, zr, zq;
};

// Reorders items already sorted by half-height (descending) within each run
// of equal half-height, so that the LDS words they stage spread over the
// banks: each next item takes the word residue (of 16) used least so far by
// its aligned group of 16 threads, then the residue (of 32) used least by its
// group of 32 (ties: the given order).  word_of(item) is the item's LDS word
// index up to a constant; consecutive items go to consecutive threads.
template <typename Item, typename H, typename W>
void bank_order(std::vector<Item>& items, H height_of, W word_of) {
  auto res = [&](const Item& it) { return (word_of(it) % 32 + 32) % 32; };
  std::vector<Item> ordered;
  ordered.reserve(items.size());
  for (size_t g0 = 0; g0 < items.size();) {
    size_t g1 = g0;
    while (g1 < items.size() && height_of(items[g1]) == height_of(items[g0])) ++g1;
    std::vector<Item> pending(items.begin() + g0, items.begin() + g1);
    while (!pending.empty()) {
      int used16[16] = {0}, used32[32] = {0};
      for (size_t t = ordered.size() / 16 * 16; t < ordered.size(); ++t) ++used16[res(ordered[t]) % 16];
      for (size_t t = ordered.size() / 32 * 32; t < ordered.size(); ++t) ++used32[res(ordered[t])];
      auto key = [&](const Item& it) { return 64 * used16[res(it) % 16] + used32[res(it)]; };
      size_t best = 0;
      for (size_t i = 1; i < pending.size(); ++i)
        if (key(pending[i]) < key(pending[best])) best = i;
      ordered.push_back(pending[best]);
      pending.erase(pending.begin() + best);
    }
    g0 = g1;
  }
  items.swap(ordered);
}

// The quad layout's columns (see the file comment) for a cross-section whose
// column (x, y), |x| <= Rx, |y| <= Ry, has half-height zr_of(x, y), or -1
// outside the sphere: runs of four x-adjacent columns in their processing
// order, each column with its own half-height and its run's.
std::vector<LayCol> quad_runs(int Rx, int Ry, const std::function<int(int, int)>& zr_of) {
  std::vector<LayCol> out;
  auto floor4 = [](int v) { return v >= 0 ? v / 4 : -((-v + 3) / 4); };
  // Runs start at x = 4k + s with s = 0 on even rows and 2 on odd rows, so
  // that the runs' 8-byte halves in the LDS plane fall on every bank pair,
  // not only on every other one.
  auto shift = [](int oy) { return 2 * (oy & 1); };
  struct Run { int x0, oy, zq; };
  std::vector<Run> runs;
  for (int oy = -Ry; oy <= Ry; ++oy)
    for (int k = floor4(-Rx - shift(oy)); 4 * k + shift(oy) <= Rx; ++k) {
      const int x0 = 4 * k + shift(oy);
      int zq = -1;
      for (int j = 0; j < 4; ++j) zq = std::max(zq, zr_of(x0 + j, oy));
      if (zq >= 0) runs.push_back({x0, oy, zq});
    }
  // by run height (descending; plane z is a prefix), then within one height
  // over the banks of the 8-byte halves the runs stage (row order first)
  std::stable_sort(runs.begin(), runs.end(), [](const Run& a, const Run& b) {
    if (a.zq != b.zq) return a.zq > b.zq;
    if (a.oy != b.oy) return a.oy < b.oy;
    return a.x0 < b.x0;
  });
  bank_order(runs, [](const Run& r) { return r.zq; }, [](const Run& r) { return (r.x0 + kLdsWX * r.oy) / 2; });
  for (const Run& r : runs)
    for (int j = 0; j < 4; ++j) out.push_back({r.x0 + j, r.oy, zr_of(r.x0 + j, r.oy), r.zq});
  return out;
}

}  // namespace

std::string build_class(const double L[3], const int N[3], double R_PE, double R_ME, int n, bool quads,
                        ClassHost* out) {
  ClassHost& C = *out;
  C = ClassHost();
  C.R_PE = R_PE;
  C.quads = quads;
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
  const int Wr = 2 * C.Rg[0] + 1;
  std::vector<int> zr_at((size_t)Wr * (2 * C.Rg[1] + 1), -1);
  for (int oy = -C.Rg[1]; oy <= C.Rg[1]; ++oy)
    for (int ox = -C.Rg[0]; ox <= C.Rg[0]; ++ox) {
      int zr = -1;
      for (int oz = 0; oz <= C.Rg[2]; ++oz)
        if (r2_of(L, N, ox, oy, oz) <= pe2) zr = oz; else break;
      if (zr >= 0) cols.push_back({ox, oy, zr, std::atan2((double)oy, (double)ox)});
      zr_at[(size_t)(ox + C.Rg[0]) + (size_t)Wr * (oy + C.Rg[1])] = zr;
    }
  std::stable_sort(cols.begin(), cols.end(), [](const Col& a, const Col& b) {
    if (a.zr != b.zr) return a.zr > b.zr;
    if (a.ang != b.ang) return a.ang < b.ang;
    if (a.oy != b.oy) return a.oy < b.oy;
    return a.ox < b.ox;
  });

  // the layout's columns: (ox, oy, half-height zr of the column itself or -1
  // outside the sphere, half-height zq of the unit the prefix is taken over)
  std::vector<LayCol> lay;
  if (!quads) {
    bank_order(cols, [](const Col& c) { return c.zr; }, [](const Col& c) { return c.ox + kLdsWX * c.oy; });
    for (const Col& c : cols) lay.push_back({c.ox, c.oy, c.zr, c.zr});
  } else {
    auto zr_of = [&](int ox, int oy) {
      if (std::abs(ox) > C.Rg[0]) return -1;
      return zr_at[(size_t)(ox + C.Rg[0]) + (size_t)Wr * (oy + C.Rg[1])];
    };
    lay = quad_runs(C.Rg[0], C.Rg[1], zr_of);
  }
  C.n_cols = (int)lay.size();
  C.cols.resize(lay.size());
  for (size_t c = 0; c < lay.size(); ++c) C.cols[c] = make_int4(lay[c].ox, lay[c].oy, lay[c].zr, lay[c].zq);

  // planes: plane z holds the prefix of the layout that reaches it
  C.plane_start.assign(2 * C.Zmax + 2, 0);
  long long acc = 0;
  for (int z = -C.Zmax; z <= C.Zmax; ++z) {
    C.plane_start[z + C.Zmax] = (int)acc;
    int nz = 0;
    while (nz < C.n_cols && lay[nz].zq >= std::abs(z)) ++nz;
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
    if (lay[c].zr < 0) continue;
    size_t m = (size_t)(lay[c].ox + cx) + (size_t)W0 * (lay[c].oy + cy);
    C.zr_map[m] = lay[c].zr;
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
  C.n_real = 0;
  for (int z = -C.Zmax; z <= C.Zmax; ++z) {
    const int nz = C.plane_start[z + C.Zmax + 1] - C.plane_start[z + C.Zmax];
    for (int c = 0; c < nz; ++c) {
      if (lay[c].zr < std::abs(z)) {   // dead slot of a padded run
        C.me_off.push_back(make_short4(0, 0, 0, 1));
        continue;
      }
      C.me_off.push_back(make_short4((short)lay[c].ox, (short)lay[c].oy, (short)z, 0));
      ++C.n_real;
    }
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
  for (int a = 0; a < 3; ++a) C.Rc[a] = C.Rg[a];
  build_sweep_tables(n, &C);
  build_scan_order(&C);
  return std::string();
}

void build_scan_order(ClassHost* out) {
  ClassHost& C = *out;
  C.me_scan.clear();
  C.me_scan.reserve(C.me_off.size());
  for (size_t k = 0; k < C.me_off.size(); ++k)
    if (!C.me_off[k].w) C.me_scan.push_back((int)k);
  std::sort(C.me_scan.begin(), C.me_scan.end(), [&](int a, int b) {
    const short4 p = C.me_off[(size_t)a], q = C.me_off[(size_t)b];
    if (p.z != q.z) return p.z < q.z;
    if (p.y != q.y) return p.y < q.y;
    return p.x < q.x;
  });
  C.scan_off.resize(C.me_scan.size());
  for (size_t k = 0; k < C.me_scan.size(); ++k) C.scan_off[k] = C.me_off[(size_t)C.me_scan[k]];
}

void build_sweep_tables(int n, ClassHost* out) {
  ClassHost& C = *out;
  // the Dirichlet points grouped by plane (the plane-sweep E/sigma kernel
  // stages each plane's far-field values beside its PE values)
  const int Zh = C.Zmax + n;
  C.halo_zstart.assign(2 * Zh + 2, 0);
  for (const short4& o : C.halo_off) C.halo_zstart[o.z + Zh + 1]++;
  for (int z = 0; z < 2 * Zh + 1; ++z) C.halo_zstart[z + 1] += C.halo_zstart[z];
  std::vector<int> fill(C.halo_zstart.begin(), C.halo_zstart.end() - 1);
  C.halo_zidx.assign(C.halo_off.size(), 0);
  for (size_t h = 0; h < C.halo_off.size(); ++h) C.halo_zidx[fill[C.halo_off[h].z + Zh]++] = (int)h;
  // the real columns (without the quad layout's padding columns)
  C.fin_cols.clear();
  for (int c = 0; c < C.n_cols; ++c)
    if (C.cols[c].z >= 0) C.fin_cols.push_back(make_int4(c, C.cols[c].z, C.cols[c].x, C.cols[c].y));
  // the Dirichlet terms of each PE slot's right-hand side: every axis
  // neighbour within n steps that is not a PE point is a Dirichlet point
  C.rhs_ptr.assign((size_t)C.n_pe + 1, 0);
  C.rhs_ent.clear();
  const int W0 = C.Wm[0], W1 = C.Wm[1];
  const int cx = C.Rg[0] + n, cy = C.Rg[1] + n, cz = C.Rg[2] + n;
  auto in_pe = [&](int ox, int oy, int oz) {
    if (std::abs(ox) > C.Rg[0] || std::abs(oy) > C.Rg[1]) return false;
    const int zr = C.zr_map[(size_t)(ox + cx) + (size_t)W0 * (oy + cy)];
    return zr >= 0 && std::abs(oz) <= zr;
  };
  for (long long k = 0; k < C.n_pe; ++k) {
    const short4 o = C.me_off[(size_t)k];
    if (!o.w) {
      for (int al = 0; al < 3; ++al)
        for (int q = 1; q <= n; ++q)
          for (int sgn = -1; sgn <= 1; sgn += 2) {
            int u[3] = {o.x, o.y, o.z};
            u[al] += sgn * q;
            if (in_pe(u[0], u[1], u[2])) continue;
            const int h = C.halo_map[(size_t)(u[0] + cx) + (size_t)W0 * ((u[1] + cy) + (size_t)W1 * (u[2] + cz))];
            if (h >= 0) C.rhs_ent.push_back(make_int2(h, 4 * al + q));
          }
    }
    C.rhs_ptr[(size_t)k + 1] = (int)C.rhs_ent.size();
  }
}

void build_moment_table(const ClassHost& C, const double A[9], int l_max, int rows, int group,
                        std::vector<double>* out) {
  const long long kpad = (C.n_pe + 31) / 32 * 32;
  out->assign((size_t)(kpad * rows), 0.0);
  std::vector<double> ones(kMaxLM, 1.0), v(kMaxLM, 0.0);
  const int nlm = (l_max + 1) * (l_max + 1);
  for (long long k = 0; k < C.n_pe; ++k) {
    const short4 o = C.me_off[(size_t)k];
    if (o.w) continue;   // dead slot
    const double x = A[0] * o.x + A[3] * o.y + A[6] * o.z;
    const double y = A[1] * o.x + A[4] * o.y + A[7] * o.z;
    const double z = A[2] * o.x + A[5] * o.y + A[8] * o.z;
    solid_harmonics_host(l_max, x, y, z, ones.data(), v.data());
    double* dst = out->data() + (size_t)((k / group) * rows * group + (k % group));
    for (int lm = 0; lm < nlm; ++lm) dst[(size_t)lm * group] = v[lm];
  }
}

void build_boundary_table(const ClassHost& C, const double A[9], const double* norm, int l_max,
                          std::vector<double>* out) {
  const int nlm = (l_max + 1) * (l_max + 1), steps = (nlm + 3) / 4;
  const long long tiles = (C.n_halo + 15) / 16;
  out->assign((size_t)(tiles * steps * 64), 0.0);
  std::vector<double> v(kMaxLM, 0.0);
  for (long long h = 0; h < C.n_halo; ++h) {
    const short4 o = C.halo_off[(size_t)h];
    const double x = A[0] * o.x + A[3] * o.y + A[6] * o.z;
    const double y = A[1] * o.x + A[4] * o.y + A[7] * o.z;
    const double z = A[2] * o.x + A[5] * o.y + A[8] * o.z;
    solid_harmonics_host(l_max, x, y, z, norm, v.data());
    const double rinv = 1.0 / std::sqrt(x * x + y * y + z * z);
    double rp = rinv;   // |r|^-(2l + 1)
    for (int l = 0; l <= l_max; ++l) {
      for (int m = -l; m <= l; ++m) {
        const int lm = l * l + l + m;
        const double t = v[lm] * rp * (4.0 * 3.14159265358979323846 / (2.0 * l + 1.0));
        (*out)[(size_t)(((h / 16) * steps + lm / 4) * 64 + (lm % 4) * 16 + (h % 16))] = t;
      }
      rp *= rinv * rinv;
    }
  }
}

// ---------------------------------------------------------------------------
// General (non-orthogonal) cells, Sec. III B 1: the PE sphere is the set of
// grid offsets o with |r(o)| <= R_PE, r(o) = sum_al (o_al / N_al) L_al, an
// ellipsoid in index space whose columns along one grid axis need not be
// symmetric about 0.  The CG sweeps along a chosen grid axis ("z'", the other
// two in ascending order are x', y').  Each (x', y') column holds the interval
// [lo, hi] of z'; it is padded to the symmetric range [-zr, zr], zr = max(|lo|,
// |hi|), so that plane z' is again a prefix of the columns sorted by zr.  The
// padding slots ("dead", me_off.w = 1) hold no point: their density, right-hand
// side and solution are zero and every kernel skips them.

namespace {

inline double r2_general(const double h[9], const int N[3], int o0, int o1, int o2) {
  const double s0 = (double)o0 / N[0], s1 = (double)o1 / N[1], s2 = (double)o2 / N[2];
  const double x = h[0] * s0 + h[3] * s1 + h[6] * s2;
  const double y = h[1] * s0 + h[4] * s1 + h[7] * s2;
  const double z = h[2] * s0 + h[5] * s1 + h[8] * s2;
  return x * x + y * y + z * z;
}

// |o_al| <= N_al |row al of h^-1| R bounds the sphere of radius R
void sphere_box(const double h[9], const int N[3], double R, int K[3]) {
  const double d = h[0] * (h[4] * h[8] - h[7] * h[5]) - h[3] * (h[1] * h[8] - h[7] * h[2]) +
                   h[6] * (h[1] * h[5] - h[4] * h[2]);
  for (int al = 0; al < 3; ++al) {
    // row al of h^-1 = (cross product of the other two columns) / det
    const int b = (al + 1) % 3, c = (al + 2) % 3;
    const double cx = h[1 + 3 * b] * h[2 + 3 * c] - h[2 + 3 * b] * h[1 + 3 * c];
    const double cy = h[2 + 3 * b] * h[0 + 3 * c] - h[0 + 3 * b] * h[2 + 3 * c];
    const double cz = h[0 + 3 * b] * h[1 + 3 * c] - h[1 + 3 * b] * h[0 + 3 * c];
    K[al] = (int)std::ceil(R * N[al] * std::sqrt(cx * cx + cy * cy + cz * cz) / std::fabs(d)) + 1;
  }
}

}  // namespace

std::string build_class_general(const double h[9], const int N[3], int sweep, double R_PE, double R_ME, int n,
                                const std::vector<NkArm>& arms, bool all_dirs, bool quads, ClassHost* out) {
  ClassHost& C = *out;
  C = ClassHost();
  C.R_PE = R_PE;
  C.general = true;
  const double pe2 = R_PE * R_PE * (1.0 + kSlack);
  const double me2 = R_ME * R_ME * (1.0 + kSlack);
  int perm[3];
  {
    int k = 0;
    for (int a = 0; a < 3; ++a)
      if (a != sweep) perm[k++] = a;
    perm[2] = sweep;
  }
  for (int a = 0; a < 3; ++a) C.perm[a] = perm[a];

  // PE points (true-frame offsets)
  int KP[3];
  sphere_box(h, N, R_PE, KP);
  std::vector<std::array<int, 3>> pts;
  for (int a = 0; a < 3; ++a) C.Rg[a] = 0;
  for (int o2 = -KP[2]; o2 <= KP[2]; ++o2)
    for (int o1 = -KP[1]; o1 <= KP[1]; ++o1)
      for (int o0 = -KP[0]; o0 <= KP[0]; ++o0)
        if (r2_general(h, N, o0, o1, o2) <= pe2) {
          pts.push_back({o0, o1, o2});
          C.Rg[0] = std::max(C.Rg[0], std::abs(o0));
          C.Rg[1] = std::max(C.Rg[1], std::abs(o1));
          C.Rg[2] = std::max(C.Rg[2], std::abs(o2));
        }
  for (int a = 0; a < 3; ++a) {
    C.Rc[a] = C.Rg[perm[a]];
    if (2 * (C.Rg[a] + n) + 1 > 32000) return "sphere too large for 16-bit offsets";
  }
  C.n_real = (long long)pts.size();

  // columns of the CG frame: interval [lo, hi] of z' per (x', y')
  const int Wc0 = 2 * C.Rc[0] + 1, Wc1 = 2 * C.Rc[1] + 1;
  std::vector<int> lo((size_t)Wc0 * Wc1, INT32_MAX), hi((size_t)Wc0 * Wc1, INT32_MIN), cnt((size_t)Wc0 * Wc1, 0);
  for (const auto& p : pts) {
    const size_t m = (size_t)(p[perm[0]] + C.Rc[0]) + (size_t)Wc0 * (p[perm[1]] + C.Rc[1]);
    lo[m] = std::min(lo[m], p[perm[2]]);
    hi[m] = std::max(hi[m], p[perm[2]]);
    cnt[m]++;
  }
  struct Col { int x, y, lo, hi, zr; double ang; };
  std::vector<Col> cols;
  for (int y = -C.Rc[1]; y <= C.Rc[1]; ++y)
    for (int x = -C.Rc[0]; x <= C.Rc[0]; ++x) {
      const size_t m = (size_t)(x + C.Rc[0]) + (size_t)Wc0 * (y + C.Rc[1]);
      if (!cnt[m]) continue;
      if (cnt[m] != hi[m] - lo[m] + 1) return "PE sphere column is not an interval";
      cols.push_back({x, y, lo[m], hi[m], std::max(std::abs(lo[m]), std::abs(hi[m])),
                      std::atan2((double)y, (double)x)});
    }
  std::stable_sort(cols.begin(), cols.end(), [](const Col& a, const Col& b) {
    if (a.zr != b.zr) return a.zr > b.zr;
    if (a.ang != b.ang) return a.ang < b.ang;
    if (a.y != b.y) return a.y < b.y;
    return a.x < b.x;
  });
  C.Zmax = 0;
  for (const Col& c : cols) C.Zmax = std::max(C.Zmax, c.zr);
  // The quad layout takes symmetric columns only (lo = -hi: no padding, as
  // when the sweep axis is perpendicular to the other two lattice vectors);
  // its phantom columns (outside the sphere) hold the empty interval [1, 0].
  bool sym = true;
  for (const Col& c : cols) sym = sym && c.lo == -c.hi;
  C.quads = quads && sym;
  struct GCol { int x, y, lo, hi, zq; };
  std::vector<GCol> lay;
  if (!C.quads) {
    bank_order(cols, [](const Col& c) { return c.zr; }, [](const Col& c) { return c.x + kLdsWX * c.y; });
    for (const Col& c : cols) lay.push_back({c.x, c.y, c.lo, c.hi, c.zr});
    C.cols.resize(cols.size());
    for (size_t c = 0; c < cols.size(); ++c) C.cols[c] = make_int4(cols[c].x, cols[c].y, cols[c].lo, cols[c].hi);
  } else {
    auto zr_of = [&](int x, int y) {
      if (std::abs(x) > C.Rc[0] || std::abs(y) > C.Rc[1]) return -1;
      const size_t m = (size_t)(x + C.Rc[0]) + (size_t)Wc0 * (y + C.Rc[1]);
      return cnt[m] ? hi[m] : -1;
    };
    for (const LayCol& q : quad_runs(C.Rc[0], C.Rc[1], zr_of))
      lay.push_back({q.ox, q.oy, q.zr >= 0 ? -q.zr : 1, q.zr >= 0 ? q.zr : 0, q.zq});
    C.cols.resize(lay.size());
    for (size_t c = 0; c < lay.size(); ++c)
      C.cols[c] = make_int4(lay[c].x, lay[c].y, lay[c].lo <= lay[c].hi ? lay[c].hi : -1, lay[c].zq);
  }
  C.n_cols = (int)lay.size();

  // planes: prefix of the padded columns (or runs); slots outside [lo, hi] are dead
  C.plane_start.assign(2 * C.Zmax + 2, 0);
  long long acc = 0;
  for (int z = -C.Zmax; z <= C.Zmax; ++z) {
    C.plane_start[z + C.Zmax] = (int)acc;
    int nz = 0;
    while (nz < C.n_cols && lay[nz].zq >= std::abs(z)) ++nz;
    acc += nz;
  }
  C.plane_start[2 * C.Zmax + 1] = (int)acc;
  C.n_pe = acc;
  if (acc > 0x7fffffffLL) return "PE sphere too large";

  // true-frame lookup maps over the PE extents plus the stencil reach
  int umax = 1;
  for (const NkArm& A : arms)
    for (int a = 0; a < 3; ++a) umax = std::max(umax, std::abs(A.u[a]));
  for (int a = 0; a < 3; ++a) C.Wm[a] = 2 * (C.Rg[a] + n * umax) + 1;
  const int W0 = C.Wm[0], W1 = C.Wm[1], W2 = C.Wm[2];
  const int c0 = C.Rg[0] + n * umax, c1 = C.Rg[1] + n * umax, c2 = C.Rg[2] + n * umax;
  auto midx = [&](int o0, int o1, int o2) {
    return (size_t)(o0 + c0) + (size_t)W0 * ((size_t)(o1 + c1) + (size_t)W1 * (o2 + c2));
  };
  C.pe_map.assign((size_t)W0 * W1 * W2, -1);
  C.me_off.reserve((size_t)C.n_pe);
  for (int z = -C.Zmax; z <= C.Zmax; ++z) {
    const int nz = C.plane_start[z + C.Zmax + 1] - C.plane_start[z + C.Zmax];
    for (int c = 0; c < nz; ++c) {
      const GCol& cc = lay[c];
      if (z < cc.lo || z > cc.hi) {
        C.me_off.push_back(make_short4(0, 0, 0, 1));
        continue;
      }
      int o[3];
      o[perm[0]] = cc.x;
      o[perm[1]] = cc.y;
      o[perm[2]] = z;
      C.pe_map[midx(o[0], o[1], o[2])] = (int)C.me_off.size();
      C.me_off.push_back(make_short4((short)o[0], (short)o[1], (short)o[2], 0));
    }
  }
  auto in_pe = [&](int o0, int o1, int o2) {
    if (std::abs(o0) > C.Rg[0] || std::abs(o1) > C.Rg[1] || std::abs(o2) > C.Rg[2]) return false;
    return C.pe_map[midx(o0, o1, o2)] >= 0;
  };

  // Dirichlet points: outside PE, reached from a PE point by q <= n steps along
  // a Laplacian arm or along a lattice axis (the first-derivative stencil of
  // sigma)
  std::vector<std::array<int, 3>> dirs;
  if (all_dirs) {
    for (int u2 = -1; u2 <= 1; ++u2)
      for (int u1 = -1; u1 <= 1; ++u1)
        for (int u0 = -1; u0 <= 1; ++u0)
          if (u0 || u1 || u2) dirs.push_back({u0, u1, u2});
  } else {
    for (const NkArm& A : arms) dirs.push_back({A.u[0], A.u[1], A.u[2]});
    for (int a = 0; a < 3; ++a) {
      std::array<int, 3> e{0, 0, 0};
      e[a] = 1;
      if (std::find(dirs.begin(), dirs.end(), e) == dirs.end()) dirs.push_back(e);
    }
  }
  C.halo_map.assign((size_t)W0 * W1 * W2, -1);
  for (int o2 = -c2; o2 <= c2; ++o2)
    for (int o1 = -c1; o1 <= c1; ++o1)
      for (int o0 = -c0; o0 <= c0; ++o0) {
        if (in_pe(o0, o1, o2)) continue;
        bool reach = false;
        for (size_t d = 0; d < dirs.size() && !reach; ++d)
          for (int q = 1; q <= n && !reach; ++q)
            reach = in_pe(o0 + q * dirs[d][0], o1 + q * dirs[d][1], o2 + q * dirs[d][2]) ||
                    in_pe(o0 - q * dirs[d][0], o1 - q * dirs[d][1], o2 - q * dirs[d][2]);
        if (!reach) continue;
        if (r2_general(h, N, o0, o1, o2) > me2) return "R_ME does not cover the stencil reach of the PE sphere";
        C.halo_map[midx(o0, o1, o2)] = (int)C.halo_off.size();
        C.halo_off.push_back(make_short4((short)o0, (short)o1, (short)o2, 0));
      }
  C.n_halo = (long long)C.halo_off.size();
  // the plane-sweep E/sigma kernel's tables, in the CG frame: the Dirichlet
  // points by plane z' and the real columns (slot, lo, hi, x' | y' << 16)
  {
    auto comp = [](const short4& o, int a) { return a == 0 ? (int)o.x : a == 1 ? (int)o.y : (int)o.z; };
    const int Zh = C.Zmax + n;
    C.halo_zstart.assign(2 * Zh + 2, 0);
    for (const short4& o : C.halo_off) {
      const int zp = comp(o, perm[2]);
      if (std::abs(zp) > Zh) return "Dirichlet point beyond n planes of the PE sphere";
      C.halo_zstart[zp + Zh + 1]++;
    }
    for (int z = 0; z < 2 * Zh + 1; ++z) C.halo_zstart[z + 1] += C.halo_zstart[z];
    std::vector<int> fill(C.halo_zstart.begin(), C.halo_zstart.end() - 1);
    C.halo_zidx.assign(C.halo_off.size(), 0);
    for (size_t hh = 0; hh < C.halo_off.size(); ++hh) C.halo_zidx[fill[comp(C.halo_off[hh], perm[2]) + Zh]++] = (int)hh;
    C.fin_cols.clear();
    for (int c = 0; c < C.n_cols; ++c)
      if (lay[c].lo <= lay[c].hi)
        C.fin_cols.push_back(
            make_int4(c, lay[c].lo, lay[c].hi, (int)(((unsigned)lay[c].x & 0xffffu) | ((unsigned)lay[c].y << 16))));
  }
  // the PE slots whose arm sums can reach a Dirichlet point: within n steps
  // of a non-PE point along one of those directions
  C.rhs_edge.assign((size_t)((C.n_pe + 31) / 32), 0u);
  for (long long k = 0; k < C.n_pe; ++k) {
    const short4 o = C.me_off[(size_t)k];
    if (o.w) continue;
    bool edge = false;
    for (size_t d = 0; d < dirs.size() && !edge; ++d)
      for (int q = 1; q <= n && !edge; ++q)
        edge = !in_pe(o.x + q * dirs[d][0], o.y + q * dirs[d][1], o.z + q * dirs[d][2]) ||
               !in_pe(o.x - q * dirs[d][0], o.y - q * dirs[d][1], o.z - q * dirs[d][2]);
    if (edge) C.rhs_edge[(size_t)(k >> 5)] |= 1u << (k & 31);
  }

  // ME shell after the PE slots
  int KM[3];
  sphere_box(h, N, R_ME, KM);
  for (int o2 = -KM[2]; o2 <= KM[2]; ++o2)
    for (int o1 = -KM[1]; o1 <= KM[1]; ++o1)
      for (int o0 = -KM[0]; o0 <= KM[0]; ++o0) {
        if (r2_general(h, N, o0, o1, o2) > me2) continue;
        if (r2_general(h, N, o0, o1, o2) <= pe2) continue;
        if (std::abs(o0) > 32000 || std::abs(o1) > 32000 || std::abs(o2) > 32000) return "ME sphere too large";
        C.me_off.push_back(make_short4((short)o0, (short)o1, (short)o2, 0));
      }
  C.n_me = (long long)C.me_off.size();
  build_scan_order(&C);
  return std::string();
}

}  // namespace exx
