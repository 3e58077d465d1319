// Drives the plan-time host code (sphere-class tables of orthorhombic and
// general cells in both layouts, the NK arms, the moment and boundary tables)
// for a build with AddressSanitizer and UndefinedBehaviorSanitizer, and checks the
// invariants every table entry must satisfy on the way: indices in range,
// planes stored as prefixes, each PE point once, the D scatter's raster
// order.  Exits non-zero on a failed check (the sanitizers abort on their own
// findings).
#include <cmath>
#include <cstdio>
#include <set>
#include <string>
#include <vector>

#include "exx_internal.h"

namespace {

int g_fail = 0;

void check(bool ok, const char* what, const char* name) {
  if (!ok) {
    std::printf("  FAIL %s: %s\n", name, what);
    ++g_fail;
  }
}

// Every PE slot of a class: plane_start is non-decreasing, every halo_map and
// pe_map entry indexes its table, every column holds its plane prefix.
void check_class(const exx::ClassHost& C, int n, const char* name) {
  check(C.n_pe > 0 && C.n_halo > 0 && C.n_me > 0, "non-empty sets", name);
  check((int)C.plane_start.size() == 2 * C.Zmax + 2, "plane_start size", name);
  for (size_t z = 1; z < C.plane_start.size(); ++z) check(C.plane_start[z] >= C.plane_start[z - 1], "plane order", name);
  check(C.plane_start.back() == C.n_pe, "plane_start ends at n_pe", name);
  for (int h : C.halo_map) check(h >= -1 && h < C.n_halo, "halo_map range", name);
  for (int p : C.pe_map) check(p >= -1 && p < C.n_pe, "pe_map range", name);
  check((long long)C.halo_off.size() == C.n_halo, "halo_off size", name);
  check((long long)C.me_off.size() >= C.n_pe, "me_off holds the PE slots", name);
  std::set<long long> seen;
  long long real = 0;
  for (long long k = 0; k < C.n_pe; ++k) {
    const short4 o = C.me_off[k];
    if (o.w) continue;   // dead slot
    ++real;
    check(seen.insert(((long long)o.x * 4096 + o.y) * 4096 + o.z).second, "PE point stored once", name);
  }
  check(real == C.n_real || C.n_real == 0, "real point count", name);
  // the D scatter's order: every live ME entry once, in raster order (z, y, x)
  long long live = 0;
  for (const short4& o : C.me_off) live += o.w ? 0 : 1;
  check((long long)C.me_scan.size() == live, "scan order holds every live ME entry", name);
  check(C.scan_off.size() == C.me_scan.size(), "scan offsets beside the scan order", name);
  for (size_t k = 0; k < C.scan_off.size() && k < C.me_scan.size(); ++k) {
    const short4 a = C.scan_off[k], b = C.me_off[(size_t)C.me_scan[k]];
    check(a.x == b.x && a.y == b.y && a.z == b.z, "scan offset of its entry", name);
  }
  std::set<int> scanned;
  for (size_t k = 0; k < C.me_scan.size(); ++k) {
    const int e = C.me_scan[k];
    check(e >= 0 && e < (int)C.me_off.size() && !C.me_off[e].w, "scan entry is a live ME entry", name);
    check(scanned.insert(e).second, "scan entry once", name);
    if (k > 0) {
      const short4 p = C.me_off[C.me_scan[k - 1]], q = C.me_off[e];
      check(p.z < q.z || (p.z == q.z && (p.y < q.y || (p.y == q.y && p.x < q.x))), "scan in raster order", name);
    }
  }
  if (!C.general) {
    check((int)C.halo_zstart.size() == 2 * (C.Zmax + n) + 2, "halo_zstart size", name);
    check((long long)C.halo_zidx.size() == C.n_halo, "halo_zidx holds every Dirichlet point", name);
    for (int h : C.halo_zidx) check(h >= 0 && h < C.n_halo, "halo_zidx range", name);
    check((long long)C.rhs_ptr.size() == C.n_pe + 1, "rhs_ptr size", name);
    for (const int2& e : C.rhs_ent) check(e.x >= 0 && e.x < C.n_halo && e.y >= 0 && e.y < 4 * 3, "rhs entry", name);
    for (const int4& c : C.fin_cols) check(c.x >= 0 && c.y >= 0 && c.y <= C.Zmax, "finalize column", name);
  } else {
    check(C.rhs_ptr.empty(), "no right-hand side table for general cells", name);
    check((long long)C.rhs_edge.size() == (C.n_pe + 31) / 32, "rhs_edge size", name);
    check((int)C.halo_zstart.size() == 2 * (C.Zmax + n) + 2, "halo_zstart size", name);
    check((long long)C.halo_zidx.size() == C.n_halo, "halo_zidx holds every Dirichlet point", name);
    for (int h : C.halo_zidx) check(h >= 0 && h < C.n_halo, "halo_zidx range", name);
    // the real columns: every PE point once across [lo, hi] of its column
    long long pts = 0;
    for (const int4& c : C.fin_cols) {
      check(c.x >= 0 && c.x < C.n_cols && c.y <= c.z && c.y >= -C.Zmax && c.z <= C.Zmax, "general finalize column",
            name);
      pts += c.z - c.y + 1;
    }
    check(pts == C.n_real, "finalize columns cover the PE points", name);
  }
}

// General cells: every PE slot with a Dirichlet point among its arm
// neighbours (q <= n steps along an NK arm) is marked in rhs_edge, so the
// right-hand side kernel, which skips unmarked slots, misses no coupling.
void check_edges(const exx::ClassHost& C, const std::vector<exx::NkArm>& arms, int n, const char* name) {
  const int c0 = (C.Wm[0] - 1) / 2, c1 = (C.Wm[1] - 1) / 2, c2 = (C.Wm[2] - 1) / 2;
  auto halo_at = [&](int o0, int o1, int o2) {
    if (std::abs(o0) > c0 || std::abs(o1) > c1 || std::abs(o2) > c2) return false;
    return C.halo_map[(size_t)(o0 + c0) + (size_t)C.Wm[0] * ((size_t)(o1 + c1) + (size_t)C.Wm[1] * (o2 + c2))] >= 0;
  };
  long long marked = 0, needed = 0;
  for (long long k = 0; k < C.n_pe; ++k) {
    const short4 o = C.me_off[(size_t)k];
    if (o.w) continue;
    bool need = false;
    for (const exx::NkArm& A : arms)
      for (int q = 1; q <= n; ++q)
        for (int s = -1; s <= 1; s += 2)
          need = need || halo_at(o.x + s * q * A.u[0], o.y + s * q * A.u[1], o.z + s * q * A.u[2]);
    const bool bit = (C.rhs_edge[(size_t)(k >> 5)] >> (k & 31)) & 1u;
    marked += bit;
    needed += need;
    if (need) check(bit, "slot with a Dirichlet arm neighbour is marked", name);
  }
  check(marked < C.n_real, "interior slots unmarked", name);
  std::printf("  %s: %lld of %lld PE points marked (%lld need it)\n", name, marked, C.n_real, needed);
}

void boundary(const exx::ClassHost& C, const double A[9], const char* name) {
  std::vector<double> norm(exx::kMaxLM, 1.0), tab;
  for (int l_max : {0, 6, 8}) {
    exx::build_boundary_table(C, A, norm.data(), l_max, &tab);
    const long long steps = ((l_max + 1) * (l_max + 1) + 3) / 4;
    check((long long)tab.size() == (C.n_halo + 15) / 16 * steps * 64, "boundary table size", name);
    for (double v : tab) check(std::isfinite(v), "boundary table finite", name);
  }
}

void moments(const exx::ClassHost& C, const double A[9], const char* name) {
  for (int group : {4, 8}) {
    std::vector<double> tab;
    const int l_max = 6, rows = 52;
    exx::build_moment_table(C, A, l_max, rows, group, &tab);
    const long long npad = (C.n_pe + 31) / 32 * 32;
    check((long long)tab.size() == npad * rows, "moment table size", name);
    for (double v : tab) check(std::isfinite(v), "moment table finite", name);
  }
}

}  // namespace

int main() {
  // orthorhombic: both layouts, every stencil half-width
  const double L[3] = {10.0, 11.0, 12.5};
  const int N[3] = {40, 44, 48};
  const double A[9] = {L[0] / N[0], 0, 0, 0, L[1] / N[1], 0, 0, 0, L[2] / N[2]};
  for (int n = 1; n <= 3; ++n)
    for (bool quads : {false, true})
      for (double R : {1.2, 2.9}) {
        exx::ClassHost C;
        char name[96];
        std::snprintf(name, sizeof name, "orthorhombic n=%d quads=%d R_PE=%.1f", n, (int)quads, R);
        const std::string e = exx::build_class(L, N, R, R + n * 0.35 + 0.5, n, quads, &C);
        std::printf("%s: %s n_pe %lld halo %lld me %lld cols %d\n", name, e.empty() ? "ok" : e.c_str(), C.n_pe,
                    C.n_halo, C.n_me, C.n_cols);
        check(e.empty(), "build_class", name);
        if (!e.empty()) continue;
        check_class(C, n, name);
        moments(C, A, name);
        boundary(C, A, name);
      }

  // triclinic: NK arms, then the general tables along each sweep axis
  const double h[9] = {10.0, 0.0, 0.0, 1.6, 10.4, 0.0, 1.1, -1.3, 11.0};
  const int Ng[3] = {40, 42, 44};
  std::vector<exx::NkArm> arms;
  std::string e = exx::build_nk_arms(h, Ng, &arms);
  std::printf("nk arms: %s %zu\n", e.empty() ? "ok" : e.c_str(), arms.size());
  check(e.empty() && arms.size() >= 3 && arms.size() <= 6, "build_nk_arms", "triclinic");
  double Ag[9];
  for (int a = 0; a < 3; ++a)
    for (int al = 0; al < 3; ++al) Ag[a + 3 * al] = h[a + 3 * al] / Ng[al];
  for (int sweep = 0; sweep < 3; ++sweep)
    for (bool all_dirs : {false, true})
      for (bool quads : {false, true}) {
        exx::ClassHost C;
        char name[96];
        std::snprintf(name, sizeof name, "triclinic sweep=%d all_dirs=%d quads=%d", sweep, (int)all_dirs, (int)quads);
        e = exx::build_class_general(h, Ng, sweep, 2.4, 4.6, 3, arms, all_dirs, quads, &C);
        std::printf("%s: %s n_pe %lld halo %lld me %lld cols %d quads %d\n", name, e.empty() ? "ok" : e.c_str(), C.n_pe,
                    C.n_halo, C.n_me, C.n_cols, (int)C.quads);
        check(e.empty(), "build_class_general", name);
        if (!e.empty()) continue;
        check_class(C, 3, name);
        check_edges(C, arms, 3, name);
        moments(C, Ag, name);
        boundary(C, Ag, name);
      }

  // a monoclinic cell whose columns are symmetric about the sweep plane
  const double hm[9] = {10.0, 0.0, 0.0, 2.0, 10.0, 0.0, 0.0, 0.0, 10.0};
  arms.clear();
  e = exx::build_nk_arms(hm, Ng, &arms);
  check(e.empty(), "build_nk_arms", "monoclinic");
  {
    exx::ClassHost C;
    e = exx::build_class_general(hm, Ng, 2, 2.4, 4.6, 3, arms, false, true, &C);
    std::printf("monoclinic quads: %s n_pe %lld quads %d\n", e.empty() ? "ok" : e.c_str(), C.n_pe, (int)C.quads);
    check(e.empty(), "build_class_general", "monoclinic");
    if (e.empty()) {
      check_class(C, 3, "monoclinic");
      check_edges(C, arms, 3, "monoclinic");
    }
  }
  std::printf("failures %d\n", g_fail);
  return g_fail ? 1 : 0;
}
