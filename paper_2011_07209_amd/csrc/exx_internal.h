// Internal types of the gfx950 EXX library (host and device).
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <cstdint>
#include <string>
#include <vector>

#include "exx.h"

namespace exx {

constexpr int kMaxL = 8;                       // l_max limit of the multipole expansion
constexpr int kMaxLM = (kMaxL + 1) * (kMaxL + 1);
constexpr int kMaxClasses = 16;
// values k_reduce writes per evaluation (see launch_reduce)
constexpr int kStatsLen = 13;
constexpr double kSlack = 1e-12;               // relative slack of sphere membership on |r|^2
// Row stride of the LDS planes of the CG, a compile-time constant so that the
// y-neighbour reads use immediate offsets.  It bounds the sphere:
// 2 (R_PE / spacing + n) + 1 <= 88.
constexpr int kLdsWX = 88;

// Geometry and stencil constants, passed by value to every kernel.
struct Geo {
  double h[9];        // cell tensor, column-major: h[a + 3*al] = (L_al)_a
  double L[3];        // orthorhombic edge lengths
  double hinv[9];     // h^-1, column-major: hinv[al + 3*a] = (h^-1)_{al a}
  double J[9];        // Jacobian J[a + 3*al] = |L_al| (h^-1)_{al a}
  double d[3];        // grid spacing |L_al| / N_al
  double inv_d2[3];   // 1 / d^2
  double inv_d[3];    // 1 / d
  double dV;          // cell volume / number of grid points
  int N[3];
  long long ngrid;
  double w2[4];       // second-derivative weights w_0..w_n
  double w1[4];       // first-derivative weights (w_q, q >= 1)
  int n;              // stencil half-width
  int l_max;
  int n_lm;
  int lds_cx, lds_cy, lds_wx, lds_wy;   // LDS plane origin and size (lds_wx = kLdsWX)
  double ylm_norm[kMaxLM];              // N_l0 for m == 0, sqrt(2) N_l|m| otherwise
  // General (non-orthogonal) cells.  gen == 0: orthorhombic, offsets are
  // r = (o_x d_x, o_y d_y, o_z d_z) and the Laplacian is the axis stencil.
  int gen;
  double A[9];          // r = A o, A[a + 3 al] = h_{a al} / N_al
  int perm[3];          // CG frame: (x', y', z') = (o[perm[0]], o[perm[1]], o[perm[2]])
  int n_arms;           // NK Laplacian: sum over arms of coef * eq. d2_1 along u
  int arm_u[6][3];
  double arm_coef[6];   // beta / step^2
};

// One arm of the NK Laplacian (Sec. III C 2, eq. lapG_mod_nk3d): the pure
// second derivative along the grid direction u (integer steps along L_1, L_2,
// L_3) of Cartesian length step, with weight beta.
struct NkArm {
  int u[3];
  double beta;
  double step;
};

// A sphere class (one PE radius).  All arrays live in one device block.
struct ClassDev {
  double R_PE;
  int n_cols;         // columns (x,y) of the PE sphere
  int Zmax;           // largest |z| offset in PE
  int Rg[3];          // largest |offset| per axis in PE
  int Wm[3];          // lookup-map dims: 2 (Rg + n) + 1
  long long n_pe, n_halo, n_me;
  // n_pe counts the slots of a PE vector; general cells pad their columns with
  // dead slots (me_off.w = 1), n_real counts the PE points proper
  long long n_real;
  int Rc[3];                 // extents in the CG frame (= Rg for orthorhombic cells)
  const int* pe_map;         // general cells: [Wm2][Wm1][Wm0] (true frame) -> slot, or -1
  const int4* cols;          // [n_cols] (ox, oy, zr, 0), sorted by zr descending; general cells:
                             // (x', y', lo, hi) in the CG frame, sorted by max(|lo|, |hi|)
  const int* plane_start;    // [2 Zmax + 2] packed index of the first point of plane z (index z + Zmax)
  const short4* halo_off;    // [n_halo] offsets of the Dirichlet points reached by the stencil
  const short4* me_off;      // [n_me] PE points in packed order, then the ME shell
  const int* halo_map;       // [Wm2][Wm1][Wm0] -> halo index or -1
  const int* col_map;        // [Wm1][Wm0] -> column index or -1
  const int* zr_map;         // [Wm1][Wm0] -> column half-height or -1
  // the Dirichlet points plane by plane (z in the CG frame), halo_zidx[halo_zstart[z + Zh] ..
  // halo_zstart[z + Zh + 1]) the halo indices of plane z, Zh = Zmax + n
  const int* halo_zidx;
  const int* halo_zstart;
  int Zh;
  // the sphere's columns without the quad layout's padding columns, n_fin of them: (slot in
  // the layout, half-height, x, y) each for orthorhombic cells, (slot, lo, hi, x | y << 16) in
  // the CG frame for general cells
  const int4* fin_cols;
  int n_fin;
  // orthorhombic cells: the Dirichlet terms of the right-hand side as a CSR
  // table over the PE slots: slot k takes w_q / d_al^2 v_h for the entries
  // rhs_ent[rhs_ptr[k] .. rhs_ptr[k + 1]) = (halo index h, 4 al + q)
  const int* rhs_ptr;
  const int2* rhs_ent;
  // general cells: bit k (word k / 32) set for the PE slots within n steps of a
  // non-PE point along a direction the tables hold Dirichlet points for (the
  // only slots whose right-hand side takes Dirichlet terms)
  const unsigned* rhs_edge;
  // the live entries of me_off (no dead slots) in grid raster order of their
  // offsets (z, then y, then x), n_scan of them: the D scatter's order; and
  // their offsets in that order (so that a point's offset and entry are two
  // independent loads)
  const int* me_scan;
  const short4* scan_off;
  long long n_scan;
  // moment table: unnormalised solid harmonics P_lm of the PE offsets over
  // mom_rows rows and n_pe rounded up to 32 points (zeros beyond); FP64 in
  // layout [k/4][row][4] for FP64 plans, split BF16 (hi, lo) in layout
  // [k/8][row][8] for mixed plans
  int mom_rows;
  // boundary table: the far field's kernel at the Dirichlet points,
  // 4 pi / (2l + 1) R_lm(rbar_h) / |rbar_h|^(2l + 1), FP64 in the operand order of
  // the matrix cores: [h / 16][lm / 4][lm mod 4][h mod 16] over (l_max + 1)^2 rows
  // rounded up to 4 and n_halo rounded up to 16 (zeros beyond)
  const double* bnd_tab;
  const double* mom_f64;
  const unsigned short* mom_hi;
  const unsigned short* mom_lo;
};

struct PairDev {
  int i, j;
  int c[3];
  int cls;
};

struct ClassHost {
  double R_PE = 0;
  int n_cols = 0, Zmax = 0;
  int Rg[3] = {0, 0, 0};
  int Wm[3] = {0, 0, 0};
  int Rc[3] = {0, 0, 0};
  bool general = false;
  bool quads = false;         // orthorhombic quad layout (runs of four columns per CG thread)
  int perm[3] = {0, 1, 2};
  std::vector<int4> cols;
  std::vector<int> plane_start;
  std::vector<short4> halo_off;
  std::vector<short4> me_off;
  std::vector<int> halo_map, col_map, zr_map, pe_map;
  std::vector<int> halo_zidx, halo_zstart;   // the Dirichlet points by plane (CG frame)
  std::vector<int4> fin_cols;                // the real columns (slot, zr, x, y) or (slot, lo, hi, x | y << 16)
  std::vector<int> rhs_ptr;                  // orthorhombic: CSR of the Dirichlet terms per PE slot
  std::vector<int2> rhs_ent;
  std::vector<unsigned> rhs_edge;            // general: PE slots near the Dirichlet points (bits)
  std::vector<int> me_scan;                  // the live ME entries in grid raster order (z, y, x)
  std::vector<short4> scan_off;              // their offsets, in that order
  long long n_pe = 0, n_halo = 0, n_me = 0, n_real = 0;
};

// Builds the tables of one class of an orthorhombic cell; returns an empty
// string or an error message.
// quads: columns grouped into runs of four x-adjacent columns of one row
// (starting at x = 4k on even rows, 4k + 2 on odd ones), each run padded to
// its tallest column with dead slots, the runs sorted by that height.
std::string build_class(const double L[3], const int N[3], double R_PE, double R_ME, int n, bool quads,
                        ClassHost* out);
// The tables of an orthorhombic class's plane-sweep kernels (build_class
// calls it): the Dirichlet points by plane (halo_zidx, halo_zstart), the real
// columns (fin_cols) and the CSR of each PE slot's Dirichlet couplings
// (rhs_ptr, rhs_ent: halo index and 4 * axis + step).
void build_sweep_tables(int n, ClassHost* out);
// The D scatter's order of a class (both builders call it): me_scan.
void build_scan_order(ClassHost* out);
// The same for a general cell h with the NK arms of its Laplacian; the CG
// sweeps along grid axis `sweep`.
// all_dirs: Dirichlet points along every nearest-neighbour direction (for
// cells that may change later), else along the arms and the lattice axes.
// quads: the quad layout when every column is symmetric about the sweep
// plane z' = 0 (else, and without quads, padded single columns; ClassHost.quads
// tells which).
std::string build_class_general(const double h[9], const int N[3], int sweep, double R_PE, double R_ME, int n,
                                const std::vector<NkArm>& arms, bool all_dirs, bool quads, ClassHost* out);
// The NK Laplacian of cell h on grid N (Algorithm 1 and eq. lapG_mod_nk3d).
std::string build_nk_arms(const double h[9], const int N[3], std::vector<NkArm>* arms);
// Unnormalised solid harmonics P_lm(A o) of the class's PE points, laid out
// [k/G][row][G] (G = group, 4 or 8) with rows >= (l_max + 1)^2 and n_pe
// rounded up to 32, zeros in the padding and at dead slots.
void build_moment_table(const ClassHost& C, const double A[9], int l_max, int rows, int group,
                        std::vector<double>* out);
// The boundary table of a class (see ClassDev::bnd_tab) for the grid map A
// (rbar = A o) and the harmonic normalisation norm.
void build_boundary_table(const ClassHost& C, const double A[9], const double* norm, int l_max,
                          std::vector<double>* out);

// The device workspace of an evaluation that the plan holds pointers to: the
// plan's own allocations, or, for exx_eval_noalloc, pieces of the library's
// static scratch array (the two are swapped in and out as a whole).
struct EvalWork {
  long long pair_cap = 0;
  PairDev* pairs = nullptr;
  int* order = nullptr;
  int* pair_count = nullptr;
  int orb_cap = 0;
  int* n_eff = nullptr;
  int* d_slot = nullptr;
  double* pE = nullptr;
  double* pS = nullptr;
  int* pIt = nullptr;
  double* pRes = nullptr;
  int* pUpd = nullptr;
  int* pSav = nullptr;
  int* pExit = nullptr;
  long long batch_cap = 0;
  double* rho_ws = nullptr;
  double* bx_ws = nullptr;
  double* halo_ws = nullptr;
  double* Q_ws = nullptr;
  double* rho_scale = nullptr;
  double* Qp_ws = nullptr;
  long long qp_rows = 0;
  int n_slots = 0;
  void* slot_ws = nullptr;
};

}  // namespace exx

struct exx_plan_s {
  exx_options opt;
  double h[9];        // the current cell
  double h0[9];       // the cell the proto-subdomain tables were built for
  double cell_strain = 0.0;   // max |h h0^-1 - I|
  int reassemblies = 0;
  bool all_dirs = false;      // Dirichlet points along every nearest-neighbour direction
  std::vector<std::array<int, 3>> arm_dirs;   // arms the tables were built for (general layout)
  int grid[3];
  double R_pair, R_PE, R_ME;
  int l_max;
  int device = 0;
  hipStream_t stream = nullptr;
  exx::Geo geo;
  std::vector<exx::ClassHost> classes;
  std::vector<exx::ClassDev> class_dev_host;   // with device pointers
  exx::ClassDev* class_dev = nullptr;          // device copy of class_dev_host
  void* class_block = nullptr;                 // device block holding every class table
  int self_class = -1;   // class of the self pairs when they have their own radii
  long long max_pe = 0, max_halo = 0, max_me = 0, max_cols = 0;
  long long max_fin = 0;   // most real columns of a class (orthorhombic; the E/sigma sweep)
  long long rstride = 0;   // row stride of the per-pair workspaces: max_pe rounded up to 32
  int max_zmax = 0;

  // pair list
  long long pair_cap = 0;
  exx::PairDev* pairs = nullptr;   // canonical order
  int* order = nullptr;            // processing order (class descending)
  int* pair_count = nullptr;       // per-orbital counts and offsets [2 * orb_cap + 1 + classes]
  int orb_cap = 0;
  int* n_eff = nullptr;            // device: pairs stored in the processing order
  // warm start: two FP32 solution stores [2][pair_cap][rstride] (which one holds
  // the previous evaluation's solutions is the device parity in warm_state),
  // the previous pair list and per-orbital offsets, and the match of each pair
  // to its row in the previous list
  float* warm_store = nullptr;
  long long warm_cap = 0;          // pair rows per store
  int* warm_map = nullptr;         // [pair_cap]
  exx::PairDev* prev_pairs = nullptr;
  int* prev_offs = nullptr;        // [orb_cap + 1]
  int* warm_state = nullptr;       // device: parity, previous list valid, previous n_orb, previous stored pairs
  int warm_orb_cap = 0;
  int* d_slot = nullptr;           // device [orb_cap]: D row of each orbital (subset evaluations)
  int warm_orb = 0;                // largest n_orb of a completed eager eval with a fixed capacity
  bool capturing = false;          // inside an exx_eval recorded into a graph
  bool last_captured = false;      // the last exx_eval was recorded into a graph

  // per-pair results
  double* pE = nullptr;
  double* pS = nullptr;
  int* pIt = nullptr;
  double* pRes = nullptr;
  int* pUpd = nullptr;
  int* pSav = nullptr;   // per pair: CG sweeps that saved two vector accesses per point (fused, or x left alone)
  int* pExit = nullptr;  // CG exit reason per pair (EXX_CG_*) | restarts << 8

  // batch workspace
  long long batch_cap = 0;
  double* rho_ws = nullptr;    // [batch][max_pe] pair densities
  double* bx_ws = nullptr;     // [batch][max_pe] right-hand sides, then potentials
  double* halo_ws = nullptr;   // [batch][max_halo]
  double* Q_ws = nullptr;      // [batch][kMaxLM]
  double* rho_scale = nullptr; // [batch] power-of-two scale of each pair density
  double* Qp_ws = nullptr;     // [chunks][batch][kMaxLM] partial moments of the point chunks
  long long qp_rows = 0;
  int n_slots = 0;
  std::vector<int> class_groups;   // persistent solve workgroups of each class's launch
  std::vector<int> class_threads;  // CG variant of each class: workgroup size ...
  std::vector<int> class_depth;    // ... and load depth
  std::vector<double> class_delta; // ... and (mixed) reliable-update threshold; 0: the plan's
  int n_cus = 1;
  int solve_threads = 1024, solve_depth = 1;   // CG variant in use
  bool tuned = false;
  double tune_ms = 0;
  void* slot_ws = nullptr;     // [slots] CG vectors: FP64 r, p; mixed: FP64 x, FP32 r, p, y
  int* queue = nullptr;
  double* stats_dev = nullptr;     // the eight values of k_reduce (see launch_reduce)
  int last_n_orb = 0;

  // eval begin, workspace ready, reductions begin, eval end, pair list done
  hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  std::vector<hipEvent_t> solve_ev;   // begin/end pairs around each solve launch of the last eval
  int solve_ev_used = 0;
  std::vector<hipEvent_t> mom_ev;     // begin/end pairs around each moment launch of the last eval
  int mom_ev_used = 0;
  double last_moment_ms = 0;
  long long last_class_pairs[exx::kMaxClasses] = {0};
  bool timing_valid = false;
  bool harvested = true;              // last eval's events already added to the totals
  double last_solve_ms = 0, last_eval_ms = 0, last_alg_bytes = 0, last_pairlist_ms = 0, last_reduce_ms = 0;
  double last_stats[exx::kStatsLen] = {0};
  long long n_evals = 0, solve_launches = 0;
  double solve_ms_total = 0, eval_ms_total = 0, alg_bytes_total = 0;
  std::string err;

  // exx_eval_noalloc: the plan's own workspace while the scratch array's
  // pieces are the active one (on_scratch), the guard that turns any device
  // allocation into an error, and the batch and CG-workgroup limits of the
  // scratch layout (0: none)
  exx::EvalWork own_work;
  bool on_scratch = false;
  bool no_alloc = false;
  long long batch_limit = 0;
  int slot_limit = 0;
};
