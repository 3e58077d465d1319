// Host-side launchers of the gfx950 kernels (kernels.hip, moments.hip,
// solve.hip).
//
// Every per-batch launcher takes a Batch: rows [p0, p0 + nb) of the processing
// order, where nb is the launch's capacity and the kernels themselves skip rows
// at or beyond the device-side pair count *n_eff.  No launcher needs the pair
// count on the host, so an evaluation can be recorded into a HIP graph.
#pragma once

#include "exx_internal.h"

namespace exx {

struct PairParams {
  double R_pair2;           // R_pair^2 (1 + slack)
  double R_PE;              // fixed radius (class 0) when no per-orbital radii
  double R_min, R_step;     // variable radii rungs
  int n_class;              // <= 0: fixed radius
  int self_class;           // class of the self pairs (i == j), or -1: by radius like the others
  unsigned long long seed;
  double frac;
};

struct Batch {
  const ClassDev* cls;
  const PairDev* pairs;
  const int* order;     // processing order (class descending)
  const int* n_eff;     // device: pairs in the order (the stored ones, at most the capacity)
  long long p0, nb;     // first row and capacity of the batch
};

// counts[0 .. n_orb) per-orbital pair counts, counts[n_orb .. 2 n_orb] offsets
// (exclusive, with the total at index 2 n_orb), then per-class counts.
hipError_t launch_pairlist(const Geo& g, const PairParams& pp, const double* centres, const double* R_orb, int n_orb,
                           int* counts, PairDev* pairs, long long cap, hipStream_t s);
// Processing order of the stored pairs (at most cap) and its length *n_eff.
hipError_t launch_order(const PairDev* pairs, const int* counts, int n_orb, int n_class, int* order, long long cap,
                        int* n_eff, hipStream_t s);
// slot[i] = position of orbital i in subset[0 .. n_subset), else -1.
hipError_t launch_dslot(int* slot, int n_orb, const int* subset, int n_subset, hipStream_t s);

// rho_scale[b]: power of two at or above max |rho| of pair b (see k_gather)
hipError_t launch_gather(const Geo& g, const Batch& B, const void* orb, int dt, double* rho_ws, long long rstride,
                         double* rho_scale, hipStream_t s);
// Rows of the moment tables, and how many of them the matrix cores take:
// (l_max + 1)^2 padded to a multiple of 16, except that FP64 tables keep up to
// 4 rows past the last full 16-row tile for the vector ALU.
void moment_layout(int l_max, bool mixed, int* rows, int* mfma_rows);
// Number of point chunks the moment launch of a batch of nb pairs uses.
int moment_splits(long long nb, int ncls, long long max_pe);
// Moments of the batch into Q_ws; class_cnt holds the per-class pair counts of
// the order (device); Qp holds splits * nb * kMaxLM partial sums; rho rows are
// zero-padded to 32 points.
hipError_t launch_moments(const Geo& g, const Batch& B, const int* class_cnt, int ncls, bool mixed,
                          const double* rho_ws, long long rstride, const double* rho_scale, double* Qp, int splits,
                          double* Q_ws, hipStream_t s);
// Far-field values at the Dirichlet points of every pair of the batch, from
// its moments and the class's boundary table, on the matrix cores.
hipError_t launch_boundary(const Geo& g, const Batch& B, const int* class_cnt, int ncls, long long max_halo,
                           const double* Q_ws, double* halo_ws, long long hstride, hipStream_t s);

struct SolveArgs {
  Geo g;
  const ClassDev* cls = nullptr;
  const PairDev* pairs = nullptr;
  const int* order = nullptr;
  long long p0 = 0, npair = 0;   // batch start and capacity
  const int* n_eff = nullptr;    // device pair count of the processing order
  int cls_id = -1;               // >= 0: solve only this class's rows of the batch
  const int* class_cnt = nullptr;   // device per-class pair counts of the order
  int ncls = 1;
  int* queue = nullptr;
  double* bx_ws = nullptr;     // per pair: right-hand side in, solution out
  long long rstride = 0;
  void* slot_ws = nullptr;     // per workgroup CG vectors
  long long sstride = 0;
  int* outIt = nullptr;
  double* outRes = nullptr;
  int* outUpd = nullptr;       // reliable updates per pair (mixed)
  int* outSav = nullptr;       // per pair: sweeps that saved two vector accesses per point
  int* outExit = nullptr;      // per pair: exit reason (EXX_CG_*) | restarts << 8
  double tol = 0;
  int max_iter = 0;
  bool mixed = false;
  double delta = 0.01;         // mixed: reliable-update threshold
  // warm start (warm_store null: every solve starts from zero)
  const float* warm_store = nullptr;   // [2][warm_cap][rstride] FP32 solutions
  long long warm_cap = 0;
  const int* warm_state = nullptr;     // device parity at [0]
  const int* warm_map = nullptr;
  const PairDev* prev_pairs = nullptr;
  int threads = 1024;          // workgroup size of the solve (512 or 1024)
  int depth = 1;               // planes of loads in flight ahead of their use (1 or 2)
  bool quads = false;          // the class's vectors are in the quad layout
};

hipError_t launch_rhs(const Geo& g, const Batch& B, long long max_pe, const double* rho_ws, double* b_ws,
                      long long rstride, const double* halo_ws, long long hstride, hipStream_t s);
hipError_t launch_solve(const SolveArgs& a, int max_cols, int max_zmax, int groups, hipStream_t s);
size_t solve_lds_bytes(const Geo& g, int max_zmax);
int solve_groups_per_cu(const Geo& g, int max_cols, int max_zmax, bool mixed, bool quads, int threads, int depth);
bool solve_supported(int max_cols, int threads);
long long solve_slot_bytes(bool mixed, long long sstride);
hipError_t launch_finalize(const Geo& g, const Batch& B, const double* rho_ws, const double* v_ws, long long rstride,
                           const double* halo_ws, long long hstride, double* outE, double* outS, hipStream_t s);
// E_xx and sigma_xx of the batch's pairs as one plane sweep per pair
// (finalize.hip): orthorhombic cells whose classes have at most 4096 columns
// (finalize_sweep_supported); launch_finalize serves the others.
bool finalize_sweep_supported(const Geo& g, long long max_cols);
hipError_t launch_finalize_sweep(const Geo& g, const Batch& B, long long max_cols, const double* rho_ws,
                                 const double* v_ws, long long rstride, const double* halo_ws, long long hstride,
                                 double* outE, double* outS, hipStream_t s);
// D^i += v phi_j (and D^j += v phi_i) into row d_slot[i] of D, or row i when
// d_slot is null; rows with d_slot = -1 are not written.
hipError_t launch_dscatter(const Geo& g, const Batch& B, long long max_me, const void* orb, void* D,
                           const int* d_slot, int dt, const double* v_ws, long long rstride, const double* Q_ws,
                           hipStream_t s);

// Warm start: warm_map[p] = row of pair p in the previous evaluation's list,
// or -1; state = (parity, previous list valid, previous n_orb, previous
// stored pairs).  launch_warm_commit makes this evaluation's list the previous
// one and flips the store parity.
hipError_t launch_warm_match(const Geo& g, const PairDev* pairs, const int* n_eff, long long cap,
                             const PairDev* prev_pairs, const int* prev_offs, const int* state, int* warm_map,
                             hipStream_t s);
hipError_t launch_warm_commit(const PairDev* pairs, const int* counts, int n_orb, const int* n_eff, long long cap,
                              PairDev* prev_pairs, int* prev_offs, int* state, hipStream_t s);

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);
hipError_t launch_set_int(int* p, int v, hipStream_t s);

// E_xx and sigma from per-pair results in canonical order; stats[kStatsLen]
// receives (iter_sum, iter_max, n_unconverged, max_res, n_pairs kept (also
// beyond the capacity), sum iters*N_PE, refinement passes max, sum N_PE,
// warm-started pairs, pairs stopped at the iteration cap, by a breakdown, by a
// non-finite norm, restarts) as doubles.  A pair is unconverged when its exit
// reason (pExit, low byte) is not EXX_CG_CONVERGED.  warm_map may be null.
hipError_t launch_reduce(const double* pE, const double* pS, const int* pIt, const double* pRes, const int* pUpd,
                         const int* pSav, const int* pExit, const PairDev* pairs, const ClassDev* cls,
                         const int* counts, int n_orb, const int* n_eff, const int* warm_map, double* E, double* sigma,
                         double* stats, hipStream_t s);

}  // namespace exx
