// C ABI of the gfx950 EXX library (declared in include/exx.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "exx_launch.h"

using namespace exx;

namespace {

thread_local std::string g_plan_error;

exx_status fail(exx_plan_t P, exx_status st, const std::string& msg) {
  if (P) P->err = msg; else g_plan_error = msg;
  return st;
}

#define EXX_HIP(P, expr)                                                                              \
  do {                                                                                                \
    hipError_t e_ = (expr);                                                                           \
    if (e_ != hipSuccess) return fail((P), EXX_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

double det3(const double* m) {
  auto M = [&](int r, int c) { return m[r + 3 * c]; };
  return M(0, 0) * (M(1, 1) * M(2, 2) - M(1, 2) * M(2, 1)) - M(0, 1) * (M(1, 0) * M(2, 2) - M(1, 2) * M(2, 0)) +
         M(0, 2) * (M(1, 0) * M(2, 1) - M(1, 1) * M(2, 0));
}

void inv3(const double* m, double* inv) {
  auto M = [&](int r, int c) { return m[r + 3 * c]; };
  const double d = det3(m);
  inv[0 + 3 * 0] = (M(1, 1) * M(2, 2) - M(1, 2) * M(2, 1)) / d;
  inv[0 + 3 * 1] = (M(0, 2) * M(2, 1) - M(0, 1) * M(2, 2)) / d;
  inv[0 + 3 * 2] = (M(0, 1) * M(1, 2) - M(0, 2) * M(1, 1)) / d;
  inv[1 + 3 * 0] = (M(1, 2) * M(2, 0) - M(1, 0) * M(2, 2)) / d;
  inv[1 + 3 * 1] = (M(0, 0) * M(2, 2) - M(0, 2) * M(2, 0)) / d;
  inv[1 + 3 * 2] = (M(0, 2) * M(1, 0) - M(0, 0) * M(1, 2)) / d;
  inv[2 + 3 * 0] = (M(1, 0) * M(2, 1) - M(1, 1) * M(2, 0)) / d;
  inv[2 + 3 * 1] = (M(0, 1) * M(2, 0) - M(0, 0) * M(2, 1)) / d;
  inv[2 + 3 * 2] = (M(0, 0) * M(1, 1) - M(0, 1) * M(1, 0)) / d;
}

// Central-difference weights (Fornberg 1988): second derivative (the n = 3 set
// is the one printed with eq. d2_1) and antisymmetric first derivative (the
// n = 3 set printed with eq. d1_1).
void stencil_weights(int n, double* w2, double* w1) {
  for (int q = 0; q < 4; ++q) w2[q] = w1[q] = 0.0;
  switch (n) {
    case 1:
      w2[0] = -2.0; w2[1] = 1.0;
      w1[1] = 1.0 / 2.0;
      break;
    case 2:
      w2[0] = -5.0 / 2.0; w2[1] = 4.0 / 3.0; w2[2] = -1.0 / 12.0;
      w1[1] = 2.0 / 3.0; w1[2] = -1.0 / 12.0;
      break;
    default:
      w2[0] = -49.0 / 18.0; w2[1] = 3.0 / 2.0; w2[2] = -3.0 / 20.0; w2[3] = 1.0 / 90.0;
      w1[1] = 3.0 / 4.0; w1[2] = -3.0 / 20.0; w1[3] = 1.0 / 60.0;
      break;
  }
}

// normalisation of the real orthonormal harmonics: N_l0, and sqrt(2) N_lm for m != 0,
// N_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!)
void harmonic_norms(int L, double* out) {
  for (int l = 0; l <= L; ++l)
    for (int m = 0; m <= l; ++m) {
      double ratio = 1.0;
      for (int k = l - m + 1; k <= l + m; ++k) ratio /= (double)k;
      const double N = std::sqrt((2.0 * l + 1.0) / (4.0 * M_PI) * ratio);
      if (m == 0) {
        out[l * l + l] = N;
      } else {
        out[l * l + l + m] = std::sqrt(2.0) * N;
        out[l * l + l - m] = std::sqrt(2.0) * N;
      }
    }
}

// bfloat16 of a finite float, rounded to nearest even
unsigned short bf16_rne(float f) {
  unsigned u;
  std::memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
double bf16_value(unsigned short h) {
  const unsigned u = (unsigned)h << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return (double)f;
}

template <typename T>
exx_status dev_alloc(exx_plan_t P, T** p, size_t count, const char* what) {
  if (P && P->no_alloc)
    return fail(P, EXX_EINVAL, std::string("exx_eval_noalloc would need a device allocation (") + what +
                                   "); its workspace must come from the scratch array");
  if (P && P->capturing)
    return fail(P, EXX_EINVAL, std::string("exx_eval needs a device allocation (") + what +
                                   ") while its stream is recorded into a graph; run one eager exx_eval with the "
                                   "same sizes first");
  if (*p) (void)hipFree(*p);
  *p = nullptr;
  if (count == 0) return EXX_OK;
  hipError_t e = hipMalloc((void**)p, count * sizeof(T));
  if (e != hipSuccess) {
    *p = nullptr;
    return fail(P, EXX_ENOMEM, std::string("device allocation failed: ") + what);
  }
  return EXX_OK;
}

// Marks the plan as recording into a graph for the lifetime of one exx_eval.
struct CaptureGuard {
  exx_plan_t P;
  CaptureGuard(exx_plan_t p, bool on) : P(p) { P->capturing = on; }
  ~CaptureGuard() { P->capturing = false; }
};

// The plan's active workspace pointers as one EvalWork, and back.
EvalWork get_work(exx_plan_t P) {
  EvalWork w;
  w.pair_cap = P->pair_cap;
  w.pairs = P->pairs;
  w.order = P->order;
  w.pair_count = P->pair_count;
  w.orb_cap = P->orb_cap;
  w.n_eff = P->n_eff;
  w.d_slot = P->d_slot;
  w.pE = P->pE;
  w.pS = P->pS;
  w.pIt = P->pIt;
  w.pRes = P->pRes;
  w.pUpd = P->pUpd;
  w.pSav = P->pSav;
  w.pExit = P->pExit;
  w.batch_cap = P->batch_cap;
  w.rho_ws = P->rho_ws;
  w.bx_ws = P->bx_ws;
  w.halo_ws = P->halo_ws;
  w.Q_ws = P->Q_ws;
  w.rho_scale = P->rho_scale;
  w.Qp_ws = P->Qp_ws;
  w.qp_rows = P->qp_rows;
  w.n_slots = P->n_slots;
  w.slot_ws = P->slot_ws;
  return w;
}

void put_work(exx_plan_t P, const EvalWork& w) {
  P->pair_cap = w.pair_cap;
  P->pairs = w.pairs;
  P->order = w.order;
  P->pair_count = w.pair_count;
  P->orb_cap = w.orb_cap;
  P->n_eff = w.n_eff;
  P->d_slot = w.d_slot;
  P->pE = w.pE;
  P->pS = w.pS;
  P->pIt = w.pIt;
  P->pRes = w.pRes;
  P->pUpd = w.pUpd;
  P->pSav = w.pSav;
  P->pExit = w.pExit;
  P->batch_cap = w.batch_cap;
  P->rho_ws = w.rho_ws;
  P->bx_ws = w.bx_ws;
  P->halo_ws = w.halo_ws;
  P->Q_ws = w.Q_ws;
  P->rho_scale = w.rho_scale;
  P->Qp_ws = w.Qp_ws;
  P->qp_rows = w.qp_rows;
  P->n_slots = w.n_slots;
  P->slot_ws = w.slot_ws;
}

// After an exx_eval_noalloc the scratch array's pieces stay the active
// workspace (the statistics and per-pair results of that call live there);
// every call that may allocate or free workspace first makes the plan's own
// allocations active again.
void use_own_work(exx_plan_t P) {
  if (!P->on_scratch) return;
  put_work(P, P->own_work);
  P->own_work = EvalWork();
  P->on_scratch = false;
  P->timing_valid = false;   // the last evaluation's results were in the scratch array
  P->harvested = true;
  P->last_captured = false;
}

void free_plan(exx_plan_t P) {
  if (!P) return;
  use_own_work(P);
  void* ptrs[] = {P->class_dev, P->class_block, P->pairs, P->order, P->pair_count, P->pE, P->pS, P->pIt,
                  P->pRes, P->pUpd, P->pSav, P->pExit, P->rho_ws, P->bx_ws, P->halo_ws, P->Q_ws, P->Qp_ws, P->rho_scale, P->n_eff, P->d_slot, P->warm_store,
                  P->warm_map, P->prev_pairs, P->prev_offs, P->warm_state, P->slot_ws, P->queue,
                  P->stats_dev};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  for (auto& e : P->ev)
    if (e) (void)hipEventDestroy(e);
  for (auto& e : P->solve_ev)
    if (e) (void)hipEventDestroy(e);
  for (auto& e : P->mom_ev)
    if (e) (void)hipEventDestroy(e);
  delete P;
}

// Copies the device statistics of the last evaluation (k_reduce's eight
// values and the per-class pair counts).  The caller has synchronized.
exx_status read_device_stats(exx_plan_t P) {
  double st[kStatsLen] = {0};
  EXX_HIP(P, hipMemcpy(st, P->stats_dev, sizeof(st), hipMemcpyDeviceToHost));
  for (int k = 0; k < kStatsLen; ++k) P->last_stats[k] = st[k];
  int cc[kMaxClasses] = {0};
  const int ncls = (int)P->classes.size();
  EXX_HIP(P, hipMemcpy(cc, P->pair_count + 2 * P->last_n_orb + 1, sizeof(int) * ncls, hipMemcpyDeviceToHost));
  for (int k = 0; k < kMaxClasses; ++k) P->last_class_pairs[k] = k < ncls ? cc[k] : 0;
  return EXX_OK;
}

// Adds the finished evaluation's device times and algorithmic bytes to the
// running totals (once per evaluation).  The caller has synchronized the stream.
exx_status harvest(exx_plan_t P) {
  if (!P->timing_valid || P->harvested) return EXX_OK;
  float ms = 0;
  double solve = 0.0;
  for (int k = 0; k + 1 < P->solve_ev_used; k += 2) {
    EXX_HIP(P, hipEventElapsedTime(&ms, P->solve_ev[k], P->solve_ev[k + 1]));
    solve += ms;
  }
  double mom = 0.0;
  for (int k = 0; k + 1 < P->mom_ev_used; k += 2) {
    EXX_HIP(P, hipEventElapsedTime(&ms, P->mom_ev[k], P->mom_ev[k + 1]));
    mom += ms;
  }
  P->last_moment_ms = mom;
  float pl_ms = 0, red_ms = 0;
  EXX_HIP(P, hipEventElapsedTime(&pl_ms, P->ev[0], P->ev[4]));
  EXX_HIP(P, hipEventElapsedTime(&red_ms, P->ev[2], P->ev[3]));
  P->last_pairlist_ms = pl_ms;
  P->last_reduce_ms = red_ms;
  EXX_HIP(P, hipEventElapsedTime(&ms, P->ev[0], P->ev[3]));
  exx_status ds = read_device_stats(P);
  if (ds != EXX_OK) return ds;
  const double b = (P->opt.precision == EXX_PREC_MIXED) ? 4.0 : 8.0;
  P->last_solve_ms = solve;
  P->last_eval_ms = ms;
  P->last_alg_bytes = P->last_stats[5] * 8.0 * b;
  P->n_evals += 1;
  P->solve_launches += P->solve_ev_used / 2;
  P->solve_ms_total += solve;
  P->eval_ms_total += ms;
  P->alg_bytes_total += P->last_alg_bytes;
  P->harvested = true;
  return EXX_OK;
}

// Sizes each class's persistent solve grid from the occupancy of its CG
// variant (class_threads, class_depth; its columns per thread select the
// kernel instance).  The slot workspace, sized for the largest grid, is
// resized on the next eval.
// Elements per CG vector in a workgroup's slot: the largest class's points,
// rounded up to 8 so that every vector of the slot starts 32-byte aligned (the
// quad layout reads a run's four values as one vector).
long long slot_stride(exx_plan_t P) { return (P->max_pe + 7) / 8 * 8; }

// Whether the plan's Laplacian has arms leaving the sweep plane: those classes
// run the tilted-arm CG, which has one load depth (1).
static bool tilted_arms(const Geo& g) {
  if (!g.gen) return false;
  for (int m = 0; m < g.n_arms; ++m)
    if (g.arm_u[m][g.perm[2]] != 0) return true;
  return false;
}

exx_status apply_solve_variants(exx_plan_t P) {
  const bool mixed = P->opt.precision == EXX_PREC_MIXED;
  const size_t ncls = P->classes.size();
  P->class_groups.assign(ncls, 0);
  int slots = 0;
  for (size_t k = 0; k < ncls; ++k) {
    const ClassHost& C = P->classes[k];
    if (!C.quads && tilted_arms(P->geo)) P->class_depth[k] = 1;
    const int per_cu =
        solve_groups_per_cu(P->geo, C.n_cols, C.Zmax, mixed, C.quads, P->class_threads[k], P->class_depth[k]);
    if (per_cu < 1) return fail(P, EXX_EDEVICE, "solve kernel cannot be resident (occupancy 0)");
    P->class_groups[k] = P->opt.solve_groups > 0 ? P->opt.solve_groups : P->n_cus * per_cu;
    slots = std::max(slots, P->class_groups[k]);
  }
  if (slots != P->n_slots && P->slot_ws) {
    (void)hipFree(P->slot_ws);
    P->slot_ws = nullptr;
  }
  P->n_slots = slots;
  // the variant reported by exx_stats: that of the class with the most columns
  const int big = (int)(std::max_element(P->classes.begin(), P->classes.end(),
                                         [](const ClassHost& a, const ClassHost& b) { return a.n_cols < b.n_cols; }) -
                        P->classes.begin());
  P->solve_threads = P->class_threads[big];
  P->solve_depth = P->class_depth[big];
  return EXX_OK;
}

// Sets the CG variant of class cls and resizes the grids.
exx_status select_solve(exx_plan_t P, int threads, int depth, int cls) {
  P->class_threads[cls] = threads;
  P->class_depth[cls] = depth;
  return apply_solve_variants(P);
}

exx_status ensure_slots(exx_plan_t P) {
  if (P->slot_ws) return EXX_OK;
  char* sw = nullptr;
  const long long sb = solve_slot_bytes(P->opt.precision == EXX_PREC_MIXED, slot_stride(P));
  if (dev_alloc(P, &sw, (size_t)P->n_slots * sb, "CG vectors")) return EXX_ENOMEM;
  P->slot_ws = sw;
  return EXX_OK;
}

// The CG solve of a batch: one persistent launch per sphere class, in
// processing order, each with the kernel instance of its class's column count
// and finding its rows of the batch on the device.
exx_status launch_solves(exx_plan_t P, SolveArgs a, hipStream_t s) {
  const int ncls = (int)P->classes.size();
  a.ncls = ncls;
  a.class_cnt = P->pair_count + 2 * P->last_n_orb + 1;
  for (int k = ncls - 1; k >= 0; --k) {
    const ClassHost& C = P->classes[k];
    a.cls_id = ncls > 1 ? k : -1;
    a.threads = P->class_threads[k];
    a.depth = P->class_depth[k];
    if (P->class_delta[k] > 0.0) a.delta = P->class_delta[k];   // chosen by the autotuner
    a.quads = C.quads;
    EXX_HIP(P, launch_set_int(P->queue, 0, s));
    long long groups = std::min<long long>(P->class_groups[k], a.npair);
    if (P->slot_limit > 0) groups = std::min<long long>(groups, P->slot_limit);   // CG slots of the scratch layout
    EXX_HIP(P, launch_solve(a, C.n_cols, C.Zmax, (int)groups, s));
  }
  return EXX_OK;
}

// Autotuner: for each sphere class with pairs in this batch, times every CG
// variant (workgroup size x load depth) that can run it on a sample of the
// class's pairs (one per workgroup of the grid), and keeps the fastest for
// that class; mixed plans without a fixed refine_delta then time the chosen
// variant with reliable-update thresholds of 0.1 and 0.001 beside the default
// 0.01 (fewer FP64 updates against a few more FP32 iterations).  The class's
// current (default) choice is timed first and is replaced only by one at
// least 3% faster, so that repeated plans settle on the same choice when
// timings are close.  Densities and boundary values are in the workspace;
// right-hand sides are rebuilt before each trial (the solve overwrites them)
// and once more by the caller.
exx_status autotune_solve(exx_plan_t P, const SolveArgs& base, long long nb, hipStream_t s) {
  static const int cand[6][2] = {{1024, 1}, {1024, 2}, {768, 1}, {768, 2}, {512, 1}, {512, 2}};
  static const double deltas[2] = {0.1, 0.001};
  hipEvent_t e0 = nullptr, e1 = nullptr, t0 = nullptr, t1 = nullptr;
  EXX_HIP(P, hipEventCreate(&e0));
  EXX_HIP(P, hipEventCreate(&e1));
  EXX_HIP(P, hipEventCreate(&t0));
  EXX_HIP(P, hipEventCreate(&t1));
  EXX_HIP(P, hipEventRecord(t0, s));
  const int ncls = (int)P->classes.size();
  int cc[kMaxClasses] = {0};
  EXX_HIP(P, hipMemcpyAsync(cc, P->pair_count + 2 * P->last_n_orb + 1, sizeof(int) * ncls, hipMemcpyDeviceToHost, s));
  EXX_HIP(P, hipStreamSynchronize(s));
  long long start = 0;
  for (int k = ncls - 1; k >= 0; --k) {
    const long long lo = std::max(start, base.p0), hi = std::min(start + cc[k], base.p0 + nb);
    start += cc[k];
    if (hi <= lo) continue;
    // one trial: the sample's solve time per pair with variant (threads,
    // depth) and threshold delta, or a negative value when it cannot run
    auto trial = [&](int threads, int depth, double delta, float* per_pair) -> exx_status {
      *per_pair = -1.0f;
      if (solve_groups_per_cu(P->geo, P->classes[k].n_cols, P->classes[k].Zmax, base.mixed, P->classes[k].quads,
                              threads, depth) < 1)
        return EXX_OK;
      exx_status st = select_solve(P, threads, depth, k);
      if (st != EXX_OK) return st;
      st = ensure_slots(P);
      if (st != EXX_OK) return st;
      const long long sample = std::min<long long>(hi - lo, P->class_groups[k]);
      SolveArgs a = base;
      a.npair = lo + sample - base.p0;   // batch rows up to the end of the sample
      a.slot_ws = P->slot_ws;
      a.ncls = ncls;
      a.class_cnt = P->pair_count + 2 * P->last_n_orb + 1;
      a.cls_id = ncls > 1 ? k : -1;
      a.threads = threads;
      a.depth = depth;
      a.delta = delta;
      a.quads = P->classes[k].quads;
      Batch B;
      B.cls = P->class_dev;
      B.pairs = P->pairs;
      B.order = P->order;
      B.n_eff = P->n_eff;
      B.p0 = base.p0;
      B.nb = a.npair;
      EXX_HIP(P, launch_rhs(P->geo, B, P->max_pe, P->rho_ws, P->bx_ws, P->rstride, P->halo_ws,
                            std::max<long long>(P->max_halo, 1), s));
      EXX_HIP(P, launch_set_int(P->queue, 0, s));
      EXX_HIP(P, hipEventRecord(e0, s));
      EXX_HIP(P, launch_solve(a, P->classes[k].n_cols, P->classes[k].Zmax,
                              (int)std::min<long long>(P->class_groups[k], sample), s));
      EXX_HIP(P, hipEventRecord(e1, s));
      EXX_HIP(P, hipEventSynchronize(e1));
      float ms = 0;
      EXX_HIP(P, hipEventElapsedTime(&ms, e0, e1));
      *per_pair = ms / (float)sample;
      return EXX_OK;
    };
    const double d0 = P->class_delta[k] > 0.0 ? P->class_delta[k] : base.delta;
    float best = 1e30f;
    int bt = P->class_threads[k], bd = P->class_depth[k];
    int order[7][2] = {{bt, bd}};
    int nc = 1;
    const bool one_depth = !P->classes[k].quads && tilted_arms(P->geo);   // no deeper variant to try
    for (const auto& c : cand)
      if ((c[0] != bt || c[1] != bd) && !(one_depth && c[1] != 1)) {
        order[nc][0] = c[0];
        order[nc][1] = c[1];
        ++nc;
      }
    for (int ci = 0; ci < nc; ++ci) {
      float per_pair;
      exx_status st = trial(order[ci][0], order[ci][1], d0, &per_pair);
      if (st != EXX_OK) return st;
      if (per_pair < 0.0f) continue;
      if (ci == 0 ? per_pair < best : per_pair < 0.97f * best) {
        best = per_pair;
        bt = order[ci][0];
        bd = order[ci][1];
      }
    }
    double bdelta = d0;
    if (base.mixed && P->opt.refine_delta <= 0.0) {
      for (double dl : deltas) {
        float per_pair;
        exx_status st = trial(bt, bd, dl, &per_pair);
        if (st != EXX_OK) return st;
        if (per_pair >= 0.0f && per_pair < 0.97f * best) {
          best = per_pair;
          bdelta = dl;
        }
      }
    }
    P->class_delta[k] = bdelta;
    exx_status st = select_solve(P, bt, bd, k);
    if (st != EXX_OK) return st;
  }
  EXX_HIP(P, hipEventRecord(t1, s));
  EXX_HIP(P, hipEventSynchronize(t1));
  float tms = 0;
  EXX_HIP(P, hipEventElapsedTime(&tms, t0, t1));
  P->tune_ms = tms;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  P->tuned = true;
  return ensure_slots(P);
}

// Records the next event of a begin/end list (solve or moment launches).
exx_status record_event(exx_plan_t P, std::vector<hipEvent_t>& evs, int& used, hipStream_t s) {
  if (used >= (int)evs.size()) {
    hipEvent_t e = nullptr;
    EXX_HIP(P, hipEventCreate(&e));
    evs.push_back(e);
  }
  EXX_HIP(P, hipEventRecord(evs[used++], s));
  return EXX_OK;
}
exx_status record_solve_event(exx_plan_t P, hipStream_t s) { return record_event(P, P->solve_ev, P->solve_ev_used, s); }
exx_status record_moment_event(exx_plan_t P, hipStream_t s) { return record_event(P, P->mom_ev, P->mom_ev_used, s); }

// ---------------------------------------------------------------------------
// The cell (Sec. III B): geometry, Laplacian arms and sphere-class tables.

bool off_diagonal(const double h[9]) {
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c)
      if (r != c && h[r + 3 * c] != 0.0) return true;
  return false;
}

// Cell-dependent fields of the geometry: h, h^-1, edge lengths and spacings,
// the Jacobian of eq. jacb, the offset map r = A o and the volume element.
void set_cell_geometry(Geo& g, const double h[9], bool general) {
  std::memcpy(g.h, h, sizeof(g.h));
  inv3(h, g.hinv);
  for (int a = 0; a < 3; ++a) {
    g.L[a] = general ? std::sqrt(h[3 * a] * h[3 * a] + h[1 + 3 * a] * h[1 + 3 * a] + h[2 + 3 * a] * h[2 + 3 * a])
                     : h[a + 3 * a];
    g.d[a] = g.L[a] / g.N[a];
    g.inv_d2[a] = 1.0 / (g.d[a] * g.d[a]);
    g.inv_d[a] = 1.0 / g.d[a];
  }
  for (int a = 0; a < 3; ++a)
    for (int al = 0; al < 3; ++al) {
      g.J[a + 3 * al] = g.L[al] * g.hinv[al + 3 * a];
      g.A[a + 3 * al] = h[a + 3 * al] / g.N[al];
    }
  g.dV = std::fabs(det3(h)) / (double)g.ngrid;
  g.gen = general ? 1 : 0;
}

// NK arms of cell h into g (general layout); every arm must be a nearest grid
// neighbour direction.  Returns an empty string or the reason.
std::string set_cell_arms(Geo& g, const double h[9], std::vector<NkArm>* arms) {
  std::string e = build_nk_arms(h, g.N, arms);
  if (!e.empty()) return e;
  if (arms->size() > 6) return "more than six NK arms";
  g.n_arms = (int)arms->size();
  for (size_t k = 0; k < arms->size(); ++k) {
    for (int a = 0; a < 3; ++a) {
      if (std::abs((*arms)[k].u[a]) > 1) return "an NK auxiliary direction beyond the first shell of grid neighbours";
      g.arm_u[k][a] = (*arms)[k].u[a];
    }
    g.arm_coef[k] = (*arms)[k].beta / ((*arms)[k].step * (*arms)[k].step);
  }
  return std::string();
}

double cell_strain(const double h[9], const double h0[9]) {
  double h0inv[9];
  inv3(h0, h0inv);
  double m = 0.0;
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += h[r + 3 * k] * h0inv[k + 3 * c];
      m = std::max(m, std::fabs(s - (r == c ? 1.0 : 0.0)));
    }
  return m;
}

// Moment and boundary tables of every class for the plan's current offset
// map, into the class block (same sizes as at assembly).
exx_status upload_moment_tables(exx_plan_t P, const Geo& g) {
  const bool mixed = P->opt.precision == EXX_PREC_MIXED;
  int mom_rows = 0, mom_mfma_rows = 0;
  moment_layout(P->l_max, mixed, &mom_rows, &mom_mfma_rows);
  for (size_t k = 0; k < P->classes.size(); ++k) {
    std::vector<double> btab;
    build_boundary_table(P->classes[k], g.A, g.ylm_norm, P->l_max, &btab);
    EXX_HIP(P, hipMemcpy((void*)P->class_dev_host[k].bnd_tab, btab.data(), btab.size() * sizeof(double),
                         hipMemcpyHostToDevice));
    std::vector<double> tab;
    build_moment_table(P->classes[k], g.A, P->l_max, mom_rows, mixed ? 8 : 4, &tab);
    const ClassDev& D = P->class_dev_host[k];
    if (mixed) {
      std::vector<unsigned short> hi(tab.size()), lo(tab.size());
      for (size_t e = 0; e < tab.size(); ++e) {
        hi[e] = bf16_rne((float)tab[e]);
        lo[e] = bf16_rne((float)(tab[e] - bf16_value(hi[e])));
      }
      EXX_HIP(P, hipMemcpy((void*)D.mom_hi, hi.data(), hi.size() * sizeof(unsigned short), hipMemcpyHostToDevice));
      EXX_HIP(P, hipMemcpy((void*)D.mom_lo, lo.data(), lo.size() * sizeof(unsigned short), hipMemcpyHostToDevice));
    } else {
      EXX_HIP(P, hipMemcpy((void*)D.mom_f64, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice));
    }
  }
  return EXX_OK;
}

// Builds the cell-dependent part of the plan for cell h: geometry, Laplacian
// arms, the sphere classes and their device tables.  Everything is built
// aside and replaces the plan's tables only on success.  Host-side checks run
// before any device call.
exx_status assemble_cell(exx_plan_t P, const double h[9]) {
  const exx_options& opt = P->opt;
  const int n = opt.stencil_n;
  const bool general = opt.cell_fluctuation != 0 || off_diagonal(h);
  Geo g = P->geo;
  set_cell_geometry(g, h, general);
  for (int a = 0; a < 3; ++a) g.perm[a] = a;
  g.n_arms = 0;
  double maxd = std::max(g.d[0], std::max(g.d[1], g.d[2]));
  std::vector<NkArm> arms;
  if (general) {
    std::string e = set_cell_arms(g, h, &arms);
    if (!e.empty()) return fail(P, EXX_EINVAL, e);
    for (const NkArm& A : arms) maxd = std::max(maxd, A.step);
  }
  if (opt.cell_fluctuation) {
    // Dirichlet points along every nearest-neighbour direction
    for (int u2 = -1; u2 <= 1; ++u2)
      for (int u1 = -1; u1 <= 1; ++u1)
        for (int u0 = -1; u0 <= 1; ++u0) {
          const int u[3] = {u0, u1, u2};
          double v[3] = {0, 0, 0};
          for (int al = 0; al < 3; ++al)
            for (int a = 0; a < 3; ++a) v[a] += u[al] * g.A[a + 3 * al];
          maxd = std::max(maxd, std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]));
        }
  }

  // sphere classes: the fixed radius or the variable-radius rungs, then (with
  // self radii) one class of the self pairs with their own PE and ME spheres
  std::vector<double> radii, me_radii;
  if (opt.R_PE_nclass > 0) {
    for (int k = 0; k < opt.R_PE_nclass; ++k) radii.push_back(opt.R_PE_min + k * opt.R_PE_step);
  } else {
    radii.push_back(P->R_PE);
  }
  const double rmax = *std::max_element(radii.begin(), radii.end());
  if (P->R_ME < rmax + n * maxd) return fail(P, EXX_EINVAL, "R_ME must be >= R_PE + n * (longest stencil step)");
  me_radii.assign(radii.size(), P->R_ME);
  int self_class = -1;
  if (opt.R_PE_self > 0.0 || opt.R_ME_self > 0.0) {
    const double rpe = opt.R_PE_self > 0.0 ? opt.R_PE_self : P->R_PE;
    const double rme = opt.R_ME_self > 0.0 ? opt.R_ME_self : P->R_ME;
    if (rme < rpe + n * maxd)
      return fail(P, EXX_EINVAL, "R_ME_self must be >= R_PE_self + n * (longest stencil step)");
    self_class = (int)radii.size();
    radii.push_back(rpe);
    me_radii.push_back(rme);
  }
  std::vector<ClassHost> classes(radii.size());
  const bool all_dirs = opt.cell_fluctuation != 0;
  if (general) {
    // sweep axis of the CG: the one whose padded columns hold the fewest
    // slots (zero padding when it is perpendicular to the other two), then the
    // fewest arms that leave the sweep plane, then the last axis
    const size_t big = (size_t)(std::max_element(radii.begin(), radii.end()) - radii.begin());
    long long best_slots = -1;
    int best_tilt = 0;
    for (int sw = 2; sw >= 0; --sw) {
      ClassHost T;
      std::string e = build_class_general(h, g.N, sw, radii[big], me_radii[big], n, arms, all_dirs, false, &T);
      if (!e.empty()) return fail(P, EXX_EINVAL, e);
      int tilt = 0;
      for (const NkArm& A : arms)
        if (A.u[sw] != 0 && (A.u[(sw + 1) % 3] != 0 || A.u[(sw + 2) % 3] != 0)) ++tilt;
      if (best_slots < 0 || T.n_pe < best_slots || (T.n_pe == best_slots && tilt < best_tilt)) {
        best_slots = T.n_pe;
        best_tilt = tilt;
        for (int a = 0; a < 3; ++a) g.perm[a] = T.perm[a];
      }
    }
  }
  // CG layout of each sphere class of an orthorhombic cell: runs of four
  // columns per thread (the quad layout) for mixed plans by default or when
  // asked, if the class's runs fit one workgroup of 1024 threads and its row
  // fits the LDS plane with the runs' 4-point neighbour vectors (R / spacing + 7
  // points on both sides of an origin that is a multiple of 4, so that runs
  // start at even positions); else single columns
  // General cells take the quad layout when no arm leaves the sweep plane and
  // the in-plane arms are the two axes and at most one diagonal (|u_x'| =
  // |u_y'| = 1), and the columns need no padding (checked by the builder);
  // not with cell_fluctuation, whose later cells may bring other arms.
  bool arms_fit = true;
  if (general) {
    int diagonals = 0;
    for (const NkArm& A : arms) {
      const int ux = A.u[g.perm[0]], uy = A.u[g.perm[1]], uz = A.u[g.perm[2]];
      if (uz != 0 && (ux != 0 || uy != 0)) arms_fit = false;
      if (ux != 0 && uy != 0) {
        ++diagonals;
        if (std::abs(ux) != 1 || std::abs(uy) != 1) arms_fit = false;
      }
    }
    arms_fit = arms_fit && diagonals <= 1 && !opt.cell_fluctuation;
  }
  const bool want_quads = arms_fit && (opt.cg_layout == 2 || (opt.cg_layout == 0 && opt.precision == EXX_PREC_MIXED));
  if (opt.cg_layout == 2 && !arms_fit)
    return fail(P, EXX_EINVAL, "quad layout: an arm of the cell's Laplacian leaves the sweep plane, or more than one "
                               "diagonal arm lies in it");
  auto quads_fit = [&](const ClassHost& C) {
    return C.n_cols <= 4 * 1024 && (C.Rc[0] + 7 + 3) / 4 * 4 + C.Rc[0] + 7 <= kLdsWX - 1;
  };
  long long max_pe = 0, max_halo = 0, max_me = 0, max_cols = 0;
  int max_zmax = 0, maxRq = -1, maxRc = -1, maxRc1 = 0;
  for (size_t k = 0; k < radii.size(); ++k) {
    auto build = [&](bool q) {
      return general ? build_class_general(h, g.N, g.perm[2], radii[k], me_radii[k], n, arms, all_dirs, q, &classes[k])
                     : build_class(g.L, g.N, radii[k], me_radii[k], n, q, &classes[k]);
    };
    std::string e = build(want_quads);
    if (!e.empty()) return fail(P, EXX_EINVAL, e);
    if (want_quads && opt.cg_layout == 2 && !classes[k].quads)
      return fail(P, EXX_EINVAL, "quad layout: the cell's columns are not symmetric about the sweep plane");
    if (classes[k].quads && !quads_fit(classes[k])) {
      if (opt.cg_layout == 2)
        return fail(P, EXX_EINVAL, "quad layout: the PE sphere needs more than 1024 runs or a wider LDS row");
      e = build(false);
      if (!e.empty()) return fail(P, EXX_EINVAL, e);
    }
  }
  auto class_extents = [&]() {
    max_pe = max_halo = max_me = max_cols = 0;
    max_zmax = maxRc1 = 0;
    maxRq = maxRc = -1;
    for (const ClassHost& C : classes) {
      max_pe = std::max(max_pe, C.n_pe);
      max_halo = std::max(max_halo, C.n_halo);
      max_me = std::max(max_me, C.n_me);
      max_cols = std::max<long long>(max_cols, C.n_cols);
      max_zmax = std::max(max_zmax, C.Zmax);
      if (C.quads) maxRq = std::max(maxRq, C.Rc[0]); else maxRc = std::max(maxRc, C.Rc[0]);
      maxRc1 = std::max(maxRc1, C.Rc[1]);
    }
  };
  class_extents();
  // one LDS plane origin for every class: a multiple of 4 at least R + 7 from
  // the left edge for quad classes (R + n for column classes), and the row
  // must hold R + 7 (R + n) points right of it
  if (maxRq >= 0) {
    g.lds_cx = (std::max(maxRq + 7, maxRc + n) + 3) / 4 * 4;
    if (g.lds_cx + maxRq + 7 > kLdsWX - 1 || (maxRc >= 0 && g.lds_cx + maxRc + n > kLdsWX - 1)) {
      // the classes do not share a plane origin: every class in columns
      if (opt.cg_layout == 2)
        return fail(P, EXX_EINVAL, "quad layout: the sphere classes do not fit one LDS row");
      for (size_t k = 0; k < radii.size(); ++k)
        if (classes[k].quads) {
          std::string e = general ? build_class_general(h, g.N, g.perm[2], radii[k], me_radii[k], n, arms, all_dirs,
                                                        false, &classes[k])
                                  : build_class(g.L, g.N, radii[k], me_radii[k], n, false, &classes[k]);
          if (!e.empty()) return fail(P, EXX_EINVAL, e);
        }
      class_extents();
    }
  }
  if (maxRq < 0) g.lds_cx = maxRc + n;
  g.lds_cy = maxRc1 + n;
  g.lds_wx = kLdsWX;
  g.lds_wy = 2 * g.lds_cy + 1;
  if (maxRq < 0 && 2 * g.lds_cx + 1 > kLdsWX)
    return fail(P, EXX_EINVAL, "PE sphere too wide: need 2 (R_PE / spacing + n) + 1 <= 88 grid points");
  if (!solve_supported((int)std::min<long long>(max_cols, 1 << 30), 512))
    return fail(P, EXX_EINVAL, "PE sphere has too many columns for one workgroup (R_PE / spacing too large)");
  if (solve_lds_bytes(g, max_zmax) > 160 * 1024) return fail(P, EXX_EINVAL, "PE sphere too wide for the LDS plane buffers");

  if (!P->class_block && hipGetDevice(&P->device) != hipSuccess) return fail(P, EXX_EDEVICE, "no HIP device");
  // upload the class tables into one block
  auto align = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const bool mixed = opt.precision == EXX_PREC_MIXED;
  int mom_rows = 0, mom_mfma_rows = 0;
  moment_layout(P->l_max, mixed, &mom_rows, &mom_mfma_rows);
  auto mom_bytes = [&](const ClassHost& C) {
    const size_t entries = (size_t)((C.n_pe + 31) / 32 * 32) * mom_rows;
    return mixed ? 2 * align(entries * sizeof(unsigned short)) : align(entries * sizeof(double));
  };
  size_t total = 0;
  for (const ClassHost& C : classes) {
    total += align(C.cols.size() * sizeof(int4)) + align(C.plane_start.size() * sizeof(int)) +
             align(C.halo_off.size() * sizeof(short4)) + align(C.me_off.size() * sizeof(short4)) +
             align(C.halo_map.size() * sizeof(int)) + align(C.col_map.size() * sizeof(int)) +
             align(C.zr_map.size() * sizeof(int)) + align(C.pe_map.size() * sizeof(int)) +
             align(C.halo_zidx.size() * sizeof(int)) + align(C.halo_zstart.size() * sizeof(int)) +
             align(C.fin_cols.size() * sizeof(int4)) + align(C.rhs_ptr.size() * sizeof(int)) +
             align(C.rhs_ent.size() * sizeof(int2)) + align(C.me_scan.size() * sizeof(int)) +
             align(C.scan_off.size() * sizeof(short4)) + align(C.rhs_edge.size() * sizeof(unsigned)) + mom_bytes(C) +
             align((size_t)((C.n_halo + 15) / 16) * ((g.n_lm + 3) / 4) * 64 * sizeof(double));
  }
  void* block = nullptr;
  ClassDev* class_dev = nullptr;
  if (hipMalloc(&block, total) != hipSuccess) return fail(P, EXX_ENOMEM, "device allocation of the subdomain tables failed");
  auto give_up = [&](exx_status st, const char* msg) {
    (void)hipFree(block);
    if (class_dev) (void)hipFree(class_dev);
    return fail(P, st, msg);
  };
  char* base = (char*)block;
  size_t off = 0;
  // an empty table has no device address (null): kernels tell the general
  // layout by a non-null pe_map
  auto put = [&](const void* src, size_t bytes) -> const void* {
    if (!bytes) return nullptr;
    void* dst = base + off;
    if (hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice) != hipSuccess) return nullptr;
    off += align(bytes);
    return dst;
  };
  std::vector<ClassDev> class_dev_host;
  for (const ClassHost& C : classes) {
    ClassDev D;
    std::memset(&D, 0, sizeof(D));
    D.R_PE = C.R_PE;
    D.n_cols = C.n_cols;
    D.Zmax = C.Zmax;
    for (int a = 0; a < 3; ++a) {
      D.Rg[a] = C.Rg[a];
      D.Wm[a] = C.Wm[a];
      D.Rc[a] = C.Rc[a];
    }
    D.n_pe = C.n_pe;
    D.n_real = C.n_real;
    D.n_halo = C.n_halo;
    D.n_me = C.n_me;
    D.cols = (const int4*)put(C.cols.data(), C.cols.size() * sizeof(int4));
    D.plane_start = (const int*)put(C.plane_start.data(), C.plane_start.size() * sizeof(int));
    D.halo_off = (const short4*)put(C.halo_off.data(), C.halo_off.size() * sizeof(short4));
    D.me_off = (const short4*)put(C.me_off.data(), C.me_off.size() * sizeof(short4));
    D.halo_map = (const int*)put(C.halo_map.data(), C.halo_map.size() * sizeof(int));
    D.col_map = (const int*)put(C.col_map.data(), C.col_map.size() * sizeof(int));
    D.zr_map = (const int*)put(C.zr_map.data(), C.zr_map.size() * sizeof(int));
    D.pe_map = general ? (const int*)put(C.pe_map.data(), C.pe_map.size() * sizeof(int)) : nullptr;
    D.halo_zidx = (const int*)put(C.halo_zidx.data(), C.halo_zidx.size() * sizeof(int));
    D.halo_zstart = (const int*)put(C.halo_zstart.data(), C.halo_zstart.size() * sizeof(int));
    D.Zh = C.Zmax + n;
    D.fin_cols = (const int4*)put(C.fin_cols.data(), C.fin_cols.size() * sizeof(int4));
    D.n_fin = (int)C.fin_cols.size();
    D.rhs_ptr = (const int*)put(C.rhs_ptr.data(), C.rhs_ptr.size() * sizeof(int));
    D.rhs_ent = (const int2*)put(C.rhs_ent.data(), C.rhs_ent.size() * sizeof(int2));
    D.rhs_edge = (const unsigned*)put(C.rhs_edge.data(), C.rhs_edge.size() * sizeof(unsigned));
    D.me_scan = (const int*)put(C.me_scan.data(), C.me_scan.size() * sizeof(int));
    D.scan_off = (const short4*)put(C.scan_off.data(), C.scan_off.size() * sizeof(short4));
    D.n_scan = (long long)C.me_scan.size();
    D.mom_rows = mom_rows;
    std::vector<double> btab;
    build_boundary_table(C, g.A, g.ylm_norm, P->l_max, &btab);
    D.bnd_tab = (const double*)put(btab.data(), btab.size() * sizeof(double));
    std::vector<double> tab;
    build_moment_table(C, g.A, P->l_max, mom_rows, mixed ? 8 : 4, &tab);
    bool tab_ok;
    if (mixed) {
      std::vector<unsigned short> hi(tab.size()), lo(tab.size());
      for (size_t e = 0; e < tab.size(); ++e) {
        hi[e] = bf16_rne((float)tab[e]);
        lo[e] = bf16_rne((float)(tab[e] - bf16_value(hi[e])));
      }
      D.mom_hi = (const unsigned short*)put(hi.data(), hi.size() * sizeof(unsigned short));
      D.mom_lo = (const unsigned short*)put(lo.data(), lo.size() * sizeof(unsigned short));
      tab_ok = D.mom_hi && D.mom_lo;
    } else {
      D.mom_f64 = (const double*)put(tab.data(), tab.size() * sizeof(double));
      tab_ok = D.mom_f64 != nullptr;
    }
    if (!D.cols || !D.plane_start || !D.me_off || !D.me_scan || !D.scan_off || !D.bnd_tab || !D.halo_map ||
        (!general && (!D.col_map || !D.zr_map)) ||
        (general != (D.pe_map != nullptr)) || !tab_ok)
      return give_up(EXX_EDEVICE, "upload of the subdomain tables failed");
    class_dev_host.push_back(D);
  }
  if (hipMalloc(&class_dev, sizeof(ClassDev) * class_dev_host.size()) != hipSuccess ||
      hipMemcpy(class_dev, class_dev_host.data(), sizeof(ClassDev) * class_dev_host.size(),
                hipMemcpyHostToDevice) != hipSuccess)
    return give_up(EXX_EDEVICE, "upload of the class descriptors failed");

  // commit
  if (P->class_block) (void)hipFree(P->class_block);
  if (P->class_dev) (void)hipFree(P->class_dev);
  P->class_block = block;
  P->class_dev = class_dev;
  P->class_dev_host = class_dev_host;
  P->classes.swap(classes);
  P->geo = g;
  P->self_class = self_class;
  P->max_pe = max_pe;
  P->rstride = (max_pe + 31) / 32 * 32;
  P->max_halo = max_halo;
  P->max_me = max_me;
  P->max_cols = max_cols;
  P->max_fin = 0;
  for (const ClassHost& C : P->classes) P->max_fin = std::max<long long>(P->max_fin, (long long)C.fin_cols.size());
  P->max_zmax = max_zmax;
  std::memcpy(P->h, h, sizeof(P->h));
  std::memcpy(P->h0, h, sizeof(P->h0));
  P->cell_strain = 0.0;
  P->all_dirs = all_dirs;
  P->arm_dirs.clear();
  for (const NkArm& A : arms) P->arm_dirs.push_back({A.u[0], A.u[1], A.u[2]});
  return EXX_OK;
}

// Default CG variant of each class (measured on MI355X): 1024 threads up to
// three columns each for orthorhombic cells (1024 x 4 spills), up to four for
// general cells (whose passes keep fewer values per column), else 512; quad
// layout classes of mixed plans 768 threads (one run each) where the runs fit,
// else 512 (two runs each), both with fused sweeps; FP64 quad classes 1024
// threads; an explicit solve_threads that can run the class is kept.  FP64
// loads one plane ahead, mixed two (512-thread quad classes, and cells with
// arms leaving the sweep plane, one).
void default_solve_variants(exx_plan_t P) {
  const exx_options& opt = P->opt;
  const int dp = opt.solve_depth > 0 ? opt.solve_depth : (opt.precision == EXX_PREC_MIXED ? 2 : 1);
  const int cpt = P->geo.gen ? 4 : 3;
  P->class_threads.assign(P->classes.size(), 1024);
  P->class_depth.assign(P->classes.size(), dp);
  P->class_delta.assign(P->classes.size(), 0.0);
  for (size_t k = 0; k < P->classes.size(); ++k) {
    const int nc = P->classes[k].n_cols;
    if (P->classes[k].quads) {
      // mixed plans fuse each pass B with the next pass A in workgroups of
      // 768 (one run per thread) or 512 threads (two runs per thread)
      int t = opt.precision == EXX_PREC_MIXED ? (nc <= 4 * 768 ? 768 : 512) : 1024;
      if (opt.solve_threads == 512 || opt.solve_threads == 1024 || (opt.solve_threads == 768 && nc <= 4 * 768))
        t = opt.solve_threads;
      P->class_threads[k] = t;
      // two runs per thread: loads one plane ahead (the registers of a
      // second plane of loads cost more than they hide)
      if (t == 512 && opt.solve_depth == 0) P->class_depth[k] = 1;
      continue;
    }
    P->class_threads[k] = (opt.solve_threads == 512 || opt.solve_threads == 1024) ? opt.solve_threads
                          : (nc <= cpt * 1024 ? 1024 : 512);
  }
}

// A new cell for the same proto-subdomains (fixed grid offsets, Sec. III B 2):
// geometry, arms and moment tables.
exx_status update_cell(exx_plan_t P, const double h[9]) {
  Geo g = P->geo;
  const bool general = g.gen != 0;
  if (!general && off_diagonal(h))
    return fail(P, EXX_EINVAL, "the plan holds orthorhombic tables (build it with cell_fluctuation for other cells)");
  set_cell_geometry(g, h, general);
  if (general) {
    std::vector<NkArm> arms;
    std::string e = set_cell_arms(g, h, &arms);
    if (!e.empty()) return fail(P, EXX_EINVAL, e);
    if (!P->all_dirs) {
      // the Dirichlet points cover the arms (and axes) the tables were built for
      for (const NkArm& A : arms) {
        const int nz = (A.u[0] != 0) + (A.u[1] != 0) + (A.u[2] != 0);
        bool known = nz == 1;
        for (const auto& d : P->arm_dirs)
          known = known || (d[0] == A.u[0] && d[1] == A.u[1] && d[2] == A.u[2]) ||
                  (d[0] == -A.u[0] && d[1] == -A.u[1] && d[2] == -A.u[2]);
        if (!known)
          return fail(P, EXX_EINVAL, "the new cell's Laplacian needs Dirichlet points the tables do not hold "
                                     "(build the plan with cell_fluctuation, or re-assemble)");
      }
    }
  }
  exx_status st = upload_moment_tables(P, g);
  if (st != EXX_OK) return st;
  P->geo = g;
  std::memcpy(P->h, h, sizeof(P->h));
  P->cell_strain = cell_strain(h, P->h0);
  return EXX_OK;
}

// Pairs per batch of an evaluation over `span` rows of the processing order:
// as many as the workspace cap (exx_options.workspace_gb) holds.
long long eval_batch(exx_plan_t P, long long span) {
  const long long per_pair = 2 * P->rstride + P->max_halo + kMaxLM;
  const double budget = (P->opt.workspace_gb > 0 ? P->opt.workspace_gb : 24.0) * 1e9;
  long long batch = std::max<long long>(1, (long long)(budget / (8.0 * per_pair)));
  batch = std::min<long long>(batch, std::max<long long>(span, 1));
  return std::min<long long>(batch, 65535);   // pair index on grid y of the per-point kernels
}

// ---------------------------------------------------------------------------
// The scratch array of exx_eval_noalloc: the whole device workspace of an
// evaluation (pair list, per-pair results, batch workspace, CG slots) in one
// file-scope array that every plan on a device shares.  Host code never names
// it in a kernel argument or copy: its device address on each device comes
// from hipGetSymbolAddress, looked up once per device when a plan is made.
constexpr size_t kScratchBytes = (size_t)EXX_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 256;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
std::string g_scratch_err[kMaxDevices];

// Looks up the scratch array's address on the current device dev (once).
void scratch_lookup(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] || !g_scratch_err[dev].empty()) return;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    g_scratch_err[dev] = std::string("hipGetSymbolAddress of the scratch array failed: ") + hipGetErrorString(e);
  else
    g_scratch_ptr[dev] = ptr;
}

// Pieces of the scratch array (from base; base null: sizes only) for n_orb
// orbitals, the plan's pair capacity, k batch rows and g CG slots.  Returns
// the bytes the layout spans.
size_t scratch_carve(exx_plan_t P, char* base, int n_orb, long long k, int g, EvalWork* w) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    off = (off + 255) & ~(size_t)255;
    char* p = base ? base + off : nullptr;
    off += bytes;
    return p;
  };
  const long long cap = P->opt.max_pairs;
  const int ncls = (int)P->classes.size();
  w->orb_cap = n_orb;
  w->pair_count = (int*)take(sizeof(int) * ((size_t)2 * n_orb + 1 + kMaxClasses));
  w->d_slot = (int*)take(sizeof(int) * (size_t)n_orb);
  w->n_eff = (int*)take(sizeof(int));
  w->pair_cap = cap;
  w->pairs = (PairDev*)take(sizeof(PairDev) * (size_t)cap);
  w->order = (int*)take(sizeof(int) * (size_t)cap);
  w->pE = (double*)take(sizeof(double) * (size_t)cap);
  w->pS = (double*)take(sizeof(double) * 9 * (size_t)cap);
  w->pIt = (int*)take(sizeof(int) * (size_t)cap);
  w->pRes = (double*)take(sizeof(double) * (size_t)cap);
  w->pUpd = (int*)take(sizeof(int) * (size_t)cap);
  w->pSav = (int*)take(sizeof(int) * (size_t)cap);
  w->pExit = (int*)take(sizeof(int) * (size_t)cap);
  w->batch_cap = k;
  w->rho_ws = (double*)take(sizeof(double) * (size_t)(k * P->rstride));
  w->bx_ws = (double*)take(sizeof(double) * (size_t)(k * P->rstride));
  w->halo_ws = (double*)take(sizeof(double) * (size_t)(k * std::max<long long>(P->max_halo, 1)));
  w->Q_ws = (double*)take(sizeof(double) * (size_t)(k * kMaxLM));
  w->rho_scale = (double*)take(sizeof(double) * (size_t)k);
  // partial moments of the point chunks: full batches and the last one, as exx_eval sizes them
  const long long tail = cap % k;
  w->qp_rows = std::max<long long>(moment_splits(k, ncls, P->max_pe) * k,
                                   tail ? moment_splits(tail, ncls, P->max_pe) * tail : 0);
  w->Qp_ws = (double*)take(sizeof(double) * (size_t)(w->qp_rows * kMaxLM));
  w->n_slots = g;
  w->slot_ws =
      take((size_t)g * (size_t)solve_slot_bytes(P->opt.precision == EXX_PREC_MIXED, slot_stride(P)));
  return off;
}

}  // namespace

extern "C" {

void exx_default_options(exx_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->stencil_n = 3;
  o->precision = EXX_PREC_FP64;
  o->cg_tol = 1e-10;
  o->cg_max_iter = 5000;
  o->pair_sample_frac = 1.0;
}

exx_status exx_plan(const double h[9], const int grid[3], double R_pair, double R_PE, double R_ME, int l_max,
                    const exx_options* opt_in, exx_plan_t* out) {
  if (!out) return fail(nullptr, EXX_EINVAL, "out is NULL");
  *out = nullptr;
  if (!h || !grid) return fail(nullptr, EXX_EINVAL, "h or grid is NULL");
  exx_options opt;
  if (opt_in) opt = *opt_in; else exx_default_options(&opt);
  for (int k = 0; k < 9; ++k)
    if (!std::isfinite(h[k])) return fail(nullptr, EXX_EINVAL, "cell tensor is not finite");
  bool general = false;   // any off-diagonal element: the NK Laplacian of Sec. III C
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c)
      if (r != c && h[r + 3 * c] != 0.0) general = true;
  for (int a = 0; a < 3; ++a) {
    if (!general && !(h[a + 3 * a] > 0.0)) return fail(nullptr, EXX_EINVAL, "cell edges must be positive");
    if (grid[a] <= 0 || grid[a] > 32000) return fail(nullptr, EXX_EINVAL, "grid dimensions out of range");
  }
  if (general && !(det3(h) > 0.0))
    return fail(nullptr, EXX_EINVAL, "the cell tensor must have a positive determinant (right-handed L_1, L_2, L_3)");
  if (!(R_pair >= 0.0) || !(R_PE > 0.0) || !(R_ME >= R_PE)) return fail(nullptr, EXX_EINVAL, "radii out of range");
  if (l_max < 0 || l_max > kMaxL) return fail(nullptr, EXX_EINVAL, "l_max must be in [0, 8]");
  if (opt.stencil_n < 1 || opt.stencil_n > 3) return fail(nullptr, EXX_EINVAL, "stencil_n must be 1, 2 or 3");
  if (!(opt.cg_tol > 0.0) || opt.cg_max_iter < 1) return fail(nullptr, EXX_EINVAL, "CG tolerance/iterations invalid");
  if (!(opt.refine_delta >= 0.0 && opt.refine_delta < 1.0))
    return fail(nullptr, EXX_EINVAL, "refine_delta must lie in [0, 1)");
  if (opt.precision != EXX_PREC_FP64 && opt.precision != EXX_PREC_MIXED)
    return fail(nullptr, EXX_EINVAL, "unknown precision");
  if (opt.R_PE_nclass < 0 || opt.R_PE_nclass > kMaxClasses) return fail(nullptr, EXX_EINVAL, "R_PE_nclass out of range");
  if (opt.R_PE_nclass > 0 && (!(opt.R_PE_min > 0.0) || !(opt.R_PE_step > 0.0)))
    return fail(nullptr, EXX_EINVAL, "variable radii need R_PE_min > 0 and R_PE_step > 0");
  if (opt.R_PE_nclass > 0 && (opt.R_PE_self > 0.0 || opt.R_ME_self > 0.0))
    return fail(nullptr, EXX_EINVAL, "self radii are not combined with variable radii");
  if (opt.R_PE_nclass + (opt.R_PE_self > 0.0 || opt.R_ME_self > 0.0 ? 1 : 0) > kMaxClasses)
    return fail(nullptr, EXX_EINVAL, "too many sphere classes");
  if (opt.max_pairs < 0 || opt.workspace_gb < 0 || opt.solve_groups < 0)
    return fail(nullptr, EXX_EINVAL, "negative capacity option");
  if (opt.solve_threads != 0 && opt.solve_threads != 512 && opt.solve_threads != 768 && opt.solve_threads != 1024)
    return fail(nullptr, EXX_EINVAL, "solve_threads must be 0, 512, 768 or 1024");
  if (opt.solve_depth < 0 || opt.solve_depth > 2) return fail(nullptr, EXX_EINVAL, "solve_depth must be 0, 1 or 2");
  if (opt.warm_start != 0 && opt.warm_start != 1) return fail(nullptr, EXX_EINVAL, "warm_start must be 0 or 1");
  if (opt.warm_start && opt.max_pairs <= 0)
    return fail(nullptr, EXX_EINVAL, "warm_start needs a fixed pair capacity (max_pairs > 0)");
  if (opt.cell_fluctuation != 0 && opt.cell_fluctuation != 1)
    return fail(nullptr, EXX_EINVAL, "cell_fluctuation must be 0 or 1");
  if (!(opt.reassemble_strain >= 0.0) || !std::isfinite(opt.reassemble_strain))
    return fail(nullptr, EXX_EINVAL, "reassemble_strain must be >= 0");
  if (opt.cg_layout < 0 || opt.cg_layout > 2) return fail(nullptr, EXX_EINVAL, "cg_layout must be 0, 1 or 2");
  if (opt.cg_layout == 2 && opt.cell_fluctuation)
    return fail(nullptr, EXX_EINVAL, "the quad layout (cg_layout 2) is not combined with cell_fluctuation");

  exx_plan_t P = new (std::nothrow) exx_plan_s();
  if (!P) return fail(nullptr, EXX_ENOMEM, "host allocation failed");
  P->opt = opt;
  std::memcpy(P->h, h, sizeof(P->h));
  std::memcpy(P->grid, grid, sizeof(P->grid));
  P->R_pair = R_pair;
  P->R_PE = R_PE;
  P->R_ME = R_ME;
  P->l_max = l_max;

  Geo& g = P->geo;
  std::memset(&g, 0, sizeof(g));
  for (int a = 0; a < 3; ++a) g.N[a] = grid[a];
  g.ngrid = (long long)grid[0] * grid[1] * grid[2];
  stencil_weights(opt.stencil_n, g.w2, g.w1);
  g.n = opt.stencil_n;
  g.l_max = l_max;
  g.n_lm = (l_max + 1) * (l_max + 1);
  harmonic_norms(l_max, g.ylm_norm);
  {
    exx_status st = assemble_cell(P, h);
    if (st != EXX_OK) {
      std::string m = P->err;
      free_plan(P);
      return fail(nullptr, st, m);
    }
  }
  for (auto& e : P->ev)
    if (hipEventCreate(&e) != hipSuccess) {
      free_plan(P);
      return fail(nullptr, EXX_EDEVICE, "event creation failed");
    }
  if (hipMalloc(&P->queue, sizeof(int)) != hipSuccess || hipMalloc(&P->stats_dev, kStatsLen * sizeof(double)) != hipSuccess) {
    free_plan(P);
    return fail(nullptr, EXX_ENOMEM, "device allocation failed");
  }
  // the device address of exx_eval_noalloc's scratch array on this device
  // (a failure is reported by exx_eval_noalloc; exx_eval does not need it)
  scratch_lookup(P->device);
  int cus = 0;
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, P->device);
  P->n_cus = std::max(1, cus);
  {
    // defaults measured on MI355X: FP64 1024 x 1, mixed 1024 x 2
    default_solve_variants(P);
    exx_status st = apply_solve_variants(P);
    if (st != EXX_OK) {
      std::string m = P->err;
      free_plan(P);
      return fail(nullptr, st, m);
    }
  }
  *out = P;
  return EXX_OK;
}

exx_status exx_set_cell(exx_plan_t P, const double h[9]) {
  if (!P) return fail(nullptr, EXX_EINVAL, "plan is NULL");
  if (!h) return fail(P, EXX_EINVAL, "h is NULL");
  for (int k = 0; k < 9; ++k)
    if (!std::isfinite(h[k])) return fail(P, EXX_EINVAL, "cell tensor is not finite");
  if (!(det3(h) > 0.0))
    return fail(P, EXX_EINVAL, "the cell tensor must have a positive determinant (right-handed L_1, L_2, L_3)");
  int dev = -1;
  EXX_HIP(P, hipGetDevice(&dev));
  if (dev != P->device) return fail(P, EXX_EINVAL, "current device differs from the plan's device");
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  EXX_HIP(P, hipStreamIsCapturing(P->stream, &cs));
  if (cs != hipStreamCaptureStatusNone) return fail(P, EXX_EINVAL, "exx_set_cell is not capturable");
  // the tables are rewritten: no evaluation may still read them
  EXX_HIP(P, hipStreamSynchronize(P->stream));
  use_own_work(P);
  if (P->opt.reassemble_strain > 0.0 && cell_strain(h, P->h0) > P->opt.reassemble_strain) {
    // re-assembly (Sec. III B 2): new proto-subdomains for h from the plan's radii
    exx_status st = assemble_cell(P, h);
    if (st != EXX_OK) return st;
    // workspaces, CG slots and warm-start stores are sized for the old tables
    // and are made again by the next eval, which also drops the warm-start
    // history; graphs need a new eager call
    P->batch_cap = 0;
    P->qp_rows = 0;
    if (P->slot_ws) (void)hipFree(P->slot_ws);
    P->slot_ws = nullptr;
    P->warm_cap = 0;
    P->warm_orb = 0;
    P->tuned = false;
    default_solve_variants(P);
    st = apply_solve_variants(P);
    if (st != EXX_OK) return st;
    P->reassemblies++;
    return EXX_OK;
  }
  return update_cell(P, h);
}

exx_status exx_pressure(const double h[9], const double sigma[9], double* Pi, double* p_int) {
  if (!h || !sigma) return fail(nullptr, EXX_EINVAL, "h or sigma is NULL");
  const double V = std::fabs(det3(h));
  if (!(V > 0.0) || !std::isfinite(V)) return fail(nullptr, EXX_EINVAL, "singular cell");
  double T[9];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      double s = 0.0;
      for (int al = 0; al < 3; ++al) s += sigma[a + 3 * al] * h[b + 3 * al];
      T[a + 3 * b] = -s / V;   // eq. pixx_working
    }
  if (Pi) std::memcpy(Pi, T, sizeof(T));
  if (p_int) *p_int = (T[0] + T[4] + T[8]) / 3.0;   // eq. pxx_working
  return EXX_OK;
}

exx_status exx_set_stream(exx_plan_t P, void* s) {
  if (!P) return fail(nullptr, EXX_EINVAL, "plan is NULL");
  P->stream = (hipStream_t)s;
  return EXX_OK;
}

exx_status exx_eval(exx_plan_t P, int n_orb, const void* orbitals, exx_dtype dt, const double* centres,
                    const double* R_PE_orb, const int* d_subset, int n_subset, double* E_xx, void* D_xx,
                    double* sigma) {
  if (!P) return fail(nullptr, EXX_EINVAL, "plan is NULL");
  if (n_orb < 1) return fail(P, EXX_EINVAL, "n_orb must be >= 1");
  if (!orbitals || !centres || !E_xx) return fail(P, EXX_EINVAL, "orbitals, centres and E_xx are required");
  if (dt != EXX_F64 && dt != EXX_F32) return fail(P, EXX_EINVAL, "unknown dtype");
  if (P->opt.R_PE_nclass > 0 && !R_PE_orb)
    return fail(P, EXX_EINVAL, "variable radii need per-orbital radii (R_PE_orb)");
  if (n_subset < 0 || n_subset > n_orb || (n_subset > 0 && !d_subset))
    return fail(P, EXX_EINVAL, "d_subset must hold n_subset (0 .. n_orb) orbital indices");
  const Geo& g = P->geo;
  hipStream_t s = P->stream;
  int dev = -1;
  EXX_HIP(P, hipGetDevice(&dev));
  if (dev != P->device) return fail(P, EXX_EINVAL, "current device differs from the plan's device");
  hipStreamCaptureStatus cap_status = hipStreamCaptureStatusNone;
  EXX_HIP(P, hipStreamIsCapturing(s, &cap_status));
  const bool capturing = cap_status != hipStreamCaptureStatusNone;
  const bool fixed = P->opt.max_pairs > 0;
  if (capturing) {
    if (!fixed) return fail(P, EXX_EINVAL, "recording exx_eval in a graph needs a fixed pair capacity (max_pairs > 0)");
    // (exx_eval_noalloc sizes its scratch layout in the call itself)
    if (n_orb > P->warm_orb && !P->no_alloc)
      return fail(P, EXX_EINVAL, "recording exx_eval in a graph needs one eager exx_eval with at least as many "
                                 "orbitals first");
  } else if (P->timing_valid && !P->harvested) {
    EXX_HIP(P, hipEventSynchronize(P->ev[3]));
    exx_status hs = harvest(P);
    if (hs != EXX_OK) return hs;
  }
  if (!P->no_alloc) use_own_work(P);
  P->timing_valid = false;
  P->last_captured = capturing;
  P->solve_ev_used = 0;
  P->mom_ev_used = 0;
  CaptureGuard guard(P, capturing);   // dev_alloc refuses while the stream is captured
  auto event = [&](hipEvent_t e) { return capturing ? hipSuccess : hipEventRecord(e, s); };

  // pair list
  if (n_orb > P->orb_cap) {
    if (dev_alloc(P, &P->pair_count, (size_t)2 * n_orb + 1 + kMaxClasses, "pair counts") ||
        dev_alloc(P, &P->d_slot, (size_t)n_orb, "D subset slots"))
      return EXX_ENOMEM;
    P->orb_cap = n_orb;
  }
  if (!P->n_eff) {
    if (dev_alloc(P, &P->n_eff, 1, "pair count")) return EXX_ENOMEM;
  }
  PairParams pp;
  pp.R_pair2 = P->R_pair * P->R_pair * (1.0 + kSlack);
  pp.R_PE = P->R_PE;
  pp.R_min = P->opt.R_PE_min;
  pp.R_step = P->opt.R_PE_step;
  pp.n_class = P->opt.R_PE_nclass;
  pp.self_class = P->self_class;
  pp.seed = P->opt.pair_sample_seed;
  pp.frac = P->opt.pair_sample_frac;
  EXX_HIP(P, event(P->ev[0]));
  auto alloc_pairs = [&](long long cap) -> exx_status {
    if (dev_alloc(P, &P->pairs, (size_t)cap, "pairs") || dev_alloc(P, &P->order, (size_t)cap, "order") ||
        dev_alloc(P, &P->pE, (size_t)cap, "pair E") || dev_alloc(P, &P->pS, (size_t)9 * cap, "pair sigma") ||
        dev_alloc(P, &P->pIt, (size_t)cap, "pair iters") || dev_alloc(P, &P->pRes, (size_t)cap, "pair res") ||
        dev_alloc(P, &P->pUpd, (size_t)cap, "pair updates") || dev_alloc(P, &P->pSav, (size_t)cap, "pair saved sweeps") ||
        dev_alloc(P, &P->pExit, (size_t)cap, "pair exit reasons"))
      return EXX_ENOMEM;
    P->pair_cap = cap;
    return EXX_OK;
  };
  if (fixed && P->pair_cap < P->opt.max_pairs) {
    if (alloc_pairs(P->opt.max_pairs) != EXX_OK) return EXX_ENOMEM;
  }
  EXX_HIP(P, launch_pairlist(g, pp, centres, R_PE_orb, n_orb, P->pair_count, P->pairs, P->pair_cap, s));
  // rows of the processing order that the batch loop covers: the capacity,
  // or (without one) the pair count, read back once to size the workspace
  long long span = P->pair_cap;
  if (!fixed) {
    int total = 0;
    EXX_HIP(P, hipMemcpyAsync(&total, P->pair_count + 2 * n_orb, sizeof(int), hipMemcpyDeviceToHost, s));
    EXX_HIP(P, hipStreamSynchronize(s));
    if (total < 0) return fail(P, EXX_EINVAL, "pair count overflow");
    if (total > P->pair_cap) {
      if (alloc_pairs(std::max<long long>(total, 1) + total / 8) != EXX_OK) return EXX_ENOMEM;
      EXX_HIP(P, launch_pairlist(g, pp, centres, R_PE_orb, n_orb, P->pair_count, P->pairs, P->pair_cap, s));
    }
    span = total;
  }
  P->last_n_orb = n_orb;
  const int ncls = (int)P->classes.size();
  EXX_HIP(P, launch_order(P->pairs, P->pair_count, n_orb, ncls, P->order, P->pair_cap, P->n_eff, s));
  EXX_HIP(P, event(P->ev[4]));
  if (P->opt.warm_start) {
    // the stores and the previous list keep their contents between calls;
    // they are (re)made only when the capacity grows, which drops the history
    if (P->warm_cap < P->pair_cap || !P->warm_state) {
      if (dev_alloc(P, &P->warm_store, (size_t)2 * P->pair_cap * P->rstride, "warm-start solutions") ||
          dev_alloc(P, &P->warm_map, (size_t)P->pair_cap, "warm-start map") ||
          dev_alloc(P, &P->prev_pairs, (size_t)P->pair_cap, "previous pairs") ||
          dev_alloc(P, &P->warm_state, 4, "warm-start state"))
        return EXX_ENOMEM;
      P->warm_cap = P->pair_cap;
      EXX_HIP(P, launch_zero(P->warm_state, 4 * sizeof(int), s));
    }
    if (n_orb + 1 > P->warm_orb_cap) {
      if (dev_alloc(P, &P->prev_offs, (size_t)n_orb + 1, "previous offsets")) return EXX_ENOMEM;
      P->warm_orb_cap = n_orb + 1;
      EXX_HIP(P, launch_zero(P->warm_state, 4 * sizeof(int), s));   // no usable previous list
    }
    EXX_HIP(P, launch_warm_match(g, P->pairs, P->n_eff, P->pair_cap, P->prev_pairs, P->prev_offs, P->warm_state,
                                 P->warm_map, s));
  }

  // workspace
  long long batch = eval_batch(P, span);
  if (P->batch_limit > 0) batch = std::min<long long>(batch, P->batch_limit);   // rows of the scratch layout
  if (batch > P->batch_cap) {
    if (dev_alloc(P, &P->rho_ws, (size_t)batch * P->rstride, "pair densities") ||
        dev_alloc(P, &P->bx_ws, (size_t)batch * P->rstride, "pair potentials") ||
        dev_alloc(P, &P->halo_ws, (size_t)batch * std::max<long long>(P->max_halo, 1), "boundary values") ||
        dev_alloc(P, &P->Q_ws, (size_t)batch * kMaxLM, "moments") ||
        dev_alloc(P, &P->rho_scale, (size_t)batch, "density scales"))
      return EXX_ENOMEM;
    P->batch_cap = batch;
  }
  {
    // partial moments of the point chunks: the full batches and the last one
    const long long tail = span % batch;
    const long long rows = std::max<long long>(moment_splits(batch, ncls, P->max_pe) * batch,
                                               tail ? moment_splits(tail, ncls, P->max_pe) * tail : 0);
    if (rows > P->qp_rows) {
      if (dev_alloc(P, &P->Qp_ws, (size_t)rows * kMaxLM, "partial moments")) return EXX_ENOMEM;
      P->qp_rows = rows;
    }
  }
  {
    exx_status st = ensure_slots(P);
    if (st != EXX_OK) return st;
  }

  const int* d_slot = nullptr;
  if (D_xx) {
    const long long rows = d_subset ? n_subset : n_orb;
    if (d_subset) {
      EXX_HIP(P, launch_dslot(P->d_slot, n_orb, d_subset, n_subset, s));
      d_slot = P->d_slot;
    }
    EXX_HIP(P, launch_zero(D_xx, (size_t)rows * g.ngrid * (dt == EXX_F64 ? 8 : 4), s));
  }
  EXX_HIP(P, event(P->ev[1]));
  const bool mixed = P->opt.precision == EXX_PREC_MIXED;
  for (long long p0 = 0; p0 < span; p0 += batch) {
    Batch B;
    B.cls = P->class_dev;
    B.pairs = P->pairs;
    B.order = P->order;
    B.n_eff = P->n_eff;
    B.p0 = p0;
    B.nb = std::min(batch, span - p0);
    EXX_HIP(P, launch_gather(g, B, orbitals, (int)dt, P->rho_ws, P->rstride, P->rho_scale, s));
    // (exx_eval_noalloc records no per-launch events: new ones would be created)
    const bool launch_events = !capturing && !P->no_alloc;
    if (launch_events) { exx_status es = record_moment_event(P, s); if (es != EXX_OK) return es; }
    EXX_HIP(P, launch_moments(g, B, P->pair_count + 2 * n_orb + 1, ncls, mixed, P->rho_ws, P->rstride, P->rho_scale,
                              P->Qp_ws, moment_splits(B.nb, ncls, P->max_pe), P->Q_ws, s));
    if (launch_events) { exx_status es = record_moment_event(P, s); if (es != EXX_OK) return es; }
    EXX_HIP(P, launch_boundary(g, B, P->pair_count + 2 * n_orb + 1, ncls, P->max_halo, P->Q_ws, P->halo_ws,
                               std::max<long long>(P->max_halo, 1), s));
    SolveArgs a;
    a.g = g;
    a.cls = P->class_dev;
    a.pairs = P->pairs;
    a.order = P->order;
    a.p0 = p0;
    a.npair = B.nb;
    a.n_eff = P->n_eff;
    a.queue = P->queue;
    a.bx_ws = P->bx_ws;
    a.rstride = P->rstride;
    a.slot_ws = P->slot_ws;
    a.sstride = slot_stride(P);
    a.outIt = P->pIt;
    a.outRes = P->pRes;
    a.outUpd = P->pUpd;
    a.outSav = P->pSav;
    a.outExit = P->pExit;
    a.mixed = mixed;
    a.delta = P->opt.refine_delta > 0.0 ? P->opt.refine_delta : 0.01;
    a.threads = P->solve_threads;
    a.depth = P->solve_depth;
    a.tol = P->opt.cg_tol;
    a.max_iter = P->opt.cg_max_iter;
    if (P->opt.warm_start) {
      a.warm_store = P->warm_store;
      a.warm_cap = P->warm_cap;
      a.warm_state = P->warm_state;
      a.warm_map = P->warm_map;
      a.prev_pairs = P->prev_pairs;
    }
    if (P->opt.autotune && !P->tuned && !P->no_alloc) {   // (exx_eval_noalloc keeps the variants it finds)
      if (capturing) return fail(P, EXX_EINVAL, "the autotuner runs in an eager exx_eval, not in a graph");
      exx_status st = autotune_solve(P, a, B.nb, s);
      if (st != EXX_OK) return st;
      a.slot_ws = P->slot_ws;
      a.threads = P->solve_threads;
      a.depth = P->solve_depth;
    }
    EXX_HIP(P, launch_rhs(g, B, P->max_pe, P->rho_ws, P->bx_ws, P->rstride, P->halo_ws,
                          std::max<long long>(P->max_halo, 1), s));
    if (launch_events) { exx_status es = record_solve_event(P, s); if (es != EXX_OK) return es; }
    { exx_status es = launch_solves(P, a, s); if (es != EXX_OK) return es; }
    if (launch_events) { exx_status es = record_solve_event(P, s); if (es != EXX_OK) return es; }
    if (finalize_sweep_supported(g, P->max_fin))
      EXX_HIP(P, launch_finalize_sweep(g, B, P->max_fin, P->rho_ws, P->bx_ws, P->rstride, P->halo_ws,
                                       std::max<long long>(P->max_halo, 1), P->pE, P->pS, s));
    else
      EXX_HIP(P, launch_finalize(g, B, P->rho_ws, P->bx_ws, P->rstride, P->halo_ws,
                                 std::max<long long>(P->max_halo, 1), P->pE, P->pS, s));
    if (D_xx)
      EXX_HIP(P, launch_dscatter(g, B, P->max_me, orbitals, D_xx, d_slot, (int)dt, P->bx_ws, P->rstride, P->Q_ws, s));
  }
  EXX_HIP(P, event(P->ev[2]));
  EXX_HIP(P, launch_reduce(P->pE, P->pS, P->pIt, P->pRes, P->pUpd, P->pSav, P->pExit, P->pairs, P->class_dev,
                           P->pair_count, n_orb, P->n_eff, P->opt.warm_start ? P->warm_map : nullptr, E_xx, sigma,
                           P->stats_dev, s));
  if (P->opt.warm_start)
    EXX_HIP(P, launch_warm_commit(P->pairs, P->pair_count, n_orb, P->n_eff, P->pair_cap, P->prev_pairs, P->prev_offs,
                                  P->warm_state, s));
  EXX_HIP(P, event(P->ev[3]));
  if (!capturing) {
    P->timing_valid = true;
    P->harvested = false;
    if (fixed && !P->no_alloc) P->warm_orb = std::max(P->warm_orb, n_orb);
  }
  return EXX_OK;
}

exx_status exx_eval_noalloc(exx_plan_t P, int n_orb, const void* orbitals, exx_dtype dt, const double* centres,
                            const double* R_PE_orb, const int* d_subset, int n_subset, double* E_xx, void* D_xx,
                            double* sigma) {
  if (!P) return fail(nullptr, EXX_EINVAL, "plan is NULL");
  if (P->opt.max_pairs <= 0)
    return fail(P, EXX_EINVAL, "exx_eval_noalloc needs a plan with a fixed pair capacity (max_pairs > 0)");
  if (P->opt.warm_start)
    return fail(P, EXX_EINVAL, "exx_eval_noalloc keeps no warm-start stores (make the plan without warm_start)");
  if (n_orb < 1) return fail(P, EXX_EINVAL, "n_orb must be >= 1");
  int dev = -1;
  EXX_HIP(P, hipGetDevice(&dev));
  if (dev != P->device) return fail(P, EXX_EINVAL, "current device differs from the plan's device");
  char* base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (dev >= 0 && dev < kMaxDevices) base = (char*)g_scratch_ptr[dev];
    if (!base)
      return fail(P, EXX_EDEVICE, dev >= 0 && dev < kMaxDevices && !g_scratch_err[dev].empty()
                                      ? g_scratch_err[dev]
                                      : std::string("no scratch array address for this device"));
  }
  hipStreamCaptureStatus cap_status = hipStreamCaptureStatusNone;
  EXX_HIP(P, hipStreamIsCapturing(P->stream, &cap_status));
  if (cap_status == hipStreamCaptureStatusNone && P->timing_valid && !P->harvested) {
    // the previous evaluation's statistics, from the workspace it used
    EXX_HIP(P, hipEventSynchronize(P->ev[3]));
    exx_status hs = harvest(P);
    if (hs != EXX_OK) return hs;
  }
  // the largest batch (and as many CG slots, up to the plan's solve grid) that
  // the scratch array holds
  int max_groups = 1;
  for (int g : P->class_groups) max_groups = std::max(max_groups, g);
  const long long span = P->opt.max_pairs;
  long long lo = 1, hi = std::max<long long>(1, eval_batch(P, span));
  EvalWork w;
  auto bytes_for = [&](long long k) {
    return scratch_carve(P, nullptr, n_orb, k, (int)std::min<long long>(k, max_groups), &w);
  };
  if (bytes_for(1) > kScratchBytes)
    return fail(P, EXX_EINVAL, "exx_eval_noalloc: one pair's workspace with " + std::to_string(n_orb) +
                                   " orbitals and max_pairs " + std::to_string(span) + " needs " +
                                   std::to_string(bytes_for(1)) + " bytes, beyond the scratch array's " +
                                   std::to_string(kScratchBytes));
  while (lo < hi) {   // largest k in [1, hi] that fits
    const long long mid = (lo + hi + 1) / 2;
    if (bytes_for(mid) <= kScratchBytes) lo = mid; else hi = mid - 1;
  }
  const long long k = lo;
  const int g = (int)std::min<long long>(k, max_groups);
  scratch_carve(P, base, n_orb, k, g, &w);
  if (!P->on_scratch) {
    P->own_work = get_work(P);
    P->on_scratch = true;
  }
  put_work(P, w);
  P->no_alloc = true;
  P->batch_limit = k;
  P->slot_limit = g;
  const exx_status st = exx_eval(P, n_orb, orbitals, dt, centres, R_PE_orb, d_subset, n_subset, E_xx, D_xx, sigma);
  P->no_alloc = false;
  P->batch_limit = 0;
  P->slot_limit = 0;
  return st;
}

exx_status exx_count_pairs(exx_plan_t P, int n_orb, const double* centres, const double* R_PE_orb,
                           long long* n_pairs) {
  if (!P || !n_pairs) return fail(P, EXX_EINVAL, "plan or n_pairs is NULL");
  if (n_orb < 1 || !centres) return fail(P, EXX_EINVAL, "n_orb >= 1 and centres are required");
  if (P->opt.R_PE_nclass > 0 && !R_PE_orb)
    return fail(P, EXX_EINVAL, "variable radii need per-orbital radii (R_PE_orb)");
  int dev = -1;
  EXX_HIP(P, hipGetDevice(&dev));
  if (dev != P->device) return fail(P, EXX_EINVAL, "current device differs from the plan's device");
  hipStreamCaptureStatus cap_status = hipStreamCaptureStatusNone;
  EXX_HIP(P, hipStreamIsCapturing(P->stream, &cap_status));
  if (cap_status != hipStreamCaptureStatusNone) return fail(P, EXX_EINVAL, "exx_count_pairs waits on the host");
  if (P->timing_valid && !P->harvested) {   // keep the last evaluation's statistics
    EXX_HIP(P, hipEventSynchronize(P->ev[3]));
    exx_status hs = harvest(P);
    if (hs != EXX_OK) return hs;
  }
  use_own_work(P);
  if (n_orb > P->orb_cap) {
    if (dev_alloc(P, &P->pair_count, (size_t)2 * n_orb + 1 + kMaxClasses, "pair counts") ||
        dev_alloc(P, &P->d_slot, (size_t)n_orb, "D subset slots"))
      return EXX_ENOMEM;
    P->orb_cap = n_orb;
  }
  PairParams pp;
  pp.R_pair2 = P->R_pair * P->R_pair * (1.0 + kSlack);
  pp.R_PE = P->R_PE;
  pp.R_min = P->opt.R_PE_min;
  pp.R_step = P->opt.R_PE_step;
  pp.n_class = P->opt.R_PE_nclass;
  pp.self_class = P->self_class;
  pp.seed = P->opt.pair_sample_seed;
  pp.frac = P->opt.pair_sample_frac;
  // capacity 0: count and scan only, nothing is stored
  EXX_HIP(P, launch_pairlist(P->geo, pp, centres, R_PE_orb, n_orb, P->pair_count, nullptr, 0, P->stream));
  int total = 0;
  EXX_HIP(P, hipMemcpyAsync(&total, P->pair_count + 2 * n_orb, sizeof(int), hipMemcpyDeviceToHost, P->stream));
  EXX_HIP(P, hipStreamSynchronize(P->stream));
  *n_pairs = total;
  return EXX_OK;
}

exx_status exx_pair_results(exx_plan_t P, long long cap, int* ij, double* E, double* sigma, int* iters,
                            double* rel_res, int* exit_code, int* updates, long long* n_pairs) {
  if (!P) return fail(nullptr, EXX_EINVAL, "plan is NULL");
  EXX_HIP(P, hipStreamSynchronize(P->stream));
  int stored = 0;
  if (P->n_eff) EXX_HIP(P, hipMemcpy(&stored, P->n_eff, sizeof(int), hipMemcpyDeviceToHost));
  const long long n = std::min<long long>(stored, std::max<long long>(cap, 0));
  if (n_pairs) *n_pairs = stored;
  if (n <= 0) return EXX_OK;
  if (ij) {
    std::vector<PairDev> pd((size_t)n);
    EXX_HIP(P, hipMemcpy(pd.data(), P->pairs, sizeof(PairDev) * n, hipMemcpyDeviceToHost));
    for (long long k = 0; k < n; ++k) {
      ij[2 * k] = pd[k].i;
      ij[2 * k + 1] = pd[k].j;
    }
  }
  if (E) EXX_HIP(P, hipMemcpy(E, P->pE, sizeof(double) * n, hipMemcpyDeviceToHost));
  if (sigma) EXX_HIP(P, hipMemcpy(sigma, P->pS, sizeof(double) * 9 * n, hipMemcpyDeviceToHost));
  if (iters) EXX_HIP(P, hipMemcpy(iters, P->pIt, sizeof(int) * n, hipMemcpyDeviceToHost));
  if (rel_res) EXX_HIP(P, hipMemcpy(rel_res, P->pRes, sizeof(double) * n, hipMemcpyDeviceToHost));
  if (exit_code) EXX_HIP(P, hipMemcpy(exit_code, P->pExit, sizeof(int) * n, hipMemcpyDeviceToHost));
  if (updates) EXX_HIP(P, hipMemcpy(updates, P->pUpd, sizeof(int) * n, hipMemcpyDeviceToHost));
  return EXX_OK;
}

exx_status exx_stats_fetch(exx_plan_t P, exx_stats* out) {
  if (!P || !out) return fail(P, EXX_EINVAL, "plan or out is NULL");
  std::memset(out, 0, sizeof(*out));
  EXX_HIP(P, hipStreamSynchronize(P->stream));
  if (!P->timing_valid && !P->last_captured) return fail(P, EXX_EINVAL, "no evaluation to report");
  if (P->timing_valid) {
    exx_status hs = harvest(P);
    if (hs != EXX_OK) return hs;
  } else {
    // the last call was recorded in a graph: device results of its latest replay, no timings
    exx_status hs = read_device_stats(P);
    if (hs != EXX_OK) return hs;
    P->last_solve_ms = P->last_eval_ms = P->last_moment_ms = 0.0;
    P->last_alg_bytes = P->last_stats[5] * 8.0 * (P->opt.precision == EXX_PREC_MIXED ? 4.0 : 8.0);
  }
  const double* st = P->last_stats;
  out->n_pairs = std::min<long long>((long long)st[4], P->pair_cap);
  out->cg_iter_sum = (long long)st[0];
  out->cg_iter_max = (int)st[1];
  out->n_unconverged = (int)st[2];
  out->max_rel_residual = st[3];
  out->n_classes = (int)P->classes.size();
  out->refine_passes_max = (int)st[6];
  out->solve_ms = P->last_solve_ms;
  out->eval_ms = P->last_eval_ms;
  out->cg_alg_bytes = P->last_alg_bytes;
  out->moment_flops = 2.0 * P->geo.n_lm * st[7];
  out->moment_ms = P->last_moment_ms;
  {
    // executed MFMA work: every point step of every pair, all padded rows
    const bool mixed = P->opt.precision == EXX_PREC_MIXED;
    double padded = 0.0;
    for (int k = 0; k < (int)P->classes.size(); ++k)
      padded += (double)P->last_class_pairs[k] * (double)((P->classes[k].n_pe + (mixed ? 31 : 15)) /
                                                            (mixed ? 32 : 16) * (mixed ? 32 : 16));
    int rows = 0, mrows = 0;
    moment_layout(P->geo.l_max, mixed, &rows, &mrows);
    out->moment_mfma_flops = 2.0 * mrows * padded * (mixed ? 3.0 : 1.0);
  }
  out->n_evals = P->n_evals;
  out->solve_launches = P->solve_launches;
  out->solve_ms_total = P->solve_ms_total;
  out->cg_alg_bytes_total = P->alg_bytes_total;
  out->eval_ms_total = P->eval_ms_total;
  out->cell_strain = P->cell_strain;
  out->reassemblies = P->reassemblies;
  out->n_arms = P->geo.gen ? P->geo.n_arms : 3;
  {
    int nq = 0;
    for (const ClassHost& C : P->classes) nq += C.quads ? 1 : 0;
    out->cg_layout = nq == 0 ? 1 : (nq == (int)P->classes.size() ? 2 : 3);
  }
  out->solve_threads = P->solve_threads;
  out->solve_depth = P->solve_depth;
  out->tune_ms = P->tune_ms;
  out->pairs_kept = (long long)st[4];
  out->graph_recorded = P->last_captured ? 1 : 0;
  out->warm_pairs = (long long)st[8];
  out->n_cg_cap = (int)st[9];
  out->n_cg_breakdown = (int)st[10];
  out->n_cg_nonfinite = (int)st[11];
  out->cg_restarts = (long long)st[12];
  out->t_pairlist_ms = P->last_pairlist_ms;
  out->t_reduce_ms = P->last_reduce_ms;
  for (int k = 0; k < (int)P->classes.size() && k < kMaxClasses; ++k) {
    out->class_threads[k] = P->class_threads[k];
    out->class_depth[k] = P->class_depth[k];
    out->class_layout[k] = P->classes[k].quads ? 2 : 1;
    out->class_pairs[k] = P->last_class_pairs[k];
    out->class_refine_delta[k] = P->opt.precision != EXX_PREC_MIXED ? 0.0
                                 : P->class_delta[k] > 0.0       ? P->class_delta[k]
                                 : P->opt.refine_delta > 0.0     ? P->opt.refine_delta
                                                                 : 0.01;
  }
  if (st[4] > (double)P->pair_cap)
    return fail(P, EXX_ECAPACITY, "more pairs than the fixed capacity (max_pairs); results cover the first ones");
  return out->n_unconverged > 0 ? fail(P, EXX_ENOCONV, "CG did not converge for some pairs") : EXX_OK;
}

exx_status exx_plan_geometry(exx_plan_t P, int cls, long long* n_pe, long long* n_halo, long long* n_me) {
  if (!P) return fail(nullptr, EXX_EINVAL, "plan is NULL");
  if (cls < 0 || cls >= (int)P->classes.size()) return fail(P, EXX_EINVAL, "class out of range");
  const ClassHost& C = P->classes[cls];
  if (n_pe) *n_pe = C.n_real;
  if (n_halo) *n_halo = C.n_halo;
  if (n_me) *n_me = C.n_me - (C.n_pe - C.n_real);   // without the dead slots of padded columns
  return EXX_OK;
}

exx_status exx_subdomain_counts(const double h[9], const int grid[3], double R_PE, double R_ME, int stencil_n,
                                long long* n_pe, long long* n_halo, long long* n_me) {
  if (!h || !grid) return fail(nullptr, EXX_EINVAL, "h or grid is NULL");
  bool general = false;
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c)
      if (r != c && h[r + 3 * c] != 0.0) general = true;
  if (stencil_n < 1 || stencil_n > 3 || !(R_PE > 0.0) || !(R_ME >= R_PE))
    return fail(nullptr, EXX_EINVAL, "invalid radii or stencil");
  double L[3];
  int N[3];
  for (int a = 0; a < 3; ++a) {
    L[a] = h[a + 3 * a];
    N[a] = grid[a];
    if ((!general && !(L[a] > 0.0)) || N[a] <= 0) return fail(nullptr, EXX_EINVAL, "invalid cell or grid");
  }
  ClassHost C;
  std::string e;
  if (general) {
    if (!(det3(h) > 0.0)) return fail(nullptr, EXX_EINVAL, "the cell tensor must have a positive determinant");
    std::vector<NkArm> arms;
    e = build_nk_arms(h, N, &arms);
    if (e.empty()) e = build_class_general(h, N, 2, R_PE, R_ME, stencil_n, arms, false, false, &C);
  } else {
    e = build_class(L, N, R_PE, R_ME, stencil_n, false, &C);
  }
  if (!e.empty()) return fail(nullptr, EXX_EINVAL, e);
  if (n_pe) *n_pe = C.n_real;
  if (n_halo) *n_halo = C.n_halo;
  if (n_me) *n_me = C.n_me - (C.n_pe - C.n_real);
  return EXX_OK;
}

exx_status exx_nk_stencil(const double h[9], const int grid[3], int* n_arms, int* u, double* beta, double* step) {
  if (!h || !grid || !n_arms) return fail(nullptr, EXX_EINVAL, "h, grid or n_arms is NULL");
  for (int a = 0; a < 3; ++a)
    if (grid[a] <= 0) return fail(nullptr, EXX_EINVAL, "invalid grid");
  std::vector<NkArm> arms;
  std::string e = build_nk_arms(h, grid, &arms);
  if (!e.empty()) return fail(nullptr, EXX_EINVAL, e);
  *n_arms = (int)arms.size();
  for (size_t k = 0; k < arms.size(); ++k) {
    for (int a = 0; a < 3; ++a)
      if (u) u[3 * k + a] = arms[k].u[a];
    if (beta) beta[k] = arms[k].beta;
    if (step) step[k] = arms[k].step;
  }
  return EXX_OK;
}

exx_status exx_destroy(exx_plan_t P) {
  if (!P) return EXX_OK;
  (void)hipStreamSynchronize(P->stream);
  free_plan(P);
  return EXX_OK;
}

const char* exx_last_error(exx_plan_t P) { return P ? P->err.c_str() : g_plan_error.c_str(); }

}  // extern "C"
