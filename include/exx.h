/*
 * exx.h -- C ABI of the MI355X (gfx950) exact-exchange pair kernel.
 *
 * The library evaluates the exact-exchange (EXX) energy E_xx, the orbital
 * forces D_xx^i and the cell derivatives sigma_xx of a set of real localized
 * orbitals, by the subdomain method of Ko, Santra and DiStasio (arXiv:2011.07209):
 * for every unique pair of orbitals whose centres lie within R_pair it forms
 * the pair density on a sphere of radius R_PE about the pair's grid centre,
 * sets far-field values on the shell R_PE < r <= R_ME from a multipole
 * expansion, solves the finite-difference Poisson equation on the sphere by
 * conjugate gradient, and accumulates E_xx, D_xx and sigma_xx.
 *
 * Units: bohr and Hartree.  Cell tensor h is column-major, h[a + 3*al] is the
 * Cartesian component a of lattice vector L_al (Sec. II B 1).  Grid arrays are
 * [N3][N2][N1] with the L_1 index fastest; grid point g sits at h (g / N).
 *
 * Ownership: the caller owns every buffer passed in or out; the plan owns its
 * tables and its device workspace.  Device pointers are HIP device (or managed)
 * memory on the device current when the plan was made.  Calls on one plan are
 * not thread-safe.  Errors are returned as status codes, never thrown; the
 * message of the last failure on a plan is available from exx_last_error().
 */
#ifndef EXX_H_
#define EXX_H_

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct exx_plan_s* exx_plan_t;

typedef enum {
  EXX_OK = 0,
  EXX_EINVAL = 1,      /* an argument is out of range or inconsistent            */
  EXX_ENOMEM = 2,      /* a device or host allocation failed                     */
  EXX_ENOCONV = 3,     /* at least one pair's CG did not converge: it hit
                          cg_max_iter, broke down, or met a non-finite norm
                          (exx_stats tells which; outputs are kept, each such
                          pair with its last FP64 solution)                    */
  EXX_EDEVICE = 4,     /* a HIP runtime call failed                              */
  EXX_ECAPACITY = 5    /* more pairs than the plan's fixed capacity              */
} exx_status;

typedef enum { EXX_F64 = 0, EXX_F32 = 1 } exx_dtype;

/* Why a pair's CG stopped (exx_pair_results exit_code, low byte; the bits
   above it count the mixed solve's restarts). */
typedef enum {
  EXX_CG_CONVERGED = 0,   /* ||b - A x|| <= cg_tol ||b|| (or b = 0)                  */
  EXX_CG_CAP = 1,         /* cg_max_iter iterations without converging                */
  EXX_CG_BREAKDOWN = 2,   /* p.Ap not positive and finite (in FP64 only a non-finite
                             input does this; the mixed solve first restarts from
                             its last FP64 solution, at most 3 times)                 */
  EXX_CG_NONFINITE = 3    /* a NaN or infinity in the right-hand side or in a
                             residual norm (mixed: after its restarts)                */
} exx_cg_exit;

typedef enum {
  EXX_PREC_FP64 = 0,   /* every step in double precision                          */
  EXX_PREC_MIXED = 1   /* FP32 stencil/vector work with FP64 dots and an FP64
                          residual-correction pass per solve                      */
} exx_precision;

typedef struct {
  int stencil_n;              /* half-width n of the axis stencils, 1..3 (Sec. III C,
                                 eq. d2_1; the paper's default is 3)               */
  int precision;              /* exx_precision                                      */
  double cg_tol;              /* stop when ||r||_2 <= cg_tol ||b||_2 (FP64 residual)  */
  int cg_max_iter;            /* per solve; hitting it is reported as EXX_ENOCONV
                                 (a pair that converges on its last permitted
                                 iteration counts as converged)                     */
  /* variable sphere radii: with per-orbital radii passed to exx_eval, the pair
     radius is the rung R_PE_min + k R_PE_step (k < R_PE_nclass) nearest to
     (R_i + R_j)/2; R_PE_nclass <= 0 keeps the single plan radius R_PE          */
  double R_PE_min, R_PE_step;
  int R_PE_nclass;
  /* deterministic pair subset: pair (i,j) is kept when the top 53 bits of one
     SplitMix64 output on the state seed ^ (i << 32) ^ j, read as a fraction,
     fall below pair_sample_frac; >= 1 keeps every pair                        */
  unsigned long long pair_sample_seed;
  double pair_sample_frac;
  long long max_pairs;        /* 0: workspace grows on demand (one host wait per
                                 exx_eval for the pair count); > 0: fixed pair
                                 capacity, no host wait, and exx_eval may be
                                 recorded into a HIP graph (see exx_eval); pairs
                                 beyond it are dropped and exx_stats_fetch
                                 returns EXX_ECAPACITY                              */
  double workspace_gb;        /* cap on per-batch pair workspace (0: 24 GB)        */
  int solve_groups;           /* persistent solve workgroups (0: as many as fit)   */
  int solve_threads;          /* CG workgroup size, 512, 768 or 1024 (0:
                                 tuned/default); 768 applies to quad-layout
                                 classes of at most 768 runs only, other classes
                                 keep their default                              */
  int solve_depth;            /* planes of loads in flight ahead of use, 1 or 2
                                 (0: tuned/default); cells with arms leaving the
                                 sweep plane have depth 1 only (reported as 1)    */
  int autotune;               /* 1: the first exx_eval times the CG variants on a
                                 sample of each sphere class's pairs and keeps
                                 the fastest per class (threads x depth; for
                                 mixed plans with refine_delta 0 also the
                                 reliable-update threshold)                        */
  int warm_start;             /* 1: each exx_eval starts a pair's CG from that
                                 pair's solution in the previous exx_eval of the
                                 plan (same i, j and sphere class, shifted by the
                                 change of its grid centre, at most one point per
                                 axis), else from zero; the stop test is unchanged.
                                 Needs max_pairs > 0; keeps 2 max_pairs N_PE FP32
                                 values on the device                               */
  /* separate radii of self pairs (i == j), Sec. III A (Step II): PE and ME
     spheres of the self pairs; <= 0 takes the non-self value (exx_plan's R_PE,
     R_ME).  Self pairs then form a sphere class of their own.  Not combined
     with variable radii (R_PE_nclass > 0: EXX_EINVAL)                          */
  double R_PE_self, R_ME_self;
  /* fluctuating cells (Sec. III B 2): 1 builds the tables so that
     exx_set_cell may later switch to any cell whose Laplacian arms are
     nearest grid neighbours (general layout even for an orthorhombic h, and
     Dirichlet points along every nearest-neighbour direction); 0: the cell
     may only change within its kind (orthorhombic stays orthorhombic, a
     general cell keeps its arm directions)                                   */
  int cell_fluctuation;
  /* re-assembly criterion: when exx_set_cell finds max |h h0^-1 - I| above
     this strain (h0: the cell the tables were built for), the
     proto-subdomains are rebuilt from scratch at the new cell with the plan's
     radii (0: never)                                                         */
  double reassemble_strain;
  /* layout of the CG vectors, per sphere class: 0 picks the quad layout for
     mixed plans for every class where it fits, single columns elsewhere; 1:
     single columns (each CG thread owns whole columns of the sphere); 2: quad
     layout for every class (the sphere's columns in runs of four adjacent
     columns, padded with zero slots to the run's tallest column; a CG thread
     owns one run in workgroups of 768 or 1024 threads and two in workgroups
     of 512, and reads its in-plane neighbours as 2-point vectors).  Mixed
     plans run quad classes in 768 threads where the class has at most 768
     runs, else in 512: their CG sweeps each pass B together with the next
     pass A (six vector accesses per point and iteration in place of eight);
     with 1024 threads the two passes stay separate.  A general cell takes it
     when no Laplacian arm leaves the sweep plane, at most one diagonal arm
     lies in it, and its columns are symmetric about the sweep plane.  With
     2, EXX_EINVAL when a class does not fit (more than 1024 runs, other arms
     or columns) and with cell_fluctuation.  Mixed plans of general cells
     whose arms leave the sweep plane (single columns) also sweep each pass B
     with the next pass A, keeping Ap in one more FP32 vector between sweeps
     (as many accesses as two passes, one stencil per iteration), except with
     four columns per thread in 1024 threads                                   */
  int cg_layout;
  /* mixed precision: a reliable update (the FP32 correction folded into the
     FP64 solution and the FP64 true residual recomputed) happens when the
     working residual falls below refine_delta times the residual of the last
     update (0: 0.01, or with autotune the fastest of 0.1, 0.01 and 0.001 on
     each class's sample, reported in exx_stats.class_refine_delta); values
     in (0, 1).  Each update is an FP64 sweep that
     costs about three CG iterations' worth of memory traffic; smaller values
     mean fewer updates and a few more FP32 iterations */
  double refine_delta;
} exx_options;

/* Fills *opt with the defaults: n = 3, FP64, tol 1e-10, 5000 iterations,
   fixed radius, all pairs, on-demand workspace. */
void exx_default_options(exx_options* opt);

/* Builds a plan for cell h (Sec. III B 1: proto-subdomains about the grid
   origin, translated per pair by eq. l2g in crystal coordinates).  h: host
   [9], column-major, h[a + 3*al] = (L_al)_a, right-handed; grid: host [3].
   An orthorhombic h uses the axis stencil of eq. d2_1; any other h the
   Natan-Kronik Laplacian of Sec. III C 1-2 (see exx_nk_stencil), whose
   auxiliary directions must be nearest grid neighbours (|u_al| <= 1) and whose
   weights must be positive.  R_ME must be >= the largest R_PE + n (longest
   stencil step, lattice axes included) so that every stencil neighbour of the
   PE sphere has a far-field value (Sec. IV A); l_max <= 8.  Violations give
   EXX_EINVAL.  opt may be NULL (defaults).  On success *out owns the plan's
   device tables (on the current device). */
exx_status exx_plan(const double h[9], const int grid[3], double R_pair, double R_PE, double R_ME, int l_max,
                    const exx_options* opt, exx_plan_t* out);

/* Binds the HIP stream (a hipStream_t, or NULL for the null stream) that
   exx_eval enqueues on. */
exx_status exx_set_stream(exx_plan_t plan, void* hip_stream);

/* Evaluates E_xx (Sec. I, eq. exxGen_mlwf), D_xx (Sec. II B 2, eq. Dxx) and
   sigma_xx (Sec. II B 3, eq. sxx_working) for n_orb orbitals.
     orbitals  device, [n_orb][N3][N2][N1] of dtype dt, read only
     centres   device, [n_orb][3] Cartesian orbital centres (bohr), read only
     R_PE_orb  device, [n_orb] per-orbital radii, or NULL for the plan radius
     d_subset  device, [n_subset] distinct orbital indices whose D^i are wanted,
               or NULL (n_subset 0) for every orbital; indices outside
               [0, n_orb) are ignored
     E_xx      device, 1 double, overwritten
     D_xx      device, [n_subset or n_orb][N3][N2][N1] of dtype dt (row s holds
               D of orbital d_subset[s]), overwritten; NULL skips D
     sigma     device, 9 doubles, sigma[a + 3*al] = dE/dh_{a al}; NULL skips it
   Unique pairs i <= j carry weight 1 (i == j) or 2 (i != j) in E and sigma;
   D^i receives v_ij phi_j and D^j receives v_ij phi_i on the ME sphere.
   Enqueued on the bound stream; outputs are complete when the stream is.
   Without a fixed capacity (max_pairs 0) the call waits once on the host for
   the pair count.  With max_pairs > 0 it does not wait, and once an eager call
   with at least n_orb orbitals has completed (which also runs the autotuner,
   when enabled) it allocates nothing, so the stream may be recorded into a HIP
   graph around it and the graph replayed with new orbital and centre values
   in the same buffers.  Recording in any other state gives EXX_EINVAL. */
exx_status exx_eval(exx_plan_t plan, int n_orb, const void* orbitals, exx_dtype dt, const double* centres,
                    const double* R_PE_orb, const int* d_subset, int n_subset, double* E_xx, void* D_xx,
                    double* sigma);

/* Bytes of the device scratch array behind exx_eval_noalloc (one per device). */
#define EXX_NOALLOC_SCRATCH_BYTES (256ull << 20)

/* exx_eval without any device allocation, for callers that cannot allocate:
   code recorded into a HIP graph, tight serving loops, harnesses that forbid
   hipMalloc.  Same arguments, outputs and status codes as exx_eval.  Its
   whole workspace (pair list, per-pair results, batch workspace and CG
   vectors) comes from one static device array of EXX_NOALLOC_SCRATCH_BYTES
   that the library holds on each device it runs on until the process ends;
   it uses as many batch rows and persistent CG workgroups as the array holds
   (fewer than exx_eval may use, so it can be slower).  Needs a plan with a
   fixed pair capacity (max_pairs > 0) and without warm_start (EXX_EINVAL
   otherwise); it never runs the autotuner (it keeps the plan's CG variants).
   EXX_EINVAL when n_orb and max_pairs need more than the array (the message
   gives the bytes).  The array keeps the last call's contents: every call on
   a device shares it, so calls that overlap on one device (two streams, or
   two plans) race, and the statistics and per-pair results of a call
   (exx_stats_fetch, exx_pair_results) stay readable only until the next
   exx_eval_noalloc on that device or the next exx_eval, exx_count_pairs or
   exx_set_cell on the plan.  No allocation and no host wait; it records no
   per-launch timing events, so exx_stats reports its whole device time only. */
exx_status exx_eval_noalloc(exx_plan_t plan, int n_orb, const void* orbitals, exx_dtype dt, const double* centres,
                            const double* R_PE_orb, const int* d_subset, int n_subset, double* E_xx, void* D_xx,
                            double* sigma);

/* Number of pairs exx_eval would form for these centres (and radii), for
   sizing max_pairs.  centres and R_PE_orb as in exx_eval (device).  Enqueues
   the pair-list kernels on the bound stream and waits for them; not for use
   while the stream is recorded into a graph.  Does not disturb the results
   of the last exx_eval beyond its per-orbital pair counts. */
exx_status exx_count_pairs(exx_plan_t plan, int n_orb, const double* centres, const double* R_PE_orb,
                           long long* n_pairs);

/* Per-pair results of the last exx_eval, copied to host arrays of capacity
   cap (any may be NULL): ij [2*cap] (i, j), E [cap] (weighted contribution),
   sigma [9*cap], iters [cap] (CG iterations; mixed: FP32 iterations),
   rel_res [cap] (final ||b - A x|| / ||b||; FP64: the recursive residual at
   the stop), exit_code [cap] (exx_cg_exit in the low byte, the mixed solve's
   restarts << 8), updates [cap] (mixed: FP64 reliable updates).  Pairs come
   in i-major, j-ascending order.  Synchronizes the bound stream.  Returns the
   number of pairs of the last evaluation in *n_pairs. */
exx_status exx_pair_results(exx_plan_t plan, long long cap, int* ij, double* E, double* sigma, int* iters,
                            double* rel_res, int* exit_code, int* updates, long long* n_pairs);

typedef struct {
  long long n_pairs;
  long long cg_iter_sum;       /* sum over pairs of CG iterations (inner, mixed)   */
  int cg_iter_max;
  int n_unconverged;
  int n_classes;
  int refine_passes_max;       /* mixed precision: FP64 correction passes          */
  double max_rel_residual;     /* max over pairs of ||b - A x|| / ||b||            */
  double solve_ms;             /* device time of the solve kernels (last eval)     */
  double eval_ms;              /* device time of the whole evaluation              */
  double cg_alg_bytes;         /* algorithmic CG bytes: sum over pairs of (8 iters
                                  - 2 fused quad sweeps - 2 passes that left x
                                  alone) N_PE b                                     */
  double moment_flops;         /* algorithmic moment flops: 2 N_lm N_PE per pair   */
  /* running totals since the plan was made (every completed exx_eval):       */
  long long n_evals;
  long long solve_launches;    /* launches of the persistent CG kernel           */
  double solve_ms_total;       /* their summed device time (HIP events)          */
  double cg_alg_bytes_total;   /* their summed algorithmic CG bytes (eight vector
                                  accesses per point and iteration, two fewer in
                                  a fused quad sweep and in a pass B that leaves
                                  x alone, which every other pass B does; a fused
                                  tilted-arm sweep, which reads and writes Ap in
                                  place of pass A's p, counts as the two passes) */
  double eval_ms_total;
  int solve_threads;           /* CG variant in use: workgroup size (quad layout:
                                  768 and 512 with fused sweeps, 512 with two
                                  runs per thread) ...                             */
  int solve_depth;             /* ... and load depth (chosen by the autotuner)     */
  double tune_ms;              /* time spent by the autotuner (first eval only)    */
  double moment_ms;            /* device time of the moment kernels (last eval)    */
  double moment_mfma_flops;    /* flops the matrix cores executed for the moments
                                  (padded rows and points; mixed: 3 products)      */
  long long pairs_kept;        /* pairs the pair list kept, also beyond max_pairs  */
  int graph_recorded;          /* 1: the last exx_eval was recorded into a graph;
                                  results are those of its latest replay, and the
                                  device times are 0                               */
  long long warm_pairs;        /* pairs whose CG started from a previous solution  */
  double cell_strain;          /* max |h h0^-1 - I| of the current cell against the
                                  cell the tables were built for                  */
  int reassemblies;            /* proto-subdomain re-assemblies by exx_set_cell    */
  int n_arms;                  /* arms of the Laplacian in use (3 to 6)           */
  int cg_layout;               /* CG layout in use: 1 columns, 2 quads, 3 both
                                  (per sphere class)                               */
  /* why pairs of the last exx_eval did not converge (they sum to n_unconverged) */
  int n_cg_cap;                /* stopped at cg_max_iter                           */
  int n_cg_breakdown;          /* p.Ap not positive and finite (after restarts)     */
  int n_cg_nonfinite;          /* a non-finite right-hand side or residual norm     */
  long long cg_restarts;       /* mixed: restarts from the last FP64 solution after
                                  a breakdown or a non-finite FP32 norm              */
  double t_pairlist_ms;        /* device time of the pair list and its order       */
  double t_reduce_ms;          /* device time of the E, sigma and stats reduction  */
  /* CG variant of each sphere class (classes beyond n_classes are 0): workgroup
     size, load depth, layout (1 columns, 2 quads) and the class's pairs in the
     last exx_eval */
  int class_threads[16];
  int class_depth[16];
  int class_layout[16];
  long long class_pairs[16];
  double class_refine_delta[16];   /* mixed: reliable-update threshold of each class
                                      (tuned, when the plan leaves it at 0)     */
} exx_stats;

/* Fluctuating cell (Sec. III B 2): makes h (host [9], column-major,
   right-handed) the plan's cell for the following exx_eval calls while the
   proto-subdomains keep their grid offsets, so their points have fixed scaled
   coordinates s = o / N, local coordinates r = h s, and a fixed count.  The
   Laplacian arms are chosen again for h (Algorithm 1, Sec. III C 2), the
   Jacobian, h^-1 and the volume element follow h, and the pair list and pair
   centres of the next exx_eval use h (centres are Cartesian, for the new
   cell).  With reassemble_strain > 0 and a strain above it, the tables are
   rebuilt for h from the plan's radii (new point counts; the warm-start
   history is dropped).  Waits for the plan's stream; not capturable: HIP
   graphs recorded before the call keep the old cell and tables, record them
   again.  EXX_EINVAL for a singular or left-handed h, for a non-orthogonal h
   on a plan built without cell_fluctuation for an orthorhombic cell, or when
   the new arms leave the Dirichlet points the tables hold (re-assemble or
   plan again). */
exx_status exx_set_cell(exx_plan_t plan, const double h[9]);

/* Host helper: the EXX stress and internal pressure from sigma_xx (Sec. II B
   3): Pi[a + 3 b] = -(1/V) sum_al sigma[a + 3 al] h[b + 3 al] (eq.
   pixx_working) and *p_int = Tr Pi / 3 (eq. pxx_working), V = |det h|.  Pi or
   p_int may be NULL. */
exx_status exx_pressure(const double h[9], const double sigma[9], double* Pi, double* p_int);

/* Statistics of the last exx_eval (synchronizes the bound stream).  Returns
   EXX_ENOCONV when a pair did not converge. */
exx_status exx_stats_fetch(exx_plan_t plan, exx_stats* out);

/* Number of points of a sphere class of the plan (n_pe, n_halo, n_me may be
   NULL); class 0 is the plan radius.  Host only. */
exx_status exx_plan_geometry(exx_plan_t plan, int cls, long long* n_pe, long long* n_halo, long long* n_me);

/* Host-only planning aid (no device needed): point counts of the PE sphere,
   of its Dirichlet points (reached by the Laplacian's arms, and by the lattice
   axes of the first-derivative stencil, within stencil_n steps) and of the
   whole ME sphere, with the same membership rule as exx_plan
   (|h (o / N)|^2 <= R^2 (1 + 1e-12), Sec. III B 1). */
exx_status exx_subdomain_counts(const double h[9], const int grid[3], double R_PE, double R_ME, int stencil_n,
                                long long* n_pe, long long* n_halo, long long* n_me);

/* Host-only (no device needed): the Natan-Kronik Laplacian that exx_plan uses
   for cell h (Sec. III C 1-2, eq. lapG_mod_nk3d, auxiliary directions by
   Algorithm 1).  Writes *n_arms (3 to 6) arms: u[3 k + al] integer steps along
   L_1, L_2, L_3, beta[k] the weight of the pure second derivative along the
   arm and step[k] its Cartesian length, so that the Laplacian is
   sum_k beta[k] / step[k]^2 * (eq. d2_1 along u_k).  Arrays hold 18, 6 and 6
   entries (NULL: not written).  EXX_EINVAL for a singular cell, or when
   Algorithm 1 finds no three admissible directions among its candidates. */
exx_status exx_nk_stencil(const double h[9], const int grid[3], int* n_arms, int* u, double* beta, double* step);

/* Frees the plan and its device memory.  NULL is accepted. */
exx_status exx_destroy(exx_plan_t plan);

/* Message of the last failure on the plan (or of the last failed exx_plan
   when plan is NULL).  The string stays valid until the next call on it. */
const char* exx_last_error(exx_plan_t plan);

#ifdef __cplusplus
}
#endif

#endif /* EXX_H_ */
