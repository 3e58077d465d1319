/*
 * exx_oracle.c -- FP64 CPU oracle for the exact-exchange (EXX) pair kernel of
 * Ko, Santra and DiStasio, "Enabling Large-Scale Condensed-Phase Hybrid DFT Based
 * AIMD II: Extensions to the Isobaric-Isoenthalpic and Isobaric-Isothermal
 * Ensembles" (arXiv:2011.07209).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the correctness reference for the
 * HIP path.  Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark load it; the product path never calls it and shares no code with it.
 *
 * It is deliberately plain and slow: every pair is handled on a dense local box
 * around its grid centre with a membership mask, in double precision, following
 * the steps of the method in the paper's order:
 *
 *   pair list              Sec. III A (Step II): |C_i - C_j| <= R_pair, i <= j
 *   pair grid centre       Sec. III B 1, eq. l2g: NINT of the crystal coordinate
 *   pair density           Sec. I, eq. rho_from_phi_mlwf, on the PE sphere (Step III)
 *   multipole moments      Sec. I, eq. mepole
 *   far-field potential    Sec. I, eq. me, on the ME shell (Step IV)
 *   near-field potential   Sec. I, eq. pe with the Natan-Kronik (NK) Laplacian
 *                          of Sec. III C 1-2 (eq. lapG_mod_nk3d: pure second
 *                          derivatives by eq. d2_1 along the lattice directions
 *                          and the auxiliary directions of Algorithm 1), solved
 *                          by conjugate gradient (Step IV)
 *   energy                 Sec. I, eq. exxGen_mlwf (Step V)
 *   wavefunction forces    Sec. II B 2, eq. Dxx, on the ME sphere (Step V)
 *   cell derivatives       Sec. II B 3, eq. sxx_working, gradient by Sec. III D,
 *                          eq. d1_1 with the Jacobian of eq. jacb
 *
 * Readings where the paper is silent (unique pairs carry weight 1 for i == j and
 * 2 otherwise; unpreconditioned CG from a zero start with a relative residual
 * stop; expansion about the grid-resolved centre; real orthonormal harmonics;
 * inclusive sphere membership with a relative slack of 1e-12 on |r|^2; NINT
 * rounds half away from zero; scatter-adds of periodic aliases accumulate) are
 * listed with their reasons in the design notes of the repository.
 *
 * Any non-singular cell is accepted.  For an orthorhombic cell the NK Laplacian
 * reduces to the axis stencil.  The cell used to build pairs, centres and
 * offset sets may differ from the physical cell, so that strain derivatives can
 * be taken at frozen subdomains (Sec. III B 2); the Laplacian, the Jacobian and
 * the local coordinates always use the physical cell.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_PI 3.14159265358979323846
#define OR_MAXL 12
#define OR_SLACK 1e-12

typedef struct {
  double h[9];       /* physical cell, column-major: h[a + 3*al] = (L_al)_a     */
  double h_geom[9];  /* cell used for pairs, centres and offset membership       */
  int grid[3];       /* N_1, N_2, N_3 points along L_1, L_2, L_3                 */
  double R_pair, R_PE, R_ME;
  int l_max;
  int stencil_n;     /* half-width n of the axis stencils, 1..3                  */
  double cg_tol;     /* stop when ||r||_2 <= cg_tol * ||b||_2                   */
  int cg_max_iter;
  /* variable radii: with per-orbital radii given, the pair radius is the rung
     R_PE_min + k * R_PE_step (k = 0..R_PE_nclass-1) nearest to (R_i + R_j)/2   */
  double R_PE_min, R_PE_step;
  int R_PE_nclass;
  unsigned long long sample_seed;  /* deterministic pair subset                  */
  double sample_frac;              /* >= 1: all pairs                            */
  int n_threads;                   /* <= 0: OpenMP default                       */
  /* separate radii of self pairs (i == j), Sec. III A (Step II): <= 0 takes
     the non-self value; not combined with variable radii                      */
  double R_PE_self, R_ME_self;
} oracle_params;

typedef struct {
  int i, j;
  int c[3];          /* grid centre of the pair                                */
  double R_PE;
  int n_pe, n_me;
  int cg_iters;
  int converged;
  double rel_res;        /* recursive residual / ||b|| at exit                 */
  double true_rel_res;   /* ||b - A x|| / ||b|| recomputed at exit             */
  double E;              /* this pair's contribution to E_xx (weight included) */
  double sigma[9];       /* this pair's contribution to sigma, [a + 3*al]      */
  double shell_rho_v;    /* w * dV * sum over ME\PE of rho * v                 */
} oracle_pair_result;

/* ------------------------------------------------------------------------- */
/* small linear algebra on 3x3 column-major matrices                          */

#define M3(m, r, c) ((m)[(r) + 3 * (c)])

static double det3(const double* m) {
  return M3(m, 0, 0) * (M3(m, 1, 1) * M3(m, 2, 2) - M3(m, 1, 2) * M3(m, 2, 1)) -
         M3(m, 0, 1) * (M3(m, 1, 0) * M3(m, 2, 2) - M3(m, 1, 2) * M3(m, 2, 0)) +
         M3(m, 0, 2) * (M3(m, 1, 0) * M3(m, 2, 1) - M3(m, 1, 1) * M3(m, 2, 0));
}

/* inverse by the adjugate */
static void inv3(const double* m, double* inv) {
  double d = det3(m);
  M3(inv, 0, 0) = (M3(m, 1, 1) * M3(m, 2, 2) - M3(m, 1, 2) * M3(m, 2, 1)) / d;
  M3(inv, 0, 1) = (M3(m, 0, 2) * M3(m, 2, 1) - M3(m, 0, 1) * M3(m, 2, 2)) / d;
  M3(inv, 0, 2) = (M3(m, 0, 1) * M3(m, 1, 2) - M3(m, 0, 2) * M3(m, 1, 1)) / d;
  M3(inv, 1, 0) = (M3(m, 1, 2) * M3(m, 2, 0) - M3(m, 1, 0) * M3(m, 2, 2)) / d;
  M3(inv, 1, 1) = (M3(m, 0, 0) * M3(m, 2, 2) - M3(m, 0, 2) * M3(m, 2, 0)) / d;
  M3(inv, 1, 2) = (M3(m, 0, 2) * M3(m, 1, 0) - M3(m, 0, 0) * M3(m, 1, 2)) / d;
  M3(inv, 2, 0) = (M3(m, 1, 0) * M3(m, 2, 1) - M3(m, 1, 1) * M3(m, 2, 0)) / d;
  M3(inv, 2, 1) = (M3(m, 0, 1) * M3(m, 2, 0) - M3(m, 0, 0) * M3(m, 2, 1)) / d;
  M3(inv, 2, 2) = (M3(m, 0, 0) * M3(m, 1, 1) - M3(m, 0, 1) * M3(m, 1, 0)) / d;
}

static void matvec3(const double* m, const double* v, double* out) {
  for (int r = 0; r < 3; ++r)
    out[r] = M3(m, r, 0) * v[0] + M3(m, r, 1) * v[1] + M3(m, r, 2) * v[2];
}

static double col_norm(const double* h, int al) {
  return sqrt(M3(h, 0, al) * M3(h, 0, al) + M3(h, 1, al) * M3(h, 1, al) +
              M3(h, 2, al) * M3(h, 2, al));
}

/* ------------------------------------------------------------------------- */
/* central-difference weights (Fornberg 1988).  Second derivative: the n = 3  */
/* set is printed with eq. d2_1; first derivative: the n = 3 set is printed   */
/* with eq. d1_1.  Lower orders are the textbook Taylor-matched sets.          */

void oracle_stencil_weights(int n, double* w2, double* w1) {
  for (int q = 0; q < 4; ++q) w2[q] = w1[q] = 0.0;
  if (n == 1) {
    w2[0] = -2.0; w2[1] = 1.0;
    w1[1] = 0.5;
  } else if (n == 2) {
    w2[0] = -5.0 / 2.0; w2[1] = 4.0 / 3.0; w2[2] = -1.0 / 12.0;
    w1[1] = 2.0 / 3.0; w1[2] = -1.0 / 12.0;
  } else if (n == 3) {
    w2[0] = -49.0 / 18.0; w2[1] = 3.0 / 2.0; w2[2] = -3.0 / 20.0; w2[3] = 1.0 / 90.0;
    w1[1] = 3.0 / 4.0; w1[2] = -3.0 / 20.0; w1[3] = 1.0 / 60.0;
  }
}

/* ------------------------------------------------------------------------- */
/* The Natan-Kronik (NK) Laplacian on a general grid (Sec. III C 1-2).        */
/*                                                                            */
/* A grid direction u (integer steps along L_1, L_2, L_3) has the Cartesian    */
/* step sum_al u_al L_al / N_al of length dl.  The Laplacian is written as     */
/* sum over arms of beta * d^2/dl^2 with the pure second derivative along each */
/* arm taken by eq. d2_1: beta / dl^2 * sum_q w_q f(o + q u).  The arms are    */
/* the three lattice directions (eq. lapG_mod_nk3d, first sum) and up to three */
/* auxiliary directions chosen by Algorithm 1 (second sum).                   */

#define OR_MAX_ARMS 6
#define OR_NQ 15          /* candidate auxiliary directions handed to Algorithm 1 */
#define OR_MAX_SHELL 8
#define OR_TIE 1e-10      /* relative tolerance of equal spacings and of the
                             parallel / singular tests of Algorithm 1          */
#define OR_ZERO_W 1e-12   /* arm weights below this times max F_al,al are zero */

typedef struct {
  int u[3];
  double beta;   /* weight of d^2/dl^2 along the arm                          */
  double step;   /* dl                                                         */
  double coef;   /* beta / dl^2                                                */
} nk_arm;

typedef struct {
  int n_arms;
  nk_arm arm[OR_MAX_ARMS];
  int aux_u[3][3];   /* the three directions Algorithm 1 accepted             */
  double b[3];       /* their weights from M b = (F12, F13, F23)              */
  double F[9];       /* F = J^T J                                             */
} nk_stencil;

typedef struct {
  int u[3];
  double len;
  int seq;           /* position in the shell sweep                          */
} nk_cand;

static double step_len(const double* h, const int* N, const int* u) {
  double v[3] = {0.0, 0.0, 0.0};
  for (int al = 0; al < 3; ++al)
    for (int a = 0; a < 3; ++a) v[a] += u[al] * M3(h, a, al) / N[al];
  return sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
}

/* candidate order: shorter step first; equal steps (within OR_TIE) keep the
   order of the shell sweep */
static int cand_before(const nk_cand* x, const nk_cand* y) {
  double m = x->len > y->len ? x->len : y->len;
  if (x->len < y->len - OR_TIE * m) return 1;
  if (y->len < x->len - OR_TIE * m) return 0;
  return x->seq < y->seq;
}

/* Builds the NK arms of cell h on grid N.  Returns 0, or -2 when Algorithm 1
   finds no three admissible auxiliary directions among its candidates. */
static int nk_build(const double* h, const int* N, nk_stencil* S) {
  memset(S, 0, sizeof(*S));
  double hinv[9], J[9];
  inv3(h, hinv);
  double dxi[3];
  for (int al = 0; al < 3; ++al) dxi[al] = col_norm(h, al) / N[al];
  /* Jacobian J_{a al} = |L_al| (h^-1)_{al a} (eq. jacb); F = J^T J (eq. lapG_) */
  for (int a = 0; a < 3; ++a)
    for (int al = 0; al < 3; ++al) M3(J, a, al) = col_norm(h, al) * M3(hinv, al, a);
  for (int al = 0; al < 3; ++al)
    for (int be = 0; be < 3; ++be) {
      double s = 0.0;
      for (int a = 0; a < 3; ++a) s += M3(J, a, al) * M3(J, a, be);
      M3(S->F, al, be) = s;
    }

  /* candidate auxiliary directions: non-axial grid points in shells
     S = max_al |u_al| = 1, 2, ... about a reference point, one of each +-u
     pair; the sweep stops at the first shell whose points all lie farther than
     the largest step of the first shell (and holds at least OR_NQ candidates) */
  static const int kMaxCand = 4 * (2 * OR_MAX_SHELL + 1) * (2 * OR_MAX_SHELL + 1) * (2 * OR_MAX_SHELL + 1);
  nk_cand* cand = (nk_cand*)malloc(sizeof(nk_cand) * kMaxCand);
  if (!cand) return -4;
  int nc = 0;
  double big1 = 0.0;
  for (int sh = 1; sh <= OR_MAX_SHELL; ++sh) {
    double shell_min = INFINITY;
    int u[3];
    for (u[2] = -sh; u[2] <= sh; ++u[2])
      for (u[1] = -sh; u[1] <= sh; ++u[1])
        for (u[0] = -sh; u[0] <= sh; ++u[0]) {
          int m = abs(u[0]) > abs(u[1]) ? abs(u[0]) : abs(u[1]);
          if (abs(u[2]) > m) m = abs(u[2]);
          if (m != sh) continue;
          double len = step_len(h, N, u);
          if (len < shell_min) shell_min = len;
          if (sh == 1 && len > big1) big1 = len;
          int nz = (u[0] != 0) + (u[1] != 0) + (u[2] != 0);
          if (nz < 2) continue;   /* axial */
          int lead = u[0] != 0 ? u[0] : (u[1] != 0 ? u[1] : u[2]);
          if (lead < 0) continue; /* -u is the same direction */
          nk_cand* c = &cand[nc];
          c->u[0] = u[0]; c->u[1] = u[1]; c->u[2] = u[2];
          c->len = len;
          c->seq = nc;
          ++nc;
        }
    if (sh >= 2 && shell_min > big1 && nc >= OR_NQ) break;
  }
  /* ascending step (insertion sort: stable, so ties keep the sweep order) */
  for (int i = 1; i < nc; ++i) {
    nk_cand t = cand[i];
    int j = i - 1;
    while (j >= 0 && cand_before(&t, &cand[j])) {
      cand[j + 1] = cand[j];
      --j;
    }
    cand[j + 1] = t;
  }
  int nq = nc < OR_NQ ? nc : OR_NQ;

  /* Algorithm 1: accept the shortest candidate, then the next whose column of M
     is not parallel to the first (Cauchy-Schwarz), then the next that makes M
     non-singular */
  double Mm[9] = {0};   /* column p: (a_p1 a_p2, a_p1 a_p3, a_p2 a_p3) */
  double a_sel[3][3];
  int p = 0;
  for (int q = 0; q < nq && p < 3; ++q) {
    double ap[3];
    for (int al = 0; al < 3; ++al) ap[al] = cand[q].u[al] * dxi[al] / cand[q].len;
    double col[3] = {ap[0] * ap[1], ap[0] * ap[2], ap[1] * ap[2]};
    int ok = 0;
    if (p == 0) {
      ok = 1;
    } else if (p == 1) {
      double d = 0.0, n1 = 0.0, n2 = 0.0;
      for (int r = 0; r < 3; ++r) {
        d += M3(Mm, r, 0) * col[r];
        n1 += M3(Mm, r, 0) * M3(Mm, r, 0);
        n2 += col[r] * col[r];
      }
      ok = fabs(d) < (1.0 - OR_TIE) * sqrt(n1 * n2);
    } else {
      double T[9];
      memcpy(T, Mm, sizeof(T));
      for (int r = 0; r < 3; ++r) M3(T, r, 2) = col[r];
      double n0 = 0.0, n1 = 0.0, n2 = 0.0;
      for (int r = 0; r < 3; ++r) {
        n0 += M3(T, r, 0) * M3(T, r, 0);
        n1 += M3(T, r, 1) * M3(T, r, 1);
        n2 += M3(T, r, 2) * M3(T, r, 2);
      }
      ok = fabs(det3(T)) > OR_TIE * sqrt(n0 * n1 * n2);
    }
    if (!ok) continue;
    for (int r = 0; r < 3; ++r) M3(Mm, r, p) = col[r];
    for (int al = 0; al < 3; ++al) {
      a_sel[p][al] = ap[al];
      S->aux_u[p][al] = cand[q].u[al];
    }
    ++p;
  }
  double aux_len[3];
  for (int k = 0; k < p; ++k) aux_len[k] = step_len(h, N, S->aux_u[k]);
  free(cand);
  if (p < 3) return -2;

  /* M b = (F12, F13, F23) (eq. nk3d_Mb_f), by Cramer's rule */
  double f[3] = {M3(S->F, 0, 1), M3(S->F, 0, 2), M3(S->F, 1, 2)};
  double dM = det3(Mm);
  for (int k = 0; k < 3; ++k) {
    double T[9];
    memcpy(T, Mm, sizeof(T));
    for (int r = 0; r < 3; ++r) M3(T, r, k) = f[r];
    S->b[k] = det3(T) / dM;
  }

  /* eq. lapG_mod_nk3d: weight F_al,al - sum_p b_p a_p,al^2 on each lattice
     direction, b_p on each auxiliary direction; zero weights are dropped */
  double fmax = 0.0;
  for (int al = 0; al < 3; ++al) if (M3(S->F, al, al) > fmax) fmax = M3(S->F, al, al);
  S->n_arms = 0;
  for (int al = 0; al < 3; ++al) {
    double beta = M3(S->F, al, al);
    for (int k = 0; k < 3; ++k) beta -= S->b[k] * a_sel[k][al] * a_sel[k][al];
    if (fabs(beta) <= OR_ZERO_W * fmax) continue;
    nk_arm* A = &S->arm[S->n_arms++];
    A->u[0] = A->u[1] = A->u[2] = 0;
    A->u[al] = 1;
    A->beta = beta;
    A->step = dxi[al];
    A->coef = beta / (dxi[al] * dxi[al]);
  }
  for (int k = 0; k < 3; ++k) {
    if (fabs(S->b[k]) <= OR_ZERO_W * fmax) continue;
    nk_arm* A = &S->arm[S->n_arms++];
    for (int al = 0; al < 3; ++al) A->u[al] = S->aux_u[k][al];
    A->beta = S->b[k];
    A->step = aux_len[k];
    A->coef = S->b[k] / (aux_len[k] * aux_len[k]);
  }
  return 0;
}

/* The NK arms of cell h on grid N, for the checks: u_out[3 k + al], beta_out,
   step_out per arm; aux_out[3 p + al] and b_out[p] for the three directions
   Algorithm 1 accepted.  Returns the number of arms or a negative error. */
int oracle_nk_stencil(const double* h, const int* N, int* u_out, double* beta_out, double* step_out, int* aux_out,
                      double* b_out) {
  if (fabs(det3(h)) <= 0.0 || N[0] <= 0 || N[1] <= 0 || N[2] <= 0) return -1;
  nk_stencil S;
  int rc = nk_build(h, N, &S);
  if (rc) return rc;
  for (int k = 0; k < S.n_arms; ++k) {
    for (int al = 0; al < 3; ++al) u_out[3 * k + al] = S.arm[k].u[al];
    beta_out[k] = S.arm[k].beta;
    step_out[k] = S.arm[k].step;
  }
  for (int p = 0; p < 3; ++p) {
    for (int al = 0; al < 3; ++al) aux_out[3 * p + al] = S.aux_u[p][al];
    b_out[p] = S.b[p];
  }
  return S.n_arms;
}

/* ------------------------------------------------------------------------- */
/* real orthonormal spherical harmonics S_lm(theta, phi), index l*l + l + m.  */
/* Associated Legendre functions without the Condon-Shortley phase, from the  */
/* textbook three-term recurrence in l; normalisation                          */
/* N_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!), sqrt(2) N_lm cos/sin(m phi) for   */
/* m > 0 / m < 0.  For real densities these give the same Q_lm Y_lm products   */
/* as the complex harmonics of eq. me and eq. mepole.                          */

void oracle_ylm(int lmax, double x, double y, double z, double* out) {
  double P[OR_MAXL + 1][OR_MAXL + 1];
  double r = sqrt(x * x + y * y + z * z);
  double ct = 1.0, st = 0.0, ph = 0.0;
  if (r > 0.0) {
    ct = z / r;
    st = sqrt(x * x + y * y) / r;
    ph = atan2(y, x);
  }
  for (int l = 0; l <= lmax; ++l)
    for (int m = 0; m <= lmax; ++m) P[l][m] = 0.0;
  P[0][0] = 1.0;
  for (int m = 1; m <= lmax; ++m) P[m][m] = (2.0 * m - 1.0) * st * P[m - 1][m - 1];
  for (int m = 0; m < lmax; ++m) P[m + 1][m] = (2.0 * m + 1.0) * ct * P[m][m];
  for (int m = 0; m <= lmax; ++m)
    for (int l = m + 2; l <= lmax; ++l)
      P[l][m] = ((2.0 * l - 1.0) * ct * P[l - 1][m] - (l + m - 1.0) * P[l - 2][m]) / (double)(l - m);
  for (int l = 0; l <= lmax; ++l) {
    for (int m = 0; m <= l; ++m) {
      double ratio = 1.0; /* (l-m)!/(l+m)! */
      for (int k = l - m + 1; k <= l + m; ++k) ratio /= (double)k;
      double N = sqrt((2.0 * l + 1.0) / (4.0 * OR_PI) * ratio);
      if (m == 0) {
        out[l * l + l] = N * P[l][0];
      } else {
        out[l * l + l + m] = sqrt(2.0) * N * P[l][m] * cos(m * ph);
        out[l * l + l - m] = sqrt(2.0) * N * P[l][m] * sin(m * ph);
      }
    }
  }
}

/* ------------------------------------------------------------------------- */
/* deterministic pair subset: one output of SplitMix64 (Steele, Lea and Flood  */
/* 2014) on the state seed ^ (i << 32) ^ j; keep the pair when the top 53 bits */
/* read as a fraction fall below sample_frac.                                  */

static uint64_t splitmix64_once(uint64_t state) {
  uint64_t z = state + 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

static int pair_selected(const oracle_params* P, int i, int j) {
  if (P->sample_frac >= 1.0) return 1;
  uint64_t u = splitmix64_once(P->sample_seed ^ ((uint64_t)(uint32_t)i << 32) ^ (uint64_t)(uint32_t)j);
  double f = (double)(u >> 11) * (1.0 / 9007199254740992.0);
  return f < P->sample_frac;
}

/* ------------------------------------------------------------------------- */
/* geometry                                                                   */

typedef struct {
  oracle_params P;
  double hinv[9], hginv[9];
  double dxi[3];       /* physical spacing |L_al| / N_al                        */
  double dV;           /* |det h| / N                                           */
  long ngrid;
  double w2[4], w1[4];
  nk_stencil S;        /* Laplacian arms of the physical cell               */
  int umax;            /* largest |u_al| over the arms                      */
} ctx_t;

static int ctx_init(ctx_t* X, const oracle_params* P) {
  X->P = *P;
  if (P->grid[0] <= 0 || P->grid[1] <= 0 || P->grid[2] <= 0) return -1;
  if (P->stencil_n < 1 || P->stencil_n > 3) return -1;
  if (P->l_max < 0 || P->l_max > OR_MAXL) return -1;
  if (fabs(det3(P->h)) <= 0.0 || fabs(det3(P->h_geom)) <= 0.0) return -1;
  inv3(P->h, X->hinv);
  inv3(P->h_geom, X->hginv);
  X->ngrid = (long)P->grid[0] * P->grid[1] * P->grid[2];
  int nk = nk_build(P->h, P->grid, &X->S);
  if (nk) return nk;
  /* the longest stencil step in the geometry cell: Laplacian arms, and the
     lattice directions of the first-derivative stencil of sigma */
  double maxd = 0.0;
  X->umax = 1;
  for (int al = 0; al < 3; ++al) {
    X->dxi[al] = col_norm(P->h, al) / P->grid[al];
    double dg = col_norm(P->h_geom, al) / P->grid[al];
    if (dg > maxd) maxd = dg;
  }
  for (int k = 0; k < X->S.n_arms; ++k) {
    double dg = step_len(P->h_geom, P->grid, X->S.arm[k].u);
    if (dg > maxd) maxd = dg;
    for (int al = 0; al < 3; ++al)
      if (abs(X->S.arm[k].u[al]) > X->umax) X->umax = abs(X->S.arm[k].u[al]);
  }
  X->dV = fabs(det3(P->h)) / (double)X->ngrid;
  oracle_stencil_weights(P->stencil_n, X->w2, X->w1);
  double rmax = P->R_PE;
  if (P->R_PE_nclass > 0) rmax = P->R_PE_min + (P->R_PE_nclass - 1) * P->R_PE_step;
  if (P->R_PE_nclass > 0 && (P->R_PE_self > 0.0 || P->R_ME_self > 0.0)) return -1;
  /* the ME shell must hold every stencil neighbour of the PE sphere, for the
     self radii as for the others */
  if (P->R_ME < rmax + P->stencil_n * maxd) return -3;
  const double rpe_s = P->R_PE_self > 0.0 ? P->R_PE_self : P->R_PE;
  const double rme_s = P->R_ME_self > 0.0 ? P->R_ME_self : P->R_ME;
  if (rme_s < rpe_s + P->stencil_n * maxd) return -3;
  return 0;
}

/* minimum-image displacement in the geometry cell */
static void mic(const ctx_t* X, const double* d, double* out) {
  double s[3];
  matvec3(X->hginv, d, s);
  for (int al = 0; al < 3; ++al) s[al] -= round(s[al]);
  matvec3(X->P.h_geom, s, out);
}

static double pair_radius(const ctx_t* X, const double* R_orb, int i, int j) {
  if (i == j && X->P.R_PE_self > 0.0 && X->P.R_PE_nclass <= 0) return X->P.R_PE_self;
  if (!R_orb || X->P.R_PE_nclass <= 0) return X->P.R_PE;
  double r = 0.5 * (R_orb[i] + R_orb[j]);
  double k = round((r - X->P.R_PE_min) / X->P.R_PE_step);
  if (k < 0) k = 0;
  if (k > X->P.R_PE_nclass - 1) k = X->P.R_PE_nclass - 1;
  return X->P.R_PE_min + k * X->P.R_PE_step;
}

/* ME radius of pair (i, j): the self value for i == j when one is given */
static double pair_me_radius(const oracle_params* P, int i, int j) {
  return (i == j && P->R_ME_self > 0.0) ? P->R_ME_self : P->R_ME;
}

/* grid centre of a point: NINT(N_al * frac((h^-1 C)_al)) mod N_al */
static void grid_centre(const ctx_t* X, const double* C, int* c) {
  double s[3];
  matvec3(X->hginv, C, s);
  for (int al = 0; al < 3; ++al) {
    double f = s[al] - floor(s[al]);
    long g = (long)round(X->P.grid[al] * f);
    g %= X->P.grid[al];
    if (g < 0) g += X->P.grid[al];
    c[al] = (int)g;
  }
}

/* Unique pair list (Step II).  Pairs come in i-major, j-ascending order.
   Returns the number of pairs (writing at most cap of them), or < 0 on error. */
static long build_pairs(const ctx_t* X, int n_orb, const double* centres, const double* R_orb,
                        oracle_pair_result* out, long cap) {
  long n = 0;
  double r2max = X->P.R_pair * X->P.R_pair * (1.0 + OR_SLACK);
  for (int i = 0; i < n_orb; ++i) {
    for (int j = i; j < n_orb; ++j) {
      double d[3], dm[3];
      for (int a = 0; a < 3; ++a) d[a] = centres[3 * j + a] - centres[3 * i + a];
      mic(X, d, dm);
      double d2 = dm[0] * dm[0] + dm[1] * dm[1] + dm[2] * dm[2];
      if (i != j && d2 > r2max) continue;
      if (!pair_selected(&X->P, i, j)) continue;
      if (out && n < cap) {
        oracle_pair_result* pr = &out[n];
        memset(pr, 0, sizeof(*pr));
        pr->i = i;
        pr->j = j;
        double Cij[3];
        for (int a = 0; a < 3; ++a) Cij[a] = centres[3 * i + a] + 0.5 * dm[a];
        grid_centre(X, Cij, pr->c);
        pr->R_PE = pair_radius(X, R_orb, i, j);
      }
      ++n;
    }
  }
  return n;
}

long oracle_pair_list(const oracle_params* P, int n_orb, const double* centres, const double* R_orb,
                      oracle_pair_result* out, long cap) {
  ctx_t X;
  int rc = ctx_init(&X, P);
  if (rc) return rc;
  return build_pairs(&X, n_orb, centres, R_orb, out, cap);
}

/* ------------------------------------------------------------------------- */
/* the local box around a pair's grid centre                                  */

typedef struct {
  int K[3], B[3];
  long n;
  long s[3];  /* strides */
} box_t;

static void box_make(const ctx_t* X, box_t* bx) {
  for (int al = 0; al < 3; ++al) {
    /* |o_al| = N_al |(h_g^-1 r)_al| <= N_al |row al of h_g^-1| R_ME */
    double rn = sqrt(M3(X->hginv, al, 0) * M3(X->hginv, al, 0) + M3(X->hginv, al, 1) * M3(X->hginv, al, 1) +
                     M3(X->hginv, al, 2) * M3(X->hginv, al, 2));
    const double rme = X->P.R_ME_self > X->P.R_ME ? X->P.R_ME_self : X->P.R_ME;   /* the larger ME sphere */
    bx->K[al] = (int)ceil(rme * X->P.grid[al] * rn) + X->P.stencil_n * X->umax + 1;
    bx->B[al] = 2 * bx->K[al] + 1;
  }
  bx->s[0] = 1;
  bx->s[1] = bx->B[0];
  bx->s[2] = (long)bx->B[0] * bx->B[1];
  bx->n = (long)bx->B[0] * bx->B[1] * bx->B[2];
}

/* offset o -> local coordinate h (o / N) for a given cell */
static void rbar_of(const double* h, const int* N, const int* o, double* r) {
  double s[3] = {(double)o[0] / N[0], (double)o[1] / N[1], (double)o[2] / N[2]};
  matvec3(h, s, r);
}

/* ------------------------------------------------------------------------- */
/* the discrete operator A = -(NK Laplacian) restricted to the PE points      */
/* (Dirichlet zero elsewhere), and plain CG on it                              */

static long arm_stride(const box_t* bx, const int* u) {
  return u[0] * bx->s[0] + u[1] * bx->s[1] + u[2] * bx->s[2];
}

static void apply_A(const ctx_t* X, const box_t* bx, const long* pe, long npe, const double* p, double* q) {
  int n = X->P.stencil_n;
  for (long k = 0; k < npe; ++k) {
    long o = pe[k];
    double acc = 0.0;
    for (int m = 0; m < X->S.n_arms; ++m) {
      long st = arm_stride(bx, X->S.arm[m].u);
      double t = X->w2[0] * p[o];
      for (int qq = 1; qq <= n; ++qq) t += X->w2[qq] * (p[o + qq * st] + p[o - qq * st]);
      acc += X->S.arm[m].coef * t;
    }
    q[o] = -acc;
  }
}

static double dot_pe(const long* pe, long npe, const double* a, const double* b) {
  double s = 0.0;
  for (long k = 0; k < npe; ++k) s += a[pe[k]] * b[pe[k]];
  return s;
}

/* Solves A x = b on the PE points.  x, r, p, q are box arrays that are zero
   off the PE points.  Returns the number of iterations taken. */
static int cg_solve(const ctx_t* X, const box_t* bx, const long* pe, long npe, const double* b, double* x,
                    double* r, double* p, double* q, double* rel_res, int* converged) {
  double bb = dot_pe(pe, npe, b, b);
  double bnorm = sqrt(bb);
  for (long k = 0; k < npe; ++k) {
    long o = pe[k];
    x[o] = 0.0;
    r[o] = b[o];
    p[o] = b[o];
  }
  *converged = 1;
  *rel_res = 0.0;
  if (bnorm == 0.0) return 0;
  double rr = bb;
  int it = 0;
  *converged = 0;
  while (it < X->P.cg_max_iter) {
    apply_A(X, bx, pe, npe, p, q);
    double alpha = rr / dot_pe(pe, npe, p, q);
    for (long k = 0; k < npe; ++k) {
      long o = pe[k];
      x[o] += alpha * p[o];
      r[o] -= alpha * q[o];
    }
    double rr_new = dot_pe(pe, npe, r, r);
    ++it;
    if (sqrt(rr_new) <= X->P.cg_tol * bnorm) {
      *converged = 1;
      rr = rr_new;
      break;
    }
    double beta = rr_new / rr;
    for (long k = 0; k < npe; ++k) {
      long o = pe[k];
      p[o] = r[o] + beta * p[o];
    }
    rr = rr_new;
  }
  *rel_res = sqrt(rr) / bnorm;
  return it;
}

/* ------------------------------------------------------------------------- */
/* one pair                                                                   */

typedef struct {
  long cap;
  long n;
  long* g;      /* global grid index of each ME point                       */
  double* v;    /* potential at that point                                  */
  double* pi;   /* phi_i there                                              */
  double* pj;   /* phi_j there                                              */
} me_list_t;

typedef struct {
  box_t bx;
  unsigned char* mask; /* 0 outside ME, 1 shell (ME\PE), 2 PE                 */
  double *rho, *vb, *b, *x, *r, *p, *q;
  long* pe;
  long npe_cap;
} work_t;

static void work_free(work_t* W) {
  free(W->mask); free(W->rho); free(W->vb); free(W->b);
  free(W->x); free(W->r); free(W->p); free(W->q); free(W->pe);
  memset(W, 0, sizeof(*W));
}

static int work_alloc(work_t* W, const box_t* bx) {
  memset(W, 0, sizeof(*W));
  W->bx = *bx;
  W->mask = (unsigned char*)calloc(bx->n, 1);
  W->rho = (double*)calloc(bx->n, sizeof(double));
  W->vb = (double*)calloc(bx->n, sizeof(double));
  W->b = (double*)calloc(bx->n, sizeof(double));
  W->x = (double*)calloc(bx->n, sizeof(double));
  W->r = (double*)calloc(bx->n, sizeof(double));
  W->p = (double*)calloc(bx->n, sizeof(double));
  W->q = (double*)calloc(bx->n, sizeof(double));
  W->pe = (long*)malloc(bx->n * sizeof(long));
  if (!W->mask || !W->rho || !W->vb || !W->b || !W->x || !W->r || !W->p || !W->q || !W->pe) {
    work_free(W);
    return -1;
  }
  return 0;
}

static inline long wrap(long g, int N) {
  g %= N;
  return g < 0 ? g + N : g;
}

/* Evaluates one pair.  Fills res (E, sigma, diagnostics), and, when me is not
   NULL, the potential on every ME point for the wavefunction forces.  When
   vout is not NULL it receives the box array of v (PE: CG solution, shell:
   far field) and rout the box array of rho. */
static int eval_pair(const ctx_t* X, work_t* W, const double* orb, oracle_pair_result* res, me_list_t* me,
                     double* vout, double* rout) {
  const oracle_params* P = &X->P;
  const box_t* bx = &W->bx;
  const int* N = P->grid;
  int n = P->stencil_n;
  int L = P->l_max;
  int nlm = (L + 1) * (L + 1);
  const double* phi_i = orb + (long)res->i * X->ngrid;
  const double* phi_j = orb + (long)res->j * X->ngrid;
  double w = (res->i == res->j) ? 1.0 : 2.0;
  double rpe2 = res->R_PE * res->R_PE * (1.0 + OR_SLACK);
  const double rme = pair_me_radius(P, res->i, res->j);
  double rme2 = rme * rme * (1.0 + OR_SLACK);

  memset(W->mask, 0, bx->n);
  memset(W->rho, 0, bx->n * sizeof(double));
  memset(W->vb, 0, bx->n * sizeof(double));
  memset(W->b, 0, bx->n * sizeof(double));
  memset(W->x, 0, bx->n * sizeof(double));
  memset(W->r, 0, bx->n * sizeof(double));
  memset(W->p, 0, bx->n * sizeof(double));
  memset(W->q, 0, bx->n * sizeof(double));

  /* subdomains: PE and ME spheres about the grid centre (Sec. III A Step II,
     Sec. III B 1); the pair density on PE (Step III) */
  long npe = 0, nme = 0;
  int o[3];
  for (o[2] = -bx->K[2]; o[2] <= bx->K[2]; ++o[2])
    for (o[1] = -bx->K[1]; o[1] <= bx->K[1]; ++o[1])
      for (o[0] = -bx->K[0]; o[0] <= bx->K[0]; ++o[0]) {
        double rg[3];
        rbar_of(P->h_geom, N, o, rg);
        double r2 = rg[0] * rg[0] + rg[1] * rg[1] + rg[2] * rg[2];
        if (r2 > rme2) continue;
        long bi = (o[0] + bx->K[0]) + bx->s[1] * (o[1] + bx->K[1]) + bx->s[2] * (o[2] + bx->K[2]);
        ++nme;
        if (r2 <= rpe2) {
          W->mask[bi] = 2;
          W->pe[npe++] = bi;
          long g = wrap(res->c[0] + o[0], N[0]) + (long)N[0] * (wrap(res->c[1] + o[1], N[1]) +
                                                                (long)N[1] * wrap(res->c[2] + o[2], N[2]));
          W->rho[bi] = phi_i[g] * phi_j[g];
        } else {
          W->mask[bi] = 1;
        }
      }
  res->n_pe = (int)npe;
  res->n_me = (int)nme;

  /* multipole moments Q_lm = dV sum_PE S_lm(rhat) |r|^l rho (eq. mepole) */
  double Q[(OR_MAXL + 1) * (OR_MAXL + 1)];
  double Y[(OR_MAXL + 1) * (OR_MAXL + 1)];
  for (int k = 0; k < nlm; ++k) Q[k] = 0.0;
  for (long k = 0; k < npe; ++k) {
    long bi = W->pe[k];
    o[0] = (int)(bi % bx->B[0]) - bx->K[0];
    o[1] = (int)((bi / bx->B[0]) % bx->B[1]) - bx->K[1];
    o[2] = (int)(bi / bx->s[2]) - bx->K[2];
    double rv[3];
    rbar_of(P->h, N, o, rv);
    double r = sqrt(rv[0] * rv[0] + rv[1] * rv[1] + rv[2] * rv[2]);
    oracle_ylm(L, rv[0], rv[1], rv[2], Y);
    double rl = 1.0;
    for (int l = 0; l <= L; ++l) {
      for (int m = -l; m <= l; ++m) Q[l * l + l + m] += X->dV * Y[l * l + l + m] * rl * W->rho[bi];
      rl *= r;
    }
  }

  /* far-field potential on ME\PE (eq. me):
     v = 4 pi sum_lm Q_lm S_lm(rhat) / ((2l+1) |r|^(l+1)) */
  for (long bi = 0; bi < bx->n; ++bi) {
    if (W->mask[bi] != 1) continue;
    o[0] = (int)(bi % bx->B[0]) - bx->K[0];
    o[1] = (int)((bi / bx->B[0]) % bx->B[1]) - bx->K[1];
    o[2] = (int)(bi / bx->s[2]) - bx->K[2];
    double rv[3];
    rbar_of(P->h, N, o, rv);
    double r = sqrt(rv[0] * rv[0] + rv[1] * rv[1] + rv[2] * rv[2]);
    oracle_ylm(L, rv[0], rv[1], rv[2], Y);
    double v = 0.0, rinv = 1.0 / r, rp = rinv; /* rp = r^-(l+1) */
    for (int l = 0; l <= L; ++l) {
      double s = 0.0;
      for (int m = -l; m <= l; ++m) s += Q[l * l + l + m] * Y[l * l + l + m];
      v += 4.0 * OR_PI * s * rp / (2.0 * l + 1.0);
      rp *= rinv;
    }
    W->vb[bi] = v;
  }

  /* right-hand side of the PE problem: 4 pi rho plus the stencil reach into
     the shell, where v takes its far-field values (eq. pe with eq. d2_1 along
     every arm of the NK Laplacian) */
  for (long k = 0; k < npe; ++k) {
    long bi = W->pe[k];
    double acc = 4.0 * OR_PI * W->rho[bi];
    for (int m = 0; m < X->S.n_arms; ++m) {
      long st = arm_stride(bx, X->S.arm[m].u);
      for (int qq = 1; qq <= n; ++qq)
        acc += X->S.arm[m].coef * X->w2[qq] * (W->vb[bi + qq * st] + W->vb[bi - qq * st]);
    }
    W->b[bi] = acc;
  }

  int conv = 0;
  double rel = 0.0;
  res->cg_iters = cg_solve(X, bx, W->pe, npe, W->b, W->x, W->r, W->p, W->q, &rel, &conv);
  res->converged = conv;
  res->rel_res = rel;
  /* true residual */
  apply_A(X, bx, W->pe, npe, W->x, W->q);
  {
    double t = 0.0, bb = 0.0;
    for (long k = 0; k < npe; ++k) {
      long bi = W->pe[k];
      double d = W->b[bi] - W->q[bi];
      t += d * d;
      bb += W->b[bi] * W->b[bi];
    }
    res->true_rel_res = bb > 0.0 ? sqrt(t / bb) : 0.0;
  }

  /* full potential on ME: CG solution on PE, far field on the shell */
  for (long k = 0; k < npe; ++k) W->vb[W->pe[k]] = W->x[W->pe[k]];

  /* energy (eq. exxGen_mlwf): -w dV sum_PE rho v */
  double e = 0.0;
  for (long k = 0; k < npe; ++k) e += W->rho[W->pe[k]] * W->vb[W->pe[k]];
  res->E = -w * X->dV * e;

  /* cell derivatives (eq. sxx_working): the Cartesian gradient of v from the
     first-derivative stencil along each lattice direction (eq. d1_1) and the
     Jacobian J_{a al} = |L_al| (h^-1)_{al a} (eq. jacb) */
  double J[9];
  for (int a = 0; a < 3; ++a)
    for (int al = 0; al < 3; ++al) M3(J, a, al) = col_norm(P->h, al) * M3(X->hinv, al, a);
  double T[9] = {0}; /* T[a + 3b] = sum_PE rbar_b rho dv/dr_a */
  for (long k = 0; k < npe; ++k) {
    long bi = W->pe[k];
    o[0] = (int)(bi % bx->B[0]) - bx->K[0];
    o[1] = (int)((bi / bx->B[0]) % bx->B[1]) - bx->K[1];
    o[2] = (int)(bi / bx->s[2]) - bx->K[2];
    double rv[3];
    rbar_of(P->h, N, o, rv);
    double dxi[3];
    for (int al = 0; al < 3; ++al) {
      double t = 0.0;
      for (int qq = 1; qq <= n; ++qq) t += X->w1[qq] * (W->vb[bi + qq * bx->s[al]] - W->vb[bi - qq * bx->s[al]]);
      dxi[al] = t / X->dxi[al];
    }
    for (int a = 0; a < 3; ++a) {
      double ga = M3(J, a, 0) * dxi[0] + M3(J, a, 1) * dxi[1] + M3(J, a, 2) * dxi[2];
      for (int b = 0; b < 3; ++b) T[a + 3 * b] += rv[b] * W->rho[bi] * ga;
    }
  }
  for (int a = 0; a < 3; ++a)
    for (int al = 0; al < 3; ++al) {
      double s = 0.0;
      for (int b = 0; b < 3; ++b) s += M3(X->hinv, al, b) * T[a + 3 * b];
      res->sigma[a + 3 * al] = -2.0 * w * X->dV * s;
    }

  /* shell term of the wavefunction-force identity and the ME list for D */
  double shell = 0.0;
  if (me) me->n = 0;
  for (long bi = 0; bi < bx->n; ++bi) {
    if (!W->mask[bi]) continue;
    o[0] = (int)(bi % bx->B[0]) - bx->K[0];
    o[1] = (int)((bi / bx->B[0]) % bx->B[1]) - bx->K[1];
    o[2] = (int)(bi / bx->s[2]) - bx->K[2];
    long g = wrap(res->c[0] + o[0], N[0]) +
             (long)N[0] * (wrap(res->c[1] + o[1], N[1]) + (long)N[1] * wrap(res->c[2] + o[2], N[2]));
    if (W->mask[bi] == 1) shell += phi_i[g] * phi_j[g] * W->vb[bi];
    if (me) {
      long t = me->n++;
      me->g[t] = g;
      me->v[t] = W->vb[bi];
      me->pi[t] = phi_i[g];
      me->pj[t] = phi_j[g];
    }
  }
  res->shell_rho_v = w * X->dV * shell;
  if (vout) memcpy(vout, W->vb, bx->n * sizeof(double));
  if (rout) memcpy(rout, W->rho, bx->n * sizeof(double));
  return 0;
}

/* ------------------------------------------------------------------------- */
/* public entry points                                                        */

void oracle_box_dims(const oracle_params* P, int* K) {
  ctx_t X;
  memset(&X, 0, sizeof(X));
  if (ctx_init(&X, P)) {
    K[0] = K[1] = K[2] = -1;
    return;
  }
  box_t bx;
  box_make(&X, &bx);
  for (int a = 0; a < 3; ++a) K[a] = bx.K[a];
}

/* Fields of a single pair (i, j) on the local box of oracle_box_dims (half-widths
   K, so (2K_0+1)(2K_1+1)(2K_2+1) points, x fastest, offset = index - K):
   rho_box (PE only), v_box (PE: CG solution, shell: far field, elsewhere 0),
   mask_box (0 outside ME, 1 shell, 2 PE).  res receives E, sigma and the CG
   diagnostics. */
int oracle_pair_fields(const oracle_params* P, int n_orb, const double* orb, const double* centres,
                       const double* R_orb, int i, int j, double* rho_box, double* v_box,
                       unsigned char* mask_box, oracle_pair_result* res) {
  ctx_t X;
  int rc = ctx_init(&X, P);
  if (rc) return rc;
  if (i < 0 || j < 0 || i >= n_orb || j >= n_orb) return -1;
  if (i > j) { int t = i; i = j; j = t; }
  double d[3], dm[3];
  for (int a = 0; a < 3; ++a) d[a] = centres[3 * j + a] - centres[3 * i + a];
  mic(&X, d, dm);
  memset(res, 0, sizeof(*res));
  res->i = i;
  res->j = j;
  double Cij[3];
  for (int a = 0; a < 3; ++a) Cij[a] = centres[3 * i + a] + 0.5 * dm[a];
  grid_centre(&X, Cij, res->c);
  res->R_PE = pair_radius(&X, R_orb, i, j);
  box_t bx;
  box_make(&X, &bx);
  work_t W;
  if (work_alloc(&W, &bx)) return -4;
  eval_pair(&X, &W, orb, res, NULL, v_box, rho_box);
  if (mask_box) memcpy(mask_box, W.mask, bx.n);
  work_free(&W);
  return 0;
}

/* Full evaluation: E_xx, D (may be NULL; [n_orb][N3][N2][N1], overwritten),
   sigma[9] (may be NULL), per-pair results (may be NULL, capacity cap).
   Pairs are evaluated in parallel; all accumulations run in pair order, so the
   result does not depend on the thread count.  Returns the number of pairs or
   a negative error code. */
long oracle_eval(const oracle_params* P, int n_orb, const double* orb, const double* centres,
                 const double* R_orb, double* E, double* D, double* sigma, oracle_pair_result* pairs_out,
                 long cap) {
  ctx_t X;
  int rc = ctx_init(&X, P);
  if (rc) return rc;
  long npairs = build_pairs(&X, n_orb, centres, R_orb, NULL, 0);
  oracle_pair_result* pr = (oracle_pair_result*)calloc(npairs > 0 ? npairs : 1, sizeof(oracle_pair_result));
  if (!pr) return -4;
  build_pairs(&X, n_orb, centres, R_orb, pr, npairs);
  box_t bx;
  box_make(&X, &bx);

  int nth = 1;
#ifdef _OPENMP
  nth = P->n_threads > 0 ? P->n_threads : omp_get_max_threads();
#endif
  long chunk = (long)nth * 2;
  me_list_t* me = (me_list_t*)calloc(chunk, sizeof(me_list_t));
  int fail = 0;
  for (long c = 0; c < chunk; ++c) {
    me[c].cap = bx.n;
    me[c].g = (long*)malloc(bx.n * sizeof(long));
    me[c].v = (double*)malloc(bx.n * sizeof(double));
    me[c].pi = (double*)malloc(bx.n * sizeof(double));
    me[c].pj = (double*)malloc(bx.n * sizeof(double));
    if (!me[c].g || !me[c].v || !me[c].pi || !me[c].pj) fail = 1;
  }
  if (D) memset(D, 0, (size_t)n_orb * X.ngrid * sizeof(double));

  for (long base = 0; base < npairs && !fail; base += chunk) {
    long cnt = npairs - base < chunk ? npairs - base : chunk;
#pragma omp parallel num_threads(nth)
    {
      work_t W;
      int ok = work_alloc(&W, &bx) == 0;
      if (!ok) {
#pragma omp atomic write
        fail = 1;
      }
#pragma omp for schedule(dynamic, 1)
      for (long k = 0; k < cnt; ++k) {
        if (ok) eval_pair(&X, &W, orb, &pr[base + k], D ? &me[k] : NULL, NULL, NULL);
      }
      if (ok) work_free(&W);
    }
    if (D) {
      for (long k = 0; k < cnt; ++k) {
        const oracle_pair_result* r = &pr[base + k];
        double* Di = D + (long)r->i * X.ngrid;
        double* Dj = D + (long)r->j * X.ngrid;
        for (long t = 0; t < me[k].n; ++t) {
          /* D^i += v phi_j, D^j += v phi_i (eq. Dxx for both orderings) */
          Di[me[k].g[t]] += me[k].v[t] * me[k].pj[t];
          if (r->i != r->j) Dj[me[k].g[t]] += me[k].v[t] * me[k].pi[t];
        }
      }
    }
  }
  for (long c = 0; c < chunk; ++c) {
    free(me[c].g); free(me[c].v); free(me[c].pi); free(me[c].pj);
  }
  free(me);
  if (fail) {
    free(pr);
    return -4;
  }
  double e = 0.0, s[9] = {0};
  for (long k = 0; k < npairs; ++k) {
    e += pr[k].E;
    for (int t = 0; t < 9; ++t) s[t] += pr[k].sigma[t];
  }
  if (E) *E = e;
  if (sigma) memcpy(sigma, s, sizeof(s));
  if (pairs_out) memcpy(pairs_out, pr, (npairs < cap ? npairs : cap) * sizeof(oracle_pair_result));
  free(pr);
  return npairs;
}

/* Operator pieces exposed for the stencil and CG checks: A applied on a box
   with a membership mask (2 = unknown point), and CG on that mask.  K holds
   the box's half-widths: 2K_a+1 points along axis a, x fastest. */
static int box_from_dims(const int* K, box_t* bx) {
  for (int a = 0; a < 3; ++a) {
    if (K[a] < 0) return -1;
    bx->K[a] = K[a];
    bx->B[a] = 2 * K[a] + 1;
  }
  bx->s[0] = 1;
  bx->s[1] = bx->B[0];
  bx->s[2] = (long)bx->B[0] * bx->B[1];
  bx->n = (long)bx->B[0] * bx->B[1] * bx->B[2];
  return 0;
}

static long mask_list(const box_t* bx, int reach, const unsigned char* mask, long* pe) {
  long npe = 0;
  for (int z = reach; z < bx->B[2] - reach; ++z)
    for (int y = reach; y < bx->B[1] - reach; ++y)
      for (int x = reach; x < bx->B[0] - reach; ++x) {
        long bi = x + bx->s[1] * y + bx->s[2] * z;
        if (mask[bi] == 2) pe[npe++] = bi;
      }
  return npe;
}

/* the three axis arms of an orthorhombic grid with the given spacings */
static void axis_arms(ctx_t* X, const double* spacing) {
  memset(&X->S, 0, sizeof(X->S));
  X->S.n_arms = 3;
  X->umax = 1;
  for (int a = 0; a < 3; ++a) {
    X->dxi[a] = spacing[a];
    nk_arm* A = &X->S.arm[a];
    A->u[a] = 1;
    A->beta = 1.0;
    A->step = spacing[a];
    A->coef = 1.0 / (spacing[a] * spacing[a]);
  }
}

/* -(sum over arms of coef * eq. d2_1 along u) on the mask == 2 points of a box;
   n_arms arms with steps u[3 k + al] and coefficients coef[k] */
int oracle_apply_arms(const int* K, int n, int n_arms, const int* u, const double* coef, const unsigned char* mask,
                      const double* p, double* q) {
  ctx_t X;
  memset(&X, 0, sizeof(X));
  box_t bx;
  if (box_from_dims(K, &bx) || n < 1 || n > 3 || n_arms < 1 || n_arms > OR_MAX_ARMS) return -1;
  X.P.stencil_n = n;
  oracle_stencil_weights(n, X.w2, X.w1);
  X.S.n_arms = n_arms;
  X.umax = 1;
  for (int k = 0; k < n_arms; ++k) {
    for (int al = 0; al < 3; ++al) {
      X.S.arm[k].u[al] = u[3 * k + al];
      if (abs(u[3 * k + al]) > X.umax) X.umax = abs(u[3 * k + al]);
    }
    X.S.arm[k].coef = coef[k];
  }
  long* pe = (long*)malloc(bx.n * sizeof(long));
  if (!pe) return -4;
  long npe = mask_list(&bx, n * X.umax, mask, pe);
  double* pm = (double*)calloc(bx.n, sizeof(double));
  for (long k = 0; k < npe; ++k) pm[pe[k]] = p[pe[k]];
  memset(q, 0, bx.n * sizeof(double));
  apply_A(&X, &bx, pe, npe, pm, q);
  free(pm);
  free(pe);
  return 0;
}

int oracle_apply_A(const int* K, const double* spacing, int n, const unsigned char* mask, const double* p,
                   double* q) {
  ctx_t X;
  memset(&X, 0, sizeof(X));
  box_t bx;
  if (box_from_dims(K, &bx) || n < 1 || n > 3) return -1;
  X.P.stencil_n = n;
  axis_arms(&X, spacing);
  oracle_stencil_weights(n, X.w2, X.w1);
  long* pe = (long*)malloc(bx.n * sizeof(long));
  if (!pe) return -4;
  long npe = mask_list(&bx, n, mask, pe);
  double* pm = (double*)calloc(bx.n, sizeof(double));
  for (long k = 0; k < npe; ++k) pm[pe[k]] = p[pe[k]];
  memset(q, 0, bx.n * sizeof(double));
  apply_A(&X, &bx, pe, npe, pm, q);
  free(pm);
  free(pe);
  return 0;
}

int oracle_cg_mask(const int* K, const double* spacing, int n, const unsigned char* mask, const double* b,
                   double tol, int max_iter, double* x, int* iters, double* rel_res) {
  ctx_t X;
  memset(&X, 0, sizeof(X));
  box_t bx;
  if (box_from_dims(K, &bx) || n < 1 || n > 3) return -1;
  X.P.stencil_n = n;
  X.P.cg_tol = tol;
  X.P.cg_max_iter = max_iter;
  axis_arms(&X, spacing);
  oracle_stencil_weights(n, X.w2, X.w1);
  long* pe = (long*)malloc(bx.n * sizeof(long));
  double* r = (double*)calloc(bx.n, sizeof(double));
  double* p = (double*)calloc(bx.n, sizeof(double));
  double* q = (double*)calloc(bx.n, sizeof(double));
  if (!pe || !r || !p || !q) { free(pe); free(r); free(p); free(q); return -4; }
  long npe = mask_list(&bx, n, mask, pe);
  memset(x, 0, bx.n * sizeof(double));
  int conv = 0;
  *iters = cg_solve(&X, &bx, pe, npe, b, x, r, p, q, rel_res, &conv);
  free(pe); free(r); free(p); free(q);
  return conv ? 0 : 1;
}
