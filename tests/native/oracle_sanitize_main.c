/* Drives every entry point of the FP64 oracle on small cells, for a build
   with AddressSanitizer and UndefinedBehaviorSanitizer: orthorhombic and
   triclinic cells, variable and self radii, a sampled pair subset, the masked
   stencil and CG checks.  Prints one line per case and exits non-zero on a
   failed return code (the sanitizers abort on their own findings). */
#include <stdio.h>

#include "../../oracle/exx_oracle.c"

static void gauss_orbitals(const double* h, const int* N, int n_orb, const double* C, double* orb) {
  const long ng = (long)N[0] * N[1] * N[2];
  for (int o = 0; o < n_orb; ++o)
    for (int k = 0; k < N[2]; ++k)
      for (int j = 0; j < N[1]; ++j)
        for (int i = 0; i < N[0]; ++i) {
          const double f[3] = {(double)i / N[0], (double)j / N[1], (double)k / N[2]};
          double r2 = 0.0;
          for (int a = 0; a < 3; ++a) {
            double d = 0.0;
            for (int al = 0; al < 3; ++al) d += h[a + 3 * al] * f[al];
            d -= C[3 * o + a];
            r2 += d * d;   /* no minimum image: the centres sit mid-cell */
          }
          orb[o * ng + ((long)k * N[1] + j) * N[0] + i] = exp(-0.8 * r2) * (1.0 + 0.1 * o);
        }
}

static int run_eval(const char* name, const oracle_params* P, int n_orb, const double* C, const double* R_orb) {
  const long ng = (long)P->grid[0] * P->grid[1] * P->grid[2];
  double* orb = (double*)malloc(sizeof(double) * n_orb * ng);
  double* D = (double*)malloc(sizeof(double) * n_orb * ng);
  oracle_pair_result pr[64];
  gauss_orbitals(P->h, P->grid, n_orb, C, orb);
  double E = 0.0, sigma[9];
  const long np = oracle_eval(P, n_orb, orb, C, R_orb, &E, D, sigma, pr, 64);
  int K[3];
  oracle_box_dims(P, K);
  if (K[0] <= 0) {
    printf("%s: invalid parameters (oracle_eval returned %ld)\n", name, np);
    free(orb);
    free(D);
    return 1;
  }
  const long nb = (2L * K[0] + 1) * (2L * K[1] + 1) * (2L * K[2] + 1);   /* K: half-widths */
  double* rho = (double*)malloc(sizeof(double) * nb);
  double* v = (double*)malloc(sizeof(double) * nb);
  unsigned char* mask = (unsigned char*)malloc(nb);
  oracle_pair_result one;
  const int rc = oracle_pair_fields(P, n_orb, orb, C, R_orb, 0, n_orb - 1, rho, v, mask, &one);
  const long npl = oracle_pair_list(P, n_orb, C, R_orb, NULL, 0);
  printf("%s: pairs %ld (list %ld) E %.12e box %dx%dx%d fields rc %d E01 %.6e\n", name, np, npl, E, K[0], K[1], K[2],
         rc, one.E);
  free(orb);
  free(D);
  free(rho);
  free(v);
  free(mask);
  return (np > 0 && rc == 0 && np == npl) ? 0 : 1;
}

static void base_params(oracle_params* P, const double* h, int N) {
  memset(P, 0, sizeof(*P));
  memcpy(P->h, h, sizeof(double) * 9);
  memcpy(P->h_geom, h, sizeof(double) * 9);
  P->grid[0] = P->grid[1] = P->grid[2] = N;
  P->R_pair = 6.0;
  P->R_PE = 2.6;
  P->R_ME = 4.8;
  P->l_max = 4;
  P->stencil_n = 3;
  P->cg_tol = 1e-8;
  P->cg_max_iter = 400;
  P->sample_frac = 1.0;
  P->n_threads = 2;
}

int main(void) {
  int fails = 0;
  const double ortho[9] = {10, 0, 0, 0, 11, 0, 0, 0, 12};
  const double tric[9] = {10, 0, 0, 1.5, 10, 0, 1.0, -1.2, 10};
  const double C[9] = {5.0, 5.5, 6.0, 6.1, 5.2, 6.4, 4.4, 6.3, 5.1};
  const double R_orb[3] = {2.2, 2.9, 2.5};
  oracle_params P;

  base_params(&P, ortho, 20);
  fails += run_eval("orthorhombic n=3", &P, 3, C, NULL);
  P.stencil_n = 1;
  fails += run_eval("orthorhombic n=1", &P, 3, C, NULL);
  base_params(&P, tric, 20);
  fails += run_eval("triclinic", &P, 3, C, NULL);
  P.grid[0] = 18;
  P.grid[2] = 23;
  P.l_max = 6;
  fails += run_eval("triclinic 18x20x23", &P, 3, C, NULL);
  base_params(&P, ortho, 20);
  P.R_PE_min = 2.0;
  P.R_PE_step = 0.4;
  P.R_PE_nclass = 3;
  fails += run_eval("variable radii", &P, 3, C, R_orb);
  base_params(&P, ortho, 20);
  P.R_PE_self = 2.0;
  P.R_ME_self = 4.0;
  fails += run_eval("self radii", &P, 3, C, NULL);
  base_params(&P, ortho, 20);
  P.sample_frac = 0.5;
  P.sample_seed = 7;
  {
    /* a sampled subset may hold any number of pairs, also none */
    const long ng = 20L * 20 * 20;
    double* orb = (double*)malloc(sizeof(double) * 3 * ng);
    gauss_orbitals(P.h, P.grid, 3, C, orb);
    double E = 0.0;
    const long np = oracle_eval(&P, 3, orb, C, NULL, &E, NULL, NULL, NULL, 0);
    printf("sampled: pairs %ld E %.12e\n", np, E);
    fails += np < 0;
    free(orb);
  }

  /* the NK stencil of the triclinic cell */
  {
    int N[3] = {20, 20, 20}, u[3 * 16], aux[9];
    double beta[16], step[16], b[3];
    const int na = oracle_nk_stencil(tric, N, u, beta, step, aux, b);
    printf("nk arms %d\n", na);
    fails += na <= 0;
  }

  /* the masked stencil and CG on a 13^3 box with a spherical mask */
  {
    const int K[3] = {6, 6, 6};   /* half-widths: a 13^3 box */
    const double sp[3] = {0.5, 0.55, 0.6};
    const long n = 13L * 13 * 13;
    unsigned char* mask = (unsigned char*)calloc(n, 1);
    double *p = (double*)malloc(sizeof(double) * n), *q = (double*)malloc(sizeof(double) * n);
    double *bb = (double*)malloc(sizeof(double) * n), *x = (double*)malloc(sizeof(double) * n);
    for (int k = 0; k < 13; ++k)
      for (int j = 0; j < 13; ++j)
        for (int i = 0; i < 13; ++i) {
          const long t = ((long)k * 13 + j) * 13 + i;
          const int r2 = (i - 6) * (i - 6) + (j - 6) * (j - 6) + (k - 6) * (k - 6);
          mask[t] = r2 <= 9 ? 2 : 0;
          p[t] = sin(0.3 * t);
          bb[t] = mask[t] ? cos(0.7 * t) : 0.0;
        }
    int rc = oracle_apply_A(K, sp, 3, mask, p, q);
    const int u[9] = {1, 0, 0, 0, 1, 0, 1, 1, 0};
    const double coef[3] = {1.0, 0.8, 0.3};
    rc |= oracle_apply_arms(K, 2, 3, u, coef, mask, p, q);
    int it = 0;
    double rr = 0.0;
    rc |= oracle_cg_mask(K, sp, 3, mask, bb, 1e-10, 500, x, &it, &rr);
    printf("mask stencil rc %d, cg iterations %d rel %.3e\n", rc, it, rr);
    fails += rc != 0;
    free(mask);
    free(p);
    free(q);
    free(bb);
    free(x);
  }
  {
    double w2[4], w1[4], y[(OR_MAXL + 1) * (OR_MAXL + 1)];
    for (int n = 1; n <= 3; ++n) oracle_stencil_weights(n, w2, w1);
    oracle_ylm(OR_MAXL, 0.3, -0.4, 0.5, y);
    oracle_ylm(4, 0.0, 0.0, 0.0, y);
  }
  printf("failures %d\n", fails);
  return fails ? 1 : 0;
}
