/* oracle_check.c -- drives every entry point of the CPU oracle (double and
 * complex-step builds) over small and ragged sizes, both boundary types,
 * flat and bed, every scheme, order and form, so that a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer checks the oracle's
 * memory accesses and arithmetic (test infrastructure: built and run by
 * tests/test_sanitize.py).  Prints one line per case; exits non-zero on
 * an unexpected return code. */
#include <complex.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "hsgn_oracle.h"

int or_stage_cs(int n, const or_params* p, double tau, const double complex* b,
                const double complex* hE, const double complex* qE, const double complex* mE,
                const double complex* WE, const double complex* ho, const double complex* qo,
                const double complex* mo, const double complex* Wo, double complex* hn,
                double complex* qn, double complex* mn, double complex* Wn, or_stage_dbg* dbg);
int or_run_cs(int n, const or_params* p, const double complex* b, double complex* h,
              double complex* q, double complex* m, double complex* W, double* t, int nsteps);
int or_tridiag_cs(int n, int cyclic, const double complex* lo, const double complex* di,
                  const double complex* up, const double complex* rhs, double complex* x);

static int failures = 0;

static void check(const char* what, int n, int rc, int want) {
  printf("%-28s n=%5d rc=%d\n", what, n, rc);
  fflush(stdout);
  if (rc != want) {
    fprintf(stderr, "%s n=%d: rc %d, expected %d\n", what, n, rc, want);
    ++failures;
  }
}

/* a smooth positive state: a hump on h0 over an optional bar-like bed */
static void state(int n, double dx, int bed, double* b, double* h, double* q, double* m,
                  double* W) {
  const double L = n * dx;
  for (int i = 0; i < n; ++i) {
    const double x = (i + 0.5) * dx;
    b[i] = bed ? 0.1 * exp(-pow((x - 0.6 * L) / (0.1 * L), 2)) : 0.0;
    const double z = 0.5 + 0.05 * exp(-pow((x - 0.3 * L) / (0.08 * L), 2));
    h[i] = z - b[i];
    q[i] = 0.02 * h[i] * sin(6.283185307179586 * x / L);
    m[i] = h[i] * h[i];
    W[i] = 0.0;
  }
}

static or_params params(int bc, int bed, int order, int scheme, int form) {
  or_params p;
  p.g = 9.81;
  p.lambda = 300.0;
  p.dx = 0.05;
  p.cfl = scheme == 1 ? 0.4 : 0.9;
  p.mcfl = 0.5;
  p.dt_fixed = 0.0;
  p.t_end = 0.0;
  p.bc = bc;
  p.has_b = bed;
  p.order = order;
  p.scheme = scheme;
  p.form = form;
  return p;
}

int main(void) {
  const int sizes[] = {4, 5, 7, 8, 31, 64, 257};
  const int nsz = (int)(sizeof sizes / sizeof sizes[0]);
  double tab[5];
  or_tableau(tab);
  printf("gamma %.17g threads %d\n", or_gamma(), or_max_threads());
  for (int si = 0; si < nsz; ++si) {
    const int n = sizes[si];
    double *b = malloc(n * sizeof(double)), *h = malloc(n * sizeof(double)),
           *q = malloc(n * sizeof(double)), *m = malloc(n * sizeof(double)),
           *W = malloc(n * sizeof(double));
    double *hn = malloc(n * sizeof(double)), *qn = malloc(n * sizeof(double)),
           *mn = malloc(n * sizeof(double)), *Wn = malloc(n * sizeof(double)),
           *phi = malloc(n * sizeof(double));
    double *dbgc[14], *dbgf[3];
    for (int k = 0; k < 14; ++k) dbgc[k] = malloc(n * sizeof(double));
    for (int k = 0; k < 3; ++k) dbgf[k] = malloc((n + 1) * sizeof(double));
    for (int bc = 0; bc <= 1; ++bc) {
      for (int bed = 0; bed <= 1; ++bed) {
        /* one stage with every intermediate recorded */
        or_params p = params(bc, bed, 2, 0, 0);
        state(n, p.dx, bed, b, h, q, m, W);
        or_stage_dbg d = {.qd = dbgc[0], .md = dbgc[1], .Wd = dbgc[2], .beta = dbgc[3],
                          .S = dbgc[4], .phi = dbgc[5], .T = dbgc[6], .P0 = dbgc[7],
                          .pt0 = dbgc[8], .lo = dbgc[9], .di = dbgc[10], .up = dbgc[11],
                          .rhs = dbgc[12], .hbar = dbgc[13], .Fq = dbgf[0], .Fm = dbgf[1],
                          .FW = dbgf[2]};
        check("or_stage", n, or_stage(n, &p, 0.01, b, h, q, m, W, h, q, m, W, hn, qn, mn, Wn, &d),
              OR_OK);
        /* every scheme, order and form over a few steps */
        for (int scheme = 0; scheme <= 2; ++scheme) {
          for (int order = 1; order <= 2; ++order) {
            for (int form = 0; form <= 1; ++form) {
              if (scheme != 0 && (order == 1 || form == 1)) continue;
              const int want_bed_ok = scheme == 0 && form == 0;
              or_params ps = params(bc, bed && want_bed_ok, order, scheme, form);
              state(n, ps.dx, bed && want_bed_ok, b, h, q, m, W);
              double t = 0.0, dt = 0.0;
              char name[64];
              snprintf(name, sizeof name, "or_step s%d o%d f%d bc%d b%d", scheme, order, form, bc,
                       bed && want_bed_ok);
              check(name, n, or_step(n, &ps, b, h, q, m, W, &t, &dt), OR_OK);
              snprintf(name, sizeof name, "or_run s%d o%d f%d", scheme, order, form);
              check(name, n, or_run(n, &ps, b, h, q, m, W, &t, 3), OR_OK);
            }
          }
        }
        /* time steps, t_end clamp, fixed step */
        p = params(bc, bed, 2, 0, 0);
        p.t_end = 0.05;
        state(n, p.dx, bed, b, h, q, m, W);
        printf("or_dt %g or_dt_ex %g\n", or_dt(n, &p, h, q, 0.0), or_dt_ex(n, &p, h, q, m, 0.0));
        p.dt_fixed = 0.004;
        p.t_end = 0.0;
        /* gauge recorder and loss */
        int gauge[2] = {0, n - 1};
        double* target = malloc(6 * sizeof(double));
        double* series = malloc(6 * sizeof(double));
        for (int k = 0; k < 6; ++k) target[k] = 0.5;
        check("or_run_gauges", n, or_run_gauges(n, &p, b, h, q, m, W, 3, 2, gauge, series), OR_OK);
        double loss = 0.0;
        check("or_run_loss", n, or_run_loss(n, &p, b, h, q, m, W, 3, 2, gauge, target, &loss),
              OR_OK);
        free(target);
        free(series);
        /* SGN elliptic problem */
        or_params pg = params(bc, 0, 2, 2, 0);
        state(n, pg.dx, 0, b, h, q, m, W);
        check("or_sgn_phi", n, or_sgn_phi(n, &pg, h, q, phi), OR_OK);
        /* tridiagonal solves */
        for (int i = 0; i < n; ++i) {
          dbgc[0][i] = -1.0;
          dbgc[1][i] = 4.0;
          dbgc[2][i] = -1.0;
          dbgc[3][i] = 1.0 + i;
        }
        check("or_tridiag", n, or_tridiag(n, bc == 0, dbgc[0], dbgc[1], dbgc[2], dbgc[3], phi),
              OR_OK);
        /* complex-step build */
        double complex *cb = malloc(n * sizeof(double complex)),
                       *ch = malloc(n * sizeof(double complex)),
                       *cq = malloc(n * sizeof(double complex)),
                       *cm = malloc(n * sizeof(double complex)),
                       *cW = malloc(n * sizeof(double complex)),
                       *cx = malloc(n * sizeof(double complex));
        state(n, p.dx, bed, b, h, q, m, W);
        for (int i = 0; i < n; ++i) {
          cb[i] = b[i];
          ch[i] = h[i] + 1e-30 * I;
          cq[i] = q[i];
          cm[i] = m[i];
          cW[i] = W[i];
        }
        double t = 0.0;
        or_params pc = params(bc, bed, 2, 0, 0);
        check("or_run_cs", n, or_run_cs(n, &pc, cb, ch, cq, cm, cW, &t, 2), OR_OK);
        check("or_stage_cs", n,
              or_stage_cs(n, &pc, 0.01, cb, ch, cq, cm, cW, ch, cq, cm, cW, cx, cq, cm, cW, NULL),
              OR_OK);
        for (int i = 0; i < n; ++i) {
          cb[i] = -1.0;
          ch[i] = 4.0;
          cq[i] = -1.0;
          cm[i] = 1.0 + i * I;
        }
        check("or_tridiag_cs", n, or_tridiag_cs(n, bc == 0, cb, ch, cq, cm, cx), OR_OK);
        free(cb); free(ch); free(cq); free(cm); free(cW); free(cx);
      }
    }
    /* invalid input is rejected: a stage with dx = 0, a solve of no rows */
    or_params bad = params(1, 0, 2, 0, 0);
    bad.dx = 0.0;
    state(n, 0.05, 0, b, h, q, m, W);
    check("or_stage (dx = 0)", n,
          or_stage(n, &bad, 0.01, b, h, q, m, W, h, q, m, W, hn, qn, mn, Wn, NULL), OR_EINVAL);
    check("or_tridiag (0 rows)", 0, or_tridiag(0, 0, h, h, h, h, phi), OR_EINVAL);
    for (int k = 0; k < 14; ++k) free(dbgc[k]);
    for (int k = 0; k < 3; ++k) free(dbgf[k]);
    free(b); free(h); free(q); free(m); free(W); free(hn); free(qn); free(mn); free(Wn);
    free(phi);
  }
  /* the batch runner with two threads over uneven instances */
  {
    const int ni = 3;
    long long off[4] = {0, 9, 40, 297};
    const int nt = (int)off[ni];
    double *b = calloc(nt, sizeof(double)), *h = malloc(nt * sizeof(double)),
           *q = malloc(nt * sizeof(double)), *m = malloc(nt * sizeof(double)),
           *W = malloc(nt * sizeof(double)), *t = calloc(ni, sizeof(double));
    int status[3];
    or_params p[3] = {params(0, 0, 2, 0, 0), params(1, 1, 2, 0, 0), params(1, 0, 1, 0, 0)};
    for (int j = 0; j < ni; ++j)
      state((int)(off[j + 1] - off[j]), p[j].dx, p[j].has_b, b + off[j], h + off[j], q + off[j],
            m + off[j], W + off[j]);
    check("or_run_batch", nt, or_run_batch(ni, off, p, b, h, q, m, W, t, 4, 2, status), OR_OK);
    free(b); free(h); free(q); free(m); free(W); free(t);
  }
  printf("%s\n", failures ? "FAILED" : "all cases ran");
  return failures ? 1 : 0;
}
