/*
 * hsgn_oracle.h -- plain FP64 CPU oracle for the semi-implicit IMEX scheme
 * for the hyperbolic Serre-Green-Naghdi (hSGN) equations
 * (Macca, Boscheri, Ricchiuto, arXiv 2510.07539).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this code: only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code, header, constant or helper with
 * the HIP library.
 *
 * State per cell: h (depth), q = hu, m = h*eta, W = h*w; optional bed b.
 * All arrays are FP64, one instance = n contiguous cells.
 */
#ifndef HSGN_ORACLE_H
#define HSGN_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  double g;        /* gravity */
  double lambda;   /* relaxation parameter of the hSGN system */
  double dx;       /* uniform cell width */
  double cfl;      /* CFL on max(|u| + sqrt(g h)) */
  double mcfl;     /* material CFL cap on max|u| dt / dx (<= 0: no cap) */
  double dt_fixed; /* > 0: use this time step */
  double t_end;    /* > 0: clamp the last step to t_end; <= 0: no clamp */
  int bc;          /* 0 periodic, 1 transmissive */
  int has_b;       /* 1: bed b is used; 0: flat bottom (b ignored) */
  int order;       /* 1: first-order scheme (one stage, tau = dt, no
                      reconstruction); otherwise the two-stage IMEX step */
  int scheme;      /* 0: semi-implicit (above); 1: fully explicit hSGN with
                      Heun's method (flat bottom; cfl applies to |u| + c);
                      2: standard SGN, elliptic-hyperbolic form, Heun's
                      method (flat bottom; lambda unused; m, W untouched) */
  int form;        /* semi-implicit stage only.  0: the implicit pressure
                      differenced in conservative P-form (the oracle of the
                      library).  1: "mode A", the printed lines of Sec. 4.2
                      (eq. GN_hyp_eq_semi_fully_discrete: the beta
                      Laplacian Delta[h], the delta Laplacian of h*eta in
                      h-dagger with weight lambda tau^2/dx^2 on face means,
                      and the printed momentum update); flat bottom only.
                      CPU only: it exists to compare the P-form with the
                      print. */
} or_params;

/* Optional per-stage intermediates (any pointer may be NULL). Cell arrays
 * have n entries; face arrays have n+1 entries (face k sits between cells
 * k-1 and k). */
typedef struct {
  double *qd, *md, *Wd;              /* q-dagger, m-dagger, W-dagger */
  double *beta, *S, *phi, *T;        /* linearisation coefficients */
  double *P0, *pt0;                  /* pressure and p-tilde at h = h_E */
  double *lo, *di, *up, *rhs;        /* assembled rows of the h-bar system */
  double *hbar;                      /* solved depth */
  double *Fq, *Fm, *FW;              /* explicit Rusanov face fluxes */
} or_stage_dbg;

enum { OR_OK = 0, OR_ENONPHYS = 1, OR_ENONCOERCIVE = 2, OR_EINVAL = 3 };

/* IMEX tableau constants (gamma = 1 - 1/sqrt(2), c = 1/(2 gamma)). */
double or_gamma(void);
/* out[5] = {gamma, 1 - c/gamma, c/gamma, 1 - (1-gamma)/gamma, (1-gamma)/gamma} */
void or_tableau(double* out);

/* One first-order semi-implicit stage with step tau:
 * U_new = U_old + tau * H(U_E, U_new), explicit terms from U_E. */
int or_stage(int n, const or_params* p, double tau, const double* b,
             const double* hE, const double* qE, const double* mE, const double* WE,
             const double* ho, const double* qo, const double* mo, const double* Wo,
             double* hn, double* qn, double* mn, double* Wn, or_stage_dbg* dbg);

/* Time step from the state (CFL, material-CFL cap, t_end clamp). */
double or_dt(int n, const or_params* p, const double* h, const double* q, double t);

/* Time step of the explicit scheme: CFL on |u| + c, c^2 = g h + (lambda/3)(m/h^2)^2. */
double or_dt_ex(int n, const or_params* p, const double* h, const double* q, const double* m,
                double t);

/* One full step, in place: the two-stage IMEX step, the first-order
 * semi-implicit step (order 1), the explicit Heun step (scheme 1), or the
 * standard SGN Heun step (scheme 2).
 * *t advances by the step used; *dt_out (may be NULL) receives it.  A zero
 * step leaves the state frozen. */
int or_step(int n, const or_params* p, const double* b,
            double* h, double* q, double* m, double* W, double* t, double* dt_out);

/* nsteps steps of one instance. */
int or_run(int n, const or_params* p, const double* b,
           double* h, double* q, double* m, double* W, double* t, int nsteps);

/* Gauge misfit of nsteps steps: after step s the loss gains
 * (1/2) sum_g (h[gauge[g]] - target[s*ng + g])^2.  State updated in place. */
int or_run_loss(int n, const or_params* p, const double* b, double* h, double* q,
                double* m, double* W, int nsteps, int ng, const int* gauge,
                const double* target, double* loss);

/* Gauge series of nsteps steps: series[s*ng + g] = h[gauge[g]] after step
 * s + 1 (double build only).  State updated in place. */
int or_run_gauges(int n, const or_params* p, const double* b, double* h, double* q,
                  double* m, double* W, int nsteps, int ng, const int* gauge, double* series);

/* Complex-step build (hsgn_oracle_cs.c, library liboracle_cs.so): the same
 * functions on double complex state with the suffix _cs (or_stage_cs,
 * or_step_cs, or_run_cs, or_run_loss_cs, or_tridiag_cs, or_dt_cs).  Im of the result
 * for an input perturbed by i*eps*v, divided by eps, is the directional
 * derivative of the double build to rounding. */

/* Independent instances concatenated: instance j owns cells
 * [offsets[j], offsets[j+1]).  OpenMP over instances with nthreads threads
 * (<= 0: library default).  status[j] receives each instance's code. */
int or_run_batch(int n_inst, const long long* offsets, const or_params* p,
                 const double* b, double* h, double* q, double* m, double* W,
                 double* t, int nsteps, int nthreads, int* status);

/* phi of the standard SGN elliptic problem (scheme 2) for the state (h, q). */
int or_sgn_phi(int n, const or_params* p, const double* h, const double* q, double* phi);

/* Tridiagonal solve: row i reads lo[i] x[i-1] + di[i] x[i] + up[i] x[i+1].
 * cyclic != 0: lo[0] couples x[n-1] and up[n-1] couples x[0]. */
int or_tridiag(int n, int cyclic, const double* lo, const double* di,
               const double* up, const double* rhs, double* x);

/* Number of OpenMP threads the batch runner would use. */
int or_max_threads(void);

#ifdef __cplusplus
}
#endif
#endif
