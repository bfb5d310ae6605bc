/*
 * hsgn_oracle.c -- plain, slow, obviously-correct FP64 CPU oracle of the
 * semi-implicit (IMEX) hSGN time step of Macca, Boscheri & Ricchiuto,
 * "Semi-implicit strategies for the Serre-Green-Naghdi equations in
 * hyperbolic form" (arXiv 2510.07539).
 *
 * TEST INFRASTRUCTURE ONLY: it exists to check the HIP library; the product
 * path never links or calls it.  No blocking, fusion or reordering: every
 * stage follows the paper's order (explicit convective predictor, exact
 * relaxation elimination, linearised elliptic problem for the new depth,
 * back-substitution), one loop per formula.
 *
 * Readings of the paper taken here:
 *  - the stage is the fully discrete first-order semi-implicit step of
 *    Sec. 4.2 (eq. GN_hyp_eq_semi_fully_discrete) with dt -> tau, explicit
 *    terms and frozen coefficients taken from the explicit stage value U_E,
 *    "old" values from the implicit combination (Sec. 3.2, eq. tableau);
 *  - the implicit pressure is differenced in conservative form: the
 *    linearised pressure P = P0 + beta (hbar - h_E), with the paper's beta
 *    (Sec. 4.2) and P0 the exact pressure at hbar = h_E, is differenced at
 *    faces, instead of applying central differences to hbar and h*eta
 *    separately;
 *  - the Rusanov speed is max(|u| + sqrt(g h)) over the two face states
 *    (the paper writes "alpha ~ |u|", which leaves the explicit acoustic
 *    coupling undamped at rest);
 *  - with a bed, m = h*eta is stored and its equation carries the exact
 *    rewrite source -(3/2) q b_x of the h*eta-tilde equation (eq. hSGNb_eq);
 *    the momentum source (g h + (3/2) p~) b_x is treated implicitly with
 *    p~ linearised like P; the m-diffusion of the Rusanov flux subtracts the
 *    face-local lake-at-rest moment so that rest is preserved;
 *  - boundary conditions: periodic, or transmissive (zero-order copy into
 *    two ghost cells, zero implicit force at the boundary face).
 *
 * The fully explicit hSGN scheme of Sec. 4.1 (eq. GN_hyp_eq_explicit) with
 * Heun's method is here too (scheme = 1, flat bottom), with two departures
 * from the print, both needed for linear stability at rest: the mass flux is
 * a Rusanov flux like the other three (the print differences q centrally),
 * and the Rusanov speed is max(|u| + c) over the two face states with the
 * hSGN celerity c^2 = g h + (lambda/3) (eta/h)^2 (eq. hSGN_c), the
 * eigenvalues of the system it treats explicitly (the print has |u|).  At
 * rest and CFL 0.4 one step as printed grows by a factor 1.0014 (lambda =
 * 100) and 1.0012 (lambda = 1000); with speed |u| + c but the central mass
 * flux by 1.011 and 1.029.  The pressure terms stay central as printed.
 *
 * The standard SGN equations in the elliptic-hyperbolic form of Sec. 4.3
 * (eq. SGN_standard; scheme = 2, flat bottom, lambda unused) are here as the
 * explicit scheme of Sec. 4.4 with Heun's method.  Readings: the g-term of
 * the right-hand side h* carries h^3 (as its derivation from eq. SGN_standard
 * and the units require; the print has h); h^3 at a face is the mean of the
 * two cell values; the Rusanov speed of the shallow-water fluxes is
 * max(|u| + sqrt(g h)); at a transmissive boundary phi has zero gradient
 * (the ghost copies the boundary cell, as for the state).
 */
#include "hsgn_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* The same source builds twice: with real_t = double (the oracle), and with
 * real_t = double complex (OR_COMPLEX) for complex-step derivatives
 * (Im f(x + i e v) / e = f'(x) v to rounding for e ~ 1e-30): branches and
 * comparisons act on real parts, |x| is x sign(Re x), max picks by real part,
 * so the complex build differentiates exactly the double build's arithmetic.
 * Exported names of the complex build carry the suffix _cs. */
#ifdef OR_COMPLEX
#include <complex.h>
typedef double complex real_t;
#define RE(x) creal(x)
#define RSQRT(x) csqrt(x)
#define FN(name) name##_cs
#else
typedef double real_t;
#define RE(x) (x)
#define RSQRT(x) sqrt(x)
#define FN(name) name
#endif
#define RABS(x) (RE(x) < 0.0 ? -(x) : (x))
#define RMAX(a, b) (RE(a) > RE(b) ? (a) : (b))

/* Double Butcher tableau of Sec. 3.2 (eq. tableau): gamma = 1 - 1/sqrt(2),
 * c = 1/(2 gamma).  Efficient form of the remark after the tableau:
 *   U_E^(2) = (1 - c/gamma) U^n + (c/gamma) U_I^(1)
 *   U~      = (1 - (1-gamma)/gamma) U^n + ((1-gamma)/gamma) U_I^(1)
 * with c/gamma = 3 + 2 sqrt(2) and (1-gamma)/gamma = 1 + sqrt(2). */
static const double OR_GAMMA = 0.29289321881345247560;
static const double OR_E0 = -4.82842712474619009760; /* 1 - c/gamma */
static const double OR_E1 = 5.82842712474619009760;  /* c/gamma */
static const double OR_T0 = -1.41421356237309504880; /* 1 - (1-gamma)/gamma */
static const double OR_T1 = 2.41421356237309504880;  /* (1-gamma)/gamma */

#ifndef OR_COMPLEX
double or_gamma(void) { return OR_GAMMA; }

void or_tableau(double* out) {
  out[0] = OR_GAMMA;
  out[1] = OR_E0;
  out[2] = OR_E1;
  out[3] = OR_T0;
  out[4] = OR_T1;
}

int or_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
#endif

/* Cell index with ghosts: periodic wrap or zero-order copy (transmissive). */
static int gidx(int i, int n, int bc) {
  if (bc == 0) return ((i % n) + n) % n;
  if (i < 0) return 0;
  if (i > n - 1) return n - 1;
  return i;
}

/* ---------------------------------------------------------------------- */
/* Tridiagonal solvers: Thomas, and Sherman-Morrison for the cyclic case.   */
/* ---------------------------------------------------------------------- */
static int thomas(int n, const real_t* lo, const real_t* di, const real_t* up,
                  const real_t* rhs, real_t* x) {
  real_t* cp = (real_t*)malloc(sizeof(real_t) * (size_t)n);
  real_t* dp = (real_t*)malloc(sizeof(real_t) * (size_t)n);
  if (!cp || !dp) { free(cp); free(dp); return OR_EINVAL; }
  cp[0] = up[0] / di[0];
  dp[0] = rhs[0] / di[0];
  for (int i = 1; i < n; ++i) {
    real_t den = di[i] - lo[i] * cp[i - 1];
    cp[i] = up[i] / den;
    dp[i] = (rhs[i] - lo[i] * dp[i - 1]) / den;
  }
  x[n - 1] = dp[n - 1];
  for (int i = n - 2; i >= 0; --i) x[i] = dp[i] - cp[i] * x[i + 1];
  free(cp);
  free(dp);
  return OR_OK;
}

int FN(or_tridiag)(int n, int cyclic, const real_t* lo, const real_t* di,
               const real_t* up, const real_t* rhs, real_t* x) {
  if (n < 1) return OR_EINVAL;
  if (n == 1) {
    real_t d = di[0] + (cyclic ? lo[0] + up[0] : 0.0);
    x[0] = rhs[0] / d;
    return OR_OK;
  }
  if (!cyclic || n == 2) {
    if (!cyclic) return thomas(n, lo, di, up, rhs, x);
    /* n == 2 cyclic: both couplings hit the other unknown. */
    real_t a00 = di[0], a01 = up[0] + lo[0];
    real_t a10 = lo[1] + up[1], a11 = di[1];
    real_t det = a00 * a11 - a01 * a10;
    x[0] = (rhs[0] * a11 - a01 * rhs[1]) / det;
    x[1] = (a00 * rhs[1] - a10 * rhs[0]) / det;
    return OR_OK;
  }
  /* Cyclic: A = B + u v^T with u = (gam, 0..0, up[n-1]),
   * v = (1, 0..0, lo[0]/gam); B has the corners removed and the two
   * diagonal ends corrected. */
  real_t gam = -di[0];
  real_t* dd = (real_t*)malloc(sizeof(real_t) * (size_t)n);
  real_t* u = (real_t*)malloc(sizeof(real_t) * (size_t)n);
  real_t* y = (real_t*)malloc(sizeof(real_t) * (size_t)n);
  real_t* z = (real_t*)malloc(sizeof(real_t) * (size_t)n);
  real_t* l2 = (real_t*)malloc(sizeof(real_t) * (size_t)n);
  real_t* u2 = (real_t*)malloc(sizeof(real_t) * (size_t)n);
  if (!dd || !u || !y || !z || !l2 || !u2) {
    free(dd); free(u); free(y); free(z); free(l2); free(u2);
    return OR_EINVAL;
  }
  for (int i = 0; i < n; ++i) {
    dd[i] = di[i];
    u[i] = 0.0;
    l2[i] = lo[i];
    u2[i] = up[i];
  }
  l2[0] = 0.0;
  u2[n - 1] = 0.0;
  dd[0] = di[0] - gam;
  dd[n - 1] = di[n - 1] - up[n - 1] * lo[0] / gam;
  u[0] = gam;
  u[n - 1] = up[n - 1];
  int rc = thomas(n, l2, dd, u2, rhs, y);
  if (rc == OR_OK) rc = thomas(n, l2, dd, u2, u, z);
  if (rc == OR_OK) {
    real_t vy = y[0] + lo[0] / gam * y[n - 1];
    real_t vz = z[0] + lo[0] / gam * z[n - 1];
    real_t f = vy / (1.0 + vz);
    for (int i = 0; i < n; ++i) x[i] = y[i] - f * z[i];
  }
  free(dd); free(u); free(y); free(z); free(l2); free(u2);
  return rc;
}

/* ---------------------------------------------------------------------- */
/* One semi-implicit stage (Sec. 4.2, eq. GN_hyp_eq_semi_fully_discrete).   */
/* ---------------------------------------------------------------------- */
int FN(or_stage)(int n, const or_params* p, double tau, const real_t* bin,
             const real_t* hE, const real_t* qE, const real_t* mE, const real_t* WE,
             const real_t* ho, const real_t* qo, const real_t* mo, const real_t* Wo,
             real_t* hn, real_t* qn, real_t* mn, real_t* Wn, or_stage_dbg* dbg) {
  if (n < 1 || !p || p->dx <= 0.0) return OR_EINVAL;
  const int bc = p->bc;
  const double g = p->g, lam = p->lambda, dx = p->dx;
  const int useb = p->has_b && bin;
  int rc = OR_OK;

  size_t nc = (size_t)n, nf = (size_t)n + 1;
  real_t* bz = (real_t*)calloc(nc, sizeof(real_t));
  real_t* Fq = (real_t*)malloc(nf * sizeof(real_t));
  real_t* Fm = (real_t*)malloc(nf * sizeof(real_t));
  real_t* FW = (real_t*)malloc(nf * sizeof(real_t));
  real_t* qd = (real_t*)malloc(nc * sizeof(real_t));
  real_t* md = (real_t*)malloc(nc * sizeof(real_t));
  real_t* Wd = (real_t*)malloc(nc * sizeof(real_t));
  real_t* beta = (real_t*)malloc(nc * sizeof(real_t));
  real_t* S = (real_t*)malloc(nc * sizeof(real_t));
  real_t* phi = (real_t*)malloc(nc * sizeof(real_t));
  real_t* T = (real_t*)malloc(nc * sizeof(real_t));
  real_t* P0 = (real_t*)malloc(nc * sizeof(real_t));
  real_t* pt0 = (real_t*)malloc(nc * sizeof(real_t));
  real_t* gL = (real_t*)malloc(nf * sizeof(real_t));
  real_t* gR = (real_t*)malloc(nf * sizeof(real_t));
  real_t* g0 = (real_t*)malloc(nf * sizeof(real_t));
  real_t* qf = (real_t*)malloc(nf * sizeof(real_t));
  real_t* lo = (real_t*)malloc(nc * sizeof(real_t));
  real_t* di = (real_t*)malloc(nc * sizeof(real_t));
  real_t* up = (real_t*)malloc(nc * sizeof(real_t));
  real_t* rhs = (real_t*)malloc(nc * sizeof(real_t));
  real_t* hb = (real_t*)malloc(nc * sizeof(real_t));
  real_t* dl = (real_t*)malloc(nc * sizeof(real_t));
  if (!bz || !Fq || !Fm || !FW || !qd || !md || !Wd || !beta || !S || !phi ||
      !T || !P0 || !pt0 || !gL || !gR || !g0 || !qf || !lo || !di || !up ||
      !rhs || !hb || !dl) {
    rc = OR_EINVAL;
    goto done;
  }
  if (p->form == 1 && useb) { /* the print has no bathymetric SI scheme */
    rc = OR_EINVAL;
    goto done;
  }
  const real_t* b = useb ? bin : bz;

  /* (1) Explicit Rusanov fluxes of q u, m u, W u at every face, from the
   * unlimited component-wise linear reconstruction of U_E (Sec. 4.1:
   * slope (v_{i+1} - v_{i-1})/(2 dx), face values v_i +- slope dx/2); the
   * first-order scheme uses the cell values (sl = 0). */
  const double sl = p->order == 1 ? 0.0 : 0.25;
  for (int k = 0; k <= n; ++k) {
    int im1 = gidx(k - 2, n, bc), i0 = gidx(k - 1, n, bc);
    int i1 = gidx(k, n, bc), i2 = gidx(k + 1, n, bc);
    /* left state: cell k-1 at its right face; right state: cell k at its
     * left face. */
    real_t hL = hE[i0] + sl * (hE[i1] - hE[im1]);
    real_t hR = hE[i1] - sl * (hE[i2] - hE[i0]);
    real_t qL = qE[i0] + sl * (qE[i1] - qE[im1]);
    real_t qR = qE[i1] - sl * (qE[i2] - qE[i0]);
    real_t mL = mE[i0] + sl * (mE[i1] - mE[im1]);
    real_t mR = mE[i1] - sl * (mE[i2] - mE[i0]);
    real_t WL = WE[i0] + sl * (WE[i1] - WE[im1]);
    real_t WR = WE[i1] - sl * (WE[i2] - WE[i0]);
    if (!(RE(hL) > 0.0) || !(RE(hR) > 0.0)) rc = OR_ENONPHYS;
    real_t uL = qL / hL, uR = qR / hR;
    real_t sL = RABS(uL) + RSQRT(g * hL), sR = RABS(uR) + RSQRT(g * hR);
    real_t a = RMAX(sL, sR);
    /* Face-local lake-at-rest moment: mhat_j = (zeta_f - b_j)^2 with
     * zeta_f the mean free surface of the two face cells, reconstructed
     * like m; identically zero jump on a flat bed. */
    real_t zf = 0.5 * ((hE[i0] + b[i0]) + (hE[i1] + b[i1]));
    real_t r_m1 = (zf - b[im1]) * (zf - b[im1]);
    real_t r_0 = (zf - b[i0]) * (zf - b[i0]);
    real_t r_1 = (zf - b[i1]) * (zf - b[i1]);
    real_t r_2 = (zf - b[i2]) * (zf - b[i2]);
    real_t mhL = r_0 + sl * (r_1 - r_m1);
    real_t mhR = r_1 - sl * (r_2 - r_0);
    Fq[k] = 0.5 * (qL * uL + qR * uR - a * (qR - qL));
    FW[k] = 0.5 * (WL * uL + WR * uR - a * (WR - WL));
    Fm[k] = 0.5 * (mL * uL + mR * uR - a * ((mR - mL) - (mhR - mhL)));
  }

  /* (2) Convective predictor with the exact relaxation elimination
   * (Sec. 3.1 eq. hSGN_eq-ustar and eq. b1; Sec. 4.2 first three lines). */
  for (int i = 0; i < n; ++i) {
    real_t dbc = (b[gidx(i + 1, n, bc)] - b[gidx(i - 1, n, bc)]) / (2.0 * dx);
    Wd[i] = Wo[i] - tau / dx * (FW[i + 1] - FW[i]) + lam * tau;
    md[i] = mo[i] - tau / dx * (Fm[i + 1] - Fm[i]) - tau * 1.5 * qE[i] * dbc +
            tau * Wd[i];
    qd[i] = qo[i] - tau / dx * (Fq[i + 1] - Fq[i]);
  }

  /* (3) Frozen coefficients at U_E (Sec. 2.2 eq. hSGN_alpha, hSGN_px;
   * Sec. 4.2 beta_1, beta_2, beta).  P0 is the pressure p(h, m) of
   * eq. hSGN_p at h = h_E and m = m-dagger / beta_1 (eq. b1 at h = h_E);
   * phi is d p~/d h of p~ = (lambda/3)(1 - eta/h) along the same
   * relaxation closure (bed form, eq. hSGNb_eq). */
  for (int i = 0; i < n; ++i) {
    real_t h = hE[i];
    if (!(RE(h) > 0.0)) rc = OR_ENONPHYS;
    real_t eta = mE[i] / h;
    real_t alpha = -(2.0 * eta / h - 1.0) / (3.0 * h);
    real_t c2 = g * h + lam / 3.0 * eta * eta / (h * h);
    real_t a2 = c2 - lam * eta * alpha;
    real_t beta1 = 1.0 + lam * tau * tau / (h * h);
    real_t beta2 = 2.0 * lam * tau * tau / (beta1 * beta1 * h * h * h);
    beta[i] = a2 + lam * alpha * beta2 * md[i];
    if (!(RE(beta[i]) > 0.0)) rc = rc ? rc : OR_ENONCOERCIVE;
    real_t eta0 = md[i] / (beta1 * h);
    pt0[i] = lam / 3.0 * (1.0 - eta0 / h);
    P0[i] = 0.5 * g * h * h + eta0 * pt0[i];
    S[i] = P0[i] - beta[i] * h;
    real_t den = h * h + lam * tau * tau;
    phi[i] = 2.0 * lam / 3.0 * md[i] * h / (den * den);
    T[i] = pt0[i] - phi[i] * h;
    dl[i] = alpha / beta1; /* delta of Sec. 4.2 (mode A only) */
  }

  if (p->form == 1) {
    /* Mode A: the remaining printed lines of Sec. 4.2 (eq.
     * GN_hyp_eq_semi_fully_discrete), flat bottom.  Face values are means of
     * the two cells; the delta Laplacian of h*eta-dagger carries the weight
     * lambda tau^2 / dx^2 on those means (with the printed 1/2 the implicit
     * coefficients at rest would not add up to g h).  Ghost cells as for the
     * fluxes: periodic wrap, or copies of the boundary cell (transmissive),
     * which folds the outer coupling of a boundary row into its diagonal. */
    const real_t r = tau * tau / (dx * dx);
    for (int i = 0; i < n; ++i) {
      int im = gidx(i - 1, n, bc), ip = gidx(i + 1, n, bc);
      real_t bp = 0.5 * (beta[i] + beta[ip]), bm = 0.5 * (beta[i] + beta[im]);
      real_t dp = 0.5 * (dl[i] + dl[ip]), dm = 0.5 * (dl[i] + dl[im]);
      /* Delta[h]_i = h_i (1 + r (beta_{i+1/2} + beta_{i-1/2}))
       *              - r beta_{i+1/2} h_{i+1} - r beta_{i-1/2} h_{i-1} */
      lo[i] = -r * bm;
      up[i] = -r * bp;
      di[i] = 1.0 + r * (bp + bm);
      /* h-dagger */
      rhs[i] = ho[i] - tau / (2.0 * dx) * (qd[ip] - qd[im]) +
               lam * r * (dp * (md[ip] - md[i]) - dm * (md[i] - md[im]));
      if (bc != 0 && i == 0) { di[i] += lo[i]; lo[i] = 0.0; }
      if (bc != 0 && i == n - 1) { di[i] += up[i]; up[i] = 0.0; }
    }
    {
      int trc = FN(or_tridiag)(n, bc == 0, lo, di, up, rhs, hb);
      if (trc) rc = trc;
    }
    /* momentum as printed, then the relaxation pair as in the P-form */
    for (int i = 0; i < n; ++i) {
      int im = gidx(i - 1, n, bc), ip = gidx(i + 1, n, bc);
      real_t hbi = hb[i];
      if (!(RE(hbi) > 0.0)) rc = OR_ENONPHYS;
      qn[i] = qd[i] - tau / (2.0 * dx) * beta[i] * (hb[ip] - hb[im]) -
              lam * tau / (2.0 * dx) * dl[i] * (md[ip] - md[im]);
      mn[i] = md[i] / (1.0 + lam * tau * tau / (hbi * hbi));
      Wn[i] = Wd[i] - lam * tau * mn[i] / (hbi * hbi);
      hn[i] = hbi;
      if (!isfinite(RE(qn[i])) || !isfinite(RE(mn[i])) || !isfinite(RE(Wn[i])) ||
          !isfinite(RE(hn[i])))
        rc = OR_ENONPHYS;
    }
    goto debug_out;
  }

  /* (4) Implicit face force G = [P_R - P_L + (g/2)(hb_L + hb_R) db
   * + (3/4)(p~_L + p~_R) db] / dx, affine in hbar:
   * G = gL hbar_L + gR hbar_R + g0, and face momentum
   * Q = (q-dagger_L + q-dagger_R)/2 - tau G (Sec. 3.1 eq. hSGN_eq-split-I).
   * Transmissive boundary faces carry no implicit force and Q = q-dagger of
   * the boundary cell. */
  for (int k = 0; k <= n; ++k) {
    int L = gidx(k - 1, n, bc), R = gidx(k, n, bc);
    int boundary = (bc != 0) && (k == 0 || k == n);
    if (boundary) {
      gL[k] = gR[k] = g0[k] = 0.0;
      qf[k] = qd[k == 0 ? 0 : n - 1];
      continue;
    }
    real_t db = b[R] - b[L];
    gL[k] = (-beta[L] + db * (0.5 * g + 0.75 * phi[L])) / dx;
    gR[k] = (beta[R] + db * (0.5 * g + 0.75 * phi[R])) / dx;
    g0[k] = (S[R] - S[L] + 0.75 * db * (T[L] + T[R])) / dx;
    qf[k] = 0.5 * (qd[L] + qd[R]);
  }

  /* (5) Mass balance hbar_i = h_old,i - tau/dx (Q_{i+1/2} - Q_{i-1/2}),
   * collected as rows of the tridiagonal (cyclic if periodic) system. */
  for (int i = 0; i < n; ++i) {
    real_t c = tau * tau / dx;
    up[i] = -c * gR[i + 1];
    lo[i] = c * gL[i];
    di[i] = 1.0 - c * (gL[i + 1] - gR[i]);
    rhs[i] = ho[i] - tau / dx * (qf[i + 1] - qf[i]) + c * (g0[i + 1] - g0[i]);
  }
  {
    int trc = FN(or_tridiag)(n, bc == 0, lo, di, up, rhs, hb);
    if (trc) rc = trc;
  }

  /* (6) Back-substitution (Sec. 4.2 last three lines): momentum from the
   * linearised pressure and bed force, then the relaxation pair with hbar
   * treated implicitly: m = m-dagger / (1 + lambda tau^2 / hbar^2),
   * W = W-dagger - lambda tau m / hbar^2. */
  for (int i = 0; i < n; ++i) {
    int im = gidx(i - 1, n, bc), ip = gidx(i + 1, n, bc);
    real_t Pm = P0[im] + beta[im] * (hb[im] - hE[im]);
    real_t Pp = P0[ip] + beta[ip] * (hb[ip] - hE[ip]);
    real_t pti = pt0[i] + phi[i] * (hb[i] - hE[i]);
    real_t dbc = (b[ip] - b[im]) / (2.0 * dx);
    real_t hbi = hb[i];
    if (!(RE(hbi) > 0.0)) rc = OR_ENONPHYS;
    qn[i] = qd[i] - tau * ((Pp - Pm) / (2.0 * dx) +
                           0.5 * g * (hb[ip] + hb[im]) * dbc + 1.5 * pti * dbc);
    mn[i] = md[i] / (1.0 + lam * tau * tau / (hbi * hbi));
    Wn[i] = Wd[i] - lam * tau * mn[i] / (hbi * hbi);
    hn[i] = hbi;
    if (!isfinite(RE(qn[i])) || !isfinite(RE(mn[i])) || !isfinite(RE(Wn[i])) ||
        !isfinite(RE(hn[i])))
      rc = OR_ENONPHYS;
  }

debug_out:
#ifndef OR_COMPLEX
  if (dbg) {
#define OR_CP(dst, src, cnt) \
  if (dbg->dst) memcpy(dbg->dst, src, (cnt) * sizeof(double))
    OR_CP(qd, qd, nc); OR_CP(md, md, nc); OR_CP(Wd, Wd, nc);
    OR_CP(beta, beta, nc); OR_CP(S, S, nc); OR_CP(phi, phi, nc);
    OR_CP(T, T, nc); OR_CP(P0, P0, nc); OR_CP(pt0, pt0, nc);
    OR_CP(lo, lo, nc); OR_CP(di, di, nc); OR_CP(up, up, nc);
    OR_CP(rhs, rhs, nc); OR_CP(hbar, hb, nc);
    OR_CP(Fq, Fq, nf); OR_CP(Fm, Fm, nf); OR_CP(FW, FW, nf);
#undef OR_CP
  }
#else
  (void)dbg;
#endif

done:
  free(bz); free(Fq); free(Fm); free(FW); free(qd); free(md); free(Wd);
  free(beta); free(S); free(phi); free(T); free(P0); free(pt0);
  free(gL); free(gR); free(g0); free(qf); free(lo); free(di); free(up);
  free(rhs); free(hb); free(dl);
  return rc;
}

/* ---------------------------------------------------------------------- */
/* Explicit hSGN space operator (Sec. 4.1, eq. GN_hyp_eq_explicit), flat    */
/* bottom, U = (h, q, m = h eta, W = h w):                                  */
/*   L_h = -Dhat_x(q)      (Rusanov; the print has the central D_x(q))      */
/*   L_q = -Dhat_x(q u) - a^2 D_x(h) - lambda alpha D_x(m)                  */
/*   L_m = -Dhat_x(m u) + W                                                 */
/*   L_W = -Dhat_x(W u) - lambda (m / h^2 - 1)                              */
/* D_x: central difference (mean of the cell fluxes at the faces); Dhat_x:  */
/* Rusanov flux difference on the unlimited linear reconstruction of U,     */
/* speed max(|u| + c) over the face states, c^2 = g h + (lambda/3)(m/h^2)^2.*/
/* a^2 = dp/dh and lambda alpha = dp/d(h eta) of the pressure (eq. hSGN_p): */
/* a^2 = g h + lambda (eta/h)^2 - (lambda/3) eta/h, alpha = -(2 eta/h - 1)/(3 h). */
/* ---------------------------------------------------------------------- */
static int FN(or_ex_rhs)(int n, const or_params* p, const real_t* h, const real_t* q,
                         const real_t* m, const real_t* W, real_t* Lh, real_t* Lq,
                         real_t* Lm, real_t* LW) {
  const double g = p->g, lam = p->lambda, dx = p->dx;
  const int bc = p->bc;
  size_t nf = (size_t)n + 1;
  real_t* Fq = (real_t*)malloc(nf * sizeof(real_t));
  real_t* Fm = (real_t*)malloc(nf * sizeof(real_t));
  real_t* FW = (real_t*)malloc(nf * sizeof(real_t));
  real_t* Fh = (real_t*)malloc(nf * sizeof(real_t)); /* mass flux */
  int rc = OR_OK;
  if (!Fq || !Fm || !FW || !Fh) { rc = OR_EINVAL; goto done; }
  /* face k lies between cells k-1 and k */
  for (int k = 0; k <= n; ++k) {
    int a = gidx(k - 2, n, bc), b0 = gidx(k - 1, n, bc), b1 = gidx(k, n, bc), c = gidx(k + 1, n, bc);
    real_t hL = h[b0] + 0.25 * (h[b1] - h[a]), hR = h[b1] - 0.25 * (h[c] - h[b0]);
    real_t qL = q[b0] + 0.25 * (q[b1] - q[a]), qR = q[b1] - 0.25 * (q[c] - q[b0]);
    real_t mL = m[b0] + 0.25 * (m[b1] - m[a]), mR = m[b1] - 0.25 * (m[c] - m[b0]);
    real_t WL = W[b0] + 0.25 * (W[b1] - W[a]), WR = W[b1] - 0.25 * (W[c] - W[b0]);
    if (!(RE(hL) > 0.0) || !(RE(hR) > 0.0)) { rc = OR_ENONPHYS; goto done; }
    real_t uL = qL / hL, uR = qR / hR;
    real_t eL = mL / (hL * hL), eR = mR / (hR * hR); /* eta/h */
    real_t cL = RSQRT(g * hL + (lam / 3.0) * eL * eL);
    real_t cR = RSQRT(g * hR + (lam / 3.0) * eR * eR);
    real_t sL = RABS(uL) + cL, sR = RABS(uR) + cR;
    real_t al = RMAX(sL, sR);
    Fh[k] = 0.5 * (qL + qR - al * (hR - hL));
    Fq[k] = 0.5 * (qL * uL + qR * uR - al * (qR - qL));
    Fm[k] = 0.5 * (mL * uL + mR * uR - al * (mR - mL));
    FW[k] = 0.5 * (WL * uL + WR * uR - al * (WR - WL));
  }
  for (int i = 0; i < n; ++i) {
    int im = gidx(i - 1, n, bc), ip = gidx(i + 1, n, bc);
    if (!(RE(h[i]) > 0.0)) { rc = OR_ENONPHYS; goto done; }
    real_t eh = m[i] / (h[i] * h[i]);
    real_t a2 = g * h[i] + lam * eh * eh - (lam / 3.0) * eh;
    real_t alpha = -(2.0 * eh - 1.0) / (3.0 * h[i]);
    real_t dh = (h[ip] - h[im]) / (2.0 * dx);
    real_t dm = (m[ip] - m[im]) / (2.0 * dx);
    Lh[i] = -(Fh[i + 1] - Fh[i]) / dx;
    Lq[i] = -(Fq[i + 1] - Fq[i]) / dx - a2 * dh - lam * alpha * dm;
    Lm[i] = -(Fm[i + 1] - Fm[i]) / dx + W[i];
    LW[i] = -(FW[i + 1] - FW[i]) / dx - lam * (eh - 1.0);
  }
done:
  free(Fq); free(Fm); free(FW); free(Fh);
  return rc;
}

/* Time step of the explicit scheme (Sec. 5: dt = CFL dx / max mu, with mu =
 * |u| + c the spectral radius of the hSGN system, eq. CFL_ex), then the
 * same material cap and t_end clamp as the semi-implicit step. */
double FN(or_dt_ex)(int n, const or_params* p, const real_t* h, const real_t* q,
                    const real_t* m, double t) {
  double dt;
  if (p->dt_fixed > 0.0) {
    dt = p->dt_fixed;
  } else {
    double smax = 0.0, umax = 0.0;
    for (int i = 0; i < n; ++i) {
      double hh = RE(h[i]);
      double u = fabs(RE(q[i]) / hh);
      double e = RE(m[i]) / (hh * hh);
      double s = u + sqrt(p->g * hh + (p->lambda / 3.0) * e * e);
      if (s > smax) smax = s;
      if (u > umax) umax = u;
    }
    dt = p->cfl * p->dx / smax;
    if (p->mcfl > 0.0 && umax * dt / p->dx > p->mcfl) dt = p->mcfl * p->dx / umax;
  }
  if (p->t_end > 0.0) {
    if (t >= p->t_end) dt = 0.0;
    else if (t + dt > p->t_end) dt = p->t_end - t;
  }
  return dt;
}

/* One explicit step with Heun's method (second order, Sec. 4.1):
 * U1 = U^n + dt L(U^n);  U^{n+1} = (U^n + U1 + dt L(U1)) / 2. */
static int FN(or_ex_step)(int n, const or_params* p, real_t* h, real_t* q, real_t* m,
                          real_t* W, double dt) {
  size_t nc = (size_t)n;
  real_t* buf = (real_t*)malloc(8 * nc * sizeof(real_t));
  if (!buf) return OR_EINVAL;
  real_t *Lh = buf, *Lq = buf + nc, *Lm = buf + 2 * nc, *LW = buf + 3 * nc;
  real_t *h1 = buf + 4 * nc, *q1 = buf + 5 * nc, *m1 = buf + 6 * nc, *W1 = buf + 7 * nc;
  int rc = FN(or_ex_rhs)(n, p, h, q, m, W, Lh, Lq, Lm, LW);
  if (rc == OR_OK) {
    for (size_t i = 0; i < nc; ++i) {
      h1[i] = h[i] + dt * Lh[i];
      q1[i] = q[i] + dt * Lq[i];
      m1[i] = m[i] + dt * Lm[i];
      W1[i] = W[i] + dt * LW[i];
    }
    rc = FN(or_ex_rhs)(n, p, h1, q1, m1, W1, Lh, Lq, Lm, LW);
  }
  if (rc == OR_OK) {
    for (size_t i = 0; i < nc; ++i) {
      h[i] = 0.5 * (h[i] + (h1[i] + dt * Lh[i]));
      q[i] = 0.5 * (q[i] + (q1[i] + dt * Lq[i]));
      m[i] = 0.5 * (m[i] + (m1[i] + dt * Lm[i]));
      W[i] = 0.5 * (W[i] + (W1[i] + dt * LW[i]));
    }
  }
  free(buf);
  return rc;
}

/* ---------------------------------------------------------------------- */
/* Standard SGN (Sec. 4.3-4.4), flat bottom, state (h, q = h u):            */
/*   h_t + q_x = 0,  q_t + (q u + g h^2/2)_x = h phi,                       */
/*   h phi - (h^3/3 phi_x)_x = -(h^3/3 g h_xx + 2 h^3/3 u_x^2)_x            */
/* discretised as                                                           */
/*   h_i phi_i - (H_{i+1/2}(phi_{i+1} - phi_i) - H_{i-1/2}(phi_i - phi_{i-1})) */
/*        / (3 dx^2) = h*_i,   H_{i+1/2} = (h_i^3 + h_{i+1}^3) / 2,          */
/*   h*_i = -(G_{i+1} - G_{i-1}) / (6 dx^3),                                */
/*   G_j = g h_j^3 (h_{j+1} - 2 h_j + h_{j-1}) + (h_j^3 / 2)(u_{j+1} - u_{j-1})^2, */
/* and L_h = -Dhat_x(q), L_q = -Dhat_x(q u + g h^2/2) + h phi with Rusanov  */
/* fluxes on the unlimited linear reconstruction of (h, q).                 */
/* ---------------------------------------------------------------------- */
static int FN(or_sgn_rhs)(int n, const or_params* p, const real_t* h, const real_t* q,
                          real_t* Lh, real_t* Lq, real_t* phi_out) {
  const double g = p->g, dx = p->dx;
  const int bc = p->bc;
  size_t nc = (size_t)n, nf = (size_t)n + 1;
  real_t* Fh = (real_t*)malloc(nf * sizeof(real_t));
  real_t* Fq = (real_t*)malloc(nf * sizeof(real_t));
  real_t* G = (real_t*)malloc((nc + 2) * sizeof(real_t)); /* G[j + 1], j = -1 .. n */
  real_t* lo = (real_t*)calloc(nc, sizeof(real_t));
  real_t* di = (real_t*)calloc(nc, sizeof(real_t));
  real_t* up = (real_t*)calloc(nc, sizeof(real_t));
  real_t* rhs = (real_t*)calloc(nc, sizeof(real_t));
  real_t* phi = (real_t*)calloc(nc, sizeof(real_t));
  int rc = OR_OK;
  if (!Fh || !Fq || !G || !lo || !di || !up || !rhs || !phi) { rc = OR_EINVAL; goto done; }
  for (int i = 0; i < n; ++i)
    if (!(RE(h[i]) > 0.0)) { rc = OR_ENONPHYS; goto done; }
  /* shallow-water Rusanov fluxes, face k between cells k-1 and k */
  for (int k = 0; k <= n; ++k) {
    int a = gidx(k - 2, n, bc), b0 = gidx(k - 1, n, bc), b1 = gidx(k, n, bc), c = gidx(k + 1, n, bc);
    real_t hL = h[b0] + 0.25 * (h[b1] - h[a]), hR = h[b1] - 0.25 * (h[c] - h[b0]);
    real_t qL = q[b0] + 0.25 * (q[b1] - q[a]), qR = q[b1] - 0.25 * (q[c] - q[b0]);
    if (!(RE(hL) > 0.0) || !(RE(hR) > 0.0)) { rc = OR_ENONPHYS; goto done; }
    real_t uL = qL / hL, uR = qR / hR;
    real_t sL = RABS(uL) + RSQRT(g * hL), sR = RABS(uR) + RSQRT(g * hR);
    real_t al = RMAX(sL, sR);
    Fh[k] = 0.5 * (qL + qR - al * (hR - hL));
    Fq[k] = 0.5 * (qL * uL + 0.5 * g * hL * hL + qR * uR + 0.5 * g * hR * hR - al * (qR - qL));
  }
  /* G_j at every cell and at the first ghost on each side (ghost states are
   * the copies or wrapped cells that every stencil reads) */
  for (int j = -1; j <= n; ++j) {
    int jc = gidx(j, n, bc), jm = gidx(j - 1, n, bc), jp = gidx(j + 1, n, bc);
    real_t h3 = h[jc] * h[jc] * h[jc];
    real_t du = q[jp] / h[jp] - q[jm] / h[jm];
    G[j + 1] = g * h3 * (h[jp] - 2.0 * h[jc] + h[jm]) + 0.5 * h3 * du * du;
  }
  /* rows of the phi system */
  for (int i = 0; i < n; ++i) {
    int im = gidx(i - 1, n, bc), ip = gidx(i + 1, n, bc);
    real_t Hm = 0.5 * (h[im] * h[im] * h[im] + h[i] * h[i] * h[i]);
    real_t Hp = 0.5 * (h[i] * h[i] * h[i] + h[ip] * h[ip] * h[ip]);
    real_t c3 = 1.0 / (3.0 * dx * dx);
    lo[i] = -c3 * Hm;
    up[i] = -c3 * Hp;
    di[i] = h[i] + c3 * (Hm + Hp);
    rhs[i] = -(G[i + 2] - G[i]) / (6.0 * dx * dx * dx); /* G_{i+1} - G_{i-1} */
    if (bc != 0) { /* zero-gradient phi at a transmissive end */
      if (i == 0) { di[i] += lo[i]; lo[i] = 0.0; }
      if (i == n - 1) { di[i] += up[i]; up[i] = 0.0; }
    }
  }
  rc = FN(or_tridiag)(n, bc == 0, lo, di, up, rhs, phi);
  if (rc != OR_OK) goto done;
  for (int i = 0; i < n; ++i) {
    Lh[i] = -(Fh[i + 1] - Fh[i]) / dx;
    Lq[i] = -(Fq[i + 1] - Fq[i]) / dx + h[i] * phi[i];
    if (phi_out) phi_out[i] = phi[i];
  }
done:
  free(Fh); free(Fq); free(G); free(lo); free(di); free(up); free(rhs); free(phi);
  return rc;
}

/* One SGN step with Heun's method (Sec. 4.4), m and W untouched. */
static int FN(or_sgn_step)(int n, const or_params* p, real_t* h, real_t* q, double dt) {
  size_t nc = (size_t)n;
  real_t* buf = (real_t*)malloc(4 * nc * sizeof(real_t));
  if (!buf) return OR_EINVAL;
  real_t *Lh = buf, *Lq = buf + nc, *h1 = buf + 2 * nc, *q1 = buf + 3 * nc;
  int rc = FN(or_sgn_rhs)(n, p, h, q, Lh, Lq, NULL);
  if (rc == OR_OK) {
    for (size_t i = 0; i < nc; ++i) {
      h1[i] = h[i] + dt * Lh[i];
      q1[i] = q[i] + dt * Lq[i];
    }
    rc = FN(or_sgn_rhs)(n, p, h1, q1, Lh, Lq, NULL);
  }
  if (rc == OR_OK) {
    for (size_t i = 0; i < nc; ++i) {
      h[i] = 0.5 * (h[i] + (h1[i] + dt * Lh[i]));
      q[i] = 0.5 * (q[i] + (q1[i] + dt * Lq[i]));
    }
  }
  free(buf);
  return rc;
}

#ifndef OR_COMPLEX
/* phi of the SGN elliptic problem for a state (for the pins). */
int or_sgn_phi(int n, const or_params* p, const double* h, const double* q, double* phi) {
  size_t nc = (size_t)n;
  double* tmp = (double*)malloc(2 * nc * sizeof(double));
  if (!tmp) return OR_EINVAL;
  int rc = or_sgn_rhs(n, p, h, q, tmp, tmp + nc, phi);
  free(tmp);
  return rc;
}
#endif

/* ---------------------------------------------------------------------- */
/* Time step (Sec. 5: dt = CFL dx / max speed, then the material CFL cap).  */
/* The speed is |u| + sqrt(g h): the lambda-independent rule of the remark  */
/* after the coercivity proposition (Sec. 3.1).                             */
/* ---------------------------------------------------------------------- */
double FN(or_dt)(int n, const or_params* p, const real_t* h, const real_t* q, double t) {
  double dt;
  if (p->dt_fixed > 0.0) {
    dt = p->dt_fixed;
  } else {
    double smax = 0.0, umax = 0.0;
    for (int i = 0; i < n; ++i) {
      double u = fabs(RE(q[i]) / RE(h[i]));
      double s = u + sqrt(p->g * RE(h[i]));
      if (s > smax) smax = s;
      if (u > umax) umax = u;
    }
    dt = p->cfl * p->dx / smax;
    if (p->mcfl > 0.0 && umax * dt / p->dx > p->mcfl) dt = p->mcfl * p->dx / umax;
  }
  if (p->t_end > 0.0) {
    if (t >= p->t_end) dt = 0.0;
    else if (t + dt > p->t_end) dt = p->t_end - t;
  }
  return dt;
}

/* ---------------------------------------------------------------------- */
/* Two-stage IMEX step (Sec. 3.2, eq. tableau, steps 1-5 + efficient form). */
/* ---------------------------------------------------------------------- */
int FN(or_step)(int n, const or_params* p, const real_t* b,
            real_t* h, real_t* q, real_t* m, real_t* W, double* t, double* dt_out) {
  if (p->scheme == 2) {
    if (p->has_b) return OR_EINVAL; /* flat bottom only */
    double dts = FN(or_dt)(n, p, h, q, *t); /* same rule as the semi-implicit step */
    if (dt_out) *dt_out = dts;
    if (!(dts > 0.0)) return OR_OK;
    int rcs = FN(or_sgn_step)(n, p, h, q, dts);
    *t += dts;
    return rcs;
  }
  if (p->scheme == 1) {
    if (p->has_b) return OR_EINVAL; /* the explicit scheme is for a flat bottom */
    double dte = FN(or_dt_ex)(n, p, h, q, m, *t);
    if (dt_out) *dt_out = dte;
    if (!(dte > 0.0)) return OR_OK;
    int rce = FN(or_ex_step)(n, p, h, q, m, W, dte);
    *t += dte;
    return rce;
  }
  double dt = FN(or_dt)(n, p, h, q, *t);
  if (dt_out) *dt_out = dt;
  if (!(dt > 0.0)) return OR_OK; /* frozen instance */
  if (p->order == 1) {
    /* first-order scheme (Sec. 4.2 as printed): one stage with tau = dt,
     * explicit terms and old values both from U^n */
    size_t n1 = (size_t)n;
    real_t* o = (real_t*)malloc(4 * n1 * sizeof(real_t));
    if (!o) return OR_EINVAL;
    int rc1 = FN(or_stage)(n, p, dt, b, h, q, m, W, h, q, m, W, o, o + n1, o + 2 * n1,
                           o + 3 * n1, NULL);
    memcpy(h, o, n1 * sizeof(real_t));
    memcpy(q, o + n1, n1 * sizeof(real_t));
    memcpy(m, o + 2 * n1, n1 * sizeof(real_t));
    memcpy(W, o + 3 * n1, n1 * sizeof(real_t));
    free(o);
    *t += dt;
    return rc1;
  }
  double tau = OR_GAMMA * dt;
  size_t nc = (size_t)n;
  real_t* buf = (real_t*)malloc(12 * nc * sizeof(real_t));
  if (!buf) return OR_EINVAL;
  real_t *h1 = buf, *q1 = buf + nc, *m1 = buf + 2 * nc, *W1 = buf + 3 * nc;
  real_t *hE = buf + 4 * nc, *qE = buf + 5 * nc, *mE = buf + 6 * nc, *WE = buf + 7 * nc;
  real_t *ht = buf + 8 * nc, *qt = buf + 9 * nc, *mt = buf + 10 * nc, *Wt = buf + 11 * nc;

  /* stage 1: U_E^(1) = U^n, U_I^(1) = U^n + gamma dt H(U_E^(1), U_I^(1)) */
  int rc = FN(or_stage)(n, p, tau, b, h, q, m, W, h, q, m, W, h1, q1, m1, W1, NULL);
  int rc2 = OR_OK;
  if (rc == OR_OK) {
    /* efficient-form combinations */
    for (size_t i = 0; i < nc; ++i) {
      hE[i] = OR_E0 * h[i] + OR_E1 * h1[i];
      qE[i] = OR_E0 * q[i] + OR_E1 * q1[i];
      mE[i] = OR_E0 * m[i] + OR_E1 * m1[i];
      WE[i] = OR_E0 * W[i] + OR_E1 * W1[i];
      ht[i] = OR_T0 * h[i] + OR_T1 * h1[i];
      qt[i] = OR_T0 * q[i] + OR_T1 * q1[i];
      mt[i] = OR_T0 * m[i] + OR_T1 * m1[i];
      Wt[i] = OR_T0 * W[i] + OR_T1 * W1[i];
    }
    /* stage 2: U^{n+1} = U_I^(2) = U~ + gamma dt H(U_E^(2), U_I^(2))
     * (stiffly accurate: the last implicit stage is the new state) */
    rc2 = FN(or_stage)(n, p, tau, b, hE, qE, mE, WE, ht, qt, mt, Wt, h, q, m, W, NULL);
  }
  free(buf);
  *t += dt;
  return rc ? rc : rc2;
}

int FN(or_run)(int n, const or_params* p, const real_t* b,
           real_t* h, real_t* q, real_t* m, real_t* W, double* t, int nsteps) {
  for (int s = 0; s < nsteps; ++s) {
    int rc = FN(or_step)(n, p, b, h, q, m, W, t, NULL);
    if (rc) return rc;
  }
  return OR_OK;
}

/* Gauge misfit: nsteps steps from the given state; after step s the loss
 * gains (1/2) sum_g (h[gauge[g]] - target[s*ng + g])^2. */
int FN(or_run_loss)(int n, const or_params* p, const real_t* b, real_t* h, real_t* q,
                    real_t* m, real_t* W, int nsteps, int ng, const int* gauge,
                    const double* target, real_t* loss) {
  double t = 0.0;
  real_t J = 0.0;
  for (int s = 0; s < nsteps; ++s) {
    int rc = FN(or_step)(n, p, b, h, q, m, W, &t, NULL);
    if (rc) return rc;
    for (int g = 0; g < ng; ++g) {
      real_t d = h[gauge[g]] - target[(size_t)s * ng + g];
      J += 0.5 * d * d;
    }
  }
  *loss = J;
  return OR_OK;
}

#ifndef OR_COMPLEX
int or_run_gauges(int n, const or_params* p, const double* b, double* h, double* q, double* m,
                  double* W, int nsteps, int ng, const int* gauge, double* series) {
  double t = 0.0;
  for (int s = 0; s < nsteps; ++s) {
    int rc = or_step(n, p, b, h, q, m, W, &t, NULL);
    if (rc) return rc;
    for (int g = 0; g < ng; ++g) series[(size_t)s * ng + g] = h[gauge[g]];
  }
  return OR_OK;
}

int or_run_batch(int n_inst, const long long* offsets, const or_params* p,
                 const double* b, double* h, double* q, double* m, double* W,
                 double* t, int nsteps, int nthreads, int* status) {
  int worst = OR_OK;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1) reduction(max : worst)
#endif
  for (int j = 0; j < n_inst; ++j) {
    long long o = offsets[j];
    int n = (int)(offsets[j + 1] - o);
    int rc = or_run(n, &p[j], b ? b + o : NULL, h + o, q + o, m + o, W + o,
                    &t[j], nsteps);
    if (status) status[j] = rc;
    if (rc > worst) worst = rc;
  }
  (void)nthreads;
  return worst;
}
#endif
