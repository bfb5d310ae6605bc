// hsgn_adjoint.hpp -- hand-written discrete adjoint of one semi-implicit stage.
//
// The stage maps (U_old, U_E; b) to U_new (Sec. 4.2, eq.
// GN_hyp_eq_semi_fully_discrete, with the readings of the forward kernels).
// Its reverse takes the adjoint of U_new and returns the adjoints of U_old,
// U_E and b.  One workgroup owns one instance and runs, separated by
// barriers:
//   forward recompute: face fluxes -> cell records -> rows -> solve (hbar)
//   reverse: back-substitution -> transposed tridiagonal solve A^T lam = hbar^a
//            -> rows -> records -> face fluxes -> cells.
// Every phase is a per-cell or per-face function of global scratch arrays;
// contributions to neighbours are written per source and gathered per
// target (no floating-point atomics: the result does not depend on timing).
// Boundary conditions follow the forward: periodic wrap, or transmissive
// ghost copies with the boundary rows folded.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "hsgn_kernels.hpp"

namespace hsgn {
namespace adj {

// scratch arrays (per cell unless marked face)
enum {
  HE, QE, ME, WE, HO, QO, MO, WO, BB,                 // stage inputs (+ bed)
  QD, MD, WD, BETA, SS, PHI, TT,                      // records
  LO, DI, UP, RHS, HB,                                // rows (folded) and hbar
  AH, AQ, AM, AW,                                     // adjoint of U_new
  WDA, MDA, QDA0, TA0, PHIA0, HBA0, FA, DBA,          // reverse back-substitution
  SA0, BETAA0, HBA, BAB,                              // ... gathered
  LOT, DIT, UPT, LAM, SCP, SY, SV, SW,                // transposed solve
  RLB, RLS, RLQ, RLP, RLT,                            // row parts to the left cell
  RRB, RRS, RRQ, RRP, RRT,                            // row parts to the right cell
  RCB, RCS, RCQ, RCP, RCT, HOA, DBMA, DBPA,           // row parts to the own cell
  BETAT, STT, QDT, PHIT, TTT, BAR,                    // record adjoints (totals)
  OAH, OAQ, OAM, OAW, EAH0, EAM0, EAQ0,               // reverse records
  FLQ, FLM, FLW, FRQ, FRM, FRW, DB2A,
  EAH, EAQ, EAM, EAW, BAS,                            // adjoint of U_E, b (stage)
  NCELL_ARR
};
enum {  // face arrays
  FQ, FM, FW, FAQ, FAM, FAW,
  PF0,  // 20 arrays: PF0 + 5*k + fld, k = 0..3 (cells f-2..f+1), fld = h, q, m, W, b
  NFACE_ARR = PF0 + 20
};

struct Inst {
  int64_t off, foff;  // first cell, first face
  int n, nf, bc, has_b;
  double g, lam, dx, tau, tdx, lt2, rr, tdx2, i2dx;
};

struct Arr {
  double* c[NCELL_ARR];
  double* f[NFACE_ARR];
};

__host__ __device__ inline Inst make_inst(int64_t off, int64_t foff, int n, int bc, int has_b,
                                          double g, double lam, double dx, double tau) {
  Inst I;
  I.off = off; I.foff = foff; I.n = n; I.nf = bc == 0 ? n : n + 1; I.bc = bc; I.has_b = has_b;
  I.g = g; I.lam = lam; I.dx = dx; I.tau = tau;
  I.tdx = tau / dx;
  I.lt2 = lam * tau * tau;
  I.rr = I.tdx * I.tdx;
  I.tdx2 = 0.5 * I.tdx;
  I.i2dx = 1.0 / (2.0 * dx);
  return I;
}

// cell index with ghosts (|i| small): periodic wrap or transmissive copy
__host__ __device__ inline int cid(const Inst& I, int i) {
  if (I.bc == 0) {
    int r = i % I.n;
    return r < 0 ? r + I.n : r;
  }
  return i < 0 ? 0 : (i > I.n - 1 ? I.n - 1 : i);
}
__host__ __device__ inline int face_r(const Inst& I, int i) { return I.bc == 0 ? (i + 1) % I.n : i + 1; }

#define CA(k, i) A.c[k][I.off + (i)]
#define FAR(k, fi) A.f[k][I.foff + (fi)]

__host__ __device__ inline double bed(const Inst& I, const Arr& A, int i) {
  return I.has_b ? CA(BB, i) : 0.0;
}

// ---------------------------------------------------------------- forward
__host__ __device__ inline void f_face(const Inst& I, Arr& A, int f) {
  const int cm = cid(I, f - 2), c0 = cid(I, f - 1), c1 = cid(I, f), c2 = cid(I, f + 1);
  const double hm = CA(HE, cm), h0 = CA(HE, c0), h1 = CA(HE, c1), h2 = CA(HE, c2);
  const double qm = CA(QE, cm), q0 = CA(QE, c0), q1 = CA(QE, c1), q2 = CA(QE, c2);
  const double mm = CA(ME, cm), m0 = CA(ME, c0), m1 = CA(ME, c1), m2 = CA(ME, c2);
  const double wm = CA(WE, cm), w0 = CA(WE, c0), w1 = CA(WE, c1), w2 = CA(WE, c2);
  const double hL = h0 + 0.25 * (h1 - hm), hR = h1 - 0.25 * (h2 - h0);
  const double qL = q0 + 0.25 * (q1 - qm), qR = q1 - 0.25 * (q2 - q0);
  const double mL = m0 + 0.25 * (m1 - mm), mR = m1 - 0.25 * (m2 - m0);
  const double WL = w0 + 0.25 * (w1 - wm), WR = w1 - 0.25 * (w2 - w0);
  const double uL = qL / hL, uR = qR / hR;
  const double sL = fabs(uL) + sqrt(I.g * hL), sR = fabs(uR) + sqrt(I.g * hR);
  const double a = sL >= sR ? sL : sR;
  double jm = mR - mL;
  if (I.has_b) {
    const double bm = CA(BB, cm), b0 = CA(BB, c0), b1 = CA(BB, c1), b2 = CA(BB, c2);
    const double zf = 0.5 * ((h0 + b0) + (h1 + b1));
    const double rm = (zf - bm) * (zf - bm), r0 = (zf - b0) * (zf - b0);
    const double r1 = (zf - b1) * (zf - b1), r2 = (zf - b2) * (zf - b2);
    jm -= (r1 - 0.25 * (r2 - r0)) - (r0 + 0.25 * (r1 - rm));
  }
  FAR(FQ, f) = 0.5 * (qL * uL + qR * uR - a * (qR - qL));
  FAR(FM, f) = 0.5 * (mL * uL + mR * uR - a * jm);
  FAR(FW, f) = 0.5 * (WL * uL + WR * uR - a * (WR - WL));
}

struct Coef {
  double ih, eh, alpha, a2, b1, ib1, b2, beta, eta0, pt0, P0, S, phi, T;
};
__host__ __device__ inline Coef coefs(const Inst& I, double h, double m, double md) {
  Coef c;
  c.ih = 1.0 / h;
  c.eh = m * c.ih * c.ih;
  c.alpha = -(2.0 * c.eh - 1.0) * c.ih * (1.0 / 3.0);
  c.a2 = I.g * h + I.lam * c.eh * c.eh - (I.lam / 3.0) * c.eh;
  c.b1 = 1.0 + I.lt2 * c.ih * c.ih;
  c.ib1 = 1.0 / c.b1;
  c.b2 = 2.0 * I.lt2 * c.ib1 * c.ib1 * c.ih * c.ih * c.ih;
  c.beta = c.a2 + I.lam * c.alpha * c.b2 * md;
  c.eta0 = md * c.ib1 * c.ih;
  c.pt0 = (I.lam / 3.0) * (1.0 - c.eta0 * c.ih);
  c.P0 = 0.5 * I.g * h * h + c.eta0 * c.pt0;
  c.S = c.P0 - c.beta * h;
  if (I.has_b) {
    c.phi = (2.0 * I.lam / 3.0) * md * c.ih * c.ih * c.ih * c.ib1 * c.ib1;
    c.T = c.pt0 - c.phi * h;
  } else {
    c.phi = 0.0;
    c.T = 0.0;
  }
  return c;
}

__host__ __device__ inline void f_rec(const Inst& I, Arr& A, int i) {
  const int fl = i, fr = face_r(I, i);
  const double Db = (bed(I, A, cid(I, i + 1)) - bed(I, A, cid(I, i - 1))) * I.i2dx;
  const double Wd = CA(WO, i) - I.tdx * (FAR(FW, fr) - FAR(FW, fl)) + I.lam * I.tau;
  double md = CA(MO, i) - I.tdx * (FAR(FM, fr) - FAR(FM, fl));
  if (I.has_b) md -= I.tau * 1.5 * CA(QE, i) * Db;
  md += I.tau * Wd;
  const double qd = CA(QO, i) - I.tdx * (FAR(FQ, fr) - FAR(FQ, fl));
  const Coef c = coefs(I, CA(HE, i), CA(ME, i), md);
  CA(QD, i) = qd; CA(MD, i) = md; CA(WD, i) = Wd;
  CA(BETA, i) = c.beta; CA(SS, i) = c.S; CA(PHI, i) = c.phi; CA(TT, i) = c.T;
}

__host__ __device__ inline void f_row(const Inst& I, Arr& A, int i) {
  const int L = cid(I, i - 1), R = cid(I, i + 1);
  const double rr = I.rr;
  double lo = -rr * CA(BETA, L), up = -rr * CA(BETA, R), di = 1.0 + 2.0 * rr * CA(BETA, i);
  double rhs = CA(HO, i) - I.tdx2 * (CA(QD, R) - CA(QD, L)) +
               rr * ((CA(SS, R) - CA(SS, i)) - (CA(SS, i) - CA(SS, L)));
  if (I.has_b) {
    const double hg = 0.5 * I.g;
    const double bL = CA(BB, L), bC = CA(BB, i), bR = CA(BB, R);
    const double dbm = bC - bL, dbp = bR - bC;
    const double eL = hg + 0.75 * CA(PHI, L), eC = hg + 0.75 * CA(PHI, i), eR = hg + 0.75 * CA(PHI, R);
    lo = -rr * (CA(BETA, L) - dbm * eL);
    up = -rr * (CA(BETA, R) + dbp * eR);
    di = 1.0 + rr * (2.0 * CA(BETA, i) - (dbp - dbm) * eC);
    rhs += rr * 0.75 * (dbp * (CA(TT, i) + CA(TT, R)) - dbm * (CA(TT, L) + CA(TT, i)));
  }
  if (I.bc != 0 && i == 0) { di += lo; lo = 0.0; }
  if (I.bc != 0 && i == I.n - 1) { di += up; up = 0.0; }
  CA(LO, i) = lo; CA(DI, i) = di; CA(UP, i) = up; CA(RHS, i) = rhs;
}

// ---------------------------------------------------------------- reverse
__host__ __device__ inline void r_back(const Inst& I, Arr& A, int i) {
  const double h = CA(HB, i), ih = 1.0 / h, ih2 = ih * ih, md = CA(MD, i);
  const double rden = 1.0 / (1.0 + I.lt2 * ih2);
  const double mn = md * rden;
  const double aW = CA(AW, i), aM = CA(AM, i), aQ = CA(AQ, i);
  double hA = CA(AH, i);
  CA(WDA, i) = aW;
  const double mnA = aM - I.lam * I.tau * ih2 * aW;
  hA += 2.0 * I.lam * I.tau * mn * ih2 * ih * aW;
  CA(MDA, i) = mnA * rden;
  hA += mnA * md * (2.0 * I.lt2 * ih2 * ih) * rden * rden;
  CA(QDA0, i) = aQ;
  const double fa = -I.tau * aQ;
  CA(FA, i) = fa;
  if (I.has_b) {
    const int L = cid(I, i - 1), R = cid(I, i + 1);
    const double Db = (CA(BB, R) - CA(BB, L)) * I.i2dx;
    const double pt = CA(TT, i) + CA(PHI, i) * h;
    CA(TA0, i) = 1.5 * fa * Db;
    CA(PHIA0, i) = 1.5 * fa * Db * h;
    hA += 1.5 * fa * Db * CA(PHI, i);
    CA(DBA, i) = fa * (0.5 * I.g * (CA(HB, R) + CA(HB, L)) + 1.5 * pt);
  } else {
    CA(TA0, i) = 0.0; CA(PHIA0, i) = 0.0; CA(DBA, i) = 0.0;
  }
  CA(HBA0, i) = hA;
}

// distinct candidate cells j-1, j, j+1 (wrapped or clipped); returns count
__host__ __device__ inline int near3(const Inst& I, int j, int out[3]) {
  int k = 0;
  for (int d = -1; d <= 1; ++d) {
    int i = j + d;
    if (I.bc == 0) {
      i = cid(I, i);
    } else if (i < 0 || i > I.n - 1) {
      continue;
    }
    bool dup = false;
    for (int e = 0; e < k; ++e) dup |= out[e] == i;
    if (!dup) out[k++] = i;
  }
  return k;
}

__host__ __device__ inline void r_back_gather(const Inst& I, Arr& A, int j) {
  double PA = 0.0, hA = CA(HBA0, j), bA = 0.0;
  int cand[3];
  const int nc = near3(I, j, cand);
  for (int e = 0; e < nc; ++e) {
    const int i = cand[e];
    const int L = cid(I, i - 1), R = cid(I, i + 1);
    const double fa = CA(FA, i);
    double hb_term = 0.0;
    if (I.has_b) hb_term = fa * 0.5 * I.g * (CA(BB, R) - CA(BB, L)) * I.i2dx;
    if (R == j) { PA += fa * I.i2dx; hA += hb_term; bA += CA(DBA, i) * I.i2dx; }
    if (L == j) { PA -= fa * I.i2dx; hA += hb_term; bA -= CA(DBA, i) * I.i2dx; }
  }
  CA(SA0, j) = PA;
  CA(BETAA0, j) = PA * CA(HB, j);
  hA += PA * CA(BETA, j);
  CA(HBA, j) = hA;
  CA(BAB, j) = bA;
}

__host__ __device__ inline void r_transpose(const Inst& I, Arr& A, int i) {
  const bool per = I.bc == 0;
  CA(LOT, i) = (per || i > 0) ? CA(UP, cid(I, i - 1)) : 0.0;
  CA(UPT, i) = (per || i < I.n - 1) ? CA(LO, cid(I, i + 1)) : 0.0;
  CA(DIT, i) = CA(DI, i);
}

__host__ __device__ inline void r_row(const Inst& I, Arr& A, int i) {
  const int L = cid(I, i - 1), R = cid(I, i + 1);
  const double lam = CA(LAM, i);
  double loA = -lam * CA(HB, L), diA = -lam * CA(HB, i), upA = -lam * CA(HB, R);
  const double rhsA = lam;
  if (I.bc != 0 && i == 0) loA = diA;         // folded: di = di_raw + lo_raw
  if (I.bc != 0 && i == I.n - 1) upA = diA;   // folded: di = di_raw + up_raw
  const double rr = I.rr;
  double bLA = -rr * loA, bRA = -rr * upA, bCA = 2.0 * rr * diA;
  double eLA = 0.0, eCA = 0.0, eRA = 0.0, dbmA = 0.0, dbpA = 0.0;
  double tLA = 0.0, tCA = 0.0, tRA = 0.0;
  if (I.has_b) {
    const double hg = 0.5 * I.g;
    const double bL = CA(BB, L), bC = CA(BB, i), bR = CA(BB, R);
    const double dbm = bC - bL, dbp = bR - bC;
    const double eL = hg + 0.75 * CA(PHI, L), eC = hg + 0.75 * CA(PHI, i), eR = hg + 0.75 * CA(PHI, R);
    eLA = rr * dbm * loA;
    dbmA = rr * eL * loA;
    eRA = -rr * dbp * upA;
    dbpA = -rr * eR * upA;
    eCA = -rr * (dbp - dbm) * diA;
    dbpA += -rr * eC * diA;
    dbmA += rr * eC * diA;
    tCA = 0.75 * rr * (dbp - dbm) * rhsA;
    tRA = 0.75 * rr * dbp * rhsA;
    tLA = -0.75 * rr * dbm * rhsA;
    dbpA += 0.75 * rr * (CA(TT, i) + CA(TT, R)) * rhsA;
    dbmA += -0.75 * rr * (CA(TT, L) + CA(TT, i)) * rhsA;
  }
  CA(RLB, i) = bLA; CA(RLS, i) = rr * rhsA; CA(RLQ, i) = I.tdx2 * rhsA; CA(RLP, i) = 0.75 * eLA; CA(RLT, i) = tLA;
  CA(RRB, i) = bRA; CA(RRS, i) = rr * rhsA; CA(RRQ, i) = -I.tdx2 * rhsA; CA(RRP, i) = 0.75 * eRA; CA(RRT, i) = tRA;
  CA(RCB, i) = bCA; CA(RCS, i) = -2.0 * rr * rhsA; CA(RCQ, i) = 0.0; CA(RCP, i) = 0.75 * eCA; CA(RCT, i) = tCA;
  CA(HOA, i) = rhsA;
  CA(DBMA, i) = dbmA;
  CA(DBPA, i) = dbpA;
}

__host__ __device__ inline void r_row_gather(const Inst& I, Arr& A, int j) {
  double bt = CA(BETAA0, j), st = CA(SA0, j), qt = CA(QDA0, j), pt = CA(PHIA0, j), tt = CA(TA0, j);
  double bA = 0.0;
  int cand[3];
  const int nc = near3(I, j, cand);
  for (int e = 0; e < nc; ++e) {
    const int i = cand[e];
    if (i == j) {
      bt += CA(RCB, i); st += CA(RCS, i); qt += CA(RCQ, i); pt += CA(RCP, i); tt += CA(RCT, i);
      bA += CA(DBMA, i) - CA(DBPA, i);
    }
    if (cid(I, i - 1) == j) {
      bt += CA(RLB, i); st += CA(RLS, i); qt += CA(RLQ, i); pt += CA(RLP, i); tt += CA(RLT, i);
      bA -= CA(DBMA, i);
    }
    if (cid(I, i + 1) == j) {
      bt += CA(RRB, i); st += CA(RRS, i); qt += CA(RRQ, i); pt += CA(RRP, i); tt += CA(RRT, i);
      bA += CA(DBPA, i);
    }
  }
  CA(BETAT, j) = bt; CA(STT, j) = st; CA(QDT, j) = qt; CA(PHIT, j) = pt; CA(TTT, j) = tt;
  CA(BAR, j) = bA;
}

__host__ __device__ inline void r_rec(const Inst& I, Arr& A, int i) {
  const double h = CA(HE, i), m = CA(ME, i), q = CA(QE, i), md = CA(MD, i);
  const Coef c = coefs(I, h, m, md);
  const double lam = I.lam;
  double hA = 0.0, mA = 0.0, ihA = 0.0, ib1A = 0.0, mdA = 0.0;
  const double TA = CA(TTT, i), SA = CA(STT, i);
  double phiA = CA(PHIT, i), betaA = CA(BETAT, i);
  double pt0A = 0.0;
  if (I.has_b) {
    pt0A += TA;
    phiA += -h * TA;
    hA += -c.phi * TA;
  }
  const double P0A = SA;
  betaA += -h * SA;
  hA += -c.beta * SA;
  hA += I.g * h * P0A;
  double eta0A = c.pt0 * P0A;
  pt0A += c.eta0 * P0A;
  eta0A += -(lam / 3.0) * c.ih * pt0A;
  ihA += -(lam / 3.0) * c.eta0 * pt0A;
  if (I.has_b) {
    const double k = 2.0 * lam / 3.0;
    mdA += k * c.ih * c.ih * c.ih * c.ib1 * c.ib1 * phiA;
    ihA += 3.0 * k * md * c.ih * c.ih * c.ib1 * c.ib1 * phiA;
    ib1A += 2.0 * k * md * c.ih * c.ih * c.ih * c.ib1 * phiA;
  }
  mdA += c.ib1 * c.ih * eta0A;
  ib1A += md * c.ih * eta0A;
  ihA += md * c.ib1 * eta0A;
  const double a2A = betaA;
  const double alphaA = lam * c.b2 * md * betaA;
  const double b2A = lam * c.alpha * md * betaA;
  mdA += lam * c.alpha * c.b2 * betaA;
  ib1A += 4.0 * I.lt2 * c.ib1 * c.ih * c.ih * c.ih * b2A;
  ihA += 6.0 * I.lt2 * c.ib1 * c.ib1 * c.ih * c.ih * b2A;
  const double b1A = -c.ib1 * c.ib1 * ib1A;
  ihA += 2.0 * I.lt2 * c.ih * b1A;
  hA += I.g * a2A;
  double ehA = (2.0 * lam * c.eh - lam / 3.0) * a2A;
  ehA += -(2.0 / 3.0) * c.ih * alphaA;
  ihA += -(2.0 * c.eh - 1.0) * (1.0 / 3.0) * alphaA;
  mA += c.ih * c.ih * ehA;
  ihA += 2.0 * m * c.ih * ehA;
  hA += -c.ih * c.ih * ihA;
  const double mdT = CA(MDA, i) + mdA;
  const double tdx = I.tdx;
  CA(OAM, i) = mdT;
  CA(FRM, i) = -tdx * mdT;
  CA(FLM, i) = tdx * mdT;
  double qEA = 0.0, DbA = 0.0;
  if (I.has_b) {
    const double Db = (CA(BB, cid(I, i + 1)) - CA(BB, cid(I, i - 1))) * I.i2dx;
    qEA = -1.5 * I.tau * Db * mdT;
    DbA = -1.5 * I.tau * q * mdT;
  }
  const double WdT = CA(WDA, i) + I.tau * mdT;
  CA(OAW, i) = WdT;
  CA(FRW, i) = -tdx * WdT;
  CA(FLW, i) = tdx * WdT;
  const double qdA = CA(QDT, i);
  CA(OAQ, i) = qdA;
  CA(FRQ, i) = -tdx * qdA;
  CA(FLQ, i) = tdx * qdA;
  CA(OAH, i) = CA(HOA, i);
  CA(EAH0, i) = hA;
  CA(EAM0, i) = mA;
  CA(EAQ0, i) = qEA;
  CA(DB2A, i) = DbA;
}

__host__ __device__ inline void r_face_gather(const Inst& I, Arr& A, int f) {
  double aq = 0.0, am = 0.0, aw = 0.0;
  const bool per = I.bc == 0;
  if (per || f >= 1) {  // cell left of the face: this is its right face
    const int cl = cid(I, f - 1);
    aq += CA(FRQ, cl); am += CA(FRM, cl); aw += CA(FRW, cl);
  }
  if (per || f <= I.n - 1) {  // cell right of the face: this is its left face
    const int cr = per ? f % I.n : f;
    aq += CA(FLQ, cr); am += CA(FLM, cr); aw += CA(FLW, cr);
  }
  FAR(FAQ, f) = aq; FAR(FAM, f) = am; FAR(FAW, f) = aw;
}

__host__ __device__ inline void r_flux(const Inst& I, Arr& A, int f) {
  const int cs[4] = {cid(I, f - 2), cid(I, f - 1), cid(I, f), cid(I, f + 1)};
  double h[4], q[4], m[4], w[4], b[4];
  for (int k = 0; k < 4; ++k) {
    h[k] = CA(HE, cs[k]); q[k] = CA(QE, cs[k]); m[k] = CA(ME, cs[k]); w[k] = CA(WE, cs[k]);
    b[k] = I.has_b ? CA(BB, cs[k]) : 0.0;
  }
  const double hL = h[1] + 0.25 * (h[2] - h[0]), hR = h[2] - 0.25 * (h[3] - h[1]);
  const double qL = q[1] + 0.25 * (q[2] - q[0]), qR = q[2] - 0.25 * (q[3] - q[1]);
  const double mL = m[1] + 0.25 * (m[2] - m[0]), mR = m[2] - 0.25 * (m[3] - m[1]);
  const double WL = w[1] + 0.25 * (w[2] - w[0]), WR = w[2] - 0.25 * (w[3] - w[1]);
  const double uL = qL / hL, uR = qR / hR;
  const double gsL = sqrt(I.g * hL), gsR = sqrt(I.g * hR);
  const double sL = fabs(uL) + gsL, sR = fabs(uR) + gsR;
  const bool leftmax = sL >= sR;
  const double a = leftmax ? sL : sR;
  double rk[4] = {0, 0, 0, 0}, zf = 0.0, jm = mR - mL;
  if (I.has_b) {
    zf = 0.5 * ((h[1] + b[1]) + (h[2] + b[2]));
    for (int k = 0; k < 4; ++k) rk[k] = (zf - b[k]) * (zf - b[k]);
    jm -= (rk[2] - 0.25 * (rk[3] - rk[1])) - (rk[1] + 0.25 * (rk[2] - rk[0]));
  }
  const double aq = FAR(FAQ, f), am = FAR(FAM, f), aw = FAR(FAW, f);
  double qLA = 0.5 * (uL + a) * aq, qRA = 0.5 * (uR - a) * aq;
  double uLA = 0.5 * qL * aq, uRA = 0.5 * qR * aq;
  double aA = -0.5 * (qR - qL) * aq;
  const double mLA = 0.5 * (uL + a) * am, mRA = 0.5 * (uR - a) * am;
  uLA += 0.5 * mL * am;
  uRA += 0.5 * mR * am;
  aA += -0.5 * jm * am;
  const double mhRA = 0.5 * a * am, mhLA = -0.5 * a * am;
  const double WLA = 0.5 * (uL + a) * aw, WRA = 0.5 * (uR - a) * aw;
  uLA += 0.5 * WL * aw;
  uRA += 0.5 * WR * aw;
  aA += -0.5 * (WR - WL) * aw;
  const double sLA = leftmax ? aA : 0.0, sRA = leftmax ? 0.0 : aA;
  uLA += (uL < 0.0 ? -1.0 : 1.0) * sLA;
  uRA += (uR < 0.0 ? -1.0 : 1.0) * sRA;
  double hLA = I.g / (2.0 * gsL) * sLA, hRA = I.g / (2.0 * gsR) * sRA;
  qLA += uLA / hL;
  hLA += -uL / hL * uLA;
  qRA += uRA / hR;
  hRA += -uR / hR * uRA;
  double pa[5][4];  // fld x cell
  auto rec = [&](int fld, double vLA, double vRA) {
    pa[fld][0] = -0.25 * vLA;
    pa[fld][1] = vLA + 0.25 * vRA;
    pa[fld][2] = 0.25 * vLA + vRA;
    pa[fld][3] = -0.25 * vRA;
  };
  rec(0, hLA, hRA);
  rec(1, qLA, qRA);
  rec(2, mLA, mRA);
  rec(3, WLA, WRA);
  for (int k = 0; k < 4; ++k) pa[4][k] = 0.0;
  if (I.has_b) {
    const double rA[4] = {-0.25 * mhLA, mhLA + 0.25 * mhRA, 0.25 * mhLA + mhRA, -0.25 * mhRA};
    double zfA = 0.0;
    for (int k = 0; k < 4; ++k) {
      zfA += 2.0 * (zf - b[k]) * rA[k];
      pa[4][k] += -2.0 * (zf - b[k]) * rA[k];
    }
    pa[0][1] += 0.5 * zfA;
    pa[0][2] += 0.5 * zfA;
    pa[4][1] += 0.5 * zfA;
    pa[4][2] += 0.5 * zfA;
  }
  for (int k = 0; k < 4; ++k)
    for (int fld = 0; fld < 5; ++fld) FAR(PF0 + 5 * k + fld, f) = pa[fld][k];
}

// cell gather of face partials and bed-source terms; writes the stage's
// adjoint of U_E and b
__host__ __device__ inline void r_cell_gather(const Inst& I, Arr& A, int j) {
  double ea[5] = {CA(EAH0, j), CA(EAQ0, j), CA(EAM0, j), 0.0, 0.0};
  for (int d = -1; d <= 2; ++d) {
    int f = j + d;
    if (I.bc == 0) {
      f = cid(I, f);
    } else if (f < 0 || f > I.n) {
      continue;
    }
    // periodic faces are distinct for n >= 4
    for (int k = 0; k < 4; ++k) {
      if (cid(I, f - 2 + k) == j)
        for (int fld = 0; fld < 5; ++fld) ea[fld] += FAR(PF0 + 5 * k + fld, f);
    }
  }
  double bA = CA(BAB, j) + CA(BAR, j) + ea[4];
  if (I.has_b) {
    int cand[3];
    const int nc = near3(I, j, cand);
    for (int e = 0; e < nc; ++e) {
      const int i = cand[e];
      if (cid(I, i + 1) == j) bA += CA(DB2A, i) * I.i2dx;
      if (cid(I, i - 1) == j) bA -= CA(DB2A, i) * I.i2dx;
    }
  }
  CA(EAH, j) = ea[0];
  CA(EAQ, j) = ea[1];
  CA(EAM, j) = ea[2];
  CA(EAW, j) = ea[3];
  CA(BAS, j) = I.has_b ? bA : 0.0;
}

#undef CA
#undef FAR

}  // namespace adj

// ---------------------------------------------------------------------------
// Tridiagonal solve of one system of M rows held in global arrays, by one
// workgroup (chunked Thomas in global scratch + level-1 PCR in LDS; cyclic
// couplings handled by the two end rows).  All threads must call it.
// ---------------------------------------------------------------------------
template <int NT>
__device__ void wg_tri_solve(Lds<NT>& S, const double* __restrict__ lo, const double* __restrict__ di,
                             const double* __restrict__ up, const double* __restrict__ rhs,
                             double* __restrict__ x, int M, bool cyclic, double* __restrict__ scp,
                             double* __restrict__ sy, double* __restrict__ sv,
                             double* __restrict__ sw) {
  const int t = threadIdx.x;
  const Chunk ch = chunk_of(M, NT, t);
  const int k = ch.k;
  const int f = ch.first;
  const bool act = t < ch.active;
  if (act) {
    double cprev = 0.0, yprev = 0.0, vprev = 1.0, wprev = 0.0;
    for (int i = 1; i <= k - 2; ++i) {
      const double l = lo[f + i], d = di[f + i], u = up[f + i], r = rhs[f + i];
      const double inv = 1.0 / (d - l * cprev);
      const bool lastint = (i == k - 2);
      cprev = lastint ? 0.0 : u * inv;
      yprev = (r - l * yprev) * inv;
      vprev = (-l * vprev) * inv;
      wprev = (-l * wprev) * inv - (lastint ? u * inv : 0.0);
      scp[f + i] = cprev;
      sy[f + i] = yprev;
      sv[f + i] = vprev;
      sw[f + i] = wprev;
    }
    double yn = 0.0, vn = 0.0, wn = 0.0;
    for (int i = k - 2; i >= 1; --i) {
      const double c = scp[f + i];
      yn = sy[f + i] - c * yn;
      vn = sv[f + i] - c * vn;
      wn = sw[f + i] - c * wn;
      sy[f + i] = yn;
      sv[f + i] = vn;
      sw[f + i] = wn;
    }
    const int l = f + k - 1;
    double R0[4] = {lo[f], di[f], up[f], rhs[f]};
    double R1[4] = {lo[l], di[l], up[l], rhs[l]};
    if (k > 2) {
      const double v1 = sv[f + 1], w1 = sw[f + 1], y1 = sy[f + 1];
      const double vk = sv[l - 1], wk = sw[l - 1], yk = sy[l - 1];
      R0[1] = R0[1] + R0[2] * v1;
      R0[3] = R0[3] - R0[2] * y1;
      R0[2] = R0[2] * w1;
      R1[1] = R1[1] + R1[0] * wk;
      R1[3] = R1[3] - R1[0] * yk;
      R1[0] = R1[0] * vk;
    }
    S.a[2 * t] = R0[0]; S.b[2 * t] = R0[1]; S.c[2 * t] = R0[2]; S.d0[2 * t] = R0[3];
    S.d1[2 * t] = 0.0; S.d2[2 * t] = 0.0;
    S.a[2 * t + 1] = R1[0]; S.b[2 * t + 1] = R1[1]; S.c[2 * t + 1] = R1[2];
    S.d0[2 * t + 1] = R1[3]; S.d1[2 * t + 1] = 0.0; S.d2[2 * t + 1] = 0.0;
  }
  __syncthreads();
  const int n1 = 2 * ch.active;
  level1_interior<NT>(S, n1);
  if (t == 0) {
    double R0[4], R1[4], z0, zl;
    tile_rows<NT>(S, n1, R0, R1);
    if (!cyclic) {
      R0[0] = 0.0;
      R1[2] = 0.0;
    }
    solve_ends(R0, R1, cyclic, z0, zl);
    S.s[0] = z0;
    S.s[1] = zl;
  }
  __syncthreads();
  const double z0 = S.s[0], zl = S.s[1];
  if (act) {
    const int j0 = 2 * t, j1 = 2 * t + 1;
    const double zf = (j0 == 0) ? z0 : S.d0[j0] + S.d1[j0] * z0 + S.d2[j0] * zl;
    const double zb = (j1 == n1 - 1) ? zl : S.d0[j1] + S.d1[j1] * z0 + S.d2[j1] * zl;
    x[f] = zf;
    x[f + k - 1] = zb;
    for (int i = 1; i <= k - 2; ++i) x[f + i] = sy[f + i] + sv[f + i] * zf + sw[f + i] * zb;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Reverse of one stage for every instance (one workgroup each).  STAGE 2
// reads the stage inputs U_E = E0 U^n + E1 U^(1), U_old = T0 U^n + T1 U^(1)
// from the tape and writes abar(U^(1)) and the U^n part of the step's
// adjoint; STAGE 1 (U_E = U_old = U^n) adds its part and writes abar(U^n).
// b-bar of the stage is added to gb.
// ---------------------------------------------------------------------------
struct AdjStageArgs {
  const InstDesc* inst;
  const double* dt;
  const double* un[4];   // tape U^n
  const double* u1[4];   // tape U^(1) (stage 2)
  const double* b;
  const double* abar[4];  // adjoint of the stage output
  double* out1[4];        // STAGE 2: abar of U^(1)
  double* outn[4];        // STAGE 2: U^n part (written); STAGE 1: abar of U^n (= outn + ...)
  double* gb;             // accumulated bed adjoint (may be null)
  adj::Arr arr;
};

template <int NT, int STAGE>
__global__ __launch_bounds__(NT) void k_adj_stage(AdjStageArgs P) {
  __shared__ Lds<NT> S;
  const int j = blockIdx.x;
  const InstDesc D = P.inst[j];
  const double dt = P.dt[j];
  const int t = threadIdx.x;
  const int n = D.n;
  const int64_t off = D.off;
  const int64_t foff = D.off + j;  // n+1 face slots per instance
  adj::Inst I = adj::make_inst(off, foff, n, D.bc, D.has_b && P.b != nullptr, D.g, D.lam, D.dx,
                               kGamma * dt);
  adj::Arr& A = P.arr;
  using namespace adj;
  if (!(dt > 0.0)) {  // frozen instance: identity map
    for (int i = t; i < n; i += NT) {
      const int64_t gi = off + i;
      for (int fld = 0; fld < 4; ++fld) {
        if (STAGE == 2) {
          P.out1[fld][gi] = 0.0;
          P.outn[fld][gi] = P.abar[fld][gi];
        } else {
          P.outn[fld][gi] = P.outn[fld][gi] + P.abar[fld][gi];
        }
      }
    }
    return;
  }
  // stage inputs
  for (int i = t; i < n; i += NT) {
    const int64_t gi = off + i;
    double* E[4] = {A.c[HE], A.c[QE], A.c[ME], A.c[WE]};
    double* O[4] = {A.c[HO], A.c[QO], A.c[MO], A.c[WO]};
    for (int fld = 0; fld < 4; ++fld) {
      const double a = P.un[fld][gi];
      if (STAGE == 1) {
        E[fld][gi] = a;
        O[fld][gi] = a;
      } else {
        const double b = P.u1[fld][gi];
        E[fld][gi] = kE0 * a + kE1 * b;
        O[fld][gi] = kT0 * a + kT1 * b;
      }
      A.c[AH + fld][gi] = P.abar[fld][gi];
    }
    A.c[BB][gi] = I.has_b ? P.b[gi] : 0.0;
  }
  __syncthreads();
  for (int f = t; f < I.nf; f += NT) f_face(I, A, f);
  __syncthreads();
  for (int i = t; i < n; i += NT) f_rec(I, A, i);
  __syncthreads();
  for (int i = t; i < n; i += NT) f_row(I, A, i);
  __syncthreads();
  wg_tri_solve<NT>(S, A.c[LO] + off, A.c[DI] + off, A.c[UP] + off, A.c[RHS] + off, A.c[HB] + off,
                   n, I.bc == 0, A.c[SCP] + off, A.c[SY] + off, A.c[SV] + off, A.c[SW] + off);
  for (int i = t; i < n; i += NT) r_back(I, A, i);
  __syncthreads();
  for (int i = t; i < n; i += NT) r_back_gather(I, A, i);
  __syncthreads();
  for (int i = t; i < n; i += NT) r_transpose(I, A, i);
  __syncthreads();
  wg_tri_solve<NT>(S, A.c[LOT] + off, A.c[DIT] + off, A.c[UPT] + off, A.c[HBA] + off,
                   A.c[LAM] + off, n, I.bc == 0, A.c[SCP] + off, A.c[SY] + off, A.c[SV] + off,
                   A.c[SW] + off);
  for (int i = t; i < n; i += NT) r_row(I, A, i);
  __syncthreads();
  for (int i = t; i < n; i += NT) r_row_gather(I, A, i);
  __syncthreads();
  for (int i = t; i < n; i += NT) r_rec(I, A, i);
  __syncthreads();
  for (int f = t; f < I.nf; f += NT) r_face_gather(I, A, f);
  __syncthreads();
  for (int f = t; f < I.nf; f += NT) r_flux(I, A, f);
  __syncthreads();
  for (int i = t; i < n; i += NT) {
    r_cell_gather(I, A, i);
    const int64_t gi = off + i;
    const double ao[4] = {A.c[OAH][gi], A.c[OAQ][gi], A.c[OAM][gi], A.c[OAW][gi]};
    const double ae[4] = {A.c[EAH][gi], A.c[EAQ][gi], A.c[EAM][gi], A.c[EAW][gi]};
    for (int fld = 0; fld < 4; ++fld) {
      if (STAGE == 2) {
        P.out1[fld][gi] = kE1 * ae[fld] + kT1 * ao[fld];
        P.outn[fld][gi] = kE0 * ae[fld] + kT0 * ao[fld];
      } else {
        P.outn[fld][gi] = P.outn[fld][gi] + ae[fld] + ao[fld];
      }
    }
    if (P.gb && I.has_b) P.gb[gi] += A.c[BAS][gi];
  }
}

}  // namespace hsgn
