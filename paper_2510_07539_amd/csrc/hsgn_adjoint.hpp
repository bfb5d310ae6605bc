// hsgn_adjoint.hpp -- hand-written discrete adjoint of one semi-implicit stage.
//
// The stage maps (U_old, U_E; b) to U_new (Sec. 4.2, eq.
// GN_hyp_eq_semi_fully_discrete, with the readings of the forward kernels):
//   faces:   reconstruction + Rusanov fluxes of U_E
//   records: q+, m+, W+ (explicit predictor) and the linearisation beta, S,
//            phi, T of the pressure at U_E
//   rows:    A hbar = rhs (tridiagonal, cyclic when periodic)
//   back-substitution: q, m, W of U_new from hbar and the records.
// Its reverse takes the adjoint of U_new and returns the adjoints of U_old,
// U_E and b, in three launches per stage:
//   R1 (tiles): recompute faces, records, rows; reverse back-substitution;
//               write the transposed rows A^T and their right-hand side
//               hbar^a (adjoint of hbar)
//   R2 (one workgroup per instance): solve A^T lam = hbar^a
//   R3 (tiles): recompute, then reverse rows (A^a = -lam hbar^T,
//               rhs^a = lam), records and faces; write the adjoints.
// hbar is not solved again: it is the depth of the stage output, which the
// caller keeps.
//
// A tile owns a core of cells and recomputes a halo of H = 6 cells on each
// side; each thread owns one cell position (and the face on its left).  Cell
// positions are "virtual": a periodic instance is unrolled onto a line, every
// position holding the values of its cell modulo n, so stencils never wrap
// inside the tile; transmissive positions are the cells themselves, with the
// ghost copies expressed by clipping.  Values read at neighbouring positions
// live in LDS, values used only by their own cell in registers.  Every
// contribution to a neighbour is written by its source and gathered by its
// target (no floating-point atomics: results do not depend on timing).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "hsgn_kernels.hpp"
#include "hsgn_window.hpp"

namespace hsgn {
namespace adj {

constexpr int H = 6;  // halo cells on each side of a tile core (core <= NT - 2H)

struct TileA {
  int32_t inst;  // instance
  int32_t ts;    // first core cell (instance-relative)
  int32_t te;    // one past the last core cell
  int32_t pad;
};

// per-tile constants
struct TC {
  int n, bc, has_b, lo0;  // lo0: virtual cell of slot 0
  double g, lam, dx, tau, tdx, lt2, rr, tdx2, i2dx;
  double lam3, lam23;  // lambda / 3 and 2 lambda / 3
};

// virtual cell -> the position holding its values: periodic positions are
// their own; transmissive ghosts clip to the end cell
__device__ __forceinline__ int vcl(const TC& T, int v) {
  if (T.bc == 0) return v;
  return v < 0 ? 0 : (v > T.n - 1 ? T.n - 1 : v);
}
__device__ __forceinline__ int slot(const TC& T, int v) { return vcl(T, v) - T.lo0; }

// cells and faces that exist at virtual position v (face v: left of cell v)
__device__ __forceinline__ bool cell_ok(const TC& T, int v) { return T.bc == 0 || (v >= 0 && v < T.n); }
__device__ __forceinline__ bool face_ok(const TC& T, int f) { return T.bc == 0 || (f >= 0 && f <= T.n); }

struct Coef {
  double ih, eh, alpha, a2, b1, ib1, b2, beta, eta0, pt0, P0, S, phi, T;
};
__device__ __forceinline__ Coef coefs(const TC& I, double h, double m, double md) {
  Coef c;
  c.ih = frcp(h);
  c.eh = m * c.ih * c.ih;
  c.alpha = -(2.0 * c.eh - 1.0) * c.ih * (1.0 / 3.0);
  c.a2 = I.g * h + I.lam * c.eh * c.eh - I.lam3 * c.eh;
  c.b1 = 1.0 + I.lt2 * c.ih * c.ih;
  c.ib1 = frcp(c.b1);
  c.b2 = 2.0 * I.lt2 * c.ib1 * c.ib1 * c.ih * c.ih * c.ih;
  c.beta = c.a2 + I.lam * c.alpha * c.b2 * md;
  c.eta0 = md * c.ib1 * c.ih;
  c.pt0 = I.lam3 * (1.0 - c.eta0 * c.ih);
  c.P0 = 0.5 * I.g * h * h + c.eta0 * c.pt0;
  c.S = c.P0 - c.beta * h;
  if (I.has_b) {
    c.phi = I.lam23 * md * c.ih * c.ih * c.ih * c.ib1 * c.ib1;
    c.T = c.pt0 - c.phi * h;
  } else {
    c.phi = 0.0;
    c.T = 0.0;
  }
  return c;
}

// LDS of a tile: arrays read at neighbouring positions.  The unions hold
// arrays whose lifetimes do not overlap (barriers separate them).
template <int NT>
struct TileLds1 {  // R1
  double he[NT], qe[NT], me[NT], we[NT], bb[NT], hb[NT];  // U_E, bed, hbar
  double phi[NT], tt[NT];                                 // records read by rows
  double fa[NT], dba[NT];                                 // reverse back-substitution
  union {
    struct { double fq[NT], fm[NT], fw[NT]; } face;  // fluxes
    struct { double beta[NT], lo[NT], up[NT]; } row; // rows
  } u;
};
template <int NT>
struct TileLds3 {  // R3: 15 arrays (30 KB at NT = 256), so five workgroups fit a CU
  union {
    struct { double he[NT], qe[NT], me[NT], we[NT], bb[NT], hb[NT]; };  // U_E, bed, hbar
    double pf[5][NT];  // face partials, one stencil cell at a time (after the reverse faces)
  };
  double phi[NT], tt[NT];
  double fa[NT], dba[NT];
  double lam[NT];   // solution of the transposed system
  double db2a[NT];  // bed-slope source adjoint
  union {
    struct { double fq[NT], fm[NT], fw[NT]; } face;  // fluxes
    struct { double fr[3][NT]; } rface;              // adjoints of each cell's right face
  } u;
};

// instance cell of virtual position v (periodic: modulo n)
__device__ __forceinline__ int real_cell(const TC& T, int v) {
  if (T.bc != 0) return v;
  int c = v % T.n;
  return c < 0 ? c + T.n : c;
}

// Load the tile: U_E, the old state, the bed, hbar and the output adjoint.
template <int STAGE, class LT>
__device__ __forceinline__ void load_tile(const TC& T, LT& L, int64_t off, int v,
                                          const double* const* un, const double* const* u1,
                                          const double* b, const double* hbs,
                                          const double* const* abar, double E[4], double O[4],
                                          double aU[4]) {
  const int t = threadIdx.x;
  if (!cell_ok(T, v)) return;
  const int64_t gi = off + real_cell(T, v);
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    const double a = un[f][gi];
    if (STAGE == 1) {
      E[f] = a;
      O[f] = a;
    } else {
      const double d = u1[f][gi];
      E[f] = kE0 * a + kE1 * d;
      O[f] = kT0 * a + kT1 * d;
    }
    aU[f] = abar[f][gi];
  }
  L.he[t] = E[0];
  L.qe[t] = E[1];
  L.me[t] = E[2];
  L.we[t] = E[3];
  L.bb[t] = T.has_b ? b[gi] : 0.0;
  L.hb[t] = hbs[gi];
}

// Rusanov flux of face f (between virtual cells f-1 and f).
template <class LT>
__device__ __forceinline__ void face_flux(const TC& I, const LT& L, int f, double& Fq,
                                          double& Fm, double& Fw) {
  const int cm = slot(I, f - 2), c0 = slot(I, f - 1), c1 = slot(I, f), c2 = slot(I, f + 1);
  const double hm = L.he[cm], h0 = L.he[c0], h1 = L.he[c1], h2 = L.he[c2];
  const double qm = L.qe[cm], q0 = L.qe[c0], q1 = L.qe[c1], q2 = L.qe[c2];
  const double mm = L.me[cm], m0 = L.me[c0], m1 = L.me[c1], m2 = L.me[c2];
  const double wm = L.we[cm], w0 = L.we[c0], w1 = L.we[c1], w2 = L.we[c2];
  const double hL = h0 + 0.25 * (h1 - hm), hR = h1 - 0.25 * (h2 - h0);
  const double qL = q0 + 0.25 * (q1 - qm), qR = q1 - 0.25 * (q2 - q0);
  const double mL = m0 + 0.25 * (m1 - mm), mR = m1 - 0.25 * (m2 - m0);
  const double WL = w0 + 0.25 * (w1 - wm), WR = w1 - 0.25 * (w2 - w0);
  const double uL = qL * frcp(hL), uR = qR * frcp(hR);
  const double sL = fabs(uL) + fsqrt(I.g * hL), sR = fabs(uR) + fsqrt(I.g * hR);
  const double a = sL >= sR ? sL : sR;
  double jm = mR - mL;
  if (I.has_b) {
    const double bm = L.bb[cm], b0 = L.bb[c0], b1 = L.bb[c1], b2 = L.bb[c2];
    const double zf = 0.5 * ((h0 + b0) + (h1 + b1));
    const double rm = (zf - bm) * (zf - bm), r0 = (zf - b0) * (zf - b0);
    const double r1 = (zf - b1) * (zf - b1), r2 = (zf - b2) * (zf - b2);
    jm -= (r1 - 0.25 * (r2 - r0)) - (r0 + 0.25 * (r1 - rm));
  }
  Fq = 0.5 * (qL * uL + qR * uR - a * (qR - qL));
  Fm = 0.5 * (mL * uL + mR * uR - a * jm);
  Fw = 0.5 * (WL * uL + WR * uR - a * (WR - WL));
}

// Per-cell values of the forward records and the reverse back-substitution.
struct Own {
  double qd, md, Wd, beta, S, phi, T;       // records
  double WDA, MDA, QDA0, TA0, PHIA0, HBA0;  // reverse back-substitution (own part)
};

// Records of cell i (own thread) from the fluxes of faces i and i+1.
template <class LT>
__device__ __forceinline__ void records(const TC& I, const LT& L, int i, const double E[4],
                                        const double O[4], Own& w) {
  const int t = i - I.lo0;
  const double Db = (L.bb[slot(I, i + 1)] - L.bb[slot(I, i - 1)]) * I.i2dx;
  const double Wd = O[3] - I.tdx * (L.u.face.fw[t + 1] - L.u.face.fw[t]) + I.lam * I.tau;
  double md = O[2] - I.tdx * (L.u.face.fm[t + 1] - L.u.face.fm[t]);
  if (I.has_b) md -= I.tau * 1.5 * E[1] * Db;
  md += I.tau * Wd;
  const double qd = O[1] - I.tdx * (L.u.face.fq[t + 1] - L.u.face.fq[t]);
  const Coef c = coefs(I, E[0], E[2], md);
  w.qd = qd; w.md = md; w.Wd = Wd;
  w.beta = c.beta; w.S = c.S; w.phi = c.phi; w.T = c.T;
}

// Reverse back-substitution at cell i: own adjoints, and the parts that
// neighbours gather (fa, dba).
template <class LT>
__device__ __forceinline__ void rev_back(const TC& I, LT& L, int i, const double aU[4],
                                         Own& w) {
  const int t = i - I.lo0;
  const double h = L.hb[t], ih = frcp(h), ih2 = ih * ih, md = w.md;
  const double rden = frcp(1.0 + I.lt2 * ih2);
  const double mn = md * rden;
  const double aW = aU[3], aM = aU[2], aQ = aU[1];
  double hA = aU[0];
  w.WDA = aW;
  const double mnA = aM - I.lam * I.tau * ih2 * aW;
  hA += 2.0 * I.lam * I.tau * mn * ih2 * ih * aW;
  w.MDA = mnA * rden;
  hA += mnA * md * (2.0 * I.lt2 * ih2 * ih) * rden * rden;
  w.QDA0 = aQ;
  const double fa = -I.tau * aQ;
  L.fa[t] = fa;
  if (I.has_b) {
    const int sL = slot(I, i - 1), sR = slot(I, i + 1);
    const double Db = (L.bb[sR] - L.bb[sL]) * I.i2dx;
    const double pt = w.T + w.phi * h;
    w.TA0 = 1.5 * fa * Db;
    w.PHIA0 = 1.5 * fa * Db * h;
    hA += 1.5 * fa * Db * w.phi;
    L.dba[t] = fa * (0.5 * I.g * (L.hb[sR] + L.hb[sL]) + 1.5 * pt);
  } else {
    w.TA0 = 0.0;
    w.PHIA0 = 0.0;
    L.dba[t] = 0.0;
  }
  w.HBA0 = hA;
}

// Gather of the back-substitution parts at cell j: adjoints of S, beta and
// hbar, and the bed part.  Source rows are j-1, j, j+1 (those that exist).
template <class LT>
__device__ __forceinline__ void gather_back(const TC& I, const LT& L, int j,
                                            const Own& w, double& SA0, double& BETAA0,
                                            double& HBA, double& BAB) {
  double PA = 0.0, hA = w.HBA0, bA = 0.0;
#pragma unroll
  for (int d = -1; d <= 1; ++d) {
    const int i = j + d;
    if (!cell_ok(I, i)) continue;
    const int Lc = vcl(I, i - 1), Rc = vcl(I, i + 1);
    const int s = i - I.lo0;
    const double fa = L.fa[s];
    double hb_term = 0.0;
    if (I.has_b) hb_term = fa * 0.5 * I.g * (L.bb[Rc - I.lo0] - L.bb[Lc - I.lo0]) * I.i2dx;
    if (Rc == j) { PA += fa * I.i2dx; hA += hb_term; bA += L.dba[s] * I.i2dx; }
    if (Lc == j) { PA -= fa * I.i2dx; hA += hb_term; bA -= L.dba[s] * I.i2dx; }
  }
  SA0 = PA;
  BETAA0 = PA * L.hb[j - I.lo0];
  HBA = hA + PA * w.beta;
  BAB = bA;
}

// Parts of the reverse of row i (A^a = -lam hbar^T, rhs^a = lam) that
// belong to the records (beta, S, q+, phi, T) of cells i-1 (l), i+1 (r) and
// i (c), and to the bed differences (dbm, dbp).
struct RowParts {
  double l[5], r[5], c[5], dbm, dbp;
};
template <class LT>
__device__ __forceinline__ RowParts row_parts(const TC& I, const LT& L, int i) {
  const int t = i - I.lo0;
  const int sL = slot(I, i - 1), sR = slot(I, i + 1);
  const double lamv = L.lam[t];
  double loA = -lamv * L.hb[sL], diA = -lamv * L.hb[t], upA = -lamv * L.hb[sR];
  const double rhsA = lamv;
  if (I.bc != 0 && i == 0) loA = diA;        // folded: di = di_raw + lo_raw
  if (I.bc != 0 && i == I.n - 1) upA = diA;  // folded: di = di_raw + up_raw
  const double rr = I.rr;
  const double bLA = -rr * loA, bRA = -rr * upA, bCA = 2.0 * rr * diA;
  double eLA = 0.0, eCA = 0.0, eRA = 0.0, dbmA = 0.0, dbpA = 0.0;
  double tLA = 0.0, tCA = 0.0, tRA = 0.0;
  if (I.has_b) {
    const double hg = 0.5 * I.g;
    const double bL = L.bb[sL], bC = L.bb[t], bR = L.bb[sR];
    const double dbm = bC - bL, dbp = bR - bC;
    const double eL = hg + 0.75 * L.phi[sL], eC = hg + 0.75 * L.phi[t], eR = hg + 0.75 * L.phi[sR];
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
    dbpA += 0.75 * rr * (L.tt[t] + L.tt[sR]) * rhsA;
    dbmA += -0.75 * rr * (L.tt[sL] + L.tt[t]) * rhsA;
  }
  RowParts p;
  p.l[0] = bLA; p.l[1] = rr * rhsA; p.l[2] = I.tdx2 * rhsA; p.l[3] = 0.75 * eLA; p.l[4] = tLA;
  p.r[0] = bRA; p.r[1] = rr * rhsA; p.r[2] = -I.tdx2 * rhsA; p.r[3] = 0.75 * eRA; p.r[4] = tRA;
  p.c[0] = bCA; p.c[1] = -2.0 * rr * rhsA; p.c[2] = 0.0; p.c[3] = 0.75 * eCA; p.c[4] = tCA;
  p.dbm = dbmA;
  p.dbp = dbpA;
  return p;
}

__device__ __forceinline__ TC make_tc(const InstDesc& D, int lo0, double dt) {
  TC T;
  T.n = D.n; T.bc = D.bc; T.has_b = D.has_b; T.lo0 = lo0;
  T.g = D.g; T.lam = D.lam; T.dx = D.dx; T.tau = kGamma * dt;
  T.tdx = T.tau / T.dx;
  T.lt2 = T.lam * T.tau * T.tau;
  T.rr = T.tdx * T.tdx;
  T.tdx2 = 0.5 * T.tdx;
  T.i2dx = 1.0 / (2.0 * T.dx);
  T.lam3 = T.lam / 3.0;
  T.lam23 = 2.0 * T.lam / 3.0;
  return T;
}

}  // namespace adj

struct AdjTileArgs {
  const InstDesc* inst;
  const adj::TileA* tiles;
  const double* dt;
  const double* un[4];    // tape U^n
  const double* u1[4];    // tape U^(1) (stage 2)
  const double* hbar;     // depth of the stage output (hbar)
  const double* b;        // bed (null if none)
  const double* abar[4];  // adjoint of the stage output
  // transposed system (R1 writes it, R2 solves it, R3 reads lam)
  double* lot;
  double* dit;
  double* upt;
  double* hba;
  const double* lam;
  double* out1[4];  // STAGE 2: adjoint of U^(1)
  double* outn[4];  // STAGE 2: U^n part (written); STAGE 1: adds its part
  double* gb;       // accumulated bed adjoint (null if not wanted)
};

// ---------------------------------------------------------------------------
// R1: transposed rows and their right-hand side hbar^a on the tile core.
// Valid ranges (slots): faces [2, NT-2], records [2, NT-3], rows [3, NT-4].
// ---------------------------------------------------------------------------
template <int NT, int STAGE>
__global__ __launch_bounds__(NT) void k_adj_r1(AdjTileArgs P) {
  using namespace adj;
  __shared__ TileLds1<NT> L;
  const TileA tl = P.tiles[blockIdx.x];
  const InstDesc D = P.inst[tl.inst];
  const double dt = P.dt[tl.inst];
  if (!(dt > 0.0)) return;  // frozen instance: R3 passes the adjoint through
  const int t = threadIdx.x;
  const TC I = make_tc(D, tl.ts - H, dt);
  const int v = I.lo0 + t;
  double E[4] = {0, 0, 0, 0}, O[4] = {0, 0, 0, 0}, aU[4] = {0, 0, 0, 0};
  load_tile<STAGE>(I, L, D.off, v, P.un, P.u1, P.b, P.hbar, P.abar, E, O, aU);
  __syncthreads();
  if (t >= 2 && t <= NT - 2 && face_ok(I, v))
    face_flux(I, L, v, L.u.face.fq[t], L.u.face.fm[t], L.u.face.fw[t]);
  __syncthreads();
  Own w;
  const bool rec_ok = t >= 2 && t <= NT - 3 && cell_ok(I, v);
  if (rec_ok) records(I, L, v, E, O, w);
  __syncthreads();  // fluxes are dead: the union now holds rows
  if (rec_ok) {
    L.u.row.beta[t] = w.beta;
    L.phi[t] = w.phi;
    L.tt[t] = w.T;
    rev_back(I, L, v, aU, w);
  }
  __syncthreads();
  // rows (the forward's expressions, right-hand side not needed)
  double di = 0.0, hbarA = 0.0;
  const bool row_ok = t >= 3 && t <= NT - 4 && cell_ok(I, v);
  if (row_ok) {
    const int sL = slot(I, v - 1), sR = slot(I, v + 1);
    const double rr = I.rr;
    double lo = -rr * L.u.row.beta[sL], up = -rr * L.u.row.beta[sR];
    di = 1.0 + 2.0 * rr * L.u.row.beta[t];
    if (I.has_b) {
      const double hg = 0.5 * I.g;
      const double bL = L.bb[sL], bC = L.bb[t], bR = L.bb[sR];
      const double dbm = bC - bL, dbp = bR - bC;
      const double eL = hg + 0.75 * L.phi[sL], eC = hg + 0.75 * L.phi[t], eR = hg + 0.75 * L.phi[sR];
      lo = -rr * (L.u.row.beta[sL] - dbm * eL);
      up = -rr * (L.u.row.beta[sR] + dbp * eR);
      di = 1.0 + rr * (2.0 * L.u.row.beta[t] - (dbp - dbm) * eC);
    }
    if (I.bc != 0 && v == 0) { di += lo; lo = 0.0; }
    if (I.bc != 0 && v == I.n - 1) { di += up; up = 0.0; }
    double SA0, BETAA0, BAB;
    gather_back(I, L, v, w, SA0, BETAA0, hbarA, BAB);
    L.u.row.lo[t] = lo;  // no storage shared with beta
    L.u.row.up[t] = up;
  }
  __syncthreads();
  if (row_ok && v >= tl.ts && v < tl.te) {
    const bool per = I.bc == 0;
    const int64_t gi = D.off + v;
    P.lot[gi] = (per || v > 0) ? L.u.row.up[slot(I, v - 1)] : 0.0;
    P.upt[gi] = (per || v < I.n - 1) ? L.u.row.lo[slot(I, v + 1)] : 0.0;
    P.dit[gi] = di;
    P.hba[gi] = hbarA;
  }
}

// ---------------------------------------------------------------------------
// R3: reverse rows, records and faces on the tile core; writes the stage's
// adjoints of U_old and U_E folded into those of U^n and U^(1), and the bed.
// Valid ranges (slots): faces [2, NT-2], records [2, NT-3], rows [3, NT-4],
// row gathers and reverse records [4, NT-5], reverse faces [5, NT-5], cell
// gathers [6, NT-7] (the core).
// ---------------------------------------------------------------------------
template <int NT, int STAGE>
__global__ __launch_bounds__(NT) void k_adj_r3(AdjTileArgs P) {
  using namespace adj;
  __shared__ TileLds3<NT> L;
  const TileA tl = P.tiles[blockIdx.x];
  const InstDesc D = P.inst[tl.inst];
  const double dt = P.dt[tl.inst];
  const int t = threadIdx.x;
  const TC I = make_tc(D, tl.ts - H, dt);
  const int v = I.lo0 + t;
  const bool core = v >= tl.ts && v < tl.te;
  if (!(dt > 0.0)) {  // frozen instance: identity map
    if (core) {
      const int64_t gi = D.off + v;
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        if (STAGE == 2) {
          P.out1[f][gi] = 0.0;
          P.outn[f][gi] = P.abar[f][gi];
        } else {
          P.outn[f][gi] = P.outn[f][gi] + P.abar[f][gi];
        }
      }
    }
    return;
  }
  double E[4] = {0, 0, 0, 0}, O[4] = {0, 0, 0, 0}, aU[4] = {0, 0, 0, 0};
  load_tile<STAGE>(I, L, D.off, v, P.un, P.u1, P.b, P.hbar, P.abar, E, O, aU);
  L.lam[t] = cell_ok(I, v) ? P.lam[D.off + real_cell(I, v)] : 0.0;
  __syncthreads();
  if (t >= 2 && t <= NT - 2 && face_ok(I, v))
    face_flux(I, L, v, L.u.face.fq[t], L.u.face.fm[t], L.u.face.fw[t]);
  __syncthreads();
  Own w;
  const bool rec_ok = t >= 2 && t <= NT - 3 && cell_ok(I, v);
  if (rec_ok) records(I, L, v, E, O, w);
  __syncthreads();  // fluxes are dead
  if (rec_ok) {
    L.phi[t] = w.phi;
    L.tt[t] = w.T;
    rev_back(I, L, v, aU, w);
  }
  __syncthreads();
  // gathers of the back-substitution parts and of the reverse rows (rows
  // j-1, j, j+1 recomputed from lam), then the reverse records
  const bool grec_ok = t >= 4 && t <= NT - 5 && cell_ok(I, v);
  double OA[4] = {0, 0, 0, 0}, EA0[3] = {0, 0, 0}, BAR = 0.0, DbA = 0.0, BAB = 0.0;
  double FLv[3] = {0, 0, 0}, FRv[3] = {0, 0, 0};
  if (grec_ok) {
    double SA0, BETAA0, HBA;
    gather_back(I, L, v, w, SA0, BETAA0, HBA, BAB);
    double bt = BETAA0, st = SA0, qt = w.QDA0, pt = w.PHIA0, tt = w.TA0;
    double bA = 0.0;
#pragma unroll
    for (int d = -1; d <= 1; ++d) {
      const int i = v + d;
      if (!cell_ok(I, i)) continue;
      const RowParts rp = row_parts(I, L, i);
      if (i == v) {
        bt += rp.c[0]; st += rp.c[1]; qt += rp.c[2]; pt += rp.c[3]; tt += rp.c[4];
        bA += rp.dbm - rp.dbp;
      }
      if (vcl(I, i - 1) == v) {
        bt += rp.l[0]; st += rp.l[1]; qt += rp.l[2]; pt += rp.l[3]; tt += rp.l[4];
        bA -= rp.dbm;
      }
      if (vcl(I, i + 1) == v) {
        bt += rp.r[0]; st += rp.r[1]; qt += rp.r[2]; pt += rp.r[3]; tt += rp.r[4];
        bA += rp.dbp;
      }
    }
    BAR = bA;
    const double HOA = L.lam[t];
    // reverse of the coefficients at U_E and of the explicit predictor
    const double h = E[0], m = E[2], q = E[1], md = w.md;
    const Coef c = coefs(I, h, m, md);
    const double lam = I.lam;
    double hA = 0.0, mA = 0.0, ihA = 0.0, ib1A = 0.0, mdA = 0.0;
    const double TA = tt, SA = st;
    double phiA = pt, betaA = bt;
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
    eta0A += -I.lam3 * c.ih * pt0A;
    ihA += -I.lam3 * c.eta0 * pt0A;
    if (I.has_b) {
      const double k = I.lam23;
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
    double ehA = (2.0 * lam * c.eh - I.lam3) * a2A;
    ehA += -(2.0 / 3.0) * c.ih * alphaA;
    ihA += -(2.0 * c.eh - 1.0) * (1.0 / 3.0) * alphaA;
    mA += c.ih * c.ih * ehA;
    ihA += 2.0 * m * c.ih * ehA;
    hA += -c.ih * c.ih * ihA;
    const double mdT = w.MDA + mdA;
    const double tdx = I.tdx;
    OA[2] = mdT;
    FRv[1] = -tdx * mdT;
    FLv[1] = tdx * mdT;
    double qEA = 0.0;
    if (I.has_b) {
      const double Db = (L.bb[slot(I, v + 1)] - L.bb[slot(I, v - 1)]) * I.i2dx;
      qEA = -1.5 * I.tau * Db * mdT;
      DbA = -1.5 * I.tau * q * mdT;
    }
    const double WdT = w.WDA + I.tau * mdT;
    OA[3] = WdT;
    FRv[2] = -tdx * WdT;
    FLv[2] = tdx * WdT;
    const double qdA = qt;
    OA[1] = qdA;
    FRv[0] = -tdx * qdA;
    FLv[0] = tdx * qdA;
    OA[0] = HOA;
    EA0[0] = hA;
    EA0[1] = mA;
    EA0[2] = qEA;
  }
  if (grec_ok) {  // no barrier needed: the union last held fluxes
#pragma unroll
    for (int k = 0; k < 3; ++k) L.u.rface.fr[k][t] = FRv[k];
    L.db2a[t] = DbA;
  }
  __syncthreads();
  // face adjoints and the reverse fluxes
  const bool rf_ok = t >= 5 && t <= NT - 5 && face_ok(I, v);
  double pa[5][4];
#pragma unroll
  for (int fl = 0; fl < 5; ++fl)
#pragma unroll
    for (int k = 0; k < 4; ++k) pa[fl][k] = 0.0;
  if (rf_ok) {
    const int f = v;
    const bool per = I.bc == 0;
    double aq = 0.0, am = 0.0, aw = 0.0;
    if (per || f >= 1) {  // cell left of the face: this is its right face
      const int s = f - 1 - I.lo0;
      aq += L.u.rface.fr[0][s]; am += L.u.rface.fr[1][s]; aw += L.u.rface.fr[2][s];
    }
    if (per || f <= I.n - 1) {  // cell right of the face (this thread's): its left face
      aq += FLv[0]; am += FLv[1]; aw += FLv[2];
    }
    const int cs[4] = {slot(I, f - 2), slot(I, f - 1), slot(I, f), slot(I, f + 1)};
    double h[4], q[4], m[4], wv[4], b[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      h[k] = L.he[cs[k]]; q[k] = L.qe[cs[k]]; m[k] = L.me[cs[k]]; wv[k] = L.we[cs[k]];
      b[k] = L.bb[cs[k]];
    }
    const double hL = h[1] + 0.25 * (h[2] - h[0]), hR = h[2] - 0.25 * (h[3] - h[1]);
    const double qL = q[1] + 0.25 * (q[2] - q[0]), qR = q[2] - 0.25 * (q[3] - q[1]);
    const double mL = m[1] + 0.25 * (m[2] - m[0]), mR = m[2] - 0.25 * (m[3] - m[1]);
    const double WL = wv[1] + 0.25 * (wv[2] - wv[0]), WR = wv[2] - 0.25 * (wv[3] - wv[1]);
    const double ihL = frcp(hL), ihR = frcp(hR);
    const double uL = qL * ihL, uR = qR * ihR;
    const double gsL = fsqrt(I.g * hL), gsR = fsqrt(I.g * hR);
    const double sL = fabs(uL) + gsL, sR = fabs(uR) + gsR;
    const bool leftmax = sL >= sR;
    const double a = leftmax ? sL : sR;
    double rk[4] = {0, 0, 0, 0}, zf = 0.0, jm = mR - mL;
    if (I.has_b) {
      zf = 0.5 * ((h[1] + b[1]) + (h[2] + b[2]));
#pragma unroll
      for (int k = 0; k < 4; ++k) rk[k] = (zf - b[k]) * (zf - b[k]);
      jm -= (rk[2] - 0.25 * (rk[3] - rk[1])) - (rk[1] + 0.25 * (rk[2] - rk[0]));
    }
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
    double hLA = 0.5 * I.g * frcp(gsL) * sLA, hRA = 0.5 * I.g * frcp(gsR) * sRA;
    qLA += uLA * ihL;
    hLA += -uL * ihL * uLA;
    qRA += uRA * ihR;
    hRA += -uR * ihR * uRA;
    const double vLA[4] = {hLA, qLA, mLA, WLA}, vRA[4] = {hRA, qRA, mRA, WRA};
#pragma unroll
    for (int fl = 0; fl < 4; ++fl) {
      pa[fl][0] = -0.25 * vLA[fl];
      pa[fl][1] = vLA[fl] + 0.25 * vRA[fl];
      pa[fl][2] = 0.25 * vLA[fl] + vRA[fl];
      pa[fl][3] = -0.25 * vRA[fl];
    }
    if (I.has_b) {
      const double rA[4] = {-0.25 * mhLA, mhLA + 0.25 * mhRA, 0.25 * mhLA + mhRA, -0.25 * mhRA};
      double zfA = 0.0;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        zfA += 2.0 * (zf - b[k]) * rA[k];
        pa[4][k] += -2.0 * (zf - b[k]) * rA[k];
      }
      pa[0][1] += 0.5 * zfA;
      pa[0][2] += 0.5 * zfA;
      pa[4][1] += 0.5 * zfA;
      pa[4][2] += 0.5 * zfA;
    }
  }
  // gather of the face partials on the core, one stencil position k at a
  // time (cell j takes position k of the faces f with f - 2 + k -> j)
  const int j = v;
  double ea[5] = {EA0[0], EA0[2], EA0[1], 0.0, 0.0};  // h, q, m, W, b
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    // the previous round is read; before round 0, the reverse faces have
    // read the staged tile, whose storage pf takes over
    __syncthreads();
    if (rf_ok) {
#pragma unroll
      for (int fl = 0; fl < 5; ++fl) L.pf[fl][t] = pa[fl][k];
    }
    __syncthreads();
    if (core) {
#pragma unroll
      for (int d = -1; d <= 2; ++d) {
        const int f = j + d;
        if (!face_ok(I, f) || vcl(I, f - 2 + k) != j) continue;
        const int s = f - I.lo0;
#pragma unroll
        for (int fl = 0; fl < 5; ++fl) ea[fl] += L.pf[fl][s];
      }
    }
  }
  if (core) {
    double bA = BAB + BAR + ea[4];
    if (I.has_b) {
#pragma unroll
      for (int d = -1; d <= 1; ++d) {
        const int i = j + d;
        if (!cell_ok(I, i)) continue;
        const int s = i - I.lo0;
        if (vcl(I, i + 1) == j) bA += L.db2a[s] * I.i2dx;
        if (vcl(I, i - 1) == j) bA -= L.db2a[s] * I.i2dx;
      }
    }
    const int64_t gi = D.off + j;
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      if (STAGE == 2) {
        P.out1[f][gi] = kE1 * ea[f] + kT1 * OA[f];
        P.outn[f][gi] = kE0 * ea[f] + kT0 * OA[f];
      } else {
        P.outn[f][gi] = P.outn[f][gi] + ea[f] + OA[f];
      }
    }
    if (P.gb && I.has_b) P.gb[gi] += bA;
  }
}

// ---------------------------------------------------------------------------
// R2: tridiagonal solve of one system of M rows held in global arrays, by
// one workgroup (chunked Thomas in global scratch + level-1 PCR in LDS;
// cyclic couplings handled by the two end rows).  All threads call it.
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
  // The chunk's rows are read (and its scratch rows written back) in blocks
  // of B rows whose loads are issued together: one memory latency per block
  // instead of one per row of the recurrence.
  constexpr int B = 8;
  if (act) {
    double cprev = 0.0, yprev = 0.0, vprev = 1.0, wprev = 0.0;
    for (int i0 = 1; i0 <= k - 2; i0 += B) {
      double L[B], D[B], U[B], R[B];
#pragma unroll
      for (int b = 0; b < B; ++b) {
        const int i = i0 + b <= k - 2 ? i0 + b : k - 2;
        L[b] = lo[f + i];
        D[b] = di[f + i];
        U[b] = up[f + i];
        R[b] = rhs[f + i];
      }
#pragma unroll
      for (int b = 0; b < B; ++b) {
        const int i = i0 + b;
        if (i <= k - 2) {
          const double l = L[b], d = D[b], u = U[b], r = R[b];
          const double inv = frcp(d - l * cprev);
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
      }
    }
    double yn = 0.0, vn = 0.0, wn = 0.0;
    for (int i1 = k - 2; i1 >= 1; i1 -= B) {
      double Cc[B], Y[B], V[B], W[B];
#pragma unroll
      for (int b = 0; b < B; ++b) {
        const int i = i1 - b >= 1 ? i1 - b : 1;
        Cc[b] = scp[f + i];
        Y[b] = sy[f + i];
        V[b] = sv[f + i];
        W[b] = sw[f + i];
      }
#pragma unroll
      for (int b = 0; b < B; ++b) {
        const int i = i1 - b;
        if (i >= 1) {
          const double c = Cc[b];
          yn = Y[b] - c * yn;
          vn = V[b] - c * vn;
          wn = W[b] - c * wn;
          sy[f + i] = yn;
          sv[f + i] = vn;
          sw[f + i] = wn;
        }
      }
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
    for (int i0 = 1; i0 <= k - 2; i0 += B) {
      double Y[B], V[B], W[B];
#pragma unroll
      for (int b = 0; b < B; ++b) {
        const int i = i0 + b <= k - 2 ? i0 + b : k - 2;
        Y[b] = sy[f + i];
        V[b] = sv[f + i];
        W[b] = sw[f + i];
      }
#pragma unroll
      for (int b = 0; b < B; ++b)
        if (i0 + b <= k - 2) x[f + i0 + b] = Y[b] + V[b] * zf + W[b] * zb;
    }
  }
  __syncthreads();
}

struct AdjSolveArgs {
  const InstDesc* inst;
  const double* dt;
  const double* lot;
  const double* dit;
  const double* upt;
  const double* hba;
  double* lam;
  double* scp;
  double* sy;
  double* sv;
  double* sw;
};

// Register-resident chunk elimination of n <= NT * K rows (a whole system or
// one tile of it): each thread eliminates its chunk (consecutive rows) into
// two rows of the level-1 system in LDS,
// keeping the chunk's interior spikes (y, v, w) in registers.  All threads
// call it; the caller synchronises before the level-1 solve.
//
// The rows come from rows(f, k, Lo, Di, Up, Rh), which fills the K rows of
// the chunk of k rows starting at row f (rows k .. K - 1 repeat row k - 1).
template <int NT, int K, class Rows>
__device__ __forceinline__ Chunk reg_chunk_elim_rows(Lds<NT>& S, int n, double (&y)[K],
                                                     double (&v)[K], double (&w)[K], Rows rows) {
  const int t = threadIdx.x;
  const Chunk ch = chunk_of(n, NT, t);
  const int k = ch.k;  // 2 <= k <= K for active threads
  const int f = ch.first;
  if (t < ch.active) {
    double Lo[K], Di[K], Up[K], Rh[K];
    rows(f, k, Lo, Di, Up, Rh);

    double cp[K];
    double cprev = 0.0, yprev = 0.0, vprev = 1.0, wprev = 0.0;
#pragma unroll
    for (int i = 1; i < K - 1; ++i) {
      if (i <= k - 2) {
        const double l = Lo[i], d = Di[i], u = Up[i], r = Rh[i];
        const double inv = frcp(d - l * cprev);
        const bool lastint = (i == k - 2);
        cprev = lastint ? 0.0 : u * inv;
        yprev = (r - l * yprev) * inv;
        vprev = (-l * vprev) * inv;
        wprev = (-l * wprev) * inv - (lastint ? u * inv : 0.0);
        cp[i] = cprev;
        y[i] = yprev;
        v[i] = vprev;
        w[i] = wprev;
      }
    }
    double yn = 0.0, vn = 0.0, wn = 0.0;
#pragma unroll
    for (int i = K - 2; i >= 1; --i) {
      if (i <= k - 2) {
        const double c = cp[i];
        yn = y[i] - c * yn;
        vn = v[i] - c * vn;
        wn = w[i] - c * wn;
        y[i] = yn;
        v[i] = vn;
        w[i] = wn;
      }
    }
    double R0[4] = {Lo[0], Di[0], Up[0], Rh[0]};
    double R1[4] = {Lo[K - 1], Di[K - 1], Up[K - 1], Rh[K - 1]};  // row k-1 (clamped)
    if (k > 2) {
      double vk = 0.0, wk = 0.0, yk = 0.0;
#pragma unroll
      for (int i = 1; i < K - 1; ++i) {
        if (i == k - 2) { vk = v[i]; wk = w[i]; yk = y[i]; }
      }
      R0[1] = R0[1] + R0[2] * v[1];
      R0[3] = R0[3] - R0[2] * y[1];
      R0[2] = R0[2] * w[1];
      R1[1] = R1[1] + R1[0] * wk;
      R1[3] = R1[3] - R1[0] * yk;
      R1[0] = R1[0] * vk;
    }
    S.a[2 * t] = R0[0]; S.b[2 * t] = R0[1]; S.c[2 * t] = R0[2]; S.d0[2 * t] = R0[3];
    S.d1[2 * t] = 0.0; S.d2[2 * t] = 0.0;
    S.a[2 * t + 1] = R1[0]; S.b[2 * t + 1] = R1[1]; S.c[2 * t + 1] = R1[2];
    S.d0[2 * t + 1] = R1[3]; S.d1[2 * t + 1] = 0.0; S.d2[2 * t + 1] = 0.0;
  }
  return ch;
}

// The same with the rows read from global arrays lo, di, up, rhs.
template <int NT, int K>
__device__ __forceinline__ Chunk reg_chunk_elim(Lds<NT>& S, const double* __restrict__ lo,
                                                const double* __restrict__ di,
                                                const double* __restrict__ up,
                                                const double* __restrict__ rhs, int n,
                                                double (&y)[K], double (&v)[K], double (&w)[K]) {
  return reg_chunk_elim_rows<NT, K>(
      S, n, y, v, w,
      [&](int f, int k, double (&Lo)[K], double (&Di)[K], double (&Up)[K], double (&Rh)[K]) {
        // every row of the chunk is loaded before the elimination starts
        // (the K loads of one lane share cache lines; issued together they
        // are served by one fetch)
        if (k == K && K % 2 == 0) {
          // a full chunk: two rows per 16-byte load (8-byte alignment
          // suffices for global memory on this target; measured: transposed
          // solve of the gradient -9 %, SGN solve -10 %)
          typedef double d2a8 __attribute__((ext_vector_type(2), aligned(8)));
#pragma unroll
          for (int i = 0; i < K; i += 2) {
            const d2a8 a = *(const d2a8*)(lo + f + i);
            const d2a8 b = *(const d2a8*)(di + f + i);
            const d2a8 c = *(const d2a8*)(up + f + i);
            const d2a8 d = *(const d2a8*)(rhs + f + i);
            Lo[i] = a.x; Lo[i + 1] = a.y;
            Di[i] = b.x; Di[i + 1] = b.y;
            Up[i] = c.x; Up[i + 1] = c.y;
            Rh[i] = d.x; Rh[i + 1] = d.y;
          }
        } else {
#pragma unroll
          for (int i = 0; i < K; ++i) {
            const int r = f + (i < k ? i : k - 1);
            Lo[i] = lo[r];
            Di[i] = di[r];
            Up[i] = up[r];
            Rh[i] = rhs[r];
          }
        }
      });
}

// Level-1 system of a whole system that is not cyclic (the first row's lower
// and the last row's upper coupling are zero): parallel cyclic reduction of
// all n1 rows with one right-hand side, stopped once every coupling is below
// 2^-66 of its diagonal (as the interior solve); on exit S.d0[j] holds z_j.
// It replaces the interior solve with its two spike columns and the 2x2 end
// solve where no spike is needed.  All threads call it.
template <int NT>
__device__ void level1_full(Lds<NT>& S, int n1) {
  const int t = threadIdx.x;
  for (int s = 1; s < n1; s <<= 1) {
    double na[2], nb[2], nc[2], nd[2];
    bool own[2];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int j = t + r * NT;
      own[r] = j < n1;
      if (own[r]) {
        const int jm = j - s, jp = j + s;
        const bool hm = jm >= 0, hp = jp < n1;
        const double a = S.a[j], c = S.c[j];
        const double k1 = hm ? a * frcp(S.b[jm]) : 0.0;
        const double k2 = hp ? c * frcp(S.b[jp]) : 0.0;
        na[r] = hm ? -k1 * S.a[jm] : 0.0;
        nc[r] = hp ? -k2 * S.c[jp] : 0.0;
        double bb = S.b[j], dd = S.d0[j];
        if (hm) {
          bb -= k1 * S.c[jm];
          dd -= k1 * S.d0[jm];
        }
        if (hp) {
          bb -= k2 * S.a[jp];
          dd -= k2 * S.d0[jp];
        }
        nb[r] = bb;
        nd[r] = dd;
      }
    }
    __syncthreads();
    bool more = false;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int j = t + r * NT;
      if (own[r]) {
        S.a[j] = na[r];
        S.b[j] = nb[r];
        S.c[j] = nc[r];
        S.d0[j] = nd[r];
        const double lim = 1.3552527156068805e-20 * fabs(nb[r]);  // 2^-66
        more |= !(fabs(na[r]) <= lim) || !(fabs(nc[r]) <= lim);
      }
    }
    if (!__syncthreads_or(more)) break;
  }
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int j = t + r * NT;
    if (j < n1) S.d0[j] *= frcp(S.b[j]);
  }
  __syncthreads();
}

// Unknowns of a thread's chunk from the system's end values z0, zl (after
// the level-1 solve): chunk ends from the level-1 spikes, interiors from
// the chunk spikes.  FULL: the level-1 solve was level1_full, whose d0
// holds the chunk ends themselves (z0 and zl are not used).
template <int NT, int K, bool FULL = false>
__device__ __forceinline__ void reg_chunk_write(const Lds<NT>& S, const Chunk& ch,
                                                double* __restrict__ x, double z0, double zl,
                                                const double (&y)[K], const double (&v)[K],
                                                const double (&w)[K]) {
  const int t = threadIdx.x;
  if (t >= ch.active) return;
  const int k = ch.k, f = ch.first;
  const int n1 = 2 * ch.active;
  const int j0 = 2 * t, j1 = 2 * t + 1;
  const double zf = FULL ? S.d0[j0]
                         : ((j0 == 0) ? z0 : S.d0[j0] + S.d1[j0] * z0 + S.d2[j0] * zl);
  const double zb = FULL ? S.d0[j1]
                         : ((j1 == n1 - 1) ? zl : S.d0[j1] + S.d1[j1] * z0 + S.d2[j1] * zl);
  if (k == K && K % 2 == 0) {
    // a full chunk: two rows per 16-byte store
    typedef double d2a8 __attribute__((ext_vector_type(2), aligned(8)));
    double xr[K];
    xr[0] = zf;
    xr[K - 1] = zb;
#pragma unroll
    for (int i = 1; i < K - 1; ++i) xr[i] = y[i] + v[i] * zf + w[i] * zb;
#pragma unroll
    for (int i = 0; i < K; i += 2) {
      d2a8 a;
      a.x = xr[i];
      a.y = xr[i + 1];
      *(d2a8*)(x + f + i) = a;
    }
    return;
  }
  x[f] = zf;
  x[f + k - 1] = zb;
#pragma unroll
  for (int i = 1; i < K - 1; ++i)
    if (i <= k - 2) x[f + i] = y[i] + v[i] * zf + w[i] * zb;
}

// Register-resident solve of one instance of n <= NT * K rows (chunks in
// registers, level-1 PCR in LDS stopping once every coupling is below 2^-66
// of its diagonal, 2x2 end solve, cyclic when periodic).  Longer instances
// use the global-scratch solve.
template <int NT, int K>
__global__ __launch_bounds__(NT) void k_adj_r2(AdjSolveArgs P) {
  __shared__ Lds<NT> S;
  const InstDesc D = P.inst[blockIdx.x];
  if (!(P.dt[blockIdx.x] > 0.0)) return;  // frozen: lam is not used
  const int64_t o = D.off;
  const int n = D.n;
  const bool cyclic = D.bc == 0;
  if (n > NT * K) {
    wg_tri_solve<NT>(S, P.lot + o, P.dit + o, P.upt + o, P.hba + o, P.lam + o, n, cyclic,
                     P.scp + o, P.sy + o, P.sv + o, P.sw + o);
    return;
  }
  double y[K], v[K], w[K];
  const Chunk ch = reg_chunk_elim<NT, K>(S, P.lot + o, P.dit + o, P.upt + o, P.hba + o, n, y, v, w);
  __syncthreads();
  if (!cyclic) {  // no spikes needed: one right-hand side over all level-1 rows
    level1_full<NT>(S, 2 * ch.active);
    reg_chunk_write<NT, K, true>(S, ch, P.lam + o, 0.0, 0.0, y, v, w);
    return;
  }
  level1_interior_fast<NT>(S, 2 * ch.active);
  if (threadIdx.x == 0) {
    double R0[4], R1[4], z0, zl;
    tile_rows<NT>(S, 2 * ch.active, R0, R1);
    if (!cyclic) {
      R0[0] = 0.0;
      R1[2] = 0.0;
    }
    solve_ends(R0, R1, cyclic, z0, zl);
    S.s[0] = z0;
    S.s[1] = zl;
  }
  __syncthreads();
  reg_chunk_write<NT, K>(S, ch, P.lam + o, S.s[0], S.s[1], y, v, w);
}

}  // namespace hsgn
