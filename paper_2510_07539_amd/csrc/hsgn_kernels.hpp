// hsgn_kernels.hpp -- device code of the gfx950 hSGN IMEX step.
//
// One workgroup handles one tile: a contiguous run of at most NT*KMAX cells
// of one instance.  Each thread owns a chunk of 2..KMAX consecutive cells and
// keeps everything it computes for them in registers:
//
//   1. explicit sweep (Sec. 4.1 reconstruction + Rusanov fluxes; Sec. 4.2
//      dagger updates; exact relaxation elimination, Sec. 3.1 eq. b1) and the
//      frozen coefficients beta, P0 (Sec. 2.2 eq. hSGN_px, Sec. 4.2);
//   2. the rows of the linear system for the new depth (Sec. 3.1 eq. hnew,
//      differenced in conservative pressure form, bed terms implicit);
//   3. a two-level partition solve: every thread eliminates the interior of
//      its chunk (Thomas on the chunk with two coupling columns), the 2*NT
//      chunk-boundary unknowns form a tridiagonal system that parallel cyclic
//      reduction solves in LDS with three right-hand sides, which leaves the
//      tile reduced to two rows in its first and last unknowns;
//   4. those two rows are either solved on the spot (instance = one tile;
//      cyclic if periodic) or written out for a per-instance reduced solve
//      across tiles, after which a second pass recomputes 1-3 and finishes;
//   5. back-substitution (Sec. 4.2 last three lines) and the stage output.
//
// The arithmetic follows the paper's formulas; only the solver's elimination
// order differs from a sequential Thomas solve.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hsgn {

// Double Butcher tableau of Sec. 3.2: gamma = 1 - 1/sqrt(2), c = 1/(2 gamma).
// Efficient form: U_E^(2) = (1 - c/gamma) U^n + (c/gamma) U^(1),
//                 U~      = (1 - (1-gamma)/gamma) U^n + ((1-gamma)/gamma) U^(1).
constexpr double kGamma = 0.29289321881345247560;
constexpr double kE0 = -4.82842712474619009760;  // 1 - c/gamma = -2 - 2 sqrt 2
constexpr double kE1 = 5.82842712474619009760;   // c/gamma = 3 + 2 sqrt 2
constexpr double kT0 = -1.41421356237309504880;  // 1 - (1-gamma)/gamma = -sqrt 2
constexpr double kT1 = 2.41421356237309504880;   // (1-gamma)/gamma = 1 + sqrt 2

constexpr int32_t kFlagNonPhys = 1;
constexpr int32_t kFlagNonCoercive = 2;

struct InstDesc {
  int64_t off;       // first cell in the concatenated arrays
  int32_t n;         // cells
  int32_t bc;        // 0 periodic, 1 transmissive
  int32_t has_b;     // bed used
  int32_t ntiles;    // tiles of this instance
  int32_t red_off;   // first reduced row (2 per tile), -1 for one tile
  int32_t pad;
  double g, lam, dx, cfl, mcfl, dt_fixed, t_end;
};

struct TileDesc {
  int32_t inst;   // instance
  int32_t tidx;   // tile index within the instance
  int32_t start;  // first cell, relative to the instance
  int32_t len;    // cells
};

struct StageArgs {
  const double* __restrict__ un_h;
  const double* __restrict__ un_q;
  const double* __restrict__ un_m;
  const double* __restrict__ un_W;
  const double* __restrict__ u1_h;  // stage 2 only
  const double* __restrict__ u1_q;
  const double* __restrict__ u1_m;
  const double* __restrict__ u1_W;
  double* __restrict__ o_h;
  double* __restrict__ o_q;
  double* __restrict__ o_m;
  double* __restrict__ o_W;
  const double* __restrict__ b;
  const InstDesc* __restrict__ inst;
  const TileDesc* __restrict__ tiles;
  const double* __restrict__ dt;
  double* __restrict__ rlo;  // reduced rows (written by the reduce pass)
  double* __restrict__ rdi;
  double* __restrict__ rup;
  double* __restrict__ rrhs;
  const double* __restrict__ rx;  // reduced solution (read by the finish pass)
  double tau_factor;  // stage step tau = tau_factor dt (gamma for the IMEX step, 1 first order)
  double slope;       // reconstruction slope factor (1/4, or 0 first order)
  unsigned long long* __restrict__ smax;  // stage-2 speed bound accumulators
  unsigned long long* __restrict__ umax;
  int32_t* __restrict__ status;
};

struct Cell {
  double h, q, m, W;
};

// Per-cell results of the explicit sweep that the rows and the
// back-substitution need.
struct Rec {
  double qd, md, Wd;  // q-dagger, m-dagger, W-dagger
  double beta, S;     // P = S + beta * hbar (linearised pressure)
  double phi, T;      // p~ = T + phi * hbar (bed only)
  double b;           // bed
};

struct Flux {
  double q, m, W;
};

__device__ __forceinline__ int wrap_idx(int i, int n, int bc) {
  if (bc == 0) {
    if (i < 0) i += n;
    else if (i >= n) i -= n;
    return i;
  }
  return i < 0 ? 0 : (i > n - 1 ? n - 1 : i);
}

template <int STAGE>
__device__ __forceinline__ Cell load_E(const StageArgs& A, int64_t gi) {
  Cell c;
  if (STAGE == 1) {
    c.h = A.un_h[gi];
    c.q = A.un_q[gi];
    c.m = A.un_m[gi];
    c.W = A.un_W[gi];
  } else {
    c.h = kE0 * A.un_h[gi] + kE1 * A.u1_h[gi];
    c.q = kE0 * A.un_q[gi] + kE1 * A.u1_q[gi];
    c.m = kE0 * A.un_m[gi] + kE1 * A.u1_m[gi];
    c.W = kE0 * A.un_W[gi] + kE1 * A.u1_W[gi];
  }
  return c;
}

template <int STAGE>
__device__ __forceinline__ Cell load_old(const StageArgs& A, int64_t gi) {
  Cell c;
  if (STAGE == 1) {
    c.h = A.un_h[gi];
    c.q = A.un_q[gi];
    c.m = A.un_m[gi];
    c.W = A.un_W[gi];
  } else {
    c.h = kT0 * A.un_h[gi] + kT1 * A.u1_h[gi];
    c.q = kT0 * A.un_q[gi] + kT1 * A.u1_q[gi];
    c.m = kT0 * A.un_m[gi] + kT1 * A.u1_m[gi];
    c.W = kT0 * A.un_W[gi] + kT1 * A.u1_W[gi];
  }
  return c;
}

// Rusanov flux at the face between cells c0 and c1 from the unlimited
// component-wise linear reconstruction (slope (v_{i+1} - v_{i-1}) / (2 dx)):
// face values v_i +/- sl (v_{i+1} - v_{i-1}) with sl = 1/4, or sl = 0 for
// the first-order scheme (cell values).
// The m-diffusion subtracts the jump of the face-local lake-at-rest moment
// (zeta_f - b_j)^2, zeta_f = mean free surface of the two face cells.
template <bool BED>
__device__ __forceinline__ Flux face_flux(const Cell& cm, const Cell& c0, const Cell& c1,
                                          const Cell& c2, double bm, double b0, double b1,
                                          double b2, double g, double sl, bool& bad) {
  const double hL = c0.h + sl * (c1.h - cm.h);
  const double hR = c1.h - sl * (c2.h - c0.h);
  const double qL = c0.q + sl * (c1.q - cm.q);
  const double qR = c1.q - sl * (c2.q - c0.q);
  const double mL = c0.m + sl * (c1.m - cm.m);
  const double mR = c1.m - sl * (c2.m - c0.m);
  const double WL = c0.W + sl * (c1.W - cm.W);
  const double WR = c1.W - sl * (c2.W - c0.W);
  bad |= !(hL > 0.0) || !(hR > 0.0);
  const double uL = qL / hL;
  const double uR = qR / hR;
  const double sL = fabs(uL) + sqrt(g * hL);
  const double sR = fabs(uR) + sqrt(g * hR);
  const double a = fmax(sL, sR);
  double jm = mR - mL;
  if (BED) {
    const double zf = 0.5 * ((c0.h + b0) + (c1.h + b1));
    const double rm = (zf - bm) * (zf - bm);
    const double r0 = (zf - b0) * (zf - b0);
    const double r1 = (zf - b1) * (zf - b1);
    const double r2 = (zf - b2) * (zf - b2);
    const double mhL = r0 + sl * (r1 - rm);
    const double mhR = r1 - sl * (r2 - r0);
    jm = jm - (mhR - mhL);
  }
  Flux F;
  F.q = 0.5 * (qL * uL + qR * uR - a * (qR - qL));
  F.m = 0.5 * (mL * uL + mR * uR - a * jm);
  F.W = 0.5 * (WL * uL + WR * uR - a * (WR - WL));
  return F;
}

struct PhysC {
  double g, lam, dx, tau, tdx, lt2, rr, tdx2;
  double sl;  // reconstruction slope factor (1/4, or 0 for the first-order scheme)
  double lam3, lam23;  // lambda/3 and 2 lambda/3 (set by the window kernel only)
};

// Dagger updates (Sec. 4.2, first three lines, with tau for dt) and frozen
// coefficients at U_E: eta = m/h, alpha = -(2 eta/h - 1)/(3 h),
// a^2 = g h + lambda (eta/h)^2 - (lambda/3) eta/h  (= c^2 - lambda eta alpha),
// beta_1 = 1 + lambda tau^2/h^2, beta_2 = 2 lambda tau^2/(beta_1^2 h^3),
// beta = a^2 + lambda alpha beta_2 m-dagger; P0 = p(h_E, m-dagger/beta_1);
// S = P0 - beta h_E; bed: phi = d p~/dh, T = p~(h_E) - phi h_E.
template <bool BED>
__device__ __forceinline__ Rec cell_record(const Cell& e, const Cell& o, const Flux& Fl,
                                           const Flux& Fr, double bm, double bc, double bp,
                                           const PhysC& P, bool& bad, bool& noncoer) {
  Rec r;
  r.Wd = o.W - P.tdx * (Fr.W - Fl.W) + P.lam * P.tau;
  double md = o.m - P.tdx * (Fr.m - Fl.m);
  if (BED) md -= P.tau * 1.5 * e.q * (bp - bm) / (2.0 * P.dx);
  md += P.tau * r.Wd;
  r.md = md;
  r.qd = o.q - P.tdx * (Fr.q - Fl.q);
  const double h = e.h;
  bad |= !(h > 0.0);
  const double ih = 1.0 / h;
  const double eh = e.m * ih * ih;  // eta / h
  const double alpha = -(2.0 * eh - 1.0) * ih * (1.0 / 3.0);
  const double a2 = P.g * h + P.lam * eh * eh - (P.lam / 3.0) * eh;
  const double b1 = 1.0 + P.lt2 * ih * ih;
  const double ib1 = 1.0 / b1;
  const double b2 = 2.0 * P.lt2 * ib1 * ib1 * ih * ih * ih;
  r.beta = a2 + P.lam * alpha * b2 * md;
  noncoer |= !(r.beta > 0.0);
  const double eta0 = md * ib1 * ih;
  const double pt0 = (P.lam / 3.0) * (1.0 - eta0 * ih);
  const double P0 = 0.5 * P.g * h * h + eta0 * pt0;
  r.S = P0 - r.beta * h;
  if (BED) {
    r.phi = (2.0 * P.lam / 3.0) * md * ih * ih * ih * ib1 * ib1;
    r.T = pt0 - r.phi * h;
  } else {
    r.phi = 0.0;
    r.T = 0.0;
  }
  r.b = bc;
  return r;
}

// Row of the depth system at cell C with neighbours L and R:
// hbar_i - tau^2/dx (G_{i+1/2} - G_{i-1/2}) = h_old - tau/(2 dx)(qd_{i+1} - qd_{i-1}),
// G the face force of the linearised pressure and bed terms.
template <bool BED>
__device__ __forceinline__ void make_row(const Rec& L, const Rec& C, const Rec& R, double ho,
                                         const PhysC& P, double& lo, double& di, double& up,
                                         double& rhs) {
  if (BED) {
    const double hg = 0.5 * P.g;
    const double dbm = C.b - L.b;
    const double dbp = R.b - C.b;
    const double eL = hg + 0.75 * L.phi;
    const double eC = hg + 0.75 * C.phi;
    const double eR = hg + 0.75 * R.phi;
    lo = -P.rr * (L.beta - dbm * eL);
    up = -P.rr * (R.beta + dbp * eR);
    di = 1.0 + P.rr * (2.0 * C.beta - (dbp - dbm) * eC);
    rhs = ho - P.tdx2 * (R.qd - L.qd) +
          P.rr * ((R.S - C.S) - (C.S - L.S) + 0.75 * (dbp * (C.T + R.T) - dbm * (L.T + C.T)));
  } else {
    lo = -P.rr * L.beta;
    up = -P.rr * R.beta;
    di = 1.0 + 2.0 * P.rr * C.beta;
    rhs = ho - P.tdx2 * (R.qd - L.qd) + P.rr * ((R.S - C.S) - (C.S - L.S));
  }
}

template <bool BED>
__device__ __forceinline__ double loadb(const StageArgs& A, bool useb, int64_t gi) {
  if (!BED) return 0.0;
  return useb ? A.b[gi] : 0.0;
}

// Record of one cell, with its own two faces (used for the tile's outer
// neighbours).
template <bool BED, int STAGE>
__device__ Rec single_record(const StageArgs& A, int64_t base, int n, int bc, bool useb, int ir,
                             const PhysC& P, bool& bad, bool& noncoer) {
  Cell c[5];
  double bb[5];
#pragma unroll
  for (int d = 0; d < 5; ++d) {
    const int jj = wrap_idx(ir - 2 + d, n, bc);
    c[d] = load_E<STAGE>(A, base + jj);
    bb[d] = loadb<BED>(A, useb, base + jj);
  }
  const Flux Fl = face_flux<BED>(c[0], c[1], c[2], c[3], bb[0], bb[1], bb[2], bb[3], P.g, P.sl, bad);
  const Flux Fr = face_flux<BED>(c[1], c[2], c[3], c[4], bb[1], bb[2], bb[3], bb[4], P.g, P.sl, bad);
  const Cell o = load_old<STAGE>(A, base + wrap_idx(ir, n, bc));
  return cell_record<BED>(c[2], o, Fl, Fr, bb[1], bb[2], bb[3], P, bad, noncoer);
}

// ---------------------------------------------------------------------------
// Level-1 (chunk-boundary) system in LDS: rows z_0..z_{n1-1}.
// ---------------------------------------------------------------------------
template <int NT>
struct Lds {
  double a[2 * NT], b[2 * NT], c[2 * NT], d0[2 * NT], d1[2 * NT], d2[2 * NT];
  double s[8];  // broadcast scalars
};

// Solve the interior rows 1..n1-2 for three right-hand sides by parallel
// cyclic reduction: d0 = rhs, d1 = coupling to z_0, d2 = coupling to
// z_{n1-1}.  On exit d0, d1, d2 hold Y, V, W with
// z_j = Y_j + V_j z_0 + W_j z_{n1-1}.  All threads must call it.
template <int NT>
__device__ void level1_interior(Lds<NT>& S, int n1) {
  const int t = threadIdx.x;
  const int last = n1 - 2;  // last interior row
  const int m = n1 - 2;
  if (m <= 0) return;
  if (t == 0) {
    S.d1[1] = -S.a[1];
    S.a[1] = 0.0;
    S.d2[last] = -S.c[last];
    S.c[last] = 0.0;
  }
  __syncthreads();
  for (int s = 1; s < m; s <<= 1) {
    double na[2], nb[2], nc[2], n0[2], n1v[2], n2[2];
    bool own[2];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int j = 1 + t + r * NT;
      own[r] = j <= last;
      if (own[r]) {
        const int jm = j - s, jp = j + s;
        const bool hm = jm >= 1, hp = jp <= last;
        const double a = S.a[j], b = S.b[j], c = S.c[j];
        const double k1 = hm ? a / S.b[jm] : 0.0;
        const double k2 = hp ? c / S.b[jp] : 0.0;
        na[r] = hm ? -k1 * S.a[jm] : 0.0;
        nc[r] = hp ? -k2 * S.c[jp] : 0.0;
        double bb = b;
        double e0 = S.d0[j], e1 = S.d1[j], e2 = S.d2[j];
        if (hm) {
          bb -= k1 * S.c[jm];
          e0 -= k1 * S.d0[jm];
          e1 -= k1 * S.d1[jm];
          e2 -= k1 * S.d2[jm];
        }
        if (hp) {
          bb -= k2 * S.a[jp];
          e0 -= k2 * S.d0[jp];
          e1 -= k2 * S.d1[jp];
          e2 -= k2 * S.d2[jp];
        }
        nb[r] = bb;
        n0[r] = e0;
        n1v[r] = e1;
        n2[r] = e2;
      }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int j = 1 + t + r * NT;
      if (own[r]) {
        S.a[j] = na[r];
        S.b[j] = nb[r];
        S.c[j] = nc[r];
        S.d0[j] = n0[r];
        S.d1[j] = n1v[r];
        S.d2[j] = n2[r];
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int j = 1 + t + r * NT;
    if (j <= last) {
      const double ib = 1.0 / S.b[j];
      S.d0[j] *= ib;
      S.d1[j] *= ib;
      S.d2[j] *= ib;
    }
  }
  __syncthreads();
}

// The tile's two reduced rows (first and last unknown), from the level-1
// system after level1_interior.  Only thread 0 calls it.
template <int NT>
__device__ __forceinline__ void tile_rows(const Lds<NT>& S, int n1, double R0[4], double R1[4]) {
  const int l = n1 - 1;
  if (n1 == 2) {
    R0[0] = S.a[0]; R0[1] = S.b[0]; R0[2] = S.c[0]; R0[3] = S.d0[0];
    R1[0] = S.a[1]; R1[1] = S.b[1]; R1[2] = S.c[1]; R1[3] = S.d0[1];
    return;
  }
  R0[0] = S.a[0];
  R0[1] = S.b[0] + S.c[0] * S.d1[1];
  R0[2] = S.c[0] * S.d2[1];
  R0[3] = S.d0[0] - S.c[0] * S.d0[1];
  R1[0] = S.a[l] * S.d1[l - 1];
  R1[1] = S.b[l] + S.a[l] * S.d2[l - 1];
  R1[2] = S.c[l];
  R1[3] = S.d0[l] - S.a[l] * S.d0[l - 1];
}

// 2x2 system of a tile that is a whole instance (cyclic couplings folded).
__device__ __forceinline__ void solve_ends(const double R0[4], const double R1[4], bool periodic,
                                          double& z0, double& zl) {
  double m00 = R0[1], m01 = R0[2], m10 = R1[0], m11 = R1[1];
  if (periodic) {
    m01 += R0[0];
    m10 += R1[2];
  }
  const double det = m00 * m11 - m01 * m10;
  z0 = (R0[3] * m11 - m01 * R1[3]) / det;
  zl = (m00 * R1[3] - m10 * R0[3]) / det;
}

// Chunk distribution: `active` threads own 2..KMAX consecutive rows each.
struct Chunk {
  int active, k, first;
};
__device__ __forceinline__ Chunk chunk_of(int n_t, int NT, int t) {
  int active = n_t / 2;
  if (active > NT) active = NT;
  if (active < 1) active = 1;
  const int base = n_t / active;
  const int rem = n_t - base * active;
  Chunk c;
  c.active = active;
  c.k = t < active ? base + (t < rem ? 1 : 0) : 0;
  c.first = t * base + (t < rem ? t : rem);
  return c;
}

// ---------------------------------------------------------------------------
// The stage kernel.  REDUCE: write the tile's two reduced rows and stop.
// Otherwise: tile = whole instance (solve its ends here) or one of several
// tiles (ends come from the reduced solve), then back-substitute and store.
// ---------------------------------------------------------------------------
// The finishing pass of stage 1 runs at two workgroups per CU (at most 256
// registers; left to itself the compiler takes up to 302 and one): measured
// 25 % faster with a bed.  The other variants measured slower so bounded
// (stage 2's finishing pass spills), and keep the compiler's choice.
template <int NT, int KMAX, bool BED, int STAGE, bool REDUCE>
__global__ __launch_bounds__(NT, (STAGE == 1 && !REDUCE) ? 2 : 1) void k_stage(StageArgs A) {
  __shared__ Lds<NT> S;
  __shared__ double nb_beta[2][NT], nb_S[2][NT], nb_qd[2][NT], nb_phi[2][NT], nb_T[2][NT],
      nb_b[2][NT];

  const TileDesc td = A.tiles[blockIdx.x];
  const InstDesc I = A.inst[td.inst];
  const double dt = A.dt[td.inst];
  const int t = threadIdx.x;
  const int n = I.n, bc = I.bc;
  const int64_t base = I.off;
  const Chunk ch = chunk_of(td.len, NT, t);
  const int k = ch.k;
  const int c0 = td.start + ch.first;  // instance-relative first cell of the chunk
  const bool act = t < ch.active;

  if (!(dt > 0.0)) {  // frozen instance: state unchanged
    if (!REDUCE && act) {
#pragma unroll
      for (int j = 0; j < KMAX; ++j) {
        if (j < k) {
          const int64_t gi = base + c0 + j;
          A.o_h[gi] = A.un_h[gi];
          A.o_q[gi] = A.un_q[gi];
          A.o_m[gi] = A.un_m[gi];
          A.o_W[gi] = A.un_W[gi];
        }
      }
    }
    return;
  }

  PhysC P;
  P.g = I.g;
  P.lam = I.lam;
  P.dx = I.dx;
  P.tau = A.tau_factor * dt;
  P.sl = A.slope;
  P.tdx = P.tau / P.dx;
  P.lt2 = P.lam * P.tau * P.tau;
  P.rr = P.tdx * P.tdx;
  P.tdx2 = 0.5 * P.tdx;
  const bool useb = BED && I.has_b;
  const bool first_tile = td.tidx == 0;
  const bool last_tile = td.tidx == I.ntiles - 1;
  const bool trans = bc != 0;
  bool bad = false, noncoer = false;

  // ---- 1. explicit sweep over the chunk (rolling window of 4 cells) ----
  Rec rec[KMAX];
  double ho[KMAX];
  Rec rec_last;  // rec[k-1]
  if (act) {
    Cell w0 = load_E<STAGE>(A, base + wrap_idx(c0 - 2, n, bc));
    Cell w1 = load_E<STAGE>(A, base + wrap_idx(c0 - 1, n, bc));
    Cell w2 = load_E<STAGE>(A, base + wrap_idx(c0, n, bc));
    Cell w3 = load_E<STAGE>(A, base + wrap_idx(c0 + 1, n, bc));
    double b0 = loadb<BED>(A, useb, base + wrap_idx(c0 - 2, n, bc));
    double b1 = loadb<BED>(A, useb, base + wrap_idx(c0 - 1, n, bc));
    double b2 = loadb<BED>(A, useb, base + wrap_idx(c0, n, bc));
    double b3 = loadb<BED>(A, useb, base + wrap_idx(c0 + 1, n, bc));
    Flux Fl = face_flux<BED>(w0, w1, w2, w3, b0, b1, b2, b3, P.g, P.sl, bad);
#pragma unroll
    for (int j = 0; j < KMAX; ++j) {
      if (j < k) {
        const int64_t g4 = base + wrap_idx(c0 + j + 2, n, bc);
        const Cell w4 = load_E<STAGE>(A, g4);
        const double b4 = loadb<BED>(A, useb, g4);
        const Flux Fr = face_flux<BED>(w1, w2, w3, w4, b1, b2, b3, b4, P.g, P.sl, bad);
        const Cell o = load_old<STAGE>(A, base + c0 + j);
        ho[j] = o.h;
        rec[j] = cell_record<BED>(w2, o, Fl, Fr, b1, b2, b3, P, bad, noncoer);
        if (j == k - 1) rec_last = rec[j];
        w0 = w1; w1 = w2; w2 = w3; w3 = w4;
        b0 = b1; b1 = b2; b2 = b3; b3 = b4;
        Fl = Fr;
      }
    }
    // share the chunk's end records with the neighbouring chunks
    nb_beta[0][t] = rec[0].beta; nb_S[0][t] = rec[0].S; nb_qd[0][t] = rec[0].qd;
    nb_phi[0][t] = rec[0].phi; nb_T[0][t] = rec[0].T; nb_b[0][t] = rec[0].b;
    nb_beta[1][t] = rec_last.beta; nb_S[1][t] = rec_last.S; nb_qd[1][t] = rec_last.qd;
    nb_phi[1][t] = rec_last.phi; nb_T[1][t] = rec_last.T; nb_b[1][t] = rec_last.b;
  }
  // outer neighbours of the tile
  Rec recL, recR;
  bool foldL = false, foldR = false;
  if (act && t == 0) {
    if (first_tile && trans) {
      recL = rec[0];
      foldL = true;
    } else {
      recL = single_record<BED, STAGE>(A, base, n, bc, useb, c0 - 1, P, bad, noncoer);
    }
  }
  if (act && t == ch.active - 1) {
    if (last_tile && trans) {
      recR = rec_last;
      foldR = true;
    } else {
      recR = single_record<BED, STAGE>(A, base, n, bc, useb, c0 + k, P, bad, noncoer);
    }
  }
  __syncthreads();
  if (act && t > 0) {
    recL.beta = nb_beta[1][t - 1]; recL.S = nb_S[1][t - 1]; recL.qd = nb_qd[1][t - 1];
    recL.phi = nb_phi[1][t - 1]; recL.T = nb_T[1][t - 1]; recL.b = nb_b[1][t - 1];
  }
  if (act && t < ch.active - 1) {
    recR.beta = nb_beta[0][t + 1]; recR.S = nb_S[0][t + 1]; recR.qd = nb_qd[0][t + 1];
    recR.phi = nb_phi[0][t + 1]; recR.T = nb_T[0][t + 1]; recR.b = nb_b[0][t + 1];
  }

  // ---- 2+3. rows and chunk elimination ----
  // interior rows 1..k-2: x_j = y_j + v_j x_0 + w_j x_{k-1}
  double cp[KMAX], y[KMAX], v[KMAX], w[KMAX];
  double r0[4], rl[4];  // first and last row of the chunk
  double yk2 = 0.0, vk2 = 0.0, wk2 = 0.0;
  if (act) {
    double cprev = 0.0, yprev = 0.0, vprev = 1.0, wprev = 0.0;
#pragma unroll
    for (int j = 0; j < KMAX; ++j) {
      if (j < k) {
        const Rec Lr = (j == 0) ? recL : rec[j > 0 ? j - 1 : 0];
        const Rec Rr = (j == k - 1) ? recR : rec[j + 1 < KMAX ? j + 1 : KMAX - 1];
        double lo, di, up, rhs;
        make_row<BED>(Lr, rec[j], Rr, ho[j], P, lo, di, up, rhs);
        if (j == 0 && foldL) {
          di += lo;
          lo = 0.0;
        }
        if (j == k - 1 && foldR) {
          di += up;
          up = 0.0;
        }
        if (j == 0) {
          r0[0] = lo; r0[1] = di; r0[2] = up; r0[3] = rhs;
        } else if (j == k - 1) {
          rl[0] = lo; rl[1] = di; rl[2] = up; rl[3] = rhs;
        } else {
          const double den = di - lo * cprev;
          const double inv = 1.0 / den;
          const bool lastint = (j == k - 2);
          cp[j] = lastint ? 0.0 : up * inv;
          y[j] = (rhs - lo * yprev) * inv;
          v[j] = (-lo * vprev) * inv;
          w[j] = (-lo * wprev) * inv - (lastint ? up * inv : 0.0);
          cprev = cp[j];
          yprev = y[j];
          vprev = v[j];
          wprev = w[j];
        }
      }
    }
    // back pass over the interior
    double yn = 0.0, vn = 0.0, wn = 0.0;
#pragma unroll
    for (int j = KMAX - 2; j >= 1; --j) {
      if (j <= k - 2) {
        y[j] = y[j] - cp[j] * yn;
        v[j] = v[j] - cp[j] * vn;
        w[j] = w[j] - cp[j] * wn;
        yn = y[j];
        vn = v[j];
        wn = w[j];
        if (j == k - 2) {
          yk2 = y[j];
          vk2 = v[j];
          wk2 = w[j];
        }
      }
    }
    double R0[4], R1[4];
    if (k > 2) {
      R0[0] = r0[0];
      R0[1] = r0[1] + r0[2] * v[1];
      R0[2] = r0[2] * w[1];
      R0[3] = r0[3] - r0[2] * y[1];
      R1[0] = rl[0] * vk2;
      R1[1] = rl[1] + rl[0] * wk2;
      R1[2] = rl[2];
      R1[3] = rl[3] - rl[0] * yk2;
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        R0[e] = r0[e];
        R1[e] = rl[e];
      }
    }
    S.a[2 * t] = R0[0]; S.b[2 * t] = R0[1]; S.c[2 * t] = R0[2]; S.d0[2 * t] = R0[3];
    S.d1[2 * t] = 0.0; S.d2[2 * t] = 0.0;
    S.a[2 * t + 1] = R1[0]; S.b[2 * t + 1] = R1[1]; S.c[2 * t + 1] = R1[2];
    S.d0[2 * t + 1] = R1[3]; S.d1[2 * t + 1] = 0.0; S.d2[2 * t + 1] = 0.0;
  }
  __syncthreads();
  const int n1 = 2 * ch.active;
  level1_interior<NT>(S, n1);

  // ---- 4. the tile's end unknowns ----
  if (t == 0) {
    double R0[4], R1[4];
    tile_rows<NT>(S, n1, R0, R1);
    if (REDUCE) {
      const int r = I.red_off + 2 * td.tidx;
      A.rlo[r] = R0[0]; A.rdi[r] = R0[1]; A.rup[r] = R0[2]; A.rrhs[r] = R0[3];
      A.rlo[r + 1] = R1[0]; A.rdi[r + 1] = R1[1]; A.rup[r + 1] = R1[2]; A.rrhs[r + 1] = R1[3];
    } else {
      double z0, zl, xl, xr;
      if (I.ntiles == 1) {
        solve_ends(R0, R1, !trans, z0, zl);
        xl = trans ? z0 : zl;
        xr = trans ? zl : z0;
      } else {
        const int r = I.red_off + 2 * td.tidx;
        const int M = 2 * I.ntiles;
        z0 = A.rx[r];
        zl = A.rx[r + 1];
        xl = first_tile ? (trans ? z0 : A.rx[I.red_off + M - 1]) : A.rx[r - 1];
        xr = last_tile ? (trans ? zl : A.rx[I.red_off]) : A.rx[r + 2];
      }
      S.s[0] = z0;
      S.s[1] = zl;
      S.s[2] = xl;
      S.s[3] = xr;
    }
  }
  if (REDUCE) return;
  __syncthreads();
  const double z0 = S.s[0], zl = S.s[1], xl_ext = S.s[2], xr_ext = S.s[3];
  // level-1 values of this thread's two rows
  double zf = 0.0, zb = 0.0;
  if (act) {
    const int j0 = 2 * t, j1 = 2 * t + 1;
    zf = (j0 == 0) ? z0 : S.d0[j0] + S.d1[j0] * z0 + S.d2[j0] * zl;
    zb = (j1 == n1 - 1) ? zl : S.d0[j1] + S.d1[j1] * z0 + S.d2[j1] * zl;
  }
  __syncthreads();
  if (act) {
    S.a[2 * t] = zf;
    S.a[2 * t + 1] = zb;
  }
  __syncthreads();

  // ---- 5. back-substitution ----
  double smax = 0.0, umax = 0.0;
  if (act) {
    const double hl_nb = (t > 0) ? S.a[2 * t - 1] : xl_ext;
    const double hr_nb = (t < ch.active - 1) ? S.a[2 * t + 2] : xr_ext;
    double hb[KMAX];
#pragma unroll
    for (int j = 0; j < KMAX; ++j) {
      if (j < k) hb[j] = (j == 0) ? zf : ((j == k - 1) ? zb : y[j] + v[j] * zf + w[j] * zb);
    }
    const double i2dx = 1.0 / (2.0 * P.dx);
#pragma unroll
    for (int j = 0; j < KMAX; ++j) {
      if (j < k) {
        const Rec Lr = (j == 0) ? recL : rec[j > 0 ? j - 1 : 0];
        const Rec Rr = (j == k - 1) ? recR : rec[j + 1 < KMAX ? j + 1 : KMAX - 1];
        const double hm = (j == 0) ? hl_nb : hb[j > 0 ? j - 1 : 0];
        const double hp = (j == k - 1) ? hr_nb : hb[j + 1 < KMAX ? j + 1 : KMAX - 1];
        const double h = hb[j];
        const double Pm = Lr.S + Lr.beta * hm;
        const double Pp = Rr.S + Rr.beta * hp;
        double force = (Pp - Pm) * i2dx;
        if (BED) {
          const double dbc = (Rr.b - Lr.b) * i2dx;
          const double pti = rec[j].T + rec[j].phi * h;
          force += 0.5 * P.g * (hp + hm) * dbc + 1.5 * pti * dbc;
        }
        const double qn = rec[j].qd - P.tau * force;
        const double ih = 1.0 / h;
        const double mn = rec[j].md / (1.0 + P.lt2 * ih * ih);
        const double Wn = rec[j].Wd - P.lam * P.tau * mn * ih * ih;
        bad |= !(h > 0.0) || !isfinite(qn) || !isfinite(mn) || !isfinite(Wn);
        const int64_t gi = base + c0 + j;
        A.o_h[gi] = h;
        A.o_q[gi] = qn;
        A.o_m[gi] = mn;
        A.o_W[gi] = Wn;
        if (STAGE == 2) {
          const double u = fabs(qn * ih);
          smax = fmax(smax, u + sqrt(P.g * h));
          umax = fmax(umax, u);
        }
      }
    }
  }
  if (STAGE == 2) {
    // all lanes take part; idle lanes contribute 0 (speeds are >= 0)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      smax = fmax(smax, __shfl_xor(smax, off));
      umax = fmax(umax, __shfl_xor(umax, off));
    }
    if ((t & 63) == 0 && smax > 0.0) {
      atomicMax(&A.smax[td.inst], (unsigned long long)__double_as_longlong(smax));
      atomicMax(&A.umax[td.inst], (unsigned long long)__double_as_longlong(umax));
    }
  }
  if (bad || noncoer) {
    atomicOr(&A.status[td.inst], (bad ? kFlagNonPhys : 0) | (noncoer ? kFlagNonCoercive : 0));
  }
}

// ---------------------------------------------------------------------------
// Reduced system across the tiles of one instance (2 rows per tile,
// cyclic when periodic): same two-level partition solve, with the chunk
// data kept in global scratch since chunks may be long.
// ---------------------------------------------------------------------------
template <int NT>
__global__ __launch_bounds__(NT) void k_rsolve(const InstDesc* __restrict__ inst,
                                               const int32_t* __restrict__ multi,
                                               const double* __restrict__ dt,
                                               const double* __restrict__ rlo,
                                               const double* __restrict__ rdi,
                                               const double* __restrict__ rup,
                                               const double* __restrict__ rrhs,
                                               double* __restrict__ rx, double* __restrict__ scp,
                                               double* __restrict__ sy, double* __restrict__ sv,
                                               double* __restrict__ sw) {
  __shared__ Lds<NT> S;
  const int j = multi[blockIdx.x];
  const InstDesc I = inst[j];
  if (!(dt[j] > 0.0)) return;
  const int M = 2 * I.ntiles;
  const int t = threadIdx.x;
  const Chunk ch = chunk_of(M, NT, t);
  const int k = ch.k;
  const int f = I.red_off + ch.first;
  const bool act = t < ch.active;
  if (act) {
    double cprev = 0.0, yprev = 0.0, vprev = 1.0, wprev = 0.0;
    for (int i = 1; i <= k - 2; ++i) {
      const double lo = rlo[f + i], di = rdi[f + i], up = rup[f + i], rhs = rrhs[f + i];
      const double inv = 1.0 / (di - lo * cprev);
      const bool lastint = (i == k - 2);
      cprev = lastint ? 0.0 : up * inv;
      yprev = (rhs - lo * yprev) * inv;
      vprev = (-lo * vprev) * inv;
      wprev = (-lo * wprev) * inv - (lastint ? up * inv : 0.0);
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
    double R0[4] = {rlo[f], rdi[f], rup[f], rrhs[f]};
    double R1[4] = {rlo[l], rdi[l], rup[l], rrhs[l]};
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
    solve_ends(R0, R1, I.bc == 0, z0, zl);
    S.s[0] = z0;
    S.s[1] = zl;
  }
  __syncthreads();
  const double z0 = S.s[0], zl = S.s[1];
  if (act) {
    const int j0 = 2 * t, j1 = 2 * t + 1;
    const double zf = (j0 == 0) ? z0 : S.d0[j0] + S.d1[j0] * z0 + S.d2[j0] * zl;
    const double zb = (j1 == n1 - 1) ? zl : S.d0[j1] + S.d1[j1] * z0 + S.d2[j1] * zl;
    rx[f] = zf;
    rx[f + k - 1] = zb;
    for (int i = 1; i <= k - 2; ++i) rx[f + i] = sy[f + i] + sv[f + i] * zf + sw[f + i] * zb;
  }
}

// Time step per instance from the speed bound of the current state
// (CFL on |u| + sqrt(g h), material-CFL cap, t_end clamp).  Resets the
// accumulators for the next step.
// (nstep counts the steps each instance has taken since its state was
// loaded: a flagged instance stops counting, so its count names the step in
// which the flag was raised)
static __global__ void k_dt(int n_inst, const InstDesc* __restrict__ inst, double* __restrict__ dt,
                     double* __restrict__ tt, unsigned long long* __restrict__ smax,
                     unsigned long long* __restrict__ umax, const int32_t* __restrict__ status,
                     int32_t* __restrict__ nstep) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_inst) return;
  const InstDesc I = inst[j];
  double d;
  if (status[j] != 0) {
    d = 0.0;
  } else if (I.dt_fixed > 0.0) {
    d = I.dt_fixed;
  } else {
    const double s = __longlong_as_double((long long)smax[j]);
    const double u = __longlong_as_double((long long)umax[j]);
    d = I.cfl * I.dx / s;
    if (I.mcfl > 0.0 && u * d / I.dx > I.mcfl) d = I.mcfl * I.dx / u;
  }
  const double t0 = tt[j];
  if (I.t_end > 0.0) {
    if (t0 >= I.t_end) d = 0.0;
    else if (t0 + d > I.t_end) d = I.t_end - t0;
  }
  if (!(d > 0.0) || !isfinite(d)) d = 0.0;
  if (d > 0.0) nstep[j] += 1;
  dt[j] = d;
  tt[j] = t0 + d;
  smax[j] = 0ull;
  umax[j] = 0ull;
}

// Speed bound of a given state (first step after a state is loaded).
template <int NT>
__global__ __launch_bounds__(NT) void k_speed(const InstDesc* __restrict__ inst,
                                              const TileDesc* __restrict__ tiles,
                                              const double* __restrict__ h,
                                              const double* __restrict__ q,
                                              unsigned long long* __restrict__ smax,
                                              unsigned long long* __restrict__ umax,
                                              unsigned long long* __restrict__ hmax) {
  const TileDesc td = tiles[blockIdx.x];
  const InstDesc I = inst[td.inst];
  double s = 0.0, u = 0.0, hx = 0.0;
  for (int i = threadIdx.x; i < td.len; i += NT) {
    const int64_t gi = I.off + td.start + i;
    const double hh = h[gi];
    const double uu = fabs(q[gi] / hh);
    s = fmax(s, uu + sqrt(I.g * hh));
    u = fmax(u, uu);
    hx = fmax(hx, hh);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    s = fmax(s, __shfl_xor(s, off));
    u = fmax(u, __shfl_xor(u, off));
    hx = fmax(hx, __shfl_xor(hx, off));
  }
  if ((threadIdx.x & 63) == 0 && s > 0.0) {
    atomicMax(&smax[td.inst], (unsigned long long)__double_as_longlong(s));
    atomicMax(&umax[td.inst], (unsigned long long)__double_as_longlong(u));
    atomicMax(&hmax[td.inst], (unsigned long long)__double_as_longlong(hx));
  }
}

// m = h^2 and W = 0 where the caller gave none.
// Default auxiliary variables of a loaded state (initial data of Sec. 6.3:
// eta = h and w = -h u_x): m = h^2 and W = -h^2 u_x with the central
// difference u_x,i = (u_{i+1} - u_{i-1}) / (2 dx) of u = q/h; periodic
// instances wrap, transmissive ones use a copy of the boundary cell beyond
// each end.  One workgroup per two-pass tile.
template <int NT>
__global__ __launch_bounds__(NT) void k_default_mW(const InstDesc* __restrict__ inst,
                                                   const TileDesc* __restrict__ tiles,
                                                   const double* __restrict__ h,
                                                   const double* __restrict__ q,
                                                   double* __restrict__ m, double* __restrict__ W,
                                                   int set_m, int set_W) {
  const TileDesc td = tiles[blockIdx.x];
  const InstDesc I = inst[td.inst];
  for (int k = threadIdx.x; k < td.len; k += NT) {
    const int i = td.start + k;
    const int64_t gi = I.off + i;
    const double hi = h[gi];
    if (set_m) m[gi] = hi * hi;
    if (set_W) {
      int im = i - 1, ip = i + 1;
      if (I.bc == 0) {
        if (im < 0) im += I.n;
        if (ip >= I.n) ip -= I.n;
      } else {
        if (im < 0) im = 0;
        if (ip >= I.n) ip = I.n - 1;
      }
      const double um = q[I.off + im] / h[I.off + im];
      const double up = q[I.off + ip] / h[I.off + ip];
      W[gi] = -hi * hi * (up - um) / (2.0 * I.dx);
    }
  }
}

// Fill (used instead of memset so that the calls stay capturable).
static __global__ void k_fill_u64(int n, unsigned long long* __restrict__ p, unsigned long long v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
static __global__ void k_fill_i32(int n, int32_t* __restrict__ p, int32_t v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace hsgn
