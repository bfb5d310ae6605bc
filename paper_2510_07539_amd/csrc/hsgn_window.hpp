// hsgn_window.hpp -- single-pass windowed stage kernel.
//
// A tile writes the cells of its core [cs, cs + cl) but solves the depth
// system on a window that extends the core by L cells on every side that is
// not a physical boundary.  Beyond a window edge that is not physical the
// unknown depth is replaced by the explicit-stage depth h_E (its coupling
// moves to the right-hand side).  The system is diagonally dominant, so the
// influence of that replacement on the core decays geometrically with the
// distance L; the kernel computes that influence exactly at both core edges
// (the derivatives of the window solve with respect to the two edge
// guesses) and flags the instance (status bit 4) if the resulting bound
// exceeds 2^-56 of the local depth.  Instances that fit in one window are
// solved exactly (no truncation).
//
// Each of the NT threads owns exactly K consecutive window rows (K is a
// compile-time constant); rows past the window's real length are identity
// rows, decoupled from the rest.  Inputs are staged through LDS with
// coalesced loads.  The sweep and the rows are the same arithmetic as the
// two-pass kernel in hsgn_kernels.hpp; the solve eliminates each thread's
// chunk in registers and solves the resulting level-1 system (two rows per
// thread) in LDS.
#pragma once

#include "hsgn_kernels.hpp"

namespace hsgn {

constexpr int32_t kFlagWindow = 4;

struct WinDesc {
  int64_t off;    // the instance's first cell, its length, boundary and bed flag
  int32_t n;      // (copies of its descriptor, so that the first loads of a
  int32_t bc;     // window wait for this descriptor only)
  int32_t has_b;
  int32_t inst;
  int32_t ws;     // window start, relative to the instance (may be < 0 if periodic)
  int32_t wl;     // real rows of the window (<= NT*K)
  int32_t cs;     // core start (relative to the instance, in [0, n))
  int32_t cl;     // core length
  int32_t flags;  // bit 0: left edge truncated; bit 1: right edge truncated
  int32_t pad;
};

struct WinArgs {
  StageArgs s;
  const WinDesc* __restrict__ win;
  int32_t nwin;
  int32_t xcd_stride;  // consecutive windows go to one XCD: see k_win
  int32_t* queue;      // k_win_persist: 8 queue counters + 1 count of ended
                       // workgroups (zero between launches)
};

// A value that is the same in every lane, computed on the vector unit (the
// scalar unit has no FP64 arithmetic), moved to scalar registers so that it
// occupies no vector registers while it stays live.
__device__ __forceinline__ double to_sgpr(double x) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(x);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)u);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(u >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Fast reciprocal: hardware estimate and two Newton steps (error of a few
// ulp at most for the normal, finite operands that reach it).
__device__ __forceinline__ double frcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(e, r, r);
  e = fma(-x, r, 1.0);
  r = fma(e, r, r);
  return r;
}

// Square root of a positive normal operand: hardware reciprocal square-root
// estimate (about 2^-24 relative), one Goldschmidt step (2^-48) and one
// residual correction (about 1 ulp).  The operands here are g h with h
// checked positive, so the library's scaling for tiny and special operands
// is not needed; a non-positive h yields a NaN, on an instance that is
// flagged anyway.
__device__ __forceinline__ double fsqrt(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y;
  double h = 0.5 * y;
  const double r = fma(-h, g, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  const double d = fma(-g, g, x);
  return fma(d, h, g);
}

template <bool BED>
__device__ __forceinline__ Flux face_flux_fast(const Cell& cm, const Cell& c0, const Cell& c1,
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
  const double uL = qL * frcp(hL);
  const double uR = qR * frcp(hR);
  const double sL = fabs(uL) + fsqrt(g * hL);
  const double sR = fabs(uR) + fsqrt(g * hR);
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

// Frozen coefficients of a row (beta, S and, with a bed, phi and T) from
// h_E, m_E and m-dagger (already in r.md); the bed value goes along.
template <bool BED>
__device__ __forceinline__ void rec_coefs_fast(Rec& r, double h, double em, double bc,
                                               const PhysC& P, bool& bad, bool& noncoer) {
  const double md = r.md;
  bad |= !(h > 0.0);
  const double ih = frcp(h);
  const double eh = em * ih * ih;
  const double alpha = -(2.0 * eh - 1.0) * ih * (1.0 / 3.0);
  const double a2 = P.g * h + P.lam * eh * eh - P.lam3 * eh;
  const double b1 = 1.0 + P.lt2 * ih * ih;
  const double ib1 = frcp(b1);
  const double b2 = 2.0 * P.lt2 * ib1 * ib1 * ih * ih * ih;
  r.beta = a2 + P.lam * alpha * b2 * md;
  noncoer |= !(r.beta > 0.0);
  const double eta0 = md * ib1 * ih;
  const double pt0 = P.lam3 * (1.0 - eta0 * ih);
  const double P0 = 0.5 * P.g * h * h + eta0 * pt0;
  r.S = P0 - r.beta * h;
  if (BED) {
    r.phi = P.lam23 * md * ih * ih * ih * ib1 * ib1;
    r.T = pt0 - r.phi * h;
  } else {
    r.phi = 0.0;
    r.T = 0.0;
  }
  r.b = bc;
}

template <bool BED>
__device__ __forceinline__ Rec cell_record_fast(const Cell& e, const Cell& o, const Flux& Fl,
                                                const Flux& Fr, double bm, double bc, double bp,
                                                const PhysC& P, double i2dx, bool& bad,
                                                bool& noncoer) {
  Rec r;
  r.Wd = o.W - P.tdx * (Fr.W - Fl.W) + P.lam * P.tau;
  double md = o.m - P.tdx * (Fr.m - Fl.m);
  if (BED) md -= P.tau * 1.5 * e.q * ((bp - bm) * i2dx);
  md += P.tau * r.Wd;
  r.md = md;
  r.qd = o.q - P.tdx * (Fr.q - Fl.q);
  rec_coefs_fast<BED>(r, e.h, e.m, bc, P, bad, noncoer);
  return r;
}

// Level-1 interior solve with one reciprocal per row and level.
template <int NT>
__device__ void level1_interior_fast(Lds<NT>& S, int n1, const int t = threadIdx.x) {
  const int last = n1 - 2;
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
        const double a = S.a[j], c = S.c[j];
        const double k1 = hm ? a * frcp(S.b[jm]) : 0.0;
        const double k2 = hp ? c * frcp(S.b[jp]) : 0.0;
        na[r] = hm ? -k1 * S.a[jm] : 0.0;
        nc[r] = hp ? -k2 * S.c[jp] : 0.0;
        double bb = S.b[j];
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
    // couplings left after this level; once every one is below 2^-66 of
    // its diagonal the remaining levels change no digit of the solution
    bool more = false;
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
        const double lim = 1.3552527156068805e-20 * fabs(nb[r]);  // 2^-66
        more |= !(fabs(na[r]) <= lim) || !(fabs(nc[r]) <= lim);
      }
    }
    if (!__syncthreads_or(more)) break;
  }
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int j = 1 + t + r * NT;
    if (j <= last) {
      const double ib = frcp(S.b[j]);
      S.d0[j] *= ib;
      S.d1[j] *= ib;
      S.d2[j] *= ib;
    }
  }
  __syncthreads();
}

// Ordering of LDS accesses among the lanes of one wavefront: a wavefront's
// LDS operations are performed in the order it issues them, so its lanes
// exchange values through LDS without a workgroup barrier.  The fences
// only keep the compiler from moving loads and stores across this point
// (at wavefront scope they emit no instruction).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Level-1 solve of one wavefront's segment of rows [F, E] (F < E): the
// interior rows F + 1 .. E - 1 are eliminated by parallel cyclic reduction
// in terms of the segment's end unknowns x_F and x_E, by the wavefront's
// 64 lanes (lane l) and with no workgroup barrier.  On exit d0, d1, d2 of an
// interior row hold Y, V, W with x_j = Y_j + V_j x_F + W_j x_E; the end rows
// keep their coefficients.  The reduction stops at the first level after
// which every coupling left is below 2^-66 of its diagonal: the levels after
// it would change no digit of the solution.
template <int NT>
__device__ void segment_pcr(Lds<NT>& S, const int F, const int E, const int l) {
  const int m = E - F - 1;  // interior rows
  if (m <= 0) return;
  if (l == 0) {
    S.d1[F + 1] = -S.a[F + 1];
    S.a[F + 1] = 0.0;
    S.d2[E - 1] = -S.c[E - 1];
    S.c[E - 1] = 0.0;
  }
  wave_lds_sync();
  for (int s = 1; s < m; s <<= 1) {
    double na[2], nb[2], nc[2], n0[2], n1v[2], n2[2];
    bool own[2];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int jr = 1 + l + 64 * r;  // segment-relative row
      own[r] = jr <= m;
      if (own[r]) {
        const int j = F + jr;
        const int jm = j - s, jp = j + s;
        const bool hm = jr - s >= 1, hp = jr + s <= m;
        const double a = S.a[j], c = S.c[j];
        const double k1 = hm ? a * frcp(S.b[jm]) : 0.0;
        const double k2 = hp ? c * frcp(S.b[jp]) : 0.0;
        na[r] = hm ? -k1 * S.a[jm] : 0.0;
        nc[r] = hp ? -k2 * S.c[jp] : 0.0;
        double bb = S.b[j];
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
    wave_lds_sync();
    bool more = false;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      if (own[r]) {
        const int j = F + 1 + l + 64 * r;
        S.a[j] = na[r];
        S.b[j] = nb[r];
        S.c[j] = nc[r];
        S.d0[j] = n0[r];
        S.d1[j] = n1v[r];
        S.d2[j] = n2[r];
        const double lim = 1.3552527156068805e-20 * fabs(nb[r]);  // 2^-66
        more |= !(fabs(na[r]) <= lim) || !(fabs(nc[r]) <= lim);
      }
    }
    const bool again = __ballot(more) != 0;  // the same in every lane
    wave_lds_sync();
    if (!again) break;
  }
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int jr = 1 + l + 64 * r;
    if (jr <= m) {
      const int j = F + jr;
      const double ib = frcp(S.b[j]);
      S.d0[j] *= ib;
      S.d1[j] *= ib;
      S.d2[j] *= ib;
    }
  }
  wave_lds_sync();
}

// The end rows F and E of a segment solved by segment_pcr, with its
// interior substituted (x_{F+1} and x_{E-1} from Y, V, W): rows of the
// tridiagonal system in the segments' end unknowns (x_{F_0}, x_{E_0},
// x_{F_1}, x_{E_1}, ...) as (lower, diagonal, upper, right-hand side).
template <int NT>
__device__ __forceinline__ void segment_ends(const Lds<NT>& S, int F, int E, double R0[4],
                                             double R1[4]) {
  if (E == F + 1) {
    R0[0] = S.a[F]; R0[1] = S.b[F]; R0[2] = S.c[F]; R0[3] = S.d0[F];
    R1[0] = S.a[E]; R1[1] = S.b[E]; R1[2] = S.c[E]; R1[3] = S.d0[E];
    return;
  }
  R0[0] = S.a[F];
  R0[1] = S.b[F] + S.c[F] * S.d1[F + 1];
  R0[2] = S.c[F] * S.d2[F + 1];
  R0[3] = S.d0[F] - S.c[F] * S.d0[F + 1];
  R1[0] = S.a[E] * S.d1[E - 1];
  R1[1] = S.b[E] + S.a[E] * S.d2[E - 1];
  R1[2] = S.c[E];
  R1[3] = S.d0[E] - S.a[E] * S.d0[E - 1];
}

// LDS layout of a staged window field: one pad double after every 8 so that
// a thread reading its K consecutive values does not collide on banks.
__device__ __forceinline__ int spad(int i) { return i + (i >> 3); }

// Cell index of instance-relative position i for any i (a periodic window
// may be longer than the ring).
__device__ __forceinline__ int wrap_any(int i, int n, int bc) {
  if (bc == 0) {
    int r = i % n;
    return r < 0 ? r + n : r;
  }
  return i < 0 ? 0 : (i > n - 1 ? n - 1 : i);
}

template <int NT, int K, bool BED>
struct WinLds {
  static constexpr int WN = NT * K;
  static constexpr int SL = WN + 8;              // staged cells: window + 3 halo each side (+2)
  static constexpr int SP = SL + (SL >> 3) + 1;  // padded length
  union {
    struct {
      double e[SP];             // staged explicit-state field (window + halo)
      double o[SP];             // staged old-state field (stage 2)
      double b[BED ? SP : 1];   // staged bed (kept through the sweep)
      double ho[SP];            // old depth (kept until the rows are built)
    } st;
    Lds<NT> sys;
    struct {
      double beta[2][NT], S[2][NT], qd[2][NT], phi[2][NT], T[2][NT], b[2][NT];
    } nb;
  } u;
  // The record exchange (nb) and the level-1 system (sys) reuse the storage
  // of the staging buffers e and o, and must not reach the bed or the old
  // depth, which are still read after them.
  static_assert(sizeof(Lds<NT>) <= 2 * SP * sizeof(double) &&
                    12 * NT * sizeof(double) <= 2 * SP * sizeof(double),
                "the level-1 system and the record exchange must fit in the staging buffers "
                "e and o");
  double misc[16];
  // system of the wavefront segments' end unknowns: rows (lower, diagonal,
  // upper, right-hand side), then its solution and the solution's
  // derivatives with respect to the left and right edge guesses
  static constexpr int NW = NT / 64;
  double l2[4][2 * NW];
  double l2x[3][2 * NW];
  // inputs of the outer rows of truncated edges (window rows -1 and wl):
  // U_E of five staged cells, the row's old state, the bed (side 0 left,
  // side 1 right)
  double side[2][4][5], sideo[2][4], sideb[2][5];
};

// One window of a stage: the body of k_win (one window per workgroup) and of
// the persistent k_win_persist below.  t is the thread index (passed in so
// that the persistent loop can keep it opaque).
template <int NT, int K, bool BED, int STAGE>
__device__ __forceinline__ void win_one(const WinArgs& W, WinLds<NT, K, BED>& L, const int bid,
                                        const int t) {
  // Register budget: 256 per lane (two waves per SIMD).  Both stages
  // address the staged loads with 32-bit offsets from per-instance base
  // pointers.  Stage 1 also reads neighbour beds from the staged bed instead
  // of carrying them in the records (kLean); stage 2 carries them (measured
  // faster) and parks m-dagger and W-dagger in LDS through the solve
  // (kStash below).  Both forms give the same values.
  constexpr bool kLean = STAGE == 1;
  const StageArgs& A = W.s;
  const WinDesc wd = W.win[bid];
  // Warm this XCD's L2 with the descriptor of the window that starts about
  // one block lifetime later (64 blocks run at once per XCD): a vector load
  // by one thread (its index made opaque, so the load is not scalarised and
  // does not hold up the waits for LDS) whose value only feeds an empty asm
  // statement after the last staging round.
  int ahead = 0;
  {
    int zero = t;
    asm volatile("" : "+v"(zero));
    zero >>= 31;
    const int wa_ = bid + 64;
    const int lim = W.xcd_stride > 0 ? min(W.nwin, (bid / W.xcd_stride + 1) * W.xcd_stride) : W.nwin;
    if (t == 0 && wa_ < lim) ahead = W.win[wa_ + zero].inst;
  }
  const int n = wd.n, bc = wd.bc;
  const int64_t base = wd.off;
  constexpr int WN = NT * K;
  const int na = (wd.wl + K - 1) / K;  // threads with real rows
  const bool act = t < na;
  const int p0 = t * K;                 // first window row of this thread
  const bool truncL = (wd.flags & 1) != 0, truncR = (wd.flags & 2) != 0;
  const bool useb = BED && wd.has_b;
  const bool physL = !truncL, physR = !truncR;

  // ---- staging and explicit sweep, one field per round: h (with the bed),
  // q, m, W.  A round stages the explicit state E (stage 2: kE0 U^n + kE1 U(1))
  // and the old state O (stage 2: kT0 U^n + kT1 U(1)) of window rows
  // [-3, wl + 3) through LDS with coalesced loads; each thread then reads the
  // values of its K + 1 faces and K rows and keeps only per-face and per-row
  // partial results.  The loads of the next round are in flight meanwhile.
  // Staged index i <-> window row i - 3; rows past the window's real end
  // repeat row wl + 2 (their values only feed identity padding rows).
  if (t == 0) {
    L.misc[0] = 0.0;  // depth guesses beyond truncated edges (0 if physical)
    L.misc[1] = 0.0;
  }
  const int SLn = na * K + 6;
  // instance cell of staged index i: rows past wl + 2 repeat row wl + 2; the
  // periodic wrap needs a true modulo only when the window is longer than
  // the ring
  const bool fast_wrap = (bc != 0) || (n >= WN + 8);
  auto cell_of = [&](int i) -> int {
    int p = i - 3;
    if (p > wd.wl + 2) p = wd.wl + 2;
    const int c = wd.ws + p;
    if (!fast_wrap) return wrap_any(c, n, bc);
    if (bc == 0) return c < 0 ? c + n : (c >= n ? c - n : c);
    return c < 0 ? 0 : (c > n - 1 ? n - 1 : c);
  };
  constexpr int NR = (WinLds<NT, K, BED>::SL + NT - 1) / NT;  // staged elements per thread
  auto fld = [&](int f, bool second) -> const double* {
    if (second) return f == 0 ? A.u1_h : f == 1 ? A.u1_q : f == 2 ? A.u1_m : A.u1_W;
    return f == 0 ? A.un_h : f == 1 ? A.un_q : f == 2 ? A.un_m : A.un_W;
  };
  double va[NR], vb[NR], vc[NR];
  // instance-relative cells of the staged elements; past the window's
  // staged cells cell_of repeats the last one, so every load is in bounds
  // and the loads need no guard (the guards cost more than the few extra
  // loads), except stage 1's first two rounds, which are loaded together
  // and spill registers unguarded.  The LDS writes of every round but the
  // last stay inside the buffers and need no guard either: no row reads
  // the elements past the staged cells.
  constexpr bool kNoGuard = STAGE == 2;
  int cidx[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int i = t + r * NT;
    cidx[r] = cell_of(i);
  }
  // loads of round f into (xa, xb, xc): U^n, U(1) and the bed
  auto load_into = [&](int f, double* xa, double* xb, double* xc) {
    const double* un = fld(f, false);
    const double* u1 = fld(f, true);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      if (kNoGuard || f >= 2 || t + r * NT < SLn) {
        xa[r] = (un + base)[cidx[r]];
        if (STAGE == 2) xb[r] = (u1 + base)[cidx[r]];
        if (BED && f == 0 && useb) xc[r] = (A.b + base)[cidx[r]];
      }
    }
  };
  // staging buffer of round f: stage 1 (which stages no old state) alternates
  // between two, so a round's writes need no barrier after the previous
  // round's reads
  auto ebuf = [&](int f) -> double* { return (STAGE == 1 && (f & 1)) ? L.u.st.o : L.u.st.e; };
  auto put_from = [&](int f, const double* xa, const double* xb, const double* xc) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int i = t + r * NT;
      if (r < NR - 1 || i < SLn) {
        double* od = f == 0 ? L.u.st.ho : L.u.st.o;  // the old depth stays until the rows
        if (STAGE == 1) {
          ebuf(f)[spad(i)] = xa[r];
          if (f == 0) od[spad(i)] = xa[r];
        } else {
          L.u.st.e[spad(i)] = kE0 * xa[r] + kE1 * xb[r];
          od[spad(i)] = kT0 * xa[r] + kT1 * xb[r];
        }
        if (BED && f == 0 && useb) L.u.st.b[spad(i)] = xc[r];
      }
    }
  };
  auto load_round = [&](int f) { load_into(f, va, vb, vc); };
  auto put_round = [&](int f) { put_from(f, va, vb, vc); };
  // face f (0..K) lies between rows p0 + f - 1 and p0 + f; its stencil is
  // x[f .. f + 3] with x[i] the staged value of row p0 + i - 2
  auto read_x = [&](double* x, const double* src) {
#pragma unroll
    for (int i = 0; i < K + 4; ++i) x[i] = src[spad(p0 + 1 + i)];
  };
  auto old_of = [&](const double* x, int j) -> double {
    return STAGE == 1 ? x[j + 2] : L.u.st.o[spad(p0 + 3 + j)];
  };
  // bed of row p0 - 1 + i (i = 0..K+1); the staged bed stays in LDS
  auto bed_row = [&](int i) -> double {
    return (BED && useb) ? L.u.st.b[spad(p0 + 2 + i)] : 0.0;
  };
  // while field f is staged, the edge threads copy what the outer row of a
  // truncated edge needs (staged cells i0 .. i0 + 4, i0 = 0 on the left and
  // wl + 1 on the right) aside
  auto save_side = [&](int f) {
#pragma unroll
    for (int sd = 0; sd < 2; ++sd) {
      const bool need = sd == 0 ? (t == 0 && truncL) : (t == na - 1 && truncR);
      if (!need) continue;
      const int i0 = sd == 0 ? 0 : wd.wl + 1;
#pragma unroll
      for (int d = 0; d < 5; ++d) L.side[sd][f][d] = ebuf(f)[spad(i0 + d)];
      const double* od = f == 0 ? L.u.st.ho : L.u.st.o;
      L.sideo[sd][f] = STAGE == 1 ? ebuf(f)[spad(i0 + 2)] : od[spad(i0 + 2)];
      if (f == 0) {
#pragma unroll
        for (int d = 0; d < 5; ++d) L.sideb[sd][d] = (BED && useb) ? L.u.st.b[spad(i0 + d)] : 0.0;
      }
    }
  };

  // stage 1: rounds 0 and 1 are in flight together (the second set of
  // registers lives only until round 1 is staged, where few other values
  // are live); stage 2, which loads two states per round, issues round 1
  // once round 0 is staged, like the later rounds (measured 0.7 % faster)
  double wa[NR], wb[NR];
  load_round(0);
  if (STAGE == 1) load_into(1, wa, wb, vc);
  // the instance's parameters and step arrive while the first rounds load;
  // a frozen instance (no step) copies its core and leaves
  const InstDesc I = A.inst[wd.inst];
  const double dt = A.dt[wd.inst];
  if (!(dt > 0.0)) {  // frozen: copy the core
    for (int i = t; i < wd.cl; i += NT) {
      const int64_t gi = base + wd.cs + i;
      A.o_h[gi] = A.un_h[gi];
      A.o_q[gi] = A.un_q[gi];
      A.o_m[gi] = A.un_m[gi];
      A.o_W[gi] = A.un_W[gi];
    }
    return;
  }
  PhysC P;
  P.g = I.g;
  P.lam = I.lam;
  P.dx = I.dx;
  // per-window constants, computed once (the same values as in every row)
  // and held in scalar registers
  P.tau = to_sgpr(A.tau_factor * dt);
  P.sl = A.slope;
  P.tdx = to_sgpr(P.tau / P.dx);
  P.lt2 = to_sgpr(P.lam * P.tau * P.tau);
  P.rr = to_sgpr(P.tdx * P.tdx);
  P.tdx2 = to_sgpr(0.5 * P.tdx);
  P.lam3 = to_sgpr(P.lam / 3.0);
  P.lam23 = to_sgpr(2.0 * P.lam / 3.0);
  const double i2dx = to_sgpr(0.5 / P.dx);
  bool bad = false, noncoer = false;

  put_round(0);
  if (STAGE == 2) load_round(1);
  __syncthreads();
  // round h: face depths, depths of rows p0 - 1 .. p0 + K
  double hL[K + 1], hR[K + 1], hf[K + 2];
  unsigned badf = 0;  // bit f: a face depth of face f is not positive
  if (act) {
    save_side(0);
    double xh[K + 4];
    read_x(xh, ebuf(0));
#pragma unroll
    for (int f = 0; f <= K; ++f) {
      hL[f] = xh[f + 1] + P.sl * (xh[f + 2] - xh[f]);
      hR[f] = xh[f + 2] - P.sl * (xh[f + 3] - xh[f + 1]);
      if (!(hL[f] > 0.0) || !(hR[f] > 0.0)) badf |= 1u << f;
    }
#pragma unroll
    for (int i = 0; i < K + 2; ++i) hf[i] = xh[i + 1];
  }
  if (STAGE == 2) __syncthreads();
  if (STAGE == 1) put_from(1, wa, wb, vc);
  else put_round(1);
  load_round(2);
  __syncthreads();
  // round q: face velocities and Rusanov speeds, q-dagger
  double uL[K + 1], uR[K + 1], ap[K + 1], qd[K], eq[K];
  if (act) {
    save_side(1);
    double xq[K + 4], Fq[K + 1];
    read_x(xq, ebuf(1));
#pragma unroll
    for (int f = 0; f <= K; ++f) {
      const double qL = xq[f + 1] + P.sl * (xq[f + 2] - xq[f]);
      const double qR = xq[f + 2] - P.sl * (xq[f + 3] - xq[f + 1]);
      uL[f] = qL * frcp(hL[f]);
      uR[f] = qR * frcp(hR[f]);
      const double sL = fabs(uL[f]) + fsqrt(P.g * hL[f]);
      const double sR = fabs(uR[f]) + fsqrt(P.g * hR[f]);
      ap[f] = fmax(sL, sR);
      Fq[f] = 0.5 * (qL * uL[f] + qR * uR[f] - ap[f] * (qR - qL));
    }
#pragma unroll
    for (int j = 0; j < K; ++j) {
      qd[j] = old_of(xq, j) - P.tdx * (Fq[j + 1] - Fq[j]);
      eq[j] = xq[j + 2];
    }
  }
  if (STAGE == 2) __syncthreads();
  put_round(2);
  load_round(3);
  __syncthreads();
  // round m: m-dagger before the relaxation term; with a bed the m-diffusion
  // subtracts the jump of the face-local rest moment (zeta_f - b)^2, formed
  // here from the depths kept since the h round and the staged bed (held
  // from the h round instead, the jumps spilled registers in stage 2)
  double mdp[K], em[K];
  if (act) {
    save_side(2);
    double xm[K + 4], xb[K + 4], Fm[K + 1];
    read_x(xm, ebuf(2));
    if (BED && useb) {
      read_x(xb, L.u.st.b);
    } else {
#pragma unroll
      for (int i = 0; i < K + 4; ++i) xb[i] = 0.0;
    }
#pragma unroll
    for (int f = 0; f <= K; ++f) {
      const double mL = xm[f + 1] + P.sl * (xm[f + 2] - xm[f]);
      const double mR = xm[f + 2] - P.sl * (xm[f + 3] - xm[f + 1]);
      double jm = mR - mL;
      if (BED) {
        const double zf = 0.5 * ((hf[f] + xb[f + 1]) + (hf[f + 1] + xb[f + 2]));
        const double rm = (zf - xb[f]) * (zf - xb[f]);
        const double r0 = (zf - xb[f + 1]) * (zf - xb[f + 1]);
        const double r1 = (zf - xb[f + 2]) * (zf - xb[f + 2]);
        const double r2 = (zf - xb[f + 3]) * (zf - xb[f + 3]);
        const double mhL = r0 + P.sl * (r1 - rm);
        const double mhR = r1 - P.sl * (r2 - r0);
        jm = jm - (mhR - mhL);
      }
      Fm[f] = 0.5 * (mL * uL[f] + mR * uR[f] - ap[f] * jm);
    }
#pragma unroll
    for (int j = 0; j < K; ++j) {
      double md = old_of(xm, j) - P.tdx * (Fm[j + 1] - Fm[j]);
      if (BED) {
        const double db = xb[j + 3] - xb[j + 1];
        md -= P.tau * 1.5 * eq[j] * (db * i2dx);
      }
      mdp[j] = md;
      em[j] = xm[j + 2];
    }
  }
  if (STAGE == 2) __syncthreads();
  put_round(3);
  asm volatile("" ::"v"(ahead));
  __syncthreads();
  // round W: W-dagger, m-dagger, and the rows' frozen coefficients
  Rec rec[K];
  Rec recL, recR;
  if (act) {
    save_side(3);
    double xw[K + 4], Fw[K + 1];
    read_x(xw, ebuf(3));
#pragma unroll
    for (int f = 0; f <= K; ++f) {
      const double WL = xw[f + 1] + P.sl * (xw[f + 2] - xw[f]);
      const double WR = xw[f + 2] - P.sl * (xw[f + 3] - xw[f + 1]);
      Fw[f] = 0.5 * (WL * uL[f] + WR * uR[f] - ap[f] * (WR - WL));
    }
    bad |= (badf & 1u) != 0;
#pragma unroll
    for (int j = 0; j < K; ++j) {
      Rec r;
      r.Wd = old_of(xw, j) - P.tdx * (Fw[j + 1] - Fw[j]) + P.lam * P.tau;
      r.md = mdp[j] + P.tau * r.Wd;
      r.qd = qd[j];
      bool bj = ((badf >> (j + 1)) & 1u) != 0, nj = false;  // flags of padding rows are dropped
      rec_coefs_fast<BED>(r, hf[j + 1], em[j], bed_row(j + 1), P, bj, nj);
      rec[j] = r;
      if (p0 + j < wd.wl) {
        bad |= bj;
        noncoer |= nj;
      }
    }
  }
  // outer neighbours (row -1 and row wl) of truncated edges: record of the
  // row from its five cells and its old state, as copied aside (side 0 left,
  // side 1 right)
  auto outer_record = [&](int sd, double& hrow) -> Rec {
    Cell c[5];
    double bb[5];
#pragma unroll
    for (int d = 0; d < 5; ++d) {
      c[d].h = L.side[sd][0][d];
      c[d].q = L.side[sd][1][d];
      c[d].m = L.side[sd][2][d];
      c[d].W = L.side[sd][3][d];
      bb[d] = L.sideb[sd][d];
    }
    const Flux Fa = face_flux_fast<BED>(c[0], c[1], c[2], c[3], bb[0], bb[1], bb[2], bb[3], P.g,
                                        P.sl, bad);
    const Flux Fb = face_flux_fast<BED>(c[1], c[2], c[3], c[4], bb[1], bb[2], bb[3], bb[4], P.g,
                                        P.sl, bad);
    Cell o;
    o.h = L.sideo[sd][0];
    o.q = L.sideo[sd][1];
    o.m = L.sideo[sd][2];
    o.W = L.sideo[sd][3];
    hrow = c[2].h;
    return cell_record_fast<BED>(c[2], o, Fa, Fb, bb[1], bb[2], bb[3], P, i2dx, bad, noncoer);
  };
  if (act && t == 0) {
    if (physL) {
      recL = rec[0];
    } else {
      double hg;
      recL = outer_record(0, hg);
      L.misc[0] = hg;  // depth guess beyond the left edge
    }
  }
  if (act && t == na - 1) {
    const int jl = wd.wl - 1 - p0;  // last real row in this thread (0..K-1)
    Rec last = rec[0];
#pragma unroll
    for (int j = 0; j < K; ++j)
      if (j == jl) last = rec[j];
    if (physR) {
      recR = last;
    } else {
      double hg;
      recR = outer_record(1, hg);
      L.misc[1] = hg;  // depth guess beyond the right edge
    }
  }
  __syncthreads();  // the staging buffers are reused below
  // share chunk-end records
  if (act) {
    L.u.nb.beta[0][t] = rec[0].beta; L.u.nb.S[0][t] = rec[0].S; L.u.nb.qd[0][t] = rec[0].qd;
    L.u.nb.phi[0][t] = rec[0].phi; L.u.nb.T[0][t] = rec[0].T;
    if (!kLean) L.u.nb.b[0][t] = rec[0].b;
    L.u.nb.beta[1][t] = rec[K - 1].beta; L.u.nb.S[1][t] = rec[K - 1].S;
    L.u.nb.qd[1][t] = rec[K - 1].qd; L.u.nb.phi[1][t] = rec[K - 1].phi;
    L.u.nb.T[1][t] = rec[K - 1].T;
    if (!kLean) L.u.nb.b[1][t] = rec[K - 1].b;
  }
  __syncthreads();
  if (act && t > 0) {
    recL.beta = L.u.nb.beta[1][t - 1]; recL.S = L.u.nb.S[1][t - 1]; recL.qd = L.u.nb.qd[1][t - 1];
    recL.phi = L.u.nb.phi[1][t - 1]; recL.T = L.u.nb.T[1][t - 1];
    if (!kLean) recL.b = L.u.nb.b[1][t - 1];
  }
  if (act && t < na - 1) {
    recR.beta = L.u.nb.beta[0][t + 1]; recR.S = L.u.nb.S[0][t + 1]; recR.qd = L.u.nb.qd[0][t + 1];
    recR.phi = L.u.nb.phi[0][t + 1]; recR.T = L.u.nb.T[0][t + 1];
    if (!kLean) recR.b = L.u.nb.b[0][t + 1];
  }
  // The last active thread may own padding rows after its last real row jl;
  // their records are never used, so the slot after row jl takes recR, the
  // right neighbour of row jl, and the rows and the back-substitution below
  // read rec[j + 1] for every j < K - 1 without a per-row select.  Only the
  // wave holding that thread takes this branch.
  if (act) {
    const int jl = wd.wl - 1 - p0;
    if (jl < K - 1) {
#pragma unroll
      for (int j = 0; j < K - 1; ++j)
        if (j == jl) rec[j + 1] = recR;
    }
  }
  const double gL = L.misc[0], gR = L.misc[1];
  __syncthreads();  // nb region is reused by the level-1 system below

  // ---- rows and chunk elimination (K rows per thread, all real or identity)
  constexpr bool kStash = STAGE == 2 && BED;
  double cp[K], y[K], v[K], w[K];
  double loE = 0.0, upE = 0.0;  // couplings moved to the right-hand side
  if (act) {
    const int jl = wd.wl - 1 - p0;  // last real row of this thread (>= K-1 if full)
    double r0[4], rl[4];
    double cprev = 0.0, yprev = 0.0, vprev = 1.0, wprev = 0.0;
#pragma unroll
    for (int j = 0; j < K; ++j) {
      const bool real = j <= jl;
      const Rec Lr = (j == 0) ? recL : rec[j > 0 ? j - 1 : 0];
      const Rec Rr = (j == K - 1) ? recR : rec[j + 1 < K ? j + 1 : K - 1];
      double lo, di, up, rhs;
      // lean form: the beds of the row and its neighbours come from the
      // staged bed (the records carry no copy of it)
      Rec Lb = Lr, Cb = rec[j], Rb = Rr;
      if (kLean) {
        Lb.b = bed_row(j);
        Cb.b = bed_row(j + 1);
        Rb.b = bed_row(j + 2);
      }
      make_row<BED>(Lb, Cb, Rb, L.u.st.ho[spad(p0 + 3 + j)], P, lo, di, up, rhs);
      if (kStash) {
        // m-dagger and W-dagger wait in this row's slots of the old-depth and
        // bed buffers (read by no one after the rows) until the
        // back-substitution, instead of in registers through the solve
        L.u.st.ho[spad(p0 + 3 + j)] = rec[j].Wd;
        L.u.st.b[spad(p0 + 3 + j)] = rec[j].md;
      }
      if (t == 0 && j == 0) {
        if (physL) {
          di += lo;
        } else {
          loE = lo;
          rhs -= lo * gL;
        }
        lo = 0.0;
      }
      if (t == na - 1 && j == jl) {
        if (physR) {
          di += up;
        } else {
          upE = up;
          rhs -= up * gR;
        }
        up = 0.0;
      }
      if (!real) {
        lo = 0.0; di = 1.0; up = 0.0; rhs = 0.0;
      }
      if (j == 0) {
        r0[0] = lo; r0[1] = di; r0[2] = up; r0[3] = rhs;
      } else if (j == K - 1) {
        rl[0] = lo; rl[1] = di; rl[2] = up; rl[3] = rhs;
      } else {
        const double inv = frcp(di - lo * cprev);
        const bool lastint = (j == K - 2);
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
    double yn = 0.0, vn = 0.0, wn = 0.0;
#pragma unroll
    for (int j = K - 2; j >= 1; --j) {
      y[j] = y[j] - cp[j] * yn;
      v[j] = v[j] - cp[j] * vn;
      w[j] = w[j] - cp[j] * wn;
      yn = y[j];
      vn = v[j];
      wn = w[j];
    }
    double R0[4], R1[4];
    if (K > 2) {
      R0[0] = r0[0];
      R0[1] = r0[1] + r0[2] * v[1];
      R0[2] = r0[2] * w[1];
      R0[3] = r0[3] - r0[2] * y[1];
      R1[0] = rl[0] * v[K - 2];
      R1[1] = rl[1] + rl[0] * w[K - 2];
      R1[2] = rl[2];
      R1[3] = rl[3] - rl[0] * y[K - 2];
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        R0[e] = r0[e];
        R1[e] = rl[e];
      }
    }
    Lds<NT>& S = L.u.sys;
    S.a[2 * t] = R0[0]; S.b[2 * t] = R0[1]; S.c[2 * t] = R0[2]; S.d0[2 * t] = R0[3];
    S.d1[2 * t] = 0.0; S.d2[2 * t] = 0.0;
    S.a[2 * t + 1] = R1[0]; S.b[2 * t + 1] = R1[1]; S.c[2 * t + 1] = R1[2];
    S.d0[2 * t + 1] = R1[3]; S.d1[2 * t + 1] = 0.0; S.d2[2 * t + 1] = 0.0;
    if (t == 0) L.misc[2] = loE;
    if (t == na - 1) L.misc[3] = upE;
  }
  // ---- level-1 system (rows 2t, 2t + 1 of every active thread).  It yields
  // the depths zf, zb of this thread's two level-1 rows and their
  // derivatives with respect to the left and right edge guesses.
  const int n1 = 2 * na;
  double zf = 0.0, zb = 0.0, GfL = 0.0, GfR = 0.0, GbL = 0.0, GbR = 0.0;
  // Windows of 256 threads solve it by wavefront segments: wavefront w
  // eliminates the interior of its rows [128 w, 128 w + 128) by PCR (no
  // workgroup barrier), one thread solves the system of the segments' end
  // unknowns (two per wavefront), and every row follows from its segment's
  // ends.  Windows of 512 threads (16 end unknowns for the one thread)
  // measured faster with the workgroup-wide PCR of the interior rows in
  // terms of the window's two end unknowns.
  constexpr bool kWaveSeg = NT <= 256;
  if constexpr (kWaveSeg) {
    const int wv = t >> 6, ln = t & 63;
    const int F = 128 * wv, E = min(F + 127, n1 - 1);
    wave_lds_sync();  // this wavefront's rows are written
    if (F < n1) {
      segment_pcr<NT>(L.u.sys, F, E, ln);
      if (ln == 0) {
        double R0[4], R1[4];
        segment_ends<NT>(L.u.sys, F, E, R0, R1);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          L.l2[e][2 * wv] = R0[e];
          L.l2[e][2 * wv + 1] = R1[e];
        }
      }
    }
    __syncthreads();
    if (t == 0) {
      // Thomas on the end unknowns, for the right-hand side and for unit
      // changes of the edge guesses (the left guess enters the first row as
      // -loE, the right guess the last row as -upE)
      const int nr = 2 * ((n1 + 127) / 128);
      const double loE = L.misc[2], upE = L.misc[3];
      double cp = 0.0, y0 = 0.0, yl = 0.0, yr = 0.0;
      for (int k = 0; k < nr; ++k) {
        const double lo = L.l2[0][k];
        const double inv = frcp(L.l2[1][k] - lo * cp);
        cp = L.l2[2][k] * inv;
        L.l2[2][k] = cp;
        y0 = (L.l2[3][k] - lo * y0) * inv;
        yl = ((k == 0 ? -loE : 0.0) - lo * yl) * inv;
        yr = ((k == nr - 1 ? -upE : 0.0) - lo * yr) * inv;
        L.l2x[0][k] = y0;
        L.l2x[1][k] = yl;
        L.l2x[2][k] = yr;
      }
      for (int k = nr - 2; k >= 0; --k) {
        const double c = L.l2[2][k];
        y0 = L.l2x[0][k] - c * y0;
        yl = L.l2x[1][k] - c * yl;
        yr = L.l2x[2][k] - c * yr;
        L.l2x[0][k] = y0;
        L.l2x[1][k] = yl;
        L.l2x[2][k] = yr;
      }
    }
    __syncthreads();
    if (act) {
      const Lds<NT>& S = L.u.sys;
      const double uF = L.l2x[0][2 * wv], uE = L.l2x[0][2 * wv + 1];
      const double lF = L.l2x[1][2 * wv], lE = L.l2x[1][2 * wv + 1];
      const double rF = L.l2x[2][2 * wv], rE = L.l2x[2][2 * wv + 1];
      const int j0 = 2 * t, j1 = 2 * t + 1;
      if (j0 == F) {
        zf = uF; GfL = lF; GfR = rF;
      } else {
        const double V = S.d1[j0], Wv = S.d2[j0];
        zf = S.d0[j0] + V * uF + Wv * uE;
        GfL = V * lF + Wv * lE;
        GfR = V * rF + Wv * rE;
      }
      if (j1 == E) {
        zb = uE; GbL = lE; GbR = rE;
      } else {
        const double V = S.d1[j1], Wv = S.d2[j1];
        zb = S.d0[j1] + V * uF + Wv * uE;
        GbL = V * lF + Wv * lE;
        GbR = V * rF + Wv * rE;
      }
    }
  } else {
    __syncthreads();
    level1_interior_fast<NT>(L.u.sys, n1, t);
    // the window's end unknowns (couplings already on the right-hand side)
    if (t == 0) {
      double R0[4], R1[4];
      tile_rows<NT>(L.u.sys, n1, R0, R1);
      const double m00 = R0[1], m01 = R0[2], m10 = R1[0], m11 = R1[1];
      const double idet = 1.0 / (m00 * m11 - m01 * m10);
      const double i00 = m11 * idet, i01 = -m01 * idet, i10 = -m10 * idet, i11 = m00 * idet;
      L.misc[4] = i00 * R0[3] + i01 * R1[3];  // z0
      L.misc[5] = i10 * R0[3] + i11 * R1[3];  // zl
      // d(z0, zl)/d(guess): left guess enters row 0 as -loE, right as -upE
      L.misc[6] = -L.misc[2] * i00;
      L.misc[7] = -L.misc[2] * i10;
      L.misc[8] = -L.misc[3] * i01;
      L.misc[9] = -L.misc[3] * i11;
    }
    __syncthreads();
    if (act) {
      const double z0 = L.misc[4], zl = L.misc[5];
      const double dz0L = L.misc[6], dzlL = L.misc[7], dz0R = L.misc[8], dzlR = L.misc[9];
      const Lds<NT>& S = L.u.sys;
      const int j0 = 2 * t, j1 = 2 * t + 1;
      double Vf, Wf, Vb, Wb;  // d(zf, zb) / d(z0, zl)
      if (j0 == 0) { zf = z0; Vf = 1.0; Wf = 0.0; }
      else { zf = S.d0[j0] + S.d1[j0] * z0 + S.d2[j0] * zl; Vf = S.d1[j0]; Wf = S.d2[j0]; }
      if (j1 == n1 - 1) { zb = zl; Vb = 0.0; Wb = 1.0; }
      else { zb = S.d0[j1] + S.d1[j1] * z0 + S.d2[j1] * zl; Vb = S.d1[j1]; Wb = S.d2[j1]; }
      GfL = Vf * dz0L + Wf * dzlL;
      GfR = Vf * dz0R + Wf * dzlR;
      GbL = Vb * dz0L + Wb * dzlL;
      GbR = Vb * dz0R + Wb * dzlR;
    }
    __syncthreads();  // every thread has read its rows before a[] takes the depths
  }
  if (act) {
    // a[] of this thread's rows takes their depths (no other thread reads
    // this thread's rows at this point)
    L.u.sys.a[2 * t] = zf;
    L.u.sys.a[2 * t + 1] = zb;
  }
  __syncthreads();

  // ---- back-substitution over the core rows
  double smax = 0.0, umax = 0.0;
  double on[4][K];  // new state of this thread's rows (core rows only are stored)
  const int c0 = wd.cs - wd.ws;    // first core row (window-relative)
  const int c1 = c0 + wd.cl;       // one past the last core row
  const bool has_core = act && p0 < c1 && p0 + K > c0;
  if (has_core) {
    const double hl_nb = (t > 0) ? L.u.sys.a[2 * t - 1] : (physL ? zf : gL);
    const double hr_nb = (t < na - 1) ? L.u.sys.a[2 * t + 2] : (physR ? zb : gR);
    double hb[K];
#pragma unroll
    for (int j = 0; j < K; ++j)
      hb[j] = (j == 0) ? zf : ((j == K - 1) ? zb : y[j] + v[j] * zf + w[j] * zb);
    const int jl = wd.wl - 1 - p0;
    // certificate at the core's edge rows
    if ((truncL || truncR) && ((p0 <= c0 && c0 < p0 + K) || (p0 <= c1 - 1 && c1 - 1 < p0 + K))) {
      const double X = 4.0 * fmax(fabs(gL), fabs(gR));
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const int p = p0 + j;
        if (p == c0 || p == c1 - 1) {
          double sgL, sgR;  // d x_p / d (left guess), d x_p / d (right guess)
          if (j == 0) { sgL = GfL; sgR = GfR; }
          else if (j == K - 1) { sgL = GbL; sgR = GbR; }
          else { sgL = v[j] * GfL + w[j] * GbL; sgR = v[j] * GfR + w[j] * GbR; }
          const double sens = fabs(sgL) + fabs(sgR);
          if (!(sens * X <= 1.3877787807814457e-17 * fabs(hb[j]))) {  // 2^-56
            atomicOr(&A.status[wd.inst], kFlagWindow);
          }
        }
      }
    }
#pragma unroll
    for (int j = 0; j < K; ++j) {
      const int p = p0 + j;
      if (p >= c0 && p < c1) {
        const Rec Lr = (j == 0) ? recL : rec[j > 0 ? j - 1 : 0];
        const Rec Rr = (j == K - 1) ? recR : rec[j + 1 < K ? j + 1 : K - 1];
        const double hm = (j == 0) ? hl_nb : hb[j > 0 ? j - 1 : 0];
        const double hp = (j == K - 1) ? hr_nb : ((j == jl && physR) ? hb[j] : hb[j + 1 < K ? j + 1 : K - 1]);
        const double h = hb[j];
        const double Pm = Lr.S + Lr.beta * hm;
        const double Pp = Rr.S + Rr.beta * hp;
        double force = (Pp - Pm) * i2dx;
        if (BED) {
          const double dbc = (kLean ? bed_row(j + 2) - bed_row(j) : Rr.b - Lr.b) * i2dx;
          const double pti = rec[j].T + rec[j].phi * h;
          force += 0.5 * P.g * (hp + hm) * dbc + 1.5 * pti * dbc;
        }
        const double qn = rec[j].qd - P.tau * force;
        const double ih = frcp(h);
        const double ih2 = ih * ih;
        const double md = kStash ? L.u.st.b[spad(p0 + 3 + j)] : rec[j].md;
        const double Wd = kStash ? L.u.st.ho[spad(p0 + 3 + j)] : rec[j].Wd;
        const double mn = md * frcp(1.0 + P.lt2 * ih2);
        const double Wn = Wd - P.lam * P.tau * mn * ih2;
        bad |= !(h > 0.0) || !isfinite(qn) || !isfinite(mn) || !isfinite(Wn);
        on[0][j] = h;
        on[1][j] = qn;
        on[2][j] = mn;
        on[3][j] = Wn;
        if (STAGE == 2) {
          const double u = fabs(qn * ih);
          smax = fmax(smax, u + fsqrt(P.g * h));
          umax = fmax(umax, u);
        }
      }
    }
  }
  // ---- coalesced stores of the core through LDS: two fields per round in
  // the staging buffers e and o, or (with a bed) all four in one round, the bed
  // and old-depth buffers being free by now.  The stores are non-temporal: the
  // stage's output is next read a whole launch later, far beyond what the
  // caches hold (measured: stage 2 -14 % on a flat periodic 2^24-cell mesh,
  // -0.6 % on the batched bar; the per-row phi stores of the SGN solve, which
  // are not coalesced, became slower this way, so they stay ordinary)
  __syncthreads();  // level-1 values (a) are no longer read
  double* out[4] = {A.o_h, A.o_q, A.o_m, A.o_W};
  constexpr int NS = (WN + NT - 1) / NT;
  constexpr bool kOneRound = BED;
  constexpr int kPer = kOneRound ? 4 : 2;
  double* const sb[4] = {L.u.st.e, L.u.st.o, kOneRound ? L.u.st.b : L.u.st.e, L.u.st.ho};
#pragma unroll
  for (int f = 0; f < 4; f += kPer) {
    if (has_core) {
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const int p = p0 + j;
        if (p >= c0 && p < c1) {
#pragma unroll
          for (int e = 0; e < kPer; ++e) sb[e][spad(p)] = on[f + e][j];
        }
      }
    }
    __syncthreads();
    if (STAGE == 2) {
      // two consecutive cells per lane, one 16-byte store (8-byte alignment
      // suffices for global memory on this target); a pair that wraps around
      // a periodic ring, or a last odd cell, is stored one cell at a time
      // (measured: stage 2 -2.8 %; stage 1, whose records live in fewer
      // registers, +0.7 %, and +0.2 % again once the stores were
      // non-temporal, so it keeps single-cell stores)
      typedef double d2a8 __attribute__((ext_vector_type(2), aligned(8)));
      static_assert(NS % 2 == 0, "paired stores cover the window in NS / 2 rounds");
#pragma unroll
      for (int r = 0; r < NS / 2; ++r) {
        const int i = 2 * (t + r * NT);
        if (i < wd.cl) {
          int c = wd.cs + i;
          if (c >= n) c -= n;
          if (i + 1 < wd.cl && c + 1 < n) {
#pragma unroll
            for (int e = 0; e < kPer; ++e) {
              d2a8 v;
              v.x = sb[e][spad(c0 + i)];
              v.y = sb[e][spad(c0 + i + 1)];
              __builtin_nontemporal_store(v, (d2a8*)(out[f + e] + base + c));
            }
          } else {
            int c1 = c + 1;
            if (c1 >= n) c1 -= n;
#pragma unroll
            for (int e = 0; e < kPer; ++e) {
              __builtin_nontemporal_store(sb[e][spad(c0 + i)], out[f + e] + base + c);
              if (i + 1 < wd.cl)
                __builtin_nontemporal_store(sb[e][spad(c0 + i + 1)], out[f + e] + base + c1);
            }
          }
        }
      }
    } else {
#pragma unroll
      for (int r = 0; r < NS; ++r) {
        const int i = t + r * NT;
        if (i < wd.cl) {
          int c = wd.cs + i;
          if (c >= n) c -= n;
#pragma unroll
          for (int e = 0; e < kPer; ++e)
            __builtin_nontemporal_store(sb[e][spad(c0 + i)], out[f + e] + base + c);
        }
      }
    }
    __syncthreads();
  }
  if (STAGE == 2) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      smax = fmax(smax, __shfl_xor(smax, off));
      umax = fmax(umax, __shfl_xor(umax, off));
    }
    if ((t & 63) == 0 && smax > 0.0) {
      atomicMax(&A.smax[wd.inst], (unsigned long long)__double_as_longlong(smax));
      atomicMax(&A.umax[wd.inst], (unsigned long long)__double_as_longlong(umax));
    }
  }
  if (bad || noncoer) {
    atomicOr(&A.status[wd.inst], (bad ? kFlagNonPhys : 0) | (noncoer ? kFlagNonCoercive : 0));
  }
}

// Stage kernel, one window per workgroup: consecutive windows of an
// instance run on the same XCD (blocks are dealt round-robin over the 8
// XCDs), so the halo rows they share hit that XCD's L2.
template <int NT, int K, bool BED, int STAGE>
__global__ __launch_bounds__(NT, NT <= 256 ? 2 : 1) void k_win(WinArgs W) {
  __shared__ WinLds<NT, K, BED> L;
  int bid = blockIdx.x;
  if (W.xcd_stride > 0) {
    const int x = bid & 7, r = bid >> 3;
    bid = x * W.xcd_stride + r;
  }
  if (bid >= W.nwin) return;
  win_one<NT, K, BED, STAGE>(W, L, bid, threadIdx.x);
}

// Persistent stage kernel: a grid of as many workgroups as are resident at
// once (a multiple of 8) walks the windows through eight work queues, one
// per XCD.  Queue x holds the contiguous window range [x stride,
// (x + 1) stride), so consecutive windows of an instance stay on one XCD
// (blocks are dealt round-robin over the XCDs).  A workgroup takes windows
// from its own XCD's queue (one atomic ticket per window), then from the
// others in turn; every workgroup ends once all eight are exhausted, and the
// last to end resets the nine counters (queue[8] counts ended workgroups),
// so the next launch, or graph replay, starts from zero.
template <int NT, int K, bool BED, int STAGE>
__global__ __launch_bounds__(NT, NT <= 256 ? 2 : 1) void k_win_persist(WinArgs W) {
  __shared__ WinLds<NT, K, BED> L;
  __shared__ int ticket;
  const int x = blockIdx.x & 7;
  for (int k = 0; k < 8; ++k) {
    const int q = (x + k) & 7;
    const int lo = q * W.xcd_stride;
    const int hi = min(W.nwin, lo + W.xcd_stride);
    while (true) {
      __syncthreads();  // the previous window is done with the LDS and the ticket
      if (threadIdx.x == 0) ticket = atomicAdd(&W.queue[q], 1);
      __syncthreads();
      const int w = lo + ticket;
      if (w >= hi) break;
      // the arguments are read again from the kernel-argument segment in
      // every iteration (the pointer is made opaque), so the compiler does
      // not keep them in scalar registers across the loop; likewise the
      // thread index, so that no address derived from it is hoisted out of
      // the loop and held in vector registers
      typedef const WinArgs __attribute__((address_space(4)))* KargPtr;
      KargPtr Wp = (KargPtr)__builtin_amdgcn_kernarg_segment_ptr();
      asm volatile("" : "+s"(Wp));
      int tid = threadIdx.x;
      asm volatile("" : "+v"(tid));
      win_one<NT, K, BED, STAGE>(*(const WinArgs*)Wp, L, w, tid);
    }
  }
  if (threadIdx.x == 0) {
    __threadfence();
    if (atomicAdd(&W.queue[8], 1) == (int)gridDim.x - 1) {
#pragma unroll
      for (int i = 0; i < 9; ++i) atomicExch(&W.queue[i], 0);
    }
  }
}

}  // namespace hsgn
