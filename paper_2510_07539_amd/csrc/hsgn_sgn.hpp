// hsgn_sgn.hpp -- the standard SGN equations in elliptic-hyperbolic form
// (Sec. 4.3-4.4), flat bottom, Heun's method: the phi solve (windowed single
// pass, or exact on the two-pass tiling) and the flux update, for the cost
// comparison the paper makes against the hSGN relaxation.
#pragma once

#include "hsgn_kernels.hpp"
#include "hsgn_window.hpp"
#include "hsgn_adjoint.hpp"
#include "hsgn_explicit.hpp"

namespace hsgn {

// The SGN update kernels walk the same 1024-cell tiles with 512 threads of two
// cells each: measured faster for them than 256 x 4, unlike k_ex.
constexpr int kSgnNT = 512;
constexpr int kSgnK = 2;
static_assert(kSgnNT * kSgnK == kExTile, "SGN and explicit kernels share one tile list");

// ---------------------------------------------------------------------------
// Standard SGN equations, elliptic-hyperbolic form (Sec. 4.3-4.4), flat
// bottom, Heun's method.  Per stage, the phi solve forms the tridiagonal
// system of phi,
//   h_i phi_i - (H_{i+1/2}(phi_{i+1} - phi_i) - H_{i-1/2}(phi_i - phi_{i-1})) / (3 dx^2)
//     = h*_i = -(G_{i+1} - G_{i-1}) / (6 dx^3),
//   H_{i+1/2} = (h_i^3 + h_{i+1}^3) / 2,
//   G_j = g h_j^3 (h_{j+1} - 2 h_j + h_{j-1}) + (h_j^3 / 2)(u_{j+1} - u_{j-1})^2,
// (zero-gradient phi at transmissive ends; cyclic when periodic) and solves
// it, in windows (k_sgn_win) or exactly on the two-pass tiling (k_sgn_tri);
// k_sgn_update applies
//   L_h = -Dhat_x(q),  L_q = -Dhat_x(q u + g h^2 / 2) + h phi
// with Rusanov fluxes (speed max(|u| + sqrt(g h))) on the linear
// reconstruction of (h, q).  m and W are carried unchanged.
// ---------------------------------------------------------------------------
struct SgnArgs {
  const double* __restrict__ un_h;  // U^n (stage 2; also the m, W carried along)
  const double* __restrict__ un_q;
  const double* __restrict__ un_m;
  const double* __restrict__ un_W;
  const double* __restrict__ in_h;  // stage operand
  const double* __restrict__ in_q;
  double* __restrict__ o_h;         // stage output
  double* __restrict__ o_q;
  double* __restrict__ o_m;
  double* __restrict__ o_W;
  const double* __restrict__ phi;   // solution (k_sgn_update)
  const InstDesc* __restrict__ inst;
  const TileDesc* __restrict__ tiles;
  const double* __restrict__ dt;
  unsigned long long* __restrict__ smax;
  unsigned long long* __restrict__ umax;
  int32_t* __restrict__ status;
};

// Stage h and q of tile cells -2 .. len + 1 (wrapped or copied ghosts).
template <int NT, int SL>
__device__ __forceinline__ void sgn_stage(double (*X)[SL], const double* __restrict__ h,
                                          const double* __restrict__ q, const InstDesc& I,
                                          const TileDesc& td) {
  const int t = threadIdx.x;
#pragma unroll
  for (int r = 0; r < (SL + NT - 1) / NT; ++r) {
    const int si = t + r * NT;
    if (si < td.len + 4) {
      int c = td.start - 2 + si;
      if (I.bc == 0) c = c < 0 ? c + I.n : (c >= I.n ? c - I.n : c);
      else c = c < 0 ? 0 : (c > I.n - 1 ? I.n - 1 : c);
      X[0][si] = h[I.off + c];
      X[1][si] = q[I.off + c];
    }
  }
}

// Solve of the phi system on the two-pass tiling (tiles of at most NT * K
// rows), with the rows formed in the solve: the tile stages h and q of its
// cells and two ghost cells per side, each thread forms the rows of its
// chunk (H, G and h^3 from the staged cells, the expressions above) and
// eliminates them in registers, and the tile continues as an exact tiled
// solve.  REDUCE: the tile writes its two reduced rows for the per-instance
// reduced solve (k_rsolve).  Otherwise the tile takes its end unknowns from
// that solve (or solves them itself when it is the whole instance) and
// writes phi.  The rows never go through global memory.
struct SgnTriArgs {
  const InstDesc* __restrict__ inst;
  const TileDesc* __restrict__ tiles;
  const double* __restrict__ dt;
  const double* __restrict__ h;  // stage operand
  const double* __restrict__ q;
  double* __restrict__ phi;
  double* __restrict__ rlo;  // reduced rows (2 per tile at red_off + 2 tidx)
  double* __restrict__ rdi;
  double* __restrict__ rup;
  double* __restrict__ rrhs;
  const double* __restrict__ rx;  // reduced solution
  int32_t* __restrict__ status;
};

// Rows of the phi system (the expressions above) for a chunk of k rows
// starting at row f, from h and q staged with two ghost cells per side
// (staged index = row + 2), in one pass over the stencil cells: row ii needs
// h at rows ii - 1 .. ii + 1 and G at rows ii - 1 and ii + 1, so only three
// h and u values and two G values are live at a time (the whole stencil kept
// at once spills registers).  Past the chunk's last stencil cell f + k + 3
// the last one repeats.  edit(ii, l, d, u) applies the boundary rules of row
// ii.  Slot K - 1 receives row k - 1 (the chunk's last row, where the
// elimination takes it).  Returns whether a depth of the chunk is not > 0.
template <int K, class Edit>
__device__ __forceinline__ bool sgn_chunk_rows(const double* Xh, const double* Xq, int f, int k,
                                               double g, double c3, double c6, double (&Lo)[K],
                                               double (&Di)[K], double (&Up)[K], double (&Rh)[K],
                                               Edit edit) {
  auto cell = [&](int i, double& hh, double& uu) {
    const int si = f + (i < k + 4 ? i : k + 3);
    hh = Xh[spad(si)];
    uu = Xq[spad(si)] / hh;
  };
  auto gfun = [&](double hm, double h0, double hp, double um, double up) {
    const double du = up - um;
    const double c = h0 * h0 * h0;
    return g * c * (hp - 2.0 * h0 + hm) + 0.5 * c * du * du;
  };
  bool bad = false;
  double hA, hB, hC, uA, uB, uC, hX, uX;
  cell(0, hX, uX);
  cell(1, hA, uA);
  cell(2, hB, uB);
  cell(3, hC, uC);
  double Gm = gfun(hX, hA, hB, uX, uB);  // G at staged cell 1
  double G0 = gfun(hA, hB, hC, uA, uC);  // G at staged cell 2
#pragma unroll
  for (int ii = 0; ii < K; ++ii) {  // hA, hB, hC: h at staged cells ii + 1 .. ii + 3
    double hD, uD;
    cell(ii + 4, hD, uD);
    const double Gp = gfun(hB, hC, hD, uB, uD);
    const double cA = hA * hA * hA, cB = hB * hB * hB, cC = hC * hC * hC;
    const double Hm = 0.5 * (cA + cB);
    const double Hp = 0.5 * (cB + cC);
    double l = -c3 * Hm, u = -c3 * Hp, d = hB + c3 * (Hm + Hp);
    const double rh = -(Gp - Gm) * c6;
    edit(ii, l, d, u);
    if (ii < k) bad |= !(hB > 0.0);
    if (ii < K - 1 || k == K) {
      Lo[ii] = l;
      Di[ii] = d;
      Up[ii] = u;
      Rh[ii] = rh;
    }
    if (ii < K - 1 && ii == k - 1) {
      Lo[K - 1] = l;
      Di[K - 1] = d;
      Up[K - 1] = u;
      Rh[K - 1] = rh;
    }
    Gm = G0;
    G0 = Gp;
    hA = hB; hB = hC; hC = hD;
    uA = uB; uB = uC; uC = uD;
  }
  return bad;
}

template <int NT, int K>
struct SgnTriLds {
  static constexpr int SL = NT * K + 4;          // staged cells: rows and two ghosts per side
  static constexpr int SP = SL + (SL >> 3) + 1;  // padded (one pad double after every 8)
  union {
    double X[2][SP];  // h, q; staged index s <-> tile cell s - 2
    Lds<NT> S;        // the level-1 system, once every chunk has its rows
  } u;
};

// Four workgroups per CU (at most 128 registers per lane; 37 KB of LDS
// each): measured 15 % faster than the 136 registers, three workgroups per
// CU, that the compiler picks by itself.
template <int NT, int K, bool REDUCE>
__global__ __launch_bounds__(NT, 4) void k_sgn_tri(SgnTriArgs P) {
  using LT = SgnTriLds<NT, K>;
  __shared__ LT L;
  const TileDesc td = P.tiles[blockIdx.x];
  const InstDesc I = P.inst[td.inst];
  if (!(P.dt[td.inst] > 0.0)) return;  // frozen: phi is not used
  const int t = threadIdx.x, len = td.len;
#pragma unroll
  for (int r = 0; r < (LT::SL + NT - 1) / NT; ++r) {
    const int si = t + r * NT;
    if (si < len + 4) {
      int c = td.start - 2 + si;
      if (I.bc == 0) c = c < 0 ? c + I.n : (c >= I.n ? c - I.n : c);
      else c = c < 0 ? 0 : (c > I.n - 1 ? I.n - 1 : c);
      L.u.X[0][spad(si)] = P.h[I.off + c];
      L.u.X[1][spad(si)] = P.q[I.off + c];
    }
  }
  __syncthreads();
  const Chunk ch = chunk_of(len, NT, t);
  double Lo[K], Di[K], Up[K], Rh[K];
  bool bad = false;
  if (t < ch.active) {
    const int k = ch.k, f = ch.first;
    const double g = I.g;
    const double c3 = 1.0 / (3.0 * I.dx * I.dx);
    const double c6 = 1.0 / (6.0 * I.dx * I.dx * I.dx);
    bad = sgn_chunk_rows<K>(L.u.X[0], L.u.X[1], f, k, g, c3, c6, Lo, Di, Up, Rh,
                            [&](int ii, double& l, double& d, double& u) {
                              if (I.bc != 0) {  // zero-gradient phi at a transmissive end
                                const int c = td.start + f + ii;
                                if (c == 0) { d += l; l = 0.0; }
                                if (c == I.n - 1) { d += u; u = 0.0; }
                              }
                            });
  }
  __syncthreads();  // the staged cells are dead: the union holds the level-1 system
  Lds<NT>& S = L.u.S;
  double y[K], v[K], w[K];
  reg_chunk_elim_rows<NT, K>(
      S, len, y, v, w,
      [&](int, int, double (&lo)[K], double (&di)[K], double (&up)[K], double (&rh)[K]) {
#pragma unroll
        for (int i = 0; i < K; ++i) {
          lo[i] = Lo[i];
          di[i] = Di[i];
          up[i] = Up[i];
          rh[i] = Rh[i];
        }
      });
  __syncthreads();
  level1_interior_fast<NT>(S, 2 * ch.active);
  if (threadIdx.x == 0) {
    double R0[4], R1[4];
    tile_rows<NT>(S, 2 * ch.active, R0, R1);
    if (REDUCE) {
      const int r = I.red_off + 2 * td.tidx;
      P.rlo[r] = R0[0]; P.rdi[r] = R0[1]; P.rup[r] = R0[2]; P.rrhs[r] = R0[3];
      P.rlo[r + 1] = R1[0]; P.rdi[r + 1] = R1[1]; P.rup[r + 1] = R1[2]; P.rrhs[r + 1] = R1[3];
    } else if (I.ntiles == 1) {
      const bool cyclic = I.bc == 0;
      if (!cyclic) {
        R0[0] = 0.0;
        R1[2] = 0.0;
      }
      double z0, zl;
      solve_ends(R0, R1, cyclic, z0, zl);
      S.s[0] = z0;
      S.s[1] = zl;
    } else {
      S.s[0] = P.rx[I.red_off + 2 * td.tidx];
      S.s[1] = P.rx[I.red_off + 2 * td.tidx + 1];
    }
  }
  if (REDUCE) return;
  __syncthreads();
  reg_chunk_write<NT, K>(S, ch, P.phi + I.off + td.start, S.s[0], S.s[1], y, v, w);
  if (bad) atomicOr(&P.status[td.inst], kFlagNonPhys);
}

// Windowed single-pass solve of the phi system (instances planned into
// windows, as the depth system of the semi-implicit step): a window solves
// rows [ws, ws + wl) of its instance and writes phi on its core
// [cs, cs + cl).  Beyond a truncated window edge the unknown phi is replaced
// by 0, so its coupling leaves the row.  The phi rows are diagonally
// dominant by h_i (diagonal minus couplings), so max |phi| <= max |rhs| /
// min h, and the replacement changes a core row by at most the row's
// derivative with respect to the replaced value times that bound.  The
// window computes those derivatives at both core edges (through the 2x2 end
// solve) and flags the instance (kFlagWindow) unless their sum is below
// 2^-56: the truncation then moves phi by less than 2^-56 of max |phi|.
struct SgnWinArgs {
  const InstDesc* __restrict__ inst;
  const WinDesc* __restrict__ win;
  const double* __restrict__ dt;
  const double* __restrict__ h;  // stage operand
  const double* __restrict__ q;
  double* __restrict__ phi;
  int32_t* __restrict__ status;
};

template <int NT, int K>
__global__ __launch_bounds__(NT, 4) void k_sgn_win(SgnWinArgs P) {
  using LT = SgnTriLds<NT, K>;
  __shared__ LT L;
  __shared__ double E[8];  // couplings moved out at the edges, end unknowns, derivatives
  const WinDesc wd = P.win[blockIdx.x];
  const InstDesc I = P.inst[wd.inst];
  if (!(P.dt[wd.inst] > 0.0)) return;  // frozen: phi is not used
  const int t = threadIdx.x, wl = wd.wl, n = I.n;
  const bool truncL = (wd.flags & 1) != 0, truncR = (wd.flags & 2) != 0;
  if (t == 0) {
    E[0] = 0.0;
    E[1] = 0.0;
  }
  // h and q of window rows -2 .. wl + 1 (staged index = row + 2)
#pragma unroll
  for (int r = 0; r < (LT::SL + NT - 1) / NT; ++r) {
    const int si = t + r * NT;
    if (si < wl + 4) {
      const int c = wrap_any(wd.ws - 2 + si, n, I.bc);
      L.u.X[0][spad(si)] = P.h[I.off + c];
      L.u.X[1][spad(si)] = P.q[I.off + c];
    }
  }
  __syncthreads();
  const Chunk ch = chunk_of(wl, NT, t);
  const int k = ch.k, f = ch.first;
  double Lo[K], Di[K], Up[K], Rh[K];
  bool bad = false;
  if (t < ch.active) {
    const double g = I.g;
    const double c3 = 1.0 / (3.0 * I.dx * I.dx);
    const double c6 = 1.0 / (6.0 * I.dx * I.dx * I.dx);
    bad = sgn_chunk_rows<K>(
        L.u.X[0], L.u.X[1], f, k, g, c3, c6, Lo, Di, Up, Rh,
        [&](int ii, double& l, double& d, double& u) {
          const int p = f + ii;
          if (I.bc != 0) {  // zero-gradient phi at a transmissive end of the instance
            const int c = wd.ws + p;
            if (c == 0) { d += l; l = 0.0; }
            if (c == n - 1) { d += u; u = 0.0; }
          }
          if (ii < k) {
            if (truncL && p == 0) {  // phi beyond the left edge taken as 0
              E[0] = l;
              l = 0.0;
            }
            if (truncR && p == wl - 1) {
              E[1] = u;
              u = 0.0;
            }
          }
        });
  }
  __syncthreads();  // the staged cells are dead: the union holds the level-1 system
  Lds<NT>& S = L.u.S;
  double y[K], v[K], w[K];
  reg_chunk_elim_rows<NT, K>(
      S, wl, y, v, w,
      [&](int, int, double (&lo)[K], double (&di)[K], double (&up)[K], double (&rh)[K]) {
#pragma unroll
        for (int i = 0; i < K; ++i) {
          lo[i] = Lo[i];
          di[i] = Di[i];
          up[i] = Up[i];
          rh[i] = Rh[i];
        }
      });
  __syncthreads();
  const int n1 = 2 * ch.active;
  level1_interior_fast<NT>(S, n1);
  if (t == 0) {
    // the window's end unknowns (no coupling beyond the ends is left) and
    // their derivatives with respect to the two replaced values: the left
    // one enters the first row's right-hand side as -E[0], the right one
    // the last row's as -E[1]
    double R0[4], R1[4];
    tile_rows<NT>(S, n1, R0, R1);
    const double m00 = R0[1], m01 = R0[2], m10 = R1[0], m11 = R1[1];
    const double idet = 1.0 / (m00 * m11 - m01 * m10);
    E[2] = (m11 * R0[3] - m01 * R1[3]) * idet;  // z0
    E[3] = (m00 * R1[3] - m10 * R0[3]) * idet;  // zl
    E[4] = -E[0] * m11 * idet;                  // d z0 / d (left value)
    E[5] = E[0] * m10 * idet;                   // d zl / d (left value)
    E[6] = E[1] * m01 * idet;                   // d z0 / d (right value)
    E[7] = -E[1] * m00 * idet;                  // d zl / d (right value)
  }
  __syncthreads();
  if (t < ch.active) {
    const double z0 = E[2], zl = E[3];
    const int j0 = 2 * t, j1 = 2 * t + 1;
    double zf, zb, Vf, Wf, Vb, Wb;  // chunk ends and their derivatives by (z0, zl)
    if (j0 == 0) { zf = z0; Vf = 1.0; Wf = 0.0; }
    else { zf = S.d0[j0] + S.d1[j0] * z0 + S.d2[j0] * zl; Vf = S.d1[j0]; Wf = S.d2[j0]; }
    if (j1 == n1 - 1) { zb = zl; Vb = 0.0; Wb = 1.0; }
    else { zb = S.d0[j1] + S.d1[j1] * z0 + S.d2[j1] * zl; Vb = S.d1[j1]; Wb = S.d2[j1]; }
    const int c0 = wd.cs - wd.ws, c1 = c0 + wd.cl;  // the core's window rows
    const bool cert = truncL || truncR;
    double sens = 0.0;
#pragma unroll
    for (int i = 0; i < K; ++i) {
      if (i < k) {
        const int p = f + i;
        double x, s0, sl;  // row value and its derivatives by (z0, zl)
        if (i == 0) { x = zf; s0 = Vf; sl = Wf; }
        else if (i == k - 1) { x = zb; s0 = Vb; sl = Wb; }
        else {
          x = y[i] + v[i] * zf + w[i] * zb;
          s0 = v[i] * Vf + w[i] * Vb;
          sl = v[i] * Wf + w[i] * Wb;
        }
        if (p >= c0 && p < c1) P.phi[I.off + wd.cs + (p - c0)] = x;
        if (cert && (p == c0 || p == c1 - 1))
          sens = fmax(sens, fabs(s0 * E[4] + sl * E[5]) + fabs(s0 * E[6] + sl * E[7]));
      }
    }
    if (!(sens <= 1.3877787807814457e-17)) atomicOr(&P.status[wd.inst], kFlagWindow);  // 2^-56
  }
  if (bad) atomicOr(&P.status[wd.inst], kFlagNonPhys);
}

template <int NT, int KX, int STAGE>
__global__ __launch_bounds__(NT) void k_sgn_update(SgnArgs A) {
  constexpr int TL = NT * KX;
  constexpr int SL = TL + 4;
  __shared__ double X[2][SL];
  __shared__ double F[2][TL + 1];  // face fluxes of h and q
  const TileDesc td = A.tiles[blockIdx.x];
  const InstDesc I = A.inst[td.inst];
  const double dt = A.dt[td.inst];
  const int t = threadIdx.x, len = td.len;
  const int64_t base = I.off + td.start;
  if (!(dt > 0.0)) {  // frozen instance: the state stays
    for (int i = t; i < len; i += NT) {
      A.o_h[base + i] = A.un_h[base + i];
      A.o_q[base + i] = A.un_q[base + i];
      if (STAGE == 2) {
        A.o_m[base + i] = A.un_m[base + i];
        A.o_W[base + i] = A.un_W[base + i];
      }
    }
    return;
  }
  sgn_stage<NT, SL>(X, A.in_h, A.in_q, I, td);
  __syncthreads();
  const double g = I.g, idx = 1.0 / I.dx;
  bool bad = false;
#pragma unroll
  for (int r = 0; r <= KX; ++r) {
    const int e = t + r * NT;
    if (e <= len) {
      const double hL = X[0][e + 1] + 0.25 * (X[0][e + 2] - X[0][e]);
      const double hR = X[0][e + 2] - 0.25 * (X[0][e + 3] - X[0][e + 1]);
      const double qL = X[1][e + 1] + 0.25 * (X[1][e + 2] - X[1][e]);
      const double qR = X[1][e + 2] - 0.25 * (X[1][e + 3] - X[1][e + 1]);
      bad |= !(hL > 0.0) || !(hR > 0.0);
      const double uL = qL / hL, uR = qR / hR;
      const double al = fmax(fabs(uL) + sqrt(g * hL), fabs(uR) + sqrt(g * hR));
      F[0][e] = 0.5 * (qL + qR - al * (hR - hL));
      F[1][e] = 0.5 * (qL * uL + 0.5 * g * hL * hL + qR * uR + 0.5 * g * hR * hR - al * (qR - qL));
    }
  }
  __syncthreads();
  double smx = 0.0, umx = 0.0;
#pragma unroll
  for (int r = 0; r < KX; ++r) {
    const int i = t + r * NT;
    if (i < len) {
      const int k = i + 2;
      const double h = X[0][k];
      const double Lh = -(F[0][i + 1] - F[0][i]) * idx;
      const double Lq = -(F[1][i + 1] - F[1][i]) * idx + h * A.phi[base + i];
      double hn = h + dt * Lh, qn = X[1][k] + dt * Lq;
      if (STAGE == 2) {
        hn = 0.5 * (A.un_h[base + i] + hn);
        qn = 0.5 * (A.un_q[base + i] + qn);
        A.o_m[base + i] = A.un_m[base + i];
        A.o_W[base + i] = A.un_W[base + i];
        const double un = fabs(qn / hn);
        smx = fmax(smx, un + sqrt(g * hn));
        umx = fmax(umx, un);
      }
      bad |= !(hn > 0.0) || !isfinite(hn) || !isfinite(qn);
      A.o_h[base + i] = hn;
      A.o_q[base + i] = qn;
    }
  }
  if (STAGE == 2) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      smx = fmax(smx, __shfl_xor(smx, off));
      umx = fmax(umx, __shfl_xor(umx, off));
    }
    if ((t & 63) == 0 && smx > 0.0) {
      atomicMax(&A.smax[td.inst], (unsigned long long)__double_as_longlong(smx));
      atomicMax(&A.umax[td.inst], (unsigned long long)__double_as_longlong(umx));
    }
  }
  if (bad) atomicOr(&A.status[td.inst], kFlagNonPhys);
}

}  // namespace hsgn
