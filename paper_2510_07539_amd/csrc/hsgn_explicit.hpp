// hsgn_explicit.hpp -- the fully explicit hSGN step with Heun's method
// (Sec. 4.1, eq. GN_hyp_eq_explicit), flat bottom, for the cost comparison
// the paper makes against the semi-implicit step.
//
// Space operator L(U), U = (h, q, m = h eta, W = h w):
//   L_h = -Dhat_x(q)
//   L_q = -Dhat_x(q u) - a^2 D_x(h) - lambda alpha D_x(m)
//   L_m = -Dhat_x(m u) + W
//   L_W = -Dhat_x(W u) - lambda (m / h^2 - 1)
// Dhat_x: Rusanov flux difference on the unlimited linear reconstruction,
// speed max(|u| + c) over the two face states with the hSGN celerity
// c^2 = g h + (lambda/3) (m/h^2)^2 (eq. hSGN_c); D_x: central difference;
// a^2 = g h + lambda (eta/h)^2 - (lambda/3) eta/h and
// alpha = -(2 eta/h - 1) / (3 h) are the pressure derivatives (eq. hSGN_p).
// The mass flux is a Rusanov flux and the speed includes c: with the
// printed central mass flux and speed |u| one step at rest grows.
// Heun: U1 = U^n + dt L(U^n);  U^{n+1} = (U^n + U1 + dt L(U1)) / 2.
//
// One workgroup owns a tile of NT * KX cells of one instance.  The four
// fields of the stage operand are staged through LDS with coalesced loads
// (tile plus two ghost cells per side: periodic wrap or zero-order copy);
// every cell is updated from its two faces.  Threads take cells at stride
// NT, so every global load and store is coalesced.
#pragma once

#include "hsgn_kernels.hpp"

namespace hsgn {

constexpr int kExNT = 256;               // threads per tile
constexpr int kExK = 4;                  // cells per thread
constexpr int kExTile = kExNT * kExK;    // cells per tile

struct ExArgs {
  const double* __restrict__ un_h;  // U^n
  const double* __restrict__ un_q;
  const double* __restrict__ un_m;
  const double* __restrict__ un_W;
  const double* __restrict__ in_h;  // operand of L (stage 1: U^n, stage 2: U1)
  const double* __restrict__ in_q;
  const double* __restrict__ in_m;
  const double* __restrict__ in_W;
  double* __restrict__ o_h;         // stage output
  double* __restrict__ o_q;
  double* __restrict__ o_m;
  double* __restrict__ o_W;
  const InstDesc* __restrict__ inst;
  const TileDesc* __restrict__ tiles;
  const double* __restrict__ dt;
  unsigned long long* __restrict__ smax;  // stage 2: speed bound of the new state
  unsigned long long* __restrict__ umax;
  int32_t* __restrict__ status;
};

// Rusanov fluxes (h, q u, m u, W u) of face e (between tile cells e - 1 and
// e; stencil: staged cells e .. e + 3) at speed max(|u| + c).
template <int SL>
__device__ __forceinline__ void ex_face(const double (*X)[SL], int e, double g, double lam,
                                        double F[4], bool& bad) {
  double L[4], R[4];
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    L[f] = X[f][e + 1] + 0.25 * (X[f][e + 2] - X[f][e]);
    R[f] = X[f][e + 2] - 0.25 * (X[f][e + 3] - X[f][e + 1]);
  }
  bad |= !(L[0] > 0.0) || !(R[0] > 0.0);
  const double iL = 1.0 / L[0], iR = 1.0 / R[0];
  const double uL = L[1] * iL, uR = R[1] * iR;
  const double eL = L[2] * iL * iL, eR = R[2] * iR * iR;
  const double sL = fabs(uL) + sqrt(g * L[0] + (lam / 3.0) * eL * eL);
  const double sR = fabs(uR) + sqrt(g * R[0] + (lam / 3.0) * eR * eR);
  const double al = fmax(sL, sR);
  F[0] = 0.5 * (L[1] + R[1] - al * (R[0] - L[0]));
  F[1] = 0.5 * (L[1] * uL + R[1] * uR - al * (R[1] - L[1]));
  F[2] = 0.5 * (L[2] * uL + R[2] * uR - al * (R[2] - L[2]));
  F[3] = 0.5 * (L[3] * uL + R[3] * uR - al * (R[3] - L[3]));
}

template <int NT, int KX, int STAGE>
__global__ __launch_bounds__(NT) void k_ex(ExArgs A) {
  constexpr int TL = NT * KX;  // tile cells
  constexpr int SL = TL + 4;   // staged cells (two ghosts per side)
  __shared__ double X[4][SL];  // stage operand; staged index s <-> cell s - 2
  const TileDesc td = A.tiles[blockIdx.x];
  const InstDesc I = A.inst[td.inst];
  const double dt = A.dt[td.inst];
  const int t = threadIdx.x;
  const int n = I.n, bc = I.bc, len = td.len;
  const int64_t base = I.off + td.start;  // first cell of the tile
  const double* in[4] = {A.in_h, A.in_q, A.in_m, A.in_W};
  const double* un[4] = {A.un_h, A.un_q, A.un_m, A.un_W};
  double* out[4] = {A.o_h, A.o_q, A.o_m, A.o_W};

  if (!(dt > 0.0)) {  // frozen instance: the state stays
    for (int i = t; i < len; i += NT) {
#pragma unroll
      for (int f = 0; f < 4; ++f) out[f][base + i] = un[f][base + i];
    }
    return;
  }
  // ---- staging (instance-relative cell start - 2 + s, wrapped or clamped)
#pragma unroll
  for (int r = 0; r < (SL + NT - 1) / NT; ++r) {
    const int si = t + r * NT;
    if (si < len + 4) {
      int c = td.start - 2 + si;
      if (bc == 0) c = c < 0 ? c + n : (c >= n ? c - n : c);
      else c = c < 0 ? 0 : (c > n - 1 ? n - 1 : c);
#pragma unroll
      for (int f = 0; f < 4; ++f) X[f][si] = in[f][I.off + c];
    }
  }
  __syncthreads();
  const double g = I.g, lam = I.lam, idx = 1.0 / I.dx, i2dx = 0.5 / I.dx;
  bool bad = false;
  // ---- cells: explicit update (stage 1) or Heun average (stage 2); each
  // thread forms both faces of its cell (a face is formed twice, which
  // keeps the LDS of a tile to the staged operand)
  double smx = 0.0, umx = 0.0;
#pragma unroll
  for (int r = 0; r < KX; ++r) {
    const int i = t + r * NT;
    if (i < len) {
      double Fl[4], Fr[4];
      ex_face<SL>(X, i, g, lam, Fl, bad);
      ex_face<SL>(X, i + 1, g, lam, Fr, bad);
      const int k = i + 2;  // staged index of the cell
      const double h = X[0][k], m = X[2][k], W = X[3][k];
      bad |= !(h > 0.0);
      const double ih = 1.0 / h;
      const double eh = m * ih * ih;
      const double a2 = g * h + lam * eh * eh - (lam / 3.0) * eh;
      const double alpha = -(2.0 * eh - 1.0) * ih * (1.0 / 3.0);
      const double dh = (X[0][k + 1] - X[0][k - 1]) * i2dx;
      const double dm = (X[2][k + 1] - X[2][k - 1]) * i2dx;
      double Lv[4];
      Lv[0] = -(Fr[0] - Fl[0]) * idx;
      Lv[1] = -(Fr[1] - Fl[1]) * idx - a2 * dh - lam * alpha * dm;
      Lv[2] = -(Fr[2] - Fl[2]) * idx + W;
      Lv[3] = -(Fr[3] - Fl[3]) * idx - lam * (eh - 1.0);
      double o[4];
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        const double u1 = X[f][k] + dt * Lv[f];
        o[f] = STAGE == 1 ? u1 : 0.5 * (un[f][base + i] + u1);
        bad |= !isfinite(o[f]);
        out[f][base + i] = o[f];
      }
      if (STAGE == 2) {
        const double ihn = 1.0 / o[0];
        const double uu = fabs(o[1] * ihn);
        const double en = o[2] * ihn * ihn;
        bad |= !(o[0] > 0.0);
        smx = fmax(smx, uu + sqrt(g * o[0] + (lam / 3.0) * en * en));
        umx = fmax(umx, uu);
      }
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

// Speed bound |u| + c of a given state (first step after a state is loaded).
template <int NT>
__global__ __launch_bounds__(NT) void k_speed_ex(const InstDesc* __restrict__ inst,
                                                 const TileDesc* __restrict__ tiles,
                                                 const double* __restrict__ h,
                                                 const double* __restrict__ q,
                                                 const double* __restrict__ m,
                                                 unsigned long long* __restrict__ smax,
                                                 unsigned long long* __restrict__ umax,
                                                 unsigned long long* __restrict__ hmax) {
  const TileDesc td = tiles[blockIdx.x];
  const InstDesc I = inst[td.inst];
  double s = 0.0, u = 0.0, hx = 0.0;
  for (int i = threadIdx.x; i < td.len; i += NT) {
    const int64_t gi = I.off + td.start + i;
    const double hh = h[gi];
    const double ih = 1.0 / hh;
    const double uu = fabs(q[gi] * ih);
    const double e = m[gi] * ih * ih;
    s = fmax(s, uu + sqrt(I.g * hh + (I.lam / 3.0) * e * e));
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

}  // namespace hsgn
