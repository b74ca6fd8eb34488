// vjp_kernel.hpp -- the hand-written discrete adjoint of one Runge-Kutta stage.
//
// A stage is W = U0 + b ((V - U0) + dt L(V)) with
//   L(V) = S(V) - (F^_{i+1/2} - F^_{i-1/2}) / dx - (G^_{j+1/2} - G^_{j-1/2}) / dy,
//   F^ = W5(f+ left-biased) + W5(f- right-biased),  f+- = (F(U) +- alpha U) / 2
// (Sect. 2.1, Eq. euler2D).  With the LF speeds alpha held at their recorded
// values, its transpose applied to the adjoint lam of W is
//   dJ/dV  = b (lam + dt J_L(V)^T lam),   dJ/dU0 = (1 - b) lam,
// and J_L^T mu is assembled here from:
//   * sources: (dS/dU)^T mu per cell (gravity; cylindrical geometric terms);
//   * per face f: nu_c(f) = (mu_c(right cell) - mu_c(left cell)) / dx, the
//     adjoint of F^_c(f) (faces on the domain boundary see mu = 0 outside);
//   * per face and component: nu * dW5/dv for both reconstructions (the
//     derivative runs through the nonlinear weights: beta-adjoints
//     -2 omega_k (q_k - W) / (eps + beta_k)), gathered at every point the
//     stencils touch (by lane shifts within a wavefront: no atomics and a
//     fixed summation order);
//   * per point: dU += A(U)^T (phi+ + phi-) / 2 + alpha (phi+ - phi-) / 2 with
//     A = dF/dU the flux Jacobian;
//   * ghost points: their adjoint belongs to the cell they were copied from
//     (mirror with the normal momentum negated, or the edge cell); it is
//     written to a small side buffer and folded back in a fixed order: the y
//     ghosts by the x pass at the y-edge cells, the x ghosts by a separate
//     tiny kernel.  A periodic axis has no
//     ghost points: its lines are rings (faces and stencils wrap), so every
//     contribution lands on a cell directly.
// The x and y parts run as two passes (y: y fluxes into a partial sum; x:
// sources + x fluxes, then the stage combination), each taking grid lines along
// its own axis, one wavefront per line and one point and face per lane, with
// the line's split fluxes (six-point halo) staged in LDS.
#pragma once

#include "stage_kernel.hpp"
#include "vjp.hpp"

namespace hy {

// nu * dW5/dv_m for the reconstruction W5(v0..v4) at the right face of v2.
// With omega_k the nonlinear weights, q_k the candidate values and
// W = sum omega_k q_k: dW = sum omega_k dq_k - 2 sum omega_k (q_k - W) dbeta_k
// / (eps + beta_k).  The candidates are carried as Q_k = 6 q_k (the 1/6 folded
// into the factors below).
__device__ __forceinline__ void weno5_adj(const double v[5], double eps, double nu, double vb[5]) {
  const double c1312 = 13.0 / 12.0;
  const double d0 = v[0] - 2.0 * v[1] + v[2], e0 = v[0] - 4.0 * v[1] + 3.0 * v[2];
  const double d1 = v[1] - 2.0 * v[2] + v[3], e1 = v[1] - v[3];
  const double d2 = v[2] - 2.0 * v[3] + v[4], e2 = 3.0 * v[2] - 4.0 * v[3] + v[4];
  // (13/12) d_k and e_k / 4 serve both beta_k and its derivative below
  const double cd0 = c1312 * d0, qe0 = 0.25 * e0;
  const double cd1 = c1312 * d1, qe1 = 0.25 * e1;
  const double cd2 = c1312 * d2, qe2 = 0.25 * e2;
  const double E0 = eps + (cd0 * d0 + qe0 * e0);
  const double E1 = eps + (cd1 * d1 + qe1 * e1);
  const double E2 = eps + (cd2 * d2 + qe2 * e2);
  const double s0 = E0 * E0, s1 = E1 * E1, s2 = E2 * E2;
  // weights over the common denominator; one division gives 1/sum(w) and 1/(E0 E1 E2)
  const double w0 = s1 * s2, w1 = 6.0 * (s0 * s2), w2 = 3.0 * (s0 * s1);
  const double sw = w0 + w1 + w2;
  const double E12 = E1 * E2, E02 = E0 * E2, E01 = E0 * E1;
  const double P = E0 * E12;
  // 1 / (P sw): hardware reciprocal and two Newton steps (the adjoint needs
  // no correctly rounded quotient; P sw is a normal positive number)
  const double x = P * sw;
  double inv = __builtin_amdgcn_rcp(x);
  inv = __builtin_fma(inv, __builtin_fma(-x, inv, 1.0), inv);
  inv = __builtin_fma(inv, __builtin_fma(-x, inv, 1.0), inv);
  const double isw = P * inv, iP = sw * inv;
  const double om0 = w0 * isw, om1 = w1 * isw, om2 = w2 * isw;
  const double Q0 = 2.0 * v[0] - 7.0 * v[1] + 11.0 * v[2];
  const double Q1 = -v[1] + 5.0 * v[2] + 2.0 * v[3];
  const double Q2 = 2.0 * v[2] + 5.0 * v[3] - v[4];
  const double W6 = om0 * Q0 + om1 * Q1 + om2 * Q2;
  // twice the beta-adjoints -2 nu omega_k (q_k - W) / E_k, with 1 / E_k =
  // (product of the other two) / P; dbeta_k = 2 (13/12) d_k dd_k + 2 (e_k / 4) de_k
  const double f = (-2.0 / 3.0) * nu * iP;
  const double bb0 = f * (om0 * (Q0 - W6)) * E12;
  const double bb1 = f * (om1 * (Q1 - W6)) * E02;
  const double bb2 = f * (om2 * (Q2 - W6)) * E01;
  const double n6 = nu * (1.0 / 6.0);
  const double c0 = n6 * om0, c1 = n6 * om1, c2 = n6 * om2;
  const double t0 = bb0 * cd0, h0 = bb0 * qe0;
  const double t1 = bb1 * cd1, h1 = bb1 * qe1;
  const double t2 = bb2 * cd2, h2 = bb2 * qe2;
  vb[0] = 2.0 * c0 + t0 + h0;
  vb[1] = -7.0 * c0 - c1 - 2.0 * t0 - 4.0 * h0 + t1 + h1;
  vb[2] = 11.0 * c0 + 5.0 * c1 + 2.0 * c2 + t0 + 3.0 * h0 - 2.0 * t1 + t2 + 3.0 * h2;
  vb[3] = 2.0 * c1 + 5.0 * c2 + t1 - h1 - 2.0 * t2 - 4.0 * h2;
  vb[4] = -c2 + t2 + h2;
}

// Single precision: textbook weights with hardware reciprocals.
__device__ __forceinline__ void weno5_adj(const float v[5], float eps, float nu, float vb[5]) {
  const float c1312 = 13.0f / 12.0f;
  const float d0 = v[0] - 2.0f * v[1] + v[2], e0 = v[0] - 4.0f * v[1] + 3.0f * v[2];
  const float d1 = v[1] - 2.0f * v[2] + v[3], e1 = v[1] - v[3];
  const float d2 = v[2] - 2.0f * v[3] + v[4], e2 = 3.0f * v[2] - 4.0f * v[3] + v[4];
  const float cd0 = c1312 * d0, qe0 = 0.25f * e0;
  const float cd1 = c1312 * d1, qe1 = 0.25f * e1;
  const float cd2 = c1312 * d2, qe2 = 0.25f * e2;
  const float r0 = rcpf(eps + (cd0 * d0 + qe0 * e0));
  const float r1 = rcpf(eps + (cd1 * d1 + qe1 * e1));
  const float r2 = rcpf(eps + (cd2 * d2 + qe2 * e2));
  const float a0 = 0.1f * r0 * r0, a1 = 0.6f * r1 * r1, a2 = 0.3f * r2 * r2;
  const float ia = rcpf(a0 + a1 + a2);
  const float om0 = a0 * ia, om1 = a1 * ia, om2 = a2 * ia;
  const float q0 = (2.0f * v[0] - 7.0f * v[1] + 11.0f * v[2]) * (1.0f / 6.0f);
  const float q1 = (-v[1] + 5.0f * v[2] + 2.0f * v[3]) * (1.0f / 6.0f);
  const float q2 = (2.0f * v[2] + 5.0f * v[3] - v[4]) * (1.0f / 6.0f);
  const float W = om0 * q0 + om1 * q1 + om2 * q2;
  // twice the beta-adjoints (see the FP64 form)
  const float f = -4.0f * nu;
  const float bb0 = f * om0 * (q0 - W) * r0;
  const float bb1 = f * om1 * (q1 - W) * r1;
  const float bb2 = f * om2 * (q2 - W) * r2;
  const float c0 = nu * om0 * (1.0f / 6.0f), c1 = nu * om1 * (1.0f / 6.0f), c2 = nu * om2 * (1.0f / 6.0f);
  const float t0 = bb0 * cd0, h0 = bb0 * qe0;
  const float t1 = bb1 * cd1, h1 = bb1 * qe1;
  const float t2 = bb2 * cd2, h2 = bb2 * qe2;
  vb[0] = 2.0f * c0 + t0 + h0;
  vb[1] = -7.0f * c0 - c1 - 2.0f * t0 - 4.0f * h0 + t1 + h1;
  vb[2] = 11.0f * c0 + 5.0f * c1 + 2.0f * c2 + t0 + 3.0f * h0 - 2.0f * t1 + t2 + 3.0f * h2;
  vb[3] = 2.0f * c1 + 5.0f * c2 + t1 - h1 - 2.0f * t2 - 4.0f * h2;
  vb[4] = -c2 + t2 + h2;
}

// 1/r for the adjoint, which is not bit-exact and needs no correctly rounded
// quotient: the hardware reciprocal refined by two Newton steps (FP64; r is a
// positive normal number on every state the adjoint is defined at), the
// hardware reciprocal in FP32.
__device__ __forceinline__ double adj_rcp(double r) {
  double y = __builtin_amdgcn_rcp(r);
  y = __builtin_fma(y, __builtin_fma(-r, y, 1.0), y);
  return __builtin_fma(y, __builtin_fma(-r, y, 1.0), y);
}
__device__ __forceinline__ float adj_rcp(float r) { return rcpf(r); }

// Velocity and pressure of a point for the adjoint's split fluxes.
template <typename R>
__device__ __forceinline__ Prim<R> adj_prim(const R U[4], R gm1, R& rinv) {
  Prim<R> w;
  rinv = adj_rcp(U[0]);
  w.u = U[1] * rinv;
  w.v = U[2] * rinv;
  w.p = gm1 * (U[3] - R(0.5) * (U[1] * w.u + U[2] * w.v));
  w.c = R(0);  // (not used by the split fluxes)
  return w;
}

// Quantities of a point that the flux-Jacobian rows need.
template <typename R> struct JacPt { R u, v, H, hq; };  // hq = (gamma-1) |v|^2 / 2

template <typename R>
__device__ __forceinline__ JacPt<R> jac_point(R r, R mx, R my, R E, R gm1) {
  const R U[4] = {r, mx, my, E};
  R rinv;
  const Prim<R> w = adj_prim(U, gm1, rinv);
  JacPt<R> j;
  j.u = w.u;
  j.v = w.v;
  j.H = (E + w.p) * rinv;
  j.hq = R(0.5) * gm1 * (w.u * w.u + w.v * w.v);
  return j;
}

// dU += A_c^T psi / 2 + alpha e_c delta / 2 for component c of direction DIR
// (psi = phi+ + phi-, delta = phi+ - phi-), A = dF/dU of that direction.
template <int DIR, typename R>
__device__ __forceinline__ void jacT_row(int c, const JacPt<R>& j, R gamma, R gm1, R alpha, R psi,
                                         R delta, R dU[4]) {
  const R h = R(0.5) * psi;
  const R u = DIR == 0 ? j.u : j.v;  // normal velocity
  const R t = DIR == 0 ? j.v : j.u;  // tangential velocity
  const int cn = DIR == 0 ? 1 : 2;   // normal-momentum component
  const int ct = DIR == 0 ? 2 : 1;   // tangential-momentum component
  if (c == 0) {
    dU[cn] += h;
  } else if (c == cn) {
    dU[0] += h * (j.hq - u * u);
    dU[cn] += h * ((R(3) - gamma) * u);
    dU[ct] += h * (-gm1 * t);
    dU[3] += h * gm1;
  } else if (c == ct) {
    dU[0] += h * (-u * t);
    dU[cn] += h * t;
    dU[ct] += h * u;
  } else {
    dU[0] += h * (u * (j.hq - j.H));
    dU[cn] += h * (j.H - gm1 * u * u);
    dU[ct] += h * (-gm1 * u * t);
    dU[3] += h * (gamma * u);
  }
  dU[c] += R(0.5) * alpha * delta;
}

struct VjpPass {
  VjpArgs a;
  void* Gp;        // partial J_L^T mu in the pass precision (y pass writes, x pass reads)
  int finalize;    // this pass writes out
  double* ghost;   // ghost adjoints of this pass's axis: [2][3][n_across][4]
  const double* ghost_y;  // x pass: the y pass's ghost adjoints, merged at the y-edge cells
};

// Wavefront-wide lane shift (DPP wave_shr:1 / wave_shl:1): lane l receives
// lane l - 1 (UP) or lane l + 1 (!UP) of x; a lane with no source receives 0.
template <bool UP>
__device__ __forceinline__ int lane_shift_bits(int x) {
  return __builtin_amdgcn_update_dpp(0, x, UP ? 0x138 : 0x130, 0xF, 0xF, true);
}
template <bool UP>
__device__ __forceinline__ float lane_shift(float x) {
  return __int_as_float(lane_shift_bits<UP>(__float_as_int(x)));
}
template <bool UP>
__device__ __forceinline__ double lane_shift(double x) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(x);
  const unsigned lo = (unsigned)lane_shift_bits<UP>((int)(unsigned)b);
  const unsigned hi = (unsigned)lane_shift_bits<UP>((int)(unsigned)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// One pass (DIR 0: x, with the source adjoint; DIR 1: y) over NL lines of
// the grid along the pass axis, one wavefront per line.  Lane l of a line
// owns point k = a0 - 3 + l (the tile's NA = 58 cells are lanes 3..60; lanes
// 0..2 and 61..63 are the ghost points where the line meets the domain edge)
// and face k (between cells k - 1 and k).  Each lane differentiates both
// reconstructions of its face; the stencil derivatives are gathered at the
// points by lane shifts inside the wavefront (phi+(k) takes the f+
// derivatives of faces k - 1 .. k + 3, phi-(k) the f- derivatives of faces
// k - 2 .. k + 2), so the component loop has no barrier and no LDS writes.
// The split fluxes of the line's points a0 - 6 .. a0 + 62 are staged in LDS
// (each face reads five of each sign).  The x pass reads its own point's
// state and adjoint straight from HBM (lanes run along rows); the y pass,
// whose lanes run down columns, stages them through LDS with row-major
// loads and transposes its results back to rows before the final writes.
template <typename R, int DIR, int NL, bool STAGE_OWN>
__global__ __launch_bounds__(64 * NL) void vjp_line_kernel(VjpPass P) {
  constexpr int NT = 64 * NL;
  constexpr int NA = 58;       // cells per line and tile
  constexpr int LP = 69;       // staged points a0 - 6 .. a0 + 62
  // Row strides padded for the y pass's staging writes, where consecutive work
  // items take consecutive lines b at point p (p = t / NL): 70 and 66 doubles
  // are 6 and 2 mod 16, so the 16 work items of a 128-byte LDS cycle (8 lines
  // x 2 points) hit 16 different 8-byte bank pairs (69 and 65 put up to four
  // on one pair: 1.3M conflict cycles per 1024^2 dispatch, 0.13M padded).
  __shared__ R sF[8][NL][LP + 1];
  __shared__ R sU[STAGE_OWN ? 4 : 1][NL][66];
  __shared__ R sM[STAGE_OWN ? 4 : 1][NL][66];

  const VjpArgs& a = P.a;
  const Geom& g = a.g;
  const int tid = threadIdx.x;
  const int wv = tid >> 6, L = tid & 63;
  const int na = DIR == 0 ? g.nx : g.ny;  // cells along the pass axis
  const int nc = DIR == 0 ? g.ny : g.nx;  // lines across it
  const int bc_lo = DIR == 0 ? g.bc[0] : g.bc[2];
  const int bc_hi = DIR == 0 ? g.bc[1] : g.bc[3];
  // A periodic line is a ring: every point index is a cell (taken modulo the
  // line length), the faces wrap, and there are no ghost points whose
  // adjoints would need folding onto cells of another tile.
  const bool ring = bc_lo == PERIODIC;
  const int cn = DIR == 0 ? 1 : 2;
  const int nta = (na + NA - 1) / NA;
  // Each XCD takes a contiguous run of (segment, line group) tiles: the line
  // groups next to each other then share an L2, so a 128-byte row that two
  // groups of 8 FP64 columns split is fetched once, as are the halo points
  // that neighbouring segments of a line both read.
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int a0 = (tile % nta) * NA;
  const int b0 = (tile / nta) * NL;
  const size_t n = (size_t)g.nx * g.ny;
  const R gamma = (R)g.gamma, gm1 = (R)g.gm1, eps = (R)g.eps;
  const R alpha = (R)(DIR == 0 ? a.ax : a.ay);
  const R id = (R)(DIR == 0 ? g.idx : g.idy);

  auto gidx = [&](int along, int across) -> size_t {
    return DIR == 0 ? (size_t)across * g.nx + along : (size_t)along * g.nx + across;
  };
  // ring index of point k: the points a line segment touches lie within one
  // line length on either side once the line holds 64 cells or more, so one
  // correction does; shorter rings take the remainder
  auto wrap = [&](int k) {
    if (na >= 64) {
      k += k < 0 ? na : 0;
      return k >= na ? k - na : k;
    }
    return ((k % na) + na) % na;
  };
  // state of point k of line b (boundary conditions applied)
  auto load_state = [&](int k, int b, R u4[4]) {
    bool flip = false;
    const int s = ring ? wrap(k) : map_index(k, na, bc_lo, bc_hi, flip);
    const size_t q = gidx(s, b < nc ? b : nc - 1);
#pragma unroll
    for (int c = 0; c < 4; ++c) u4[c] = (R)a.V[c * n + q];
    if (flip) u4[cn] = -u4[cn];
  };
  // adjoint of the cells (zero outside the domain; a ring has no outside)
  auto load_mu = [&](int k, int b, R m4[4]) {
    const bool in = (ring || (k >= 0 && k < na)) && b < nc;
    const size_t q = in ? gidx(ring ? wrap(k) : k, b) : 0;
#pragma unroll
    for (int c = 0; c < 4; ++c) m4[c] = in ? (R)a.lam[c * n + q] : R(0);
  };

  const int k = a0 - 3 + L;  // this lane's point and face
  const int line = b0 + wv;
  R cu[4], mu[4];
  auto stage_point = [&](int p, int b, const R u4[4]) {
    R fp[4], fm[4];
    R rinv;
    split_flux_prim<DIR>(u4, adj_prim(u4, gm1, rinv), alpha, fp, fm);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      sF[c][b][p] = fp[c];
      sF[4 + c][b][p] = fm[c];
    }
  };
  if constexpr (!STAGE_OWN) {
    // lanes run along rows: each wavefront stages its own line, lane l its own
    // point (p = l + 3) and lanes 0..4 the five others (p = 0, 1, 2, 67, 68);
    // every load is issued before any of them is used
    const int ph = L < 3 ? L : 64 + L;
    R uh[4];
    if (L < 5) load_state(a0 - 6 + ph, line, uh);
    load_state(k, line, cu);
    load_mu(k, line, mu);
    stage_point(L + 3, wv, cu);
    if (L < 5) stage_point(ph, wv, uh);
  } else {
    // lanes run down columns: stage the workgroup's points with row-major
    // loads (consecutive work items take consecutive columns), the own
    // points' state and adjoint with them.  A work item stages at most two
    // points and one adjoint; all its loads are issued before any of them is
    // used.
    static_assert(NL * LP <= 2 * NT && NL * 64 == NT, "y staging shape");
    const int t2 = tid + NT;
    const bool two = t2 < NL * LP;
    const int b1 = tid % NL, p1 = tid / NL, b2 = t2 % NL, p2 = t2 / NL;
    R u1[4], u2[4], m4[4];
    load_state(a0 - 6 + p1, b0 + b1, u1);
    if (two) load_state(a0 - 6 + p2, b0 + b2, u2);
    load_mu(a0 - 3 + p1, b0 + b1, m4);  // (b1, p1) = (line, lane) of the adjoint
    stage_point(p1, b1, u1);
    if (p1 >= 3 && p1 < 67) {
#pragma unroll
      for (int c = 0; c < 4; ++c) sU[c][b1][p1 - 3] = u1[c];
    }
    if (two) {
      stage_point(p2, b2, u2);
      if (p2 >= 3 && p2 < 67) {
#pragma unroll
        for (int c = 0; c < 4; ++c) sU[c][b2][p2 - 3] = u2[c];
      }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) sM[c][b1][p1] = m4[c];
  }
  __syncthreads();
  if constexpr (STAGE_OWN) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      cu[c] = sU[c][wv][L];
      mu[c] = sM[c][wv][L];
    }
  }

  const bool line_ok = line < nc;
  const bool face_in = L > 0 && (ring || (k >= 0 && k <= na)) && line_ok;
  const bool is_cell = L >= 3 && L < 3 + NA && k < na && line_ok;
  const bool own_lo = a0 == 0, own_hi = a0 <= na - 1 && na - 1 < a0 + NA;
  const bool is_ghost = !ring && line_ok && ((own_lo && k < 0) || (own_hi && k >= na && k < na + NG));
  const JacPt<R> jc = jac_point<R>(cu[0], cu[1], cu[2], cu[3], gm1);
  R dU[4] = {R(0), R(0), R(0), R(0)};

#pragma unroll
  for (int c = 0; c < 4; ++c) {
    // adjoint of the face value: (mu(k) - mu(k - 1)) / dx
    const R mleft = lane_shift<true>(mu[c]);
    const R nu = face_in ? (mu[c] - mleft) * id : R(0);
    R vp[5], vm[5], gp[5], gm[5];
#pragma unroll
    for (int m = 0; m < 5; ++m) vp[m] = sF[c][wv][L + m];
    weno5_adj(vp, eps, nu, gp);
    // phi+(l) = gp0(l+3) + gp1(l+2) + gp2(l+1) + gp3(l) + gp4(l-1)
    R t = gp[0];
    t = lane_shift<false>(t) + gp[1];
    t = lane_shift<false>(t) + gp[2];
    t = lane_shift<false>(t) + gp[3];
    R php = t + lane_shift<true>(gp[4]);
    asm volatile("" : "+v"(php) : : "memory");  // the two signs one after the other
#pragma unroll
    for (int m = 0; m < 5; ++m) vm[m] = sF[4 + c][wv][L + 5 - m];
    weno5_adj(vm, eps, nu, gm);
    // phi-(l) = gm0(l-2) + gm1(l-1) + gm2(l) + gm3(l+1) + gm4(l+2)
    R u = gm[0];
    u = lane_shift<true>(u) + gm[1];
    u = lane_shift<true>(u) + gm[2];
    R w = gm[4];
    w = lane_shift<false>(w) + gm[3];
    const R phm = u + lane_shift<false>(w);
    jacT_row<DIR, R>(c, jc, gamma, gm1, alpha, php + phm, php - phm, dU);
    // one component at a time (few live registers)
    asm volatile("" : "+v"(dU[0]), "+v"(dU[1]), "+v"(dU[2]), "+v"(dU[3]) : : "memory");
  }

  // ---- ghost adjoints to the side buffer (folded onto their source cells later)
  if (is_ghost) {
    const int side = k < 0 ? 0 : 1;
    const int layer = k < 0 ? -k - 1 : k - na;
#pragma unroll
    for (int c = 0; c < 4; ++c)
      P.ghost[(((size_t)side * 3 + layer) * nc + line) * 4 + c] = (double)dU[c];
  }

  // ---- per cell.  The y pass (run first) hands its part to the x pass
  // through a partial sum; the x pass adds the sources, that partial sum and
  // the y ghosts' adjoints, and forms the stage combination.
  int ca = k, cb = line;
  bool cact = is_cell;
  double G[4];
  if (DIR == 0) {
    if (is_cell) {
      const size_t q = gidx(k, line);
      const R r = cu[0], E = cu[3];
      const R m0 = mu[0], m1 = mu[1], m2 = mu[2], m3 = mu[3];
      const R gxv = g.grav ? (R)g.grav[q] : (R)g.gx;
      const R gyv = g.grav ? (R)g.grav[n + q] : (R)g.gy;
      R S[4];
      S[0] = gxv * m1 + gyv * m2;
      S[1] = gxv * m3;
      S[2] = gyv * m3;
      S[3] = R(0);
      if (g.cyl) {
        const double ri = g.xlo + ((double)k + 0.5) * g.dx;
        const R ir = (R)(1.0 / ri);
        const R uu = jc.u, vv = jc.v;
        const R Eo = E / r;  // E / rho
        // d/dU of (m_r, m_r u, m_z u, (E + p) u), transposed onto mu, times -1/r
        S[0] -= ir * (-uu * uu * m1 - uu * vv * m2 + uu * (R(2) * jc.hq - gamma * Eo) * m3);
        S[1] -= ir * (m0 + R(2) * uu * m1 + vv * m2 + (gamma * Eo - jc.hq - gm1 * uu * uu) * m3);
        S[2] -= ir * (uu * m2 - gm1 * uu * vv * m3);
        S[3] -= ir * (gamma * uu * m3);
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) G[c] = (double)(S[c] + dU[c]);
      if (g.has_y) {
        const R* gp = static_cast<const R*>(P.Gp);
#pragma unroll
        for (int c = 0; c < 4; ++c) G[c] += (double)gp[c * n + q];
        // y-ghost adjoints whose source is this cell (only cells within three
        // of a y edge can be sources), in a fixed order
        const int I = k, J = line;
        if (g.bc[2] != PERIODIC && (J < NG || J >= g.ny - NG)) {
          for (int e = 0; e < 6; ++e) {
            const int side = e / 3, layer = e % 3;
            const int kk = side == 0 ? -1 - layer : g.ny + layer;
            bool flip;
            if (map_index(kk, g.ny, g.bc[2], g.bc[3], flip) != J) continue;
            const double* gv = P.ghost_y + (((size_t)side * 3 + layer) * g.nx + I) * 4;
#pragma unroll
            for (int c = 0; c < 4; ++c) G[c] += (flip && c == 2) ? -gv[c] : gv[c];
          }
        }
      }
    }
  } else {
    // lanes run down columns: transpose the cells' results through LDS so
    // that the partial sum is written in row segments
    R(*sT)[NA][NL + 1] = reinterpret_cast<R(*)[NA][NL + 1]>(&sF[0][0][0]);
    static_assert(4 * NA * (NL + 1) <= 8 * NL * LP, "transpose fits in the split-flux storage");
    __syncthreads();  // every wavefront is done with sF
    if (L >= 3 && L < 3 + NA) {
#pragma unroll
      for (int c = 0; c < 4; ++c) sT[c][L - 3][wv] = dU[c];
    }
    __syncthreads();
    cb = b0 + tid % NL;
    const int la = tid / NL;
    ca = a0 + la;
    cact = la < NA && ca < na && cb < nc;
    if (cact) {
#pragma unroll
      for (int c = 0; c < 4; ++c) G[c] = (double)sT[c][la][tid % NL];
    }
  }
  if (!cact) return;
  const size_t q = gidx(ca, cb);
  if (!P.finalize) {
    // (the y pass's partial sum is a value of the pass precision: exact in it)
    R* gp = static_cast<R*>(P.Gp);
#pragma unroll
    for (int c = 0; c < 4; ++c) gp[c * n + q] = (R)G[c];
    return;
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    // (in FP64 the x pass holds the cell's adjoint already)
    const double l = DIR == 0 && sizeof(R) == 8 ? (double)mu[c] : a.lam[c * n + q];
    double o = a.b * __builtin_fma(a.dt, G[c], l);
    if (a.add0) o += a.c0 * a.add0[c * n + q];
    if (a.add1) o += a.c1 * a.add1[c * n + q];
    a.out[c * n + q] = o;
  }
}

// Adds scale * (adjoint of each ghost point) onto the cell it was copied from.
// One work item per (line, component): it loads the six ghost values of its
// line first, merges those that land on the same cell (transmissive edges, or
// tiny grids where both sides reach the same cells) in a fixed order, then
// updates the distinct target cells -- deterministic, no atomics, and no
// chain of dependent read-modify-writes.
// (Templated on the pass precision only so each instantiating unit owns a copy.)
template <typename R>
__global__ void vjp_fold_kernel(Geom g, int dir, const double* __restrict__ ghost,
                                double* __restrict__ out, double scale) {
  const int na = dir == 0 ? g.nx : g.ny;
  const int nc = dir == 0 ? g.ny : g.nx;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int b = t >> 2, c = t & 3;
  if (b >= nc) return;
  const int lo = dir == 0 ? g.bc[0] : g.bc[2];
  const int hi = dir == 0 ? g.bc[1] : g.bc[3];
  const int cn = dir == 0 ? 1 : 2;
  const size_t n = (size_t)g.nx * g.ny;
  int tgt[6];
  double val[6];
#pragma unroll
  for (int e = 0; e < 6; ++e) {
    const int side = e / 3, layer = e % 3;
    const int k = side == 0 ? -1 - layer : na + layer;
    bool flip;
    tgt[e] = map_index(k, na, lo, hi, flip);
    const double v = ghost[(((size_t)side * 3 + layer) * nc + b) * 4 + c];
    val[e] = (flip && c == cn) ? -v : v;
  }
#pragma unroll
  for (int e = 0; e < 6; ++e) {
    bool first = true;
#pragma unroll
    for (int f = 0; f < e; ++f) first = first && tgt[f] != tgt[e];
    if (!first) continue;
    double sum = val[e];
#pragma unroll
    for (int f = e + 1; f < 6; ++f)
      if (tgt[f] == tgt[e]) sum += val[f];
    const size_t q = dir == 0 ? (size_t)b * g.nx + tgt[e] : (size_t)tgt[e] * g.nx + b;
    out[c * n + q] += scale * sum;
  }
}

}  // namespace hy
