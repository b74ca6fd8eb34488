// stage_kernel.hpp -- the fused Runge-Kutta stage kernel (forward), templated on
// the arithmetic type of the spatial operator.
//
// One workgroup owns a TX x TY tile of cells.  It stages the tile plus three
// ghost layers on each side (a "cross": x-halo on the tile's rows, y-halo on
// its columns; boundary conditions applied while loading) in LDS, and then,
// without touching HBM again until the store:
//   1. primitive variables and the globally Lax-Friedrichs split fluxes
//      f+- = (F(U) +- alpha_x U) / 2 of every x-point (Sect. 2.1),
//   2. WENO5 reconstruction at every x-face of the tile, a run of four
//      consecutive faces of one component per work item (the runs share the
//      stencils' second differences; the last face of every row is a task of
//      its own): F^ = W(f+ upwind-left) + W(f- upwind-right); with the
//      characteristic option one whole face per work item (char_face),
//   3. the same in y with alpha_y (skipped in the 1D limit),
//   4. per cell: divergence, sources of Eq. euler2D (gravity, cylindrical
//      geometric terms), the SSP-RK3 stage combination in FP64, the optional
//      atmosphere floors, the positivity check, and the maxima of |u|+c, |v|+c,
//      c+|u|+|v| of the new state, reduced across the workgroup and merged
//      with one atomic max per quantity: the next stage's global LF speeds and
//      the next step's CFL speed cost no extra pass over the grid.
//
// With R = double every formula below is evaluated with the same IEEE
// operations in the same order as the CPU oracle's (fma where it uses fma,
// nothing else fused: the FP64 translation unit is built with
// -ffp-contract=off), so the two agree bit for bit.  With R = float
// (HYDRO_FP32_BULK) the spatial operator is evaluated in FP32 with hardware
// reciprocal/sqrt approximations and free contraction; states, the stage
// combination and the reductions stay FP64.
#pragma once

#include "hydro_internal.hpp"
#include "ieee.hpp"

namespace hy {

__device__ __forceinline__ double as_double(unsigned long long b) { return __longlong_as_double((long long)b); }
__device__ __forceinline__ unsigned long long as_bits(double d) {
  return (unsigned long long)__double_as_longlong(d);
}

// Index of the source cell of (possibly ghost) index gi on an axis of n cells,
// and whether the momentum normal to that axis changes sign (reflecting).
// Indices beyond the three ghost layers only occur for tile cells past the
// grid edge, whose results are discarded; they are clamped into range.
__device__ __forceinline__ int map_index(int gi, int n, int lo, int hi, bool& flip) {
  flip = false;
  int s = gi;
  if (gi < 0) {
    if (lo == PERIODIC) s = gi + n;
    else if (lo == TRANSMISSIVE) s = 0;
    else { s = -gi - 1; flip = true; }
  } else if (gi >= n) {
    if (hi == PERIODIC) s = gi - n;
    else if (hi == TRANSMISSIVE) s = n - 1;
    else { s = 2 * n - 1 - gi; flip = true; }
  }
  s = s < 0 ? 0 : (s >= n ? n - 1 : s);
  return s;
}

template <typename R> struct Prim { R u, v, p, c; };

// ---------------------------------------------------------------- FP64 path
// Same operations, same order as the oracle.

__device__ __forceinline__ Prim<double> prim(double r, double mx, double my, double E,
                                             double gamma, double gm1) {
  Prim<double> w;
  double rinv = cr_rcp_pos(r);
  w.u = mx * rinv;
  w.v = my * rinv;
  double ke2 = mx * w.u + my * w.v;
  w.p = gm1 * (E - 0.5 * ke2);
  w.c = cr_sqrt_pos((gamma * w.p) * rinv);
  return w;
}

// Second difference of three consecutive stencil values (in stencil order)
// and 13/12 times it: the first term of a smoothness indicator.  Neighbouring
// faces' stencils share their middle points, so a run of faces computes each
// point's pair once.
struct D2 {
  double d, cd;
};
__device__ __forceinline__ D2 d2_at(double l, double m, double r) {
  const double d = __builtin_fma(-2.0, m, l) + r;
  return {d, (13.0 / 12.0) * d};
}

// WENO5-JS at the right face of v2 as numerator and denominator (weights over
// the common denominator 10 s0 s1 s2, s_k = (eps + beta_k)^2): W = num / den;
// given the second differences of the candidate stencils (v0 v1 v2),
// (v1 v2 v3), (v2 v3 v4).
__device__ __forceinline__ void weno5_nd_d2(double v0, double v1, double v2, double v3, double v4, D2 t0,
                                            D2 t1, D2 t2, double eps, double& num, double& den) {
  double e = __builtin_fma(3.0, v2, __builtin_fma(-4.0, v1, v0));
  double b0 = __builtin_fma(t0.cd, t0.d, (0.25 * e) * e);
  e = v1 - v3;
  double b1 = __builtin_fma(t1.cd, t1.d, (0.25 * e) * e);
  e = __builtin_fma(-4.0, v3, 3.0 * v2) + v4;
  double b2 = __builtin_fma(t2.cd, t2.d, (0.25 * e) * e);
  double p0 = __builtin_fma(11.0, v2, __builtin_fma(-7.0, v1, 2.0 * v0));
  double p1 = __builtin_fma(5.0, v2, __builtin_fma(2.0, v3, -v1));
  double p2 = __builtin_fma(5.0, v3, __builtin_fma(2.0, v2, -v4));
  double s0 = (eps + b0) * (eps + b0);
  double s1 = (eps + b1) * (eps + b1);
  double s2 = (eps + b2) * (eps + b2);
  double w0 = s1 * s2;
  double w1 = 6.0 * (s0 * s2);
  double w2 = 3.0 * (s0 * s1);
  num = __builtin_fma(w2, p2, __builtin_fma(w1, p1, w0 * p0));
  den = 6.0 * ((w0 + w1) + w2);
}

__device__ __forceinline__ void weno5_nd(double v0, double v1, double v2, double v3, double v4, double eps,
                                         double& num, double& den) {
  weno5_nd_d2(v0, v1, v2, v3, v4, d2_at(v0, v1, v2), d2_at(v1, v2, v3), d2_at(v2, v3, v4), eps, num, den);
}

// Face value of a split flux: left-biased reconstruction of the f+ stencil
// p0..p4 plus right-biased reconstruction of the f- stencil m0..m4 (upwind
// order), over one common denominator, (n+ d- + n- d+) / (d+ d-): one division
// per face; symmetric in the two sides.
__device__ __forceinline__ double weno5_face(double p0, double p1, double p2, double p3, double p4,
                                             double m0, double m1, double m2, double m3, double m4,
                                             double eps) {
  double np, dp, nm, dm;
  weno5_nd(p0, p1, p2, p3, p4, eps, np, dp);
  weno5_nd(m0, m1, m2, m3, m4, eps, nm, dm);
  return cr_div_pos_normal(np * dm + nm * dp, dp * dm);  // dp, dm > 0: sums of positive weights
}

__device__ __forceinline__ double lf_fma(double a, double b, double c) { return __builtin_fma(a, b, c); }

// ---------------------------------------------------------------- FP32 path

__device__ __forceinline__ float rcpf(float x) { return __builtin_amdgcn_rcpf(x); }

__device__ __forceinline__ Prim<float> prim(float r, float mx, float my, float E, float gamma,
                                            float gm1) {
  Prim<float> w;
  float rinv = rcpf(r);
  w.u = mx * rinv;
  w.v = my * rinv;
  w.p = gm1 * (E - 0.5f * (mx * w.u + my * w.v));
  w.c = __builtin_amdgcn_sqrtf(gamma * w.p * rinv);
  return w;
}

// Textbook weights a_k = d_k / s_k with hardware reciprocals (no overflow of
// the products in single precision); t0..t2 are 13/12 times the squared
// second differences of the three candidate stencils, which a run of faces
// shares between neighbouring stencils.
__device__ __forceinline__ float sq2_at(float l, float m, float r) {
  const float d = l - 2.0f * m + r;
  return (13.0f / 12.0f) * d * d;
}
__device__ __forceinline__ float weno5_t(float v0, float v1, float v2, float v3, float v4, float t0, float t1,
                                         float t2, float eps) {
  float e = v0 - 4.0f * v1 + 3.0f * v2;
  float b0 = t0 + 0.25f * e * e;
  e = v1 - v3;
  float b1 = t1 + 0.25f * e * e;
  e = 3.0f * v2 - 4.0f * v3 + v4;
  float b2 = t2 + 0.25f * e * e;
  float s0 = eps + b0, s1 = eps + b1, s2 = eps + b2;
  float a0 = 0.1f * rcpf(s0 * s0);
  float a1 = 0.6f * rcpf(s1 * s1);
  float a2 = 0.3f * rcpf(s2 * s2);
  float p0 = 2.0f * v0 - 7.0f * v1 + 11.0f * v2;
  float p1 = -v1 + 5.0f * v2 + 2.0f * v3;
  float p2 = 2.0f * v2 + 5.0f * v3 - v4;
  return (a0 * p0 + a1 * p1 + a2 * p2) * (rcpf(a0 + a1 + a2) * (1.0f / 6.0f));
}

__device__ __forceinline__ float weno5(float v0, float v1, float v2, float v3, float v4, float eps) {
  return weno5_t(v0, v1, v2, v3, v4, sq2_at(v0, v1, v2), sq2_at(v1, v2, v3), sq2_at(v2, v3, v4), eps);
}

__device__ __forceinline__ float lf_fma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// ---------------------------------------------------------- split fluxes

// f+- = (F(U) +- alpha U) / 2 in direction DIR (0: x, 1: y), given the
// point's primitive variables w (its sound speed is not used).
template <int DIR, typename R>
__device__ __forceinline__ void split_flux_prim(const R U[4], const Prim<R>& w, R alpha, R fp[4], R fm[4]) {
  R F[4];
  if (DIR == 0) {
    F[0] = U[1];
    F[1] = lf_fma(U[1], w.u, w.p);
    F[2] = U[2] * w.u;
    F[3] = (U[3] + w.p) * w.u;
  } else {
    F[0] = U[2];
    F[1] = U[1] * w.v;
    F[2] = lf_fma(U[2], w.v, w.p);
    F[3] = (U[3] + w.p) * w.v;
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    fp[c] = R(0.5) * lf_fma(alpha, U[c], F[c]);
    fm[c] = R(0.5) * lf_fma(-alpha, U[c], F[c]);
  }
}

template <int DIR, typename R>
__device__ __forceinline__ void split_flux(const R U[4], R gamma, R gm1, R alpha, R fp[4], R fm[4]) {
  split_flux_prim<DIR>(U, prim(U[0], U[1], U[2], U[3], gamma, gm1), alpha, fp, fm);
}

// ------------------------------------------- characteristic-wise faces (FP64)

__device__ __forceinline__ double dot4(double a0, double a1, double a2, double a3, const double b[4]) {
  return __builtin_fma(a3, b[3], __builtin_fma(a2, b[2], __builtin_fma(a1, b[1], a0 * b[0])));
}

// Face value between stencil points 2 and 3 of a line whose points sit at
// base + k * st (k = 0..5) in LDS: F = split fluxes [8][np] (f+ then f-,
// components rho, m_x, m_y, E), Q = [4][np] per point sqrt(rho), u, v,
// H = (E + p)/rho.  The split fluxes are projected on the left eigenvectors of
// the flux Jacobian at the Roe average of points 2 and 3, in the frame
// (rho, m_n, m_t, E) (n = x for DIR 0, y for DIR 1), reconstructed field by
// field, and mapped back with the right eigenvectors.  The oracle's
// operations in the oracle's order.  Returns false when the averaged sound
// speed is not real.
template <int DIR>
__device__ __forceinline__ bool char_face(const double* F, const double* Q, int np, int base, int st,
                                          double gm1, double eps, double out[4]) {
  constexpr int CN = DIR == 0 ? 1 : 2, CT = DIR == 0 ? 2 : 1;
  const int il = base + 2 * st, ir = base + 3 * st;
  const double sl = Q[il], sr = Q[ir];
  const double nl = Q[(1 + DIR) * np + il], nr = Q[(1 + DIR) * np + ir];
  const double tl = Q[(2 - DIR) * np + il], tr = Q[(2 - DIR) * np + ir];
  const double Hl = Q[3 * np + il], Hr = Q[3 * np + ir];
  // (sqrt(rho) of two positive densities: den is a positive normal number;
  // for a face with c2 <= 0, reported as unphysical, the values are not used)
  const double den = sl + sr;
  const double un = cr_div_pos_normal(sl * nl + sr * nr, den);
  const double ut = cr_div_pos_normal(sl * tl + sr * tr, den);
  const double H = cr_div_pos_normal(sl * Hl + sr * Hr, den);
  const double q2 = un * un + ut * ut;
  const double c2 = gm1 * (H - 0.5 * q2);
  const bool ok = c2 > 0.0 && __builtin_isfinite(c2);
  const double c = cr_sqrt_pos(c2), ic = cr_rcp_pos(c);
  const double b1 = cr_div_pos_normal(gm1, c2), b2 = (0.5 * q2) * b1;
  double gh[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    double l0, l1, l2, l3;
    if (m == 0) { l0 = 0.5 * (b2 + un * ic); l1 = 0.5 * (-(b1 * un) - ic); l2 = -0.5 * (b1 * ut); l3 = 0.5 * b1; }
    else if (m == 1) { l0 = 1.0 - b2; l1 = b1 * un; l2 = b1 * ut; l3 = -b1; }
    else if (m == 2) { l0 = -ut; l1 = 0.0; l2 = 1.0; l3 = 0.0; }
    else { l0 = 0.5 * (b2 - un * ic); l1 = 0.5 * (ic - b1 * un); l2 = -0.5 * (b1 * ut); l3 = 0.5 * b1; }
    // Each projection consumes its four loads at once and each field is
    // finished before the next starts (the empty asm statements), so the
    // compiler does not hold the 48 stencil values of all fields in registers
    // at once: 103 VGPRs instead of 256 plus 32 accumulation registers, four
    // waves per SIMD instead of one.
    double g[6], h[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const int p = base + k * st;
      if (k < 5) {
        const double f[4] = {F[p], F[CN * np + p], F[CT * np + p], F[3 * np + p]};
        g[k] = dot4(l0, l1, l2, l3, f);
        asm volatile("" : "+v"(g[k]) : : "memory");
      }
      if (k > 0) {
        const double f[4] = {F[4 * np + p], F[(4 + CN) * np + p], F[(4 + CT) * np + p], F[7 * np + p]};
        h[k] = dot4(l0, l1, l2, l3, f);
        asm volatile("" : "+v"(h[k]) : : "memory");
      }
    }
    gh[m] = weno5_face(g[0], g[1], g[2], g[3], g[4], h[5], h[4], h[3], h[2], h[1], eps);
    asm volatile("" : "+v"(gh[m]) : : "memory");
  }
  const double r0 = dot4(1.0, 1.0, 0.0, 1.0, gh);
  const double r1 = dot4(un - c, un, 0.0, un + c, gh);
  const double r2 = dot4(ut, ut, 1.0, ut, gh);
  const double r3 = dot4(H - un * c, 0.5 * q2, ut, H + un * c, gh);
  out[0] = r0;
  out[CN] = r1;
  out[CT] = r2;
  out[3] = r3;
  return ok;
}

// Face value of one component from its split-flux stencils in LDS: P points
// at f+ of the face's fourth-left point, M at f- of the same point, st is the
// point stride; the face lies between points 2 and 3.
template <typename R>
__device__ __forceinline__ R face_value(const R* P, const R* M, int st, R eps) {
  if constexpr (sizeof(R) == 8)
    return weno5_face(P[0], P[st], P[2 * st], P[3 * st], P[4 * st], M[5 * st], M[4 * st], M[3 * st],
                      M[2 * st], M[st], eps);
  else
    return weno5(P[0], P[st], P[2 * st], P[3 * st], P[4 * st], eps) +
           weno5(M[5 * st], M[4 * st], M[3 * st], M[2 * st], M[st], eps);
}

// Face values of a run of NR consecutive faces of one component: P and M
// point at f+ and f- of the first face's fourth-left point, st is the point
// stride; face j lies between points j + 2 and j + 3, its f+ stencil is
// P[j .. j + 4] and its f- stencil M[j + 5 .. j + 1] (upwind first).  In FP64
// each point's second differences (one pair for the f+ stencils, one for the
// f- stencils, which run the other way) are computed once for the run; every
// value is the one face_value gives.
template <int NR, typename R>
__device__ __forceinline__ void face_run(const R* P, const R* M, int st, R eps, R out[NR]) {
  if constexpr (sizeof(R) == 8) {
    D2 sp[NR + 3], sm[NR + 4];  // sp[k]: around P[k]; sm[k]: around M[k] (taken from M[k + 1] down)
#pragma unroll
    for (int j = 0; j < NR; ++j) {
      if (j == 0) {
        sp[1] = d2_at(P[0], P[st], P[2 * st]);
        sp[2] = d2_at(P[st], P[2 * st], P[3 * st]);
        sm[2] = d2_at(M[3 * st], M[2 * st], M[st]);
        sm[3] = d2_at(M[4 * st], M[3 * st], M[2 * st]);
      }
      sp[j + 3] = d2_at(P[(j + 2) * st], P[(j + 3) * st], P[(j + 4) * st]);
      sm[j + 4] = d2_at(M[(j + 5) * st], M[(j + 4) * st], M[(j + 3) * st]);
      double np, dp, nm, dm;
      weno5_nd_d2(P[j * st], P[(j + 1) * st], P[(j + 2) * st], P[(j + 3) * st], P[(j + 4) * st], sp[j + 1],
                  sp[j + 2], sp[j + 3], eps, np, dp);
      weno5_nd_d2(M[(j + 5) * st], M[(j + 4) * st], M[(j + 3) * st], M[(j + 2) * st], M[(j + 1) * st],
                  sm[j + 4], sm[j + 3], sm[j + 2], eps, nm, dm);
      out[j] = cr_div_pos_normal(np * dm + nm * dp, dp * dm);  // dp, dm > 0: sums of positive weights
      asm volatile("" : "+v"(out[j]) : : "memory");  // one face at a time: few live registers
    }
  } else {
    // single precision: the squared second-difference terms shared the same way
    R tp[NR + 3], tm[NR + 4];
#pragma unroll
    for (int j = 0; j < NR; ++j) {
      if (j == 0) {
        tp[1] = sq2_at(P[0], P[st], P[2 * st]);
        tp[2] = sq2_at(P[st], P[2 * st], P[3 * st]);
        tm[2] = sq2_at(M[3 * st], M[2 * st], M[st]);
        tm[3] = sq2_at(M[4 * st], M[3 * st], M[2 * st]);
      }
      tp[j + 3] = sq2_at(P[(j + 2) * st], P[(j + 3) * st], P[(j + 4) * st]);
      tm[j + 4] = sq2_at(M[(j + 5) * st], M[(j + 4) * st], M[(j + 3) * st]);
      out[j] = weno5_t(P[j * st], P[(j + 1) * st], P[(j + 2) * st], P[(j + 3) * st], P[(j + 4) * st],
                       tp[j + 1], tp[j + 2], tp[j + 3], eps) +
               weno5_t(M[(j + 5) * st], M[(j + 4) * st], M[(j + 3) * st], M[(j + 2) * st], M[(j + 1) * st],
                       tm[j + 4], tm[j + 3], tm[j + 2], eps);
      asm volatile("" : "+v"(out[j]) : : "memory");
    }
  }
}

// Max of a non-negative x over the wavefront, valid in lane 63 (exact: a max
// of doubles).  DPP row shifts by 1, 2, 4, 8 (a lane with no source reads 0)
// leave each 16-lane row's max in its lane 15; row_bcast:15 and
// row_bcast:31 then carry the row maxima up to the last row.  No LDS round
// trips, unlike lane shuffles.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_move(double old, double x) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(x);
  const unsigned long long o = (unsigned long long)__double_as_longlong(old);
  const unsigned lo =
      (unsigned)__builtin_amdgcn_update_dpp((int)(unsigned)o, (int)(unsigned)b, CTRL, ROWS, 0xF, true);
  const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp((int)(unsigned)(o >> 32), (int)(unsigned)(b >> 32),
                                                            CTRL, ROWS, 0xF, true);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ double wave_max_nonneg(double x) {
  x = __builtin_fmax(x, dpp_move<0x111, 0xF>(0.0, x));  // row_shr:1
  x = __builtin_fmax(x, dpp_move<0x112, 0xF>(0.0, x));  // row_shr:2
  x = __builtin_fmax(x, dpp_move<0x114, 0xF>(0.0, x));  // row_shr:4
  x = __builtin_fmax(x, dpp_move<0x118, 0xF>(0.0, x));  // row_shr:8
  x = __builtin_fmax(x, dpp_move<0x142, 0xA>(x, x));    // row_bcast:15 into rows 1, 3
  x = __builtin_fmax(x, dpp_move<0x143, 0xC>(x, x));    // row_bcast:31 into rows 2, 3
  return x;
}

// Max over the NSUB sub-slots of ring slot s, by wavefront 0, broadcast to the
// block through LDS.  Every work item of the block must call it.
__device__ __forceinline__ void read_slot(const Ctl* ctl, int s, double out[3], double* sh) {
  static_assert(NSUB == 64, "one sub-slot per lane of a wavefront");
  if (threadIdx.x < NSUB) {
    const unsigned long long* p = ctl->slot[s][threadIdx.x];
    const double m0 = wave_max_nonneg(as_double(p[0]));
    const double m1 = wave_max_nonneg(as_double(p[1]));
    const double m2 = wave_max_nonneg(as_double(p[2]));
    if (threadIdx.x == NSUB - 1) {
      sh[0] = m0;
      sh[1] = m1;
      sh[2] = m2;
    }
  }
  __syncthreads();
  out[0] = sh[0];
  out[1] = sh[1];
  out[2] = sh[2];
}

// Block index -> tile index.  Workgroups are dispatched round-robin over the
// 8 XCDs; remapping so that each XCD receives a contiguous run of tiles
// (whole tile rows) keeps neighbouring tiles' shared halo rows in the same L2.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  if (nb % 8 != 0) return b;
  return (b % 8) * (nb / 8) + b / 8;
}

// Wide grids (256 or more tile columns): within each XCD's run of whole tile
// rows, bands of 64 tile columns are taken one after another, row by row
// inside a band.  The tiles an XCD holds at once then span about three tile
// rows of one band and read their shared halo rows from its L2; in plain row
// order across such a grid a tile row's halo is evicted before the row below
// needs it (4096^2: 1.31x the algorithmic HBM bytes, 1.01x banded).
__device__ __forceinline__ int xcd_band_tile(int b, int nb, int ntx) {
  constexpr int W = 64;
  if (nb % 8 != 0 || ntx < 256 || ntx % W != 0) return xcd_tile(b, nb);
  const int per = nb / 8;  // tiles per XCD
  if (per % ntx != 0) return xcd_tile(b, nb);
  const int rows = per / ntx;
  const int x = b % 8, l = b / 8;  // XCD, index within its run
  const int band = l / (rows * W), r = (l % (rows * W)) / W, c = l % W;
  return x * per + r * ntx + band * W + c;
}

// Per-point inputs of the Roe average: sqrt(rho), u, v, H = (E + p)/rho.
template <typename R>
__device__ __forceinline__ void store_roe_inputs(const R U[4], R gamma, R gm1, R* Q, int np, int k) {
  const Prim<R> w = prim(U[0], U[1], U[2], U[3], gamma, gm1);
  Q[k] = cr_sqrt(U[0]);
  Q[np + k] = w.u;
  Q[2 * np + k] = w.v;
  Q[3 * np + k] = cr_div(U[3] + w.p, U[0]);
}

template <typename R, int TX, int TY, bool HASY, bool CHAR = false>
__global__ __launch_bounds__(TX * TY) void stage_kernel(StageArgs a) {
  constexpr int NT = TX * TY;  // work items, one per cell of the tile
  constexpr int GY = HASY ? NG : 0;
  constexpr int TXP = TX + 2 * NG;
  constexpr int TYP = TY + 2 * GY;
  constexpr int NPX = TY * TXP;
  constexpr int NPY = HASY ? TYP * TX : 0;
  constexpr int NP = NPX > NPY ? NPX : NPY;
  constexpr int NFX = TY * (TX + 1);
  constexpr int NFY = HASY ? (TY + 1) * TX : 0;
  constexpr int NF = NFX > NFY ? NFX : NFY;
  constexpr int NW = (NT + 63) / 64;
  static_assert(NT % 64 == 0, "whole wavefronts");
  static_assert(TX % 4 == 0 && (!HASY || TY % 4 == 0), "runs of four faces tile the rows and columns");

  static_assert(8 * NP >= 4 * NF, "face values fit in the split-flux storage");
  static_assert(!CHAR || sizeof(R) == 8, "characteristic faces are FP64 only");
  // split fluxes (f+ in 0..3, f- in 4..7); characteristic faces add per point
  // sqrt(rho), u, v, H (8..11)
  __shared__ R sF[CHAR ? 12 : 8][NP];
  bool fbad = false;
  __shared__ double sRed[NW][3];

  const Geom& g = a.g;
  Ctl* ctl = a.ctl;
  const int tid = threadIdx.x;
  const bool lead = (blockIdx.x == 0 && tid == 0);

  const int ntx = (g.nx + TX - 1) / TX;
  const int tile = xcd_band_tile(blockIdx.x, gridDim.x, ntx);
  const int i0 = (tile % ntx) * TX;
  const int j0 = (tile / ntx) * TY;
  const size_t n = (size_t)g.nx * g.ny;
  const R gamma = (R)g.gamma, gm1 = (R)g.gm1, eps = (R)g.eps;

  // State of a (possibly ghost) point, fetched into registers ahead of its
  // use; the boundary conditions (index map, reflection sign) are applied on
  // use.
  struct Pt {
    double v[4];
    bool fx, fy;
  };
  // A tile whose ghost layers all lie inside the grid needs no index map.
  const bool interior = i0 >= NG && i0 + TX + NG <= g.nx && (!HASY || (j0 >= NG && j0 + TY + NG <= g.ny));
  auto fetch_point = [&](int I, int J, Pt& p) {
    size_t q;
    if (interior) {
      p.fx = false;
      p.fy = false;
      q = (size_t)J * g.nx + I;
    } else {
      p.fy = false;
      const int si = map_index(I, g.nx, g.bc[0], g.bc[1], p.fx);
      const int sj = HASY ? map_index(J, g.ny, g.bc[2], g.bc[3], p.fy) : 0;
      q = (size_t)sj * g.nx + si;
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) p.v[c] = a.V[c * n + q];
  };
  auto point_state = [&](const Pt& p, R U[4]) {
    U[0] = (R)p.v[0];
    U[1] = (R)(p.fx ? -p.v[1] : p.v[1]);
    U[2] = (R)(p.fy ? -p.v[2] : p.v[2]);
    U[3] = (R)p.v[3];
  };

  // The x sweep's points and the control block are requested together, before
  // anything waits for either: their latencies overlap.  Work item (tx, ty)
  // takes the tile cell (tx, ty) (its primitive variables serve both sweeps
  // and the per-cell phase) and the first TY * 2 NG work items one x-halo
  // point each.  A cell past the grid edge is fetched through the index map
  // of both axes: it is a ghost point only along the axis it lies within, and
  // its values along the other are discarded.
  const int tx = tid % TX, ty = tid / TX;
  constexpr int NHX = TY * 2 * NG;
  Pt own, hx;
  fetch_point(i0 + tx, j0 + ty, own);
  const bool has_hx = tid < NHX;
  int khx = 0;
  if (has_hx) {
    const int j = tid / (2 * NG), c = tid - j * (2 * NG);
    const int lx = c < NG ? c : c + TX;
    khx = j * TXP + lx;
    fetch_point(i0 + lx - NG, j0 + j, hx);
  }
  const bool device_dt = !a.rhs_only && a.dt_mode == 1;
  double t_prev = 0.0, dt_prev = 0.0;
  int active_prev = 1;
  if (device_dt) {
    t_prev = ctl->t;
    dt_prev = ctl->dt;
    active_prev = ctl->active;
  }

  // ---- speeds of this stage's input (LF alphas; CFL speed for stage 0)
  __shared__ double sSlot[3];
  double sp[3] = {a.fax, a.fay, 0.0};
  const bool use_slot = !a.rhs_only && (!a.frozen || a.dt_mode == 1);
  if (use_slot) read_slot(ctl, a.stage, sp, sSlot);

  // ---- time step and whether this step is taken
  double dt = a.dt_host;
  bool active = true;
  if (device_dt) {
    if (a.stage == 0) {
      active = !(a.t_end > 0.0) || (t_prev < a.t_end);
      dt = cr_div(g.cfl_dmin, sp[2]);
      if (a.t_end > 0.0 && t_prev + dt > a.t_end) dt = a.t_end - t_prev;
      if (lead) {
        ctl->active = active ? 1 : 0;
        ctl->dt = dt;
        if (active && a.dt_rec) *a.dt_rec = dt;
      }
    } else {
      dt = dt_prev;
      active = active_prev != 0;
    }
  }
  if (!active) return;
  // In a launch whose workgroups are all resident at once, issue priority
  // falls as a workgroup advances (3: x sweep, 2: y sweep, 1: per-cell
  // phase), so the workgroups sharing a compute unit progress together
  // instead of the last one running its latency-bound tail alone.
  if (a.prio) __builtin_amdgcn_s_setprio(3);

  const double ax = a.frozen || a.rhs_only ? a.fax : sp[0];
  const double ay = a.frozen || a.rhs_only ? a.fay : sp[1];
  if (!a.rhs_only && !a.frozen && blockIdx.x == 0 && tid < NSUB) {
    // clear the slot two stages ahead (one sub-slot per lane)
    unsigned long long* z = ctl->slot[(a.stage + 2) % 3][tid];
    z[0] = 0ull;
    z[1] = 0ull;
    z[2] = 0ull;
  }
  if (lead && !a.rhs_only) {
    const int s = a.stage;
    if (a.alpha_rec) {
      a.alpha_rec[s] = ax;
      a.alpha_rec[3 + s] = ay;
    }
    if (s == 2 && a.dt_mode == 1) {
      ctl->t = t_prev + dt;
      ctl->steps = ctl->steps + 1;
    }
  }

  R D[4] = {R(0), R(0), R(0), R(0)};
  Prim<R> wo;  // primitive variables of the work item's cell (stage input)

  // ---- 1. x sweep: split fluxes of the tile rows and their x-halo points
  // (read straight from L2 into registers; only the split fluxes live in LDS),
  // then one (face, component) per work item (a whole face for the
  // characteristic option), face values parked in registers until every
  // stencil read is done, then written over the split fluxes.
  {
    const R al = (R)ax;
    {
      R U[4];
      point_state(own, U);
      wo = prim(U[0], U[1], U[2], U[3], gamma, gm1);
      R fp[4], fm[4];
      split_flux_prim<0>(U, wo, al, fp, fm);
      const int k = ty * TXP + tx + NG;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        sF[c][k] = fp[c];
        sF[4 + c][k] = fm[c];
      }
      if constexpr (CHAR) store_roe_inputs(U, gamma, gm1, &sF[8][0], NP, k);
    }
    if (has_hx) {
      R U[4];
      point_state(hx, U);
      R fp[4], fm[4];
      split_flux<0>(U, gamma, gm1, al, fp, fm);
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        sF[c][khx] = fp[c];
        sF[4 + c][khx] = fm[c];
      }
      if constexpr (CHAR) store_roe_inputs(U, gamma, gm1, &sF[8][0], NP, khx);
    }
    __syncthreads();
    // faces: work item (tx, ty) takes face tx of row ty for all four
    // components; the last face of every row (f = TX) is split into 4 * TY
    // single-component tasks for the first work items.
    R* sFh = &sF[0][0];  // [4][TY][TX + 1], reusing the split-flux storage
    if constexpr (CHAR) {
      // one whole face per work item; the last face of every row for the first TY
      R fh[4], fe[4];
      fbad |= !char_face<0>(&sF[0][0], &sF[8][0], NP, ty * TXP + tx, 1, g.gm1, g.eps, fh);
      const bool extra = tid < TY;
      if (extra) fbad |= !char_face<0>(&sF[0][0], &sF[8][0], NP, tid * TXP + TX, 1, g.gm1, g.eps, fe);
      __syncthreads();
#pragma unroll
      for (int c = 0; c < 4; ++c) sFh[c * NFX + ty * (TX + 1) + tx] = fh[c];
      if (extra) {
#pragma unroll
        for (int c = 0; c < 4; ++c) sFh[c * NFX + tid * (TX + 1) + TX] = fe[c];
      }
    } else {
      // a run of four faces of one component per work item: faces 4q .. 4q + 3
      // of row r (component c = tid / (TY TX / 4), rows in consecutive
      // lanes), then the last face of every row (f = TX) for the first 4 TY
      // work items
      R fh[4], fe = R(0);
      const int rc = tid / (TY * (TX / 4)), rrem = tid - rc * (TY * (TX / 4));
      const int rr = rrem % TY, rq = rrem / TY;
      face_run<4>(&sF[rc][rr * TXP + 4 * rq], &sF[4 + rc][rr * TXP + 4 * rq], 1, eps, fh);
      const bool extra = tid < 4 * TY;
      const int ec = tid / TY, ej = tid - ec * TY;
      if (extra) fe = face_value(&sF[ec][ej * TXP + TX], &sF[4 + ec][ej * TXP + TX], 1, eps);
      __syncthreads();
#pragma unroll
      for (int j = 0; j < 4; ++j) sFh[rc * NFX + rr * (TX + 1) + 4 * rq + j] = fh[j];
      if (extra) sFh[ec * NFX + ej * (TX + 1) + TX] = fe;
    }
    __syncthreads();
    if (a.prio) __builtin_amdgcn_s_setprio(2);
    const R idx = (R)g.idx;
    {
#pragma unroll
      for (int c = 0; c < 4; ++c)
        D[c] = (sFh[c * NFX + ty * (TX + 1) + tx + 1] - sFh[c * NFX + ty * (TX + 1) + tx]) * idx;
    }
  }

  // ---- 2. y sweep (skipped in the 1D limit), same pattern
  R Dy[4] = {R(0), R(0), R(0), R(0)};
  if (HASY) {
    __syncthreads();  // the x face values are read; sF is reused
    const R al = (R)ay;
    {
      // the work item's cell, with its primitive variables from the x sweep
      R U[4];
      point_state(own, U);
      R fp[4], fm[4];
      split_flux_prim<1>(U, wo, al, fp, fm);
      const int k = (ty + GY) * TX + tx;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        sF[c][k] = fp[c];
        sF[4 + c][k] = fm[c];
      }
      if constexpr (CHAR) store_roe_inputs(U, gamma, gm1, &sF[8][0], NP, k);
    }
    if (tid < TX * 2 * GY) {  // one y-halo point each for the first TX * 2 NG work items
      const int r = tid / TX, i = tid - r * TX;
      const int ly = r < GY ? r : r + TY;
      const int k = ly * TX + i;
      Pt pt;
      fetch_point(i0 + i, j0 + ly - GY, pt);
      R U[4];
      point_state(pt, U);
      R fp[4], fm[4];
      split_flux<1>(U, gamma, gm1, al, fp, fm);
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        sF[c][k] = fp[c];
        sF[4 + c][k] = fm[c];
      }
      if constexpr (CHAR) store_roe_inputs(U, gamma, gm1, &sF[8][0], NP, k);
    }
    __syncthreads();
    // faces: work item (tx, ty) takes face ty of column tx for all four
    // components; the last face of every column (f = TY) is split into 4 * TX
    // single-component tasks.
    R* sFh = &sF[0][0];  // [4][TY + 1][TX]
    if constexpr (CHAR) {
      R fh[4], fe[4];
      fbad |= !char_face<1>(&sF[0][0], &sF[8][0], NP, ty * TX + tx, TX, g.gm1, g.eps, fh);
      const bool extra = tid < TX;
      if (extra) fbad |= !char_face<1>(&sF[0][0], &sF[8][0], NP, TY * TX + tid, TX, g.gm1, g.eps, fe);
      __syncthreads();
#pragma unroll
      for (int c = 0; c < 4; ++c) sFh[c * NFY + ty * TX + tx] = fh[c];
      if (extra) {
#pragma unroll
        for (int c = 0; c < 4; ++c) sFh[c * NFY + TY * TX + tid] = fe[c];
      }
    } else {
      // a run of four faces 4q .. 4q + 3 of column i and one component per
      // work item (columns in consecutive lanes), then the last face of every
      // column (f = TY) for the first 4 TX work items
      R fh[4], fe = R(0);
      const int rc = tid / (TX * (TY / 4)), rrem = tid - rc * (TX * (TY / 4));
      const int ri = rrem % TX, rq = rrem / TX;
      face_run<4>(&sF[rc][4 * rq * TX + ri], &sF[4 + rc][4 * rq * TX + ri], TX, eps, fh);
      const bool extra = tid < 4 * TX;
      const int ec = tid / TX, ei = tid - ec * TX;
      if (extra) fe = face_value(&sF[ec][TY * TX + ei], &sF[4 + ec][TY * TX + ei], TX, eps);
      __syncthreads();
#pragma unroll
      for (int j = 0; j < 4; ++j) sFh[rc * NFY + (4 * rq + j) * TX + ri] = fh[j];
      if (extra) sFh[ec * NFY + TY * TX + ei] = fe;
    }
    __syncthreads();
    if (a.prio) __builtin_amdgcn_s_setprio(1);
    const R idy = (R)g.idy;
    {
#pragma unroll
      for (int c = 0; c < 4; ++c)
        Dy[c] = (sFh[c * NFY + (ty + 1) * TX + tx] - sFh[c * NFY + ty * TX + tx]) * idy;
    }
  }

  // ---- 3. per cell: sources, L, stage combination, floors, check, maxima
  const int I = i0 + tx, J = j0 + ty;
  const bool act = I < g.nx && J < g.ny;
  double amax = 0.0, bmax = 0.0, smax = 0.0;
  bool bad = false;
  if (act) {
    const size_t q = (size_t)J * g.nx + I;
    double v[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) v[c] = a.V[c * n + q];
    const R r = (R)v[0], mx = (R)v[1], my = (R)v[2], E = (R)v[3];
    const R gxv = g.grav ? (R)g.grav[q] : (R)g.gx;
    const R gyv = g.grav ? (R)g.grav[n + q] : (R)g.gy;
    R S[4];
    S[0] = R(0);
    S[1] = r * gxv;
    S[2] = r * gyv;
    S[3] = mx * gxv + my * gyv;
    if (g.cyl) {
      const Prim<R>& w = wo;  // the cell's primitive variables (stage input)
      const double ri = g.xlo + ((double)I + 0.5) * g.dx;
      const R ir = (R)cr_rcp_pos(ri);
      S[0] = S[0] - ir * mx;
      S[1] = S[1] - ir * (mx * w.u);
      S[2] = S[2] - ir * (my * w.u);
      S[3] = S[3] - ir * ((E + w.p) * w.u);
    }
    R L[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) L[c] = HASY ? S[c] - (D[c] + Dy[c]) : S[c] - D[c];
    if (a.rhs_only) {
#pragma unroll
      for (int c = 0; c < 4; ++c) a.W[c * n + q] = (double)L[c];
    } else {
      double w[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const double u0 = a.U0[c * n + q];
        w[c] = __builtin_fma(a.b, __builtin_fma(dt, (double)L[c], v[c] - u0), u0);
      }
      // primitive variables of the new state (after the floors: those of the
      // floored state are reused unless the pressure floor changed E)
      Prim<double> pw;
      bool fresh = true;
      if (g.floor_on) {  // atmosphere: minimum density, then minimum pressure
        if (w[0] < g.rho_floor) {
          w[0] = g.rho_floor;
          w[1] = 0.0;
          w[2] = 0.0;
          w[3] = g.e_floor;
        }
        pw = prim(w[0], w[1], w[2], w[3], g.gamma, g.gm1);
        if (pw.p < g.p_floor) w[3] = g.e_floor + 0.5 * (w[1] * pw.u + w[2] * pw.v);
        else fresh = false;
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) a.W[c * n + q] = w[c];
      if (fresh) pw = prim(w[0], w[1], w[2], w[3], g.gamma, g.gm1);
      bad = !(w[0] > 0.0) || !(pw.p > 0.0) || !__builtin_isfinite(pw.c);
      amax = __builtin_fabs(pw.u) + pw.c;
      bmax = __builtin_fabs(pw.v) + pw.c;
      smax = pw.c + (__builtin_fabs(pw.u) + __builtin_fabs(pw.v));
    }
  }
  bad = bad || fbad;
  if (a.rhs_only) {
    if constexpr (CHAR) {
      const int anyb = __syncthreads_or(bad ? 1 : 0);
      if (tid == 0 && anyb) atomicOr(&ctl->flag, 1);
    }
    return;
  }
  if (a.frozen) {  // a replay of recorded speeds needs no new maxima, only the check
    const int anybad = __syncthreads_or(bad ? 1 : 0);
    if (tid == 0 && anybad) atomicOr(&ctl->flag, 1);
    return;
  }

  // ---- maxima: within each wavefront (DPP), then LDS across the
  // workgroup's waves, then one atomic max per quantity (exact and
  // order-free).
  amax = wave_max_nonneg(amax);
  bmax = wave_max_nonneg(bmax);
  smax = wave_max_nonneg(smax);
  const int wave = tid / 64;
  if ((tid & 63) == 63) {
    sRed[wave][0] = amax;
    sRed[wave][1] = bmax;
    sRed[wave][2] = smax;
  }
  const int anybad = __syncthreads_or(bad ? 1 : 0);
  if (tid == 0) {
    amax = sRed[0][0];
    bmax = sRed[0][1];
    smax = sRed[0][2];
    for (int k = 1; k < NW; ++k) {
      amax = __builtin_fmax(amax, sRed[k][0]);
      bmax = __builtin_fmax(bmax, sRed[k][1]);
      smax = __builtin_fmax(smax, sRed[k][2]);
    }
    unsigned long long* slot = ctl->slot[(a.stage + 1) % 3][blockIdx.x % NSUB];
    atomicMax(&slot[0], as_bits(amax));
    atomicMax(&slot[1], as_bits(bmax));
    atomicMax(&slot[2], as_bits(smax));
    if (anybad) atomicOr(&ctl->flag, 1);
  }
}

// Whether nb workgroups of kernel k fit on the current device at once
// (resident workgroups per compute unit x compute units), cached per device in
// cap, which belongs to one kernel.
template <typename K>
bool one_round(K k, int threads, int nb, int* cap) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return false;
  if (cap[dev] == 0) {
    int per_cu = 0, ncu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, threads, 0) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return false;
    cap[dev] = per_cu * ncu > 0 ? per_cu * ncu : -1;
  }
  return nb <= cap[dev];
}

// Tile shapes: 16 x 16 cells (256 work items) in 2D; 256 x 1 in the 1D limit.
template <typename R, bool CHAR>
hipError_t launch_stage_variant(const StageArgs& a, hipStream_t s) {
  StageArgs b = a;
  if (a.g.has_y) {
    constexpr int TX = 16, TY = 16;
    static int cap[MAX_DEVICES];
    const auto k = stage_kernel<R, TX, TY, true, CHAR>;
    const int nb = ((a.g.nx + TX - 1) / TX) * ((a.g.ny + TY - 1) / TY);
    b.prio = one_round(k, TX * TY, nb, cap) ? 1 : 0;
    hipLaunchKernelGGL(k, dim3(nb), dim3(TX * TY), 0, s, b);
  } else {
    constexpr int TX = 256, TY = 1;
    static int cap[MAX_DEVICES];
    const auto k = stage_kernel<R, TX, TY, false, CHAR>;
    const int nb = (a.g.nx + TX - 1) / TX;
    b.prio = one_round(k, TX * TY, nb, cap) ? 1 : 0;
    hipLaunchKernelGGL(k, dim3(nb), dim3(TX * TY), 0, s, b);
  }
  return hipGetLastError();
}

template <typename R>
hipError_t launch_stage(const StageArgs& a, hipStream_t s) {
  if constexpr (sizeof(R) == 8) {
    if (a.g.charw) return launch_stage_variant<R, true>(a, s);
  }
  return launch_stage_variant<R, false>(a, s);
}

}  // namespace hy
