/*
 * hydro_oracle.c -- FP64 CPU oracle of the hydro update (TEST INFRASTRUCTURE).
 *
 * This file is test infrastructure.  Only the tests, the smoke entry point
 * and the CPU-baseline leg of the benchmark may load it.  The product path
 * (the HIP library) never links, calls or reads anything from here, and this
 * file shares no code, header or constant table with it.
 *
 * What it computes, one step of the semi-discrete Euler system of Sect. 2.1
 * (Eq. euler2D, with Qdot = 0 and a fixed gravity field g = -grad Phi):
 *
 *   dU/dt = L(U),   U = (rho, m_x, m_y, E)   (m = rho v, E = tau of Eq. euler2D)
 *   L(U)  = S(U) - (dF/dx + dG/dy)
 *
 * discretised as the paper's Sect. 2.1 describes it: finite-difference WENO
 * (fifth order, Jiang & Shu 1996, the scheme the paper cites) applied to the
 * two halves of a global Lax-Friedrichs flux splitting, summed at each face.
 * Time stepping is the three-stage third-order SSP Runge-Kutta scheme (the
 * "original prescription" the paper names in Sect. 2.1); the CFL time step
 * is Eq. of Sect. 5.3 (dt = c_cfl Delta / max(c_s + |v_r| + |v_z|)).
 *
 * Plain, slow and explicit: every stage copies the state into an array
 * padded with three ghost layers, computes primitives, split fluxes,
 * reconstructions and divergences in separate loops, one cell at a time.
 * Built with -fopenmp, the loops over rows (x sweep), columns (y sweep) and
 * cells are shared among threads.  Each row, column or cell is computed by
 * the same operations whichever thread takes it, and the only reductions are
 * maxima (exact, order-free) and an error flag, so the result is bit for bit
 * the same for any number of threads.  The compensated totals (orc_sums)
 * stay sequential: their rounding depends on the order.
 *
 * Readings of the paper (the paper prints no WENO formula and no rounding
 * rules; these choices are ours and are listed in the design notes):
 *  - point values at cell centres (finite-difference form, Sect. 2.1);
 *  - WENO-JS with eps = p->eps (1e-6 default, at least 1e-30) and exponent 2;
 *    the face value sums the two reconstructions over a common denominator
 *    (orc_weno5_face);
 *  - "global" LF: alpha_x = max over interior cells of |u|+c, alpha_y =
 *    max of |v|+c, recomputed from every stage's input, same for all four
 *    components (Sect. 2.1);
 *  - ideal-gas EOS p = (gamma-1) rho eps (Sect. 5.1);
 *  - ghost cells: periodic, transmissive (zero gradient, the paper's "free"
 *    boundary) or reflecting (mirror, normal momentum negated; the r = 0 axis
 *    and the z = 0 plane of Eq. euler2D are reflecting);
 *  - geometric sources of Eq. euler2D evaluated at r_i = xlo + (i+1/2) dx;
 *  - the paper names its scheme "WENO-Roe": besides the component-wise
 *    reconstruction of the split fluxes (what its text describes), recon = 1
 *    reconstructs them in the characteristic fields of the flux Jacobian at
 *    the Roe average of the two cells beside each face (char_face below).
 *
 * Rounding contract.  Every formula is written in one fixed evaluation
 * order; fma(a,b,c) is a single-rounding a*b+c (C99).  Build with
 * -ffp-contract=off so that the compiler fuses nothing else.  Where x and y
 * quantities are combined (kinetic energy, gravity work, c + |u| + |v|) the
 * order is symmetric, so that the update commutes bit for bit with swapping
 * the axes.  The WENO
 * weights are written over a common denominator (one division per
 * reconstruction), which is the Jiang-Shu formula multiplied through by
 * 10 * s0*s1*s2; see weno5() below.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NG 3 /* ghost layers: the five-point WENO stencil reaches 3 cells past a face */

enum { ORC_PERIODIC = 0, ORC_TRANSMISSIVE = 1, ORC_REFLECTING = 2 };
enum { ORC_OK = 0, ORC_E_INVALID = -1, ORC_E_NOMEM = -2, ORC_E_UNPHYSICAL = -4 };

typedef struct {
  int32_t nx, ny;             /* interior cells; ny == 1 is the 1D limit (no y sweep) */
  double xlo, xhi, ylo, yhi;  /* domain; cylindrical: x = r, y = z */
  int32_t geometry;           /* 0 Cartesian, 1 cylindrical (r,z) */
  int32_t bc[4];              /* x-low, x-high, y-low, y-high */
  double gamma, cfl, eps;
  double gx, gy;              /* uniform gravity (used when no field is given) */
  double rho_floor, p_floor;  /* atmosphere floors applied after each stage when rho_floor > 0 */
  int32_t recon;              /* 0 component-wise, 1 characteristic-wise reconstruction */
} orc_params;

/* ---------------------------------------------------------------- helpers */

static int check_params(const orc_params *p) {
  if (!p) return ORC_E_INVALID;
  if (p->nx < 3 || p->ny < 1 || (p->ny > 1 && p->ny < 3)) return ORC_E_INVALID;
  if (!(p->xhi > p->xlo) || !(p->yhi > p->ylo)) return ORC_E_INVALID;
  if (!(p->gamma > 1.0) || !(p->eps >= 1e-30)) return ORC_E_INVALID;
  for (int k = 0; k < 4; ++k)
    if (p->bc[k] < 0 || p->bc[k] > 2) return ORC_E_INVALID;
  if ((p->bc[0] == ORC_PERIODIC) != (p->bc[1] == ORC_PERIODIC)) return ORC_E_INVALID;
  if ((p->bc[2] == ORC_PERIODIC) != (p->bc[3] == ORC_PERIODIC)) return ORC_E_INVALID;
  if (p->geometry == 1 && p->xlo < 0.0) return ORC_E_INVALID;
  if (p->geometry != 0 && p->geometry != 1) return ORC_E_INVALID;
  if (p->recon != 0 && p->recon != 1) return ORC_E_INVALID;
  return ORC_OK;
}

static double cell_dx(const orc_params *p) { return (p->xhi - p->xlo) / (double)p->nx; }
static double cell_dy(const orc_params *p) { return (p->yhi - p->ylo) / (double)p->ny; }

/* Primitive variables from conserved ones (Sect. 2.1: tau = rho eps + rho v^2/2,
 * Sect. 5.1: p = (gamma-1) rho eps, c^2 = gamma p / rho). */
typedef struct { double u, v, p, c; } prim_t;

static prim_t cons_to_prim(double r, double mx, double my, double E, double gamma) {
  prim_t w;
  double rinv = 1.0 / r;
  w.u = mx * rinv;
  w.v = my * rinv;
  double ke2 = mx * w.u + my * w.v; /* m.v = 2 x kinetic energy density */
  w.p = (gamma - 1.0) * (E - 0.5 * ke2);
  w.c = sqrt((gamma * w.p) * rinv);
  return w;
}

/* Fifth-order WENO reconstruction (Jiang & Shu 1996) of the value at the
 * right face of v2 from the five point values v0..v4 (upwind side first).
 *
 * Textbook form: candidates q_k (third-order, one per three-point stencil),
 * smoothness indicators beta_k, linear weights d = (1/10, 6/10, 3/10),
 * a_k = d_k / (eps + beta_k)^2, omega_k = a_k / sum a, W = sum omega_k q_k.
 * Written here with p_k = 6 q_k and a_k scaled by 10 s0 s1 s2
 * (s_k = (eps + beta_k)^2):  w0 = s1 s2, w1 = 6 s0 s2, w2 = 3 s0 s1,
 * W = (w0 p0 + w1 p1 + w2 p2) / (6 (w0 + w1 + w2)).  Same value, one division. */
static void weno5_nd(double v0, double v1, double v2, double v3, double v4, double eps, double *num_out,
                     double *den_out) {
  const double c1312 = 13.0 / 12.0;
  double d, e;
  d = fma(-2.0, v1, v0) + v2;           /* v0 - 2 v1 + v2 */
  e = fma(3.0, v2, fma(-4.0, v1, v0));  /* v0 - 4 v1 + 3 v2 */
  double b0 = fma(c1312 * d, d, (0.25 * e) * e);
  d = fma(-2.0, v2, v1) + v3;           /* v1 - 2 v2 + v3 */
  e = v1 - v3;
  double b1 = fma(c1312 * d, d, (0.25 * e) * e);
  d = fma(-2.0, v3, v2) + v4;           /* v2 - 2 v3 + v4 */
  e = fma(-4.0, v3, 3.0 * v2) + v4;     /* 3 v2 - 4 v3 + v4 */
  double b2 = fma(c1312 * d, d, (0.25 * e) * e);

  double p0 = fma(11.0, v2, fma(-7.0, v1, 2.0 * v0)); /* 2 v0 - 7 v1 + 11 v2 */
  double p1 = fma(5.0, v2, fma(2.0, v3, -v1));         /* -v1 + 5 v2 + 2 v3 */
  double p2 = fma(5.0, v3, fma(2.0, v2, -v4));         /* 2 v2 + 5 v3 - v4 */

  double s0 = (eps + b0) * (eps + b0);
  double s1 = (eps + b1) * (eps + b1);
  double s2 = (eps + b2) * (eps + b2);
  double w0 = s1 * s2;
  double w1 = 6.0 * (s0 * s2);
  double w2 = 3.0 * (s0 * s1);
  *num_out = fma(w2, p2, fma(w1, p1, w0 * p0));
  *den_out = 6.0 * ((w0 + w1) + w2);
}

double orc_weno5(double v0, double v1, double v2, double v3, double v4, double eps) {
  double num, den;
  weno5_nd(v0, v1, v2, v3, v4, eps, &num, &den);
  return num / den;
}

/* Face value of the split flux: the left-biased reconstruction of the f+
 * stencil p0..p4 plus the right-biased one of the f- stencil m0..m4 (given in
 * upwind order, m0 the farthest point), over one common denominator:
 * (n+ d- + n- d+) / (d+ d-).  Two products summed, so the value does not
 * depend on which side is called "+" (mirror symmetry stays exact); one
 * division per face instead of two.  d+ d- >= (6 eps^4)^2 stays a normal
 * double for eps >= 1e-30. */
double orc_weno5_face(double p0, double p1, double p2, double p3, double p4, double m0, double m1,
                      double m2, double m3, double m4, double eps) {
  double np, dp, nm, dm;
  weno5_nd(p0, p1, p2, p3, p4, eps, &np, &dp);
  weno5_nd(m0, m1, m2, m3, m4, eps, &nm, &dm);
  return (np * dm + nm * dp) / (dp * dm);
}

/* ---------------------------------------------------------- ghost cells */

/* Padded array: [4][ny + 2 gy][nx + 2 NG], gy = NG in 2D, 0 in 1D. */
typedef struct {
  int nx, ny, gy, px, py;
  double *a;
} padded_t;

static double *pad_at(padded_t *P, int c, int j, int i) { /* j, i interior indices */
  return &P->a[((size_t)c * P->py + (size_t)(j + P->gy)) * P->px + (size_t)(i + NG)];
}

/* Source index and sign of the momentum normal to the boundary for a ghost
 * at index g outside [0, n) (g in [-NG, -1] or [n, n+NG-1]). */
static int ghost_src(int g, int n, int bc_lo, int bc_hi, double *flip) {
  *flip = 1.0;
  if (g < 0) {
    if (bc_lo == ORC_PERIODIC) return g + n;
    if (bc_lo == ORC_TRANSMISSIVE) return 0;
    *flip = -1.0;
    return -g - 1; /* mirror about the face at index 0 */
  }
  if (bc_hi == ORC_PERIODIC) return g - n;
  if (bc_hi == ORC_TRANSMISSIVE) return n - 1;
  *flip = -1.0;
  return 2 * n - 1 - g; /* mirror about the face at index n */
}

static void fill_padded(const orc_params *p, const double *V, padded_t *P) {
  const int nx = p->nx, ny = p->ny;
  const long total = (long)4 * P->py * P->px;
#pragma omp parallel for schedule(static)
  for (long k = 0; k < total; ++k) P->a[k] = NAN; /* corners stay NaN: never read */
#pragma omp parallel for collapse(2) schedule(static)
  for (int c = 0; c < 4; ++c)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i)
        *pad_at(P, c, j, i) = V[((size_t)c * ny + j) * nx + i];
  /* x ghosts, interior rows */
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny; ++j)
    for (int g = -NG; g < nx + NG; ++g) {
      if (g >= 0 && g < nx) continue;
      double flip;
      int s = ghost_src(g, nx, p->bc[0], p->bc[1], &flip);
      for (int c = 0; c < 4; ++c) {
        double val = *pad_at(P, c, j, s);
        *pad_at(P, c, j, g) = (c == 1) ? flip * val : val;
      }
    }
  /* y ghosts, interior columns */
  if (P->gy > 0)
    for (int g = -NG; g < ny + NG; ++g) {
      if (g >= 0 && g < ny) continue;
      double flip;
      int s = ghost_src(g, ny, p->bc[2], p->bc[3], &flip);
      for (int i = 0; i < nx; ++i)
        for (int c = 0; c < 4; ++c) {
          double val = *pad_at(P, c, s, i);
          *pad_at(P, c, g, i) = (c == 2) ? flip * val : val;
        }
    }
}

/* ------------------------------------------------------------ reductions */

/* alpha_x = max |u| + c, alpha_y = max |v| + c, s_max = max c + |u| + |v|
 * over interior cells.  Returns ORC_E_UNPHYSICAL if rho <= 0 or p <= 0
 * (or a non-finite value) anywhere. */
int orc_alpha(const orc_params *p, const double *V, double out[3]) {
  int rc = check_params(p);
  if (rc) return rc;
  const long n = (long)p->nx * p->ny;
  double ax = 0.0, ay = 0.0, sm = 0.0;
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(max : ax, ay, sm) reduction(| : bad)
  for (long k = 0; k < n; ++k) {
    double r = V[k], mx = V[n + k], my = V[2 * n + k], E = V[3 * n + k];
    prim_t w = cons_to_prim(r, mx, my, E, p->gamma);
    if (!(r > 0.0) || !(w.p > 0.0) || !isfinite(w.c)) bad = 1;
    double a = fabs(w.u) + w.c;
    double b = fabs(w.v) + w.c;
    double s = w.c + (fabs(w.u) + fabs(w.v));
    if (a > ax) ax = a;
    if (b > ay) ay = b;
    if (s > sm) sm = s;
  }
  out[0] = ax;
  out[1] = ay;
  out[2] = sm;
  return bad ? ORC_E_UNPHYSICAL : ORC_OK;
}

/* CFL step of Sect. 5.3: dt = c_cfl * Delta / max(c + |u| + |v|),
 * Delta = min(dx, dy) (dx alone in the 1D limit). */
static double cfl_dt(const orc_params *p, double smax) {
  double dx = cell_dx(p);
  double dmin = dx;
  if (p->ny > 1) {
    double dy = cell_dy(p);
    if (dy < dmin) dmin = dy;
  }
  return (p->cfl * dmin) / smax;
}

int orc_cfl(const orc_params *p, const double *U, double *dt) {
  double a[3];
  int rc = orc_alpha(p, U, a);
  if (rc) return rc;
  *dt = cfl_dt(p, a[2]);
  return ORC_OK;
}

/* -------------------------------------------------------- right-hand side */

/* Flux-split values f+ and f- of one direction at every point of a padded
 * row (dir 0) or column (dir 1):  f+- = (F(U) +- alpha U) / 2. */
static void split_flux(const double U[4], double gamma, double alpha, int dir,
                       double fp[4], double fm[4]) {
  double r = U[0], mx = U[1], my = U[2], E = U[3];
  prim_t w = cons_to_prim(r, mx, my, E, gamma);
  double F[4];
  if (dir == 0) {
    F[0] = mx;
    F[1] = fma(mx, w.u, w.p);
    F[2] = my * w.u;
    F[3] = (E + w.p) * w.u;
  } else {
    F[0] = my;
    F[1] = mx * w.v;
    F[2] = fma(my, w.v, w.p);
    F[3] = (E + w.p) * w.v;
  }
  for (int c = 0; c < 4; ++c) {
    fp[c] = 0.5 * fma(alpha, U[c], F[c]);
    fm[c] = 0.5 * fma(-alpha, U[c], F[c]);
  }
}

/* Eigenvectors of the flux Jacobian in direction dir at the Roe average of
 * the states Ul, Ur (conserved, (rho, m_x, m_y, E)), in the rotated frame
 * (rho, m_n, m_t, E) with n the direction of the sweep and t the other one:
 * right eigenvectors (columns) for the speeds u_n - c, u_n, u_n, u_n + c
 *   R = [1, 1, 0, 1; u_n - c, u_n, 0, u_n + c; u_t, u_t, 1, u_t;
 *        H - u_n c, q2/2, u_t, H + u_n c],
 * and their inverse L (rows), b1 = (gamma - 1)/c^2, b2 = b1 q2/2:
 *   L = [(b2 + u_n/c)/2, (-b1 u_n - 1/c)/2, -b1 u_t/2, b1/2;
 *        1 - b2, b1 u_n, b1 u_t, -b1;  -u_t, 0, 1, 0;
 *        (b2 - u_n/c)/2, (1/c - b1 u_n)/2, -b1 u_t/2, b1/2].
 * Roe average: weights sqrt(rho); u_n, u_t and the total enthalpy
 * H = (E + p)/rho averaged, c^2 = (gamma - 1)(H - q2/2), q2 = u_n^2 + u_t^2.
 * Returns ORC_E_UNPHYSICAL when c^2 <= 0. */
int orc_char_eig(const double Ul[4], const double Ur[4], int dir, double gamma, double Lm[16],
                 double Rm[16]) {
  prim_t wl = cons_to_prim(Ul[0], Ul[1], Ul[2], Ul[3], gamma);
  prim_t wr = cons_to_prim(Ur[0], Ur[1], Ur[2], Ur[3], gamma);
  const double nl = dir == 0 ? wl.u : wl.v, tl = dir == 0 ? wl.v : wl.u;
  const double nr = dir == 0 ? wr.u : wr.v, tr = dir == 0 ? wr.v : wr.u;
  const double Hl = (Ul[3] + wl.p) / Ul[0], Hr = (Ur[3] + wr.p) / Ur[0];
  const double sl = sqrt(Ul[0]), sr = sqrt(Ur[0]);
  const double den = sl + sr;
  const double un = (sl * nl + sr * nr) / den;
  const double ut = (sl * tl + sr * tr) / den;
  const double H = (sl * Hl + sr * Hr) / den;
  const double q2 = un * un + ut * ut;
  const double c2 = (gamma - 1.0) * (H - 0.5 * q2);
  if (!(c2 > 0.0) || !isfinite(c2)) return ORC_E_UNPHYSICAL;
  const double c = sqrt(c2), ic = 1.0 / c;
  const double b1 = (gamma - 1.0) / c2, b2 = (0.5 * q2) * b1;
  const double L[16] = {0.5 * (b2 + un * ic), 0.5 * (-(b1 * un) - ic), -0.5 * (b1 * ut), 0.5 * b1,
                        1.0 - b2, b1 * un, b1 * ut, -b1,
                        -ut, 0.0, 1.0, 0.0,
                        0.5 * (b2 - un * ic), 0.5 * (ic - b1 * un), -0.5 * (b1 * ut), 0.5 * b1};
  const double R[16] = {1.0, 1.0, 0.0, 1.0,
                        un - c, un, 0.0, un + c,
                        ut, ut, 1.0, ut,
                        H - un * c, 0.5 * q2, ut, H + un * c};
  memcpy(Lm, L, sizeof(L));
  memcpy(Rm, R, sizeof(R));
  return ORC_OK;
}

/* Four-term dot product in a fixed order: ((a0 b0 + a1 b1) + a2 b2) + a3 b3,
 * each step one fma. */
static double dot4(const double *a, const double b[4]) {
  return fma(a[3], b[3], fma(a[2], b[2], fma(a[1], b[1], a[0] * b[0])));
}

/* Characteristic-wise face value between padded points i and i+1 of a line:
 * fp, fm hold the split fluxes of the line ([k][4], original component
 * order), Ul, Ur the states at i and i+1.  Each field m: the projections
 * l_m . f+ at i-2..i+2 reconstructed left-biased plus l_m . f- at i+3..i-1
 * right-biased; the face flux is R times those four values, rotated back. */
static int char_face(const double *fp, const double *fm, int i, const double Ul[4],
                     const double Ur[4], int dir, double gamma, double eps, double out[4]) {
  double L[16], R[16];
  int rc = orc_char_eig(Ul, Ur, dir, gamma, L, R);
  if (rc) return rc;
  const int cn = dir == 0 ? 1 : 2, ct = dir == 0 ? 2 : 1;
  double gp[6][4], gm[6][4]; /* rotated split fluxes at i-2 .. i+3 */
  for (int k = 0; k < 6; ++k) {
    const int q = i - 2 + k;
    gp[k][0] = fp[4 * q]; gp[k][1] = fp[4 * q + cn]; gp[k][2] = fp[4 * q + ct]; gp[k][3] = fp[4 * q + 3];
    gm[k][0] = fm[4 * q]; gm[k][1] = fm[4 * q + cn]; gm[k][2] = fm[4 * q + ct]; gm[k][3] = fm[4 * q + 3];
  }
  double gh[4];
  for (int m = 0; m < 4; ++m) {
    const double *l = &L[4 * m];
    gh[m] = orc_weno5_face(dot4(l, gp[0]), dot4(l, gp[1]), dot4(l, gp[2]), dot4(l, gp[3]), dot4(l, gp[4]),
                           dot4(l, gm[5]), dot4(l, gm[4]), dot4(l, gm[3]), dot4(l, gm[2]), dot4(l, gm[1]),
                           eps);
  }
  double rot[4];
  for (int c = 0; c < 4; ++c) rot[c] = dot4(&R[4 * c], gh);
  out[0] = rot[0];
  out[cn] = rot[1];
  out[ct] = rot[2];
  out[3] = rot[3];
  return ORC_OK;
}

/* L(V) on the interior for given LF speeds (ax, ay).  gravity: NULL or
 * [2][ny][nx] (g_x, g_y) per cell.  L: [4][ny][nx]. */
int orc_rhs(const orc_params *p, const double *gravity, const double *V,
            double ax, double ay, double *L) {
  int rc = check_params(p);
  if (rc) return rc;
  const int nx = p->nx, ny = p->ny;
  const size_t n = (size_t)nx * ny;
  const double dx = cell_dx(p), dy = cell_dy(p);
  const double idx = 1.0 / dx, idy = 1.0 / dy;
  const double eps = p->eps;

  padded_t P;
  P.nx = nx;
  P.ny = ny;
  P.gy = (ny > 1) ? NG : 0;
  P.px = nx + 2 * NG;
  P.py = ny + 2 * P.gy;
  P.a = (double *)malloc(sizeof(double) * 4 * (size_t)P.px * P.py);
  double *Dx = (double *)calloc(4 * n, sizeof(double));
  double *Dy = (double *)calloc(4 * n, sizeof(double));
  if (!P.a || !Dx || !Dy) {
    free(P.a); free(Dx); free(Dy);
    return ORC_E_NOMEM;
  }
  fill_padded(p, V, &P);
  int status = ORC_OK, nomem = 0;
  const int len = (nx > ny ? nx : ny) + 2 * NG;

#pragma omp parallel reduction(min : status) reduction(| : nomem)
  {
    /* line buffers of this thread: split fluxes of one row or column and its face values */
    double *fp = (double *)malloc(sizeof(double) * 4 * len);
    double *fm = (double *)malloc(sizeof(double) * 4 * len);
    double *Fh = (double *)malloc(sizeof(double) * 4 * (len + 1));
    const int have = fp && fm && Fh;
    if (!have) nomem = 1;

    /* x sweep, one interior row at a time.  Padded point k <-> cell k - NG.
     * Face f (0..nx) sits between cells f-1 and f. */
#pragma omp for schedule(static)
    for (int j = 0; j < ny; ++j) {
      if (!have) continue;
      for (int k = 0; k < nx + 2 * NG; ++k) {
        double U[4], a[4], b[4];
        for (int c = 0; c < 4; ++c) U[c] = *pad_at(&P, c, j, k - NG);
        split_flux(U, p->gamma, ax, 0, a, b);
        for (int c = 0; c < 4; ++c) { fp[4 * k + c] = a[c]; fm[4 * k + c] = b[c]; }
      }
      for (int f = 0; f <= nx; ++f) {
        int i = f - 1 + NG; /* padded index of the cell left of the face */
        if (p->recon == 1) {
          double Ul[4], Ur[4];
          for (int c = 0; c < 4; ++c) {
            Ul[c] = *pad_at(&P, c, j, i - NG);
            Ur[c] = *pad_at(&P, c, j, i + 1 - NG);
          }
          if (char_face(fp, fm, i, Ul, Ur, 0, p->gamma, eps, &Fh[4 * f])) status = ORC_E_UNPHYSICAL;
          continue;
        }
        for (int c = 0; c < 4; ++c) {
          Fh[4 * f + c] = orc_weno5_face(fp[4 * (i - 2) + c], fp[4 * (i - 1) + c], fp[4 * i + c],
                                         fp[4 * (i + 1) + c], fp[4 * (i + 2) + c],
                                         fm[4 * (i + 3) + c], fm[4 * (i + 2) + c], fm[4 * (i + 1) + c],
                                         fm[4 * i + c], fm[4 * (i - 1) + c], eps);
        }
      }
      for (int i = 0; i < nx; ++i)
        for (int c = 0; c < 4; ++c)
          Dx[((size_t)c * ny + j) * nx + i] = (Fh[4 * (i + 1) + c] - Fh[4 * i + c]) * idx;
    }

    /* y sweep, one interior column at a time (skipped in the 1D limit). */
    if (ny > 1) {
#pragma omp for schedule(static)
      for (int i = 0; i < nx; ++i) {
        if (!have) continue;
        for (int k = 0; k < ny + 2 * NG; ++k) {
          double U[4], a[4], b[4];
          for (int c = 0; c < 4; ++c) U[c] = *pad_at(&P, c, k - NG, i);
          split_flux(U, p->gamma, ay, 1, a, b);
          for (int c = 0; c < 4; ++c) { fp[4 * k + c] = a[c]; fm[4 * k + c] = b[c]; }
        }
        for (int f = 0; f <= ny; ++f) {
          int jj = f - 1 + NG;
          if (p->recon == 1) {
            double Ul[4], Ur[4];
            for (int c = 0; c < 4; ++c) {
              Ul[c] = *pad_at(&P, c, jj - NG, i);
              Ur[c] = *pad_at(&P, c, jj + 1 - NG, i);
            }
            if (char_face(fp, fm, jj, Ul, Ur, 1, p->gamma, eps, &Fh[4 * f])) status = ORC_E_UNPHYSICAL;
            continue;
          }
          for (int c = 0; c < 4; ++c) {
            Fh[4 * f + c] = orc_weno5_face(fp[4 * (jj - 2) + c], fp[4 * (jj - 1) + c], fp[4 * jj + c],
                                           fp[4 * (jj + 1) + c], fp[4 * (jj + 2) + c],
                                           fm[4 * (jj + 3) + c], fm[4 * (jj + 2) + c], fm[4 * (jj + 1) + c],
                                           fm[4 * jj + c], fm[4 * (jj - 1) + c], eps);
          }
        }
        for (int j = 0; j < ny; ++j)
          for (int c = 0; c < 4; ++c)
            Dy[((size_t)c * ny + j) * nx + i] = (Fh[4 * (j + 1) + c] - Fh[4 * j + c]) * idy;
      }
    }
    free(fp); free(fm); free(Fh);
  }
  if (nomem) {
    free(P.a); free(Dx); free(Dy);
    return ORC_E_NOMEM;
  }

  /* Sources of Eq. euler2D and L = S - (Dx + Dy). */
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      size_t k = (size_t)j * nx + i;
      double r = V[k], mx = V[n + k], my = V[2 * n + k], E = V[3 * n + k];
      double gxv = gravity ? gravity[k] : p->gx;
      double gyv = gravity ? gravity[n + k] : p->gy;
      double S[4];
      S[0] = 0.0;                      /* (no mass source) */
      S[1] = r * gxv;                  /* -rho dPhi/dr */
      S[2] = r * gyv;                  /* -rho dPhi/dz */
      S[3] = mx * gxv + my * gyv;      /* -rho v.grad Phi */
      if (p->geometry == 1) {
        /* -(1/r)(rho v_r, rho v_r^2, rho v_r v_z, (tau + p) v_r) */
        prim_t w = cons_to_prim(r, mx, my, E, p->gamma);
        double ri = p->xlo + ((double)i + 0.5) * dx;
        double ir = 1.0 / ri;
        S[0] = S[0] - ir * mx;
        S[1] = S[1] - ir * (mx * w.u);
        S[2] = S[2] - ir * (my * w.u);
        S[3] = S[3] - ir * ((E + w.p) * w.u);
      }
      for (int c = 0; c < 4; ++c) {
        size_t q = (size_t)c * n + k;
        L[q] = (ny > 1) ? S[c] - (Dx[q] + Dy[q]) : S[c] - Dx[q];
      }
    }

  free(P.a); free(Dx); free(Dy);
  return status;
}

/* --------------------------------------------------------------- stepping */

/* One SSP-RK3 step in place: U1 = U + dt L(U);
 * U2 = 3/4 U + 1/4 (U1 + dt L(U1));  U^{n+1} = 1/3 U + 2/3 (U2 + dt L(U2)).
 * Each stage, with input V and weight b = 1, 1/4, 2/3, is evaluated in the
 * algebraically identical increment form U + b ((V - U) + dt L(V)), i.e.
 * fma(b, fma(dt, L, V - U), U): a steady state (L = 0, V = U) is then
 * reproduced bit for bit, which the convex form with the inexact 1/3, 2/3
 * would not do.
 * alpha_in: NULL (computed from each stage's input) or [3][2] (ax, ay) per
 * stage.  alpha_out: NULL or [3][2], the speeds used. */
int orc_step(const orc_params *p, const double *gravity, double *U, double dt,
             const double *alpha_in, double *alpha_out) {
  int rc = check_params(p);
  if (rc) return rc;
  const size_t n4 = (size_t)4 * p->nx * p->ny;
  const size_t n = (size_t)p->nx * p->ny;
  const double cb[3] = {1.0, 0.25, 2.0 / 3.0};
  double *V = (double *)malloc(sizeof(double) * n4);
  double *W = (double *)malloc(sizeof(double) * n4);
  double *L = (double *)malloc(sizeof(double) * n4);
  if (!V || !W || !L) { free(V); free(W); free(L); return ORC_E_NOMEM; }
  memcpy(V, U, sizeof(double) * n4);
  int status = ORC_OK;
  for (int s = 0; s < 3 && status == ORC_OK; ++s) {
    double ax, ay;
    if (alpha_in) {
      ax = alpha_in[2 * s];
      ay = alpha_in[2 * s + 1];
    } else {
      double a[3];
      rc = orc_alpha(p, V, a);
      if (rc) { status = rc; break; }
      ax = a[0];
      ay = a[1];
    }
    if (alpha_out) { alpha_out[2 * s] = ax; alpha_out[2 * s + 1] = ay; }
    rc = orc_rhs(p, gravity, V, ax, ay, L);
    if (rc) { status = rc; break; }
#pragma omp parallel for schedule(static)
    for (long q = 0; q < (long)n4; ++q) W[q] = fma(cb[s], fma(dt, L[q], V[q] - U[q]), U[q]);
    if (p->rho_floor > 0.0) {
      /* atmosphere (Sect. 5.3 enforces a minimum density, the atmosphere's):
       * rho < rho_floor -> the atmosphere state at rest; then, for the ideal
       * gas, p < p_floor -> internal energy raised to the atmosphere's
       * pressure with rho and m kept. */
#pragma omp parallel for schedule(static)
      for (long k = 0; k < (long)n; ++k) {
        if (W[k] < p->rho_floor) {
          W[k] = p->rho_floor;
          W[n + k] = 0.0;
          W[2 * n + k] = 0.0;
          W[3 * n + k] = p->p_floor / (p->gamma - 1.0);
        }
        prim_t w = cons_to_prim(W[k], W[n + k], W[2 * n + k], W[3 * n + k], p->gamma);
        if (w.p < p->p_floor)
          W[3 * n + k] = p->p_floor / (p->gamma - 1.0) + 0.5 * (W[n + k] * w.u + W[2 * n + k] * w.v);
      }
    }
    int unphys = 0;
#pragma omp parallel for schedule(static) reduction(| : unphys)
    for (long k = 0; k < (long)n; ++k) {
      prim_t w = cons_to_prim(W[k], W[n + k], W[2 * n + k], W[3 * n + k], p->gamma);
      if (!(W[k] > 0.0) || !(w.p > 0.0) || !isfinite(w.c)) unphys = 1;
    }
    if (unphys) status = ORC_E_UNPHYSICAL;
    double *t = V; V = W; W = t;
  }
  if (status == ORC_OK) memcpy(U, V, sizeof(double) * n4);
  free(V); free(W); free(L);
  return status;
}

/* Advance up to nsteps steps with the CFL time step, each clamped so that
 * t never passes t_end (t_end <= 0: no clamp).  Stops early when t reaches
 * t_end.  dt_rec: NULL or [nsteps]; alpha_rec: NULL or [nsteps][3][2].
 * Returns the number of steps taken (>= 0) or an error code (< 0). */
int orc_run(const orc_params *p, const double *gravity, double *U, int nsteps,
            double t_end, double *t_io, double *dt_rec, double *alpha_rec) {
  int rc = check_params(p);
  if (rc) return rc;
  double t = t_io ? *t_io : 0.0;
  int k = 0;
  for (; k < nsteps; ++k) {
    if (t_end > 0.0 && !(t < t_end)) break;
    double a[3];
    rc = orc_alpha(p, U, a);
    if (rc) return rc;
    double dt = cfl_dt(p, a[2]);
    if (t_end > 0.0 && t + dt > t_end) dt = t_end - t;
    rc = orc_step(p, gravity, U, dt, NULL, alpha_rec ? alpha_rec + 6 * (size_t)k : NULL);
    if (rc) return rc;
    if (dt_rec) dt_rec[k] = dt;
    t = t + dt;
    if (t_io) *t_io = t;
  }
  return k;
}

/* Totals of rho, m_x, m_y, E over the grid (times the cell volume: dx dy in
 * Cartesian, 2 pi r_i dx dy in cylindrical), summed in row-major order with
 * Neumaier's compensated summation. */
int orc_sums(const orc_params *p, const double *U, double out[4]) {
  int rc = check_params(p);
  if (rc) return rc;
  const int nx = p->nx, ny = p->ny;
  const size_t n = (size_t)nx * ny;
  const double dx = cell_dx(p), dy = cell_dy(p);
  const double two_pi = 6.283185307179586;
  for (int c = 0; c < 4; ++c) {
    double s = 0.0, comp = 0.0;
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        double vol = dx * dy;
        if (p->geometry == 1) vol = (two_pi * (p->xlo + ((double)i + 0.5) * dx)) * vol;
        double term = U[(size_t)c * n + (size_t)j * nx + i] * vol;
        double t = s + term;
        if (fabs(s) >= fabs(term)) comp += (s - t) + term;
        else comp += (term - t) + s;
        s = t;
      }
    out[c] = s + comp;
  }
  return ORC_OK;
}

/* Number of threads the parallel loops use (n >= 1); returns the number in
 * effect (1 without OpenMP). */
int orc_set_threads(int nthreads) {
#ifdef _OPENMP
  if (nthreads >= 1) omp_set_num_threads(nthreads);
  return omp_get_max_threads();
#else
  (void)nthreads;
  return 1;
#endif
}

/* Size of the parameter struct, so the binding can check its mirror. */
int orc_params_size(void) { return (int)sizeof(orc_params); }
