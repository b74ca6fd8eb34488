/*
 * levelset_oracle.c -- FP64 CPU oracle of the level-set flame tracker
 * (TEST INFRASTRUCTURE; same rules as hydro_oracle.c: loaded only by the
 * tests, the smoke entry point and the benchmark's baseline leg, no code
 * shared with the HIP library).
 *
 * Sect. 2.3 (level-set method): a scalar S on the grid corners whose zero
 * contour is the flame front (S > 0 ash, S < 0 fuel) is
 *   (1) advected by dS/dt = -(v + v_flame) . grad S, with v_flame of magnitude
 *       s_f along the outward normal of the burnt region, -grad S / |grad S|,
 *       so that dS/dt = -(u S_x + v S_y) + s_f |grad S|; the paper advects S
 *       with the same WENO scheme as the fluid;
 *   (2) re-distanced after each update: the front points are where neighbouring
 *       corners have values of opposite sign, placed by linear interpolation;
 *       every corner takes the smallest distance d to them, and the new value
 *       is H(d) S_old + (1 - H(d)) d with
 *       H(d) = (1 - tanh((d - d0) / (D/3))) / (1 - tanh(-d0 / (D/3))), d0 = 3 D,
 *       D the grid spacing.
 *
 * Readings (the paper gives no discretisation of (1), and (2) in words):
 *  - corners (i, j), i = 0..nx, j = 0..ny, at (xlo + i dx, ylo + j dy); S and the
 *    corner velocity (u, v) are arrays [ny+1][nx+1];
 *  - (1) is a Hamilton-Jacobi equation S_t + H(S_x, S_y) = 0 with
 *    H(p, q) = u p + v q - s_f sqrt(p^2 + q^2); the WENO scheme for it is the
 *    Hamilton-Jacobi form of WENO5-JS: one-sided derivatives S_x^-/S_x^+ are the
 *    left-/right-biased fifth-order reconstructions (the same weights, epsilon
 *    and evaluation order as the flux reconstruction of the fluid) of the
 *    differences q_m = (S_m - S_{m-1}) (1/dx) (times the reciprocal of the
 *    spacing, formed once), combined by a
 *    global Lax-Friedrichs flux
 *      Hhat = H((p- + p+)/2, (q- + q+)/2) - ax (p+ - p-)/2 - ay (q+ - q-)/2,
 *    ax = max|u| + s_f, ay = max|v| + s_f over all corners; SSP-RK3 in the
 *    increment form of the fluid's step, with a given dt;
 *  - ghost corners (3 per side): periodic (corner nx is corner 0's image, so the
 *    grid is nx x ny distinct corners and corner nx/ny is overwritten by its
 *    image before the step and after each stage), reflecting (S_{-k} = S_k about the wall corner),
 *    transmissive (linear extrapolation S_{-k} = 2 S_0 - S_k, which keeps a
 *    distance function's slope);
 *  - (2): front points on corner-to-corner edges (horizontal and vertical) with
 *    S_a S_b < 0, at a + (b - a) S_a / (S_a - S_b), and at corners with S = 0;
 *    d is the Euclidean distance to the nearest one; the new value keeps the old
 *    sign: S_new = H(d) S_old + (1 - H(d)) sign(S_old) d; D = min(dx, dy); with
 *    no front point S is left unchanged.
 * Every formula has a fixed evaluation order (built with -ffp-contract=off).
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { LS_PERIODIC = 0, LS_TRANSMISSIVE = 1, LS_REFLECTING = 2 };

typedef struct {
  int32_t nx, ny;          /* cells; corners are (nx+1) x (ny+1) */
  double xlo, xhi, ylo, yhi;
  int32_t bc[4];           /* x-low, x-high, y-low, y-high */
  double eps;              /* WENO epsilon */
} orc_ls_params;

/* WENO5-JS reconstruction at the right face of v2 from v0..v4 (left-biased):
 * the fluid oracle's routine, so both uses share one evaluation order. */
double orc_weno5(double v0, double v1, double v2, double v3, double v4, double eps);

/* Ghost-padded copy: pad[(ny+1+6)][(nx+1+6)], interior corner (i, j) at
 * (i+3, j+3). */
static void pad_corners(const orc_ls_params *q, const double *S, double *pad) {
  const int mx = q->nx + 1, my = q->ny + 1, px = mx + 6;
  for (int j = 0; j < my; ++j)
    for (int i = 0; i < mx; ++i) pad[(size_t)(j + 3) * px + i + 3] = S[(size_t)j * mx + i];
  /* x ghosts, rows 3..my+2 */
  for (int j = 3; j < my + 3; ++j) {
    double *row = pad + (size_t)j * px;
    for (int k = 1; k <= 3; ++k) {
      const int lo = 3 - k, hi = mx + 2 + k; /* ghost positions */
      switch (q->bc[0]) {
        case LS_PERIODIC: row[lo] = row[3 + q->nx - k]; break;
        case LS_REFLECTING: row[lo] = row[3 + k]; break;
        default: row[lo] = 2.0 * row[3] - row[3 + k]; break;
      }
      switch (q->bc[1]) {
        case LS_PERIODIC: row[hi] = row[3 + k]; break;
        case LS_REFLECTING: row[hi] = row[mx + 2 - k]; break;
        default: row[hi] = 2.0 * row[mx + 2] - row[mx + 2 - k]; break;
      }
    }
  }
  /* y ghosts, all columns */
  for (int i = 0; i < px; ++i) {
    for (int k = 1; k <= 3; ++k) {
      double *lo = pad + (size_t)(3 - k) * px + i, *hi = pad + (size_t)(my + 2 + k) * px + i;
      const double c0 = pad[(size_t)3 * px + i], cn = pad[(size_t)(my + 2) * px + i];
      switch (q->bc[2]) {
        case LS_PERIODIC: *lo = pad[(size_t)(3 + q->ny - k) * px + i]; break;
        case LS_REFLECTING: *lo = pad[(size_t)(3 + k) * px + i]; break;
        default: *lo = 2.0 * c0 - pad[(size_t)(3 + k) * px + i]; break;
      }
      switch (q->bc[3]) {
        case LS_PERIODIC: *hi = pad[(size_t)(3 + k) * px + i]; break;
        case LS_REFLECTING: *hi = pad[(size_t)(my + 2 - k) * px + i]; break;
        default: *hi = 2.0 * cn - pad[(size_t)(my + 2 - k) * px + i]; break;
      }
    }
  }
}

/* One-sided WENO derivatives along a line of the padded array: c points at the
 * corner, s is the stride to the next corner, h the spacing. */
static void one_sided(const double *c, ptrdiff_t s, double h, double eps, double *dm, double *dp) {
  const double ih = 1.0 / h;
  double qv[6]; /* q_{m} = (S_m - S_{m-1}) * (1/h) for m = i-2 .. i+3 */
  for (int k = 0; k < 6; ++k) {
    const ptrdiff_t m = (ptrdiff_t)(k - 2);
    qv[k] = (c[m * s] - c[(m - 1) * s]) * ih;
  }
  *dm = orc_weno5(qv[0], qv[1], qv[2], qv[3], qv[4], eps);
  *dp = orc_weno5(qv[5], qv[4], qv[3], qv[2], qv[1], eps);
}

/* Global LF speeds (max|u| + s_f, max|v| + s_f) over all corners. */
void orc_ls_alpha(const orc_ls_params *q, const double *vel, double s_f, double out[2]) {
  const size_t n = (size_t)(q->nx + 1) * (size_t)(q->ny + 1);
  double mu = 0.0, mv = 0.0;
  for (size_t k = 0; k < n; ++k) {
    const double au = fabs(vel[k]), av = fabs(vel[n + k]);
    if (au > mu) mu = au;
    if (av > mv) mv = av;
  }
  out[0] = mu + s_f;
  out[1] = mv + s_f;
}

/* L = -Hhat at every corner.  vel: [2][ny+1][nx+1] (u, v). */
void orc_ls_rhs(const orc_ls_params *q, const double *S, const double *vel, double s_f, double ax,
                double ay, double *L) {
  const int mx = q->nx + 1, my = q->ny + 1, px = mx + 6;
  const double dx = (q->xhi - q->xlo) / (double)q->nx, dy = (q->yhi - q->ylo) / (double)q->ny;
  const size_t n = (size_t)mx * (size_t)my;
  double *pad = malloc(sizeof(double) * (size_t)px * (size_t)(my + 6));
  pad_corners(q, S, pad);
  for (int j = 0; j < my; ++j)
    for (int i = 0; i < mx; ++i) {
      const double *c = pad + (size_t)(j + 3) * px + i + 3;
      double pm, pp, qm, qp;
      one_sided(c, 1, dx, q->eps, &pm, &pp);
      one_sided(c, (ptrdiff_t)px, dy, q->eps, &qm, &qp);
      const double p = 0.5 * (pm + pp), qq = 0.5 * (qm + qp);
      const double u = vel[(size_t)j * mx + i], v = vel[n + (size_t)j * mx + i];
      const double grad = sqrt(p * p + qq * qq);
      const double H = (u * p + v * qq) - s_f * grad;
      const double Hhat = (H - ax * (0.5 * (pp - pm))) - ay * (0.5 * (qp - qm));
      L[(size_t)j * mx + i] = -Hhat;
    }
  free(pad);
}

/* Periodic images: corner nx equals corner 0, corner ny equals corner 0. */
static void periodic_images(const orc_ls_params *q, double *S) {
  const int mx = q->nx + 1, my = q->ny + 1;
  if (q->bc[0] == LS_PERIODIC)
    for (int j = 0; j < my; ++j) S[(size_t)j * mx + q->nx] = S[(size_t)j * mx];
  if (q->bc[2] == LS_PERIODIC)
    for (int i = 0; i < mx; ++i) S[(size_t)q->ny * mx + i] = S[i];
}

/* One SSP-RK3 step of the advection in place with time step dt; the LF speeds
 * are computed once from the corner velocity (it is frozen over the step).
 * Stage form: W = U0 + b ((V - U0) + dt L(V)), b = 1, 1/4, 2/3. */
void orc_ls_step(const orc_ls_params *q, double *S, const double *vel, double s_f, double dt) {
  const size_t n = (size_t)(q->nx + 1) * (size_t)(q->ny + 1);
  double a[2];
  orc_ls_alpha(q, vel, s_f, a);
  double *S0 = malloc(sizeof(double) * n), *V = malloc(sizeof(double) * n),
         *L = malloc(sizeof(double) * n);
  periodic_images(q, S); /* corner nx (ny) is corner 0's image from the start */
  memcpy(S0, S, sizeof(double) * n);
  memcpy(V, S, sizeof(double) * n);
  const double b[3] = {1.0, 0.25, 2.0 / 3.0};
  for (int st = 0; st < 3; ++st) {
    orc_ls_rhs(q, V, vel, s_f, a[0], a[1], L);
    for (size_t k = 0; k < n; ++k) {
      const double inc = (V[k] - S0[k]) + dt * L[k];
      V[k] = S0[k] + b[st] * inc;
    }
    periodic_images(q, V);
  }
  memcpy(S, V, sizeof(double) * n);
  free(S0);
  free(V);
  free(L);
}

/* Front points: (x, y) pairs into pts (capacity cap points).  Returns their
 * number (all of them are counted even beyond cap). Order: corners with S = 0,
 * then horizontal edges, then vertical edges, each in row-major order. */
long orc_ls_front(const orc_ls_params *q, const double *S, double *pts, long cap) {
  const int mx = q->nx + 1, my = q->ny + 1;
  const double dx = (q->xhi - q->xlo) / (double)q->nx, dy = (q->yhi - q->ylo) / (double)q->ny;
  long n = 0;
#define PUSH(X, Y)              \
  do {                          \
    if (n < cap) {              \
      pts[2 * n] = (X);         \
      pts[2 * n + 1] = (Y);     \
    }                           \
    ++n;                        \
  } while (0)
  for (int j = 0; j < my; ++j)
    for (int i = 0; i < mx; ++i)
      if (S[(size_t)j * mx + i] == 0.0) PUSH(q->xlo + (double)i * dx, q->ylo + (double)j * dy);
  for (int j = 0; j < my; ++j)
    for (int i = 0; i + 1 < mx; ++i) {
      const double a = S[(size_t)j * mx + i], b = S[(size_t)j * mx + i + 1];
      if ((a < 0.0 && b > 0.0) || (a > 0.0 && b < 0.0)) {
        const double x0 = q->xlo + (double)i * dx;
        PUSH(x0 + dx * (a / (a - b)), q->ylo + (double)j * dy);
      }
    }
  for (int j = 0; j + 1 < my; ++j)
    for (int i = 0; i < mx; ++i) {
      const double a = S[(size_t)j * mx + i], b = S[(size_t)(j + 1) * mx + i];
      if ((a < 0.0 && b > 0.0) || (a > 0.0 && b < 0.0)) {
        const double y0 = q->ylo + (double)j * dy;
        PUSH(q->xlo + (double)i * dx, y0 + dy * (a / (a - b)));
      }
    }
#undef PUSH
  return n;
}

/* The blend weight H(d), d0 = 3 D, width D / 3. */
static double blend_h(double d, double D) {
  const double w = D / 3.0, d0 = 3.0 * D;
  return (1.0 - tanh((d - d0) / w)) / (1.0 - tanh(-d0 / w));
}

/* Re-distance S in place; dist (optional, [ny+1][nx+1]) receives d.  Returns the
 * number of front points (0: S unchanged, dist untouched). */
long orc_ls_redistance(const orc_ls_params *q, double *S, double *dist) {
  const int mx = q->nx + 1, my = q->ny + 1;
  const double dx = (q->xhi - q->xlo) / (double)q->nx, dy = (q->yhi - q->ylo) / (double)q->ny;
  const double D = dx < dy ? dx : dy;
  const long cap = 3L * (long)mx * (long)my;
  double *pts = malloc(sizeof(double) * 2 * (size_t)cap);
  const long np = orc_ls_front(q, S, pts, cap);
  if (np > 0) {
    for (int j = 0; j < my; ++j)
      for (int i = 0; i < mx; ++i) {
        const double x = q->xlo + (double)i * dx, y = q->ylo + (double)j * dy;
        double best = INFINITY;
        for (long k = 0; k < np; ++k) {
          const double ex = x - pts[2 * k], ey = y - pts[2 * k + 1];
          const double r = sqrt(ex * ex + ey * ey);
          if (r < best) best = r;
        }
        const double s = S[(size_t)j * mx + i];
        const double h = blend_h(best, D);
        const double sd = s < 0.0 ? -best : best;
        S[(size_t)j * mx + i] = h * s + (1.0 - h) * sd;
        if (dist) dist[(size_t)j * mx + i] = best;
      }
  }
  free(pts);
  return np;
}

/* Corner velocity from a cell state U[4][ny][nx] (rho, m_x, m_y, E): the mean
 * of the velocities m/rho of the four cells that share the corner,
 * 0.25 ((a + b) + (c + d)) with a, b the lower-left and lower-right cell and
 * c, d the upper ones.  Beyond the grid the fluid's ghost cells stand in:
 * periodic images, copies of the edge cell (transmissive), or mirror cells
 * with the normal velocity negated (reflecting, which makes it 0 on the wall).
 * vel: [2][ny+1][nx+1]. */
static void cell_velocity(const orc_ls_params *q, const double *U, int ci, int cj, double *u, double *v) {
  const int nx = q->nx, ny = q->ny;
  double su = 1.0, sv = 1.0;
  if (ci < 0) {
    if (q->bc[0] == LS_PERIODIC) ci += nx;
    else if (q->bc[0] == LS_REFLECTING) { ci = -1 - ci; su = -1.0; }
    else ci = 0;
  } else if (ci >= nx) {
    if (q->bc[1] == LS_PERIODIC) ci -= nx;
    else if (q->bc[1] == LS_REFLECTING) { ci = 2 * nx - 1 - ci; su = -1.0; }
    else ci = nx - 1;
  }
  if (cj < 0) {
    if (q->bc[2] == LS_PERIODIC) cj += ny;
    else if (q->bc[2] == LS_REFLECTING) { cj = -1 - cj; sv = -1.0; }
    else cj = 0;
  } else if (cj >= ny) {
    if (q->bc[3] == LS_PERIODIC) cj -= ny;
    else if (q->bc[3] == LS_REFLECTING) { cj = 2 * ny - 1 - cj; sv = -1.0; }
    else cj = ny - 1;
  }
  const size_t n = (size_t)nx * (size_t)ny, k = (size_t)cj * nx + ci;
  const double rho = U[k];
  *u = su * (U[n + k] / rho);
  *v = sv * (U[2 * n + k] / rho);
}

void orc_ls_corner_velocity(const orc_ls_params *q, const double *U, double *vel) {
  const int mx = q->nx + 1, my = q->ny + 1;
  const size_t nc = (size_t)mx * (size_t)my;
  for (int j = 0; j < my; ++j)
    for (int i = 0; i < mx; ++i) {
      double ua, va, ub, vb, uc, vc, ud, vd;
      cell_velocity(q, U, i - 1, j - 1, &ua, &va);
      cell_velocity(q, U, i, j - 1, &ub, &vb);
      cell_velocity(q, U, i - 1, j, &uc, &vc);
      cell_velocity(q, U, i, j, &ud, &vd);
      vel[(size_t)j * mx + i] = 0.25 * ((ua + ub) + (uc + ud));
      vel[nc + (size_t)j * mx + i] = 0.25 * ((va + vb) + (vc + vd));
    }
}

int orc_ls_params_size(void) { return (int)sizeof(orc_ls_params); }
