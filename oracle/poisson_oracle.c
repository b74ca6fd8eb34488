/*
 * poisson_oracle.c -- FP64 CPU oracle of the gravitational potential solver
 * (TEST INFRASTRUCTURE; same rules as hydro_oracle.c: loaded only by the
 * tests, the smoke entry point and the benchmark's baseline leg, no code
 * shared with the HIP library).
 *
 * Sect. 2.1: the potential satisfies the Poisson equation
 *     (1/r) d/dr (r dPhi/dr) + d^2 Phi / dz^2 = 4 pi G rho
 * in cylindrical (r, z); it is solved by successive over-relaxation of
 * Gauss-Seidel sweeps, stopped when the relative change of every cell falls
 * below a tolerance (1e-8 in the paper); the inner boundaries (the axis r = 0
 * and the symmetry plane z = 0) are reflecting and the outer ones are fixed by
 * the Roche approximation Phi = -G M / sqrt(r^2 + z^2).
 *
 * Readings (the paper gives no discretisation):
 *  - cell-centred values on the quarter plane [0, R] x [0, Z], r_i = (i+1/2) dr,
 *    z_j = (j+1/2) dz; the r-operator in flux form with face radii
 *    r_{i-1/2} = i dr, r_{i+1/2} = (i+1) dr (the axis face has zero area, which
 *    is the reflecting condition at r = 0); at z = 0 the ghost mirrors the first
 *    row (its difference term vanishes);
 *  - outer ghost cells (i = nr or j = nz) hold the Roche value at their centres,
 *    with M the total mass of the (mirror-symmetric) configuration, an input;
 *  - sweeps in red-black order (colour (i + j) mod 2, red first), which makes
 *    the updates of one colour independent of each other;
 *  - the Gauss-Seidel value is the weighted neighbour sum minus 4 pi G rho,
 *    times the reciprocal of the diagonal weight (one reciprocal per column
 *    and row kind rather than one division per update);
 *  - relative change of a cell |Phi_new - Phi_old| / |Phi_new|, taken as 0
 *    when the value does not change (a cell that stays at 0 gives no 0/0); an
 *    iteration (red then black sweep) ends the solve when the largest one is
 *    < tol.
 * Every formula has a fixed evaluation order (built with -ffp-contract=off,
 * no fma).
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>

typedef struct {
  int32_t nr, nz;          /* cells */
  double rmax, zmax;       /* domain [0, rmax] x [0, zmax] */
  double G;                /* gravitational constant */
  double mass;             /* total mass for the Roche boundary value */
  double omega;            /* over-relaxation factor, 0 < omega < 2 */
  double tol;              /* relative-change tolerance */
  int32_t max_iter;
} orc_poisson_params;

/* Roche value -G M / sqrt(r^2 + z^2) at a ghost centre. */
static double roche(const orc_poisson_params *q, double r, double z) {
  return -(q->G * q->mass) / sqrt(r * r + z * z);
}

/* One colour sweep; returns the largest relative change of the sweep. */
static double sweep(const orc_poisson_params *q, const double *rho, double *phi, int colour) {
  const int nr = q->nr, nz = q->nz;
  const double dr = q->rmax / (double)nr, dz = q->zmax / (double)nz;
  const double idr2 = 1.0 / (dr * dr), idz2 = 1.0 / (dz * dz);
  const double four_pi_g = (4.0 * 3.141592653589793) * q->G;
  double change = 0.0;
  for (int j = 0; j < nz; ++j)
    for (int i = 0; i < nr; ++i) {
      if (((i + j) & 1) != colour) continue;
      const double r_i = ((double)i + 0.5) * dr;
      const double z_j = ((double)j + 0.5) * dz;
      const double wi = 1.0 / ((double)i + 0.5);
      const double aE = ((double)(i + 1) * wi) * idr2; /* r_{i+1/2} / (r_i dr^2) */
      const double aW = ((double)i * wi) * idr2;       /* r_{i-1/2} / (r_i dr^2) */
      const double aN = idz2;
      const double aS = j > 0 ? idz2 : 0.0;            /* mirror at z = 0 */
      const double pE = i + 1 < nr ? phi[(size_t)j * nr + i + 1] : roche(q, r_i + dr, z_j);
      const double pW = i > 0 ? phi[(size_t)j * nr + i - 1] : 0.0; /* weight 0 on the axis */
      const double pN = j + 1 < nz ? phi[(size_t)(j + 1) * nr + i] : roche(q, r_i, z_j + dz);
      const double pS = j > 0 ? phi[(size_t)(j - 1) * nr + i] : 0.0;
      const double diag = ((aE + aW) + aN) + aS;
      const double num = (((aE * pE + aW * pW) + aN * pN) + aS * pS) - four_pi_g * rho[(size_t)j * nr + i];
      const double gs = num * (1.0 / diag);
      const double old = phi[(size_t)j * nr + i];
      const double nw = old + q->omega * (gs - old);
      phi[(size_t)j * nr + i] = nw;
      const double c = nw == old ? 0.0 : fabs(nw - old) / fabs(nw);
      if (c > change) change = c;
    }
  return change;
}

/* Solve in place from the given starting potential.  Returns the number of
 * iterations done (>= 1) or -1 for invalid parameters; *last_change receives
 * the largest relative change of the last iteration. */
int orc_poisson(const orc_poisson_params *q, const double *rho, double *phi, double *last_change) {
  if (!q || q->nr < 2 || q->nz < 2 || !(q->rmax > 0.0) || !(q->zmax > 0.0) ||
      !(q->omega > 0.0 && q->omega < 2.0) || q->max_iter < 1)
    return -1;
  double ch = 0.0;
  int it = 0;
  while (it < q->max_iter) {
    double a = sweep(q, rho, phi, 0);
    double b = sweep(q, rho, phi, 1);
    ch = a > b ? a : b;
    ++it;
    if (ch < q->tol) break;
  }
  if (last_change) *last_change = ch;
  return it;
}

/* Gravitational acceleration g = -grad Phi at the cell centres, central
 * differences; the reflecting boundaries mirror Phi (zero normal gradient
 * across r = 0 and z = 0), the outer ghosts hold the Roche values.
 * g: [2][nz][nr] (g_r, g_z). */
void orc_gravity(const orc_poisson_params *q, const double *phi, double *g) {
  const int nr = q->nr, nz = q->nz;
  const double dr = q->rmax / (double)nr, dz = q->zmax / (double)nz;
  for (int j = 0; j < nz; ++j)
    for (int i = 0; i < nr; ++i) {
      const double r_i = ((double)i + 0.5) * dr;
      const double z_j = ((double)j + 0.5) * dz;
      const double pE = i + 1 < nr ? phi[(size_t)j * nr + i + 1] : roche(q, r_i + dr, z_j);
      const double pW = i > 0 ? phi[(size_t)j * nr + i - 1] : phi[(size_t)j * nr + i];
      const double pN = j + 1 < nz ? phi[(size_t)(j + 1) * nr + i] : roche(q, r_i, z_j + dz);
      const double pS = j > 0 ? phi[(size_t)(j - 1) * nr + i] : phi[(size_t)j * nr + i];
      g[(size_t)j * nr + i] = -(pE - pW) / (2.0 * dr);
      g[(size_t)nr * nz + (size_t)j * nr + i] = -(pN - pS) / (2.0 * dz);
    }
}

int orc_poisson_params_size(void) { return (int)sizeof(orc_poisson_params); }
