/*
 * hydro.h -- C ABI of the MI355X (gfx950) WENO5 Euler solver.
 *
 * The library advances the two-dimensional Euler equations in conservative
 * form with source terms (Eq. euler2D of Sect. 2.1: Cartesian (x, y) or
 * cylindrical (r, z) with the geometric terms -(1/r)(...), a fixed gravity
 * field g = -grad Phi, no heat source), using the discretisation Sect. 2.1
 * describes: finite-difference fifth-order WENO (Jiang & Shu 1996) applied to
 * both halves of a global Lax-Friedrichs flux splitting, an ideal-gas EOS
 * p = (gamma - 1) rho eps (Sect. 5.1), third-order SSP Runge-Kutta time
 * stepping and the CFL step of Sect. 5.3.
 *
 * Conventions for every entry point
 *  - Return value: HYDRO_OK (0) or a negative HYDRO_E_* code.  No call
 *    throws, aborts or prints.  hydro_strerror() names a code.
 *  - State arrays are caller-owned DEVICE buffers of 4 * ny * nx doubles,
 *    component-major [4][ny][nx] (row j = y index, i = x index, x fastest),
 *    components (rho, m_x, m_y, E): density, momentum density (m = rho v;
 *    m_r, m_z in cylindrical geometry) and total energy density
 *    E = rho eps + rho |v|^2 / 2 (the paper's tau).  Values are point values
 *    at cell centres x_i = xlo + (i + 1/2) dx, y_j = ylo + (j + 1/2) dy.
 *  - A context owns its scratch memory (stage states, reduction slots, an
 *    error flag) from hydro_create to hydro_destroy and is bound to one HIP
 *    stream.  Calls enqueue work on that stream and return without waiting
 *    unless stated ("synchronises").  A context is not thread-safe; several
 *    contexts may share a device.
 *  - Device buffers passed in must stay valid until the enqueued work has
 *    finished.  Pointers are checked for NULL only.
 *  - HYDRO_E_UNPHYSICAL is sticky: a stage that produces rho <= 0 or p <= 0
 *    (after the optional atmosphere floors) sets a device flag; the next
 *    synchronising call returns the code and hydro_check() clears it.
 *  - Magnitudes: the WENO weights of a face are summed over one common
 *    denominator, which multiplies eighth powers of the smoothness
 *    indicators, so the split fluxes (F(U) +- alpha U) / 2 must stay below
 *    about 1e17 in magnitude (FP64; about 1e9 with HYDRO_FP32_BULK).  States
 *    in units of order one, as in the paper's dimensionless tests, are far
 *    inside; beyond it the faces overflow to NaN and the step reports
 *    HYDRO_E_UNPHYSICAL.  Problems in physical units are to be scaled.
 */
#ifndef HYDRO_H
#define HYDRO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  HYDRO_OK = 0,
  HYDRO_E_INVALID = -1,    /* bad parameters, sizes or NULL pointers */
  HYDRO_E_NOMEM = -2,      /* device allocation failed */
  HYDRO_E_DEVICE = -3,     /* a HIP runtime call failed */
  HYDRO_E_UNPHYSICAL = -4, /* rho <= 0 or p <= 0 (or non-finite) was produced */
  HYDRO_E_STATE = -5       /* call not valid in the context's current state */
};

enum { HYDRO_PERIODIC = 0, HYDRO_TRANSMISSIVE = 1, HYDRO_REFLECTING = 2 };
enum { HYDRO_CARTESIAN = 0, HYDRO_CYLINDRICAL = 1 };
enum { HYDRO_FP64 = 0, HYDRO_FP32_BULK = 1 };
enum { HYDRO_COMPONENTWISE = 0, HYDRO_CHARACTERISTIC = 1 };

/* Problem description (Sect. 2.1, Eq. euler2D).
 *  nx, ny      interior cells; nx >= 3; ny == 1 is the 1D limit (no y sweep,
 *              as in the one-dimensional tests of Sect. 5.1), else ny >= 3.
 *  domain      [xlo, xhi] x [ylo, yhi]; cylindrical: x = r >= 0, y = z.
 *  geometry    HYDRO_CARTESIAN or HYDRO_CYLINDRICAL (adds -(1/r)(m_r, m_r v_r,
 *              m_z v_r, (E + p) v_r) at r_i = xlo + (i + 1/2) dx).
 *  bc[4]       x-low, x-high, y-low, y-high: periodic (both sides of an axis
 *              or neither), transmissive (zero gradient: the paper's "free"
 *              boundary) or reflecting (mirror, normal momentum negated: the
 *              r = 0 axis and z = 0 plane).  Three ghost layers.
 *  gamma       ideal-gas ratio of specific heats (> 1).
 *  cfl         Courant number c_cfl of the CFL step (Sect. 5.3).
 *  weno_eps    epsilon of the WENO weights (1e-6 is the usual choice; at least
 *              1e-30, so that the two reconstructions of a face can share one
 *              denominator without underflow; at least 1e-12 with
 *              HYDRO_FP32_BULK, whose single-precision weights reach
 *              1 / eps^2 on flat data).  HYDRO_E_INVALID otherwise.
 *  precision   HYDRO_FP64: every operation in FP64.  HYDRO_FP32_BULK: primitive
 *              variables, split fluxes, reconstructions and the divergence in
 *              FP32; stage accumulation, the CFL / LF-speed reductions and the
 *              conservation sums stay FP64; states stay FP64 in memory.
 *  gx, gy      uniform gravity, used when no gravity field is given.
 *  rho_floor   > 0 enables the atmosphere floors after every stage (Sect. 5.3:
 *  p_floor     minimum density): a cell with rho < rho_floor becomes
 *              (rho_floor, 0, 0, p_floor / (gamma - 1)); then a cell with
 *              p < p_floor gets E = p_floor / (gamma - 1) + m.v / 2 (rho and m
 *              kept).  p_floor must then be > 0.  rho_floor <= 0 disables both.
 *  reconstruction  HYDRO_COMPONENTWISE: WENO5 on each component of the split
 *              fluxes (what Sect. 2.1 describes).  HYDRO_CHARACTERISTIC: the
 *              split fluxes projected, per face, on the left eigenvectors of
 *              the flux Jacobian at the Roe average of the two cells beside
 *              the face, reconstructed field by field and mapped back (the
 *              scheme's name in Sect. 2.1, "WENO-Roe"); FP64 only, no adjoint
 *              (hydro_step_vjp* return HYDRO_E_INVALID); a face whose averaged
 *              sound speed is not real counts as an unphysical state. */
typedef struct {
  int32_t nx, ny;
  double xlo, xhi, ylo, yhi;
  int32_t geometry;
  int32_t bc[4];
  double gamma, cfl, weno_eps;
  int32_t precision;
  double gx, gy;
  double rho_floor, p_floor;
  int32_t reconstruction;
} hydro_params;

/* Global Lax-Friedrichs speeds of the three Runge-Kutta stages (Sect. 2.1:
 * alpha_x = max over interior cells of |v_x| + c, alpha_y = max |v_y| + c,
 * each taken from the stage's input state).  Recorded by the forward step and
 * replayed ("frozen") by the adjoint. */
typedef struct {
  double ax[3], ay[3];
} hydro_alpha;

typedef struct hydro_ctx hydro_ctx;

/* Create a context on the current HIP device.
 *  params   copied.
 *  gravity  NULL (uniform params->gx, gy) or a device field [2][ny][nx] of
 *           (g_x, g_y) per cell; borrowed, must outlive the context.
 *  stream   a hipStream_t, or NULL for the null stream.
 *  out      receives the context.
 * Allocates 2 state-sized scratch buffers (64 B per cell); the first
 * hydro_step_vjp_saved call adds 3 more, the first hydro_step_vjp call 5.
 * Errors: INVALID, NOMEM, DEVICE. */
int hydro_create(const hydro_params* params, const double* gravity, void* stream,
                 hydro_ctx** out);

/* Free the context's scratch (waits for its stream).  NULL is accepted. */
int hydro_destroy(hydro_ctx* ctx);

/* CFL time step of state U (Sect. 5.3): dt = cfl * min(dx, dy) / max over
 * interior cells of (c + |v_x| + |v_y|) (dx alone when ny == 1).
 * Synchronises; *dt_host receives the value.  UNPHYSICAL if U has rho <= 0
 * or p <= 0 somewhere. */
int hydro_cfl(hydro_ctx* ctx, const double* U, double* dt_host);

/* One SSP-RK3 step of size dt, in place: U <- U^{n+1}.
 *  alpha_in   NULL: each stage computes its LF speeds from its input (the
 *             method); else the given speeds are used (replay of a recorded
 *             schedule, as the adjoint requires).
 *  alpha_out  NULL, or receives the speeds used (then the call synchronises).
 * Asynchronous otherwise. */
int hydro_step(hydro_ctx* ctx, double* U, double dt, const hydro_alpha* alpha_in,
               hydro_alpha* alpha_out);

/* Largest grid (nx * ny cells) hydro_step_noalloc accepts. */
#define HYDRO_NOALLOC_MAX_CELLS (1 << 20)

/* hydro_step without a context, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): one SSP-RK3 step of U in place, exactly as hydro_step computes
 * it (same kernels, same results bit for bit), allocating nothing.
 *  params, gravity  as for hydro_create (params checked the same way; gravity
 *             NULL or a device field [2][ny][nx]); nx * ny must not exceed
 *             HYDRO_NOALLOC_MAX_CELLS (else INVALID, before any device call).
 *  stream     a hipStream_t, or NULL for the null stream.
 *  U, dt, alpha_in  as for hydro_step (alpha_in NULL: each stage computes its
 *             LF speeds; else the given speeds are replayed).
 *  unphysical NULL, or a device int32 that receives 1 if a stage produced
 *             rho <= 0 or p <= 0, else 0 (there is no context whose flag
 *             hydro_check could read).
 * The stage states and reduction slots live in one device array of the
 * library (64 MiB + 33 KiB per device, held until the process ends, set up on
 * the first call on a device).  Every call on a device uses that array:
 * calls on one device must not overlap in time (different streams race); each
 * call clears what it needs.  Asynchronous. */
int hydro_step_noalloc(const hydro_params* params, const double* gravity, void* stream, double* U,
                       double dt, const hydro_alpha* alpha_in, int32_t* unphysical);

/* Up to nsteps steps with the CFL time step computed on the device (no host
 * round trip between steps), each clamped so that t never passes t_end
 * (t_end <= 0: no clamp, exactly nsteps steps).
 *  t_io       in: start time; out: time reached.
 *  dt_rec     NULL or device [nsteps] doubles: the dt of each step taken.
 *  alpha_rec  NULL or device [nsteps][6] doubles (ax[0..2], ay[0..2] of each
 *             step, the layout of hydro_alpha).
 * Synchronises at the end.  Returns the number of steps taken (>= 0) or an
 * error code. */
int hydro_run(hydro_ctx* ctx, double* U, int32_t nsteps, double t_end, double* t_io,
              double* dt_rec, double* alpha_rec);

/* hydro_run that keeps every state the adjoint needs, so that a backward pass
 * needs no replay (the memory-for-time end of the trade that checkpointing
 * makes the other way; 96 B per cell and step).  states: device
 * [nsteps][3][4][ny][nx]: [k][0] the state at the start of step k, [k][1] and
 * [k][2] its two Runge-Kutta stage states (as hydro_step_save writes them);
 * entries of steps not taken (t_end reached) are left as they are; it must
 * not overlap U.  U: in, the initial state; out, the final one.  Other arguments, return value and
 * synchronisation as hydro_run. */
int hydro_run_save(hydro_ctx* ctx, double* U, int32_t nsteps, double t_end, double* t_io,
                   double* dt_rec, double* alpha_rec, double* states);

/* The spatial operator alone: L = S(V) - (dF/dx + dG/dy) for given LF speeds
 * (the right-hand side each Runge-Kutta stage integrates).  L: device
 * [4][ny][nx], overwritten.  Asynchronous. */
int hydro_rhs(hydro_ctx* ctx, const double* V, double ax, double ay, double* L);

/* Discrete adjoint of one step: lam_prev = (dU^{n+1}/dU^n)^T lam_next for the
 * step hydro_step(U_n, dt, alpha) performs with the given (recorded) LF speeds
 * held fixed.  Recomputes the two intermediate stage states from U_n.
 * U_n, lam_next: device [4][ny][nx], read only; lam_prev: device
 * [4][ny][nx], overwritten (may not alias the others).  The atmosphere
 * floors must be disabled (INVALID otherwise).  The first adjoint call of a
 * context allocates its adjoint scratch (NOMEM if that fails).  Asynchronous. */
int hydro_step_vjp(hydro_ctx* ctx, const double* U_n, double dt, const hydro_alpha* alpha,
                   const double* lam_next, double* lam_prev);

/* One step U_in -> U_out (U_out may equal U_in) that also keeps its two
 * intermediate stage states: U1_out and U2_out (device [4][ny][nx],
 * overwritten, distinct from each other and from U_in, U_out) receive
 * U1 = U + dt L(U) and U2 = 3/4 U + 1/4 (U1 + dt L(U1)) of the SSP-RK3 step
 * (Sect. 2.1).  alpha_in as for hydro_step.  For adjoint replays, which then
 * need not recompute the stages (see hydro_step_vjp_saved).  Asynchronous. */
int hydro_step_save(hydro_ctx* ctx, const double* U_in, double* U_out, double dt,
                    const hydro_alpha* alpha_in, double* U1_out, double* U2_out);

/* hydro_step_vjp with the step's stage states supplied (as hydro_step_save
 * wrote them for the same U_n, dt and alpha) instead of recomputed.
 * lam_prev may not alias any other argument.  Asynchronous. */
int hydro_step_vjp_saved(hydro_ctx* ctx, const double* U_n, const double* U1, const double* U2,
                         double dt, const hydro_alpha* alpha, const double* lam_next,
                         double* lam_prev);

/* Gravitational potential of a density field (Sect. 2.1): the Poisson
 * equation (1/r) d/dr (r dPhi/dr) + d^2Phi/dz^2 = 4 pi G rho on the context's
 * quarter plane (cylindrical geometry with xlo = ylo = 0: x = r, y = z),
 * solved by successive over-relaxation (factor omega in (0, 2)) of
 * Gauss-Seidel sweeps in red-black order (colour (i + j) mod 2, red first),
 * stopped after the first iteration whose largest relative change
 * |new - old| / |new| is below tol (the paper uses 1e-8), or after max_iter.
 * Reflecting at the axis and the symmetry plane; the outer ghost cells hold
 * the Roche value -G mass / sqrt(r^2 + z^2) (mass: the total mass of the
 * mirror-symmetric configuration, given by the caller).  Cell-centred
 * five-point stencil, r-operator in flux form.
 *  rho       device [ny][nx] (the density component of a state will do).
 *  phi       device [ny][nx], in: starting potential; out: the solution.
 *  iters_out, change_out: NULL or receive the iterations done and the last
 *            iteration's largest relative change (not converged when
 *            iters == max_iter and change >= tol).
 * Synchronises once per batch of iterations (batches of 8, 16, .. 256).
 * INVALID if the context is not such a quarter plane. */
int hydro_poisson(hydro_ctx* ctx, const double* rho, double* phi, double G, double mass,
                  double omega, double tol, int32_t max_iter, int32_t* iters_out,
                  double* change_out);

/* g = -grad Phi at the cell centres by central differences (mirror across the
 * axis and the plane, Roche values beyond the outer edges), for use as the
 * gravity field of hydro_create.  g_out: device [2][ny][nx] (g_r, g_z).
 * Same geometry requirement as hydro_poisson.  Asynchronous. */
int hydro_gravity(hydro_ctx* ctx, const double* phi, double G, double mass, double* g_out);

/* ---- Level set (Sect. 2.3): the flame front as the zero contour of a field S
 * on the grid corners (S > 0 burnt, S < 0 fuel).  Corner (i, j), i = 0..nx,
 * j = 0..ny, lies at (xlo + i dx, ylo + j dy); corner fields are device arrays
 * [ny+1][nx+1], corner velocities [2][ny+1][nx+1] (u, v).  Ghost corners follow
 * the context's boundary codes: periodic (corner nx is corner 0's image),
 * reflecting (mirror about the wall corner), transmissive (linear
 * extrapolation).  Two-dimensional contexts only (ny >= 3), any geometry (the
 * field is advected in the (x, y) plane).  The first level-set call allocates
 * two corner fields and room for 3 front points per corner (HYDRO_E_NOMEM when
 * that fails).  All four calls run on the context's stream. */

/* Corner velocity from a cell state U[4][ny][nx]: the mean of the velocities
 * m/rho of the four cells that share the corner, with the fluid's ghost cells
 * beyond the grid.  Asynchronous. */
int hydro_ls_velocity(hydro_ctx* ctx, const double* U, double* vel);

/* One SSP-RK3 step of dS/dt = -(v + v_flame) . grad S, v_flame = s_flame along
 * the outward normal of the burnt region, i.e. S_t + u S_x + v S_y =
 * s_flame |grad S|: Hamilton-Jacobi WENO5 (the fluid's reconstruction applied
 * to one-sided differences), global Lax-Friedrichs flux with speeds
 * max|u| + s_flame, max|v| + s_flame over the corners, velocity frozen over
 * the step, time step dt.  S in place (periodic image corners are set from
 * their sources first).  s_flame >= 0.  Asynchronous. */
int hydro_ls_step(hydro_ctx* ctx, double* S, const double* vel, double s_flame, double dt);

/* Front points of S: one where neighbouring corners (in x or in y) have values
 * of opposite sign, placed by linear interpolation, and one at every corner
 * where S = 0.  pts: device [cap][2] (x, y), filled in no particular order with
 * min(count, cap) points; *count receives the number found.  Synchronises. */
int hydro_ls_front(hydro_ctx* ctx, const double* S, double* pts, int64_t cap, int64_t* count);

/* Re-distancing: every corner takes d, its distance to the nearest front point,
 * and S = H(d) S + (1 - H(d)) sign(S) d with
 * H(d) = (1 - tanh((d - 3D) / (D/3))) / (1 - tanh(-9)), D = min(dx, dy): values
 * within about two spacings of the front are kept, far values become the
 * distance.  With no front point S is left as it is.  dist: NULL or device
 * [ny+1][nx+1] receiving d (untouched without front points).  *npoints (may be
 * NULL) receives the number of front points: then the call synchronises at
 * its end; with npoints NULL it only enqueues. */
int hydro_ls_redistance(hydro_ctx* ctx, double* S, double* dist, int64_t* npoints);

/* Conserved totals: the integrals of rho, m_x, m_y and E over the grid, i.e.
 * the mass, momentum and energy whose relative changes Delta M / M and
 * Delta E / E the paper reports for its Gresho vortex test (Sect. 5.2, Table
 * Test2D_test1).  Each value times the cell volume (dx dy; 2 pi r_i dx dy in
 * cylindrical geometry, r_i = xlo + (i + 1/2) dx), summed with compensated
 * (Neumaier) summation over a fixed partition and tree, so the result does not
 * depend on the launch.  U: device [4][ny][nx].  Synchronises; out_host[4]
 * receives the four totals. */
int hydro_sums(hydro_ctx* ctx, const double* U, double out_host[4]);

/* Synchronise and return (then clear) the sticky UNPHYSICAL flag. */
int hydro_check(hydro_ctx* ctx);

/* Static string naming an error code. */
const char* hydro_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* HYDRO_H */
