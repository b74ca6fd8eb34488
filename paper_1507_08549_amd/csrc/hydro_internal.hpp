// hydro_internal.hpp -- structures shared by the host side of the library and
// its HIP kernels.  Not part of the public ABI (include/hydro.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace hy {

constexpr int NG = 3;  // ghost layers: a five-point WENO stencil reaches 3 cells past a face

enum Bc : int { PERIODIC = 0, TRANSMISSIVE = 1, REFLECTING = 2 };

// Problem constants in the form the kernels use them.  Every derived value is
// computed once on the host with the same IEEE operations a direct
// evaluation would use (e.g. idx = 1.0 / dx), so device results do not
// depend on where a constant was formed.
struct Geom {
  int nx, ny;
  int has_y;             // ny > 1
  int bc[4];             // x-low, x-high, y-low, y-high
  int cyl;               // cylindrical (r, z): geometric sources
  double dx, dy, idx, idy;
  double xlo;
  double gamma, gm1, eps;
  double gx, gy;         // uniform gravity (when grav == nullptr)
  const double* grav;    // [2][ny][nx] or nullptr
  int floor_on;
  double rho_floor, p_floor, e_floor;  // e_floor = p_floor / (gamma - 1)
  double cfl_dmin;       // cfl * min(dx, dy) (dx in 1D)
  int charw;             // characteristic-wise reconstruction (FP64 only)
};

// Device-resident control block of a context.
// slot[k] holds the maxima (|u|+c, |v|+c, c+|u|+|v|) of one state as the bit
// patterns of non-negative doubles (their integer order is their numeric
// order, so atomicMax on the bits is an exact max).  The three slots form a
// ring over the Runge-Kutta stages: stage k reads slot k % 3 (its input's
// speeds), accumulates its output's speeds into slot (k + 1) % 3 and clears
// slot (k + 2) % 3 for the stage after it.
// Each slot is split into NSUB sub-slots on separate 128-byte lines:
// workgroup b merges into sub-slot b % NSUB, so the device-scope atomics of
// different workgroups do not queue on one address; a reader takes the max
// over the sub-slots (one wavefront, NSUB = 64 lanes).
constexpr int NSUB = 64;
// Devices per process for which per-device launch facts are cached.
constexpr int MAX_DEVICES = 16;
struct Ctl {
  double dt;       // time step of the current step (device-computed mode)
  double t;        // time reached
  double pad0;
  int active;      // current step is taken (t < t_end)
  int steps;       // steps taken by hydro_run
  int flag;        // sticky: a stage produced rho <= 0 or p <= 0
  int pad[7];
  unsigned long long slot[3][NSUB][16];
};
constexpr size_t kCtlHeader = 64;  // bytes before slot[][][]: what the host reads back
static_assert(offsetof(Ctl, slot) == kCtlHeader, "control header layout");

struct StageArgs {
  Geom g;
  const double* U0;   // state at the start of the step
  const double* V;    // stage input
  double* W;          // stage output (may alias U0: each cell reads U0 only at itself)
  double b;           // stage weight: W = U0 + b ((V - U0) + dt L(V))
  int stage;          // 0, 1, 2
  int frozen;         // use fax, fay instead of the slot
  double fax, fay;
  int dt_mode;        // 0: dt_host; 1: computed on the device from slot 0 (stage 0)
  double dt_host;
  double t_end;       // clamp of the device-computed step (<= 0: none)
  Ctl* ctl;
  double* dt_rec;     // device mode: this step's record, or nullptr
  double* alpha_rec;  // [6] for this step (ax[3], ay[3]), or nullptr
  int rhs_only;       // write L(V) to W instead of a stage
  int prio;           // set by the launcher: all workgroups resident at once
};

// Launchers (defined next to their kernels).
hipError_t launch_stage_fp64(const StageArgs& a, hipStream_t s);
hipError_t launch_stage_fp32(const StageArgs& a, hipStream_t s);
hipError_t launch_clear_slots(Ctl* ctl, hipStream_t s);
// Maxima of a state into ctl->slot[slot]; clears the other two slots.
// partial: scratch of 4 * 256 doubles.
hipError_t launch_alpha_reduce(const Geom& g, const double* U, Ctl* ctl, int slot, double* partial,
                               hipStream_t s);
hipError_t launch_sums(const Geom& g, const double* U, double* partial, int nblocks, double* out,
                       hipStream_t s);
int sums_blocks(const Geom& g);

// Potential solver (red-black over-relaxed Gauss-Seidel in (r, z)).
// Control block of the temporally blocked potential solver.
constexpr int PKMAX = 4;  // most iterations per launch
struct PoissonCtl {
  int done_launch;  // launch that ended the solve (INT_MAX while running)
  int iters;        // iterations done
  int result;       // buffer holding the result: 0 the caller's, 1 the scratch
  int pad0;
  double change;    // largest relative change of the last iteration
  double pad1[5];
  unsigned long long bank[3][PKMAX][NSUB][16];  // per launch (ring of 3), per iteration: max change
};

struct PoissonArgs {
  int nr, nz;
  double dr, dz, idr2, idz2;
  double four_pi_g, G, mass, omega, tol;
  const double* rho;
  double* phi;
  double* X[2];     // potential buffers: the caller's and a scratch one
  PoissonCtl* pc;
  int l;            // launch index (buffer parity, bank)
  int kprev;        // iterations done by launch l-1 (0: none)
  int kcur;         // iterations for this launch (0: only check launch l-1)
  int t0;           // index of this launch's first iteration
  int final_;       // no more launches follow: record the outcome
};
hipError_t launch_poisson_block_init(PoissonCtl* pc, hipStream_t s);
hipError_t launch_poisson_block(const PoissonArgs& a, int config, hipStream_t s);
int poisson_block_k(int config);
int poisson_block_config(int nr, int nz);
hipError_t launch_gravity(const PoissonArgs& a, double* g, hipStream_t s);

// Level set on the corners ([ny+1][nx+1]).  The point count and the speed
// sub-slots come in two sets that alternate between calls: a call works in
// one set and clears the other for the next call (stream order puts every use
// of a set before that clear), so no call needs a clearing launch.
struct LsCtl {
  unsigned long long npts[2];  // [set]: front points found
  unsigned long long pad[14];
  unsigned long long amax[2][NSUB][16];  // [set][sub][0]: max|u|, [1]: max|v| (bit patterns)
};
struct LsArgs {
  int mx, my;          // corners per row / column (nx + 1, ny + 1)
  int bc[4];           // fluid codes: 0 periodic, 1 transmissive (linear extrapolation), 2 reflecting
  double xlo, ylo, dx, dy, idx, idy, eps;  // idx = 1 / dx, idy = 1 / dy
  double s_f, dt, b;   // flame speed, time step, stage weight
  const double* S0;    // step input
  const double* V;     // stage input (front search: the field)
  double* W;           // stage output (distance: the field, in place; velocity: the output)
  const double* vel;   // corner velocity [2][my][mx]
  LsCtl* lc;
  int set;             // the call's set of lc
};
hipError_t launch_ls_init(LsCtl* lc, hipStream_t s);  // both sets of lc cleared
hipError_t launch_ls_alpha(const LsArgs& a, hipStream_t s);
hipError_t launch_ls_images(const LsArgs& a, double* S, hipStream_t s);
hipError_t launch_ls_stage(const LsArgs& a, hipStream_t s);
hipError_t launch_ls_front(const LsArgs& a, double* pts, hipStream_t s);
hipError_t launch_ls_distance(const LsArgs& a, const double* pts, double* dist, hipStream_t s);
hipError_t launch_ls_velocity(const LsArgs& a, const double* U, hipStream_t s);


}  // namespace hy
