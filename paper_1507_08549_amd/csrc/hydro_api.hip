// hydro_api.hip -- the C ABI declared in include/hydro.h: context management,
// parameter checks, and the launch sequences of the forward step, the
// multi-step run with a device-side CFL step, the spatial operator, the
// reductions and the discrete adjoint.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <new>

#include "hydro.h"
#include "hydro_internal.hpp"
#include "vjp.hpp"

struct hydro_ctx {
  hydro_params p;
  hy::Geom g;
  hipStream_t stream;
  int device;
  size_t n;              // cells
  double* U1;            // stage states
  double* U2;
  double* X[5];          // adjoint scratch (first adjoint call): recomputed stage states, stage adjoints, partial sum
  hy::Ctl* ctl;          // device control block
  double* rec;           // device: alpha record of hydro_step ([6])
  double* partial;       // device: per-block partial sums
  double* sum_out;       // device: [4]
  double* apart;         // device: partial maxima of the LF/CFL reduction ([256][4])
  double* ghost;         // device: adjoint of ghost cells ([2][3][max(nx, ny)][4] per axis)
  int nsum;
  hy::Ctl* h_ctl;        // pinned host staging
  double* h_buf;         // pinned host staging ([8])
  // level set (allocated by the first level-set call)
  double* ls_a;          // stage corner fields
  double* ls_b;
  double* ls_pts;        // front points, capacity 3 per corner ([2] each)
  hy::LsCtl* ls_ctl;
  unsigned long long* h_npts;  // pinned host staging
  int ls_aset, ls_pset;  // the control sets the next advection step / front search use
  // potential solver (allocated by the first call)
  double* p_scratch;     // second potential buffer
  hy::PoissonCtl* pc;
  hy::PoissonCtl* h_pc;  // pinned host staging (header)
};

namespace {

struct DeviceGuard {
  int prev = -1;
  bool ok = true;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) { ok = false; return; }
    if (prev != dev && hipSetDevice(dev) != hipSuccess) ok = false;
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

#define HY_CHECK(call)                                  \
  do {                                                  \
    if ((call) != hipSuccess) return HYDRO_E_DEVICE;    \
  } while (0)

int check_params(const hydro_params* p) {
  if (!p) return HYDRO_E_INVALID;
  if (p->nx < 3 || p->ny < 1 || (p->ny > 1 && p->ny < 3)) return HYDRO_E_INVALID;
  if ((long long)p->nx * (long long)p->ny > (1LL << 31) - 1) return HYDRO_E_INVALID;
  if (!(p->xhi > p->xlo) || !(p->yhi > p->ylo)) return HYDRO_E_INVALID;
  if (!(p->gamma > 1.0) || !(p->weno_eps >= 1e-30) || !(p->cfl > 0.0)) return HYDRO_E_INVALID;
  if (!std::isfinite(p->gx) || !std::isfinite(p->gy)) return HYDRO_E_INVALID;
  for (int k = 0; k < 4; ++k)
    if (p->bc[k] < 0 || p->bc[k] > 2) return HYDRO_E_INVALID;
  if ((p->bc[0] == HYDRO_PERIODIC) != (p->bc[1] == HYDRO_PERIODIC)) return HYDRO_E_INVALID;
  if ((p->bc[2] == HYDRO_PERIODIC) != (p->bc[3] == HYDRO_PERIODIC)) return HYDRO_E_INVALID;
  if (p->geometry != HYDRO_CARTESIAN && p->geometry != HYDRO_CYLINDRICAL) return HYDRO_E_INVALID;
  if (p->geometry == HYDRO_CYLINDRICAL && p->xlo < 0.0) return HYDRO_E_INVALID;
  if (p->precision != HYDRO_FP64 && p->precision != HYDRO_FP32_BULK) return HYDRO_E_INVALID;
  // FP32-bulk forms the weights d_k / (eps + beta_k)^2 in single precision:
  // on flat data they reach 1 / eps^2, which must stay far below FLT_MAX
  if (p->precision == HYDRO_FP32_BULK && !(p->weno_eps >= 1e-12)) return HYDRO_E_INVALID;
  if (p->rho_floor > 0.0 && !(p->p_floor > 0.0)) return HYDRO_E_INVALID;
  if (p->reconstruction != HYDRO_COMPONENTWISE && p->reconstruction != HYDRO_CHARACTERISTIC)
    return HYDRO_E_INVALID;
  if (p->reconstruction == HYDRO_CHARACTERISTIC && p->precision != HYDRO_FP64) return HYDRO_E_INVALID;
  return HYDRO_OK;
}

// Derived constants, each formed with the same operations as a direct
// evaluation (so the kernels' arithmetic does not depend on where they were
// formed).
hy::Geom make_geom(const hydro_params* p, const double* gravity) {
  hy::Geom g{};
  g.nx = p->nx;
  g.ny = p->ny;
  g.has_y = p->ny > 1;
  for (int k = 0; k < 4; ++k) g.bc[k] = p->bc[k];
  g.cyl = p->geometry == HYDRO_CYLINDRICAL;
  g.dx = (p->xhi - p->xlo) / (double)p->nx;
  g.dy = (p->yhi - p->ylo) / (double)p->ny;
  g.idx = 1.0 / g.dx;
  g.idy = 1.0 / g.dy;
  g.xlo = p->xlo;
  g.gamma = p->gamma;
  g.gm1 = p->gamma - 1.0;
  g.eps = p->weno_eps;
  g.gx = p->gx;
  g.gy = p->gy;
  g.grav = gravity;
  g.floor_on = p->rho_floor > 0.0;
  g.rho_floor = p->rho_floor;
  g.p_floor = p->p_floor;
  g.e_floor = p->p_floor / (p->gamma - 1.0);
  double dmin = g.dx;
  if (g.has_y && g.dy < dmin) dmin = g.dy;
  g.cfl_dmin = p->cfl * dmin;
  g.charw = p->reconstruction == HYDRO_CHARACTERISTIC;
  return g;
}

__global__ void set_ctl_kernel(hy::Ctl* ctl, double t) {
  if (threadIdx.x == 0) {
    ctl->t = t;
    ctl->dt = 0.0;
    ctl->active = 1;
    ctl->steps = 0;
  }
}

hipError_t launch_stage(const hydro_ctx* c, const hy::StageArgs& a) {
  return c->p.precision == HYDRO_FP64 ? hy::launch_stage_fp64(a, c->stream)
                                      : hy::launch_stage_fp32(a, c->stream);
}

const double kStageWeight[3] = {1.0, 0.25, 2.0 / 3.0};

hy::StageArgs stage_args(const hydro_ctx* c, double* U, int s) {
  hy::StageArgs a{};
  a.g = c->g;
  a.U0 = U;
  a.V = s == 0 ? U : (s == 1 ? c->U1 : c->U2);
  a.W = s == 0 ? c->U1 : (s == 1 ? c->U2 : U);
  a.b = kStageWeight[s];
  a.stage = s;
  a.ctl = c->ctl;
  return a;
}

int read_flag(hydro_ctx* c, bool clear) {
  HY_CHECK(hipMemcpyAsync(c->h_ctl, c->ctl, hy::kCtlHeader, hipMemcpyDeviceToHost, c->stream));
  HY_CHECK(hipStreamSynchronize(c->stream));
  const int f = c->h_ctl->flag;
  if (f && clear) {
    HY_CHECK(hipMemsetAsync(&c->ctl->flag, 0, sizeof(int), c->stream));
    HY_CHECK(hipStreamSynchronize(c->stream));
  }
  return f ? HYDRO_E_UNPHYSICAL : HYDRO_OK;
}

// One step U_in -> U_out (may be the same buffer) with the stage states in
// S1, S2 (the context's scratch or the caller's buffers).
int step_impl(hydro_ctx* c, const double* U_in, double* U_out, double dt, const hydro_alpha* alpha_in,
              hydro_alpha* alpha_out, double* S1, double* S2) {
  // A replay of recorded speeds neither reads nor needs the reduction slots.
  if (!alpha_in) HY_CHECK(hy::launch_alpha_reduce(c->g, U_in, c->ctl, 0, c->apart, c->stream));
  for (int s = 0; s < 3; ++s) {
    hy::StageArgs a = stage_args(c, U_out, s);
    a.U0 = U_in;
    a.V = s == 0 ? U_in : (s == 1 ? S1 : S2);
    a.W = s == 0 ? S1 : (s == 1 ? S2 : U_out);
    a.dt_mode = 0;
    a.dt_host = dt;
    if (alpha_in) {
      a.frozen = 1;
      a.fax = alpha_in->ax[s];
      a.fay = alpha_in->ay[s];
    }
    a.alpha_rec = alpha_out ? c->rec : nullptr;
    HY_CHECK(launch_stage(c, a));
  }
  if (alpha_out) {
    HY_CHECK(hipMemcpyAsync(c->h_buf, c->rec, 6 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HY_CHECK(hipStreamSynchronize(c->stream));
    for (int s = 0; s < 3; ++s) {
      alpha_out->ax[s] = c->h_buf[s];
      alpha_out->ay[s] = c->h_buf[3 + s];
    }
  }
  return HYDRO_OK;
}

// The adjoint's scratch, allocated by the first adjoint call: the two stage
// adjoints and the y pass's partial sum (X[2..4]), and with recompute the two
// recomputed stage states (X[0..1]).  Forward-only contexts never hold it.
int ensure_adj(hydro_ctx* c, bool recompute) {
  const size_t bytes = 4 * c->n * sizeof(double);
  for (int k = recompute ? 0 : 2; k < 5; ++k) {
    if (c->X[k]) continue;
    if (hipMalloc(&c->X[k], bytes) != hipSuccess) {
      c->X[k] = nullptr;
      (void)hipGetLastError();
      return HYDRO_E_NOMEM;
    }
  }
  return HYDRO_OK;
}

// Adjoint of one step given its two stage states R1, R2.
int vjp_impl(hydro_ctx* c, const double* U_n, const double* R1, const double* R2, double dt,
             const hydro_alpha* alpha, const double* lam_next, double* lam_prev) {
  double* lam2 = c->X[2];
  double* lam1 = c->X[3];
  // Stage adjoints, last to first.  With W = U0 + b ((V - U0) + dt L(V)):
  //   dJ/dV  = b (lam + dt J_L(V)^T lam),  dJ/dU0 += (1 - b) lam.
  hy::VjpArgs v{};
  v.g = c->g;
  v.dt = dt;
  v.fp32 = c->p.precision == HYDRO_FP32_BULK;
  v.ghost = c->ghost;
  v.ghost_y_offset = 2 * 3 * 4 * (size_t)(c->p.nx > c->p.ny ? c->p.nx : c->p.ny);
  v.Gp = c->X[4];
  // stage 3 (input R2): lam2 = 2/3 (lam3 + dt J^T lam3)
  v.V = R2; v.lam = lam_next; v.b = kStageWeight[2]; v.ax = alpha->ax[2]; v.ay = alpha->ay[2];
  v.out = lam2;
  HY_CHECK(hy::launch_stage_vjp(v, c->stream));
  // stage 2 (input R1): lam1 = 1/4 (lam2 + dt J^T lam2)
  v.V = R1; v.lam = lam2; v.b = kStageWeight[1]; v.ax = alpha->ax[1]; v.ay = alpha->ay[1];
  v.out = lam1;
  HY_CHECK(hy::launch_stage_vjp(v, c->stream));
  // stage 1 (input U_n = U0, b = 1), plus the U0 shares of stages 3 and 2:
  // lam_prev = (lam1 + dt J^T lam1) + 1/3 lam3 + 3/4 lam2
  v.V = U_n; v.lam = lam1; v.b = kStageWeight[0]; v.ax = alpha->ax[0]; v.ay = alpha->ay[0];
  v.out = lam_prev;
  v.add0 = lam_next; v.c0 = 1.0 - kStageWeight[2];
  v.add1 = lam2; v.c1 = 1.0 - kStageWeight[1];
  HY_CHECK(hy::launch_stage_vjp(v, c->stream));
  return HYDRO_OK;
}

void free_ctx(hydro_ctx* c) {
  if (!c) return;
  (void)hipFree(c->U1);
  (void)hipFree(c->U2);
  for (double* x : c->X) (void)hipFree(x);
  (void)hipFree(c->ctl);
  (void)hipFree(c->rec);
  (void)hipFree(c->partial);
  (void)hipFree(c->sum_out);
  (void)hipFree(c->ghost);
  (void)hipFree(c->apart);
  (void)hipHostFree(c->h_ctl);
  (void)hipHostFree(c->h_buf);
  (void)hipFree(c->ls_a);
  (void)hipFree(c->ls_b);
  (void)hipFree(c->ls_pts);
  (void)hipFree(c->ls_ctl);
  (void)hipHostFree(c->h_npts);
  (void)hipFree(c->p_scratch);
  (void)hipFree(c->pc);
  (void)hipHostFree(c->h_pc);
  delete c;
}

// ---- the allocation-free step (hydro_step_noalloc)
// Scratch of the step variant that allocates nothing: a control block
// (reduction slots, flag), the partial maxima of the speed reduction and the
// two stage states of a grid of at most HYDRO_NOALLOC_MAX_CELLS cells, in one
// file-scope device array.  Each device holds its own copy from the first
// launch of this library's code until the process ends.  In host code the
// array's name is not a device address: hydro_step_noalloc looks the address
// up once per device (hipGetSymbolAddress) and passes that pointer on.
constexpr size_t kNaCtlBytes = (sizeof(hy::Ctl) + 255) / 256 * 256;
constexpr size_t kNaPartialBytes = 256 * 4 * sizeof(double);
constexpr size_t kNaStateBytes = 4 * (size_t)HYDRO_NOALLOC_MAX_CELLS * sizeof(double);
constexpr size_t kNaScratchBytes = kNaCtlBytes + kNaPartialBytes + 2 * kNaStateBytes;
}  // namespace

static __device__ __align__(256) unsigned char scratch[kNaScratchBytes];

namespace {
std::mutex g_na_mutex;
unsigned char* g_na_ptr[hy::MAX_DEVICES];  // device address of `scratch`, per device

// Address of this device's scratch array (looked up on the first call on the device).
int noalloc_scratch(int dev, unsigned char** out) {
  if (dev < 0 || dev >= hy::MAX_DEVICES) return HYDRO_E_DEVICE;
  std::lock_guard<std::mutex> lock(g_na_mutex);
  if (!g_na_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return HYDRO_E_DEVICE;
    g_na_ptr[dev] = static_cast<unsigned char*>(p);
  }
  *out = g_na_ptr[dev];
  return HYDRO_OK;
}

// Start of a call: the error flag and the header of the control block cleared
// (a kernel, not a memset, so that the call can be captured in a graph).
__global__ void noalloc_begin_kernel(hy::Ctl* ctl) {
  if (threadIdx.x == 0) {
    ctl->t = 0.0;
    ctl->dt = 0.0;
    ctl->active = 1;
    ctl->steps = 0;
    ctl->flag = 0;
  }
}

// End of a call: the flag (1: a stage produced rho <= 0 or p <= 0) to the caller.
__global__ void noalloc_end_kernel(const hy::Ctl* ctl, int32_t* unphysical) {
  if (threadIdx.x == 0) *unphysical = ctl->flag ? 1 : 0;
}

}  // namespace

extern "C" {

int hydro_create(const hydro_params* params, const double* gravity, void* stream, hydro_ctx** out) {
  if (!out) return HYDRO_E_INVALID;
  *out = nullptr;
  int rc = check_params(params);
  if (rc) return rc;
  hydro_ctx* c = new (std::nothrow) hydro_ctx();
  if (!c) return HYDRO_E_NOMEM;
  c->p = *params;
  c->g = make_geom(params, gravity);
  c->stream = (hipStream_t)stream;
  if (hipGetDevice(&c->device) != hipSuccess) { delete c; return HYDRO_E_DEVICE; }
  c->n = (size_t)params->nx * (size_t)params->ny;
  const size_t bytes = 4 * c->n * sizeof(double);
  c->nsum = hy::sums_blocks(c->g);
  bool ok = hipMalloc(&c->U1, bytes) == hipSuccess && hipMalloc(&c->U2, bytes) == hipSuccess;
  ok = ok && hipMalloc(&c->ctl, sizeof(hy::Ctl)) == hipSuccess;
  ok = ok && hipMalloc(&c->rec, 8 * sizeof(double)) == hipSuccess;
  ok = ok && hipMalloc(&c->partial, (size_t)c->nsum * 8 * sizeof(double)) == hipSuccess;
  ok = ok && hipMalloc(&c->sum_out, 4 * sizeof(double)) == hipSuccess;
  const size_t nmax = (size_t)(params->nx > params->ny ? params->nx : params->ny);
  ok = ok && hipMalloc(&c->apart, 256 * 4 * sizeof(double)) == hipSuccess;
  ok = ok && hipMalloc(&c->ghost, 2 * 2 * 3 * nmax * 4 * sizeof(double)) == hipSuccess;
  ok = ok && hipHostMalloc((void**)&c->h_ctl, sizeof(hy::Ctl), hipHostMallocDefault) == hipSuccess;
  ok = ok && hipHostMalloc((void**)&c->h_buf, 8 * sizeof(double), hipHostMallocDefault) == hipSuccess;
  if (!ok) {
    free_ctx(c);
    (void)hipGetLastError();
    return HYDRO_E_NOMEM;
  }
  if (hipMemsetAsync(c->ctl, 0, sizeof(hy::Ctl), c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess) {
    free_ctx(c);
    return HYDRO_E_DEVICE;
  }
  *out = c;
  return HYDRO_OK;
}

int hydro_destroy(hydro_ctx* c) {
  if (!c) return HYDRO_OK;
  DeviceGuard dg(c->device);
  int rc = (hipStreamSynchronize(c->stream) == hipSuccess) ? HYDRO_OK : HYDRO_E_DEVICE;
  free_ctx(c);
  return rc;
}

int hydro_cfl(hydro_ctx* c, const double* U, double* dt_host) {
  if (!c || !U || !dt_host) return HYDRO_E_INVALID;
  DeviceGuard dg(c->device);
  if (!dg.ok) return HYDRO_E_DEVICE;
  HY_CHECK(hy::launch_alpha_reduce(c->g, U, c->ctl, 0, c->apart, c->stream));
  int rc = read_flag(c, false);
  if (rc) return rc;
  HY_CHECK(hipMemcpyAsync(c->h_buf, &c->ctl->slot[0][0][0], 3 * sizeof(double), hipMemcpyDeviceToHost,
                          c->stream));
  HY_CHECK(hipStreamSynchronize(c->stream));
  const double smax = c->h_buf[2];
  *dt_host = c->g.cfl_dmin / smax;
  return HYDRO_OK;
}

int hydro_step(hydro_ctx* c, double* U, double dt, const hydro_alpha* alpha_in,
               hydro_alpha* alpha_out) {
  if (!c || !U || !(dt >= 0.0)) return HYDRO_E_INVALID;
  DeviceGuard dg(c->device);
  if (!dg.ok) return HYDRO_E_DEVICE;
  return step_impl(c, U, U, dt, alpha_in, alpha_out, c->U1, c->U2);
}

int hydro_step_save(hydro_ctx* c, const double* U_in, double* U_out, double dt,
                    const hydro_alpha* alpha_in, double* U1_out, double* U2_out) {
  if (!c || !U_in || !U_out || !U1_out || !U2_out || !(dt >= 0.0)) return HYDRO_E_INVALID;
  if (U1_out == U2_out || U1_out == U_in || U2_out == U_in || U1_out == U_out || U2_out == U_out)
    return HYDRO_E_INVALID;
  DeviceGuard dg(c->device);
  if (!dg.ok) return HYDRO_E_DEVICE;
  return step_impl(c, U_in, U_out, dt, alpha_in, nullptr, U1_out, U2_out);
}

int hydro_step_noalloc(const hydro_params* params, const double* gravity, void* stream, double* U,
                       double dt, const hydro_alpha* alpha_in, int32_t* unphysical) {
  if (!U || !(dt >= 0.0)) return HYDRO_E_INVALID;
  int rc = check_params(params);
  if (rc) return rc;
  if ((size_t)params->nx * (size_t)params->ny > (size_t)HYDRO_NOALLOC_MAX_CELLS) return HYDRO_E_INVALID;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return HYDRO_E_DEVICE;
  unsigned char* base = nullptr;
  if ((rc = noalloc_scratch(dev, &base))) return rc;
  hy::Ctl* ctl = reinterpret_cast<hy::Ctl*>(base);
  double* apart = reinterpret_cast<double*>(base + kNaCtlBytes);
  double* S1 = reinterpret_cast<double*>(base + kNaCtlBytes + kNaPartialBytes);
  double* S2 = reinterpret_cast<double*>(base + kNaCtlBytes + kNaPartialBytes + kNaStateBytes);
  const hy::Geom g = make_geom(params, gravity);
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(noalloc_begin_kernel, dim3(1), dim3(64), 0, st, ctl);
  HY_CHECK(hipGetLastError());
  // the same launch sequence as hydro_step, on the scratch array's buffers
  if (!alpha_in) HY_CHECK(hy::launch_alpha_reduce(g, U, ctl, 0, apart, st));
  for (int s = 0; s < 3; ++s) {
    hy::StageArgs a{};
    a.g = g;
    a.U0 = U;
    a.V = s == 0 ? U : (s == 1 ? S1 : S2);
    a.W = s == 0 ? S1 : (s == 1 ? S2 : U);
    a.b = kStageWeight[s];
    a.stage = s;
    a.ctl = ctl;
    a.dt_mode = 0;
    a.dt_host = dt;
    if (alpha_in) {
      a.frozen = 1;
      a.fax = alpha_in->ax[s];
      a.fay = alpha_in->ay[s];
    }
    HY_CHECK(params->precision == HYDRO_FP64 ? hy::launch_stage_fp64(a, st) : hy::launch_stage_fp32(a, st));
  }
  if (unphysical) {
    hipLaunchKernelGGL(noalloc_end_kernel, dim3(1), dim3(64), 0, st, ctl, unphysical);
    HY_CHECK(hipGetLastError());
  }
  return HYDRO_OK;
}

int hydro_run(hydro_ctx* c, double* U, int32_t nsteps, double t_end, double* t_io, double* dt_rec,
              double* alpha_rec) {
  if (!c || !U || nsteps < 0) return HYDRO_E_INVALID;
  DeviceGuard dg(c->device);
  if (!dg.ok) return HYDRO_E_DEVICE;
  const double t0 = t_io ? *t_io : 0.0;
  hipLaunchKernelGGL(set_ctl_kernel, dim3(1), dim3(64), 0, c->stream, c->ctl, t0);
  HY_CHECK(hipGetLastError());
  HY_CHECK(hy::launch_alpha_reduce(c->g, U, c->ctl, 0, c->apart, c->stream));
  for (int k = 0; k < nsteps; ++k) {
    for (int s = 0; s < 3; ++s) {
      hy::StageArgs a = stage_args(c, U, s);
      a.dt_mode = 1;
      a.t_end = t_end;
      a.dt_rec = dt_rec ? dt_rec + k : nullptr;
      a.alpha_rec = alpha_rec ? alpha_rec + 6 * (size_t)k : nullptr;
      HY_CHECK(launch_stage(c, a));
    }
  }
  int rc = read_flag(c, false);
  if (t_io) *t_io = c->h_ctl->t;
  if (rc) return rc;
  return c->h_ctl->steps;
}

int hydro_run_save(hydro_ctx* c, double* U, int32_t nsteps, double t_end, double* t_io, double* dt_rec,
                   double* alpha_rec, double* states) {
  if (!c || !U || !states || states == U || nsteps < 0) return HYDRO_E_INVALID;
  DeviceGuard dg(c->device);
  if (!dg.ok) return HYDRO_E_DEVICE;
  const size_t n4 = 4 * c->n;
  auto S = [&](int k, int s) { return states + ((size_t)k * 3 + (size_t)s) * n4; };
  const double t0 = t_io ? *t_io : 0.0;
  hipLaunchKernelGGL(set_ctl_kernel, dim3(1), dim3(64), 0, c->stream, c->ctl, t0);
  HY_CHECK(hipGetLastError());
  if (nsteps > 0) HY_CHECK(hipMemcpyAsync(S(0, 0), U, n4 * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  HY_CHECK(hy::launch_alpha_reduce(c->g, U, c->ctl, 0, c->apart, c->stream));
  for (int k = 0; k < nsteps; ++k) {
    for (int s = 0; s < 3; ++s) {
      hy::StageArgs a{};
      a.g = c->g;
      a.U0 = S(k, 0);
      a.V = S(k, s);
      a.W = s < 2 ? S(k, s + 1) : (k + 1 < nsteps ? S(k + 1, 0) : U);
      a.b = kStageWeight[s];
      a.stage = s;
      a.ctl = c->ctl;
      a.dt_mode = 1;
      a.t_end = t_end;
      a.dt_rec = dt_rec ? dt_rec + k : nullptr;
      a.alpha_rec = alpha_rec ? alpha_rec + 6 * (size_t)k : nullptr;
      HY_CHECK(launch_stage(c, a));
    }
  }
  int rc = read_flag(c, false);
  if (t_io) *t_io = c->h_ctl->t;
  const int steps = c->h_ctl->steps;
  if (steps > 0 && steps < nsteps) {  // stopped at t_end: the last state taken is the start of step `steps`
    HY_CHECK(hipMemcpyAsync(U, S(steps, 0), n4 * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    HY_CHECK(hipStreamSynchronize(c->stream));
  }
  if (rc) return rc;
  return steps;
}

int hydro_rhs(hydro_ctx* c, const double* V, double ax, double ay, double* L) {
  if (!c || !V || !L || V == L) return HYDRO_E_INVALID;
  DeviceGuard dg(c->device);
  if (!dg.ok) return HYDRO_E_DEVICE;
  hy::StageArgs a{};
  a.g = c->g;
  a.U0 = V;
  a.V = V;
  a.W = L;
  a.rhs_only = 1;
  a.frozen = 1;
  a.fax = ax;
  a.fay = ay;
  a.ctl = c->ctl;
  HY_CHECK(launch_stage(c, a));
  return HYDRO_OK;
}

int hydro_step_vjp(hydro_ctx* c, const double* U_n, double dt, const hydro_alpha* alpha,
                   const double* lam_next, double* lam_prev) {
  if (!c || !U_n || !alpha || !lam_next || !lam_prev) return HYDRO_E_INVALID;
  if (lam_prev == lam_next || lam_prev == U_n || !(dt >= 0.0)) return HYDRO_E_INVALID;
  if (c->g.floor_on || c->g.charw) return HYDRO_E_INVALID;
  DeviceGuard dg(c->device);
  if (!dg.ok) return HYDRO_E_DEVICE;
  if (int rc = ensure_adj(c, true)) return rc;
  // Recompute the stage states with the recorded speeds.
  double* R1 = c->X[0];
  double* R2 = c->X[1];
  for (int s = 0; s < 2; ++s) {
    hy::StageArgs a{};
    a.g = c->g;
    a.U0 = U_n;
    a.V = s == 0 ? U_n : R1;
    a.W = s == 0 ? R1 : R2;
    a.b = kStageWeight[s];
    a.stage = s;
    a.frozen = 1;
    a.fax = alpha->ax[s];
    a.fay = alpha->ay[s];
    a.dt_mode = 0;
    a.dt_host = dt;
    a.ctl = c->ctl;
    HY_CHECK(launch_stage(c, a));
  }
  return vjp_impl(c, U_n, R1, R2, dt, alpha, lam_next, lam_prev);
}

int hydro_step_vjp_saved(hydro_ctx* c, const double* U_n, const double* U1, const double* U2, double dt,
                         const hydro_alpha* alpha, const double* lam_next, double* lam_prev) {
  if (!c || !U_n || !U1 || !U2 || !alpha || !lam_next || !lam_prev) return HYDRO_E_INVALID;
  if (lam_prev == lam_next || lam_prev == U_n || lam_prev == U1 || lam_prev == U2 || !(dt >= 0.0))
    return HYDRO_E_INVALID;
  if (c->g.floor_on || c->g.charw) return HYDRO_E_INVALID;
  DeviceGuard dg(c->device);
  if (!dg.ok) return HYDRO_E_DEVICE;
  if (int rc = ensure_adj(c, false)) return rc;
  return vjp_impl(c, U_n, U1, U2, dt, alpha, lam_next, lam_prev);
}

namespace {
hy::PoissonArgs poisson_args(const hydro_ctx* c, const double* rho, double* phi, double G, double mass,
                             double omega, double tol) {
  hy::PoissonArgs a{};
  a.nr = c->p.nx;
  a.nz = c->p.ny;
  a.dr = c->g.dx;  // xlo = 0: (xhi - 0) / nx
  a.dz = c->g.dy;
  a.idr2 = 1.0 / (a.dr * a.dr);
  a.idz2 = 1.0 / (a.dz * a.dz);
  a.four_pi_g = (4.0 * 3.141592653589793) * G;
  a.G = G;
  a.mass = mass;
  a.omega = omega;
  a.tol = tol;
  a.rho = rho;
  a.phi = phi;
  return a;
}

bool poisson_geometry_ok(const hydro_ctx* c) {
  return c->g.cyl && c->g.has_y && c->p.xlo == 0.0 && c->p.ylo == 0.0;
}

int ensure_poisson(hydro_ctx* c) {
  if (c->pc) return HYDRO_OK;
  hy::PoissonCtl* pc = nullptr;
  bool ok = hipMalloc(&c->p_scratch, c->n * sizeof(double)) == hipSuccess &&
            hipMalloc(&pc, sizeof(hy::PoissonCtl)) == hipSuccess &&
            hipHostMalloc((void**)&c->h_pc, sizeof(hy::PoissonCtl), hipHostMallocDefault) == hipSuccess;
  if (!ok) {
    (void)hipFree(c->p_scratch);
    (void)hipFree(pc);
    (void)hipHostFree(c->h_pc);
    c->p_scratch = nullptr;
    c->h_pc = nullptr;
    (void)hipGetLastError();
    return HYDRO_E_NOMEM;
  }
  c->pc = pc;
  return HYDRO_OK;
}

// Temporally blocked: up to K iterations per launch, launches in batches of
// 2, 4, .. 64, a check after each batch, one host synchronisation per batch.
int poisson_blocked(hydro_ctx* c, hy::PoissonArgs a, int32_t max_iter, int32_t* iters_out,
                    double* change_out) {
  if (int rc = ensure_poisson(c)) return rc;
  const int config = hy::poisson_block_config(a.nr, a.nz);
  const int K = hy::poisson_block_k(config);
  a.X[0] = a.phi;
  a.X[1] = c->p_scratch;
  a.pc = c->pc;
  HY_CHECK(hy::launch_poisson_block_init(c->pc, c->stream));
  int l = 0, t = 0, kprev = 0, batch = 2;
  for (;;) {
    for (int b = 0; b < batch && t < max_iter; ++b) {
      a.l = l;
      a.kprev = kprev;
      a.kcur = K < max_iter - t ? K : max_iter - t;
      a.t0 = t;
      a.final_ = 0;
      HY_CHECK(hy::launch_poisson_block(a, config, c->stream));
      kprev = a.kcur;
      t += a.kcur;
      ++l;
    }
    // check launch l-1 (and, after the last iteration, record the outcome)
    a.l = l;
    a.kprev = kprev;
    a.kcur = 0;
    a.t0 = t;
    a.final_ = t >= max_iter;
    HY_CHECK(hy::launch_poisson_block(a, config, c->stream));
    HY_CHECK(hipMemcpyAsync(c->h_pc, c->pc, 32, hipMemcpyDeviceToHost, c->stream));
    HY_CHECK(hipStreamSynchronize(c->stream));
    if (c->h_pc->done_launch != 0x7fffffff) break;
    batch = batch < 64 ? 2 * batch : 64;
  }
  if (c->h_pc->result == 1)
    HY_CHECK(hipMemcpyAsync(a.phi, c->p_scratch, c->n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  if (iters_out) *iters_out = c->h_pc->iters;
  if (change_out) *change_out = c->h_pc->change;
  return HYDRO_OK;
}
}  // namespace

int hydro_poisson(hydro_ctx* c, const double* rho, double* phi, double G, double mass, double omega,
                  double tol, int32_t max_iter, int32_t* iters_out, double* change_out) {
  if (!c || !rho || !phi || !(omega > 0.0 && omega < 2.0) || max_iter < 1 || !(tol >= 0.0))
    return HYDRO_E_INVALID;
  if (!poisson_geometry_ok(c) || !(mass > 0.0) || !(G > 0.0)) return HYDRO_E_INVALID;
  DeviceGuard dg(c->device);
  if (!dg.ok) return HYDRO_E_DEVICE;
  hy::PoissonArgs a = poisson_args(c, rho, phi, G, mass, omega, tol);
  return poisson_blocked(c, a, max_iter, iters_out, change_out);
}

int hydro_gravity(hydro_ctx* c, const double* phi, double G, double mass, double* g_out) {
  if (!c || !phi || !g_out || !poisson_geometry_ok(c) || !(mass > 0.0) || !(G > 0.0))
    return HYDRO_E_INVALID;
  DeviceGuard dg(c->device);
  if (!dg.ok) return HYDRO_E_DEVICE;
  hy::PoissonArgs a = poisson_args(c, nullptr, const_cast<double*>(phi), G, mass, 1.0, 0.0);
  HY_CHECK(hy::launch_gravity(a, g_out, c->stream));
  return HYDRO_OK;
}

namespace {
size_t ls_corners(const hydro_ctx* c) { return (size_t)(c->p.nx + 1) * (size_t)(c->p.ny + 1); }

int ensure_ls(hydro_ctx* c) {
  if (c->ls_ctl) return HYDRO_OK;
  const size_t nc = ls_corners(c);
  bool ok = hipMalloc(&c->ls_a, nc * sizeof(double)) == hipSuccess &&
            hipMalloc(&c->ls_b, nc * sizeof(double)) == hipSuccess &&
            hipMalloc(&c->ls_pts, 3 * nc * 2 * sizeof(double)) == hipSuccess &&
            hipHostMalloc((void**)&c->h_npts, sizeof(unsigned long long), hipHostMallocDefault) == hipSuccess;
  hy::LsCtl* lc = nullptr;
  ok = ok && hipMalloc(&lc, sizeof(hy::LsCtl)) == hipSuccess;
  if (!ok) {
    (void)hipFree(c->ls_a);
    (void)hipFree(c->ls_b);
    (void)hipFree(c->ls_pts);
    (void)hipFree(lc);
    (void)hipHostFree(c->h_npts);
    c->ls_a = c->ls_b = c->ls_pts = nullptr;
    c->h_npts = nullptr;
    (void)hipGetLastError();
    return HYDRO_E_NOMEM;
  }
  c->ls_ctl = lc;
  c->ls_aset = c->ls_pset = 0;
  HY_CHECK(hy::launch_ls_init(lc, c->stream));
  return HYDRO_OK;
}

hy::LsArgs ls_args(const hydro_ctx* c) {
  hy::LsArgs a{};
  a.mx = c->p.nx + 1;
  a.my = c->p.ny + 1;
  for (int k = 0; k < 4; ++k) a.bc[k] = c->p.bc[k];
  a.xlo = c->p.xlo;
  a.ylo = c->p.ylo;
  a.dx = c->g.dx;
  a.dy = c->g.dy;
  a.idx = c->g.idx;  // 1.0 / dx
  a.idy = c->g.idy;
  a.eps = c->p.weno_eps;
  a.lc = c->ls_ctl;
  return a;
}

// Front points of S into the context's buffer; returns their number in *np.
int ls_front(hydro_ctx* c, const double* S, long long* np) {
  hy::LsArgs a = ls_args(c);
  a.V = S;
  a.set = c->ls_pset;
  c->ls_pset ^= 1;
  HY_CHECK(hy::launch_ls_front(a, c->ls_pts, c->stream));
  HY_CHECK(hipMemcpyAsync(c->h_npts, &c->ls_ctl->npts[a.set], sizeof(unsigned long long),
                          hipMemcpyDeviceToHost, c->stream));
  HY_CHECK(hipStreamSynchronize(c->stream));
  *np = (long long)*c->h_npts;
  return HYDRO_OK;
}
}  // namespace

#define HY_LS_PROLOGUE(c)                       \
  if (!(c)) return HYDRO_E_INVALID;             \
  if ((c)->p.ny < 3) return HYDRO_E_INVALID;    \
  DeviceGuard dg((c)->device);                  \
  if (!dg.ok) return HYDRO_E_DEVICE;            \
  if (int rc_ = ensure_ls(c)) return rc_

int hydro_ls_velocity(hydro_ctx* c, const double* U, double* vel) {
  HY_LS_PROLOGUE(c);
  if (!U || !vel) return HYDRO_E_INVALID;
  hy::LsArgs a = ls_args(c);
  a.W = vel;
  HY_CHECK(hy::launch_ls_velocity(a, U, c->stream));
  return HYDRO_OK;
}

int hydro_ls_step(hydro_ctx* c, double* S, const double* vel, double s_flame, double dt) {
  HY_LS_PROLOGUE(c);
  if (!S || !vel || !(s_flame >= 0.0) || !std::isfinite(s_flame) || !std::isfinite(dt))
    return HYDRO_E_INVALID;
  hy::LsArgs a = ls_args(c);
  a.vel = vel;
  a.s_f = s_flame;
  a.dt = dt;
  a.S0 = S;
  a.set = c->ls_aset;
  c->ls_aset ^= 1;
  HY_CHECK(hy::launch_ls_images(a, S, c->stream));
  HY_CHECK(hy::launch_ls_alpha(a, c->stream));
  const double b[3] = {1.0, 0.25, 2.0 / 3.0};
  const double* in[3] = {S, c->ls_a, c->ls_b};
  double* out[3] = {c->ls_a, c->ls_b, S};
  for (int st = 0; st < 3; ++st) {
    a.V = in[st];
    a.W = out[st];
    a.b = b[st];
    HY_CHECK(hy::launch_ls_stage(a, c->stream));
  }
  return HYDRO_OK;
}

int hydro_ls_front(hydro_ctx* c, const double* S, double* pts, int64_t cap, int64_t* count) {
  HY_LS_PROLOGUE(c);
  if (!S || (cap > 0 && !pts) || cap < 0) return HYDRO_E_INVALID;
  long long np = 0;
  if (int rc = ls_front(c, S, &np)) return rc;
  const long long m = np < cap ? np : cap;
  if (m > 0)
    HY_CHECK(hipMemcpyAsync(pts, c->ls_pts, (size_t)m * 2 * sizeof(double), hipMemcpyDeviceToDevice,
                            c->stream));
  if (count) *count = np;
  return HYDRO_OK;
}

int hydro_ls_redistance(hydro_ctx* c, double* S, double* dist, int64_t* npoints) {
  HY_LS_PROLOGUE(c);
  if (!S) return HYDRO_E_INVALID;
  // the distance kernel reads the point count on the device (and leaves S and
  // dist as they are when it is 0), so nothing waits between the two launches
  hy::LsArgs a = ls_args(c);
  a.V = S;
  a.set = c->ls_pset;
  c->ls_pset ^= 1;
  HY_CHECK(hy::launch_ls_front(a, c->ls_pts, c->stream));
  a.W = S;
  HY_CHECK(hy::launch_ls_distance(a, c->ls_pts, dist, c->stream));
  if (npoints) {
    HY_CHECK(hipMemcpyAsync(c->h_npts, &c->ls_ctl->npts[a.set], sizeof(unsigned long long),
                            hipMemcpyDeviceToHost, c->stream));
    HY_CHECK(hipStreamSynchronize(c->stream));
    *npoints = (int64_t)*c->h_npts;
  }
  return HYDRO_OK;
}

int hydro_sums(hydro_ctx* c, const double* U, double out_host[4]) {
  if (!c || !U || !out_host) return HYDRO_E_INVALID;
  DeviceGuard dg(c->device);
  if (!dg.ok) return HYDRO_E_DEVICE;
  HY_CHECK(hy::launch_sums(c->g, U, c->partial, c->nsum, c->sum_out, c->stream));
  HY_CHECK(hipMemcpyAsync(c->h_buf, c->sum_out, 4 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HY_CHECK(hipStreamSynchronize(c->stream));
  for (int k = 0; k < 4; ++k) out_host[k] = c->h_buf[k];
  return HYDRO_OK;
}

int hydro_check(hydro_ctx* c) {
  if (!c) return HYDRO_E_INVALID;
  DeviceGuard dg(c->device);
  if (!dg.ok) return HYDRO_E_DEVICE;
  return read_flag(c, true);
}

const char* hydro_strerror(int code) {
  switch (code) {
    case HYDRO_OK: return "ok";
    case HYDRO_E_INVALID: return "invalid argument";
    case HYDRO_E_NOMEM: return "device allocation failed";
    case HYDRO_E_DEVICE: return "HIP runtime error";
    case HYDRO_E_UNPHYSICAL: return "unphysical state (rho <= 0 or p <= 0)";
    case HYDRO_E_STATE: return "invalid context state";
    default: return "unknown error";
  }
}

}  // extern "C"
