// poisson.hip -- the gravitational potential of Sect. 2.1: the Poisson
// equation (1/r) d/dr (r dPhi/dr) + d^2Phi/dz^2 = 4 pi G rho in (r, z), solved by
// successive over-relaxation of Gauss-Seidel sweeps until the relative change
// of every cell is below a tolerance; reflecting axis (r = 0) and symmetry
// plane (z = 0), Roche values -G M / sqrt(r^2 + z^2) beyond the outer edges.
//
// Cell-centred five-point stencil, r-operator in flux form (face radii i dr and
// (i+1) dr, so the axis face has zero weight), mirror at z = 0, Roche values at
// the outer ghost centres.  Red-black order (colour (i + j) mod 2, red first)
// makes each colour's updates independent: one launch per colour, one work
// item per cell of the colour.  Every formula has the CPU oracle's evaluation
// order (FP64, built with -ffp-contract=off, no fma), so the potential and the
// iteration count agree bit for bit.
//
// Convergence without host round trips: each sweep merges its cells' largest
// relative change |new - old| / |new| into a ring of two slots (64 sub-slots on
// separate lines, as for the LF speeds); the red sweep of iteration k reads
// iteration k-1's slot and, when it is below the tolerance, marks the solve
// done: every later launch of the batch returns at once.  The black sweep of
// iteration k clears the slot iteration k+1 will fill.
#include "stage_kernel.hpp"

namespace hy {

constexpr int PS_THREADS = 256;

__device__ __forceinline__ double roche(const PoissonArgs& a, double r, double z) {
  return cr_div(-(a.G * a.mass), cr_sqrt(r * r + z * z));
}

// Largest relative change recorded in pslot[s] (wavefront 0; broadcast).
__device__ __forceinline__ double read_pslot(const Ctl* ctl, int s, double* sh) {
  if (threadIdx.x < NSUB) {
    double m = as_double(ctl->pslot[s][threadIdx.x][0]);
#pragma unroll
    for (int off = NSUB / 2; off > 0; off >>= 1) m = __builtin_fmax(m, __shfl_xor(m, off));
    if (threadIdx.x == 0) *sh = m;
  }
  __syncthreads();
  return *sh;
}

__global__ void poisson_init_kernel(Ctl* ctl) {
  const int t = threadIdx.x;
  if (t < NSUB) {
    ctl->pslot[0][t][0] = 0ull;
    ctl->pslot[1][t][0] = 0ull;
  }
  if (t == 0) {
    ctl->pdone = 0;
    ctl->piters = 0;
    ctl->pchange = 0.0;
  }
}

hipError_t launch_poisson_init(Ctl* ctl, hipStream_t s) {
  hipLaunchKernelGGL(poisson_init_kernel, dim3(1), dim3(64), 0, s, ctl);
  return hipGetLastError();
}

__global__ __launch_bounds__(PS_THREADS) void poisson_sweep_kernel(PoissonArgs a) {
  __shared__ double sh;
  __shared__ double red[PS_THREADS / 64];
  __shared__ int done;
  Ctl* ctl = a.ctl;
  const int tid = threadIdx.x;
  // one read per workgroup, so that every wavefront takes the same branch
  if (tid == 0) done = ctl->pdone;
  __syncthreads();
  if (done) return;
  if (a.colour == 0 && a.iter > 0) {
    const double prev = read_pslot(ctl, (a.iter - 1) & 1, &sh);
    if (prev < a.tol) {  // converged after iteration iter - 1: same decision in every workgroup
      if (blockIdx.x == 0 && tid == 0) {
        ctl->pdone = 1;
        ctl->piters = a.iter;
        ctl->pchange = prev;
      }
      return;
    }
  }
  if (a.colour == 1 && blockIdx.x == 0 && tid < NSUB) ctl->pslot[(a.iter + 1) & 1][tid][0] = 0ull;

  const int half = (a.nr + 1) / 2;
  const int cell = blockIdx.x * PS_THREADS + tid;
  double change = 0.0;
  if (cell < half * a.nz) {
    const int j = cell / half;
    const int i = 2 * (cell % half) + ((j + a.colour) & 1);
    if (i < a.nr) {
      const int nr = a.nr, nz = a.nz;
      const double r_i = ((double)i + 0.5) * a.dr;
      const double z_j = ((double)j + 0.5) * a.dz;
      const double wi = cr_div(1.0, (double)i + 0.5);
      const double aE = ((double)(i + 1) * wi) * a.idr2;
      const double aW = ((double)i * wi) * a.idr2;
      const double aN = a.idz2;
      const double aS = j > 0 ? a.idz2 : 0.0;
      const double* phi = a.phi;
      const double pE = i + 1 < nr ? phi[(size_t)j * nr + i + 1] : roche(a, r_i + a.dr, z_j);
      const double pW = i > 0 ? phi[(size_t)j * nr + i - 1] : 0.0;
      const double pN = j + 1 < nz ? phi[(size_t)(j + 1) * nr + i] : roche(a, r_i, z_j + a.dz);
      const double pS = j > 0 ? phi[(size_t)(j - 1) * nr + i] : 0.0;
      const double diag = ((aE + aW) + aN) + aS;
      const double num = (((aE * pE + aW * pW) + aN * pN) + aS * pS) - a.four_pi_g * a.rho[(size_t)j * nr + i];
      const double gs = cr_div(num, diag);
      const double old = phi[(size_t)j * nr + i];
      const double nw = old + a.omega * (gs - old);
      a.phi[(size_t)j * nr + i] = nw;
      change = nw == old ? 0.0 : cr_div(__builtin_fabs(nw - old), __builtin_fabs(nw));
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) change = __builtin_fmax(change, __shfl_xor(change, off));
  if ((tid & 63) == 0) red[tid / 64] = change;
  __syncthreads();
  if (tid == 0) {
    for (int k = 1; k < PS_THREADS / 64; ++k) change = __builtin_fmax(change, red[k]);
    atomicMax(&ctl->pslot[a.iter & 1][blockIdx.x % NSUB][0], as_bits(change));
  }
}

hipError_t launch_poisson_sweep(const PoissonArgs& a, hipStream_t s) {
  const int half = (a.nr + 1) / 2;
  const int nb = (half * a.nz + PS_THREADS - 1) / PS_THREADS;
  hipLaunchKernelGGL(poisson_sweep_kernel, dim3(nb), dim3(PS_THREADS), 0, s, a);
  return hipGetLastError();
}

// After iterations 0..iter-1: record convergence of iteration iter-1 (if no
// sweep has done so already) and its change.
__global__ void poisson_check_kernel(PoissonArgs a) {
  __shared__ double sh;
  __shared__ int done;
  Ctl* ctl = a.ctl;
  if (threadIdx.x == 0) done = ctl->pdone;
  __syncthreads();
  if (done) return;
  const double prev = read_pslot(ctl, (a.iter - 1) & 1, &sh);
  if (threadIdx.x == 0) {
    ctl->pchange = prev;
    if (prev < a.tol) {
      ctl->pdone = 1;
      ctl->piters = a.iter;
    }
  }
}

hipError_t launch_poisson_check(const PoissonArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(poisson_check_kernel, dim3(1), dim3(64), 0, s, a);
  return hipGetLastError();
}

// g = -grad Phi at the cell centres (central differences; mirror across the
// axis and the plane, Roche values beyond the outer edges).  g: [2][nz][nr].
__global__ __launch_bounds__(PS_THREADS) void gravity_kernel(PoissonArgs a, double* g) {
  const int cell = blockIdx.x * PS_THREADS + threadIdx.x;
  if (cell >= a.nr * a.nz) return;
  const int nr = a.nr, nz = a.nz;
  const int j = cell / nr, i = cell % nr;
  const double* phi = a.phi;
  const double r_i = ((double)i + 0.5) * a.dr;
  const double z_j = ((double)j + 0.5) * a.dz;
  const double pE = i + 1 < nr ? phi[(size_t)j * nr + i + 1] : roche(a, r_i + a.dr, z_j);
  const double pW = i > 0 ? phi[(size_t)j * nr + i - 1] : phi[(size_t)j * nr + i];
  const double pN = j + 1 < nz ? phi[(size_t)(j + 1) * nr + i] : roche(a, r_i, z_j + a.dz);
  const double pS = j > 0 ? phi[(size_t)(j - 1) * nr + i] : phi[(size_t)j * nr + i];
  g[(size_t)j * nr + i] = cr_div(-(pE - pW), 2.0 * a.dr);
  g[(size_t)nr * nz + (size_t)j * nr + i] = cr_div(-(pN - pS), 2.0 * a.dz);
}

hipError_t launch_gravity(const PoissonArgs& a, double* g, hipStream_t s) {
  const int nb = (a.nr * a.nz + PS_THREADS - 1) / PS_THREADS;
  hipLaunchKernelGGL(gravity_kernel, dim3(nb), dim3(PS_THREADS), 0, s, a, g);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Temporally blocked solver.  A launch advances its workgroup's tile by up to K
// iterations without leaving LDS: the tile is loaded with a halo of 2K cells,
// and the red (black) half-sweep h updates the cells of its colour within
// 2K - 1 - h cells of the tile, which are exactly those whose neighbours hold
// correct values after half-sweep h - 1 (each half-sweep consumes one halo
// layer).  The overlapping halos are recomputed by the neighbouring
// workgroups with the same operations, so every tile ends bit-identical to
// the sweep-by-sweep order.  Launches alternate between two buffers (launch l
// reads X[l & 1], writes X[(l + 1) & 1]) and record each iteration's largest
// relative change (owned cells only) in a ring of three banks.
//
// Each launch first examines launch l-1's iterations: if iteration m of them
// is the first below the tolerance, the solve ends there: when m is l-1's last
// iteration its output is the result; otherwise every workgroup recomputes
// m + 1 iterations from l-1's input into l-1's output (the result).  The
// decision depends only on l-1's bank, so all workgroups of a launch take the
// same one, and the launch that ends the solve stamps its index; later
// launches then return at once.
template <int TX, int TY, int K>
__global__ __launch_bounds__(PS_THREADS) void poisson_block_kernel(PoissonArgs a) {
  constexpr int H = 2 * K;
  constexpr int PX = TX + 2 * H, PY = TY + 2 * H;
  __shared__ double PH[PY][PX];
  __shared__ double RH[PY][PX];
  __shared__ double red[PS_THREADS / 64];
  __shared__ double sm[PKMAX];
  __shared__ int s_mode, s_m;
  PoissonCtl* pc = a.pc;
  const int tid = threadIdx.x;
  enum { EXIT = 0, NORMAL = 1, REDO = 2 };

  if (tid < 64) {
    // wavefront 0: the outcome of launch l-1
    int mode = NORMAL, mm = -1;
    if (pc->done_launch < a.l) {
      mode = EXIT;
    } else if (a.kprev > 0) {
      const int b = (a.l + 2) % 3;  // (l - 1) mod 3
      for (int k = 0; k < a.kprev; ++k) {
        double m = as_double(pc->bank[b][k][tid][0]);
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) m = __builtin_fmax(m, __shfl_xor(m, off));
        if (tid == 0) sm[k] = m;
        if (mm < 0 && m < a.tol) mm = k;
      }
      if (mm >= 0) {
        mode = (mm == a.kprev - 1) ? EXIT : REDO;
        if (blockIdx.x == 0 && tid == 0) {
          pc->iters = a.t0 - a.kprev + mm + 1;
          pc->change = sm[mm];
          pc->result = a.l & 1;
          pc->done_launch = a.l;
        }
      } else if (a.kcur == 0) {
        mode = EXIT;
        if (a.final_ && blockIdx.x == 0 && tid == 0) {
          pc->iters = a.t0;
          pc->change = sm[a.kprev - 1];
          pc->result = a.l & 1;
          pc->done_launch = a.l;
        }
      }
    } else if (a.kcur == 0) {
      mode = EXIT;
    }
    if (tid == 0) {
      s_mode = mode;
      s_m = mm;
    }
  }
  __syncthreads();
  const int mode = s_mode;
  if (mode == EXIT) return;
  const bool redo = mode == REDO;
  const int kk = redo ? s_m + 1 : a.kcur;
  const double* in = redo ? a.X[(a.l + 1) & 1] : a.X[a.l & 1];
  double* out = redo ? a.X[a.l & 1] : a.X[(a.l + 1) & 1];
  const int bank = a.l % 3;
  if (!redo && blockIdx.x == 0 && tid < NSUB)
    for (int k = 0; k < PKMAX; ++k) pc->bank[(a.l + 1) % 3][k][tid][0] = 0ull;

  const int nr = a.nr, nz = a.nz;
  const int ntx = (nr + TX - 1) / TX;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int i0 = (tile % ntx) * TX, j0 = (tile / ntx) * TY;
  for (int k = tid; k < PX * PY; k += PS_THREADS) {
    const int ly = k / PX, lx = k % PX;
    const int i = i0 - H + lx, j = j0 - H + ly;
    double p = 0.0, r = 0.0;
    if (i >= 0 && i < nr && j >= 0 && j < nz) {
      p = in[(size_t)j * nr + i];
      r = a.rho[(size_t)j * nr + i];
    }
    PH[ly][lx] = p;
    RH[ly][lx] = r;
  }
  __syncthreads();

  const int ti1 = min(i0 + TX, nr) - 1, tj1 = min(j0 + TY, nz) - 1;  // owned cells (inclusive)
  double change = 0.0;
  for (int h = 0; h < 2 * kk; ++h) {
    const int c = h & 1;
    const int g = 2 * kk - 1 - h;
    const int ia = max(i0 - g, 0), ib = min(ti1 + g, nr - 1);
    const int ja = max(j0 - g, 0), jb = min(tj1 + g, nz - 1);
    const int wmax = ((ib - ia) >> 1) + 1;
    const int ncell = (jb - ja + 1) * wmax;
    for (int t = tid; t < ncell; t += PS_THREADS) {
      const int j = ja + t / wmax;
      const int i = ia + ((c + j + ia) & 1) + 2 * (t % wmax);
      if (i > ib) continue;
      const int lx = i - i0 + H, ly = j - j0 + H;
      const double r_i = ((double)i + 0.5) * a.dr;
      const double z_j = ((double)j + 0.5) * a.dz;
      const double wi = cr_div(1.0, (double)i + 0.5);
      const double aE = ((double)(i + 1) * wi) * a.idr2;
      const double aW = ((double)i * wi) * a.idr2;
      const double aN = a.idz2;
      const double aS = j > 0 ? a.idz2 : 0.0;
      const double pE = i + 1 < nr ? PH[ly][lx + 1] : roche(a, r_i + a.dr, z_j);
      const double pW = i > 0 ? PH[ly][lx - 1] : 0.0;
      const double pN = j + 1 < nz ? PH[ly + 1][lx] : roche(a, r_i, z_j + a.dz);
      const double pS = j > 0 ? PH[ly - 1][lx] : 0.0;
      const double diag = ((aE + aW) + aN) + aS;
      const double num = (((aE * pE + aW * pW) + aN * pN) + aS * pS) - a.four_pi_g * RH[ly][lx];
      const double gs = cr_div(num, diag);
      const double old = PH[ly][lx];
      const double nw = old + a.omega * (gs - old);
      PH[ly][lx] = nw;
      if (i >= i0 && i <= ti1 && j >= j0 && j <= tj1)
        change = __builtin_fmax(change, nw == old ? 0.0 : cr_div(__builtin_fabs(nw - old), __builtin_fabs(nw)));
    }
    __syncthreads();
    if (c == 1 && !redo) {
      // end of iteration h / 2: the tile's largest change into the bank
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) change = __builtin_fmax(change, __shfl_xor(change, off));
      if ((tid & 63) == 0) red[tid / 64] = change;
      __syncthreads();
      if (tid == 0) {
        double m = red[0];
        for (int k = 1; k < PS_THREADS / 64; ++k) m = __builtin_fmax(m, red[k]);
        atomicMax(&pc->bank[bank][h >> 1][blockIdx.x % NSUB][0], as_bits(m));
      }
      change = 0.0;
    }
  }
  for (int k = tid; k < TX * TY; k += PS_THREADS) {
    const int i = i0 + k % TX, j = j0 + k / TX;
    if (i < nr && j < nz) out[(size_t)j * nr + i] = PH[j - j0 + H][i - i0 + H];
  }
}

__global__ void poisson_block_init_kernel(PoissonCtl* pc) {
  const int t = threadIdx.x;
  if (t < NSUB)
    for (int b = 0; b < 3; ++b)
      for (int k = 0; k < PKMAX; ++k) pc->bank[b][k][t][0] = 0ull;
  if (t == 0) {
    pc->done_launch = 0x7fffffff;
    pc->iters = 0;
    pc->result = 0;
    pc->change = 0.0;
  }
}

namespace {
constexpr int BTX = 64, BTY = 32, BK = 4;  // large grids: 80 x 48 cells in LDS (61 KB)
constexpr int STX = 16, STY = 16, SK = 2;  // small grids: 24 x 24 cells in LDS (9 KB)
static_assert(BK <= PKMAX && SK <= PKMAX, "bank depth");
int tiles(int nr, int nz, int tx, int ty) { return ((nr + tx - 1) / tx) * ((nz + ty - 1) / ty); }
}  // namespace

bool poisson_block_big(int nr, int nz) { return tiles(nr, nz, BTX, BTY) >= 256; }
int poisson_block_k(bool big) { return big ? BK : SK; }

hipError_t launch_poisson_block_init(PoissonCtl* pc, hipStream_t s) {
  hipLaunchKernelGGL(poisson_block_init_kernel, dim3(1), dim3(64), 0, s, pc);
  return hipGetLastError();
}

hipError_t launch_poisson_block(const PoissonArgs& a, bool big, hipStream_t s) {
  if (big)
    hipLaunchKernelGGL((poisson_block_kernel<BTX, BTY, BK>), dim3(tiles(a.nr, a.nz, BTX, BTY)),
                       dim3(PS_THREADS), 0, s, a);
  else
    hipLaunchKernelGGL((poisson_block_kernel<STX, STY, SK>), dim3(tiles(a.nr, a.nz, STX, STY)),
                       dim3(PS_THREADS), 0, s, a);
  return hipGetLastError();
}

}  // namespace hy
