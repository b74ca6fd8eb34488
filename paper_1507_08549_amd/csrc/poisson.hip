// poisson.hip -- the gravitational potential of Sect. 2.1: the Poisson
// equation (1/r) d/dr (r dPhi/dr) + d^2Phi/dz^2 = 4 pi G rho in (r, z), solved by
// successive over-relaxation of Gauss-Seidel sweeps until the relative change
// of every cell is below a tolerance; reflecting axis (r = 0) and symmetry
// plane (z = 0), Roche values -G M / sqrt(r^2 + z^2) beyond the outer edges.
//
// Cell-centred five-point stencil, r-operator in flux form (face radii i dr and
// (i+1) dr, so the axis face has zero weight), mirror at z = 0, Roche values at
// the outer ghost centres.  Red-black order (colour (i + j) mod 2, red first)
// makes each colour's updates independent of each other.  The Gauss-Seidel
// value is the weighted neighbour sum minus 4 pi G rho times the reciprocal
// of the diagonal weight.  Every formula has the CPU oracle's evaluation order
// (FP64, built with -ffp-contract=off, correctly rounded divisions and roots),
// so the potential and the iteration count agree bit for bit.
#include "stage_kernel.hpp"

namespace hy {

constexpr int PS_THREADS = 256;

__device__ __forceinline__ double roche(const PoissonArgs& a, double r, double z) {
  return cr_div(-(a.G * a.mass), cr_sqrt(r * r + z * z));
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
// iterations without leaving LDS (each colour stored contiguously, so a
// half-sweep reads and writes LDS at unit stride; the r-operator weights once
// per column; Roche values in the ring beyond the outer edges): the tile is loaded with a halo of 2K cells,
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
template <int TX, int TY, int K, int NT>
__global__ __launch_bounds__(NT) void poisson_block_kernel(PoissonArgs a) {
  constexpr int H = 2 * K;
  constexpr int PX = TX + 2 * H, PY = TY + 2 * H;
  constexpr int HX = PX / 2;
  static_assert(PX % 2 == 0 && TX % 2 == 0 && TY % 2 == 0, "colour layout needs even tiles");
  // potential and density by colour: cell (lx, ly) of the tile has colour
  // (lx + ly) & 1 (tile origins are even) and sits at [colour][ly][lx / 2]
  __shared__ double PC[2][PY][HX];
  __shared__ double RC[2][PY][HX];
  __shared__ double cAE[PX], cAW[PX];  // r-operator weights of each column
  __shared__ double cID[2][PX];        // 1 / diagonal weight: row 0 (no south weight), other rows
  __shared__ double red[NT / 64];
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
  // Load.  Beyond the grid, the ring the stencil reaches holds what the
  // update takes there: the Roche value past the outer edges (the oracle's
  // formula at the ghost centre), 0 past the axis and the plane (whose
  // weights are 0).
  for (int k = tid; k < PX * PY; k += NT) {
    const int ly = k / PX, lx = k % PX;
    const int i = i0 - H + lx, j = j0 - H + ly;
    const bool iin = i >= 0 && i < nr, jin = j >= 0 && j < nz;
    double p = 0.0, r = 0.0;
    if (iin && jin) {
      p = in[(size_t)j * nr + i];
      r = a.rho[(size_t)j * nr + i];
    } else if (i == nr && jin) {
      p = roche(a, ((double)(nr - 1) + 0.5) * a.dr + a.dr, ((double)j + 0.5) * a.dz);
    } else if (j == nz && iin) {
      p = roche(a, ((double)i + 0.5) * a.dr, ((double)(nz - 1) + 0.5) * a.dz + a.dz);
    }
    const int c = (lx + ly) & 1;
    PC[c][ly][lx >> 1] = p;
    RC[c][ly][lx >> 1] = r;
  }
  for (int lx = tid; lx < PX; lx += NT) {
    const int i = i0 - H + lx;
    double e = 0.0, w = 0.0, d0 = 0.0, d1 = 0.0;
    if (i >= 0 && i < nr) {
      const double wi = cr_div(1.0, (double)i + 0.5);
      e = ((double)(i + 1) * wi) * a.idr2;  // r_{i+1/2} / (r_i dr^2)
      w = ((double)i * wi) * a.idr2;        // r_{i-1/2} / (r_i dr^2)
      d0 = cr_div(1.0, ((e + w) + a.idz2) + 0.0);
      d1 = cr_div(1.0, ((e + w) + a.idz2) + a.idz2);
    }
    cAE[lx] = e;
    cAW[lx] = w;
    cID[0][lx] = d0;
    cID[1][lx] = d1;
  }
  __syncthreads();

  const int ti1 = min(i0 + TX, nr) - 1, tj1 = min(j0 + TY, nz) - 1;  // owned cells (inclusive)
  const int ox = i0 - H, oy = j0 - H;  // tile origin of the LDS arrays
  double change = 0.0;
  for (int h = 0; h < 2 * kk; ++h) {
    const int c = h & 1;
    const int g = 2 * kk - 1 - h;
    const int lxa = max(i0 - g, 0) - ox, lxb = min(ti1 + g, nr - 1) - ox;
    const int lya = max(j0 - g, 0) - oy, lyb = min(tj1 + g, nz - 1) - oy;
    const double(*Q)[HX] = PC[1 - c];
    // the (row, colour slot) pairs of the active rows, dealt to the work items
    // in order (the cells of one colour are independent of each other)
    const int nslot = (lyb - lya + 1) * HX;
    for (int idx = tid; idx < nslot; idx += NT) {
      const int ry = idx / HX, m = idx - ry * HX;
      const int ly = lya + ry;
      const int o = (c + ly) & 1;  // cells of colour c in this row: lx = 2m + o
      if (2 * m + o < lxa || 2 * m + o > lxb) continue;
      const int j = oy + ly;
      const double aS = j > 0 ? a.idz2 : 0.0;
      const int lx = 2 * m + o;
      const double aE = cAE[lx], aW = cAW[lx], aN = a.idz2;
      const double pE = Q[ly][m + o], pW = Q[ly][m + o - 1];
      const double pN = Q[ly + 1][m], pS = Q[ly - 1][m];
      const double num = (((aE * pE + aW * pW) + aN * pN) + aS * pS) - a.four_pi_g * RC[c][ly][m];
      const double gs = num * cID[j > 0 ? 1 : 0][lx];
      const double old = PC[c][ly][m];
      const double nw = old + a.omega * (gs - old);
      PC[c][ly][m] = nw;
      const int i = ox + lx;
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
        double mx = red[0];
        for (int k = 1; k < NT / 64; ++k) mx = __builtin_fmax(mx, red[k]);
        atomicMax(&pc->bank[bank][h >> 1][blockIdx.x % NSUB][0], as_bits(mx));
      }
      change = 0.0;
    }
  }
  for (int k = tid; k < TX * TY; k += NT) {
    const int i = i0 + k % TX, j = j0 + k / TX;
    if (i < nr && j < nz) {
      const int lx = i - ox, ly = j - oy;
      out[(size_t)j * nr + i] = PC[(lx + ly) & 1][ly][lx >> 1];
    }
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
constexpr int BTX = 128, BTY = 32, BK = 4, BNT = 1024;  // large grids: 144 x 48 cells in LDS (115 KB)
constexpr int MTX = 32, MTY = 32, MK = 4, MNT = 256;    // mid-size grids: 48 x 48 cells in LDS (39 KB)
constexpr int STX = 16, STY = 16, SK = 2, SNT = 256;  // small grids: 24 x 24 cells in LDS (9 KB)
static_assert(BK <= PKMAX && MK <= PKMAX && SK <= PKMAX, "bank depth");
int tiles(int nr, int nz, int tx, int ty) { return ((nr + tx - 1) / tx) * ((nz + ty - 1) / ty); }
}  // namespace

// The largest tile shape that still gives every compute unit a workgroup.
int poisson_block_config(int nr, int nz) {
  if (tiles(nr, nz, BTX, BTY) >= 256) return 2;
  if (tiles(nr, nz, MTX, MTY) >= 256) return 1;
  return 0;
}
int poisson_block_k(int config) { return config == 2 ? BK : (config == 1 ? MK : SK); }

hipError_t launch_poisson_block_init(PoissonCtl* pc, hipStream_t s) {
  hipLaunchKernelGGL(poisson_block_init_kernel, dim3(1), dim3(64), 0, s, pc);
  return hipGetLastError();
}

hipError_t launch_poisson_block(const PoissonArgs& a, int config, hipStream_t s) {
  if (config == 2)
    hipLaunchKernelGGL((poisson_block_kernel<BTX, BTY, BK, BNT>), dim3(tiles(a.nr, a.nz, BTX, BTY)),
                       dim3(BNT), 0, s, a);
  else if (config == 1)
    hipLaunchKernelGGL((poisson_block_kernel<MTX, MTY, MK, MNT>), dim3(tiles(a.nr, a.nz, MTX, MTY)),
                       dim3(MNT), 0, s, a);
  else
    hipLaunchKernelGGL((poisson_block_kernel<STX, STY, SK, SNT>), dim3(tiles(a.nr, a.nz, STX, STY)),
                       dim3(SNT), 0, s, a);
  return hipGetLastError();
}

}  // namespace hy
