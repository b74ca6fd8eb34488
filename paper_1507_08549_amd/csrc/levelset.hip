// levelset.hip -- the level-set flame front of Sect. 2.3 on the grid corners.
//
// (1) Advection: dS/dt = -(v + v_flame) . grad S with v_flame = s_f along the
//     outward normal of the burnt region (-grad S / |grad S|), i.e. the
//     Hamilton-Jacobi equation S_t + H(S_x, S_y) = 0, H(p, q) = u p + v q -
//     s_f |(p, q)|, discretised with the WENO5-JS reconstruction of the fluid
//     (same weights, epsilon and evaluation order) applied to the one-sided
//     differences, a global Lax-Friedrichs flux with speeds max|u| + s_f and
//     max|v| + s_f, and the fluid's SSP-RK3 stages.
// (2) Re-distancing: front points where neighbouring corners change sign
//     (linear interpolation) or a corner is zero; each corner's distance d to
//     the nearest point; S <- H(d) S + (1 - H(d)) sign(S) d with
//     H(d) = (1 - tanh((d - 3D) / (D/3))) / (1 - tanh(-9)), D the spacing.
//
// Corner (i, j), i = 0..nx, j = 0..ny, sits at (xlo + i dx, ylo + j dy); fields
// are [ny+1][nx+1].  Ghost corners: periodic (corner nx is corner 0: it is read
// as corner 0 and computed as corner 0), reflecting (mirror about the wall
// corner), transmissive (linear extrapolation 2 S_0 - S_k).  Every FP64 formula
// has the CPU oracle's evaluation order (built with -ffp-contract=off), so the
// advected field and the distances agree bit for bit; the blend goes through
// tanh, whose last bits depend on the math library.
//
// Kernels:
//  ls_alpha              max|u|, max|v| of the corner velocity into 64
//                        sub-slots (bit patterns of non-negative doubles order
//                        like the values, so atomicMax on them is exact) of the
//                        step's set, clearing the other set for the next step;
//  ls_stage              one RK stage: 32 x 16 corner tile with a 3-corner
//                        halo in LDS (read without the ghost rule where the
//                        halo lies inside the grid), the one-sided differences
//                        (times 1/spacing) once per edge in LDS, four
//                        reconstructions per corner;
//  ls_front              front points, one work item per corner (its zero test,
//                        its right edge, its upper edge), one atomic per
//                        wavefront to reserve space (the order of the points is
//                        not fixed; nothing downstream depends on it);
//  ls_distance           nearest-point search and blend: 32 x 16 corners per
//                        workgroup, two per work item; points streamed through
//                        LDS.  The minimum is taken over squared distances and
//                        rooted once (the square root is monotone and correctly
//                        rounded, so this equals the minimum of the roots).
//                        A workgroup first bounds the distance of all its
//                        corners (nearest point to the tile centre plus the
//                        half diagonal) and skips every point whose distance to
//                        the tile's box exceeds that bound with a relative
//                        margin of 1e-9, far above rounding, so the skipped
//                        points can never hold the minimum.
#include "stage_kernel.hpp"

namespace hy {

namespace {

constexpr int LTX = 32, LTY = 16;  // stage tile (corners)
constexpr int LST_THREADS = LTX * LTY;  // stage kernel: one work item per corner
constexpr int LS_THREADS = 256;

// Corner index along one axis with the ghost rule; returns the corner to read
// and, for linear extrapolation, the edge corner (edge >= 0) so the value is
// 2 S(edge) - S(idx).
__device__ __forceinline__ int ls_map(int gi, int n, int blo, int bhi, int& edge) {
  edge = -1;
  if (gi < 0) {
    if (blo == 0) return gi + n;
    if (blo == 2) return -gi;
    edge = 0;
    return -gi;
  }
  if (gi > n) {
    if (bhi == 0) return gi - n;
    if (bhi == 2) return 2 * n - gi;
    edge = n;
    return 2 * n - gi;
  }
  if (gi == n && bhi == 0) return 0;  // periodic image
  return gi;
}

__device__ __forceinline__ void read_amax(const LsCtl* lc, int set, double* sh, double& mu, double& mv) {
  if (threadIdx.x < NSUB) {
    double a = as_double(lc->amax[set][threadIdx.x][0]), b = as_double(lc->amax[set][threadIdx.x][1]);
#pragma unroll
    for (int off = NSUB / 2; off > 0; off >>= 1) {
      a = __builtin_fmax(a, __shfl_xor(a, off));
      b = __builtin_fmax(b, __shfl_xor(b, off));
    }
    if (threadIdx.x == 0) {
      sh[0] = a;
      sh[1] = b;
    }
  }
  __syncthreads();
  mu = sh[0];
  mv = sh[1];
}

// WENO5-JS of the fluid (same weights and order) at the right face of v2; the
// denominator is a sum of positive weights, at least 60 eps^4, so the
// normal-denominator division gives the correctly rounded quotient.
__device__ __forceinline__ double ls_weno5(double v0, double v1, double v2, double v3, double v4, double eps) {
  double num, den;
  weno5_nd(v0, v1, v2, v3, v4, eps, num, den);
  return cr_div_pos_normal(num, den);
}

}  // namespace

__global__ void ls_init_kernel(LsCtl* lc) {
  const int t = threadIdx.x;
  if (t < NSUB) {
    for (int set = 0; set < 2; ++set) {
      lc->amax[set][t][0] = 0ull;
      lc->amax[set][t][1] = 0ull;
    }
  }
  if (t < 2) lc->npts[t] = 0ull;
}

// max |u|, max |v| into the sub-slots of set `set`; the first workgroup clears
// the other set's sub-slots for the next step.
__global__ __launch_bounds__(LS_THREADS) void ls_alpha_kernel(const double* vel, long long nc, LsCtl* lc,
                                                              int set) {
  if (blockIdx.x == 0 && threadIdx.x < NSUB) {
    lc->amax[1 - set][threadIdx.x][0] = 0ull;
    lc->amax[1 - set][threadIdx.x][1] = 0ull;
  }
  __shared__ double red[2][LS_THREADS / 64];
  double mu = 0.0, mv = 0.0;
  for (long long k = (long long)blockIdx.x * LS_THREADS + threadIdx.x; k < nc;
       k += (long long)gridDim.x * LS_THREADS) {
    mu = __builtin_fmax(mu, __builtin_fabs(vel[k]));
    mv = __builtin_fmax(mv, __builtin_fabs(vel[nc + k]));
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    mu = __builtin_fmax(mu, __shfl_xor(mu, off));
    mv = __builtin_fmax(mv, __shfl_xor(mv, off));
  }
  const int w = threadIdx.x / 64;
  if ((threadIdx.x & 63) == 0) {
    red[0][w] = mu;
    red[1][w] = mv;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < LS_THREADS / 64; ++k) {
      mu = __builtin_fmax(mu, red[0][k]);
      mv = __builtin_fmax(mv, red[1][k]);
    }
    atomicMax(&lc->amax[set][blockIdx.x % NSUB][0], as_bits(mu));
    atomicMax(&lc->amax[set][blockIdx.x % NSUB][1], as_bits(mv));
  }
}

__global__ __launch_bounds__(LST_THREADS) void ls_stage_kernel(LsArgs a) {
  constexpr int PX = LTX + 6, PY = LTY + 6;
  __shared__ double T[PY][PX];
  __shared__ double QX[LTY][LTX + 5];
  __shared__ double QY[LTY + 5][LTX];
  __shared__ double sh[2];
  const int tid = threadIdx.x;
  const int ntx = (a.mx + LTX - 1) / LTX;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int i0 = (tile % ntx) * LTX, j0 = (tile / ntx) * LTY;
  const int nx = a.mx - 1, ny = a.my - 1;

  // tile of S with a 3-corner halo; only the x halo of interior rows and the y
  // halo of interior columns are used.  A tile whose halo lies inside the
  // grid (and off a periodic image row or column) reads every corner as
  // itself.
  const bool interior = i0 >= 3 && j0 >= 3 && i0 + LTX + 2 <= nx - (a.bc[1] == 0 ? 1 : 0) &&
                        j0 + LTY + 2 <= ny - (a.bc[3] == 0 ? 1 : 0);
  if (interior) {
    const double* V = a.V + ((size_t)(j0 - 3) * a.mx + (i0 - 3));
    for (int k = tid; k < PX * PY; k += LST_THREADS) {
      const int ly = k / PX, lx = k - ly * PX;
      T[ly][lx] = V[(size_t)ly * a.mx + lx];
    }
  } else {
    for (int k = tid; k < PX * PY; k += LST_THREADS) {
      const int ly = k / PX, lx = k % PX;
      const int gi = i0 - 3 + lx, gj = j0 - 3 + ly;
      const bool xin = gi >= 0 && gi <= nx, yin = gj >= 0 && gj <= ny;
      double v = 0.0;
      if (gi >= -3 && gi <= nx + 3 && gj >= -3 && gj <= ny + 3 && (xin || yin)) {
        int ex, ey;
        const int ci = ls_map(gi, nx, a.bc[0], a.bc[1], ex);
        const int cj = ls_map(gj, ny, a.bc[2], a.bc[3], ey);
        const double* V = a.V;
        if (ex >= 0 && yin) {
          const int cjj = ls_map(gj, ny, a.bc[2], a.bc[3], ey);
          v = 2.0 * V[(size_t)cjj * a.mx + ex] - V[(size_t)cjj * a.mx + ci];
        } else if (ey >= 0 && xin) {
          v = 2.0 * V[(size_t)ey * a.mx + ci] - V[(size_t)cj * a.mx + ci];
        } else if (ex < 0 && ey < 0) {
          v = V[(size_t)cj * a.mx + ci];
        }
      }
      T[ly][lx] = v;
    }
  }
  __syncthreads();
  for (int k = tid; k < LTY * (LTX + 5); k += LST_THREADS) {
    const int r = k / (LTX + 5), e = k % (LTX + 5);
    QX[r][e] = (T[r + 3][e + 1] - T[r + 3][e]) * a.idx;
  }
  for (int k = tid; k < (LTY + 5) * LTX; k += LST_THREADS) {
    const int e = k / LTX, c = k % LTX;
    QY[e][c] = (T[e + 1][c + 3] - T[e][c + 3]) * a.idy;
  }
  double mu, mv;
  read_amax(a.lc, a.set, sh, mu, mv);  // contains a barrier
  const double ax = mu + a.s_f, ay = mv + a.s_f;

  const int tx = tid % LTX, ty = tid / LTX;
  const int i = i0 + tx, j = j0 + ty;
  if (i > nx || j > ny) return;
  const double* qx = &QX[ty][tx];
  const double pm = ls_weno5(qx[0], qx[1], qx[2], qx[3], qx[4], a.eps);
  const double pp = ls_weno5(qx[5], qx[4], qx[3], qx[2], qx[1], a.eps);
  const double qm = ls_weno5(QY[ty][tx], QY[ty + 1][tx], QY[ty + 2][tx], QY[ty + 3][tx], QY[ty + 4][tx], a.eps);
  const double qp = ls_weno5(QY[ty + 5][tx], QY[ty + 4][tx], QY[ty + 3][tx], QY[ty + 2][tx], QY[ty + 1][tx], a.eps);
  // a periodic image corner is computed as corner 0 (same stencil, same
  // velocity and stage input; the step input holds the images already, see
  // ls_images_kernel, so its own S0 is corner 0's and W may alias S0)
  const int si = (i == nx && a.bc[1] == 0) ? 0 : i;
  const int sj = (j == ny && a.bc[3] == 0) ? 0 : j;
  const size_t kc = (size_t)sj * a.mx + si;
  const size_t ko = (size_t)j * a.mx + i;
  const size_t nc = (size_t)a.mx * a.my;
  const double p = 0.5 * (pm + pp), q = 0.5 * (qm + qp);
  const double u = a.vel[kc], v = a.vel[nc + kc];
  const double grad = cr_sqrt(p * p + q * q);
  const double H = (u * p + v * q) - a.s_f * grad;
  const double Hhat = (H - ax * (0.5 * (pp - pm))) - ay * (0.5 * (qp - qm));
  const double L = -Hhat;
  const double s0 = a.S0[ko];
  const double inc = (a.V[kc] - s0) + a.dt * L;
  a.W[ko] = s0 + a.b * inc;
}

// Periodic images before a step: corner nx of every row takes corner 0's value
// (periodic in x), corner ny of every column corner 0's (periodic in y), as if
// the x images were written first.  Sources are never targets.
__global__ __launch_bounds__(LS_THREADS) void ls_images_kernel(LsArgs a, double* S) {
  const int k = blockIdx.x * LS_THREADS + threadIdx.x;
  const int nx = a.mx - 1, ny = a.my - 1;
  const bool xp = a.bc[1] == 0, yp = a.bc[3] == 0;
  int i, j;
  if (k < a.my) {
    i = nx;
    j = k;
  } else if (k < a.my + nx) {
    i = k - a.my;
    j = ny;
  } else {
    return;
  }
  const int si = (xp && i == nx) ? 0 : i;
  const int sj = (yp && j == ny) ? 0 : j;
  if (si != i || sj != j) S[(size_t)j * a.mx + i] = S[(size_t)sj * a.mx + si];
}

__global__ __launch_bounds__(LS_THREADS) void ls_front_kernel(LsArgs a, double* pts) {
  const long long nc = (long long)a.mx * a.my;
  const long long k = (long long)blockIdx.x * LS_THREADS + threadIdx.x;
  double px[3], py[3];
  int cnt = 0;
  if (k < nc) {
    const int j = (int)(k / a.mx), i = (int)(k % a.mx);
    const double* S = a.V;
    const double s = S[k];
    const double x = a.xlo + (double)i * a.dx, y = a.ylo + (double)j * a.dy;
    if (s == 0.0) {
      px[cnt] = x;
      py[cnt] = y;
      ++cnt;
    }
    if (i + 1 < a.mx) {
      const double b = S[k + 1];
      if ((s < 0.0 && b > 0.0) || (s > 0.0 && b < 0.0)) {
        px[cnt] = x + a.dx * cr_div(s, s - b);
        py[cnt] = y;
        ++cnt;
      }
    }
    if (j + 1 < a.my) {
      const double b = S[k + a.mx];
      if ((s < 0.0 && b > 0.0) || (s > 0.0 && b < 0.0)) {
        px[cnt] = x;
        py[cnt] = y + a.dy * cr_div(s, s - b);
        ++cnt;
      }
    }
  }
  // wavefront prefix sum of the counts, one atomic per wavefront
  const int lane = threadIdx.x & 63;
  int incl = cnt;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int o = __shfl_up(incl, off);
    if (lane >= off) incl += o;
  }
  const int total = __shfl(incl, 63);
  unsigned long long base = 0;
  if (lane == 63 && total > 0) base = atomicAdd(&a.lc->npts[a.set], (unsigned long long)total);
  if (blockIdx.x == 0 && threadIdx.x == 0) a.lc->npts[1 - a.set] = 0ull;  // for the next call
  base = __shfl(base, 63);
  const unsigned long long at = base + (unsigned long long)(incl - cnt);
  for (int c = 0; c < cnt; ++c) {
    pts[2 * (at + c)] = px[c];
    pts[2 * (at + c) + 1] = py[c];
  }
}

// Distance and blend.  Corner tile 32 x 16 (two corners per work item, rows
// ty and ty + 8); points staged through LDS in chunks.
constexpr int DTX = 32, DTY = 16, DCH = 512;
constexpr int DRS = LS_THREADS / DTX;  // row stride of a work item's corners
constexpr int DR = DTY / DRS;          // corners per work item
static_assert(DR * DRS == DTY && LS_THREADS % DTX == 0, "distance tile shape");

__global__ __launch_bounds__(LS_THREADS) void ls_distance_kernel(LsArgs a, const double* pts, double* dist) {
  __shared__ double P[2][DCH];
  __shared__ int nkeep;
  __shared__ double red[LS_THREADS / 64];
  const int tid = threadIdx.x;
  const int ntx = (a.mx + DTX - 1) / DTX;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int i0 = (tile % ntx) * DTX, j0 = (tile / ntx) * DTY;
  const long long np = (long long)a.lc->npts[a.set];
  if (np == 0) return;  // no front: the field stays as it is
  const int i1 = min(i0 + DTX, a.mx) - 1, j1 = min(j0 + DTY, a.my) - 1;
  // tile box and centre
  const double bx0 = a.xlo + (double)i0 * a.dx, bx1 = a.xlo + (double)i1 * a.dx;
  const double by0 = a.ylo + (double)j0 * a.dy, by1 = a.ylo + (double)j1 * a.dy;
  const double cx = 0.5 * (bx0 + bx1), cy = 0.5 * (by0 + by1);
  const double hx = 0.5 * (bx1 - bx0), hy = 0.5 * (by1 - by0);
  const double half_diag = __builtin_sqrt(hx * hx + hy * hy);

  // pass 1: nearest point to the tile centre
  double best_c = __builtin_inf();
  for (long long k = tid; k < np; k += LS_THREADS) {
    const double ex = cx - pts[2 * k], ey = cy - pts[2 * k + 1];
    best_c = __builtin_fmin(best_c, ex * ex + ey * ey);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) best_c = __builtin_fmin(best_c, __shfl_xor(best_c, off));
  if ((tid & 63) == 0) red[tid / 64] = best_c;
  __syncthreads();
  best_c = red[0];
  for (int k = 1; k < LS_THREADS / 64; ++k) best_c = __builtin_fmin(best_c, red[k]);
  // every corner of the tile is within (|centre - p*| + half diagonal) of a point
  const double ub = __builtin_sqrt(best_c) + half_diag;
  const double ub2 = (ub * ub) * (1.0 + 1e-9);

  const int tx = tid % DTX, ty = tid / DTX;
  const int i = i0 + tx;
  const double x = a.xlo + (double)i * a.dx;
  double yv[DR], best[DR];
#pragma unroll
  for (int r = 0; r < DR; ++r) {
    yv[r] = a.ylo + (double)(j0 + ty + DRS * r) * a.dy;
    best[r] = __builtin_inf();
  }
  for (long long c0 = 0; c0 < np; c0 += DCH) {
    const int m = (int)min((long long)DCH, np - c0);
    __syncthreads();  // previous chunk consumed
    if (tid == 0) nkeep = 0;
    __syncthreads();
    for (int k = tid; k < m; k += LS_THREADS) {
      const double qx = pts[2 * (c0 + k)], qy = pts[2 * (c0 + k) + 1];
      // squared distance from the point to the tile's box
      const double ddx = qx < bx0 ? bx0 - qx : (qx > bx1 ? qx - bx1 : 0.0);
      const double ddy = qy < by0 ? by0 - qy : (qy > by1 ? qy - by1 : 0.0);
      if (ddx * ddx + ddy * ddy <= ub2) {
        const int at = atomicAdd(&nkeep, 1);
        P[0][at] = qx;
        P[1][at] = qy;
      }
    }
    __syncthreads();
    const int nk = nkeep;
    for (int k = 0; k < nk; ++k) {
      const double ex = x - P[0][k];
#pragma unroll
      for (int r = 0; r < DR; ++r) {
        const double ey = yv[r] - P[1][k];
        best[r] = __builtin_fmin(best[r], ex * ex + ey * ey);
      }
    }
  }
  if (i >= a.mx) return;
  const double D = a.dx < a.dy ? a.dx : a.dy;
  const double w = D / 3.0, d0 = 3.0 * D;
  const double den = 1.0 - tanh(-d0 / w);
#pragma unroll
  for (int r = 0; r < DR; ++r) {
    const int j = j0 + ty + DRS * r;
    if (j >= a.my) continue;
    const size_t kc = (size_t)j * a.mx + i;
    const double d = cr_sqrt(best[r]);
    const double s = a.W[kc];
    const double h = (1.0 - tanh((d - d0) / w)) / den;
    const double sd = s < 0.0 ? -d : d;
    a.W[kc] = h * s + (1.0 - h) * sd;
    if (dist) dist[kc] = d;
  }
}

__global__ __launch_bounds__(LS_THREADS) void ls_velocity_kernel(LsArgs a, const double* U) {
  const long long nc = (long long)a.mx * a.my;
  const long long k = (long long)blockIdx.x * LS_THREADS + threadIdx.x;
  if (k >= nc) return;
  const int j = (int)(k / a.mx), i = (int)(k % a.mx);
  const int nx = a.mx - 1, ny = a.my - 1;
  const size_t n = (size_t)nx * (size_t)ny;
  double uu[4], vv[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    int ci = i - 1 + (c & 1), cj = j - 1 + (c >> 1);
    double su = 1.0, sv = 1.0;
    if (ci < 0) {
      if (a.bc[0] == 0) ci += nx;
      else if (a.bc[0] == 2) { ci = -1 - ci; su = -1.0; }
      else ci = 0;
    } else if (ci >= nx) {
      if (a.bc[1] == 0) ci -= nx;
      else if (a.bc[1] == 2) { ci = 2 * nx - 1 - ci; su = -1.0; }
      else ci = nx - 1;
    }
    if (cj < 0) {
      if (a.bc[2] == 0) cj += ny;
      else if (a.bc[2] == 2) { cj = -1 - cj; sv = -1.0; }
      else cj = 0;
    } else if (cj >= ny) {
      if (a.bc[3] == 0) cj -= ny;
      else if (a.bc[3] == 2) { cj = 2 * ny - 1 - cj; sv = -1.0; }
      else cj = ny - 1;
    }
    const size_t kk = (size_t)cj * nx + ci;
    const double rho = U[kk];
    uu[c] = su * cr_div(U[n + kk], rho);
    vv[c] = sv * cr_div(U[2 * n + kk], rho);
  }
  double* vel = a.W;
  vel[k] = 0.25 * ((uu[0] + uu[1]) + (uu[2] + uu[3]));
  vel[nc + k] = 0.25 * ((vv[0] + vv[1]) + (vv[2] + vv[3]));
}

hipError_t launch_ls_init(LsCtl* lc, hipStream_t s) {
  hipLaunchKernelGGL(ls_init_kernel, dim3(1), dim3(64), 0, s, lc);
  return hipGetLastError();
}

hipError_t launch_ls_alpha(const LsArgs& a, hipStream_t s) {
  const long long nc = (long long)a.mx * a.my;
  long long nb = (nc + LS_THREADS - 1) / LS_THREADS;
  if (nb > 1024) nb = 1024;
  hipLaunchKernelGGL(ls_alpha_kernel, dim3((unsigned)nb), dim3(LS_THREADS), 0, s, a.vel, nc, a.lc, a.set);
  return hipGetLastError();
}

hipError_t launch_ls_images(const LsArgs& a, double* S, hipStream_t s) {
  if (a.bc[1] != 0 && a.bc[3] != 0) return hipSuccess;
  const int n = a.my + a.mx - 1;
  hipLaunchKernelGGL(ls_images_kernel, dim3((n + LS_THREADS - 1) / LS_THREADS), dim3(LS_THREADS), 0, s, a, S);
  return hipGetLastError();
}

hipError_t launch_ls_stage(const LsArgs& a, hipStream_t s) {
  const int nb = ((a.mx + LTX - 1) / LTX) * ((a.my + LTY - 1) / LTY);
  hipLaunchKernelGGL(ls_stage_kernel, dim3(nb), dim3(LST_THREADS), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_ls_front(const LsArgs& a, double* pts, hipStream_t s) {
  const long long nc = (long long)a.mx * a.my;
  const unsigned nb = (unsigned)((nc + LS_THREADS - 1) / LS_THREADS);
  hipLaunchKernelGGL(ls_front_kernel, dim3(nb), dim3(LS_THREADS), 0, s, a, pts);
  return hipGetLastError();
}

hipError_t launch_ls_distance(const LsArgs& a, const double* pts, double* dist, hipStream_t s) {
  const int nb = ((a.mx + DTX - 1) / DTX) * ((a.my + DTY - 1) / DTY);
  hipLaunchKernelGGL(ls_distance_kernel, dim3(nb), dim3(LS_THREADS), 0, s, a, pts, dist);
  return hipGetLastError();
}

hipError_t launch_ls_velocity(const LsArgs& a, const double* U, hipStream_t s) {
  const long long nc = (long long)a.mx * a.my;
  const unsigned nb = (unsigned)((nc + LS_THREADS - 1) / LS_THREADS);
  hipLaunchKernelGGL(ls_velocity_kernel, dim3(nb), dim3(LS_THREADS), 0, s, a, U);
  return hipGetLastError();
}

}  // namespace hy
