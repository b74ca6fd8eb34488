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
//                        its right edge, its upper edge), 16 x 16 corners per
//                        workgroup, one atomic per workgroup with points to
//                        reserve space (the order of the points is not fixed;
//                        nothing downstream depends on it);
//  ls_distance           nearest-point search and blend: 32 x 16 corners per
//                        workgroup, a 16 x 8 quarter per wavefront, two corners
//                        per work item; points streamed through LDS.  The
//                        minimum is taken over squared distances and rooted
//                        once (the square root is monotone and correctly
//                        rounded, so this equals the minimum of the roots).
//                        Every corner starts from its distance to one point
//                        near the tile centre (the nearest among every fourth
//                        point); a point whose distance to the tile's box, then
//                        to the quarter's box, exceeds the largest of those
//                        starting distances over the box's corners (with a
//                        relative margin of 1e-9, far above rounding) is
//                        skipped: it cannot hold the minimum of any of them.
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
  const long long stride = (long long)gridDim.x * LS_THREADS;
  long long k = (long long)blockIdx.x * LS_THREADS + threadIdx.x;
  for (; k + 3 * stride < nc; k += 4 * stride) {  // eight loads in flight
    double u[4], v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      u[q] = vel[k + q * stride];
      v[q] = vel[nc + k + q * stride];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      mu = __builtin_fmax(mu, __builtin_fabs(u[q]));
      mv = __builtin_fmax(mv, __builtin_fabs(v[q]));
    }
  }
  for (; k < nc; k += stride) {
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

// Front points of a 16 x 16 corner tile per workgroup: a prefix sum of the
// counts over the workgroup and one atomic per workgroup that has points.
constexpr int FTX = 16, FTY = 16;
static_assert(FTX * FTY == LS_THREADS, "front tile shape");

__global__ __launch_bounds__(LS_THREADS) void ls_front_kernel(LsArgs a, double* pts) {
  __shared__ int wsum[LS_THREADS / 64];
  __shared__ unsigned long long base;
  const int ntx = (a.mx + FTX - 1) / FTX;
  const int i = (blockIdx.x % ntx) * FTX + (threadIdx.x % FTX);
  const int j = (blockIdx.x / ntx) * FTY + (threadIdx.x / FTX);
  double px[3], py[3];
  int cnt = 0;
  if (i < a.mx && j < a.my) {
    const size_t k = (size_t)j * a.mx + i;
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
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int incl = cnt;  // inclusive prefix sum over the wavefront
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int o = __shfl_up(incl, off);
    if (lane >= off) incl += o;
  }
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  int before = 0, total = 0;
#pragma unroll
  for (int q = 0; q < LS_THREADS / 64; ++q) {
    before += q < w ? wsum[q] : 0;
    total += wsum[q];
  }
  if (threadIdx.x == 0) {
    base = total > 0 ? atomicAdd(&a.lc->npts[a.set], (unsigned long long)total) : 0ull;
    if (blockIdx.x == 0) a.lc->npts[1 - a.set] = 0ull;  // for the next call
  }
  __syncthreads();
  const unsigned long long at = base + (unsigned long long)(before + incl - cnt);
  for (int c = 0; c < cnt; ++c) {
    pts[2 * (at + c)] = px[c];
    pts[2 * (at + c) + 1] = py[c];
  }
}

// Distance and blend.  Corner tile 32 x 16 per workgroup; each wavefront owns a
// 16 x 8 quarter of it, two corners per work item (rows q and q + 4 of the
// quarter, one column).  Points are streamed in chunks: the workgroup keeps
// those a corner of its tile may be nearest to, each wavefront keeps, of
// those, the ones a corner of its quarter may be nearest to, and loops over
// its own list.
constexpr int DTX = 32, DTY = 16, DQX = 16, DQY = 8;
constexpr int DW = LS_THREADS / 64;  // wavefronts per workgroup
constexpr int DCH = 496;             // points per chunk
constexpr int DPT = (DCH + LS_THREADS - 1) / LS_THREADS;  // a work item's points per chunk
constexpr int QCAP = 128;            // a wavefront's list (16 KB of LDS per workgroup in all)
static_assert((DTX / DQX) * (DTY / DQY) == DW && DQX * DQY == 2 * 64 && QCAP >= 64,
              "distance tile shape");

// Max of a non-negative x over the wavefront, in every lane.
__device__ __forceinline__ double wave_max_all(double x) {
  const long long m = __double_as_longlong(wave_max_nonneg(x));
  const unsigned lo = __builtin_amdgcn_readlane((unsigned)m, 63);
  const unsigned hi = __builtin_amdgcn_readlane((unsigned)((unsigned long long)m >> 32), 63);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Squared distance from (qx, qy) to the box [x0, x1] x [y0, y1].
// (With x0 <= x1 at most one of x0 - qx, qx - x1 is positive.)
__device__ __forceinline__ double box_dist2(double qx, double qy, double x0, double x1, double y0, double y1) {
  const double ddx = __builtin_fmax(__builtin_fmax(x0 - qx, qx - x1), 0.0);
  const double ddy = __builtin_fmax(__builtin_fmax(y0 - qy, qy - y1), 0.0);
  return ddx * ddx + ddy * ddy;
}

__global__ __launch_bounds__(LS_THREADS) void ls_distance_kernel(LsArgs a, const double* pts, double* dist) {
  __shared__ double P[2][DCH];      // the tile's candidates of a chunk
  __shared__ double Q[DW][2][QCAP];  // each wavefront's own candidates
  __shared__ double red[3][DW];     // pass 1: each wavefront's nearest point
  __shared__ double ub[DW];         // each quarter's bound
  __shared__ int nkeep[2];          // candidates of the chunk (alternating)
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform in the wavefront
  const int ntx = (a.mx + DTX - 1) / DTX;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int i0 = (tile % ntx) * DTX, j0 = (tile / ntx) * DTY;
  const long long np = (long long)a.lc->npts[a.set];
  if (np == 0) return;  // no front: the field stays as it is
  const double2* pp = reinterpret_cast<const double2*>(pts);  // (x, y) of each point
  const int i1 = min(i0 + DTX, a.mx) - 1, j1 = min(j0 + DTY, a.my) - 1;
  const double tx0 = a.xlo + (double)i0 * a.dx, tx1 = a.xlo + (double)i1 * a.dx;
  const double ty0 = a.ylo + (double)j0 * a.dy, ty1 = a.ylo + (double)j1 * a.dy;

  // pass 1: the point nearest to the tile centre among every 4th point (any
  // point bounds the corners' minima; a sample of the front is close enough)
  {
    const double cx = 0.5 * (tx0 + tx1), cy = 0.5 * (ty0 + ty1);
    double bc = __builtin_inf(), bx = 0.0, by = 0.0;
    for (long long k = (long long)tid * 4; k < np; k += 2 * 4 * LS_THREADS) {
      const double2 p0 = pp[k];
      const double2 p1 = k + 4 * LS_THREADS < np ? pp[k + 4 * LS_THREADS] : p0;
      const double ex = cx - p0.x, ey = cy - p0.y, fx = cx - p1.x, fy = cy - p1.y;
      const double d = ex * ex + ey * ey, e = fx * fx + fy * fy;
      if (d < bc) { bc = d; bx = p0.x; by = p0.y; }
      if (e < bc) { bc = e; bx = p1.x; by = p1.y; }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double od = __shfl_xor(bc, off), ox = __shfl_xor(bx, off), oy = __shfl_xor(by, off);
      if (od < bc) { bc = od; bx = ox; by = oy; }
    }
    if (lane == 0) { red[0][w] = bc; red[1][w] = bx; red[2][w] = by; }
  }
  __syncthreads();
  double px = red[1][0], py = red[2][0];
  {
    double b = red[0][0];
    for (int k = 1; k < DW; ++k)
      if (red[0][k] < b) { b = red[0][k]; px = red[1][k]; py = red[2][k]; }
  }

  // this work item's corners and its wavefront's quarter
  const int qi0 = i0 + (w % (DTX / DQX)) * DQX, qj0 = j0 + (w / (DTX / DQX)) * DQY;
  const int i = qi0 + (lane % DQX);
  const double x = a.xlo + (double)i * a.dx;
  const bool wave_on = qi0 < a.mx && qj0 < a.my;  // the quarter holds a corner of the grid
  const int qi1 = min(qi0 + DQX, a.mx) - 1, qj1 = min(qj0 + DQY, a.my) - 1;
  const double qx0 = a.xlo + (double)qi0 * a.dx, qx1 = a.xlo + (double)qi1 * a.dx;
  const double qy0 = a.ylo + (double)qj0 * a.dy, qy1 = a.ylo + (double)qj1 * a.dy;
  double yv[2], best[2];
  bool on[2];
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int j = qj0 + (lane / DQX) + 4 * r;
    yv[r] = a.ylo + (double)j * a.dy;
    on[r] = i < a.mx && j < a.my;
    // the point found in pass 1 is a candidate of every corner
    const double ex = x - px, ey = yv[r] - py;
    best[r] = ex * ex + ey * ey;
  }
  // Bounds: every corner's minimum is at most its starting distance, so a
  // point whose distance to a box exceeds the largest starting distance of the
  // box's corners (with a relative margin of 1e-9, far above rounding) is
  // nearest to none of them.
  const double qb = wave_max_all(__builtin_fmax(on[0] ? best[0] : 0.0, on[1] ? best[1] : 0.0));
  if (lane == 0) ub[w] = qb;
  if (tid == 0) nkeep[0] = 0;
  __syncthreads();
  double tb = ub[0];
  for (int k = 1; k < DW; ++k) tb = __builtin_fmax(tb, ub[k]);
  tb *= 1.0 + 1e-9;
  const double wb = qb * (1.0 + 1e-9);

  double2 q[DPT];  // this work item's points of the chunk
#pragma unroll
  for (int e = 0; e < DPT; ++e) {
    const int k = tid + e * LS_THREADS;
    q[e] = k < DCH && k < np ? pp[k] : double2{0.0, 0.0};
  }
  // a wavefront's list is run (and emptied) whenever another block of 64
  // candidates might not fit
  auto run_list = [&](int nq) {
    __syncwarp();
#pragma unroll 4
    for (int k = 0; k < nq; ++k) {
      const double ex = x - Q[w][0][k];
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        const double ey = yv[r] - Q[w][1][k];
        best[r] = __builtin_fmin(best[r], ex * ex + ey * ey);
      }
    }
  };
  int c = 0;
  for (long long c0 = 0; c0 < np; c0 += DCH, c ^= 1) {
    const int m = (int)min((long long)DCH, np - c0);
#pragma unroll
    for (int e = 0; e < DPT; ++e) {
      const int k = tid + e * LS_THREADS;
      if (k < m && box_dist2(q[e].x, q[e].y, tx0, tx1, ty0, ty1) <= tb) {
        const int at = atomicAdd(&nkeep[c], 1);
        P[0][at] = q[e].x;
        P[1][at] = q[e].y;
      }
      if (k < DCH && c0 + DCH + k < np) q[e] = pp[c0 + DCH + k];  // next chunk, loaded during this one
    }
    __syncthreads();  // the chunk's candidates are complete
    const int nk = nkeep[c];
    if (tid == 0) nkeep[c ^ 1] = 0;  // last read in the previous chunk
    if (wave_on) {
      int nq = 0;
      for (int k0 = 0; k0 < nk; k0 += 64) {
        if (nq > QCAP - 64) {
          run_list(nq);
          nq = 0;
        }
        const int k = k0 + lane;
        double sx = 0.0, sy = 0.0;
        bool keep = false;
        if (k < nk) {
          sx = P[0][k];
          sy = P[1][k];
          keep = box_dist2(sx, sy, qx0, qx1, qy0, qy1) <= wb;
        }
        const unsigned long long bal = __ballot(keep);
        if (keep) {
          const int at = nq + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(bal >> 32),
                                                             __builtin_amdgcn_mbcnt_lo((unsigned)bal, 0u));
          Q[w][0][at] = sx;
          Q[w][1][at] = sy;
        }
        nq += __popcll(bal);
      }
      run_list(nq);
    }
    __syncthreads();  // the chunk's candidates are consumed
  }
  const double D = a.dx < a.dy ? a.dx : a.dy;
  const double wd = D / 3.0, d0 = 3.0 * D;
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    if (!on[r]) continue;
    const int j = qj0 + (lane / DQX) + 4 * r;
    const size_t kc = (size_t)j * a.mx + i;
    const double d = cr_sqrt(best[r]);
    const double s = a.W[kc];
    const double t = (d - d0) / wd;
    // tanh(t) rounds to 1 from t = 22 on (1 - tanh(22) is about 1.6e-19), where
    // the blend weight is 0
    const double h = t < 22.0 ? (1.0 - tanh(t)) / (1.0 - tanh(-d0 / wd)) : 0.0;
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
  const unsigned nb = (unsigned)(((a.mx + FTX - 1) / FTX) * ((a.my + FTY - 1) / FTY));
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
