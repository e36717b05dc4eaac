// Jacobi-preconditioned CG for one or several corrector systems (gfx950).
//
// Work is cut into tiles of consecutive rows of one system; one block of
// threads owns a tile.  One kernel per iteration:
//   k_iter    every block reduces its system's partials of the last product
//             in a fixed order (identical result in every block), forms alpha
//             and beta (recurrence for the next rho, anchored on the exact
//             rho), updates x_acc, z and p of its rows, and applies A to the
//             new p at once: the new p of a neighbour row is recomputed from
//             that row's old p, z and q~ with the same operations its owner
//             uses, so no grid-wide wait separates the update from the
//             product.  p, z and q~ alternate between two buffers.
// A chunk of m iterations opens with a plain product (k_spmv) and ends with
// the m-th update folding the increments into the double-double solution
// (k_update_flush), an exact float64 residual from the CSR matrix (k_resid,
// k_sys_check) and the new direction (k_pdir).  Between them the per-iteration
// kernels synchronise only through kernel boundaries: no fences, no spin
// waits.  Where every tile of one system fits the device at once, a
// resident kernel instead runs the chunk's m - 1 iterations in one launch,
// separating iterations with a bounded grid barrier on per-tile flags:
// k_chunk holds each tile's rows (matrix and vectors) on chip; k_chunk_win,
// for larger operators, one tile per compute unit, holds the tile's column
// window of p and z and its rows' x_acc and q~, and streams the matrix.
// Chunks are captured once in a HIP graph and replayed; a system whose test
// passes is masked out of later kernels.
//
// Difference form: row i is stored as c_i = sum_j a_ij (its mass or
// Dirichlet part) and w_ij = -a_ij, and (A p)_i = c_i p_i + sum_j w_ij (p_i -
// p_j).  Rounding the weights then perturbs the quadratic form by a relative
// O(u) on every mode, which keeps float32 Krylov vectors usable on these
// M-matrices.
//
// Compiled with -ffp-contract=off.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <iterator>
#include <map>
#include <mutex>
#include <string>
#include <tuple>

#include "kernels.h"
#include "solver.h"

namespace pm {

template <typename V, typename W, typename I>
struct SetArgs {
  int N, n_sys;
  const int* tile_sys;
  const int* tile_r0;
  const int* tile_r1;
  const int* sys_tile0;
  const int* tile_lo;  // first and last column any row of the tile reaches
  const int* tile_hi;
  const int* tile_pub_lo;  // rows r < pub_lo or r >= pub_hi are in another tile's window
  const int* tile_pub_hi;
  const int* perm;
  const int* rp;
  const int* col;
  const double* val;
  const double* b;
  double* x;
  W* c;
  W* w;
  I* idx;
  double* dp;
  double* x64;
  double* xlo;
  double* b64;
  V* xacc;
  V* p[2];        // ping-pong direction, residual/D' and D'^{-1} A p buffers
  V* z[2];
  V* q[2];
  double* part[2];  // [tile][4] product partials, alternating with the buffers
  double* part3;    // [tile][4] residual partials
  V* y;             // D'^{-1} r (Chebyshev schedule)
  V* zc[3];         // Chebyshev iterates, rotating
  SysState* ss;
  uint32_t* flags;  // [tile * 16]: resident chunk kernel's published-iteration counts
};

// Fixed-order sum over the tile partials t0..t1-1 (stride 4); every thread of
// the block gets the result, so all blocks of a system agree bit for bit.
template <int NV>
__device__ __forceinline__ void sum_range(const double* __restrict__ part, int t0, int t1,
                                          double (&out)[NV]) {
  __shared__ double sh[NV][16];
  __shared__ double res[NV];
  double v[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = 0.0;
  for (int t = t0 + (int)threadIdx.x; t < t1; t += blockDim.x)
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] += part[4 * (size_t)t + k];
  wave_sum<NV>(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k) sh[k][wid] = v[k];
  __syncthreads();
  if (threadIdx.x < NV) {
    double s = 0.0;
    for (int ww = 0; ww < nw; ++ww) s += sh[threadIdx.x][ww];
    res[threadIdx.x] = s;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) out[k] = res[k];
}

template <int NV>
__device__ __forceinline__ void tile_partial(double (&v)[NV], double* part) {
  block_partial<NV>(v, part);
}

__global__ void k_sys_init(SysState* ss, int n_sys, int max_it, int stag_it) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_sys) return;
  SysState z{};
  z.max_it = max_it;
  z.stag_it = stag_it;
  z.rho_ring[0] = z.rho_ring[1] = INFINITY;  // first Chebyshev direction: beta = 0
  ss[s] = z;
}

// Difference-form rows from the float64 CSR: c_i = row sum, w = -off-diagonals
// padded to three slots (padding: w = 0 pointing at the row itself), and
// d' = c + sum w evaluated from the stored (rounded) values: the Jacobi
// diagonal the iteration uses.  Also brings b and x0 into the packed order.
template <typename V, typename W, typename I>
__global__ void __launch_bounds__(1024) k_prep(SetArgs<V, W, I> a, int x0_zero) {
  const int t = xcd_block(blockIdx.x, gridDim.x);
  const int s = a.tile_sys[t];
  const int N = a.N;
  int err = 0;
  double acc[2] = {0.0, 0.0};
  for (int i = a.tile_r0[t] + threadIdx.x; i < a.tile_r1[t]; i += blockDim.x) {
    double sum = 0.0;
    bool fin = true;
    W wv[3] = {W(0), W(0), W(0)};
    I iv[3];
    iv[0] = iv[1] = iv[2] = sizeof(I) == 2 ? I(0) : I(i);
    int nk = 0;
    for (int k = a.rp[i]; k < a.rp[i + 1]; ++k) {
      const double v = a.val[k];
      fin = fin && isfinite(v);
      sum += v;
      const int j = a.col[k];
      if (j != i && nk < 3) {
        wv[nk] = (W)(-v);
        iv[nk] = sizeof(I) == 2 ? I(j - i) : I(j);
        ++nk;
      }
    }
    const W cw = (W)sum;
    a.c[i] = cw;
    double d = (double)cw;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      a.w[(size_t)k * N + i] = wv[k];
      a.idx[(size_t)k * N + i] = iv[k];
      d += (double)wv[k];
    }
    a.dp[i] = d;
    if (!fin) err = PM_NONFINITE;
    else if (!(d > 0.0) && err == 0) err = PM_INVALID_ARG;
    const int o = a.perm[i];
    const double bi = a.b[o];
    const double xi = x0_zero ? 0.0 : a.x[o];
    a.b64[i] = bi;
    a.x64[i] = xi;
    a.xlo[i] = 0.0;
    a.xacc[i] = V(0);
    a.p[0][i] = V(0);
    a.p[1][i] = V(0);
    acc[0] += bi * bi;
    acc[1] += xi * xi;
  }
  if (err) atomicExch(&a.ss[s].err, err);
  tile_partial<2>(acc, a.part[0] + 4 * (size_t)t);
}

// One block per system: ||b||, the tolerance, the input checks.
template <typename V, typename W, typename I>
__global__ void k_sys_start(SetArgs<V, W, I> a, double tol) {
  const int s = blockIdx.x;
  double r[2];
  sum_range<2>(a.part[0], a.sys_tile0[s], a.sys_tile0[s + 1], r);
  if (threadIdx.x != 0) return;
  SysState& S = a.ss[s];
  S.bnorm2 = r[0];
  S.tol2 = tol * tol * r[0];
  if (S.err != 0) {
    S.status = S.err;
    S.done = 1;
  } else if (!isfinite(r[0]) || !isfinite(r[1])) {
    S.status = PM_NONFINITE;
    S.done = 1;
  } else if (r[0] == 0.0) {
    S.status = PM_OK;
    S.res2 = 0.0;
    S.done = 2;  // zero right-hand side: the solution is 0
  }
}

// True residuals from the float64 CSR with error-free transformations, for the
// returned vector x_hi (stopping test) and for x_hi + x_lo (replacement);
// tile partials of ||r_hi||^2, z.D'z and || |A||x_hi| ||^2 (rounding floor).
//   mode 0 (start):   z = r_dd/d', p = z   (buffer 0)
//   mode 1 (replace): z = r_dd/d'          (buffer 0)
//   mode 2 (final):   norms only, also for stopped systems
// With inv_theta > 0 (Chebyshev schedule) modes 0 and 1 write y = r_dd/d' and
// the first Chebyshev iterate z_1 = y / theta instead.
template <typename V, typename W, typename I>
__global__ void __launch_bounds__(1024) k_resid(SetArgs<V, W, I> a, int mode, double inv_theta) {
  const int t = xcd_block(blockIdx.x, gridDim.x);
  const int s = a.tile_sys[t];
  if (mode != 2 && a.ss[s].done) return;
  double acc[3] = {0.0, 0.0, 0.0};
  // Rows of these meshes hold at most kRowMax entries (three neighbours and
  // the diagonal); every load of R rows is issued before the first use, and
  // the compensated sums run over the entries in CSR order with zero padding
  // (exact no-ops), the same arithmetic as residual_row.  Longer rows finish
  // in residual_row's loop.
  constexpr int R = 2, kRowMax = 4;
  const int r0 = a.tile_r0[t], r1 = a.tile_r1[t];
  for (int base = r0 + threadIdx.x; base < r1; base += R * blockDim.x) {
    int k0[R], k1[R], cj[R][kRowMax];
    double bi[R], av[R][kRowMax], xh[R][kRowMax], xl[R][kRowMax];
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int i = base + u * (int)blockDim.x;
      const int ii = i < r1 ? i : r0;
      k0[u] = a.rp[ii];
      k1[u] = a.rp[ii + 1];
      bi[u] = a.b64[ii];
    }
#pragma unroll
    for (int u = 0; u < R; ++u)
#pragma unroll
      for (int e = 0; e < kRowMax; ++e) {
        const int k = k0[u] + e < k1[u] ? k0[u] + e : k0[u];
        cj[u][e] = a.col[k];
        av[u][e] = k0[u] + e < k1[u] ? a.val[k] : 0.0;
      }
#pragma unroll
    for (int u = 0; u < R; ++u)
#pragma unroll
      for (int e = 0; e < kRowMax; ++e) {
        xh[u][e] = a.x64[cj[u][e]];
        xl[u][e] = a.xlo[cj[u][e]];
      }
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int i = base + u * (int)blockDim.x;
      if (i >= r1) continue;
      double sum = bi[u], e = 0.0, el = 0.0, m = 0.0;
#pragma unroll
      for (int q = 0; q < kRowMax; ++q) {
        const double av_ = av[u][q], xv = xh[u][q];
        const double pr = av_ * xv;
        m += fabs(pr);
        const double pe = __builtin_fma(av_, xv, -pr);
        const double tt = sum - pr;
        const double bb = tt - sum;
        const double err = (sum - (tt - bb)) + (-pr - bb);
        sum = tt;
        e += err - pe;
        el -= av_ * xl[u][q];
      }
      double rh = sum + e, rd = sum + (e + el), ax = m;
      if (k1[u] - k0[u] > kRowMax) {  // not on triangle meshes; kept general
        double rh2, rd2, ax2;
        residual_row(0.0, a.val, a.col, a.x64, a.xlo, k0[u] + kRowMax, k1[u], rh2, rd2, ax2);
        rh += rh2;
        rd += rd2;
        ax += ax2;
      }
      acc[0] += rh * rh;
      acc[2] += ax * ax;
      if (mode == 2) continue;
      const double d = a.dp[i];
      const V zv = (V)(rd / d);
      if (inv_theta > 0.0) {
        a.y[i] = zv;
        a.zc[1][i] = (V)((double)zv * inv_theta);
      } else {
        a.z[0][i] = zv;
        if (mode == 0) a.p[0][i] = zv;
      }
      const double zd = (double)zv;
      acc[1] += d * zd * zd;
    }
  }
  tile_partial<3>(acc, a.part3 + 4 * (size_t)t);
}

// One block per system after k_resid: the convergence test on the returned
// vector; the stagnation test (the best residual norm is within 100x of the
// rounding floor u || |A||x| || and has not halved for max(stag_it, k_best)
// iterations); the scalars of the next direction, which restarts (beta = 0)
// when r.D'^{-1}r of the true residual exceeds 100 times that of the
// recursive residual it replaces (the recursion drifted away from it).
template <typename V, typename W, typename I>
__global__ void k_sys_check(SetArgs<V, W, I> a, int mode, int cheb) {
  const int s = blockIdx.x;
  SysState& S = a.ss[s];
  if (mode != 2 && S.done) return;
  if (mode == 2 && S.done == 2) return;
  double r[3];
  sum_range<3>(a.part3, a.sys_tile0[s], a.sys_tile0[s + 1], r);
  double nr[4] = {S.nu_rec, 0.0, 0.0, 0.0};
  if (cheb && mode == 1) sum_range<4>(a.part[1], a.sys_tile0[s], a.sys_tile0[s + 1], nr);
  if (threadIdx.x != 0) return;
  const bool restart = r[1] > 100.0 * nr[0];
  S.res2 = r[0];
  if (mode == 2) return;
  if (!isfinite(r[0])) {
    S.status = PM_NONFINITE;
    S.done = 1;
  } else if (r[0] <= S.tol2) {
    S.status = PM_OK;
    S.done = 1;
  } else if (mode == 0) {
    if (!cheb) S.rho = r[1];
    S.best_res2 = r[0];
    S.k_best = S.iter;
  } else {
    if (r[0] < 0.25 * S.best_res2) {
      S.best_res2 = r[0];
      S.k_best = S.iter;
    }
    const double floor2 = 0x1p-106 * r[2];
    const int window = S.stag_it > S.k_best ? S.stag_it : S.k_best;
    if (S.best_res2 < 1e4 * floor2 && S.iter - S.k_best >= window) {
      S.status = PM_STAGNATED;
      S.done = 1;
    } else {
      if (!cheb) {
        S.beta = restart ? 0.0 : r[1] / S.rho;
        S.rho = r[1];
      } else if (restart) {  // the Chebyshev direction kernel forms beta from the ring
        S.rho_ring[S.iter & 1] = INFINITY;
      }
      S.iter_base = S.iter;
    }
  }
}

// p = z + beta p after a replacement: z in buffer 0, the old p in buffer
// `src`, the new p in buffer 0.
template <typename V, typename W, typename I>
__global__ void __launch_bounds__(1024) k_pdir(SetArgs<V, W, I> a, int src) {
  const int t = xcd_block(blockIdx.x, gridDim.x);
  const SysState& S = a.ss[a.tile_sys[t]];
  if (S.done) return;
  const double be = S.beta;
  const V* ps = a.p[src];
  V* pd = a.p[0];
  for (int i = a.tile_r0[t] + threadIdx.x; i < a.tile_r1[t]; i += blockDim.x)
    pd[i] = (V)((double)a.z[0][i] + be * (double)ps[i]);
}

// Rows handled per thread and loop trip: every load of the group is issued
// before the first use, so each thread keeps R rows of memory traffic in flight.
constexpr int kUnroll = 4;

// Stop decision of an update from the reduced product partials (identical in
// every block of the system): 0 = go on, 100 = exact zero residual, else the
// status.
__device__ __forceinline__ int stop_code(int k, int max_it, double pq, double rho) {
  if (k > max_it) return PM_MAXIT;
  if (rho == 0.0) return 100;
  if (!(pq > 0.0) || !isfinite(pq) || !isfinite(rho)) return PM_BREAKDOWN;
  return 0;
}

// Plain product on buffer 0 (the first iteration of a chunk):
// q~ = D'^{-1} A p in difference form and, with q = D' q~ as stored, the tile
// partials of  s0 = p.q,  s1 = z.q (= q.D'^{-1} r),  s2 = q.D'^{-1} q,
// s3 = z.D' z (= rho), into part[0].
template <typename V, typename W, typename I>
__global__ void __launch_bounds__(1024) k_spmv(SetArgs<V, W, I> a) {
  const int t = xcd_block(blockIdx.x, gridDim.x);
  const int s = a.tile_sys[t];
  if (a.ss[s].done) return;
  const int N = a.N;
  const W* __restrict__ c = a.c;
  const W* __restrict__ w = a.w;
  const I* __restrict__ idx = a.idx;
  const V* __restrict__ p = a.p[0];
  const V* __restrict__ z = a.z[0];
  V* __restrict__ q = a.q[0];
  const int r0 = a.tile_r0[t], r1 = a.tile_r1[t];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int base = r0 + threadIdx.x; base < r1; base += kUnroll * blockDim.x) {
    int row[kUnroll];
    W w0[kUnroll], w1[kUnroll], w2[kUnroll], cc[kUnroll];
    I i0[kUnroll], i1[kUnroll], i2[kUnroll];
    V pv[kUnroll], zv[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int i0r = base + u * (int)blockDim.x;
      row[u] = i0r < r1 ? i0r : -1;
      const int i = i0r < r1 ? i0r : r0;  // a valid row keeps the loads in bounds
      w0[u] = w[i];
      w1[u] = w[(size_t)N + i];
      w2[u] = w[2 * (size_t)N + i];
      i0[u] = idx[i];
      i1[u] = idx[(size_t)N + i];
      i2[u] = idx[2 * (size_t)N + i];
      cc[u] = c[i];
      pv[u] = p[i];
      zv[u] = z[i];
    }
    V g0[kUnroll], g1[kUnroll], g2[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int i = row[u] >= 0 ? row[u] : r0;
      g0[u] = p[col_of<I>(i, i0[u])];
      g1[u] = p[col_of<I>(i, i1[u])];
      g2[u] = p[col_of<I>(i, i2[u])];
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      if (row[u] < 0) continue;
      const double pi = (double)pv[u];
      const double ci = (double)cc[u];
      double y = ci * pi;
      y += (double)w0[u] * (pi - (double)g0[u]);
      y += (double)w1[u] * (pi - (double)g1[u]);
      y += (double)w2[u] * (pi - (double)g2[u]);
      const double d = ((ci + (double)w0[u]) + (double)w1[u]) + (double)w2[u];
      const V qv = (V)(y / d);
      q[row[u]] = qv;
      const double qd = (double)qv, zi = (double)zv[u];
      const double dq = d * qd;
      acc[0] += pi * dq;
      acc[1] += zi * dq;
      acc[2] += qd * dq;
      acc[3] += d * zi * zi;
    }
  }
  tile_partial<4>(acc, a.part[0] + 4 * (size_t)t);
}

// Partials of a system's tiles, loaded by the threads of a block before they
// are needed: thread tid holds tiles t0 + tid + u * blockDim (u < kPartU) as
// two 16-byte loads each; partial_reduce() adds them in a fixed order (then
// any further tiles, then across lanes and waves), so every block of the
// system obtains the same sums.
constexpr int kPartU = 4;

template <int PU>
struct PartRegsT {
  double2 v[PU][2];
};
using PartRegs = PartRegsT<kPartU>;

// Branch-free: every thread loads a valid tile (its own, or the system's last
// one) and partial_reduce() drops the copies, so no load waits on another.
// PU tiles per thread in registers; the sum is the same for any PU.
template <int PU>
__device__ __forceinline__ void partial_load(const double* __restrict__ part, int t0, int t1,
                                             PartRegsT<PU>& P) {
  const double2* p2 = reinterpret_cast<const double2*>(part);
#pragma unroll
  for (int u = 0; u < PU; ++u) {
    const int tt = t0 + (int)threadIdx.x + u * (int)blockDim.x;
    const size_t tc = (size_t)(tt < t1 ? tt : t1 - 1);
    P.v[u][0] = p2[2 * tc];
    P.v[u][1] = p2[2 * tc + 1];
  }
}

template <int PU>
__device__ __forceinline__ void partial_reduce(const double* __restrict__ part, int t0, int t1,
                                               const PartRegsT<PU>& P, double (&out)[4]) {
  __shared__ double sh[4][16];
  __shared__ double res[4];
  double v[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int u = 0; u < PU; ++u) {
    const bool own = t0 + (int)threadIdx.x + u * (int)blockDim.x < t1;
    v[0] += own ? P.v[u][0].x : 0.0;
    v[1] += own ? P.v[u][0].y : 0.0;
    v[2] += own ? P.v[u][1].x : 0.0;
    v[3] += own ? P.v[u][1].y : 0.0;
  }
  for (int tt = t0 + (int)threadIdx.x + PU * (int)blockDim.x; tt < t1; tt += blockDim.x)
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] += part[4 * (size_t)tt + k];
  wave_sum<4>(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < 4; ++k) sh[k][wid] = v[k];
  __syncthreads();
  if (threadIdx.x < 4) {
    double acc = 0.0;
    for (int w = 0; w < nw; ++w) acc += sh[threadIdx.x][w];
    res[threadIdx.x] = acc;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 4; ++k) out[k] = res[k];
}

// The rows one thread handles in one trip of the fused iteration, with their
// neighbours' p, z and q~.
template <typename V, typename W, typename I, int R>
struct Trip {
  int row[R];
  W w0[R], w1[R], w2[R], cc[R];
  I i0[R], i1[R], i2[R];
  V pv[R], zv[R], qv[R], xv[R];
  V gp[3][R], gz[3][R], gq[3][R];
};

template <typename V, typename W, typename I, int R>
__device__ __forceinline__ void trip_direct(Trip<V, W, I, R>& T, const SetArgs<V, W, I>& a,
                                            const V* __restrict__ ps, const V* __restrict__ zs,
                                            const V* __restrict__ qs, int base, int r0, int r1) {
  const size_t N = (size_t)a.N;
#pragma unroll
  for (int u = 0; u < R; ++u) {
    const int i0r = base + u * (int)blockDim.x;
    T.row[u] = i0r < r1 ? i0r : -1;
    const int i = i0r < r1 ? i0r : r0;  // a valid row keeps the loads in bounds
    T.w0[u] = a.w[i];
    T.w1[u] = a.w[N + i];
    T.w2[u] = a.w[2 * N + i];
    T.i0[u] = a.idx[i];
    T.i1[u] = a.idx[N + i];
    T.i2[u] = a.idx[2 * N + i];
    T.cc[u] = a.c[i];
    T.pv[u] = ps[i];
    T.zv[u] = zs[i];
    T.qv[u] = qs[i];
    T.xv[u] = a.xacc[i];
  }
}

template <typename V, typename W, typename I, int R>
__device__ __forceinline__ void trip_gather(Trip<V, W, I, R>& T, const V* __restrict__ ps,
                                            const V* __restrict__ zs, const V* __restrict__ qs,
                                            int r0) {
#pragma unroll
  for (int u = 0; u < R; ++u) {
    const int i = T.row[u] >= 0 ? T.row[u] : r0;
    const int j0 = col_of<I>(i, T.i0[u]), j1 = col_of<I>(i, T.i1[u]), j2 = col_of<I>(i, T.i2[u]);
    T.gp[0][u] = ps[j0];
    T.gz[0][u] = zs[j0];
    T.gq[0][u] = qs[j0];
    T.gp[1][u] = ps[j1];
    T.gz[1][u] = zs[j1];
    T.gq[1][u] = qs[j1];
    T.gp[2][u] = ps[j2];
    T.gz[2][u] = zs[j2];
    T.gq[2][u] = qs[j2];
  }
}

// The update and product for the rows of one trip (see k_iter).
template <typename V, typename W, typename I, int R>
__device__ __forceinline__ void trip_compute(const Trip<V, W, I, R>& T, double as, double bs,
                                             V* __restrict__ pd, V* __restrict__ zd,
                                             V* __restrict__ qd, V* __restrict__ xacc,
                                             double (&acc)[4]) {
#pragma unroll
  for (int u = 0; u < R; ++u) {
    if (T.row[u] < 0) continue;
    const int i = T.row[u];
    const double pold = (double)T.pv[u];
    xacc[i] = (V)((double)T.xv[u] + as * pold);
    const V zn = (V)((double)T.zv[u] - as * (double)T.qv[u]);
    const V pn = (V)((double)zn + bs * pold);
    zd[i] = zn;
    pd[i] = pn;
    double g[3];
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      const V zj = (V)((double)T.gz[e][u] - as * (double)T.gq[e][u]);
      g[e] = (double)(V)((double)zj + bs * (double)T.gp[e][u]);
    }
    const double pi = (double)pn;
    const double ci = (double)T.cc[u];
    double y = ci * pi;
    y += (double)T.w0[u] * (pi - g[0]);
    y += (double)T.w1[u] * (pi - g[1]);
    y += (double)T.w2[u] * (pi - g[2]);
    const double d = ((ci + (double)T.w0[u]) + (double)T.w1[u]) + (double)T.w2[u];
    const V qn = (V)(y / d);
    qd[i] = qn;
    const double qq = (double)qn, zi = (double)zn;
    const double dq = d * qq;
    acc[0] += pi * dq;
    acc[1] += zi * dq;
    acc[2] += qq * dq;
    acc[3] += d * zi * zi;
  }
}

// Iteration k = iter_base + j of a chunk (1 <= j < m), reading buffer src and
// writing buffer dst = src ^ 1.  Every block reduces its system's partials of
// the last product (same order, same result): alpha = rho / p.q, the next rho
// by its recurrence anchored on the exact rho, beta = rho_next / rho.  Then,
// for the rows of the tile,
//   x_acc += alpha p;  z' = z - alpha q~;  p' = z' + beta p
// and at once q~' = D'^{-1} A p' with the tile partials of the next product.
// The p' of a neighbour row comes from that row's p, z and q~ in buffer src by
// the same expression (same roundings) its own block evaluates, so every block
// sees the same p'.  Loads are software-pipelined: the first trip's rows and
// the partials are all in flight before the reduction waits on any of them,
// and the next trip's rows are loaded while a trip is computed.  (A third
// trip in flight, and non-temporal loads of the streamed arrays, measured
// slower on MI355X.)  The
// system's first tile records the scalars and the iteration count, or the
// stop status.  `scale` multiplies alpha and beta (1 in solves, 0 when the
// kernel is timed).
template <typename V, typename W, typename I, int R>
__global__ void __launch_bounds__(512) k_iter(SetArgs<V, W, I> a, int src, int j, double scale) {
  const int t = xcd_block(blockIdx.x, gridDim.x);
  const int s = a.tile_sys[t];
  SysState& S = a.ss[s];
  if (S.done) return;
  const int r0 = a.tile_r0[t], r1 = a.tile_r1[t];
  const int t0 = a.sys_tile0[s], t1 = a.sys_tile0[s + 1];
  const V* __restrict__ ps = a.p[src];
  const V* __restrict__ zs = a.z[src];
  const V* __restrict__ qs = a.q[src];
  V* __restrict__ pd = a.p[src ^ 1];
  V* __restrict__ zd = a.z[src ^ 1];
  V* __restrict__ qd = a.q[src ^ 1];
  V* __restrict__ xacc = a.xacc;
  const int step = R * (int)blockDim.x;
  int base = r0 + (int)threadIdx.x;

  Trip<V, W, I, R> Ta, Tb;
  trip_direct<V, W, I, R>(Ta, a, ps, zs, qs, base, r0, r1);
  PartRegs P;
  partial_load(a.part[src], t0, t1, P);
  trip_gather<V, W, I, R>(Ta, ps, zs, qs, r0);
  double r[4];
  partial_reduce(a.part[src], t0, t1, P, r);

  const bool first = t == t0 && threadIdx.x == 0;
  const int k = S.iter_base + j;
  const double pq = r[0], rho = r[3];
  if (const int stop = stop_code(k, S.max_it, pq, rho)) {
    if (first) {
      S.status = stop == 100 ? PM_OK : stop;
      S.done = 1;
    }
    return;
  }
  const double al = rho / pq;
  const double rn = rho - 2.0 * al * r[1] + al * al * r[2];
  const double be = rn / rho;
  const double as = al * scale, bs = be * scale;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  // two trip buffers in turn: while one trip is computed, the next trip's row
  // loads are in flight.  Loads past the tile end are clamped to row r0 and
  // flagged, so they are always in bounds.
  for (;;) {
    trip_direct<V, W, I, R>(Tb, a, ps, zs, qs, base + step, r0, r1);
    trip_compute<V, W, I, R>(Ta, as, bs, pd, zd, qd, xacc, acc);
    base += step;
    if (base >= r1) break;
    trip_gather<V, W, I, R>(Tb, ps, zs, qs, r0);
    trip_direct<V, W, I, R>(Ta, a, ps, zs, qs, base + step, r0, r1);
    trip_compute<V, W, I, R>(Tb, as, bs, pd, zd, qd, xacc, acc);
    base += step;
    if (base >= r1) break;
    trip_gather<V, W, I, R>(Ta, ps, zs, qs, r0);
  }
  tile_partial<4>(acc, a.part[src ^ 1] + 4 * (size_t)t);
  if (first) {
    S.alpha = al;
    S.beta = be;
    S.rho = rho;
    S.iter = k;
  }
}

// LDS-staged fused iteration: the same arithmetic as k_iter, bit for bit.
// The new z and p of every row in the tile's column window [tile_lo,
// tile_hi] are formed once, by one thread, into LDS (rows of the tile also
// store them to global memory there), so the product reads its neighbours
// from LDS instead of gathering three vectors per neighbour from L2.  Every
// global load is coalesced and independent of the others: the first
// staging rows, the first product rows and the partials are all in flight
// before the reduction waits on any of them.
template <typename V, typename W, typename I>
__global__ void __launch_bounds__(512) k_iter_lds(SetArgs<V, W, I> a, int src, int j,
                                                  double scale) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const int t = xcd_block(blockIdx.x, gridDim.x);
  const int s = a.tile_sys[t];
  SysState& S = a.ss[s];
  if (S.done) return;
  const int r0 = a.tile_r0[t], r1 = a.tile_r1[t];
  const int lo = a.tile_lo[t], nwin = a.tile_hi[t] - lo + 1;
  const int t0 = a.sys_tile0[s], t1 = a.sys_tile0[s + 1];
  const int B = blockDim.x, tid = threadIdx.x;
  const size_t N = (size_t)a.N;
  V* __restrict__ lp = reinterpret_cast<V*>(lds_raw);
  V* __restrict__ lz = lp + nwin;
  const V* __restrict__ ps = a.p[src];
  const V* __restrict__ zs = a.z[src];
  const V* __restrict__ qs = a.q[src];
  V* __restrict__ pd = a.p[src ^ 1];
  V* __restrict__ zd = a.z[src ^ 1];
  V* __restrict__ qd = a.q[src ^ 1];
  V* __restrict__ xacc = a.xacc;

  constexpr int kStage = 4;  // staging rows per thread loaded before the reduction
  V sp[kStage], sz[kStage], sq[kStage];
#pragma unroll
  for (int u = 0; u < kStage; ++u) {
    const int w = tid + u * B;
    const int i = lo + (w < nwin ? w : nwin - 1);
    sp[u] = ps[i];
    sz[u] = zs[i];
    sq[u] = qs[i];
  }
  PartRegs P;
  partial_load(a.part[src], t0, t1, P);
  constexpr int R = kUnroll;
  W w0[R], w1[R], w2[R], cc[R];
  I i0[R], i1[R], i2[R];
  V xv[R], pv[R];
  auto load_rows = [&](int b0) {
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int ir = b0 + u * B;
      const int i = ir < r1 ? ir : r0;
      w0[u] = a.w[i];
      w1[u] = a.w[N + i];
      w2[u] = a.w[2 * N + i];
      i0[u] = a.idx[i];
      i1[u] = a.idx[N + i];
      i2[u] = a.idx[2 * N + i];
      cc[u] = a.c[i];
      xv[u] = xacc[i];
      pv[u] = ps[i];
    }
  };
  int base = r0 + tid;
  load_rows(base);
  double r[4];
  partial_reduce(a.part[src], t0, t1, P, r);

  const bool first = t == t0 && tid == 0;
  const int k = S.iter_base + j;
  const double pq = r[0], rho = r[3];
  if (const int stop = stop_code(k, S.max_it, pq, rho)) {
    if (first) {
      S.status = stop == 100 ? PM_OK : stop;
      S.done = 1;
    }
    return;
  }
  const double al = rho / pq;
  const double rn = rho - 2.0 * al * r[1] + al * al * r[2];
  const double be = rn / rho;
  const double as = al * scale, bs = be * scale;

  auto stage = [&](int w, V pold, V zold, V qold) {
    const V zn = (V)((double)zold - as * (double)qold);
    const V pn = (V)((double)zn + bs * (double)pold);
    lp[w] = pn;
    lz[w] = zn;
    const int i = lo + w;
    if (i >= r0 && i < r1) {
      zd[i] = zn;
      pd[i] = pn;
    }
  };
#pragma unroll
  for (int u = 0; u < kStage; ++u) {
    const int w = tid + u * B;
    if (w < nwin) stage(w, sp[u], sz[u], sq[u]);
  }
  for (int w = tid + kStage * B; w < nwin; w += B) stage(w, ps[lo + w], zs[lo + w], qs[lo + w]);
  __syncthreads();

  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (;;) {
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int i = base + u * B;
      if (i >= r1) continue;
      xacc[i] = (V)((double)xv[u] + as * (double)pv[u]);
      const int li = i - lo;
      const double pi = (double)lp[li], zi = (double)lz[li], ci = (double)cc[u];
      double y = ci * pi;
      y += (double)w0[u] * (pi - (double)lp[col_of<I>(i, i0[u]) - lo]);
      y += (double)w1[u] * (pi - (double)lp[col_of<I>(i, i1[u]) - lo]);
      y += (double)w2[u] * (pi - (double)lp[col_of<I>(i, i2[u]) - lo]);
      const double d = ((ci + (double)w0[u]) + (double)w1[u]) + (double)w2[u];
      const V qn = (V)(y / d);
      qd[i] = qn;
      const double qq = (double)qn;
      const double dq = d * qq;
      acc[0] += pi * dq;
      acc[1] += zi * dq;
      acc[2] += qq * dq;
      acc[3] += d * zi * zi;
    }
    base += R * B;
    if (base >= r1) break;
    load_rows(base);
  }
  tile_partial<4>(acc, a.part[src ^ 1] + 4 * (size_t)t);
  if (first) {
    S.alpha = al;
    S.beta = be;
    S.rho = rho;
    S.iter = k;
  }
}

// Data that blocks of the resident chunk kernel exchange within one launch
// (halo rows, tile partials) is written and read with device-coherent
// accesses (relaxed atomics at agent scope: they write through and read past
// the per-XCD L2), so the grid barrier needs no L2 write-back or invalidate.
template <typename T>
__device__ __forceinline__ T ld_agent(const T* p) {
  if constexpr (sizeof(T) == 8) {
    const unsigned long long v = __hip_atomic_load(reinterpret_cast<const unsigned long long*>(p),
                                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return __builtin_bit_cast(T, v);
  } else {
    const unsigned v = __hip_atomic_load(reinterpret_cast<const unsigned*>(p), __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
    return __builtin_bit_cast(T, v);
  }
}

template <typename T>
__device__ __forceinline__ void st_agent(T* p, T x) {
  if constexpr (sizeof(T) == 8)
    __hip_atomic_store(reinterpret_cast<unsigned long long*>(p),
                       __builtin_bit_cast(unsigned long long, x), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  else
    __hip_atomic_store(reinterpret_cast<unsigned*>(p), __builtin_bit_cast(unsigned, x),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid barrier of the resident chunk kernel.  Each wave waits until its own
// stores (halo rows, tile partials) have completed; then the block publishes
// `count` (the solve's iteration number it has just finished: increasing
// within a solve, reset at its start) in its own flag (a 64-byte slot of
// `flags`), and its threads poll the flags of all nt tiles, one flag per
// thread, until every tile has published at least `count`.  A tile one
// iteration ahead wrote the other buffer parity, so its data does not
// disturb this iteration's.  No atomics: a shared
// counter would serialise the arrivals of all blocks.  Every wait is bounded
// (max_spins polls, about a second by default): a grid that is not fully
// resident gives up instead of spinning for ever.
__device__ __forceinline__ bool grid_barrier(uint32_t* flags, int t, int nt, uint32_t count,
                                             int max_spins) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0)
    __hip_atomic_store(flags + 16 * (size_t)t, count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  int good = 1;
  for (int u = (int)threadIdx.x; u < nt; u += blockDim.x) {
    int spins = 0;
    while (__hip_atomic_load(flags + 16 * (size_t)u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
               count &&
           spins < max_spins) {
      __builtin_amdgcn_s_sleep(1);
      ++spins;
    }
    good &= spins < max_spins;
  }
  return __syncthreads_and(good) != 0;
}

// Clears the resident kernel's flags at the start of a solve (a kernel, not a
// memset, so that it can sit in a captured graph).
__global__ void k_flags_reset(uint32_t* flags, int nt) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < nt) flags[16 * (size_t)t] = 0u;
}

// partial_reduce over all nt tiles with device-coherent loads (same order)
__device__ __forceinline__ void partial_reduce_agent(const double* part, int nt,
                                                     double (&out)[4]) {
  __shared__ double sh[4][16];
  __shared__ double res[4];
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (int tt = (int)threadIdx.x; tt < nt; tt += blockDim.x)
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] += ld_agent(part + 4 * (size_t)tt + k);
  wave_sum<4>(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < 4; ++k) sh[k][wid] = v[k];
  __syncthreads();
  if (threadIdx.x < 4) {
    double acc = 0.0;
    for (int w = 0; w < nw; ++w) acc += sh[threadIdx.x][w];
    res[threadIdx.x] = acc;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 4; ++k) out[k] = res[k];
}

// block_partial with a device-coherent store of the result
__device__ __forceinline__ void tile_partial_agent(double (&v)[4], double* part) {
  __shared__ double sh[4][16];
  wave_sum<4>(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < 4; ++k) sh[k][wid] = v[k];
  __syncthreads();
  if (threadIdx.x < 4) {
    double acc = 0.0;
    for (int w = 0; w < nw; ++w) acc += sh[threadIdx.x][w];
    st_agent(part + threadIdx.x, acc);
  }
}

// Resident chunk kernel: iterations j0 .. j1-1 of a chunk of one system in
// one launch, with one block per tile and every block resident (the host
// launches it only when the whole grid fits the device at once).  Each
// iteration performs exactly the arithmetic of k_iter / k_iter_lds, bit for
// bit, with the same fixed-order partial sums; what changes is where the
// data lives between iterations:
//   - the tile's matrix rows, x_acc and q~ stay in registers, its p and z in
//     LDS (inside the staged column window), for the whole launch;
//   - per iteration a block loads only the halo of its window (rows of other
//     tiles) from the buffer its neighbours wrote, and stores only its own
//     rows that fall in another tile's window, plus its tile partials;
//   - a grid barrier replaces the kernel boundary between iterations; what
//     crosses it is stored and loaded device-coherently.
// The last iteration stores every row (p, z, q~ and x_acc), so the kernels
// after the chunk find the same state as after the one-kernel-per-iteration
// schedule.  RPT: rows per thread (RPT * blockDim >= tile rows).
template <typename V, typename W, typename I, int RPT>
__global__ void __launch_bounds__(512) k_chunk(SetArgs<V, W, I> a, int j0, int j1,
                                               double scale, int max_spins) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const int t = xcd_block(blockIdx.x, gridDim.x);
  SysState& S = a.ss[0];
  if (S.done) return;
  const int r0 = a.tile_r0[t], r1 = a.tile_r1[t];
  const int lo = a.tile_lo[t], nwin = a.tile_hi[t] - lo + 1;
  const int pub_lo = a.tile_pub_lo[t], pub_hi = a.tile_pub_hi[t];
  const int nt = gridDim.x;
  const int B = blockDim.x, tid = threadIdx.x;
  const size_t N = (size_t)a.N;
  V* __restrict__ lp = reinterpret_cast<V*>(lds_raw);
  V* __restrict__ lz = lp + nwin;
  V* __restrict__ lq = lz + nwin;  // q~ of the tile's own rows
  // 16-bit column offsets of the tile's rows live in LDS ([3][RPT * B]),
  // wider ones in registers
  constexpr bool kIdxLds = sizeof(I) == 2;
  I* __restrict__ lx = reinterpret_cast<I*>(lq + RPT * B);
  // halo: window rows below the tile (nlow of them), then above it
  const int nlow = r0 - lo, nhalo = nwin - (r1 - r0);
  auto halo_w = [&](int h) { return h < nlow ? h : h + (r1 - r0); };

  W w0[RPT], w1[RPT], w2[RPT], cc[RPT];
  I i0[kIdxLds ? 1 : RPT], i1[kIdxLds ? 1 : RPT], i2[kIdxLds ? 1 : RPT];
  V xa[RPT];
#pragma unroll
  for (int u = 0; u < RPT; ++u) {
    const int ir = r0 + tid + u * B;
    const int i = ir < r1 ? ir : r0;
    w0[u] = a.w[i];
    w1[u] = a.w[N + i];
    w2[u] = a.w[2 * N + i];
    if constexpr (kIdxLds) {
      const int l = tid + u * B;
      lx[l] = a.idx[i];
      lx[RPT * B + l] = a.idx[N + i];
      lx[2 * RPT * B + l] = a.idx[2 * N + i];
    } else {
      i0[u] = a.idx[i];
      i1[u] = a.idx[N + i];
      i2[u] = a.idx[2 * N + i];
    }
    cc[u] = a.c[i];
    xa[u] = a.xacc[i];
  }
  // own rows' p, z, q~ of the chunk's first iteration, from the buffer the
  // previous kernels wrote, into LDS (later iterations keep them there)
  {
    const int src0 = (j0 - 1) & 1;
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
      const int i = r0 + tid + u * B;
      if (i >= r1) continue;
      lp[i - lo] = a.p[src0][i];
      lz[i - lo] = a.z[src0][i];
      lq[i - r0] = a.q[src0][i];
    }
  }
  const bool first_block = t == 0 && tid == 0;
  double al = 0.0, be = 0.0, rho = 0.0;
  int k_done = -1;
  bool failed = false;
  int src = (j0 - 1) & 1;
  for (int j = j0; j < j1; ++j, src ^= 1) {
    const bool first = j == j0, last = j + 1 == j1;
    if (!first && !grid_barrier(a.flags, t, nt, (uint32_t)(S.iter_base + j - 1), max_spins)) {
      failed = true;
      break;
    }
    const V* __restrict__ ps = a.p[src];
    const V* __restrict__ zs = a.z[src];
    const V* __restrict__ qs = a.q[src];
    V* __restrict__ pd = a.p[src ^ 1];
    V* __restrict__ zd = a.z[src ^ 1];
    V* __restrict__ qd = a.q[src ^ 1];
    // the first halo rows of this thread are in flight while the partials
    // are reduced
    constexpr int HR = 4;
    V hp[HR], hz[HR], hq[HR];
#pragma unroll
    for (int u = 0; u < HR; ++u) {
      const int h = tid + u * B;
      const int i = lo + halo_w(h < nhalo ? h : (nhalo > 0 ? nhalo - 1 : 0));
      const int ic = nhalo > 0 ? i : r0;
      hp[u] = ld_agent(ps + ic);
      hz[u] = ld_agent(zs + ic);
      hq[u] = ld_agent(qs + ic);
    }
    double r[4];
    partial_reduce_agent(a.part[src], nt, r);
    const int k = S.iter_base + j;
    const double pq = r[0], rh = r[3];
    if (const int stop = stop_code(k, S.max_it, pq, rh)) {
      if (first_block) {
        S.status = stop == 100 ? PM_OK : stop;
        S.done = 1;
      }
      break;
    }
    const double a_ = rh / pq;
    const double rn = rh - 2.0 * a_ * r[1] + a_ * a_ * r[2];
    const double b_ = rn / rh;
    const double as = a_ * scale, bs = b_ * scale;
    // staging: the new z and p of the window into LDS; own rows (old values
    // in LDS) by the thread that owns them, which also adds alpha p (old p)
    // to x_acc
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
      const int i = r0 + tid + u * B;
      if (i >= r1) continue;
      const int li = i - lo;
      const V qold = lq[i - r0];
      const V pold = lp[li];
      const V zold = lz[li];
      const V zn = (V)((double)zold - as * (double)qold);
      const V pn = (V)((double)zn + bs * (double)pold);
      xa[u] = (V)((double)xa[u] + as * (double)pold);
      lp[li] = pn;
      lz[li] = zn;
      if (last) {
        zd[i] = zn;
        pd[i] = pn;
      } else if (i < pub_lo || i >= pub_hi) {
        st_agent(zd + i, zn);
        st_agent(pd + i, pn);
      }
    }
    auto stage_halo = [&](int h, V pold, V zold, V qold) {
      const V zn = (V)((double)zold - as * (double)qold);
      const V pn = (V)((double)zn + bs * (double)pold);
      const int w = halo_w(h);
      lp[w] = pn;
      lz[w] = zn;
    };
#pragma unroll
    for (int u = 0; u < HR; ++u) {
      const int h = tid + u * B;
      if (h < nhalo) stage_halo(h, hp[u], hz[u], hq[u]);
    }
    for (int h = tid + HR * B; h < nhalo; h += B) {
      const int i = lo + halo_w(h);
      stage_halo(h, ld_agent(ps + i), ld_agent(zs + i), ld_agent(qs + i));
    }
    __syncthreads();
    // product of the new direction for own rows, with the tile partials
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
      const int i = r0 + tid + u * B;
      if (i >= r1) continue;
      const int li = i - lo;
      const double pi = (double)lp[li], zi = (double)lz[li], ci = (double)cc[u];
      I o0, o1, o2;
      if constexpr (kIdxLds) {
        const int l = tid + u * B;
        o0 = lx[l];
        o1 = lx[RPT * B + l];
        o2 = lx[2 * RPT * B + l];
      } else {
        o0 = i0[u];
        o1 = i1[u];
        o2 = i2[u];
      }
      double y = ci * pi;
      y += (double)w0[u] * (pi - (double)lp[col_of<I>(i, o0) - lo]);
      y += (double)w1[u] * (pi - (double)lp[col_of<I>(i, o1) - lo]);
      y += (double)w2[u] * (pi - (double)lp[col_of<I>(i, o2) - lo]);
      const double d = ((ci + (double)w0[u]) + (double)w1[u]) + (double)w2[u];
      const V qn = (V)(y / d);
      lq[i - r0] = qn;
      if (last) qd[i] = qn;
      else if (i < pub_lo || i >= pub_hi) st_agent(qd + i, qn);
      const double qq = (double)qn;
      const double dq = d * qq;
      acc[0] += pi * dq;
      acc[1] += zi * dq;
      acc[2] += qq * dq;
      acc[3] += d * zi * zi;
    }
    tile_partial_agent(acc, a.part[src ^ 1] + 4 * (size_t)t);
    al = a_;
    be = b_;
    rho = rh;
    k_done = k;
  }
  // x_acc of the completed iterations (also after a stop, which leaves the
  // state of the last completed iteration, as the per-iteration kernels do)
#pragma unroll
  for (int u = 0; u < RPT; ++u) {
    const int i = r0 + tid + u * B;
    if (i < r1) a.xacc[i] = xa[u];
  }
  if (first_block) {
    if (k_done >= 0) {
      S.alpha = al;
      S.beta = be;
      S.rho = rho;
      S.iter = k_done;
    }
  }
  if (failed && tid == 0) {  // any block that gave up marks the solve failed
    S.status = PM_HIP_ERROR;
    S.bar_fail = 1;
    S.done = 1;
  }
}

// Resident window kernel: the form of k_chunk for systems whose operator does
// not fit on chip (one large tile per compute unit).  What stays on chip for
// the whole launch is the tile's column window of p and z (LDS) and x_acc
// and q~ of the thread's own rows (registers, RPT rows per thread); the
// matrix rows are read every iteration.  The halo exchange, partials and
// grid barrier are those of k_chunk.  Same arithmetic as k_iter /
// k_iter_lds, bit for bit.  Rows are handled R per trip, RPT / R trips.
template <typename V, typename W, typename I, int RPT>
__global__ void __launch_bounds__(512) k_chunk_win(SetArgs<V, W, I> a, int j0, int j1,
                                                   double scale, int max_spins) {
  constexpr int R = kUnroll;
  static_assert(RPT % R == 0, "rows per thread in whole trips");
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const int t = xcd_block(blockIdx.x, gridDim.x);
  SysState& S = a.ss[0];
  if (S.done) return;
  const int r0 = a.tile_r0[t], r1 = a.tile_r1[t];
  const int lo = a.tile_lo[t], nwin = a.tile_hi[t] - lo + 1;
  const int pub_lo = a.tile_pub_lo[t], pub_hi = a.tile_pub_hi[t];
  const int nt = gridDim.x;
  const int B = blockDim.x, tid = threadIdx.x;
  const size_t N = (size_t)a.N;
  V* __restrict__ lp = reinterpret_cast<V*>(lds_raw);
  V* __restrict__ lz = lp + nwin;
  const int nlow = r0 - lo, nhalo = nwin - (r1 - r0);
  auto halo_w = [&](int h) { return h < nlow ? h : h + (r1 - r0); };
  V xa[RPT], qo[RPT];
  {
    const int src0 = (j0 - 1) & 1;
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
      const int ir = r0 + tid + u * B;
      const int i = ir < r1 ? ir : r0;
      xa[u] = a.xacc[i];
      qo[u] = a.q[src0][i];
      if (ir < r1) {
        lp[i - lo] = a.p[src0][i];
        lz[i - lo] = a.z[src0][i];
      }
    }
  }
  const bool first_block = t == 0 && tid == 0;
  double al = 0.0, be = 0.0, rho = 0.0;
  int k_done = -1;
  bool failed = false;
  int src = (j0 - 1) & 1;
  for (int j = j0; j < j1; ++j, src ^= 1) {
    const bool first = j == j0, last = j + 1 == j1;
    if (!first && !grid_barrier(a.flags, t, nt, (uint32_t)(S.iter_base + j - 1), max_spins)) {
      failed = true;
      break;
    }
    const V* __restrict__ ps = a.p[src];
    const V* __restrict__ zs = a.z[src];
    const V* __restrict__ qs = a.q[src];
    V* __restrict__ pd = a.p[src ^ 1];
    V* __restrict__ zd = a.z[src ^ 1];
    V* __restrict__ qd = a.q[src ^ 1];
    // the first own row, opaque to the compiler in every iteration: the
    // rows' addresses are then formed again each iteration instead of being
    // kept live across all of them (RPT rows x every array)
    int ib = r0 + tid;
    asm volatile("" : "+v"(ib));
    constexpr int HR = 4;
    V hp[HR], hz[HR], hq[HR];
#pragma unroll
    for (int u = 0; u < HR; ++u) {
      const int h = tid + u * B;
      const int i = lo + halo_w(h < nhalo ? h : (nhalo > 0 ? nhalo - 1 : 0));
      const int ic = nhalo > 0 ? i : r0;
      hp[u] = ld_agent(ps + ic);
      hz[u] = ld_agent(zs + ic);
      hq[u] = ld_agent(qs + ic);
    }
    double r[4];
    partial_reduce_agent(a.part[src], nt, r);
    const int k = S.iter_base + j;
    const double pq = r[0], rh = r[3];
    if (const int stop = stop_code(k, S.max_it, pq, rh)) {
      if (first_block) {
        S.status = stop == 100 ? PM_OK : stop;
        S.done = 1;
      }
      break;
    }
    const double a_ = rh / pq;
    const double rn = rh - 2.0 * a_ * r[1] + a_ * a_ * r[2];
    const double b_ = rn / rh;
    const double as = a_ * scale, bs = b_ * scale;
    // own rows: x_acc += alpha p; new z, p into LDS (published where another
    // tile's window reaches them)
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
      const int i = ib + u * B;
      if (i >= r1) continue;
      const int li = i - lo;
      const V pold = lp[li];
      const V zn = (V)((double)lz[li] - as * (double)qo[u]);
      const V pn = (V)((double)zn + bs * (double)pold);
      xa[u] = (V)((double)xa[u] + as * (double)pold);
      lp[li] = pn;
      lz[li] = zn;
      if (last) {
        zd[i] = zn;
        pd[i] = pn;
      } else if (i < pub_lo || i >= pub_hi) {
        st_agent(zd + i, zn);
        st_agent(pd + i, pn);
      }
    }
    auto stage_halo = [&](int h, V pold, V zold, V qold) {
      const V zn = (V)((double)zold - as * (double)qold);
      const V pn = (V)((double)zn + bs * (double)pold);
      const int w = halo_w(h);
      lp[w] = pn;
      lz[w] = zn;
    };
#pragma unroll
    for (int u = 0; u < HR; ++u) {
      const int h = tid + u * B;
      if (h < nhalo) stage_halo(h, hp[u], hz[u], hq[u]);
    }
    for (int h = tid + HR * B; h < nhalo; h += B) {
      const int i = lo + halo_w(h);
      stage_halo(h, ld_agent(ps + i), ld_agent(zs + i), ld_agent(qs + i));
    }
    __syncthreads();
    // product of the new direction for own rows, R rows per trip
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int tr = 0; tr < RPT / R; ++tr) {
      W w0[R], w1[R], w2[R], cc[R];
      I i0[R], i1[R], i2[R];
#pragma unroll
      for (int u = 0; u < R; ++u) {
        const int ir = ib + (tr * R + u) * B;
        const int i = ir < r1 ? ir : r0;
        w0[u] = a.w[i];
        w1[u] = a.w[N + i];
        w2[u] = a.w[2 * N + i];
        i0[u] = a.idx[i];
        i1[u] = a.idx[N + i];
        i2[u] = a.idx[2 * N + i];
        cc[u] = a.c[i];
      }
#pragma unroll
      for (int u = 0; u < R; ++u) {
        const int i = ib + (tr * R + u) * B;
        if (i >= r1) continue;
        const int li = i - lo;
        const double pi = (double)lp[li], zi = (double)lz[li], ci = (double)cc[u];
        double y = ci * pi;
        y += (double)w0[u] * (pi - (double)lp[col_of<I>(i, i0[u]) - lo]);
        y += (double)w1[u] * (pi - (double)lp[col_of<I>(i, i1[u]) - lo]);
        y += (double)w2[u] * (pi - (double)lp[col_of<I>(i, i2[u]) - lo]);
        const double d = ((ci + (double)w0[u]) + (double)w1[u]) + (double)w2[u];
        const V qn = (V)(y / d);
        qo[tr * R + u] = qn;
        if (last) qd[i] = qn;
        else if (i < pub_lo || i >= pub_hi) st_agent(qd + i, qn);
        const double qq = (double)qn;
        const double dq = d * qq;
        acc[0] += pi * dq;
        acc[1] += zi * dq;
        acc[2] += qq * dq;
        acc[3] += d * zi * zi;
      }
    }
    tile_partial_agent(acc, a.part[src ^ 1] + 4 * (size_t)t);
    al = a_;
    be = b_;
    rho = rh;
    k_done = k;
  }
  // x_acc of the completed iterations
#pragma unroll
  for (int u = 0; u < RPT; ++u) {
    const int i = r0 + tid + u * B;
    if (i < r1) a.xacc[i] = xa[u];
  }
  if (first_block && k_done >= 0) {
    S.alpha = al;
    S.beta = be;
    S.rho = rho;
    S.iter = k_done;
  }
  if (failed && tid == 0) {
    S.status = PM_HIP_ERROR;
    S.bar_fail = 1;
    S.done = 1;
  }
}

// Split schedule (the tuner may prefer it where the fused kernel's extra
// neighbour gathers cost more than the pass it saves): after k_spmv on buffer
// 0, iteration k = iter_base + j updates x_acc, z and p in place with the
// scalars from part[0].
template <typename V, typename W, typename I>
__global__ void __launch_bounds__(1024) k_update(SetArgs<V, W, I> a, int j, double scale) {
  const int t = xcd_block(blockIdx.x, gridDim.x);
  const int s = a.tile_sys[t];
  SysState& S = a.ss[s];
  if (S.done) return;
  const int r0 = a.tile_r0[t], r1 = a.tile_r1[t];
  const int t0 = a.sys_tile0[s], t1 = a.sys_tile0[s + 1];
  V* __restrict__ p = a.p[0];
  V* __restrict__ z = a.z[0];
  const V* __restrict__ q = a.q[0];
  V* __restrict__ xacc = a.xacc;
  int base = r0 + (int)threadIdx.x;
  V xa[kUnroll], pp[kUnroll], zz[kUnroll], qq[kUnroll];
  auto load = [&](int b0) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int i = b0 + u * (int)blockDim.x;
      const int jj = i < r1 ? i : r0;
      xa[u] = xacc[jj];
      pp[u] = p[jj];
      zz[u] = z[jj];
      qq[u] = q[jj];
    }
  };
  load(base);
  PartRegs P;
  partial_load(a.part[0], t0, t1, P);
  double r[4];
  partial_reduce(a.part[0], t0, t1, P, r);
  const bool first = t == t0 && threadIdx.x == 0;
  const int k = S.iter_base + j;
  const double pq = r[0], rho = r[3];
  if (const int stop = stop_code(k, S.max_it, pq, rho)) {
    if (first) {
      S.status = stop == 100 ? PM_OK : stop;
      S.done = 1;
    }
    return;
  }
  const double al = rho / pq;
  const double rn = rho - 2.0 * al * r[1] + al * al * r[2];
  const double be = rn / rho;
  const double as = al * scale, bs = be * scale;
  while (base < r1) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int i = base + u * (int)blockDim.x;
      if (i >= r1) continue;
      const double pi = (double)pp[u];
      xacc[i] = (V)((double)xa[u] + as * pi);
      const V zv = (V)((double)zz[u] - as * (double)qq[u]);
      z[i] = zv;
      p[i] = (V)((double)zv + bs * pi);
    }
    base += kUnroll * (int)blockDim.x;
    if (base < r1) load(base);
  }
  if (first) {
    S.alpha = al;
    S.beta = be;
    S.rho = rho;
    S.iter = k;
  }
}

// ---------------------------------------------------------------------------
// Chebyshev-preconditioned schedule.  z = p(D'^{-1} A) D'^{-1} r replaces
// z = D'^{-1} r: y = D'^{-1} r is kept apart, z_1 = y / theta, and
//   z_{i+1} = z_i + omega_i (z_i - z_{i-1}) + gamma_i (y - D'^{-1} A z_i)
// (the three-term form of Chebyshev acceleration from z_0 = 0; the host
// computes omega_i, gamma_i).  Per CG iteration: k_cheb_dir (new direction
// and its product), k_cheb_update (x_acc, y, z_1) and degree - 1 steps
// k_cheb_step, the last of which forms the partials of rho = r.z.
// ---------------------------------------------------------------------------

// Iteration k = iter_base + j: rho_k from the last step's partials (part[1]),
// beta = rho_k / rho_{k-1} (rho_0 = inf: beta = 0), p = z + beta p_old and
// q~ = D'^{-1} A p with the tile partials of p.q in part[0].  A neighbour's
// new p is recomputed from its z and old p with the same expression.
template <typename V, typename W, typename I>
__global__ void __launch_bounds__(1024) k_cheb_dir(SetArgs<V, W, I> a, int zb, int j) {
  const int t = xcd_block(blockIdx.x, gridDim.x);
  const int s = a.tile_sys[t];
  SysState& S = a.ss[s];
  if (S.done) return;
  const int r0 = a.tile_r0[t], r1 = a.tile_r1[t];
  const int t0 = a.sys_tile0[s], t1 = a.sys_tile0[s + 1];
  const int k = S.iter_base + j;
  double r[4];
  sum_range<4>(a.part[1], t0, t1, r);
  const double rho = r[0];
  const bool first = t == t0 && threadIdx.x == 0;
  if (!(rho > 0.0) || !isfinite(rho)) {  // zero residual, or a preconditioner breakdown
    if (first) {
      S.status = rho == 0.0 ? PM_OK : PM_BREAKDOWN;
      S.done = 1;
    }
    return;
  }
  const double be = rho / S.rho_ring[(k - 1) & 1];
  const int N = a.N;
  const V* __restrict__ z = a.zc[zb];
  const V* __restrict__ po = a.p[(k - 1) & 1];
  V* __restrict__ pn = a.p[k & 1];
  V* __restrict__ q = a.q[0];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int base = r0 + threadIdx.x; base < r1; base += kUnroll * blockDim.x) {
    int row[kUnroll];
    W w0[kUnroll], w1[kUnroll], w2[kUnroll], cc[kUnroll];
    I i0[kUnroll], i1[kUnroll], i2[kUnroll];
    V zv[kUnroll], pv[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int i0r = base + u * (int)blockDim.x;
      row[u] = i0r < r1 ? i0r : -1;
      const int i = i0r < r1 ? i0r : r0;
      w0[u] = a.w[i];
      w1[u] = a.w[(size_t)N + i];
      w2[u] = a.w[2 * (size_t)N + i];
      i0[u] = a.idx[i];
      i1[u] = a.idx[(size_t)N + i];
      i2[u] = a.idx[2 * (size_t)N + i];
      cc[u] = a.c[i];
      zv[u] = z[i];
      pv[u] = po[i];
    }
    double g[3][kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int i = row[u] >= 0 ? row[u] : r0;
      const int js[3] = {col_of<I>(i, i0[u]), col_of<I>(i, i1[u]), col_of<I>(i, i2[u])};
#pragma unroll
      for (int e = 0; e < 3; ++e) g[e][u] = (double)(V)((double)z[js[e]] + be * (double)po[js[e]]);
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      if (row[u] < 0) continue;
      const V pnv = (V)((double)zv[u] + be * (double)pv[u]);
      pn[row[u]] = pnv;
      const double pi = (double)pnv, ci = (double)cc[u];
      double yv = ci * pi;
      yv += (double)w0[u] * (pi - g[0][u]);
      yv += (double)w1[u] * (pi - g[1][u]);
      yv += (double)w2[u] * (pi - g[2][u]);
      const double d = ((ci + (double)w0[u]) + (double)w1[u]) + (double)w2[u];
      const V qv = (V)(yv / d);
      q[row[u]] = qv;
      acc[0] += pi * (d * (double)qv);
    }
  }
  tile_partial<4>(acc, a.part[0] + 4 * (size_t)t);
  if (first) {
    S.rho_ring[k & 1] = rho;
    S.rho = rho;
    S.beta = be;
  }
}

// Iteration k = iter_base + j: alpha = rho_k / p.q; x_acc += alpha p,
// y -= alpha q~ and z_1 = y / theta, or on the chunk's last iteration (FLUSH)
// (x_hi, x_lo) += x_acc + alpha p, y and z_1 then coming from the true residual.
template <typename V, typename W, typename I, bool FLUSH>
__global__ void __launch_bounds__(1024) k_cheb_update(SetArgs<V, W, I> a, int j,
                                                      double inv_theta) {
  const int t = xcd_block(blockIdx.x, gridDim.x);
  const int s = a.tile_sys[t];
  SysState& S = a.ss[s];
  if (S.done) return;
  const int r0 = a.tile_r0[t], r1 = a.tile_r1[t];
  const int t0 = a.sys_tile0[s], t1 = a.sys_tile0[s + 1];
  double r[4];
  sum_range<4>(a.part[0], t0, t1, r);
  const bool first = t == t0 && threadIdx.x == 0;
  const int k = S.iter_base + j;
  const double pq = r[0], rho = S.rho_ring[k & 1];
  if (const int stop = stop_code(k, S.max_it, pq, rho)) {
    if (first) {
      S.status = stop == 100 ? PM_OK : stop;
      S.done = 1;
    }
    return;
  }
  const double al = rho / pq;
  const V* __restrict__ p = a.p[k & 1];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
    const double pi = (double)p[i];
    if (FLUSH) {
      double hi = a.x64[i], lo = a.xlo[i];
      dd_add(hi, lo, (double)a.xacc[i] + al * pi);
      a.x64[i] = hi;
      a.xlo[i] = lo;
      a.xacc[i] = V(0);
      const double yr = (double)a.y[i] - al * (double)a.q[0][i];  // recursive residual
      acc[0] += a.dp[i] * yr * yr;
    } else {
      a.xacc[i] = (V)((double)a.xacc[i] + al * pi);
      const V yv = (V)((double)a.y[i] - al * (double)a.q[0][i]);
      a.y[i] = yv;
      a.zc[1][i] = (V)((double)yv * inv_theta);
    }
  }
  // the flush's partials go to part[1] (free until the next steps): this
  // kernel's blocks are still reading part[0]
  if (FLUSH) tile_partial<4>(acc, a.part[1] + 4 * (size_t)t);
  if (first) {
    S.alpha = al;
    S.iter = k;
  }
}

// One Chebyshev step z_out = z_in + omega (z_in - z_prev) + gamma (y - D'^{-1}
// A z_in) (z_prev = 0 when from_zero); the last step of an application also
// forms the tile partials of rho = r.z = sum d' y z_out in part[1].
template <typename V, typename W, typename I>
__global__ void __launch_bounds__(1024) k_cheb_step(SetArgs<V, W, I> a, int zin, int zprev,
                                                    int zout, double omega, double gamma,
                                                    int from_zero, int last) {
  const int t = xcd_block(blockIdx.x, gridDim.x);
  const int s = a.tile_sys[t];
  if (a.ss[s].done) return;
  const int r0 = a.tile_r0[t], r1 = a.tile_r1[t];
  const int N = a.N;
  const V* __restrict__ zi_ = a.zc[zin];
  const V* __restrict__ zp_ = a.zc[zprev];
  V* __restrict__ zo_ = a.zc[zout];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int base = r0 + threadIdx.x; base < r1; base += kUnroll * blockDim.x) {
    int row[kUnroll];
    W w0[kUnroll], w1[kUnroll], w2[kUnroll], cc[kUnroll];
    I i0[kUnroll], i1[kUnroll], i2[kUnroll];
    V zv[kUnroll], zp[kUnroll], yv[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int i0r = base + u * (int)blockDim.x;
      row[u] = i0r < r1 ? i0r : -1;
      const int i = i0r < r1 ? i0r : r0;
      w0[u] = a.w[i];
      w1[u] = a.w[(size_t)N + i];
      w2[u] = a.w[2 * (size_t)N + i];
      i0[u] = a.idx[i];
      i1[u] = a.idx[(size_t)N + i];
      i2[u] = a.idx[2 * (size_t)N + i];
      cc[u] = a.c[i];
      zv[u] = zi_[i];
      zp[u] = from_zero ? V(0) : zp_[i];
      yv[u] = a.y[i];
    }
    V g0[kUnroll], g1[kUnroll], g2[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int i = row[u] >= 0 ? row[u] : r0;
      g0[u] = zi_[col_of<I>(i, i0[u])];
      g1[u] = zi_[col_of<I>(i, i1[u])];
      g2[u] = zi_[col_of<I>(i, i2[u])];
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      if (row[u] < 0) continue;
      const double zi = (double)zv[u], ci = (double)cc[u];
      double az = ci * zi;
      az += (double)w0[u] * (zi - (double)g0[u]);
      az += (double)w1[u] * (zi - (double)g1[u]);
      az += (double)w2[u] * (zi - (double)g2[u]);
      const double d = ((ci + (double)w0[u]) + (double)w1[u]) + (double)w2[u];
      const double yi = (double)yv[u];
      const V zo = (V)(zi + omega * (zi - (double)zp[u]) + gamma * (yi - az / d));
      zo_[row[u]] = zo;
      acc[0] += d * yi * (double)zo;
    }
  }
  if (last) tile_partial<4>(acc, a.part[1] + 4 * (size_t)t);
}

// Last iteration of a chunk (k = iter_base + m): the same scalars from the
// partials in part[src], then (x_hi, x_lo) += x_acc + alpha p and x_acc = 0;
// z and p are rebuilt from the true residual afterwards.
template <typename V, typename W, typename I>
__global__ void __launch_bounds__(1024) k_update_flush(SetArgs<V, W, I> a, int src, int j) {
  const int t = xcd_block(blockIdx.x, gridDim.x);
  const int s = a.tile_sys[t];
  SysState& S = a.ss[s];
  if (S.done) return;
  double r[4];
  sum_range<4>(a.part[src], a.sys_tile0[s], a.sys_tile0[s + 1], r);
  const bool first = t == a.sys_tile0[s] && threadIdx.x == 0;
  const int k = S.iter_base + j;
  const double pq = r[0], rho = r[3];
  if (const int stop = stop_code(k, S.max_it, pq, rho)) {
    if (first) {
      S.status = stop == 100 ? PM_OK : stop;
      S.done = 1;
    }
    return;
  }
  const double al = rho / pq;
  const double rn = rho - 2.0 * al * r[1] + al * al * r[2];
  const double be = rn / rho;
  const V* __restrict__ ps = a.p[src];
  const int r0 = a.tile_r0[t], r1 = a.tile_r1[t];
  for (int base = r0 + threadIdx.x; base < r1; base += kUnroll * blockDim.x) {
    double xa[kUnroll], pp[kUnroll], hi[kUnroll], lo[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int i = base + u * (int)blockDim.x;
      const int jj = i < r1 ? i : r0;
      xa[u] = (double)a.xacc[jj];
      pp[u] = (double)ps[jj];
      hi[u] = a.x64[jj];
      lo[u] = a.xlo[jj];
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int i = base + u * (int)blockDim.x;
      if (i >= r1) continue;
      dd_add(hi[u], lo[u], xa[u] + al * pp[u]);
      a.x64[i] = hi[u];
      a.xlo[i] = lo[u];
      a.xacc[i] = V(0);
    }
  }
  if (first) {
    S.alpha = al;
    S.beta = be;
    S.rho = rho;
    S.nu_rec = rn;  // r.D'^{-1}r of the recursive residual after this update
    S.iter = k;
  }
}

// End of solve: fold pending increments (limit or breakdown mid-chunk).
template <typename V, typename W, typename I>
__global__ void __launch_bounds__(1024) k_flush(SetArgs<V, W, I> a) {
  const int t = xcd_block(blockIdx.x, gridDim.x);
  for (int i = a.tile_r0[t] + threadIdx.x; i < a.tile_r1[t]; i += blockDim.x) {
    double hi = a.x64[i], lo = a.xlo[i];
    dd_add(hi, lo, (double)a.xacc[i]);
    a.x64[i] = hi;
    a.xlo[i] = lo;
    a.xacc[i] = V(0);
  }
}

template <typename V, typename W, typename I>
__global__ void __launch_bounds__(1024) k_scatter(SetArgs<V, W, I> a) {
  const int t = xcd_block(blockIdx.x, gridDim.x);
  const bool zero = a.ss[a.tile_sys[t]].done == 2;
  for (int i = a.tile_r0[t] + threadIdx.x; i < a.tile_r1[t]; i += blockDim.x)
    a.x[a.perm[i]] = zero ? 0.0 : a.x64[i];
}

// Timing support: let the iteration kernels run again on a finished state.
__global__ void k_timing_state(SysState* ss, int n_sys) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_sys) return;
  ss[s].done = 0;
  ss[s].status = PM_OK;
  ss[s].max_it = INT_MAX;
  ss[s].iter = 0;
  ss[s].iter_base = 0;
  ss[s].tol2 = -1.0;
}

// ---------------------------------------------------------------------------
// Host driver
// ---------------------------------------------------------------------------

#define PS_HIP(expr)                                                                  \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess) {                                                           \
      set_error(PM_HIP_ERROR, std::string(#expr) + ": " + hipGetErrorString(e_));     \
      return PM_HIP_ERROR;                                                            \
    }                                                                                 \
  } while (0)

namespace {

constexpr int kMinTile = 256;

template <typename T>
int salloc(SolveSet& S, T** ptr, size_t count) {
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, std::max<size_t>(count, 1) * sizeof(T));
  if (e != hipSuccess) {
    set_error(PM_HIP_ERROR, std::string("hipMalloc: ") + hipGetErrorString(e));
    return PM_HIP_ERROR;
  }
  S.allocs.push_back(p);
  *ptr = static_cast<T*>(p);
  return PM_OK;
}

// Column window of every tile: min and max column over its rows (the CSR
// holds the diagonal, so the rows themselves are inside).
__global__ void k_tile_window(const int* tile_r0, const int* tile_r1, const int* rp,
                              const int* col, int* lo, int* hi) {
  __shared__ int smn[16], smx[16];
  const int t = blockIdx.x;
  int mn = INT_MAX, mx = -1;
  for (int i = tile_r0[t] + threadIdx.x; i < tile_r1[t]; i += blockDim.x)
    for (int k = rp[i]; k < rp[i + 1]; ++k) {
      mn = min(mn, col[k]);
      mx = max(mx, col[k]);
    }
  for (int off = 32; off > 0; off >>= 1) {
    mn = min(mn, __shfl_xor(mn, off, 64));
    mx = max(mx, __shfl_xor(mx, off, 64));
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  if (lane == 0) {
    smn[wid] = mn;
    smx[wid] = mx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < nw; ++w) {
      mn = min(mn, smn[w]);
      mx = max(mx, smx[w]);
    }
    lo[t] = mn;
    hi[t] = mx;
  }
}

int build_tiles(SolveSet& S, int tile_rows) {
  if (S.tile_rows == tile_rows) return PM_OK;
  std::vector<int> ts, t0, t1, st0(S.n_sys + 1);
  for (int s = 0; s < S.n_sys; ++s) {
    st0[s] = (int)ts.size();
    for (int r = S.row0[s]; r < S.row0[s + 1]; r += tile_rows) {
      ts.push_back(s);
      t0.push_back(r);
      t1.push_back(std::min(S.row0[s + 1], r + tile_rows));
    }
  }
  st0[S.n_sys] = (int)ts.size();
  if ((int)ts.size() > S.max_tiles) {
    set_error(PM_INVALID_ARG, "tile size below the minimum");
    return PM_INVALID_ARG;
  }
  PS_HIP(hipMemcpy(S.tile_sys, ts.data(), 4 * ts.size(), hipMemcpyHostToDevice));
  PS_HIP(hipMemcpy(S.tile_r0, t0.data(), 4 * t0.size(), hipMemcpyHostToDevice));
  PS_HIP(hipMemcpy(S.tile_r1, t1.data(), 4 * t1.size(), hipMemcpyHostToDevice));
  PS_HIP(hipMemcpy(S.sys_tile0, st0.data(), 4 * st0.size(), hipMemcpyHostToDevice));
  const int nt = (int)ts.size();
  k_tile_window<<<nt, 256>>>(S.tile_r0, S.tile_r1, S.rp, S.col, S.tile_lo, S.tile_hi);
  PS_HIP(hipGetLastError());
  std::vector<int> lo(nt), hi(nt);
  PS_HIP(hipMemcpy(lo.data(), S.tile_lo, 4 * (size_t)nt, hipMemcpyDeviceToHost));
  PS_HIP(hipMemcpy(hi.data(), S.tile_hi, 4 * (size_t)nt, hipMemcpyDeviceToHost));
  S.win_max = 0;
  for (int k = 0; k < nt; ++k) S.win_max = std::max(S.win_max, hi[k] - lo[k] + 1);
  // published rows: those at or below the highest column of an earlier tile
  // of the system, and those at or above the lowest column of a later one
  std::vector<int> plo(nt), phi(nt);
  for (int sy = 0; sy < S.n_sys; ++sy) {
    int run = INT_MIN;
    for (int k = st0[sy]; k < st0[sy + 1]; ++k) {
      plo[k] = run == INT_MIN ? INT_MIN : run + 1;
      run = std::max(run, hi[k]);
    }
    run = INT_MAX;
    for (int k = st0[sy + 1] - 1; k >= st0[sy]; --k) {
      phi[k] = run;
      run = std::min(run, lo[k]);
    }
  }
  PS_HIP(hipMemcpy(S.tile_pub_lo, plo.data(), 4 * (size_t)nt, hipMemcpyHostToDevice));
  PS_HIP(hipMemcpy(S.tile_pub_hi, phi.data(), 4 * (size_t)nt, hipMemcpyHostToDevice));
  S.tile_rows = tile_rows;
  S.n_tiles = nt;
  return PM_OK;
}

template <typename V, typename W, typename I>
SetArgs<V, W, I> make_args(SolveSet& S, const double* val, const double* b, double* x) {
  SetArgs<V, W, I> a;
  a.N = S.N;
  a.n_sys = S.n_sys;
  a.tile_sys = S.tile_sys;
  a.tile_r0 = S.tile_r0;
  a.tile_r1 = S.tile_r1;
  a.sys_tile0 = S.sys_tile0;
  a.tile_lo = S.tile_lo;
  a.tile_hi = S.tile_hi;
  a.tile_pub_lo = S.tile_pub_lo;
  a.tile_pub_hi = S.tile_pub_hi;
  a.perm = S.perm;
  a.rp = S.rp;
  a.col = S.col;
  a.val = val;
  a.b = b;
  a.x = x;
  a.c = (W*)S.c;
  a.w = (W*)S.w;
  a.idx = (I*)S.idx;
  a.dp = S.dp;
  a.x64 = S.x64;
  a.xlo = S.xlo;
  a.b64 = S.b64;
  a.xacc = (V*)S.xacc;
  for (int k = 0; k < 2; ++k) {
    a.p[k] = (V*)S.p[k];
    a.z[k] = (V*)S.z[k];
    a.q[k] = (V*)S.q[k];
    a.part[k] = S.part[k];
  }
  a.part3 = S.part3;
  a.y = (V*)S.y;
  for (int k = 0; k < 3; ++k) a.zc[k] = (V*)S.zc[k];
  a.ss = S.ss;
  a.flags = S.flags;
  return a;
}

// Chebyshev coefficients: the interval [b / 30, b] with b = 2 (Gershgorin
// bound of D^{-1} A), theta and delta its centre and half width; step i of
// the three-term form uses omega_i = rho_{i-1} rho_{i-2} and gamma_i =
// 2 rho_{i-1} / delta with rho_0 = delta / theta, rho_i = 1 / (2 theta /
// delta - rho_{i-1}).
constexpr int kMaxChebDegree = 16;
struct Cheb {
  int degree = 0;
  double inv_theta = 0.0;
  double omega[kMaxChebDegree + 1] = {}, gamma[kMaxChebDegree + 1] = {};
};

Cheb make_cheb(int degree) {
  Cheb C;
  C.degree = degree;
  const double b = 2.0, a = b / 30.0;
  const double theta = 0.5 * (b + a), delta = 0.5 * (b - a), sigma = theta / delta;
  C.inv_theta = 1.0 / theta;
  double rho[kMaxChebDegree + 1];
  rho[0] = 1.0 / sigma;
  for (int i = 1; i <= kMaxChebDegree; ++i) rho[i] = 1.0 / (2.0 * sigma - rho[i - 1]);
  for (int i = 2; i <= degree; ++i) {
    C.omega[i] = rho[i - 1] * rho[i - 2];
    C.gamma[i] = 2.0 * rho[i - 1] / delta;
  }
  return C;
}

// Launch shape: rows per tile, threads per block, rows per thread and trip of
// the fused iteration kernel (0: split schedule, k_update then k_spmv).
struct Launch {
  int tile, block, rows;
};
// Launch.rows of the resident chunk kernel (k_chunk) and of the resident
// window kernel (k_chunk_win)
constexpr int kResident = 4;
constexpr int kResidentWin = 5;
inline bool is_resident(int rows) { return rows == kResident || rows == kResidentWin; }

template <typename V, typename W, typename I>
struct Ops {
  using A = SetArgs<V, W, I>;
  static void flags_reset(SolveSet& S, hipStream_t s) {
    k_flags_reset<<<(S.n_tiles + 255) / 256, 256, 0, s>>>(S.flags, S.n_tiles);
  }
  static void start(SolveSet& S, const A& a, const pm_opts& o, const Launch& L, hipStream_t s) {
    if (is_resident(L.rows)) flags_reset(S, s);
    const int checks = o.stag_checks > 0 ? o.stag_checks : 40;
    const long win = (long)checks * o.replace_every;
    k_sys_init<<<(S.n_sys + 63) / 64, 64, 0, s>>>(S.ss, S.n_sys, o.max_it,
                                                  (int)std::min<long>(win, INT_MAX));
    k_prep<V, W, I><<<S.n_tiles, L.block, 0, s>>>(a, o.x0_is_zero);
    k_sys_start<V, W, I><<<S.n_sys, 256, 0, s>>>(a, o.tol);
    resid(S, a, 0, L, s);
  }
  static void resid(SolveSet& S, const A& a, int mode, const Launch& L, hipStream_t s,
                    double inv_theta = 0.0) {
    k_resid<V, W, I><<<S.n_tiles, L.block, 0, s>>>(a, mode, inv_theta);
    k_sys_check<V, W, I><<<S.n_sys, 256, 0, s>>>(a, mode, inv_theta > 0.0 ? 1 : 0);
  }
  static void spmv(SolveSet& S, const A& a, const Launch& L, hipStream_t s) {
    k_spmv<V, W, I><<<S.n_tiles, L.block, 0, s>>>(a);
  }
  // One iteration after the product of the last: the fused kernel (buffers
  // src -> src ^ 1), or the split schedule's update then product (buffer 0).
  static void iter(SolveSet& S, const A& a, int src, int j, const Launch& L, hipStream_t s,
                   double scale) {
    if (L.rows == 0) {
      k_update<V, W, I><<<S.n_tiles, L.block, 0, s>>>(a, j, scale);
      spmv(S, a, L, s);
    } else if (L.rows == 1) {
      k_iter<V, W, I, 1><<<S.n_tiles, L.block, 0, s>>>(a, src, j, scale);
    } else if (L.rows == 3) {
      k_iter_lds<V, W, I><<<S.n_tiles, L.block, lds_bytes(S), s>>>(a, src, j, scale);
    } else {
      k_iter<V, W, I, 2><<<S.n_tiles, L.block, 0, s>>>(a, src, j, scale);
    }
  }
  // m iterations: product on buffer 0, m - 1 iterations (fused: alternating
  // the buffers), the flushing m-th update, the replacement and the new
  // direction (back in buffer 0).
  static size_t lds_bytes(const SolveSet& S) { return 2 * sizeof(V) * (size_t)S.win_max; }
  // whether the LDS-staged kernel fits the current tiles, raising the kernel's
  // dynamic LDS limit when more than the default is needed
  static bool lds_fits(const SolveSet& S) {
    const size_t need = lds_bytes(S);
    if (need > (size_t)S.lds_limit) return false;
    if (need > 65536 &&
        hipFuncSetAttribute((const void*)k_iter_lds<V, W, I>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)need) != hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
    return true;
  }
  // Resident chunk kernel (Launch.rows == kResident): rows per thread, 4 or 8.
  static int resident_rpt(int tile, int block) {
    return tile <= 4 * block ? 4 : tile <= 8 * block ? 8 : 0;
  }
  static const void* resident_fn(int rpt) {
    return rpt == 4 ? (const void*)k_chunk<V, W, I, 4> : (const void*)k_chunk<V, W, I, 8>;
  }
  // whether every tile of the current set can be resident at once (one system,
  // its window in LDS, the whole grid on the device together)
  // LDS of the resident kernel: p and z of the window, q~ of the tile's
  // RPT * block row slots, and 16-bit column offsets of those rows
  static size_t resident_lds_bytes(const SolveSet& S, const Launch& L) {
    const size_t slots = (size_t)resident_rpt(L.tile, L.block) * L.block;
    return sizeof(V) * (2 * (size_t)S.win_max + slots) + (sizeof(I) == 2 ? 3 * 2 * slots : 0);
  }
  static bool resident_fits(const SolveSet& S, const Launch& L) {
    const int rpt = resident_rpt(L.tile, L.block);
    if (S.n_sys != 1 || rpt == 0 || S.n_cu <= 0) return false;
    const size_t need = resident_lds_bytes(S, L);
    if (need > (size_t)S.lds_limit) return false;
    const void* f = resident_fn(rpt);
    if (need > 65536 &&
        hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)need) !=
            hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, L.block, need) != hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
    return (long)per_cu * S.n_cu >= (long)S.n_tiles;
  }
  // resident window kernel: one system, every tile resident at once, the
  // column windows' p and z in LDS
  static size_t win_lds_bytes(const SolveSet& S) { return 2 * sizeof(V) * (size_t)S.win_max; }
  // rows per thread of the resident window kernel: 8, 16 or 32 (0: too many)
  static int win_rpt(int tile, int block) {
    return tile <= 8 * block ? 8 : tile <= 16 * block ? 16 : tile <= 32 * block ? 32 : 0;
  }
  static const void* win_fn(int rpt) {
    return rpt == 8    ? (const void*)k_chunk_win<V, W, I, 8>
           : rpt == 16 ? (const void*)k_chunk_win<V, W, I, 16>
                       : (const void*)k_chunk_win<V, W, I, 32>;
  }
  static bool win_fits(const SolveSet& S, const Launch& L) {
    const int rpt = win_rpt(L.tile, L.block);
    if (S.n_sys != 1 || S.n_cu <= 0 || rpt == 0) return false;
    const size_t need = win_lds_bytes(S);
    if (need > (size_t)S.lds_limit) return false;
    const void* f = win_fn(rpt);
    if (need > 65536 &&
        hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)need) !=
            hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, L.block, need) != hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
    return (long)per_cu * S.n_cu >= (long)S.n_tiles;
  }
  static bool any_resident_fits(const SolveSet& S, const Launch& L) {
    return L.rows == kResident ? resident_fits(S, L) : win_fits(S, L);
  }
  // iterations j0 .. j1-1 of a chunk in one resident launch (buffer (j0-1)&1 in)
  static void resident(SolveSet& S, const A& a, int j0, int j1, const Launch& L, hipStream_t s,
                       double scale) {
    if (L.rows == kResidentWin) {
      const size_t lds = win_lds_bytes(S);
      const int sp = S.resident_spins;
      switch (win_rpt(L.tile, L.block)) {
        case 8:
          k_chunk_win<V, W, I, 8><<<S.n_tiles, L.block, lds, s>>>(a, j0, j1, scale, sp);
          break;
        case 16:
          k_chunk_win<V, W, I, 16><<<S.n_tiles, L.block, lds, s>>>(a, j0, j1, scale, sp);
          break;
        default:
          k_chunk_win<V, W, I, 32><<<S.n_tiles, L.block, lds, s>>>(a, j0, j1, scale, sp);
          break;
      }
      return;
    }
    const size_t lds = resident_lds_bytes(S, L);
    if (resident_rpt(L.tile, L.block) == 4)
      k_chunk<V, W, I, 4><<<S.n_tiles, L.block, lds, s>>>(a, j0, j1, scale, S.resident_spins);
    else
      k_chunk<V, W, I, 8><<<S.n_tiles, L.block, lds, s>>>(a, j0, j1, scale, S.resident_spins);
  }
  static void chunk(SolveSet& S, const A& a, int m, const Launch& L, hipStream_t s) {
    spmv(S, a, L, s);
    int src = 0;
    if (is_resident(L.rows)) {
      if (m > 1) resident(S, a, 1, m, L, s, 1.0);
      src = (m - 1) & 1;
    } else {
      for (int j = 1; j < m; ++j) {
        iter(S, a, src, j, L, s, 1.0);
        if (L.rows != 0) src ^= 1;
      }
    }
    k_update_flush<V, W, I><<<S.n_tiles, L.block, 0, s>>>(a, src, m);
    resid(S, a, 1, L, s);
    k_pdir<V, W, I><<<S.n_tiles, L.block, 0, s>>>(a, src);
  }
  // Chebyshev schedule (see k_cheb_dir).  degree - 1 steps from z_1 build z
  // in buffer degree % 3; the last one forms the partials of r.z.
  static void cheb_steps(SolveSet& S, const A& a, const Launch& L, hipStream_t s,
                         const Cheb& C) {
    for (int i = 2; i <= C.degree; ++i)
      k_cheb_step<V, W, I><<<S.n_tiles, L.block, 0, s>>>(a, (i - 1) % 3, (i - 2) % 3, i % 3,
                                                         C.omega[i], C.gamma[i], i == 2 ? 1 : 0,
                                                         i == C.degree ? 1 : 0);
  }
  static void cheb_start(SolveSet& S, const A& a, const pm_opts& o, const Launch& L,
                         hipStream_t s, const Cheb& C) {
    const int checks = o.stag_checks > 0 ? o.stag_checks : 40;
    const long win = (long)checks * o.replace_every;
    k_sys_init<<<(S.n_sys + 63) / 64, 64, 0, s>>>(S.ss, S.n_sys, o.max_it,
                                                  (int)std::min<long>(win, INT_MAX));
    k_prep<V, W, I><<<S.n_tiles, L.block, 0, s>>>(a, o.x0_is_zero);
    k_sys_start<V, W, I><<<S.n_sys, 256, 0, s>>>(a, o.tol);
    resid(S, a, 0, L, s, C.inv_theta);
    cheb_steps(S, a, L, s, C);
  }
  static void cheb_chunk(SolveSet& S, const A& a, int m, const Launch& L, hipStream_t s,
                         const Cheb& C) {
    for (int j = 1; j <= m; ++j) {
      k_cheb_dir<V, W, I><<<S.n_tiles, L.block, 0, s>>>(a, C.degree % 3, j);
      if (j < m) {
        k_cheb_update<V, W, I, false><<<S.n_tiles, L.block, 0, s>>>(a, j, C.inv_theta);
        cheb_steps(S, a, L, s, C);
      } else {
        k_cheb_update<V, W, I, true><<<S.n_tiles, L.block, 0, s>>>(a, j, C.inv_theta);
      }
    }
    resid(S, a, 1, L, s, C.inv_theta);
    cheb_steps(S, a, L, s, C);
  }
  static void finish(SolveSet& S, const A& a, const Launch& L, hipStream_t s) {
    k_flush<V, W, I><<<S.n_tiles, L.block, 0, s>>>(a);
    resid(S, a, 2, L, s);
    k_scatter<V, W, I><<<S.n_tiles, L.block, 0, s>>>(a);
  }
};

// Launch shapes tried by the tuner (timing the fused iteration kernel on the
// real matrix); the choice is cached per problem shape and precision.
constexpr Launch kCandidates[] = {
    {1024, 256, 1}, {2048, 256, 1}, {2048, 512, 1}, {4096, 512, 1}, {2048, 256, 2},
    {4096, 512, 2}, {8192, 512, 2}, {2048, 256, 0}, {4096, 256, 0}, {4096, 512, 0},
    {1024, 256, 3}, {2048, 256, 3}, {2048, 512, 3}, {4096, 512, 3}, {8192, 512, 3},
    {2048, 256, 4}, {2048, 512, 4}, {4096, 512, 4},
};
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int, int>, Launch> g_tuned;

template <typename V, typename W, typename I>
int tune_launch(SolveSet& S, const double* val64, const double* b, double* x, const pm_opts& o,
                hipStream_t s, Launch* best_launch) {
  const auto key = std::make_tuple(S.N, S.n_sys, o.precision, S.index_bits);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(key);
    if (it != g_tuned.end()) {
      *best_launch = it->second;
      return PM_OK;
    }
  }
  double best = 1e300;
  Launch arg = {2048, 256, 0};
  pm_opts ot = o;
  ot.max_it = INT_MAX;
  std::vector<Launch> cands(std::begin(kCandidates), std::end(kCandidates));
  // the resident window kernel with one tile per compute unit
  if (S.n_sys == 1 && S.n_cu > 0)
    cands.push_back({std::max(kMinTile, (S.N + S.n_cu - 1) / S.n_cu), 512, kResidentWin});
  for (const Launch& L : cands) {
    if (L.rows != kResidentWin && (long)L.tile * 2 > (long)S.N && L.tile != kCandidates[0].tile)
      continue;
    if (int r = build_tiles(S, L.tile)) return r;
    if (L.rows == 3 && !Ops<V, W, I>::lds_fits(S)) continue;
    if (is_resident(L.rows) && !Ops<V, W, I>::any_resident_fits(S, L)) continue;
    const auto a = make_args<V, W, I>(S, val64, b, x);
    Ops<V, W, I>::start(S, a, ot, L, s);
    Ops<V, W, I>::spmv(S, a, L, s);
    const bool res = is_resident(L.rows);
    // warm caches and clocks (the resident kernel's iteration numbers keep
    // increasing from launch to launch, as in a solve)
    if (res) Ops<V, W, I>::resident(S, a, 1, 5, L, s, 0.0);
    else
      for (int w = 0; w < 4; ++w) Ops<V, W, I>::iter(S, a, w & 1, 1, L, s, 0.0);
    // best of three rounds of twenty iterations: single rounds vary by a few
    // per cent, as much as neighbouring shapes differ
    float ms = 1e30f;
    for (int round = 0; round < 3; ++round) {
      PS_HIP(hipEventRecord(S.tev[0], s));
      if (res) Ops<V, W, I>::resident(S, a, 5 + 20 * round, 25 + 20 * round, L, s, 0.0);
      else
        for (int w = 0; w < 20; ++w) Ops<V, W, I>::iter(S, a, w & 1, 1, L, s, 0.0);
      PS_HIP(hipEventRecord(S.tev[1], s));
      PS_HIP(hipEventSynchronize(S.tev[1]));
      float r = 0.f;
      PS_HIP(hipEventElapsedTime(&r, S.tev[0], S.tev[1]));
      ms = std::min(ms, r);
    }
    if (ms < best) {
      best = ms;
      arg = L;
    }
  }
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tuned[key] = arg;
  *best_launch = arg;
  return PM_OK;
}

template <typename V, typename W, typename I>
int run(SolveSet& S, const double* val64, const double* b, double* x, const pm_opts& o,
        pm_info* infos, hipStream_t s, const Launch* force = nullptr, int pass = 0) {
  using O = Ops<V, W, I>;
  // bound of the resident kernel's barrier waits; PMCORR_RESIDENT_SPINS
  // overrides it (a diagnostic knob: 0 makes every wait give up at once)
  {
    const char* e = std::getenv("PMCORR_RESIDENT_SPINS");
    S.resident_spins = e ? std::max(0, std::atoi(e)) : 1 << 20;
  }
  Launch L;
  bool tuned = false;
  if (force) {
    L = *force;
  } else if (o.tile_rows > 0) {
    const int block = o.block > 0 ? std::min(512, std::max(64, (o.block / 64) * 64)) : 256;
    L = {std::max(kMinTile, o.tile_rows), block, o.iter_shape < 0 ? 0 : std::max(1, o.iter_shape)};
    if (o.precond == PM_PREC_CHEBYSHEV) L.rows = 1;  // the schedule applies to Jacobi only
  } else {
    if (int r = tune_launch<V, W, I>(S, val64, b, x, o, s, &L)) return r;
    tuned = true;
  }
  if (int r = build_tiles(S, L.tile)) return r;
  if (L.rows == 3 && !O::lds_fits(S)) {
    set_error(PM_INVALID_ARG, "the tile's column window does not fit the LDS of one block");
    return PM_INVALID_ARG;
  }
  if (is_resident(L.rows) && !O::any_resident_fits(S, L)) {
    set_error(PM_INVALID_ARG,
              "the resident schedule needs one system whose tiles all fit the device at once");
    return PM_INVALID_ARG;
  }
  const auto a = make_args<V, W, I>(S, val64, b, x);
  S.last_prec = o.precision;
  S.last_tile = L.tile;
  S.last_block = L.block;
  S.last_rows = L.rows;
  S.last_val = val64;

  const bool cheb = o.precond == PM_PREC_CHEBYSHEV;
  const Cheb C = make_cheb(cheb ? o.cheb_degree : 0);
  const int pc = cheb ? 100 + o.cheb_degree : 0;
  S.last_pc = pc;
  if (cheb) O::cheb_start(S, a, o, L, s, C);
  else O::start(S, a, o, L, s);
  PS_HIP(hipGetLastError());

  if (!S.graph || S.g_prec != o.precision || S.g_m != o.replace_every || S.g_tile != L.tile ||
      S.g_block != L.block || S.g_rows != L.rows || S.g_pc != pc || S.g_val != val64 ||
      S.g_spins != S.resident_spins) {
    if (S.graph) {
      (void)hipGraphExecDestroy(S.graph);
      S.graph = nullptr;
    }
    hipGraph_t g = nullptr;
    PS_HIP(hipStreamBeginCapture(S.cap, hipStreamCaptureModeThreadLocal));
    if (cheb) O::cheb_chunk(S, a, o.replace_every, L, S.cap, C);
    else O::chunk(S, a, o.replace_every, L, S.cap);
    PS_HIP(hipStreamEndCapture(S.cap, &g));
    PS_HIP(hipGraphInstantiate(&S.graph, g, nullptr, nullptr, 0));
    (void)hipGraphDestroy(g);
    S.g_prec = o.precision;
    S.g_m = o.replace_every;
    S.g_spins = S.resident_spins;
    S.g_tile = L.tile;
    S.g_block = L.block;
    S.g_rows = L.rows;
    S.g_pc = pc;
    S.g_val = val64;
  }

  // replay chunks; poll the stop flags one chunk behind so the GPU stays busy
  const size_t bytes = sizeof(SysState) * S.n_sys;
  SysState* slot[2] = {S.h_ss, S.h_ss + S.n_sys};
  auto all_done = [&](const SysState* st) {
    for (int k = 0; k < S.n_sys; ++k)
      if (!st[k].done) return false;
    return true;
  };
  PS_HIP(hipMemcpyAsync(slot[0], S.ss, bytes, hipMemcpyDeviceToHost, s));
  PS_HIP(hipEventRecord(S.ev[0], s));
  PS_HIP(hipEventSynchronize(S.ev[0]));
  bool stop = all_done(slot[0]);
  const long max_chunks = (long)o.max_it / o.replace_every + 3;
  long c = 0;
  while (!stop && c < max_chunks) {
    PS_HIP(hipGraphLaunch(S.graph, s));
    const int k = (int)(c & 1);
    PS_HIP(hipMemcpyAsync(slot[k], S.ss, bytes, hipMemcpyDeviceToHost, s));
    PS_HIP(hipEventRecord(S.ev[k], s));
    if (c >= 1) {
      PS_HIP(hipEventSynchronize(S.ev[k ^ 1]));
      if (all_done(slot[k ^ 1])) stop = true;
    }
    ++c;
  }
  O::finish(S, a, L, s);
  PS_HIP(hipGetLastError());
  SysState* fin = S.h_ss + 2 * S.n_sys;
  PS_HIP(hipMemcpyAsync(fin, S.ss, bytes, hipMemcpyDeviceToHost, s));
  PS_HIP(hipStreamSynchronize(s));
  // a resident launch whose grid was not all resident at once (a barrier
  // wait gave up): solve again, from the start, on the streaming schedule
  // with the same tiles, which computes bitwise the same iterations
  if (is_resident(L.rows) && fin[0].bar_fail) {
    const Launch L2 = {L.tile, L.block, O::lds_fits(S) ? 3 : 1};
    if (tuned) {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      g_tuned[std::make_tuple(S.N, S.n_sys, o.precision, S.index_bits)] = L2;
    }
    return run<V, W, I>(S, val64, b, x, o, infos, s, &L2, pass);
  }
  // The recursion can end a solve early while the true residual, in float64,
  // misses the tolerance: with float32 storage on a system of a few rows, the
  // recursive residual reaches exactly zero (rho = 0, taken as converged), or
  // decays until p.q underflows to zero (a breakdown after progress).  Solve
  // on from the returned iterate; each pass starts again from the true
  // residual.
  if (pass < 4) {
    bool again = false;
    int used = 0;
    for (int k = 0; k < S.n_sys; ++k) {
      const SysState& f = fin[k];
      again = again || (f.done && f.res2 > f.tol2 &&
                        (f.status == PM_OK || (f.status == PM_BREAKDOWN && f.iter > 0)));
      used = std::max(used, f.iter);
    }
    if (again && used < o.max_it) {
      std::vector<int> before(S.n_sys);
      for (int k = 0; k < S.n_sys; ++k) before[k] = fin[k].iter;
      pm_opts o2 = o;
      o2.x0_is_zero = 0;
      o2.max_it = o.max_it - used;
      const int st = run<V, W, I>(S, val64, b, x, o2, infos, s, &L, pass + 1);
      if (infos)
        for (int k = 0; k < S.n_sys; ++k) infos[k].iters += before[k];
      return st;
    }
  }
  int worst = PM_OK;
  for (int k = 0; k < S.n_sys; ++k) {
    const SysState& f = fin[k];
    int status = f.done ? f.status : PM_MAXIT;
    // CG ends within n iterations in exact arithmetic; on a system of a few
    // rows the recursion then decays to p.q = 0 before the next convergence
    // test.  A returned iterate that meets the tolerance is a converged solve.
    if (status == PM_BREAKDOWN && f.res2 <= f.tol2) status = PM_OK;
    if (infos) {
      infos[k].iters = f.iter;
      infos[k].status = status;
      infos[k].bnorm = std::sqrt(f.bnorm2);
      infos[k].rel_res_true = f.bnorm2 > 0 ? std::sqrt(f.res2 / f.bnorm2) : 0.0;
    }
    if (worst == PM_OK && status != PM_OK) worst = status;
  }
  return worst;
}

}  // namespace

int set_init(SolveSet& S, const std::vector<int>& rows, int64_t nnz, int index_bits,
             const int* perm, const int* rp, const int* col) {
  S.n_sys = (int)rows.size();
  S.row0.assign(S.n_sys + 1, 0);
  S.max_tiles = 0;
  for (int k = 0; k < S.n_sys; ++k) {
    S.row0[k + 1] = S.row0[k] + rows[k];
    S.max_tiles += (rows[k] + kMinTile - 1) / kMinTile;
  }
  S.N = S.row0[S.n_sys];
  S.nnz = nnz;
  S.index_bits = index_bits;
  S.perm = perm;
  S.rp = rp;
  S.col = col;
  const size_t N = S.N, T = S.max_tiles;
  int r;
  if ((r = salloc(S, &S.tile_sys, T)) || (r = salloc(S, &S.tile_r0, T)) ||
      (r = salloc(S, &S.tile_r1, T)) || (r = salloc(S, &S.sys_tile0, S.n_sys + 1)) ||
      (r = salloc(S, &S.tile_lo, T)) || (r = salloc(S, &S.tile_hi, T)) ||
      (r = salloc(S, &S.tile_pub_lo, T)) || (r = salloc(S, &S.tile_pub_hi, T)))
    return r;
  {
    int dev = 0, lim = 0, ncu = 0;
    PS_HIP(hipGetDevice(&dev));
    PS_HIP(hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    PS_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    S.lds_limit = lim;
    S.n_cu = ncu;
  }
  double* d;
  int32_t* i32;
  if ((r = salloc(S, &d, N))) return r;
  S.c = d;
  if ((r = salloc(S, &d, 3 * N))) return r;
  S.w = d;
  if ((r = salloc(S, &i32, 3 * N))) return r;
  S.idx = i32;
  if ((r = salloc(S, &S.dp, N)) || (r = salloc(S, &S.x64, N)) || (r = salloc(S, &S.xlo, N)) ||
      (r = salloc(S, &S.b64, N)))
    return r;
  void** vecs[] = {&S.xacc, &S.p[0], &S.p[1], &S.z[0], &S.z[1], &S.q[0],
                   &S.q[1], &S.y,    &S.zc[0], &S.zc[1], &S.zc[2]};
  for (void** v : vecs) {
    if ((r = salloc(S, &d, N))) return r;
    *v = d;
  }
  if ((r = salloc(S, &S.part[0], 4 * T)) || (r = salloc(S, &S.part[1], 4 * T)) ||
      (r = salloc(S, &S.part3, 4 * T)) || (r = salloc(S, &S.ss, (size_t)S.n_sys)) ||
      (r = salloc(S, &S.flags, 16 * T)))
    return r;
  PS_HIP(hipHostMalloc((void**)&S.h_ss, 3 * sizeof(SysState) * S.n_sys, hipHostMallocDefault));
  PS_HIP(hipStreamCreateWithFlags(&S.cap, hipStreamNonBlocking));
  for (auto& e : S.ev) PS_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  for (auto& e : S.tev) PS_HIP(hipEventCreate(&e));
  return PM_OK;
}

void set_free(SolveSet& S) {
  if (S.graph) (void)hipGraphExecDestroy(S.graph);
  for (void* p : S.allocs) (void)hipFree(p);
  S.allocs.clear();
  if (S.h_ss) (void)hipHostFree(S.h_ss);
  for (auto& e : S.ev)
    if (e) (void)hipEventDestroy(e);
  for (auto& e : S.tev)
    if (e) (void)hipEventDestroy(e);
  if (S.cap) (void)hipStreamDestroy(S.cap);
  S = SolveSet();
}

int set_solve(SolveSet& S, const double* val64, const double* b, double* x, const pm_opts& o,
              pm_info* infos, hipStream_t s) {
  const bool i16 = S.index_bits == 16;
  if (o.precision == PM_FP64)
    return i16 ? run<double, double, int16_t>(S, val64, b, x, o, infos, s)
               : run<double, double, int32_t>(S, val64, b, x, o, infos, s);
  return i16 ? run<float, float, int16_t>(S, val64, b, x, o, infos, s)
             : run<float, float, int32_t>(S, val64, b, x, o, infos, s);
}

namespace {
template <typename V, typename W, typename I>
int time_kernel(SolveSet& S, int which, int n_launch, hipStream_t s, double* ms) {
  const auto a = make_args<V, W, I>(S, S.last_val, nullptr, nullptr);
  const Launch L = {S.last_tile, S.last_block, S.last_rows};
  k_timing_state<<<(S.n_sys + 63) / 64, 64, 0, s>>>(S.ss, S.n_sys);
  if (is_resident(L.rows)) Ops<V, W, I>::flags_reset(S, s);
  Ops<V, W, I>::spmv(S, a, L, s);  // partials for the first fused iteration
  PS_HIP(hipEventRecord(S.tev[0], s));
  // the resident kernel is timed as the solve runs it: launches of m - 1
  // iterations (m of the last solve); the time returned is per iteration
  const bool res = which == 1 && is_resident(L.rows);
  const int per = res ? std::max(1, S.g_m - 1) : 1;
  if (res) {
    for (int r = 0; r < n_launch; ++r)
      Ops<V, W, I>::resident(S, a, 1 + r * per, 1 + (r + 1) * per, L, s, 0.0);
  } else {
    for (int r = 0; r < n_launch; ++r) {
      if (which == 0) Ops<V, W, I>::spmv(S, a, L, s);
      else if (which == 1) Ops<V, W, I>::iter(S, a, r & 1, 1, L, s, 0.0);
      else k_resid<V, W, I><<<S.n_tiles, L.block, 0, s>>>(a, 2, 0.0);
    }
  }
  PS_HIP(hipEventRecord(S.tev[1], s));
  PS_HIP(hipGetLastError());
  PS_HIP(hipEventSynchronize(S.tev[1]));
  float t = 0.f;
  PS_HIP(hipEventElapsedTime(&t, S.tev[0], S.tev[1]));
  *ms = (double)t / ((double)n_launch * per);
  return PM_OK;
}
}  // namespace

int set_time_kernel(SolveSet& S, int which, int n_launch, hipStream_t s, double* ms,
                    double* bytes) {
  if (S.last_prec < 0 || which < 0 || which > 2 || n_launch < 1 || (which == 1 && S.last_pc)) {
    set_error(PM_INVALID_ARG, "pm_time_kernel: no solve to time or bad kernel id");
    return PM_INVALID_ARG;
  }
  if (int r = build_tiles(S, S.last_tile)) return r;
  const bool f64 = S.last_prec == PM_FP64, i16 = S.index_bits == 16;
  double t = 0.0;
  int r;
  if (f64)
    r = i16 ? time_kernel<double, double, int16_t>(S, which, n_launch, s, &t)
            : time_kernel<double, double, int32_t>(S, which, n_launch, s, &t);
  else
    r = i16 ? time_kernel<float, float, int16_t>(S, which, n_launch, s, &t)
            : time_kernel<float, float, int32_t>(S, which, n_launch, s, &t);
  if (r) return r;
  const double sv = f64 ? 8 : 4, sw = sv, si = i16 ? 2 : 4, n = S.N;
  if (ms) *ms = t;
  if (bytes) {
    if (which == 0) *bytes = n * (4 * sw + 3 * si + 3 * sv);
    else if (which == 1 && S.last_rows == 0) *bytes = n * (4 * sw + 3 * si + 10 * sv);
    else if (which == 1) *bytes = n * (4 * sw + 3 * si + 8 * sv);
    else *bytes = 12.0 * S.nnz + 4.0 * (n + 1) + 24.0 * n;
  }
  return PM_OK;
}

}  // namespace pm
