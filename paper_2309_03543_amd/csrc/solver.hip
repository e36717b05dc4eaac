// Jacobi-preconditioned CG for one or several corrector systems (gfx950).
//
// Work is cut into tiles of consecutive rows of one system; one block of
// threads owns a tile.  An iteration is two kernels:
//   k_spmv    q~ = D'^{-1} A p in difference form, fused with the four dot
//             products the iteration needs (per-tile partials)
//   k_update  every block reduces its system's partials in a fixed order
//             (identical result in every block), forms alpha and beta
//             (recurrence for the next rho, anchored on the exact rho), and
//             updates x_acc, z and p
// Every m-th iteration the increments are folded into the double-double
// solution and the residual is recomputed exactly from the float64 CSR
// matrix (k_update<FLUSH>, k_resid, k_sys_check, k_pdir).  The kernel
// boundaries are the only grid-wide synchronisation: no fences, no spin
// waits.  Chunks of m iterations are captured once in a HIP graph and
// replayed; a system whose test passes is masked out of later kernels.
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
  V* p;
  V* z;
  V* q;
  double* part4;  // [tile][4]
  double* part3;  // [tile][4], residual partials
  SysState* ss;
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

__global__ void k_sys_init(SysState* ss, int n_sys, int max_it, int stag_checks) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_sys) return;
  SysState z{};
  z.max_it = max_it;
  z.stag_checks = stag_checks;
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
    acc[0] += bi * bi;
    acc[1] += xi * xi;
  }
  if (err) atomicExch(&a.ss[s].err, err);
  tile_partial<2>(acc, a.part4 + 4 * (size_t)t);
}

// One block per system: ||b||, the tolerance, the input checks.
template <typename V, typename W, typename I>
__global__ void k_sys_start(SetArgs<V, W, I> a, double tol) {
  const int s = blockIdx.x;
  double r[2];
  sum_range<2>(a.part4, a.sys_tile0[s], a.sys_tile0[s + 1], r);
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
//   mode 0 (start):   z = r_dd/d', p = z
//   mode 1 (replace): z = r_dd/d'
//   mode 2 (final):   norms only, also for stopped systems
template <typename V, typename W, typename I>
__global__ void __launch_bounds__(1024) k_resid(SetArgs<V, W, I> a, int mode) {
  const int t = xcd_block(blockIdx.x, gridDim.x);
  const int s = a.tile_sys[t];
  if (mode != 2 && a.ss[s].done) return;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int i = a.tile_r0[t] + threadIdx.x; i < a.tile_r1[t]; i += blockDim.x) {
    double rh, rd, ax;
    residual_row(a.b64[i], a.val, a.col, a.x64, a.xlo, a.rp[i], a.rp[i + 1], rh, rd, ax);
    acc[0] += rh * rh;
    acc[2] += ax * ax;
    if (mode != 2) {
      const double d = a.dp[i];
      const V zv = (V)(rd / d);
      a.z[i] = zv;
      if (mode == 0) a.p[i] = zv;
      const double zd = (double)zv;
      acc[1] += d * zd * zd;
    }
  }
  tile_partial<3>(acc, a.part3 + 4 * (size_t)t);
}

// One block per system after k_resid: the convergence test on the returned
// vector; the stagnation test (the residual norm has not halved for
// stag_checks replacement points although it is within 1000x of the tolerance
// or of the rounding floor u*|| |A||x| ||); the scalars of the next direction.
template <typename V, typename W, typename I>
__global__ void k_sys_check(SetArgs<V, W, I> a, int mode) {
  const int s = blockIdx.x;
  SysState& S = a.ss[s];
  if (mode != 2 && S.done) return;
  if (mode == 2 && S.done == 2) return;
  double r[3];
  sum_range<3>(a.part3, a.sys_tile0[s], a.sys_tile0[s + 1], r);
  if (threadIdx.x != 0) return;
  S.res2 = r[0];
  if (mode == 2) return;
  if (!isfinite(r[0])) {
    S.status = PM_NONFINITE;
    S.done = 1;
  } else if (r[0] <= S.tol2) {
    S.status = PM_OK;
    S.done = 1;
  } else if (mode == 0) {
    S.rho = r[1];
    S.best_res2 = r[0];
    S.stall = 0;
  } else {
    if (r[0] < 0.25 * S.best_res2) {
      S.best_res2 = r[0];
      S.stall = 0;
    } else {
      S.stall += 1;
    }
    const double floor2 = 0x1p-106 * r[2];
    if (S.best_res2 < 1e6 * fmax(S.tol2, floor2) && S.stall >= S.stag_checks) {
      S.status = PM_STAGNATED;
      S.done = 1;
    } else {
      S.beta = r[1] / S.rho;
      S.rho = r[1];
    }
  }
}

// p = z + beta p after a replacement.
template <typename V, typename W, typename I>
__global__ void __launch_bounds__(1024) k_pdir(SetArgs<V, W, I> a) {
  const int t = xcd_block(blockIdx.x, gridDim.x);
  const SysState& S = a.ss[a.tile_sys[t]];
  if (S.done) return;
  const double be = S.beta;
  for (int i = a.tile_r0[t] + threadIdx.x; i < a.tile_r1[t]; i += blockDim.x)
    a.p[i] = (V)((double)a.z[i] + be * (double)a.p[i]);
}

// Rows handled per thread and loop trip: every load of the group is issued
// before the first use, so each thread keeps R rows of memory traffic in flight.
constexpr int kUnroll = 4;

// q~ = D'^{-1} A p (difference form) and, with q = D' q~ as stored, the tile
// partials of  s0 = p.q,  s1 = z.q (= q.D'^{-1} r),  s2 = q.D'^{-1} q,
// s3 = z.D' z (= rho).
template <typename V, typename W, typename I>
__global__ void __launch_bounds__(1024) k_spmv(SetArgs<V, W, I> a) {
  const int t = xcd_block(blockIdx.x, gridDim.x);
  const int s = a.tile_sys[t];
  SysState& S = a.ss[s];
  if (S.done) return;
  const int N = a.N;
  const W* __restrict__ c = a.c;
  const W* __restrict__ w = a.w;
  const I* __restrict__ idx = a.idx;
  const V* __restrict__ p = a.p;
  const V* __restrict__ z = a.z;
  V* __restrict__ q = a.q;
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
  tile_partial<4>(acc, a.part4 + 4 * (size_t)t);
  if (t == a.sys_tile0[s] && threadIdx.x == 0) S.iter_pending = S.iter + 1;
}

// Every block reduces its system's product partials (same order, same
// result): alpha = rho / p.q, the next rho by its recurrence anchored on the
// exact rho, beta = rho_next / rho; then
//   FLUSH = false:  x_acc += alpha p;  z -= alpha q~;  p = z + beta p
//   FLUSH = true :  (x_hi, x_lo) += x_acc + alpha p; x_acc = 0 (replacement
//                   iteration: z and p are rebuilt from the true residual)
// The system's first tile records the scalars and the iteration count, or
// the stop status.  `scale` multiplies alpha and beta (1 in solves, 0 when the
// kernel is timed).
template <typename V, typename W, typename I, bool FLUSH>
__global__ void __launch_bounds__(1024) k_update(SetArgs<V, W, I> a, double scale) {
  const int t = xcd_block(blockIdx.x, gridDim.x);
  const int s = a.tile_sys[t];
  SysState& S = a.ss[s];
  if (S.done) return;
  double r[4];
  sum_range<4>(a.part4, a.sys_tile0[s], a.sys_tile0[s + 1], r);
  const bool first = t == a.sys_tile0[s] && threadIdx.x == 0;
  const int k = S.iter_pending;
  const double pq = r[0], rho = r[3];
  int stop = 0;
  if (k > S.max_it) stop = PM_MAXIT;
  else if (rho == 0.0) stop = 100;  // exact zero residual in the recurrence
  else if (!(pq > 0.0) || !isfinite(pq) || !isfinite(rho)) stop = PM_BREAKDOWN;
  if (stop) {
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
  const int r0 = a.tile_r0[t], r1 = a.tile_r1[t];
  for (int base = r0 + threadIdx.x; base < r1; base += kUnroll * blockDim.x) {
    if (FLUSH) {
      double xa[kUnroll], pp[kUnroll], hi[kUnroll], lo[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int i = base + u * (int)blockDim.x;
        const int j = i < r1 ? i : r0;
        xa[u] = (double)a.xacc[j];
        pp[u] = (double)a.p[j];
        hi[u] = a.x64[j];
        lo[u] = a.xlo[j];
      }
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int i = base + u * (int)blockDim.x;
        if (i >= r1) continue;
        dd_add(hi[u], lo[u], xa[u] + as * pp[u]);
        a.x64[i] = hi[u];
        a.xlo[i] = lo[u];
        a.xacc[i] = V(0);
      }
    } else {
      V xa[kUnroll], pp[kUnroll], zz[kUnroll], qq[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int i = base + u * (int)blockDim.x;
        const int j = i < r1 ? i : r0;
        xa[u] = a.xacc[j];
        pp[u] = a.p[j];
        zz[u] = a.z[j];
        qq[u] = a.q[j];
      }
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int i = base + u * (int)blockDim.x;
        if (i >= r1) continue;
        const double pi = (double)pp[u];
        a.xacc[i] = (V)((double)xa[u] + as * pi);
        const V zv = (V)((double)zz[u] - as * (double)qq[u]);
        a.z[i] = zv;
        a.p[i] = (V)((double)zv + bs * pi);
      }
    }
  }
  if (first) {
    S.alpha = al;
    S.beta = be;
    S.rho = rho;
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
  ss[s].iter_pending = 1;
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
  S.tile_rows = tile_rows;
  S.n_tiles = (int)ts.size();
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
  a.p = (V*)S.p;
  a.z = (V*)S.z;
  a.q = (V*)S.q;
  a.part4 = S.part4;
  a.part3 = S.part3;
  a.ss = S.ss;
  return a;
}

template <typename V, typename W, typename I>
struct Ops {
  using A = SetArgs<V, W, I>;
  static void start(SolveSet& S, const A& a, const pm_opts& o, int block, hipStream_t s) {
    const int G = S.n_tiles;
    k_sys_init<<<(S.n_sys + 63) / 64, 64, 0, s>>>(S.ss, S.n_sys, o.max_it,
                                                  o.stag_checks > 0 ? o.stag_checks : 40);
    k_prep<V, W, I><<<G, block, 0, s>>>(a, o.x0_is_zero);
    k_sys_start<V, W, I><<<S.n_sys, 256, 0, s>>>(a, o.tol);
    resid(S, a, 0, block, s);
  }
  static void resid(SolveSet& S, const A& a, int mode, int block, hipStream_t s) {
    k_resid<V, W, I><<<S.n_tiles, block, 0, s>>>(a, mode);
    k_sys_check<V, W, I><<<S.n_sys, 256, 0, s>>>(a, mode);
  }
  static void spmv(SolveSet& S, const A& a, int block, hipStream_t s) {
    k_spmv<V, W, I><<<S.n_tiles, block, 0, s>>>(a);
  }
  static void update(SolveSet& S, const A& a, int block, hipStream_t s, double scale) {
    k_update<V, W, I, false><<<S.n_tiles, block, 0, s>>>(a, scale);
  }
  static void chunk(SolveSet& S, const A& a, int mrep, int block, hipStream_t s) {
    for (int it = 0; it < mrep - 1; ++it) {
      spmv(S, a, block, s);
      update(S, a, block, s, 1.0);
    }
    spmv(S, a, block, s);
    k_update<V, W, I, true><<<S.n_tiles, block, 0, s>>>(a, 1.0);
    resid(S, a, 1, block, s);
    k_pdir<V, W, I><<<S.n_tiles, block, 0, s>>>(a);
  }
  static void finish(SolveSet& S, const A& a, int block, hipStream_t s) {
    k_flush<V, W, I><<<S.n_tiles, block, 0, s>>>(a);
    resid(S, a, 2, block, s);
    k_scatter<V, W, I><<<S.n_tiles, block, 0, s>>>(a);
  }
};

// Tile sizes tried by the tuner; the choice is cached per shape.
constexpr int kTileCandidates[] = {1024, 2048, 4096, 8192};
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int, int>, int> g_tuned;

template <typename V, typename W, typename I>
int tune_tile(SolveSet& S, const double* val64, const double* b, double* x, const pm_opts& o,
              int block, hipStream_t s, int* best_tile) {
  const auto key = std::make_tuple(S.N, S.n_sys, o.precision, S.index_bits);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(key);
    if (it != g_tuned.end()) {
      *best_tile = it->second;
      return PM_OK;
    }
  }
  double best = 1e300;
  int arg = 2048;
  pm_opts ot = o;
  ot.max_it = INT_MAX;
  for (int tile : kTileCandidates) {
    if (int r = build_tiles(S, tile)) return r;
    const auto a = make_args<V, W, I>(S, val64, b, x);
    Ops<V, W, I>::start(S, a, ot, block, s);
    for (int w = 0; w < 3; ++w) {  // warm caches and clocks
      Ops<V, W, I>::spmv(S, a, block, s);
      Ops<V, W, I>::update(S, a, block, s, 0.0);
    }
    PS_HIP(hipEventRecord(S.tev[0], s));
    const int reps = 20;
    for (int w = 0; w < reps; ++w) {
      Ops<V, W, I>::spmv(S, a, block, s);
      Ops<V, W, I>::update(S, a, block, s, 0.0);
    }
    PS_HIP(hipEventRecord(S.tev[1], s));
    PS_HIP(hipEventSynchronize(S.tev[1]));
    float ms = 0.f;
    PS_HIP(hipEventElapsedTime(&ms, S.tev[0], S.tev[1]));
    if (ms < best) {
      best = ms;
      arg = tile;
    }
  }
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tuned[key] = arg;
  *best_tile = arg;
  return PM_OK;
}

template <typename V, typename W, typename I>
int run(SolveSet& S, const double* val64, const double* b, double* x, const pm_opts& o,
        pm_info* infos, hipStream_t s) {
  using O = Ops<V, W, I>;
  const int block = o.block > 0 ? std::min(1024, std::max(64, (o.block / 64) * 64)) : 256;
  int tile = o.tile_rows > 0 ? std::max(kMinTile, o.tile_rows) : 0;
  if (tile == 0) {
    if (int r = tune_tile<V, W, I>(S, val64, b, x, o, block, s, &tile)) return r;
  }
  if (int r = build_tiles(S, tile)) return r;
  const auto a = make_args<V, W, I>(S, val64, b, x);
  S.last_prec = o.precision;
  S.last_tile = tile;
  S.last_block = block;
  S.last_val = val64;

  O::start(S, a, o, block, s);
  PS_HIP(hipGetLastError());

  if (!S.graph || S.g_prec != o.precision || S.g_m != o.replace_every || S.g_tile != tile ||
      S.g_block != block || S.g_val != val64) {
    if (S.graph) {
      (void)hipGraphExecDestroy(S.graph);
      S.graph = nullptr;
    }
    hipGraph_t g = nullptr;
    PS_HIP(hipStreamBeginCapture(S.cap, hipStreamCaptureModeThreadLocal));
    O::chunk(S, a, o.replace_every, block, S.cap);
    PS_HIP(hipStreamEndCapture(S.cap, &g));
    PS_HIP(hipGraphInstantiate(&S.graph, g, nullptr, nullptr, 0));
    (void)hipGraphDestroy(g);
    S.g_prec = o.precision;
    S.g_m = o.replace_every;
    S.g_tile = tile;
    S.g_block = block;
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
  O::finish(S, a, block, s);
  PS_HIP(hipGetLastError());
  SysState* fin = S.h_ss + 2 * S.n_sys;
  PS_HIP(hipMemcpyAsync(fin, S.ss, bytes, hipMemcpyDeviceToHost, s));
  PS_HIP(hipStreamSynchronize(s));
  int worst = PM_OK;
  for (int k = 0; k < S.n_sys; ++k) {
    const SysState& f = fin[k];
    int status = f.done ? f.status : PM_MAXIT;
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
      (r = salloc(S, &S.tile_r1, T)) || (r = salloc(S, &S.sys_tile0, S.n_sys + 1)))
    return r;
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
  void** vecs[] = {&S.xacc, &S.p, &S.z, &S.q};
  for (void** v : vecs) {
    if ((r = salloc(S, &d, N))) return r;
    *v = d;
  }
  if ((r = salloc(S, &S.part4, 4 * T)) || (r = salloc(S, &S.part3, 4 * T)) ||
      (r = salloc(S, &S.ss, (size_t)S.n_sys)))
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
  const int block = S.last_block;
  k_timing_state<<<(S.n_sys + 63) / 64, 64, 0, s>>>(S.ss, S.n_sys);
  PS_HIP(hipEventRecord(S.tev[0], s));
  for (int r = 0; r < n_launch; ++r) {
    if (which == 0) Ops<V, W, I>::spmv(S, a, block, s);
    else if (which == 1) Ops<V, W, I>::update(S, a, block, s, 0.0);
    else k_resid<V, W, I><<<S.n_tiles, block, 0, s>>>(a, 2);
  }
  PS_HIP(hipEventRecord(S.tev[1], s));
  PS_HIP(hipGetLastError());
  PS_HIP(hipEventSynchronize(S.tev[1]));
  float t = 0.f;
  PS_HIP(hipEventElapsedTime(&t, S.tev[0], S.tev[1]));
  *ms = (double)t / n_launch;
  return PM_OK;
}
}  // namespace

int set_time_kernel(SolveSet& S, int which, int n_launch, hipStream_t s, double* ms,
                    double* bytes) {
  if (S.last_prec < 0 || which < 0 || which > 2 || n_launch < 1) {
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
    else if (which == 1) *bytes = n * 7 * sv;
    else *bytes = 12.0 * S.nnz + 4.0 * (n + 1) + 24.0 * n;
  }
  return PM_OK;
}

}  // namespace pm
