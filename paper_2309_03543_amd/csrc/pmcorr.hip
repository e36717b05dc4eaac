// Corrector-system assembly and PCG on MI355X (gfx950).
//
// Hot path per PCG iteration (two kernels, one grid-wide reduction):
//   k_spmv    q~ = D'^{-1} A p in difference form, fused with the four dot
//             products the iteration needs; the last block computes alpha and
//             beta (recurrence for the next rho, anchored on the exact rho)
//   k_update  x_acc += alpha p;  z -= alpha q~;  p = z + beta p
// Every m-th iteration the increments are folded into the float64 solution
// and the residual is recomputed exactly from the float64 CSR matrix
// (k_update_flush, k_resid, k_pdir).  Chunks of m iterations are captured in
// a HIP graph and replayed until a device-side flag reports convergence.
//
// Difference form: each row is stored as c_i = sum_j a_ij (the row sum, i.e.
// the mass or Dirichlet part) and w_ij = -a_ij for the off-diagonals, and the
// product is (A p)_i = c_i p_i + sum_j w_ij (p_i - p_j).  Rounding the weights
// then perturbs the quadratic form by a relative O(u) on every mode, which is
// what keeps float32 Krylov vectors usable on these M-matrices.
//
// Compiled with -ffp-contract=off.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "kernels.h"
#include "pm_internal.h"

using pm::State;

namespace pm {

namespace {
thread_local int g_last_status = PM_OK;
thread_local std::string g_last_msg;
}  // namespace

void set_error(int status, const std::string& msg) {
  g_last_status = status;
  g_last_msg = msg;
}

int get_error(char* buf, int32_t len) {
  if (buf && len > 0) {
    std::snprintf(buf, (size_t)len, "%s", g_last_msg.c_str());
  }
  return g_last_status;
}

// ---------------------------------------------------------------------------
// Assembly kernels (eq. CS1_sys_coeff, eq. Cs2_4, eq. CS2_sys_coeff)
// ---------------------------------------------------------------------------

// Per cell, in the renumbered order: Kfrak = chi exp(-s) G, M = I/dt + nu eps Kfrak,
// S = I + nu eps dt Kfrak, Xi = eps dt S^{-1}.
__global__ void k_cell_tensors(int n, const int* __restrict__ perm, const double* __restrict__ eps,
                               const double* __restrict__ logk, const double* __restrict__ chi,
                               const double* __restrict__ g11, const double* __restrict__ g12,
                               const double* __restrict__ g22, double nu, double dt,
                               double* __restrict__ X11, double* __restrict__ X12,
                               double* __restrict__ X22, double* __restrict__ M11,
                               double* __restrict__ M22, State* st) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int o = perm[i];
  const double e = eps[o], s = logk[o];
  const double ch = chi ? chi[o] : 1.0;
  const double a11 = g11 ? g11[o] : 1.0, a12 = g12 ? g12[o] : 0.0, a22 = g22 ? g22[o] : 1.0;
  const bool finite_in = isfinite(e) && isfinite(s) && isfinite(ch) && isfinite(a11) &&
                         isfinite(a12) && isfinite(a22);
  if (!finite_in) {
    atomicExch(&st->err, PM_NONFINITE);
    return;
  }
  if (!(e > 0.0) || ch < 0.0 || !(a11 > 0.0) || !(a11 * a22 - a12 * a12 > 0.0)) {
    atomicExch(&st->err, PM_INVALID_ARG);
    return;
  }
  const double k = ch * exp(-s);
  const double K11 = k * a11, K12 = k * a12, K22 = k * a22;
  M11[i] = 1.0 / dt + nu * e * K11;
  M22[i] = 1.0 / dt + nu * e * K22;
  const double c = nu * e * dt;
  const double S11 = 1.0 + c * K11, S12 = c * K12, S22 = 1.0 + c * K22;
  const double det = S11 * S22 - S12 * S12;
  const double f = e * dt / det;
  X11[i] = f * S22;
  X12[i] = -f * S12;
  X22[i] = f * S11;
}

// n.A.n for the outward unit normal of the CCW side vector t.
__device__ __forceinline__ double normal_quadratic(double tx, double ty, double a11, double a12,
                                                   double a22) {
  return (ty * ty * a11 - 2.0 * tx * ty * a12 + tx * tx * a22) / (tx * tx + ty * ty);
}

// One thread per row (renumbered order): side weights, off-diagonals into their
// CSR slots, the diagonal, 1/diagonal and the Dirichlet lift.
__global__ void k_assemble(int n, int kind, const int* __restrict__ perm, const int* __restrict__ nb,
                           const int* __restrict__ pos, const int* __restrict__ diagpos,
                           const int8_t* __restrict__ tag, const double* __restrict__ T,
                           const double* __restrict__ tx, const double* __restrict__ ty,
                           const double* __restrict__ area, const double* __restrict__ X11,
                           const double* __restrict__ X12, const double* __restrict__ X22,
                           const double* __restrict__ M11, const double* __restrict__ M22,
                           double nu, const double* __restrict__ g, double* __restrict__ val64,
                           float* __restrict__ val32, double* __restrict__ dinv,
                           double* __restrict__ b_lift) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int bit = kind == PM_CP2 ? 2 : 1;
  const int old = perm[i];
  double w[3], lift[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const size_t s = (size_t)k * n + i;
    const int o = nb[s];
    const double Ts = T[s];
    double wk = 0.0, lk = 0.0;
    if (o >= 0) {
      if (kind == PM_CP2) {
        const double a11 = 0.5 * (X11[i] + X11[o]);
        const double a12 = 0.5 * (X12[i] + X12[o]);
        const double a22 = 0.5 * (X22[i] + X22[o]);
        wk = Ts * normal_quadratic(tx[s], ty[s], a11, a12, a22);
      } else {
        wk = nu * Ts;
      }
      const int p = pos[s];
      val64[p] = -wk;
      if (val32) val32[p] = (float)(-wk);
    } else if (tag[s] & bit) {
      if (kind == PM_CP2)
        wk = Ts * normal_quadratic(tx[s], ty[s], X11[i], X12[i], X22[i]);
      else
        wk = nu * Ts;
      if (g) lk = wk * g[3 * (size_t)old + k];
    }
    w[k] = wk;
    lift[k] = lk;
  }
  const double mass = kind == PM_CP1X ? M11[i] * area[i] : (kind == PM_CP1Y ? M22[i] * area[i] : 0.0);
  const double diag = mass + (w[0] + w[1] + w[2]);
  val64[diagpos[i]] = diag;
  if (val32) val32[diagpos[i]] = (float)diag;
  if (dinv) dinv[i] = 1.0 / diag;
  if (b_lift) b_lift[old] = (lift[0] + lift[1]) + lift[2];
}

// ---------------------------------------------------------------------------
// Solver kernels
// ---------------------------------------------------------------------------

// Difference-form rows from the float64 CSR: c_i = row sum, w = -off-diagonals
// padded to three slots (padding: w = 0 pointing at the row itself), d' = c +
// sum w evaluated from the stored (rounded) values, which is the Jacobi
// diagonal the iteration uses.
template <typename W, typename I>
__global__ void k_prep_ell(int n, const int* __restrict__ rp, const int* __restrict__ col,
                           const double* __restrict__ val, W* __restrict__ c, W* __restrict__ w,
                           I* __restrict__ idx, double* __restrict__ dp, State* st) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double sum = 0.0;
  bool finite_all = true;
  W wv[3] = {W(0), W(0), W(0)};
  I iv[3];
  const I self = sizeof(I) == 2 ? I(0) : I(i);
  iv[0] = iv[1] = iv[2] = self;
  int nk = 0;
  for (int k = rp[i]; k < rp[i + 1]; ++k) {
    const double a = val[k];
    finite_all = finite_all && isfinite(a);
    sum += a;
    const int j = col[k];
    if (j != i && nk < 3) {
      wv[nk] = (W)(-a);
      iv[nk] = sizeof(I) == 2 ? I(j - i) : I(j);
      ++nk;
    }
  }
  const W cw = (W)sum;
  c[i] = cw;
  double d = (double)cw;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    w[(size_t)k * n + i] = wv[k];
    idx[(size_t)k * n + i] = iv[k];
    d += (double)wv[k];
  }
  dp[i] = d;
  if (!finite_all) atomicExch(&st->err, PM_NONFINITE);
  else if (!(d > 0.0)) atomicExch(&st->err, PM_INVALID_ARG);
}

// b and x0 into the renumbered order; partials of ||b||^2 and ||x0||^2.
template <typename V>
__global__ void __launch_bounds__(1024) k_gather_in(int n, int rpb, const int* __restrict__ perm,
                                                   const double* __restrict__ b,
                                                   const double* __restrict__ x, int x0_zero,
                                                   double* __restrict__ b64,
                                                   double* __restrict__ x64,
                                                   double* __restrict__ xlo, V* __restrict__ xacc,
                                                   double* __restrict__ part) {
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const int r0 = lb * rpb, r1 = min(n, r0 + rpb);
  double acc[2] = {0.0, 0.0};
  for (int i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
    const int o = perm[i];
    const double bi = b[o];
    const double xi = x0_zero ? 0.0 : x[o];
    b64[i] = bi;
    x64[i] = xi;
    xlo[i] = 0.0;
    xacc[i] = V(0);
    acc[0] += bi * bi;
    acc[1] += xi * xi;
  }
  block_partial<2>(acc, part + 2 * (size_t)blockIdx.x);
}

// One block: ||b||, the tolerance, input checks.
__global__ void k_start(const double* __restrict__ part, int nb, double tol, State* st) {
  double s[2];
  sum_partials<2>(part, nb, s);
  if (threadIdx.x != 0) return;
  st->bnorm2 = s[0];
  st->tol2 = tol * tol * s[0];
  if (st->err != 0) {
    st->status = st->err;
    st->done = 1;
  } else if (!isfinite(s[0]) || !isfinite(s[1])) {
    st->status = PM_NONFINITE;
    st->done = 1;
  } else if (s[0] == 0.0) {
    st->status = PM_OK;
    st->res2 = 0.0;
    st->done = 2;  // zero right-hand side: the solution is 0
  }
}

// True residuals from the float64 CSR with error-free transformations, for the
// returned vector x_hi (stopping test) and for x_hi + x_lo (replacement);
// partials of ||r_hi||^2, z.D'z and || |A||x_hi| ||^2 (rounding-floor estimate).
//   mode 0 (start):   z = r_dd/d', p = z
//   mode 1 (replace): z = r_dd/d'
//   mode 2 (final):   norms only; runs even after the stop flag is set
template <typename V>
__global__ void __launch_bounds__(1024) k_resid(int n, int rpb, int mode, const int* __restrict__ rp,
                                               const int* __restrict__ col,
                                               const double* __restrict__ val,
                                               const double* __restrict__ b64,
                                               const double* __restrict__ x64,
                                               const double* __restrict__ xlo,
                                               const double* __restrict__ dp, V* __restrict__ z,
                                               V* __restrict__ p, double* __restrict__ part,
                                               const State* st) {
  if (mode != 2 && st->done) return;
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const int r0 = lb * rpb, r1 = min(n, r0 + rpb);
  double acc[3] = {0.0, 0.0, 0.0};
  for (int i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
    double rh, rd, ax;
    residual_row(b64[i], val, col, x64, xlo, rp[i], rp[i + 1], rh, rd, ax);
    acc[0] += rh * rh;
    acc[2] += ax * ax;
    if (mode != 2) {
      const double d = dp[i];
      const V zv = (V)(rd / d);
      z[i] = zv;
      if (mode == 0) p[i] = zv;
      const double zd = (double)zv;
      acc[1] += d * zd * zd;
    }
  }
  block_partial<3>(acc, part + 3 * (size_t)blockIdx.x);
}

// One block after k_resid: the convergence test on the returned vector, the
// stagnation test (the residual norm has not halved for stag_checks
// replacement points although it is within 1000x of the tolerance or of the
// rounding floor u*|| |A||x| ||), and the scalars for the search direction.
__global__ void k_check(int mode, const double* __restrict__ part, int nb, State* st) {
  if (mode != 2 && st->done) return;
  double s[3];
  sum_partials<3>(part, nb, s);
  if (threadIdx.x != 0) return;
  st->res2 = s[0];
  if (mode == 2) return;
  if (!isfinite(s[0])) {
    st->status = PM_NONFINITE;
    st->done = 1;
  } else if (s[0] <= st->tol2) {
    st->status = PM_OK;
    st->done = 1;
  } else if (mode == 0) {
    st->rho = s[1];
    st->best_res2 = s[0];
    st->stall = 0;
  } else {
    if (s[0] < 0.25 * st->best_res2) {
      st->best_res2 = s[0];
      st->stall = 0;
    } else {
      st->stall += 1;
    }
    const double floor2 = 0x1p-106 * s[2];
    if (st->best_res2 < 1e6 * fmax(st->tol2, floor2) && st->stall >= st->stag_checks) {
      st->status = PM_STAGNATED;
      st->done = 1;
    } else {
      st->beta = s[1] / st->rho;
      st->rho = s[1];
    }
  }
}

// p = z + beta p after a replacement.
template <typename V>
__global__ void __launch_bounds__(1024) k_pdir(int n, int rpb, const V* __restrict__ z,
                                              V* __restrict__ p, const State* st) {
  if (st->done) return;
  const double b = st->beta;
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const int r0 = lb * rpb, r1 = min(n, r0 + rpb);
  for (int i = r0 + threadIdx.x; i < r1; i += blockDim.x) p[i] = (V)((double)z[i] + b * (double)p[i]);
}

// q~ = D'^{-1} A p (difference form) and, with q = D' q~ as stored, the block
// partials of  s0 = p.q,  s1 = z.q (= q.D'^{-1} r),  s2 = q.D'^{-1} q,
// s3 = z.D' z (= rho).
template <typename V, typename W, typename I>
__global__ void __launch_bounds__(1024) k_spmv(int n, int rpb, const W* __restrict__ c,
                                              const W* __restrict__ w, const I* __restrict__ idx,
                                              const V* __restrict__ p, const V* __restrict__ z,
                                              V* __restrict__ q, double* __restrict__ part,
                                              State* st) {
  if (st->done) return;
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const int r0 = lb * rpb, r1 = min(n, r0 + rpb);
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
    const W w0 = w[i], w1 = w[(size_t)n + i], w2 = w[2 * (size_t)n + i];
    const int j0 = col_of<I>(i, idx[i]);
    const int j1 = col_of<I>(i, idx[(size_t)n + i]);
    const int j2 = col_of<I>(i, idx[2 * (size_t)n + i]);
    const double pi = (double)p[i];
    const double p0 = (double)p[j0], p1 = (double)p[j1], p2 = (double)p[j2];
    const double ci = (double)c[i];
    double y = ci * pi;
    y += (double)w0 * (pi - p0);
    y += (double)w1 * (pi - p1);
    y += (double)w2 * (pi - p2);
    const double d = ((ci + (double)w0) + (double)w1) + (double)w2;
    const V qv = (V)(y / d);
    q[i] = qv;
    const double qd = (double)qv, zi = (double)z[i];
    const double dq = d * qd;
    acc[0] += pi * dq;
    acc[1] += zi * dq;
    acc[2] += qd * dq;
    acc[3] += d * zi * zi;
  }
  block_partial<4>(acc, part + 4 * (size_t)blockIdx.x);
  if (blockIdx.x == 0 && threadIdx.x == 0) st->iter_pending = st->iter + 1;
}

// Every block reduces the product's partials (same order, same result):
// alpha = rho / p.q, the next rho by its recurrence anchored on the exact rho,
// beta = rho_next / rho; then
//   FLUSH = false:  x_acc += alpha p;  z -= alpha q~;  p = z + beta p
//   FLUSH = true :  (x_hi, x_lo) += x_acc + alpha p; x_acc = 0  (replacement
//                   iteration: z and p are rebuilt from the true residual)
// Block 0 records the scalars and the iteration count, or the stop status.
// `scale` multiplies alpha and beta (1 in solves; 0 when timing the kernel).
template <typename V, bool FLUSH>
__global__ void __launch_bounds__(1024) k_update(int n, int rpb, V* __restrict__ xacc,
                                                V* __restrict__ p, V* __restrict__ z,
                                                const V* __restrict__ q, double* __restrict__ x64,
                                                double* __restrict__ xlo,
                                                const double* __restrict__ part, int nbp,
                                                double scale, State* st) {
  if (st->done) return;
  double s[4];
  sum_partials<4>(part, nbp, s);
  const int k = st->iter_pending;
  const double pq = s[0], rho = s[3];
  int stop = 0;
  if (k > st->max_it) stop = PM_MAXIT;
  else if (rho == 0.0) stop = 100;  // exact zero residual in the recurrence
  else if (!(pq > 0.0) || !isfinite(pq) || !isfinite(rho)) stop = PM_BREAKDOWN;
  if (stop) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      st->status = stop == 100 ? PM_OK : stop;
      st->done = 1;
    }
    return;
  }
  const double a = rho / pq;
  const double rn = rho - 2.0 * a * s[1] + a * a * s[2];
  const double be = rn / rho;
  const double as = a * scale, bs = be * scale;
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const int r0 = lb * rpb, r1 = min(n, r0 + rpb);
  for (int i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
    const double pi = (double)p[i];
    if (FLUSH) {
      const double xi = (double)xacc[i] + as * pi;
      double hi = x64[i], lo = xlo[i];
      dd_add(hi, lo, xi);
      x64[i] = hi;
      xlo[i] = lo;
      xacc[i] = V(0);
    } else {
      xacc[i] = (V)((double)xacc[i] + as * pi);
      const V zv = (V)((double)z[i] - as * (double)q[i]);
      z[i] = zv;
      p[i] = (V)((double)zv + bs * pi);
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->alpha = a;
    st->beta = be;
    st->rho = rho;
    st->iter = k;
  }
}

// End of solve: fold any pending increments (limit or breakdown mid-chunk).
template <typename V>
__global__ void k_flush(int n, V* __restrict__ xacc, double* __restrict__ x64,
                        double* __restrict__ xlo) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double hi = x64[i], lo = xlo[i];
  dd_add(hi, lo, (double)xacc[i]);
  x64[i] = hi;
  xlo[i] = lo;
  xacc[i] = V(0);
}

__global__ void k_scatter_out(int n, const int* __restrict__ perm, const double* __restrict__ x64,
                              double* __restrict__ x, const State* st) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  x[perm[i]] = st->done == 2 ? 0.0 : x64[i];
}

// Timing support: make the iteration kernels run again on a finished state
// (k_update is then launched with scale 0, which leaves the vectors unchanged).
__global__ void k_timing_state(State* st) {
  st->done = 0;
  st->status = PM_OK;
  st->max_it = INT_MAX;
  st->iter = 0;
  st->iter_pending = 1;
  st->tol2 = -1.0;
}

// ---------------------------------------------------------------------------
// Adjoint gradient (one thread per cell, gathers over its three sides)
// ---------------------------------------------------------------------------
__global__ void k_adjoint_grad(int n, int kind, const int* __restrict__ perm,
                               const int* __restrict__ nb, const int8_t* __restrict__ tag,
                               const double* __restrict__ T, const double* __restrict__ tx,
                               const double* __restrict__ ty, const double* __restrict__ area,
                               const double* __restrict__ eps, const double* __restrict__ logk,
                               const double* __restrict__ chi, const double* __restrict__ g11,
                               const double* __restrict__ g12, const double* __restrict__ g22,
                               double nu, double dt, const double* __restrict__ g,
                               const double* __restrict__ eta, const double* __restrict__ lam,
                               double* __restrict__ grad_s, double* __restrict__ grad_e) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int old = perm[i];
  const double e = eps[old], s = logk[old];
  const double ch = chi ? chi[old] : 1.0;
  const double a11 = g11 ? g11[old] : 1.0, a12 = g12 ? g12[old] : 0.0, a22 = g22 ? g22[old] : 1.0;
  const double k = ch * exp(-s);
  const double K11 = k * a11, K12 = k * a12, K22 = k * a22;
  const double li = lam[old], ei = eta[old];
  if (kind != PM_CP2) {
    const double Kd = kind == PM_CP1X ? K11 : K22;
    const double base = -li * ei * area[i];
    grad_s[old] = base * (-nu * e * Kd);
    grad_e[old] = base * (nu * Kd);
    return;
  }
  const double c = nu * e * dt;
  const double S11 = 1.0 + c * K11, S12 = c * K12, S22 = 1.0 + c * K22;
  const double det = S11 * S22 - S12 * S12;
  // S^{-1}
  const double I11 = S22 / det, I12 = -S12 / det, I22 = S11 / det;
  // B = S^{-1} Kfrak S^{-1} (symmetric)
  const double t11 = I11 * K11 + I12 * K12, t12 = I11 * K12 + I12 * K22;
  const double t21 = I12 * K11 + I22 * K12, t22 = I12 * K12 + I22 * K22;
  const double B11 = t11 * I11 + t12 * I12, B12 = t11 * I12 + t12 * I22;
  const double B22 = t21 * I12 + t22 * I22;
  // dXi/ds = eps dt S^{-1} (nu eps dt Kfrak) S^{-1};  dXi/deps = dt S^{-1} - eps dt S^{-1} (nu dt Kfrak) S^{-1}
  const double fs = e * dt * c, fe = e * dt * nu * dt;
  const double ds11 = fs * B11, ds12 = fs * B12, ds22 = fs * B22;
  const double de11 = dt * I11 - fe * B11, de12 = dt * I12 - fe * B12, de22 = dt * I22 - fe * B22;
  double gs = 0.0, ge = 0.0;
#pragma unroll
  for (int kk = 0; kk < 3; ++kk) {
    const size_t sidx = (size_t)kk * n + i;
    const int o = nb[sidx];
    double f;
    if (o >= 0) {
      const int oo = perm[o];
      f = -0.5 * T[sidx] * (li - lam[oo]) * (ei - eta[oo]);
    } else if (tag[sidx] & 2) {
      f = -T[sidx] * li * (ei - (g ? g[3 * (size_t)old + kk] : 0.0));
    } else {
      continue;
    }
    gs += f * normal_quadratic(tx[sidx], ty[sidx], ds11, ds12, ds22);
    ge += f * normal_quadratic(tx[sidx], ty[sidx], de11, de12, de22);
  }
  grad_s[old] = gs;
  grad_e[old] = ge;
}

}  // namespace pm

// ===========================================================================
// Host side
// ===========================================================================

using namespace pm;

#define PM_HIP(expr)                                                                  \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess) {                                                           \
      set_error(PM_HIP_ERROR, std::string(#expr) + ": " + hipGetErrorString(e_));     \
      return PM_HIP_ERROR;                                                            \
    }                                                                                 \
  } while (0)

struct pm_mesh {
  HostStructure hs;
  int device = 0;
  int32_t n = 0, nnz = 0;
  int index_bits = 32;
  // structure, renumbered order
  int32_t *perm = nullptr, *row_ptr = nullptr, *col = nullptr;
  int32_t *nb = nullptr, *pos = nullptr, *diagpos = nullptr;  // nb/pos: [3][n]
  int8_t* tag = nullptr;                                       // [3][n]
  double *T = nullptr, *tx = nullptr, *ty = nullptr, *area = nullptr;
  // assembly scratch
  double *X11 = nullptr, *X12 = nullptr, *X22 = nullptr, *M11 = nullptr, *M22 = nullptr;
  // solver workspace (sized for float64 / int32; float32 runs use the front part)
  void *ell_c = nullptr, *ell_w = nullptr, *ell_idx = nullptr;
  double *dp = nullptr, *x64 = nullptr, *xlo = nullptr, *b64 = nullptr;
  void *xacc = nullptr, *p = nullptr, *z = nullptr, *q = nullptr;
  double* part = nullptr;   // per-block partials of the product / start kernels
  double* part2 = nullptr;  // per-block partials of the residual kernel
  State* st = nullptr;
  State* h_st = nullptr;  // pinned, 3 slots
  hipStream_t cap = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipEvent_t tev[2] = {nullptr, nullptr};
  hipGraphExec_t graph = nullptr;
  int g_prec = -1, g_m = -1, g_grid = -1, g_block = -1;
  const double* g_val = nullptr;
  // launch shape and matrix of the last solve (for pm_time_kernel)
  int last_prec = -1, last_grid = 0, last_block = 256, last_rpb = 0;
  const double* last_val = nullptr;
  std::vector<void*> allocs;
};

namespace pm {
const HostStructure* mesh_structure(const pm_mesh* m) { return &m->hs; }
}  // namespace pm

namespace {

template <typename T>
int dalloc(pm_mesh* m, T** ptr, size_t count) {
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, std::max<size_t>(count, 1) * sizeof(T));
  if (e != hipSuccess) {
    set_error(PM_HIP_ERROR, std::string("hipMalloc: ") + hipGetErrorString(e));
    return PM_HIP_ERROR;
  }
  m->allocs.push_back(p);
  *ptr = static_cast<T*>(p);
  return PM_OK;
}

void free_mesh(pm_mesh* m) {
  if (!m) return;
  if (m->graph) (void)hipGraphExecDestroy(m->graph);
  for (void* p : m->allocs) (void)hipFree(p);
  if (m->h_st) (void)hipHostFree(m->h_st);
  for (auto& e : m->ev)
    if (e) (void)hipEventDestroy(e);
  for (auto& e : m->tev)
    if (e) (void)hipEventDestroy(e);
  if (m->cap) (void)hipStreamDestroy(m->cap);
  delete m;
}

struct Launch {
  int grid, block, rpb;
};

Launch launch_shape(int n, const pm_opts* o) {
  Launch L;
  L.block = (o && o->block > 0) ? o->block : 256;
  L.block = std::min(1024, std::max(64, (L.block / 64) * 64));
  int g = (o && o->grid > 0) ? o->grid : (n + 2 * L.block - 1) / (2 * L.block);
  g = std::max(1, std::min(g, kMaxBlocks));
  L.rpb = (n + g - 1) / g;
  L.grid = (n + L.rpb - 1) / L.rpb;
  return L;
}

inline int blocks_for(int n, int b) { return (n + b - 1) / b; }

}  // namespace

// ---------------------------------------------------------------------------
// The iteration for one precision / index width
// ---------------------------------------------------------------------------
template <typename V, typename W, typename I>
struct Solver {
  static void prep(pm_mesh* m, const double* val64, hipStream_t s) {
    k_prep_ell<W, I><<<blocks_for(m->n, 256), 256, 0, s>>>(
        m->n, m->row_ptr, m->col, val64, (W*)m->ell_c, (W*)m->ell_w, (I*)m->ell_idx, m->dp, m->st);
  }
  static void start(pm_mesh* m, const Launch& L, const double* b, const double* x, int x0_zero,
                    double tol, const double* val64, hipStream_t s) {
    k_gather_in<V><<<L.grid, L.block, 0, s>>>(m->n, L.rpb, m->perm, b, x, x0_zero, m->b64, m->x64,
                                              m->xlo, (V*)m->xacc, m->part);
    k_start<<<1, 256, 0, s>>>(m->part, L.grid, tol, m->st);
    resid(m, L, 0, val64, s);
  }
  static void spmv(pm_mesh* m, const Launch& L, hipStream_t s) {
    k_spmv<V, W, I><<<L.grid, L.block, 0, s>>>(m->n, L.rpb, (const W*)m->ell_c, (const W*)m->ell_w,
                                               (const I*)m->ell_idx, (const V*)m->p,
                                               (const V*)m->z, (V*)m->q, m->part, m->st);
  }
  template <bool FLUSH>
  static void update(pm_mesh* m, const Launch& L, hipStream_t s, double scale = 1.0) {
    k_update<V, FLUSH><<<L.grid, L.block, 0, s>>>(m->n, L.rpb, (V*)m->xacc, (V*)m->p, (V*)m->z,
                                                  (const V*)m->q, m->x64, m->xlo, m->part, L.grid,
                                                  scale, m->st);
  }
  static void resid(pm_mesh* m, const Launch& L, int mode, const double* val64, hipStream_t s) {
    k_resid<V><<<L.grid, L.block, 0, s>>>(m->n, L.rpb, mode, m->row_ptr, m->col, val64, m->b64,
                                          m->x64, m->xlo, m->dp, (V*)m->z, (V*)m->p, m->part2,
                                          m->st);
    k_check<<<1, 256, 0, s>>>(mode, m->part2, L.grid, m->st);
  }
  // one chunk of m iterations ending with a replacement
  static void chunk(pm_mesh* m, const Launch& L, int mrep, const double* val64, hipStream_t s) {
    for (int it = 0; it < mrep - 1; ++it) {
      spmv(m, L, s);
      update<false>(m, L, s);
    }
    spmv(m, L, s);
    update<true>(m, L, s);
    resid(m, L, 1, val64, s);
    k_pdir<V><<<L.grid, L.block, 0, s>>>(m->n, L.rpb, (const V*)m->z, (V*)m->p, m->st);
  }
  static void finish(pm_mesh* m, const Launch& L, const double* val64, double* x, hipStream_t s) {
    k_flush<V><<<blocks_for(m->n, 256), 256, 0, s>>>(m->n, (V*)m->xacc, m->x64, m->xlo);
    resid(m, L, 2, val64, s);
    k_scatter_out<<<blocks_for(m->n, 256), 256, 0, s>>>(m->n, m->perm, m->x64, x, m->st);
  }
};

namespace {

// The graph of one chunk reads val64 through its kernel arguments, so it is
// rebuilt when the matrix pointer changes.
struct ChunkKey {
  int prec, m, grid, block;
  const double* val;
};

template <typename V, typename W, typename I>
int run_solve(pm_mesh* m, const double* val64, const double* b, double* x, const pm_opts& o,
              pm_info* info, hipStream_t s) {
  using S = Solver<V, W, I>;
  const Launch L = launch_shape(m->n, &o);
  m->last_prec = o.precision;
  m->last_grid = L.grid;
  m->last_block = L.block;
  m->last_rpb = L.rpb;
  m->last_val = val64;

  State init{};
  init.max_it = o.max_it;
  init.stag_checks = o.stag_checks > 0 ? o.stag_checks : 40;
  std::memcpy(&m->h_st[2], &init, sizeof(State));
  PM_HIP(hipMemcpyAsync(m->st, &m->h_st[2], sizeof(State), hipMemcpyHostToDevice, s));
  S::prep(m, val64, s);
  S::start(m, L, b, x, o.x0_is_zero, o.tol, val64, s);
  PM_HIP(hipGetLastError());

  // (re)build the chunk graph (its kernels take val64 as an argument)
  if (!m->graph || m->g_prec != o.precision || m->g_m != o.replace_every || m->g_grid != L.grid ||
      m->g_block != L.block || m->g_val != val64) {
    if (m->graph) {
      (void)hipGraphExecDestroy(m->graph);
      m->graph = nullptr;
    }
    hipGraph_t g = nullptr;
    PM_HIP(hipStreamBeginCapture(m->cap, hipStreamCaptureModeThreadLocal));
    S::chunk(m, L, o.replace_every, val64, m->cap);
    PM_HIP(hipStreamEndCapture(m->cap, &g));
    PM_HIP(hipGraphInstantiate(&m->graph, g, nullptr, nullptr, 0));
    (void)hipGraphDestroy(g);
    m->g_prec = o.precision;
    m->g_m = o.replace_every;
    m->g_grid = L.grid;
    m->g_block = L.block;
    m->g_val = val64;
  }

  // replay chunks; poll the stop flag one chunk behind so the GPU stays busy
  const long max_chunks = (long)o.max_it / o.replace_every + 3;
  PM_HIP(hipMemcpyAsync(&m->h_st[0], m->st, sizeof(State), hipMemcpyDeviceToHost, s));
  PM_HIP(hipEventRecord(m->ev[0], s));
  PM_HIP(hipEventSynchronize(m->ev[0]));
  bool stop = m->h_st[0].done != 0;
  long c = 0;
  while (!stop && c < max_chunks) {
    PM_HIP(hipGraphLaunch(m->graph, s));
    const int slot = (int)(c & 1);
    PM_HIP(hipMemcpyAsync(&m->h_st[slot], m->st, sizeof(State), hipMemcpyDeviceToHost, s));
    PM_HIP(hipEventRecord(m->ev[slot], s));
    if (c >= 1) {
      PM_HIP(hipEventSynchronize(m->ev[slot ^ 1]));
      if (m->h_st[slot ^ 1].done) stop = true;
    }
    ++c;
  }
  S::finish(m, L, val64, x, s);
  PM_HIP(hipGetLastError());
  PM_HIP(hipMemcpyAsync(&m->h_st[0], m->st, sizeof(State), hipMemcpyDeviceToHost, s));
  PM_HIP(hipStreamSynchronize(s));
  const State& f = m->h_st[0];
  int status = f.done ? f.status : PM_MAXIT;
  if (f.err) status = f.err;
  if (info) {
    info->iters = f.iter;
    info->status = status;
    info->bnorm = std::sqrt(f.bnorm2);
    info->rel_res_true = f.bnorm2 > 0 ? std::sqrt(f.res2 / f.bnorm2) : 0.0;
  }
  if (status < 0) set_error(status, "pcg_solve stopped with an error status");
  return status;
}

int check_opts(const pm_opts& o) {
  if (!(o.tol > 0.0) || o.max_it < 0 || o.replace_every < 1 ||
      (o.precision != PM_FP64 && o.precision != PM_MIXED)) {
    set_error(PM_INVALID_ARG, "invalid solver options");
    return PM_INVALID_ARG;
  }
  return PM_OK;
}

}  // namespace

// ===========================================================================
// C entry points
// ===========================================================================
extern "C" {

void pm_opts_default(pm_opts* o) {
  if (!o) return;
  o->tol = 1e-10;
  o->max_it = 200000;
  o->precision = PM_FP64;
  o->replace_every = 50;
  o->x0_is_zero = 1;
  o->block = 0;
  o->grid = 0;
  o->stag_checks = 40;
}

const char* pm_status_string(int s) {
  switch (s) {
    case PM_OK: return "ok";
    case PM_MAXIT: return "iteration limit reached";
    case PM_STAGNATED: return "residual stagnated above the tolerance";
    case PM_INVALID_ARG: return "invalid argument";
    case PM_BAD_MESH: return "bad mesh";
    case PM_NOT_DELAUNAY: return "mesh not Delaunay";
    case PM_SINGULAR: return "singular system";
    case PM_NONFINITE: return "non-finite input";
    case PM_BREAKDOWN: return "PCG breakdown";
    case PM_HIP_ERROR: return "HIP runtime error";
    default: return "unknown status";
  }
}

int pm_last_error(char* buf, int32_t len) { return get_error(buf, len); }

int pm_structure_host(int32_t n_nodes, const double* xy, int32_t n_cells, const int32_t* tri,
                      const int8_t* side_tag, int32_t* perm, int32_t* row_ptr, int32_t* col,
                      int32_t col_capacity, double* T, pm_mesh_stats* stats) {
  HostStructure hs;
  std::string err;
  int st = build_structure(n_nodes, xy, n_cells, tri, side_tag, hs, err);
  if (st != PM_OK) {
    set_error(st, err);
    return st;
  }
  if ((perm == nullptr) != (row_ptr == nullptr) || (row_ptr && !col) ||
      (col && hs.stats.nnz > col_capacity)) {
    set_error(PM_INVALID_ARG, "output arrays missing or col_capacity < nnz");
    return PM_INVALID_ARG;
  }
  if (perm) std::memcpy(perm, hs.perm.data(), sizeof(int32_t) * hs.n);
  if (row_ptr) std::memcpy(row_ptr, hs.row_ptr.data(), sizeof(int32_t) * (hs.n + 1));
  if (col) std::memcpy(col, hs.col.data(), sizeof(int32_t) * hs.stats.nnz);
  if (T) std::memcpy(T, hs.T.data(), sizeof(double) * 3 * (size_t)hs.n);
  if (stats) *stats = hs.stats;
  return PM_OK;
}

int pm_mesh_create(int32_t n_nodes, const double* xy, int32_t n_cells, const int32_t* tri,
                   const int8_t* side_tag, pm_mesh** out) {
  if (!out) {
    set_error(PM_INVALID_ARG, "out is null");
    return PM_INVALID_ARG;
  }
  *out = nullptr;
  pm_mesh* m = new pm_mesh();
  std::string err;
  int st = build_structure(n_nodes, xy, n_cells, tri, side_tag, m->hs, err);
  if (st != PM_OK) {
    set_error(st, err);
    delete m;
    return st;
  }
  const HostStructure& hs = m->hs;
  const size_t n = hs.n;
  m->n = hs.n;
  m->nnz = hs.stats.nnz;
  m->index_bits = hs.stats.index_bits;
  (void)hipGetDevice(&m->device);

  // per-side arrays in the renumbered order, side-major
  std::vector<int32_t> nb(3 * n), pos(3 * n), diagpos(n);
  std::vector<int8_t> tag(3 * n);
  std::vector<double> T(3 * n), tx(3 * n), ty(3 * n), area(n);
  for (size_t i = 0; i < n; ++i) {
    const size_t old = hs.perm[i];
    area[i] = hs.area[old];
    for (int32_t k = hs.row_ptr[i]; k < hs.row_ptr[i + 1]; ++k)
      if (hs.col[k] == (int32_t)i) diagpos[i] = k;
    for (int j = 0; j < 3; ++j) {
      const size_t s = (size_t)j * n + i, so = 3 * old + j;
      const int32_t o = hs.nbr[so];
      nb[s] = o >= 0 ? hs.inv[o] : -1;
      pos[s] = -1;
      if (o >= 0)
        for (int32_t k = hs.row_ptr[i]; k < hs.row_ptr[i + 1]; ++k)
          if (hs.col[k] == nb[s]) pos[s] = k;
      tag[s] = hs.tag[so];
      T[s] = hs.T[so];
      tx[s] = hs.tx[so];
      ty[s] = hs.ty[so];
    }
  }
  int r = PM_OK;
#define ALLOC(ptr, cnt)                       \
  if ((r = dalloc(m, &(ptr), (cnt))) != PM_OK) { \
    free_mesh(m);                             \
    return r;                                 \
  }
  ALLOC(m->perm, n);
  ALLOC(m->row_ptr, n + 1);
  ALLOC(m->col, (size_t)m->nnz);
  ALLOC(m->nb, 3 * n);
  ALLOC(m->pos, 3 * n);
  ALLOC(m->diagpos, n);
  ALLOC(m->tag, 3 * n);
  ALLOC(m->T, 3 * n);
  ALLOC(m->tx, 3 * n);
  ALLOC(m->ty, 3 * n);
  ALLOC(m->area, n);
  ALLOC(m->X11, n);
  ALLOC(m->X12, n);
  ALLOC(m->X22, n);
  ALLOC(m->M11, n);
  ALLOC(m->M22, n);
  double* tmp;
  ALLOC(tmp, n);
  m->ell_c = tmp;
  ALLOC(tmp, 3 * n);
  m->ell_w = tmp;
  int32_t* itmp;
  ALLOC(itmp, 3 * n);
  m->ell_idx = itmp;
  ALLOC(m->dp, n);
  ALLOC(m->x64, n);
  ALLOC(m->xlo, n);
  ALLOC(m->b64, n);
  ALLOC(tmp, n);
  m->xacc = tmp;
  ALLOC(tmp, n);
  m->p = tmp;
  ALLOC(tmp, n);
  m->z = tmp;
  ALLOC(tmp, n);
  m->q = tmp;
  ALLOC(m->part, (size_t)kMaxBlocks * 4);
  ALLOC(m->part2, (size_t)kMaxBlocks * 4);
  ALLOC(m->st, 1);
#undef ALLOC
  auto fail = [&](hipError_t e, const char* what) {
    set_error(PM_HIP_ERROR, std::string(what) + ": " + hipGetErrorString(e));
    free_mesh(m);
    return PM_HIP_ERROR;
  };
  hipError_t e;
  if ((e = hipHostMalloc((void**)&m->h_st, 3 * sizeof(State), hipHostMallocDefault)) != hipSuccess)
    return fail(e, "hipHostMalloc");
  if ((e = hipStreamCreateWithFlags(&m->cap, hipStreamNonBlocking)) != hipSuccess)
    return fail(e, "hipStreamCreate");
  for (auto& ev : m->ev)
    if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess)
      return fail(e, "hipEventCreate");
  for (auto& ev : m->tev)
    if ((e = hipEventCreate(&ev)) != hipSuccess) return fail(e, "hipEventCreate");
  struct Up {
    void* d;
    const void* h;
    size_t bytes;
  } ups[] = {
      {m->perm, hs.perm.data(), 4 * n},        {m->row_ptr, hs.row_ptr.data(), 4 * (n + 1)},
      {m->col, hs.col.data(), 4 * (size_t)m->nnz}, {m->nb, nb.data(), 12 * n},
      {m->pos, pos.data(), 12 * n},            {m->diagpos, diagpos.data(), 4 * n},
      {m->tag, tag.data(), 3 * n},             {m->T, T.data(), 24 * n},
      {m->tx, tx.data(), 24 * n},              {m->ty, ty.data(), 24 * n},
      {m->area, area.data(), 8 * n},
  };
  for (const Up& u : ups)
    if ((e = hipMemcpy(u.d, u.h, u.bytes, hipMemcpyHostToDevice)) != hipSuccess)
      return fail(e, "hipMemcpy");
  *out = m;
  return PM_OK;
}

void pm_mesh_destroy(pm_mesh* m) { free_mesh(m); }

int pm_mesh_get_stats(const pm_mesh* m, pm_mesh_stats* st) {
  if (!m || !st) {
    set_error(PM_INVALID_ARG, "null argument");
    return PM_INVALID_ARG;
  }
  *st = m->hs.stats;
  return PM_OK;
}

int pm_mesh_export(const pm_mesh* m, int32_t* perm, int32_t* row_ptr, int32_t* col) {
  if (!m) {
    set_error(PM_INVALID_ARG, "null mesh");
    return PM_INVALID_ARG;
  }
  if (perm) std::memcpy(perm, m->hs.perm.data(), 4 * (size_t)m->n);
  if (row_ptr) std::memcpy(row_ptr, m->hs.row_ptr.data(), 4 * ((size_t)m->n + 1));
  if (col) std::memcpy(col, m->hs.col.data(), 4 * (size_t)m->nnz);
  return PM_OK;
}

int assemble_corrector(pm_mesh* m, int32_t kind, const pm_cell_params* prm, double nu, double dt,
                       const double* g, double* val64, float* val32, double* dinv, double* b_lift,
                       hipStream_t s) {
  if (!m || !prm || !prm->eps || !prm->logk || !val64 || kind < 0 || kind > 2 || !(dt > 0.0) ||
      !(nu >= 0.0) || !std::isfinite(nu) || !std::isfinite(dt)) {
    set_error(PM_INVALID_ARG, "assemble_corrector: invalid argument");
    return PM_INVALID_ARG;
  }
  if (kind == PM_CP2)
    for (uint8_t bits : m->hs.comp_bits)
      if (!(bits & 2)) {
        set_error(PM_SINGULAR, "CP2: a mesh component has no CP2 Dirichlet side");
        return PM_SINGULAR;
      }
  PM_HIP(hipMemsetAsync(&m->st->err, 0, sizeof(int32_t), s));
  const int nbk = blocks_for(m->n, 256);
  k_cell_tensors<<<nbk, 256, 0, s>>>(m->n, m->perm, prm->eps, prm->logk, prm->chi, prm->g11,
                                     prm->g12, prm->g22, nu, dt, m->X11, m->X12, m->X22, m->M11,
                                     m->M22, m->st);
  k_assemble<<<nbk, 256, 0, s>>>(m->n, kind, m->perm, m->nb, m->pos, m->diagpos, m->tag, m->T,
                                 m->tx, m->ty, m->area, m->X11, m->X12, m->X22, m->M11, m->M22, nu,
                                 g, val64, val32, dinv, b_lift);
  PM_HIP(hipGetLastError());
  PM_HIP(hipMemcpyAsync(&m->h_st[2].err, &m->st->err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  PM_HIP(hipStreamSynchronize(s));
  if (m->h_st[2].err) {
    set_error(m->h_st[2].err, "assemble_corrector: invalid or non-finite cell parameters");
    return m->h_st[2].err;
  }
  return PM_OK;
}

int pcg_solve(pm_mesh* m, const double* val64, const double* b, double* x, const pm_opts* opts,
              pm_info* info, hipStream_t s) {
  if (!m || !val64 || !b || !x) {
    set_error(PM_INVALID_ARG, "pcg_solve: null argument");
    return PM_INVALID_ARG;
  }
  pm_opts o;
  pm_opts_default(&o);
  if (opts) o = *opts;
  if (int r = check_opts(o)) return r;
  const bool i16 = m->index_bits == 16;
  if (o.precision == PM_FP64)
    return i16 ? run_solve<double, double, int16_t>(m, val64, b, x, o, info, s)
               : run_solve<double, double, int32_t>(m, val64, b, x, o, info, s);
  return i16 ? run_solve<float, float, int16_t>(m, val64, b, x, o, info, s)
             : run_solve<float, float, int32_t>(m, val64, b, x, o, info, s);
}

int pcg_adjoint(pm_mesh* m, int32_t kind, const pm_cell_params* prm, double nu, double dt,
                const double* g, const double* val64, const double* eta, const double* grad_eta,
                double* lambda, double* grad_logk, double* grad_eps, const pm_opts* opts,
                pm_info* info, hipStream_t s) {
  if (!m || !prm || !prm->eps || !prm->logk || !val64 || !eta || !grad_eta || !lambda ||
      !grad_logk || !grad_eps || kind < 0 || kind > 2) {
    set_error(PM_INVALID_ARG, "pcg_adjoint: invalid argument");
    return PM_INVALID_ARG;
  }
  pm_opts o;
  pm_opts_default(&o);
  if (opts) o = *opts;
  o.x0_is_zero = 1;
  int st = pcg_solve(m, val64, grad_eta, lambda, &o, info, s);
  if (st < 0) return st;
  k_adjoint_grad<<<blocks_for(m->n, 256), 256, 0, s>>>(
      m->n, kind, m->perm, m->nb, m->tag, m->T, m->tx, m->ty, m->area, prm->eps, prm->logk,
      prm->chi, prm->g11, prm->g12, prm->g22, nu, dt, g, eta, lambda, grad_logk, grad_eps);
  PM_HIP(hipGetLastError());
  PM_HIP(hipStreamSynchronize(s));
  return st;
}

int pm_time_kernel(pm_mesh* m, int32_t which, int32_t n_launch, hipStream_t s, double* ms,
                   double* bytes) {
  if (!m || m->last_prec < 0 || which < 0 || which > 2 || n_launch < 1) {
    set_error(PM_INVALID_ARG, "pm_time_kernel: no solve to time or bad kernel id");
    return PM_INVALID_ARG;
  }
  pm_opts o;
  pm_opts_default(&o);
  o.grid = m->last_grid;
  o.block = m->last_block;
  const Launch L = launch_shape(m->n, &o);
  const bool f64 = m->last_prec == PM_FP64, i16 = m->index_bits == 16;
  const double sv = f64 ? 8 : 4, sw = sv, si = i16 ? 2 : 4, n = m->n;
  k_timing_state<<<1, 1, 0, s>>>(m->st);
  PM_HIP(hipEventRecord(m->tev[0], s));
  for (int r = 0; r < n_launch; ++r) {
    if (which == 0) {
      if (f64) {
        if (i16) Solver<double, double, int16_t>::spmv(m, L, s);
        else Solver<double, double, int32_t>::spmv(m, L, s);
      } else {
        if (i16) Solver<float, float, int16_t>::spmv(m, L, s);
        else Solver<float, float, int32_t>::spmv(m, L, s);
      }
    } else if (which == 1) {
      if (f64) Solver<double, double, int32_t>::update<false>(m, L, s, 0.0);
      else Solver<float, float, int32_t>::update<false>(m, L, s, 0.0);
    } else {
      if (f64) Solver<double, double, int32_t>::resid(m, L, 2, m->last_val, s);
      else Solver<float, float, int32_t>::resid(m, L, 2, m->last_val, s);
    }
  }
  PM_HIP(hipEventRecord(m->tev[1], s));
  PM_HIP(hipGetLastError());
  PM_HIP(hipEventSynchronize(m->tev[1]));
  float t = 0.f;
  PM_HIP(hipEventElapsedTime(&t, m->tev[0], m->tev[1]));
  if (ms) *ms = (double)t / n_launch;
  if (bytes) {
    if (which == 0) *bytes = n * (4 * sw + 3 * si + 3 * sv);
    else if (which == 1) *bytes = n * 7 * sv;
    else *bytes = 12.0 * m->nnz + 4.0 * (n + 1) + 16.0 * n;
  }
  return PM_OK;
}

}  // extern "C"
