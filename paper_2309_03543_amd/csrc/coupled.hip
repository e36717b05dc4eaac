// Conjugate gradients on the coupled CP1 system (gfx950).
//
// With anisotropic permeability the CP1 velocity components are coupled
// through the off-diagonal of each cell's mass tensor (Sec. 3.2.2,
// eq. cs1_sys2 and eq. CS1_sys_coeff):
//   A_x u + m v = b_x,   m u + A_y v = b_y,   m_e = M12_e A_e.
// The 2n x 2n matrix is nu L (x) I plus the cells' SPD mass blocks plus the
// Dirichlet terms, so it is SPD and CG applies directly; the preconditioner
// is the inverse of each cell's 2x2 diagonal block.  Both components of a
// cell sit together (double2), so each row reads its three weights, shared by
// the x and y matrices, once for both components.
//
// Work is cut into tiles of rows, one block per tile (XCD-aware order).  Two
// kernels per iteration, no grid-wide waits inside a kernel: each kernel
// reduces the per-tile partials of the previous one in a fixed order, so
// every block gets bitwise the same scalar.
//   k_cc_spmv    r.z of the last update -> beta; p = z + beta p (own rows,
//                and recomputed with the same expression for the neighbours);
//                q = C p; partial p.q
//   k_cc_update  alpha = r.z / p.q; x += alpha p; r -= alpha q; z = P^{-1} r;
//                partial r.z
// Every check_every iterations the true residual ||b - C x|| decides the stop.
//
// Precisions.  In float64 every vector and matrix value is float64 and the
// recursive residual is never replaced.  In mixed precision the Krylov
// vectors (r, z, p, q) and the per-iteration copies of the weights, diagonal
// blocks and block inverses are stored in float32 (all arithmetic in
// float64); x, b and float64 copies of the matrix stay, and every check
// replaces r by the float64 true residual b - C x, keeping the direction
// unless the replaced r.z exceeds the recursive one a hundredfold (then the
// next direction restarts, beta = 0).  A value rounded to float32 is rounded
// once, when it is stored; a neighbour's new direction is recomputed and
// rounded the same way as its owner stores it.
//
// Compiled with -ffp-contract=off.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>

#include "coupled.h"
#include "kernels.h"

namespace pm {

void set_error(int status, const std::string& msg);

namespace {

constexpr int kFlagPattern = 1;    // x and y matrices differ off the diagonal
constexpr int kFlagNotSpd = 2;     // a cell's 2x2 block is not positive definite
constexpr int kFlagNonfinite = 3;  // NaN or Inf in the right-hand side
constexpr int kFlagBreakdown = 4;  // p.q <= 0 or not finite

template <typename T>
struct Pair;
template <>
struct Pair<double> {
  using type = double2;
};
template <>
struct Pair<float> {
  using type = float2;
};

// T: storage type of the Krylov vectors and of the per-iteration matrix data.
template <typename T>
struct CA {
  using V2 = typename Pair<T>::type;
  int n, tile_rows, n_tiles;
  const int* nb;
  T* w;            // [3][n] off-diagonal magnitudes
  T* dm;           // [3][n] diagonal of x, diagonal of y, coupling m
  T* inv;          // [3][n] block inverses
  double* w64;     // float64 weights and blocks for the true residual
  double* dm64;    // (the same arrays as w, dm in float64)
  double2* b;
  double2* x;
  V2* r;
  V2* z;
  V2* q;
  V2* p0;
  V2* p1;
  double* part;  // [4][n_tiles]: p.q (or the setup / residual sums), r.z even, r.z odd,
                 // r.z of a replaced residual
  double* scal;  // r.z of even and odd iterations
  int32_t* flag;
};

__device__ __forceinline__ double2 wide(double2 v) { return v; }
__device__ __forceinline__ double2 wide(float2 v) { return make_double2(v.x, v.y); }
template <typename V2>
__device__ __forceinline__ V2 narrow(double x, double y);
template <>
__device__ __forceinline__ double2 narrow<double2>(double x, double y) {
  return make_double2(x, y);
}
template <>
__device__ __forceinline__ float2 narrow<float2>(double x, double y) {
  return make_float2((float)x, (float)y);
}

// Fixed-order block sum of NV values; every thread gets the totals.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV]) {
  __shared__ double sh[NV][16];
  __shared__ double res[NV];
  wave_sum<NV>(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k) sh[k][wid] = v[k];
  __syncthreads();
  if (threadIdx.x < NV) {
    double s = 0.0;
    for (int k = 0; k < nw; ++k) s += sh[threadIdx.x][k];
    res[threadIdx.x] = s;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = res[k];
}

// Sum of the t tile partials at part, the same in every block.
__device__ __forceinline__ double sum_tiles(const double* __restrict__ part, int t) {
  double v[1] = {0.0};
  for (int i = threadIdx.x; i < t; i += blockDim.x) v[0] += part[i];
  block_sum<1>(v);
  return v[0];
}

template <typename T>
__device__ __forceinline__ void tile_rows(const CA<T>& a, int& tile, int& r0, int& r1) {
  tile = xcd_block(blockIdx.x, gridDim.x);
  r0 = tile * a.tile_rows;
  r1 = min(a.n, r0 + a.tile_rows);
}

// (C y)_i for the cell pair y (both components of every cell), with the
// weights and blocks W / D (stored as T or as float64).  The weight of a
// missing neighbour is stored as 0 and its y_nb entry is any finite value, so
// the term vanishes exactly without a branch.
template <typename W>
__device__ __forceinline__ double2 apply_row(const W* __restrict__ w, const W* __restrict__ dm,
                                             int n, int i, double2 yi, const double2* y_nb) {
  const double dx = dm[i], dy = dm[(size_t)n + i], m = dm[2 * (size_t)n + i];
  double qx = dx * yi.x + m * yi.y, qy = m * yi.x + dy * yi.y;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double wk = w[(size_t)k * n + i];
    qx -= wk * y_nb[k].x;
    qy -= wk * y_nb[k].y;
  }
  return make_double2(qx, qy);
}

template <typename T>
__global__ void __launch_bounds__(kCoupledBlock)
k_cc_setup(CA<T> a, const int* __restrict__ perm, const int* __restrict__ pos,
           const int* __restrict__ diagpos, const double* __restrict__ val_x,
           const double* __restrict__ val_y, const double* __restrict__ mA,
           const double* __restrict__ bx, const double* __restrict__ by) {
  using V2 = typename CA<T>::V2;
  int t, r0, r1;
  tile_rows(a, t, r0, r1);
  double acc[2] = {0.0, 0.0};
  for (int i = r0 + (int)threadIdx.x; i < r1; i += blockDim.x) {
    const int o = perm[i];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const size_t s = (size_t)k * a.n + i;
      const int ps = pos[s];
      double wk = 0.0;
      if (ps >= 0) {
        wk = -val_x[ps];
        if (val_y[ps] != val_x[ps]) atomicExch(a.flag, kFlagPattern);
      }
      a.w64[s] = wk;
      a.w[s] = (T)wk;
    }
    const double dx = val_x[diagpos[i]], dy = val_y[diagpos[i]], m = mA[o];
    a.dm64[i] = dx;
    a.dm64[(size_t)a.n + i] = dy;
    a.dm64[2 * (size_t)a.n + i] = m;
    a.dm[i] = (T)dx;
    a.dm[(size_t)a.n + i] = (T)dy;
    a.dm[2 * (size_t)a.n + i] = (T)m;
    const double det = dx * dy - m * m;
    if (!(dx > 0.0) || !(det > 0.0) || !isfinite(det)) atomicExch(a.flag, kFlagNotSpd);
    const T i11 = (T)(dy / det), i12 = (T)(-m / det), i22 = (T)(dx / det);
    a.inv[i] = i11;
    a.inv[(size_t)a.n + i] = i12;
    a.inv[2 * (size_t)a.n + i] = i22;
    const double2 bb = make_double2(bx[o], by[o]);
    if (!isfinite(bb.x) || !isfinite(bb.y)) atomicExch(a.flag, kFlagNonfinite);
    const double2 rr = wide(narrow<V2>(bb.x, bb.y));
    const V2 zs = narrow<V2>((double)i11 * rr.x + (double)i12 * rr.y,
                             (double)i12 * rr.x + (double)i22 * rr.y);
    const double2 zz = wide(zs);
    a.b[i] = bb;
    a.x[i] = make_double2(0.0, 0.0);
    a.r[i] = narrow<V2>(rr.x, rr.y);
    a.z[i] = zs;
    acc[0] += bb.x * bb.x + bb.y * bb.y;
    acc[1] += rr.x * zz.x + rr.y * zz.y;
  }
  block_sum<2>(acc);
  if (threadIdx.x == 0) {
    a.part[t] = acc[0];                      // ||b||^2
    a.part[(size_t)a.n_tiles + t] = acc[1];  // r.z of iteration 0
  }
}

// Two rows per trip: the neighbour indices of both rows are loaded first, then
// every gather of both rows is issued with clamped (always valid) addresses
// before any value is used, so the loads overlap; rows past the tile and
// missing neighbours are masked only when the products are formed.
// After a replacement (replaced != 0) r.z comes from the replaced residual's
// partials, and the direction restarts when it exceeds the recursive r.z a
// hundredfold.
constexpr int kSpmvRows = 2;

template <typename T>
__global__ void __launch_bounds__(kCoupledBlock) k_cc_spmv(CA<T> a, int k, int replaced) {
  using V2 = typename CA<T>::V2;
  if (*a.flag) return;
  const double rz_rec = sum_tiles(a.part + (size_t)(1 + (k & 1)) * a.n_tiles, a.n_tiles);
  double rz = rz_rec;
  bool restart = false;
  if (replaced) {
    rz = sum_tiles(a.part + 3 * (size_t)a.n_tiles, a.n_tiles);
    restart = rz > 100.0 * rz_rec;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) a.scal[k & 1] = rz;
  const double beta = (k == 0 || restart) ? 0.0 : rz / a.scal[(k - 1) & 1];
  const V2* __restrict__ pold = (k & 1) ? a.p0 : a.p1;
  V2* __restrict__ pnew = (k & 1) ? a.p1 : a.p0;
  const bool fresh = k == 0 || restart;
  int t, r0, r1;
  tile_rows(a, t, r0, r1);
  double acc[1] = {0.0};
  for (int base = r0 + (int)threadIdx.x; base < r1; base += kSpmvRows * blockDim.x) {
    int row[kSpmvRows], nbo[kSpmvRows][3];
#pragma unroll
    for (int r = 0; r < kSpmvRows; ++r) {
      const int ir = base + r * (int)blockDim.x;
      row[r] = ir < r1 ? ir : base;
#pragma unroll
      for (int kk = 0; kk < 3; ++kk) nbo[r][kk] = a.nb[(size_t)kk * a.n + row[r]];
    }
    V2 zn[kSpmvRows][3], pn_old[kSpmvRows][3], zi[kSpmvRows], pi_old[kSpmvRows];
#pragma unroll
    for (int r = 0; r < kSpmvRows; ++r) {
      zi[r] = a.z[row[r]];
      pi_old[r] = pold[row[r]];
#pragma unroll
      for (int kk = 0; kk < 3; ++kk) {
        const int o = nbo[r][kk] >= 0 ? nbo[r][kk] : row[r];
        zn[r][kk] = a.z[o];
        pn_old[r][kk] = pold[o];
      }
    }
#pragma unroll
    for (int r = 0; r < kSpmvRows; ++r) {
      if (base + r * (int)blockDim.x >= r1) continue;
      const int i = row[r];
      double2 pn[3];
#pragma unroll
      for (int kk = 0; kk < 3; ++kk) {
        const double2 zo = wide(zn[r][kk]), po = wide(pn_old[r][kk]);
        pn[kk] = fresh ? zo : wide(narrow<V2>(zo.x + beta * po.x, zo.y + beta * po.y));
      }
      const double2 zw = wide(zi[r]);
      V2 ps = zi[r];
      if (!fresh) {
        const double2 po = wide(pi_old[r]);
        ps = narrow<V2>(zw.x + beta * po.x, zw.y + beta * po.y);
      }
      pnew[i] = ps;
      const double2 pi = wide(ps);
      const double2 qi = apply_row(a.w, a.dm, a.n, i, pi, pn);
      const V2 qs = narrow<V2>(qi.x, qi.y);
      a.q[i] = qs;
      const double2 qw = wide(qs);
      acc[0] += pi.x * qw.x + pi.y * qw.y;
    }
  }
  block_sum<1>(acc);
  if (threadIdx.x == 0) a.part[t] = acc[0];
}

template <typename T>
__global__ void __launch_bounds__(kCoupledBlock) k_cc_update(CA<T> a, int k) {
  using V2 = typename CA<T>::V2;
  if (*a.flag) return;
  const double pq = sum_tiles(a.part, a.n_tiles);
  if (!(pq > 0.0) || !isfinite(pq)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicExch(a.flag, kFlagBreakdown);
    return;
  }
  const double alpha = a.scal[k & 1] / pq;
  const V2* __restrict__ p = (k & 1) ? a.p1 : a.p0;
  int t, r0, r1;
  tile_rows(a, t, r0, r1);
  double acc[1] = {0.0};
  for (int i = r0 + (int)threadIdx.x; i < r1; i += blockDim.x) {
    const double2 pi = wide(p[i]), qi = wide(a.q[i]);
    double2 xi = a.x[i];
    const double2 rw = wide(a.r[i]);
    xi.x += alpha * pi.x;
    xi.y += alpha * pi.y;
    const V2 rs = narrow<V2>(rw.x - alpha * qi.x, rw.y - alpha * qi.y);
    const double2 ri = wide(rs);
    const double i11 = a.inv[i], i12 = a.inv[(size_t)a.n + i], i22 = a.inv[2 * (size_t)a.n + i];
    const V2 zs = narrow<V2>(i11 * ri.x + i12 * ri.y, i12 * ri.x + i22 * ri.y);
    const double2 zi = wide(zs);
    a.x[i] = xi;
    a.r[i] = rs;
    a.z[i] = zs;
    acc[0] += ri.x * zi.x + ri.y * zi.y;
  }
  block_sum<1>(acc);
  if (threadIdx.x == 0) a.part[(size_t)(1 + ((k + 1) & 1)) * a.n_tiles + t] = acc[0];
}

// Partials of ||b - C x||^2 (float64 matrix and x) into part[0 .. n_tiles).
// With replace set, r becomes the true residual (rounded to T), z its
// preconditioned value, and their r.z partials go to the fourth slot.
template <typename T>
__global__ void __launch_bounds__(kCoupledBlock) k_cc_resid(CA<T> a, int replace) {
  using V2 = typename CA<T>::V2;
  int t, r0, r1;
  tile_rows(a, t, r0, r1);
  double acc[2] = {0.0, 0.0};
  for (int i = r0 + (int)threadIdx.x; i < r1; i += blockDim.x) {
    double2 xn[3];
#pragma unroll
    for (int kk = 0; kk < 3; ++kk) {
      const int o = a.nb[(size_t)kk * a.n + i];
      xn[kk] = o >= 0 ? a.x[o] : make_double2(0.0, 0.0);
    }
    const double2 cx = apply_row(a.w64, a.dm64, a.n, i, a.x[i], xn);
    const double2 bi = a.b[i];
    const double tx = bi.x - cx.x, ty = bi.y - cx.y;
    acc[0] += tx * tx + ty * ty;
    if (replace) {
      const V2 rs = narrow<V2>(tx, ty);
      const double2 ri = wide(rs);
      const double i11 = a.inv[i], i12 = a.inv[(size_t)a.n + i],
                   i22 = a.inv[2 * (size_t)a.n + i];
      const V2 zs = narrow<V2>(i11 * ri.x + i12 * ri.y, i12 * ri.x + i22 * ri.y);
      const double2 zi = wide(zs);
      a.r[i] = rs;
      a.z[i] = zs;
      acc[1] += ri.x * zi.x + ri.y * zi.y;
    }
  }
  block_sum<2>(acc);
  if (threadIdx.x == 0) {
    a.part[t] = acc[0];
    if (replace) a.part[3 * (size_t)a.n_tiles + t] = acc[1];
  }
}

__global__ void k_cc_scatter(int n, const int* __restrict__ perm, const double2* __restrict__ x,
                             double* __restrict__ u, double* __restrict__ v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int o = perm[i];
  const double2 xi = x[i];
  u[o] = xi.x;
  v[o] = xi.y;
}

#define CC_HIP(expr)                                                               \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess) {                                                        \
      set_error(PM_HIP_ERROR, std::string(#expr) + ": " + hipGetErrorString(e_));  \
      return PM_HIP_ERROR;                                                         \
    }                                                                              \
  } while (0)

// Copies the n_tiles partials at part and the flag to the host; returns
// their fixed-order sum in *sum and the flag in *flag.
template <typename T>
int fetch_sum(const CA<T>& a, double* h_part, hipStream_t s, double* sum, int32_t* flag) {
  CC_HIP(hipMemcpyAsync(h_part, a.part, sizeof(double) * a.n_tiles, hipMemcpyDeviceToHost, s));
  CC_HIP(hipMemcpyAsync(h_part + a.n_tiles, a.flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  CC_HIP(hipStreamSynchronize(s));
  double acc = 0.0;
  for (int t = 0; t < a.n_tiles; ++t) acc += h_part[t];
  *sum = acc;
  std::memcpy(flag, h_part + a.n_tiles, sizeof(int32_t));
  return PM_OK;
}

template <typename T>
int run(const CoupledIn& in, CoupledWork& w, CA<T>& a, double tol, int max_it, int check_every,
        pm_info* info, hipStream_t s) {
  const bool mixed = sizeof(T) == sizeof(float);
  const int grid = a.n_tiles;
  CC_HIP(hipMemsetAsync(a.flag, 0, sizeof(int32_t), s));
  k_cc_setup<T><<<grid, kCoupledBlock, 0, s>>>(a, in.perm, in.pos, in.diagpos, in.val_x,
                                              in.val_y, in.mA, in.b_x, in.b_y);
  CC_HIP(hipGetLastError());
  double bb = 0.0;
  int32_t flag = 0;
  if (int r = fetch_sum(a, w.h_part, s, &bb, &flag)) return r;
  if (flag) {
    const int st = flag == kFlagNonfinite ? PM_NONFINITE : PM_INVALID_ARG;
    set_error(st, flag == kFlagPattern
                      ? "coupled CP1: the x and y matrices differ off the diagonal"
                      : (flag == kFlagNotSpd ? "coupled CP1: a cell's 2x2 block is not positive "
                                               "definite"
                                             : "coupled CP1: non-finite right-hand side"));
    return st;
  }
  pm_info res{};
  res.bnorm = std::sqrt(bb);
  int status = PM_OK;
  int k = 0;
  if (bb > 0.0) {
    status = PM_MAXIT;
    double rel = 1.0;  // x = 0
    while (k < max_it) {
      const int steps = std::min(check_every - k % check_every, max_it - k);
      for (int j = 0; j < steps; ++j, ++k) {
        k_cc_spmv<T><<<grid, kCoupledBlock, 0, s>>>(a, k, mixed && j == 0 && k > 0);
        k_cc_update<T><<<grid, kCoupledBlock, 0, s>>>(a, k);
      }
      CC_HIP(hipGetLastError());
      k_cc_resid<T><<<grid, kCoupledBlock, 0, s>>>(a, mixed ? 1 : 0);
      double r2 = 0.0;
      if (int r = fetch_sum(a, w.h_part, s, &r2, &flag)) return r;
      rel = std::sqrt(r2) / res.bnorm;
      // a breakdown on an iterate that meets the tolerance is convergence
      // (a system of a few rows: CG has ended, then p.q decays to zero)
      if (rel <= tol) {
        status = PM_OK;
        break;
      }
      if (flag == kFlagBreakdown) {
        status = PM_BREAKDOWN;
        set_error(status, "coupled CP1: p.q <= 0 or not finite before the tolerance was met");
        break;
      }
    }
    res.rel_res_true = rel;
  }
  k_cc_scatter<<<(a.n + 255) / 256, 256, 0, s>>>(a.n, in.perm, a.x, in.u, in.v);
  CC_HIP(hipGetLastError());
  CC_HIP(hipStreamSynchronize(s));
  res.iters = k;
  res.status = status;
  if (info) *info = res;
  return status;
}

}  // namespace

int coupled_pcg(const CoupledIn& in, CoupledWork& w, int precision, double tol, int max_it,
                int check_every, pm_info* info, hipStream_t s) {
  if (precision == PM_MIXED) {
    CA<float> a;
    a.n = in.n;
    a.tile_rows = w.tile_rows;
    a.n_tiles = w.n_tiles;
    a.nb = in.nb;
    a.w = w.w32;
    a.dm = w.dm32;
    a.inv = w.inv32;
    a.w64 = w.w64;
    a.dm64 = w.dm64;
    a.b = w.b;
    a.x = w.x;
    a.r = w.r32;
    a.z = w.z32;
    a.q = w.q32;
    a.p0 = w.p32[0];
    a.p1 = w.p32[1];
    a.part = w.part;
    a.scal = w.scal;
    a.flag = w.flag;
    return run(in, w, a, tol, max_it, check_every, info, s);
  }
  CA<double> a;
  a.n = in.n;
  a.tile_rows = w.tile_rows;
  a.n_tiles = w.n_tiles;
  a.nb = in.nb;
  a.w = w.w64;
  a.dm = w.dm64;
  a.inv = w.inv64;
  a.w64 = w.w64;
  a.dm64 = w.dm64;
  a.b = w.b;
  a.x = w.x;
  a.r = w.r;
  a.z = w.z;
  a.q = w.q;
  a.p0 = w.p[0];
  a.p1 = w.p[1];
  a.part = w.part;
  a.scal = w.scal;
  a.flag = w.flag;
  return run(in, w, a, tol, max_it, check_every, info, s);
}

}  // namespace pm
