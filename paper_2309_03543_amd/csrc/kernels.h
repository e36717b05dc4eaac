// Device kernels of the corrector library (gfx950, wave64).  Included by the
// HIP translation units only.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pm {

constexpr int kNumXcd = 8;        // MI355X: 8 accelerator complex dies, 32 CUs each

// Blocks are dispatched round-robin over the XCDs; renumber them so each XCD
// works on one contiguous range of rows and the neighbour gathers of adjacent
// row tiles hit the same L2.
__device__ __forceinline__ int xcd_block(int b, int nb) {
  const int x = b % kNumXcd, k = b / kNumXcd;
  const int per = nb / kNumXcd, rem = nb % kNumXcd;
  return x * per + (x < rem ? x : rem) + k;
}

template <int NV>
__device__ __forceinline__ void wave_sum(double (&v)[NV]) {
#pragma unroll
  for (int k = 0; k < NV; ++k)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
}

// Block sum of NV values (fixed order).  Thread t < NV stores component t of
// the block's partial at part[t] with a plain store: the partials are read by
// a later kernel, after the kernel boundary has made them visible to every
// XCD, so no fence is needed here.
template <int NV>
__device__ __forceinline__ void block_partial(double (&v)[NV], double* part) {
  __shared__ double sh[NV][16];
  wave_sum<NV>(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k) sh[k][wid] = v[k];
  __syncthreads();
  if (threadIdx.x < NV) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += sh[threadIdx.x][w];
    part[threadIdx.x] = s;
  }
}

template <typename I>
__device__ __forceinline__ int col_of(int i, I v);
template <>
__device__ __forceinline__ int col_of<int16_t>(int i, int16_t v) { return i + (int)v; }
template <>
__device__ __forceinline__ int col_of<int32_t>(int i, int32_t v) { return (int)v; }

// Exact residual rows for x = x_hi + x_lo: r_hi = b_i - sum_k a_k x_hi_k and
// r_dd = r_hi - sum_k a_k x_lo_k, with error-free transformations (FMA
// two-product, two-sum) on the x_hi terms, each rounded once at the end.
// The x_lo terms are below one ulp of the x_hi terms, so plain products are
// exact enough for them.  absax = sum_k |a_k x_hi_k| sets the rounding floor.
__device__ __forceinline__ void residual_row(double bi, const double* __restrict__ val,
                                             const int* __restrict__ col,
                                             const double* __restrict__ xh,
                                             const double* __restrict__ xl, int k0, int k1,
                                             double& r_hi, double& r_dd, double& absax) {
  double s = bi, e = 0.0, el = 0.0, m = 0.0;
  for (int k = k0; k < k1; ++k) {
    const int j = col[k];
    const double a = val[k], xv = xh[j];
    const double pr = a * xv;
    m += fabs(pr);
    const double pe = __builtin_fma(a, xv, -pr);
    const double t = s - pr;
    const double bb = t - s;
    const double err = (s - (t - bb)) + (-pr - bb);
    s = t;
    e += err - pe;
    el -= a * xl[j];
  }
  r_hi = s + e;
  r_dd = s + (e + el);
  absax = m;
}

// (hi, lo) += v as a double-double (two-sum, then renormalise).
__device__ __forceinline__ void dd_add(double& hi, double& lo, double v) {
  const double s = hi + v;
  const double bb = s - hi;
  const double e = ((hi - (s - bb)) + (v - bb)) + lo;
  hi = s + e;
  lo = e - (hi - s);
}

}  // namespace pm
