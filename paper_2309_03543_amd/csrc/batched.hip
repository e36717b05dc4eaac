// Batched corrector PCG: many independent systems (for instance permeability
// realisations on meshes of different sizes) solved by one persistent
// cooperative kernel, captured once in a HIP graph.
//
// The systems are packed one after another (each in its own mesh's reverse
// Cuthill-McKee order) and cut into row tiles that never straddle two
// systems.  Every phase of the iteration sweeps the tiles of the systems that
// are still active (tile t goes to block t mod G, so a large system spreads
// over the whole grid), separated by grid-wide barriers.  Per-system scalars
// live in a small state array; a system whose true residual passes the test
// at a replacement point is masked out of all later phases.  The algorithm,
// the difference-form product and the stopping rule are those of pcg_solve.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "kernels.h"
#include "pm_internal.h"

namespace pm {

struct SysState {
  double alpha, beta, rho, bnorm2, tol2, res2, best_res2;
  int32_t iter, done, status, stall;
};

struct BatchArgs {
  int n_sys, n_tiles, N, mrep, max_it, stag_checks;
  double tol;
  const int* tile_sys;
  const int* tile_r0;
  const int* tile_r1;
  const int* sys_tile0;  // [n_sys + 1]
  const int* perm;       // packed: global cell-order index of each packed row
  const int* rp;         // packed CSR row pointers into the packed values
  const int* col;        // packed CSR columns (global rows)
  const double* val;
  const double* b;
  double* x;
  void* c;
  void* w;
  void* idx;
  double* dp;
  double* x64;
  double* xlo;
  double* b64;
  void* xacc;
  void* p;
  void* z;
  void* q;
  double* tpart;  // [n_tiles][4]
  SysState* ss;
  uint32_t* bar;  // [0] arrivals, [1] generation, [2] abort flag
  uint32_t spin_limit;
};

// Grid-wide barrier for a co-resident (cooperative) grid.  The wait is
// bounded: past spin_limit polls the abort flag is raised and every block
// leaves the kernel at its next phase check.
__device__ __forceinline__ bool grid_barrier(uint32_t* bar, uint32_t nblocks, uint32_t spin_limit) {
  __shared__ int aborted;
  // every wave publishes its own stores (agent-scope release) before arriving
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    aborted = 0;
    const uint32_t gen = __hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t arrived = atomicAdd(&bar[0], 1u) + 1u;
    if (arrived == nblocks) {
      __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __threadfence();
      atomicAdd(&bar[1], 1u);
    } else {
      uint32_t spins = 0;
      while (__hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
        __builtin_amdgcn_s_sleep(2);
        if (++spins > spin_limit ||
            __hip_atomic_load(&bar[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
          atomicExch(&bar[2], 1u);
          break;
        }
      }
    }
    aborted = __hip_atomic_load(&bar[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
  }
  __syncthreads();
  // every wave acquires what the other blocks published
  __threadfence();
  return aborted == 0;
}

template <int NV>
__device__ __forceinline__ void block_sum_to(double (&v)[NV], double* out) {
  __shared__ double sh[NV][16];
  wave_sum<NV>(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k) sh[k][wid] = v[k];
  __syncthreads();
  if (threadIdx.x < NV) {
    double s = 0.0;
    for (int ww = 0; ww < nw; ++ww) s += sh[threadIdx.x][ww];
    out[threadIdx.x] = s;
  }
  __syncthreads();
}

// Fixed-order sum of the tile partials of system s (NV components, stride 4).
template <int NV>
__device__ __forceinline__ void system_sum(const BatchArgs& a, int s, double (&out)[NV]) {
  __shared__ double res[NV];
  double v[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = 0.0;
  for (int t = a.sys_tile0[s] + threadIdx.x; t < a.sys_tile0[s + 1]; t += blockDim.x)
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] += a.tpart[4 * (size_t)t + k];
  block_sum_to<NV>(v, res);
#pragma unroll
  for (int k = 0; k < NV; ++k) out[k] = res[k];
}

template <typename V, typename W, typename I>
__global__ void __launch_bounds__(256) k_pcg_batched(BatchArgs a) {
  const uint32_t G = gridDim.x;
  const int N = a.N;
  W* __restrict__ c = (W*)a.c;
  W* __restrict__ w = (W*)a.w;
  I* __restrict__ idx = (I*)a.idx;
  V* __restrict__ xacc = (V*)a.xacc;
  V* __restrict__ p = (V*)a.p;
  V* __restrict__ z = (V*)a.z;
  V* __restrict__ q = (V*)a.q;
  SysState* ss = a.ss;

  // ---- start: difference-form rows, inputs into the packed order ----
  for (int t = blockIdx.x; t < a.n_tiles; t += G) {
    double acc[2] = {0.0, 0.0};
    for (int i = a.tile_r0[t] + threadIdx.x; i < a.tile_r1[t]; i += blockDim.x) {
      double sum = 0.0;
      W wv[3] = {W(0), W(0), W(0)};
      I iv[3];
      iv[0] = iv[1] = iv[2] = sizeof(I) == 2 ? I(0) : I(i);
      int nk = 0;
      bool fin = true;
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
      c[i] = cw;
      double d = (double)cw;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        w[(size_t)k * N + i] = wv[k];
        idx[(size_t)k * N + i] = iv[k];
        d += (double)wv[k];
      }
      a.dp[i] = fin && d > 0.0 ? d : NAN;
      const int o = a.perm[i];
      const double bi = a.b[o], xi = a.x[o];
      a.b64[i] = bi;
      a.x64[i] = xi;
      a.xlo[i] = 0.0;
      xacc[i] = V(0);
      acc[0] += bi * bi;
      acc[1] += xi * xi + (fin && d > 0.0 ? 0.0 : NAN);
    }
    double out[2];
    block_sum_to<2>(acc, out);
    if (threadIdx.x < 2) a.tpart[4 * (size_t)t + threadIdx.x] = out[threadIdx.x];
  }
  if (!grid_barrier(a.bar, G, a.spin_limit)) return;
  for (int s = blockIdx.x; s < a.n_sys; s += G) {
    double r[2];
    system_sum<2>(a, s, r);
    if (threadIdx.x == 0) {
      SysState& S = ss[s];
      S.bnorm2 = r[0];
      S.tol2 = a.tol * a.tol * r[0];
      S.iter = 0;
      S.status = PM_OK;
      S.done = 0;
      if (!isfinite(r[0]) || !isfinite(r[1])) {
        S.status = PM_NONFINITE;
        S.done = 1;
      } else if (r[0] == 0.0) {
        S.res2 = 0.0;
        S.done = 2;
      }
    }
  }
  if (!grid_barrier(a.bar, G, a.spin_limit)) return;

  // ---- residual kernel body shared by start / replace / final ----
  auto residual_pass = [&](int mode) {
    for (int t = blockIdx.x; t < a.n_tiles; t += G) {
      const int s = a.tile_sys[t];
      if (mode != 2 && ss[s].done) continue;
      double acc[3] = {0.0, 0.0, 0.0};
      for (int i = a.tile_r0[t] + threadIdx.x; i < a.tile_r1[t]; i += blockDim.x) {
        double rh, rd, ax;
        residual_row(a.b64[i], a.val, a.col, a.x64, a.xlo, a.rp[i], a.rp[i + 1], rh, rd, ax);
        acc[0] += rh * rh;
        acc[2] += ax * ax;
        if (mode != 2) {
          const double d = a.dp[i];
          const V zv = (V)(rd / d);
          z[i] = zv;
          if (mode == 0) p[i] = zv;
          const double zd = (double)zv;
          acc[1] += d * zd * zd;
        }
      }
      double out[3];
      block_sum_to<3>(acc, out);
      if (threadIdx.x < 3) a.tpart[4 * (size_t)t + threadIdx.x] = out[threadIdx.x];
    }
  };
  auto residual_check = [&](int mode) {
    for (int s = blockIdx.x; s < a.n_sys; s += G) {
      if (mode != 2 && ss[s].done) continue;
      if (mode == 2 && ss[s].done == 2) continue;
      double r[3];
      system_sum<3>(a, s, r);
      if (threadIdx.x == 0) {
        SysState& S = ss[s];
        S.res2 = r[0];
        if (mode != 2) {
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
            if (S.best_res2 < 1e6 * fmax(S.tol2, 0x1p-106 * r[2]) && S.stall >= a.stag_checks) {
              S.status = PM_STAGNATED;
              S.done = 1;
            } else {
              S.beta = r[1] / S.rho;
              S.rho = r[1];
            }
          }
        }
      }
    }
  };

  residual_pass(0);
  if (!grid_barrier(a.bar, G, a.spin_limit)) return;
  residual_check(0);
  if (!grid_barrier(a.bar, G, a.spin_limit)) return;

  for (int it = 1; it <= a.max_it; ++it) {
    // every block sees the same flags after the barrier, so all leave together
    bool any = false;
    for (int s = 0; s < a.n_sys && !any; ++s) any = ss[s].done == 0;
    if (!any) break;

    // product and dot products
    for (int t = blockIdx.x; t < a.n_tiles; t += G) {
      const int s = a.tile_sys[t];
      if (ss[s].done) continue;
      double acc[4] = {0.0, 0.0, 0.0, 0.0};
      for (int i = a.tile_r0[t] + threadIdx.x; i < a.tile_r1[t]; i += blockDim.x) {
        const W w0 = w[i], w1 = w[(size_t)N + i], w2 = w[2 * (size_t)N + i];
        const int j0 = col_of<I>(i, idx[i]);
        const int j1 = col_of<I>(i, idx[(size_t)N + i]);
        const int j2 = col_of<I>(i, idx[2 * (size_t)N + i]);
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
      double out[4];
      block_sum_to<4>(acc, out);
      if (threadIdx.x < 4) a.tpart[4 * (size_t)t + threadIdx.x] = out[threadIdx.x];
    }
    if (!grid_barrier(a.bar, G, a.spin_limit)) return;
    for (int s = blockIdx.x; s < a.n_sys; s += G) {
      if (ss[s].done) continue;
      double r[4];
      system_sum<4>(a, s, r);
      if (threadIdx.x == 0) {
        SysState& S = ss[s];
        const double pq = r[0], rho = r[3];
        if (rho == 0.0) {
          S.status = PM_OK;
          S.done = 1;
        } else if (!(pq > 0.0) || !isfinite(pq) || !isfinite(rho)) {
          S.status = PM_BREAKDOWN;
          S.done = 1;
        } else {
          const double al = rho / pq;
          const double rn = rho - 2.0 * al * r[1] + al * al * r[2];
          S.alpha = al;
          S.beta = rn / rho;
          S.rho = rho;
          S.iter = it;
        }
      }
    }
    if (!grid_barrier(a.bar, G, a.spin_limit)) return;

    const bool replace = (it % a.mrep) == 0;
    for (int t = blockIdx.x; t < a.n_tiles; t += G) {
      const int s = a.tile_sys[t];
      if (ss[s].done) continue;
      const double al = ss[s].alpha, be = ss[s].beta;
      for (int i = a.tile_r0[t] + threadIdx.x; i < a.tile_r1[t]; i += blockDim.x) {
        const double pi = (double)p[i];
        if (replace) {
          const double xi = (double)xacc[i] + al * pi;
          double hi = a.x64[i], lo = a.xlo[i];
          dd_add(hi, lo, xi);
          a.x64[i] = hi;
          a.xlo[i] = lo;
          xacc[i] = V(0);
        } else {
          xacc[i] = (V)((double)xacc[i] + al * pi);
          const V zv = (V)((double)z[i] - al * (double)q[i]);
          z[i] = zv;
          p[i] = (V)((double)zv + be * pi);
        }
      }
    }
    if (!grid_barrier(a.bar, G, a.spin_limit)) return;
    if (replace) {
      residual_pass(1);
      if (!grid_barrier(a.bar, G, a.spin_limit)) return;
      residual_check(1);
      if (!grid_barrier(a.bar, G, a.spin_limit)) return;
      for (int t = blockIdx.x; t < a.n_tiles; t += G) {
        const int s = a.tile_sys[t];
        if (ss[s].done) continue;
        const double be = ss[s].beta;
        for (int i = a.tile_r0[t] + threadIdx.x; i < a.tile_r1[t]; i += blockDim.x)
          p[i] = (V)((double)z[i] + be * (double)p[i]);
      }
      if (!grid_barrier(a.bar, G, a.spin_limit)) return;
    }
  }

  // ---- finish: pending increments, final residual, scatter ----
  for (int t = blockIdx.x; t < a.n_tiles; t += G)
    for (int i = a.tile_r0[t] + threadIdx.x; i < a.tile_r1[t]; i += blockDim.x) {
      double hi = a.x64[i], lo = a.xlo[i];
      dd_add(hi, lo, (double)xacc[i]);
      a.x64[i] = hi;
      a.xlo[i] = lo;
      xacc[i] = V(0);
    }
  if (!grid_barrier(a.bar, G, a.spin_limit)) return;
  residual_pass(2);
  if (!grid_barrier(a.bar, G, a.spin_limit)) return;
  residual_check(2);
  for (int s = blockIdx.x; s < a.n_sys; s += G)
    if (threadIdx.x == 0 && ss[s].done == 0) {
      ss[s].status = PM_MAXIT;
      ss[s].done = 1;
    }
  for (int t = blockIdx.x; t < a.n_tiles; t += G) {
    const bool zero = ss[a.tile_sys[t]].done == 2;
    for (int i = a.tile_r0[t] + threadIdx.x; i < a.tile_r1[t]; i += blockDim.x)
      a.x[a.perm[i]] = zero ? 0.0 : a.x64[i];
  }
}

}  // namespace pm

using namespace pm;

#define PB_HIP(expr)                                                                  \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess) {                                                           \
      set_error(PM_HIP_ERROR, std::string(#expr) + ": " + hipGetErrorString(e_));     \
      return PM_HIP_ERROR;                                                            \
    }                                                                                 \
  } while (0)

struct pm_batch {
  int n_sys = 0, n_tiles = 0, N = 0;
  int64_t nnz = 0;
  int index_bits = 16;
  std::vector<int64_t> val_off, vec_off;
  std::vector<void*> allocs;
  BatchArgs args{};
  SysState* h_ss = nullptr;
  // cached graph: one cooperative kernel node
  hipGraphExec_t graph = nullptr;
  int g_prec = -1;
  int g_grid = 0;
  const double* g_val = nullptr;
  const double* g_b = nullptr;
  double* g_x = nullptr;
  pm_opts g_opts{};
};

namespace {
constexpr int kTile = 1024;

template <typename T>
int balloc(pm_batch* B, T** ptr, size_t count) {
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, std::max<size_t>(count, 1) * sizeof(T));
  if (e != hipSuccess) {
    set_error(PM_HIP_ERROR, std::string("hipMalloc: ") + hipGetErrorString(e));
    return PM_HIP_ERROR;
  }
  B->allocs.push_back(p);
  *ptr = static_cast<T*>(p);
  return PM_OK;
}

void free_batch(pm_batch* B) {
  if (!B) return;
  if (B->graph) (void)hipGraphExecDestroy(B->graph);
  for (void* p : B->allocs) (void)hipFree(p);
  if (B->h_ss) (void)hipHostFree(B->h_ss);
  delete B;
}

template <typename V, typename W, typename I>
const void* kernel_ptr() {
  return reinterpret_cast<const void*>(&k_pcg_batched<V, W, I>);
}

const void* pick_kernel(int prec, int bits) {
  if (prec == PM_FP64)
    return bits == 16 ? kernel_ptr<double, double, int16_t>() : kernel_ptr<double, double, int32_t>();
  return bits == 16 ? kernel_ptr<float, float, int16_t>() : kernel_ptr<float, float, int32_t>();
}
}  // namespace

extern "C" {

int pm_batch_create(int32_t n_sys, pm_mesh* const* meshes, pm_batch** out) {
  if (!out || n_sys < 1 || !meshes) {
    set_error(PM_INVALID_ARG, "pm_batch_create: invalid argument");
    return PM_INVALID_ARG;
  }
  *out = nullptr;
  std::vector<const HostStructure*> hs(n_sys);
  for (int s = 0; s < n_sys; ++s) {
    if (!meshes[s]) {
      set_error(PM_INVALID_ARG, "pm_batch_create: null mesh");
      return PM_INVALID_ARG;
    }
    hs[s] = mesh_structure(meshes[s]);
  }
  pm_batch* B = new pm_batch();
  B->n_sys = n_sys;
  B->val_off.assign(n_sys + 1, 0);
  B->vec_off.assign(n_sys + 1, 0);
  int max_bw = 0;
  for (int s = 0; s < n_sys; ++s) {
    B->val_off[s + 1] = B->val_off[s] + hs[s]->stats.nnz;
    B->vec_off[s + 1] = B->vec_off[s] + hs[s]->n;
    max_bw = std::max(max_bw, hs[s]->stats.bandwidth);
  }
  if (B->vec_off[n_sys] > INT32_MAX / 4 || B->val_off[n_sys] > INT32_MAX) {
    set_error(PM_INVALID_ARG, "pm_batch_create: batch too large for 32-bit indexing");
    free_batch(B);
    return PM_INVALID_ARG;
  }
  B->N = (int)B->vec_off[n_sys];
  B->nnz = B->val_off[n_sys];
  B->index_bits = max_bw <= 32767 ? 16 : 32;
  const size_t N = B->N;
  std::vector<int> perm(N), rp(N + 1), col(B->nnz), tsys, tr0, tr1, st0(n_sys + 1);
  for (int s = 0; s < n_sys; ++s) {
    const HostStructure& h = *hs[s];
    const int off = (int)B->vec_off[s];
    const int voff = (int)B->val_off[s];
    for (int i = 0; i < h.n; ++i) {
      perm[off + i] = off + h.perm[i];
      rp[off + i] = voff + h.row_ptr[i];
    }
    for (int k = 0; k < h.stats.nnz; ++k) col[voff + k] = off + h.col[k];
    st0[s] = (int)tsys.size();
    for (int r = 0; r < h.n; r += kTile) {
      tsys.push_back(s);
      tr0.push_back(off + r);
      tr1.push_back(off + std::min(h.n, r + kTile));
    }
  }
  rp[N] = (int)B->nnz;
  st0[n_sys] = (int)tsys.size();
  B->n_tiles = (int)tsys.size();
  BatchArgs& a = B->args;
  int r = PM_OK;
#define BALLOC(ptr, cnt)                          \
  if ((r = balloc(B, &(ptr), (cnt))) != PM_OK) { \
    free_batch(B);                                \
    return r;                                     \
  }
  int *d_tsys, *d_tr0, *d_tr1, *d_st0, *d_perm, *d_rp, *d_col;
  BALLOC(d_tsys, tsys.size());
  BALLOC(d_tr0, tr0.size());
  BALLOC(d_tr1, tr1.size());
  BALLOC(d_st0, st0.size());
  BALLOC(d_perm, N);
  BALLOC(d_rp, N + 1);
  BALLOC(d_col, (size_t)B->nnz);
  double *dc, *dw, *dp, *x64, *xlo, *b64, *xacc, *p, *z, *q, *tpart;
  int32_t* didx;
  BALLOC(dc, N);
  BALLOC(dw, 3 * N);
  BALLOC(didx, 3 * N);
  BALLOC(dp, N);
  BALLOC(x64, N);
  BALLOC(xlo, N);
  BALLOC(b64, N);
  BALLOC(xacc, N);
  BALLOC(p, N);
  BALLOC(z, N);
  BALLOC(q, N);
  BALLOC(tpart, 4 * (size_t)B->n_tiles);
  SysState* ss;
  BALLOC(ss, (size_t)n_sys);
  uint32_t* bar;
  BALLOC(bar, 4);
#undef BALLOC
  hipError_t e;
  struct Up {
    void* d;
    const void* h;
    size_t bytes;
  } ups[] = {{d_tsys, tsys.data(), 4 * tsys.size()}, {d_tr0, tr0.data(), 4 * tr0.size()},
             {d_tr1, tr1.data(), 4 * tr1.size()},    {d_st0, st0.data(), 4 * st0.size()},
             {d_perm, perm.data(), 4 * N},           {d_rp, rp.data(), 4 * (N + 1)},
             {d_col, col.data(), 4 * (size_t)B->nnz}};
  for (const Up& u : ups)
    if ((e = hipMemcpy(u.d, u.h, u.bytes, hipMemcpyHostToDevice)) != hipSuccess) {
      set_error(PM_HIP_ERROR, std::string("hipMemcpy: ") + hipGetErrorString(e));
      free_batch(B);
      return PM_HIP_ERROR;
    }
  if ((e = hipMemset(bar, 0, 4 * sizeof(uint32_t))) != hipSuccess ||
      (e = hipHostMalloc((void**)&B->h_ss, sizeof(SysState) * n_sys, hipHostMallocDefault)) !=
          hipSuccess) {
    set_error(PM_HIP_ERROR, std::string("batch setup: ") + hipGetErrorString(e));
    free_batch(B);
    return PM_HIP_ERROR;
  }
  a.n_sys = n_sys;
  a.n_tiles = B->n_tiles;
  a.N = B->N;
  a.tile_sys = d_tsys;
  a.tile_r0 = d_tr0;
  a.tile_r1 = d_tr1;
  a.sys_tile0 = d_st0;
  a.perm = d_perm;
  a.rp = d_rp;
  a.col = d_col;
  a.c = dc;
  a.w = dw;
  a.idx = didx;
  a.dp = dp;
  a.x64 = x64;
  a.xlo = xlo;
  a.b64 = b64;
  a.xacc = xacc;
  a.p = p;
  a.z = z;
  a.q = q;
  a.tpart = tpart;
  a.ss = ss;
  a.bar = bar;
  a.spin_limit = 1u << 24;
  *out = B;
  return PM_OK;
}

void pm_batch_destroy(pm_batch* B) { free_batch(B); }

int pm_batch_offsets(const pm_batch* B, int64_t* val_off, int64_t* vec_off) {
  if (!B) {
    set_error(PM_INVALID_ARG, "pm_batch_offsets: null batch");
    return PM_INVALID_ARG;
  }
  if (val_off) std::memcpy(val_off, B->val_off.data(), sizeof(int64_t) * (B->n_sys + 1));
  if (vec_off) std::memcpy(vec_off, B->vec_off.data(), sizeof(int64_t) * (B->n_sys + 1));
  return PM_OK;
}

int pcg_solve_batched(pm_batch* B, const double* val64, const double* b, double* x,
                      const pm_opts* opts, pm_info* infos, hipStream_t s) {
  if (!B || !val64 || !b || !x) {
    set_error(PM_INVALID_ARG, "pcg_solve_batched: null argument");
    return PM_INVALID_ARG;
  }
  pm_opts o;
  pm_opts_default(&o);
  if (opts) o = *opts;
  if (!(o.tol > 0.0) || o.max_it < 0 || o.replace_every < 1 ||
      (o.precision != PM_FP64 && o.precision != PM_MIXED)) {
    set_error(PM_INVALID_ARG, "pcg_solve_batched: invalid options");
    return PM_INVALID_ARG;
  }
  // x on entry is the initial guess unless x0_is_zero: zero it on the device
  if (o.x0_is_zero) PB_HIP(hipMemsetAsync(x, 0, sizeof(double) * B->N, s));
  const void* kern = pick_kernel(o.precision, B->index_bits);
  int dev = 0, ncu = 0, per_cu = 0;
  PB_HIP(hipGetDevice(&dev));
  PB_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  PB_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 256, 0));
  int grid = std::max(1, std::min(per_cu, 4) * ncu);
  if (o.grid > 0) grid = std::min(grid, o.grid);
  BatchArgs a = B->args;
  a.val = val64;
  a.b = b;
  a.x = x;
  a.tol = o.tol;
  a.mrep = o.replace_every;
  a.max_it = o.max_it;
  a.stag_checks = o.stag_checks > 0 ? o.stag_checks : 40;
  const bool same = B->graph && B->g_prec == o.precision && B->g_grid == grid &&
                    B->g_val == val64 && B->g_b == b && B->g_x == x && B->g_opts.tol == o.tol &&
                    B->g_opts.max_it == o.max_it && B->g_opts.replace_every == o.replace_every &&
                    B->g_opts.stag_checks == o.stag_checks;
  if (!same) {
    if (B->graph) {
      (void)hipGraphExecDestroy(B->graph);
      B->graph = nullptr;
    }
    hipGraph_t g = nullptr;
    PB_HIP(hipGraphCreate(&g, 0));
    void* kargs[] = {&a};
    hipKernelNodeParams kp{};
    kp.func = const_cast<void*>(kern);
    kp.gridDim = dim3(grid);
    kp.blockDim = dim3(256);
    kp.sharedMemBytes = 0;
    kp.kernelParams = kargs;
    kp.extra = nullptr;
    hipGraphNode_t node;
    PB_HIP(hipGraphAddKernelNode(&node, g, nullptr, 0, &kp));
    hipKernelNodeAttrValue v{};
    v.cooperative = 1;
    PB_HIP(hipGraphKernelNodeSetAttribute(node, hipKernelNodeAttributeCooperative, &v));
    PB_HIP(hipGraphInstantiate(&B->graph, g, nullptr, nullptr, 0));
    (void)hipGraphDestroy(g);
    B->g_prec = o.precision;
    B->g_grid = grid;
    B->g_val = val64;
    B->g_b = b;
    B->g_x = x;
    B->g_opts = o;
  }
  PB_HIP(hipMemsetAsync(B->args.bar, 0, 4 * sizeof(uint32_t), s));
  PB_HIP(hipGraphLaunch(B->graph, s));
  PB_HIP(hipMemcpyAsync(B->h_ss, B->args.ss, sizeof(SysState) * B->n_sys, hipMemcpyDeviceToHost, s));
  uint32_t abort_flag = 0;
  PB_HIP(hipMemcpyAsync(&abort_flag, B->args.bar + 2, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  PB_HIP(hipStreamSynchronize(s));
  if (abort_flag) {
    set_error(PM_HIP_ERROR, "pcg_solve_batched: grid barrier timed out");
    return PM_HIP_ERROR;
  }
  int worst = PM_OK;
  for (int k = 0; k < B->n_sys; ++k) {
    const SysState& S = B->h_ss[k];
    if (infos) {
      infos[k].iters = S.iter;
      infos[k].status = S.status;
      infos[k].bnorm = std::sqrt(S.bnorm2);
      infos[k].rel_res_true = S.bnorm2 > 0 ? std::sqrt(S.res2 / S.bnorm2) : 0.0;
    }
    if (worst == PM_OK && S.status != PM_OK) worst = S.status;
  }
  if (worst < 0) set_error(worst, "pcg_solve_batched: a system stopped with an error status");
  return worst;
}

}  // extern "C"
