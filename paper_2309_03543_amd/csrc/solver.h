// Internal: the PCG driver shared by pcg_solve (one system) and
// pcg_solve_batched (several systems packed one after another).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "pm_internal.h"

namespace pm {

// Per-system solver state (device memory).
struct SysState {
  double alpha, beta, rho;  // current CG scalars
  double bnorm2, tol2;      // ||b||^2 and tol^2 ||b||^2
  double res2;              // last true residual ||b - A x_hi||^2
  double best_res2;         // smallest res2 seen (stagnation test)
  double rho_ring[2];       // r.z of iterations k (slot k & 1), Chebyshev schedule
  double nu_rec;            // r.D'^{-1}r of the recursive residual at the last flush
  int32_t iter;             // completed iterations
  int32_t iter_base;        // completed iterations at the start of the current chunk
  int32_t max_it;
  int32_t stag_it;          // minimum stagnation window (stag_checks * m iterations)
  int32_t done;             // 0 running, 1 stopped, 2 zero right-hand side
  int32_t status;           // PM_* status once stopped
  int32_t k_best;           // iteration at which res2 last fell below best_res2 / 4
  int32_t err;              // input check failure found by the preparation kernel
  int32_t bar_fail;         // a block of the resident chunk kernel gave up waiting
};

// A set of one or more independent systems laid out one after another.
// Rows of system s occupy [row0[s], row0[s+1]); the CSR arrays are the packed
// matrices (columns are global row indices); perm maps each packed row to the
// packed cell-order index of the caller's vectors.
struct SolveSet {
  int N = 0, n_sys = 0;
  int64_t nnz = 0;
  int index_bits = 32;
  std::vector<int> row0;  // host, n_sys + 1
  const int* perm = nullptr;
  const int* rp = nullptr;
  const int* col = nullptr;
  // work tiles (rows of one system each), rebuilt when the tile size changes
  int tile_rows = 0, n_tiles = 0, max_tiles = 0;
  int *tile_sys = nullptr, *tile_r0 = nullptr, *tile_r1 = nullptr, *sys_tile0 = nullptr;
  // columns reached by each tile's rows, [tile_lo, tile_hi], and the widest
  int *tile_lo = nullptr, *tile_hi = nullptr;
  // rows of each tile that some other tile's window reaches: r < pub_lo or
  // r >= pub_hi (the resident chunk kernel publishes only these per iteration)
  int *tile_pub_lo = nullptr, *tile_pub_hi = nullptr;
  int win_max = 0;
  int n_cu = 0;       // compute units of the device (queried once)
  // resident chunk kernel: per tile, at a 64-byte stride, the number of
  // iterations whose results the tile has published in the current launch
  uint32_t* flags = nullptr;
  int resident_spins = 1 << 20;  // bound of each barrier wait (polls)
  int lds_limit = 0;  // bytes of LDS one block may use (queried once)
  // workspace: difference-form rows, vectors, partials, states
  void *c = nullptr, *w = nullptr, *idx = nullptr;
  double *dp = nullptr, *x64 = nullptr, *xlo = nullptr, *b64 = nullptr;
  void* xacc = nullptr;
  void *p[2] = {nullptr, nullptr}, *z[2] = {nullptr, nullptr}, *q[2] = {nullptr, nullptr};
  void* y = nullptr;                       // D'^{-1} r (Chebyshev schedule)
  void* zc[3] = {nullptr, nullptr, nullptr};  // Chebyshev iterates, rotating
  double *part[2] = {nullptr, nullptr}, *part3 = nullptr;
  SysState* ss = nullptr;
  SysState* h_ss = nullptr;  // pinned, 3 slots of n_sys states
  hipStream_t cap = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipEvent_t tev[2] = {nullptr, nullptr};
  hipGraphExec_t graph = nullptr;
  int g_prec = -1, g_m = -1, g_tile = -1, g_block = -1, g_rows = -1, g_pc = -1, g_spins = -1;
  const double* g_val = nullptr;
  // last solve, for the timing hook
  int last_prec = -1, last_tile = 0, last_block = 256, last_rows = 1, last_pc = 0;
  const double* last_val = nullptr;
  std::vector<void*> allocs;
};

int set_init(SolveSet& S, const std::vector<int>& rows_per_sys, int64_t nnz, int index_bits,
             const int* perm, const int* rp, const int* col);
void set_free(SolveSet& S);
int set_solve(SolveSet& S, const double* val64, const double* b, double* x, const pm_opts& o,
              pm_info* infos, hipStream_t s);
int set_time_kernel(SolveSet& S, int which, int n_launch, hipStream_t s, double* ms,
                    double* bytes);

}  // namespace pm
