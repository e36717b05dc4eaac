// Batched corrector PCG: several independent systems (for instance
// permeability realisations on meshes of different sizes) packed one after
// another and solved together by the tile-based iteration of solver.hip.
//
// Each system keeps its own reverse Cuthill-McKee order, scalars, stopping
// test and stop flag; tiles never straddle two systems, so one launch of each
// iteration kernel advances every active system, and a system that has
// converged is masked out of the launches that follow.  One replay of the
// captured HIP graph runs m iterations of the whole batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstring>
#include <string>
#include <vector>

#include "pm_internal.h"
#include "solver.h"

using namespace pm;

struct pm_batch {
  int n_sys = 0;
  std::vector<int64_t> val_off, vec_off;
  int* perm = nullptr;
  int* rp = nullptr;
  int* col = nullptr;
  SolveSet set;
  std::vector<void*> allocs;
};

namespace {

void free_batch(pm_batch* B) {
  if (!B) return;
  set_free(B->set);
  for (void* p : B->allocs) (void)hipFree(p);
  delete B;
}

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
  std::vector<int> rows(n_sys);
  for (int s = 0; s < n_sys; ++s) {
    B->val_off[s + 1] = B->val_off[s] + hs[s]->stats.nnz;
    B->vec_off[s + 1] = B->vec_off[s] + hs[s]->n;
    rows[s] = hs[s]->n;
    max_bw = std::max(max_bw, hs[s]->stats.bandwidth);
  }
  if (B->vec_off[n_sys] > INT32_MAX / 4 || B->val_off[n_sys] > INT32_MAX) {
    set_error(PM_INVALID_ARG, "pm_batch_create: batch too large for 32-bit indexing");
    free_batch(B);
    return PM_INVALID_ARG;
  }
  const size_t N = (size_t)B->vec_off[n_sys], nnz = (size_t)B->val_off[n_sys];
  std::vector<int> perm(N), rp(N + 1), col(nnz);
  for (int s = 0; s < n_sys; ++s) {
    const HostStructure& h = *hs[s];
    const int off = (int)B->vec_off[s], voff = (int)B->val_off[s];
    for (int i = 0; i < h.n; ++i) {
      perm[off + i] = off + h.perm[i];
      rp[off + i] = voff + h.row_ptr[i];
    }
    for (int k = 0; k < h.stats.nnz; ++k) col[voff + k] = off + h.col[k];
  }
  rp[N] = (int)nnz;
  int r;
  if ((r = balloc(B, &B->perm, N)) || (r = balloc(B, &B->rp, N + 1)) ||
      (r = balloc(B, &B->col, nnz))) {
    free_batch(B);
    return r;
  }
  hipError_t e;
  if ((e = hipMemcpy(B->perm, perm.data(), 4 * N, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(B->rp, rp.data(), 4 * (N + 1), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(B->col, col.data(), 4 * nnz, hipMemcpyHostToDevice)) != hipSuccess) {
    set_error(PM_HIP_ERROR, std::string("hipMemcpy: ") + hipGetErrorString(e));
    free_batch(B);
    return PM_HIP_ERROR;
  }
  if ((r = set_init(B->set, rows, (int64_t)nnz, max_bw <= 32767 ? 16 : 32, B->perm, B->rp,
                    B->col)) != PM_OK) {
    free_batch(B);
    return r;
  }
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
  if (!(o.tol > 0.0) || o.max_it < 0 || o.replace_every < 1 || o.tile_rows < 0 || o.block < 0 ||
      (o.precision != PM_FP64 && o.precision != PM_MIXED) ||
      o.iter_shape < -1 || o.iter_shape > 3 ||
      (o.precond != PM_PREC_JACOBI && o.precond != PM_PREC_CHEBYSHEV) ||
      (o.precond == PM_PREC_CHEBYSHEV && (o.cheb_degree < 2 || o.cheb_degree > 16))) {
    set_error(PM_INVALID_ARG, "pcg_solve_batched: invalid options");
    return PM_INVALID_ARG;
  }
  const int worst = set_solve(B->set, val64, b, x, o, infos, s);
  if (worst < 0) set_error(worst, "pcg_solve_batched: a system stopped with an error status");
  return worst;
}

}  // extern "C"
