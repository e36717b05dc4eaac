// Internal: the mesh handle and the host helpers shared by the HIP
// translation units of the library.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <vector>

#include "coupled.h"
#include "pm_internal.h"
#include "solver.h"

// Returns PM_HIP_ERROR with a message when a HIP runtime call fails.
#define PM_HIP(expr)                                                                  \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess) {                                                           \
      pm::set_error(PM_HIP_ERROR, std::string(#expr) + ": " + hipGetErrorString(e_)); \
      return PM_HIP_ERROR;                                                            \
    }                                                                                 \
  } while (0)

struct pm_mesh {
  pm::HostStructure hs;
  int device = 0;
  int32_t n = 0, nnz = 0;
  // structure, renumbered order
  int32_t *perm = nullptr, *row_ptr = nullptr, *col = nullptr;
  int32_t *nb = nullptr, *pos = nullptr, *diagpos = nullptr;  // nb/pos: [3][n]
  int8_t* tag = nullptr;                                       // [3][n]
  int8_t* nbs = nullptr;     // [3][n] side index of the neighbour, -1 on the boundary
  uint8_t* avail = nullptr;  // [n] bit k: the CP2 cross-term estimate of side k exists
  double *T = nullptr, *tx = nullptr, *ty = nullptr, *area = nullptr;
  // assembly scratch and its input-check flag
  double *X11 = nullptr, *X12 = nullptr, *X22 = nullptr, *M11 = nullptr, *M22 = nullptr;
  int32_t* asm_err = nullptr;
  int32_t* h_err = nullptr;  // pinned
  // CP2 cross-term workspace (renumbered order)
  double *eta_r = nullptr, *F = nullptr;  // [n], [3][n]
  double* b2 = nullptr;                   // [n] second right-hand side, cell order
  double* eta2_r = nullptr;               // [n] renumbered eta for the RT0 update
  // coupled CP1: a two-system batch of this mesh (x, y) and its packed
  // vectors, created by the first cp1_solve_coupled call
  pm_batch* pair = nullptr;
  double *pv = nullptr, *pb = nullptr, *px = nullptr, *pprev = nullptr;  // [2 nnz], [2n] x3
  double *mA = nullptr, *ppart = nullptr, *h_part = nullptr;           // [n], [blocks][4], pinned
  // coupled CP1 conjugate gradients: workspace, created by the first call
  pm::CoupledWork cw;
  // the solver workspace (a set with one system)
  pm::SolveSet set;
  std::vector<void*> allocs;
};

namespace pm {

// Device allocation owned by the mesh (freed by pm_mesh_destroy).
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

inline int blocks_for(int n, int b) { return (n + b - 1) / b; }

// PM_OK, or PM_INVALID_ARG with a message for out-of-range solver options.
int check_opts(const pm_opts& o);

}  // namespace pm
