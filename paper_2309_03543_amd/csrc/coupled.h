// Internal: conjugate gradients on the coupled CP1 system of both velocity
// components with the cells' 2x2 diagonal blocks as preconditioner.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "pm_internal.h"

namespace pm {

// Inputs (device pointers; renumbered order unless noted).
struct CoupledIn {
  int n = 0;
  const int* perm = nullptr;     // perm[new] = old
  const int* nb = nullptr;       // [3][n] neighbour (new order) or -1
  const int* pos = nullptr;      // [3][n] CSR slot of that neighbour, -1 on the boundary
  const int* diagpos = nullptr;  // [n] CSR slot of the diagonal
  const double* val_x = nullptr; // CSR values of the x and y matrices
  const double* val_y = nullptr;
  const double* mA = nullptr;    // [n] cell order: M12 A_e
  const double* b_x = nullptr;   // [n] cell order
  const double* b_y = nullptr;
  double* u = nullptr;           // [n] cell order, out
  double* v = nullptr;
};

// Workspace (device unless noted).  The float64 matrix copies, b, x and the
// partials serve both precisions; each precision has its own vectors (and,
// in mixed precision, float32 matrix copies), created on first use.
struct CoupledWork {
  int tile_rows = 0, n_tiles = 0;
  double* w64 = nullptr;    // [3][n] off-diagonal magnitudes (shared by x and y)
  double* dm64 = nullptr;   // [3][n] diagonal of x, diagonal of y, coupling m
  double* inv64 = nullptr;  // [3][n] inverse of each cell's 2x2 block
  double2 *b = nullptr, *x = nullptr;
  double2 *r = nullptr, *z = nullptr, *q = nullptr;  // float64 vectors
  double2* p[2] = {nullptr, nullptr};
  float *w32 = nullptr, *dm32 = nullptr, *inv32 = nullptr;  // mixed precision
  float2 *r32 = nullptr, *z32 = nullptr, *q32 = nullptr;
  float2* p32[2] = {nullptr, nullptr};
  double* part = nullptr;   // [4][n_tiles]: p.q (or the setup / residual sums), r.z of even
                            // and odd iterations, r.z of a replaced residual
  double* scal = nullptr;   // [2]: r.z of even and odd iterations
  int32_t* flag = nullptr;  // [1]
  double* h_part = nullptr; // pinned host [n_tiles + 1]
  bool ready = false, ready64 = false, ready32 = false;
};

constexpr int kCoupledTile = 4096;
constexpr int kCoupledBlock = 512;

inline int coupled_tiles(int n) { return (n + kCoupledTile - 1) / kCoupledTile; }

// Solves; tol, max_it, check_every as in pm_opts (tol, max_it,
// replace_every); precision PM_FP64 or PM_MIXED (its arrays must exist).
int coupled_pcg(const CoupledIn& in, CoupledWork& w, int precision, double tol, int max_it,
                int check_every, pm_info* info, hipStream_t s);

}  // namespace pm
