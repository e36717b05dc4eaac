// Meshes, assembly, single solves and the adjoint on MI355X (gfx950).
//
// This file holds the mesh handle's device structure and its creation, the
// per-cell tensors and the CP1/CP2 matrix assembly (eq. CS1_sys_coeff,
// eq. Cs2_4, eq. CS2_sys_coeff), the adjoint gradient kernel, and the C entry
// points for them and for single-system PCG.  The PCG iteration itself is in
// solver.hip, batched solves in batched.hip, the correction step around the
// solves (cross terms, coupled CP1, fluxes, RT0) in step.hip and the coupled
// CP1 conjugate gradients in coupled.hip.
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

#include "cell.h"
#include "kernels.h"
#include "mesh.h"

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

// Per cell, in the renumbered order: Xi and the diagonal of M = I/dt + nu eps Kfrak.
__global__ void k_cell_tensors(int n, const int* __restrict__ perm, const double* __restrict__ eps,
                               const double* __restrict__ logk, const double* __restrict__ chi,
                               const double* __restrict__ g11, const double* __restrict__ g12,
                               const double* __restrict__ g22, double nu, double dt,
                               double* __restrict__ X11, double* __restrict__ X12,
                               double* __restrict__ X22, double* __restrict__ M11,
                               double* __restrict__ M22, int32_t* err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double e, K11, K12, K22, x11, x12, x22;
  if (!cell_xi(perm[i], eps, logk, chi, g11, g12, g22, nu, dt, e, K11, K12, K22, x11, x12, x22,
               err))
    return;
  M11[i] = 1.0 / dt + nu * e * K11;
  M22[i] = 1.0 / dt + nu * e * K22;
  X11[i] = x11;
  X12[i] = x12;
  X22[i] = x22;
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

namespace pm {
const HostStructure* mesh_structure(const pm_mesh* m) { return &m->hs; }
}  // namespace pm

namespace {

void free_mesh(pm_mesh* m) {
  if (!m) return;
  if (m->pair) pm_batch_destroy(m->pair);
  if (m->h_part) (void)hipHostFree(m->h_part);
  if (m->cw.h_part) (void)hipHostFree(m->cw.h_part);
  set_free(m->set);
  for (void* p : m->allocs) (void)hipFree(p);
  if (m->h_err) (void)hipHostFree(m->h_err);
  delete m;
}

}  // namespace

namespace pm {

int check_opts(const pm_opts& o) {
  if (!(o.tol > 0.0) || o.max_it < 0 || o.replace_every < 1 ||
      (o.precision != PM_FP64 && o.precision != PM_MIXED) || o.tile_rows < 0 || o.block < 0 ||
      o.iter_shape < -1 || o.iter_shape > 5 ||
      (o.precond != PM_PREC_JACOBI && o.precond != PM_PREC_CHEBYSHEV) ||
      (o.precond == PM_PREC_CHEBYSHEV && (o.cheb_degree < 2 || o.cheb_degree > 16))) {
    set_error(PM_INVALID_ARG, "invalid solver options");
    return PM_INVALID_ARG;
  }
  return PM_OK;
}

}  // namespace pm

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
  o->tile_rows = 0;
  o->stag_checks = 40;
  o->iter_shape = 0;
  o->precond = PM_PREC_JACOBI;
  o->cheb_degree = 4;
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
  (void)hipGetDevice(&m->device);

  // per-side arrays in the renumbered order, side-major
  std::vector<int32_t> nb(3 * n), pos(3 * n), diagpos(n);
  std::vector<int8_t> tag(3 * n), nbs(3 * n);
  std::vector<uint8_t> avail(n);
  std::vector<double> T(3 * n), tx(3 * n), ty(3 * n), area(n);
  for (size_t i = 0; i < n; ++i) {
    const size_t old = hs.perm[i];
    area[i] = hs.area[old];
    // a cross-term estimate for side j uses the two other sides, each either
    // interior or a CP2 Dirichlet side
    uint8_t usable = 0;
    for (int j = 0; j < 3; ++j)
      if (hs.nbr[3 * old + j] >= 0 || (hs.tag[3 * old + j] & 2)) usable |= (uint8_t)(1u << j);
    for (int j = 0; j < 3; ++j) {
      const unsigned others = (1u << ((j + 1) % 3)) | (1u << ((j + 2) % 3));
      if ((usable & others) == others) avail[i] |= (uint8_t)(1u << j);
    }
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
      nbs[s] = (int8_t)hs.nbr_side[so];
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
  ALLOC(m->nbs, 3 * n);
  ALLOC(m->avail, n);
  ALLOC(m->eta_r, n);
  ALLOC(m->F, 3 * n);
  ALLOC(m->b2, n);
  ALLOC(m->eta2_r, n);
  ALLOC(m->T, 3 * n);
  ALLOC(m->tx, 3 * n);
  ALLOC(m->ty, 3 * n);
  ALLOC(m->area, n);
  ALLOC(m->X11, n);
  ALLOC(m->X12, n);
  ALLOC(m->X22, n);
  ALLOC(m->M11, n);
  ALLOC(m->M22, n);
  ALLOC(m->asm_err, 1);
#undef ALLOC
  auto fail = [&](hipError_t e, const char* what) {
    set_error(PM_HIP_ERROR, std::string(what) + ": " + hipGetErrorString(e));
    free_mesh(m);
    return PM_HIP_ERROR;
  };
  hipError_t e;
  if ((e = hipHostMalloc((void**)&m->h_err, sizeof(int32_t), hipHostMallocDefault)) != hipSuccess)
    return fail(e, "hipHostMalloc");
  struct Up {
    void* d;
    const void* h;
    size_t bytes;
  } ups[] = {
      {m->perm, hs.perm.data(), 4 * n},        {m->row_ptr, hs.row_ptr.data(), 4 * (n + 1)},
      {m->col, hs.col.data(), 4 * (size_t)m->nnz}, {m->nb, nb.data(), 12 * n},
      {m->pos, pos.data(), 12 * n},            {m->diagpos, diagpos.data(), 4 * n},
      {m->tag, tag.data(), 3 * n},             {m->T, T.data(), 24 * n},
      {m->nbs, nbs.data(), 3 * n},             {m->avail, avail.data(), n},
      {m->tx, tx.data(), 24 * n},              {m->ty, ty.data(), 24 * n},
      {m->area, area.data(), 8 * n},
  };
  for (const Up& u : ups)
    if ((e = hipMemcpy(u.d, u.h, u.bytes, hipMemcpyHostToDevice)) != hipSuccess)
      return fail(e, "hipMemcpy");
  if ((r = set_init(m->set, std::vector<int>{m->n}, m->nnz, hs.stats.index_bits, m->perm,
                    m->row_ptr, m->col)) != PM_OK) {
    free_mesh(m);
    return r;
  }
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

int pm_mesh_set_index_bits(pm_mesh* m, int32_t bits) {
  if (!m || (bits != 16 && bits != 32) || (bits == 16 && m->hs.stats.bandwidth > 32767)) {
    set_error(PM_INVALID_ARG, "pm_mesh_set_index_bits: 16 or 32 bits (16 needs bandwidth <= 32767)");
    return PM_INVALID_ARG;
  }
  set_free(m->set);
  if (int r = set_init(m->set, std::vector<int>{m->n}, m->nnz, bits, m->perm, m->row_ptr, m->col))
    return r;
  m->hs.stats.index_bits = bits;
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
  PM_HIP(hipMemsetAsync(m->asm_err, 0, sizeof(int32_t), s));
  const int nbk = blocks_for(m->n, 256);
  k_cell_tensors<<<nbk, 256, 0, s>>>(m->n, m->perm, prm->eps, prm->logk, prm->chi, prm->g11,
                                     prm->g12, prm->g22, nu, dt, m->X11, m->X12, m->X22, m->M11,
                                     m->M22, m->asm_err);
  k_assemble<<<nbk, 256, 0, s>>>(m->n, kind, m->perm, m->nb, m->pos, m->diagpos, m->tag, m->T,
                                 m->tx, m->ty, m->area, m->X11, m->X12, m->X22, m->M11, m->M22, nu,
                                 g, val64, val32, dinv, b_lift);
  PM_HIP(hipGetLastError());
  PM_HIP(hipMemcpyAsync(m->h_err, m->asm_err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  PM_HIP(hipStreamSynchronize(s));
  if (*m->h_err) {
    set_error(*m->h_err, "assemble_corrector: invalid or non-finite cell parameters");
    return *m->h_err;
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
  set_error(PM_OK, "");
  const int st = set_solve(m->set, val64, b, x, o, info, s);
  // keep a reason the driver gave; a status the device reached gets this one
  if (st < 0 && g_last_status == PM_OK) set_error(st, "pcg_solve stopped with an error status");
  return st;
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
  if (!m) {
    set_error(PM_INVALID_ARG, "pm_time_kernel: null mesh");
    return PM_INVALID_ARG;
  }
  return set_time_kernel(m->set, which, n_launch, s, ms, bytes);
}

int pm_last_launch(const pm_mesh* m, int32_t* tile_rows, int32_t* block, int32_t* iter_shape) {
  if (!m || m->set.last_prec < 0) {
    set_error(PM_INVALID_ARG, "pm_last_launch: null mesh or no solve yet");
    return PM_INVALID_ARG;
  }
  if (tile_rows) *tile_rows = m->set.last_tile;
  if (block) *block = m->set.last_block;
  if (iter_shape) *iter_shape = m->set.last_rows == 0 ? -1 : m->set.last_rows;
  return PM_OK;
}

}  // extern "C"
