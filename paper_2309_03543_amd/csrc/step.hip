// The correction step around the two corrector solves (gfx950): the CP2
// cross terms and the two-solve sequence (Sec. 3.2.3, eq. Cs2_7, eq. eta_flux;
// App. C), the coupled anisotropic CP1 (Sec. 3.2.2, eq. cs1_sys2; App. B),
// and the averaged side fluxes and RT0 velocity (eq. flux_k_+_2/3; App. A,
// eq. RT0).
//
// Compiled with -ffp-contract=off.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "cell.h"
#include "kernels.h"
#include "mesh.h"

namespace pm {

// ---------------------------------------------------------------------------
// CP2 cross terms: right-hand side of the second CP2 solve (Sec. 3.2.3,
// eq. Cs2_7 and eq. eta_flux; App. C, eq. A3.1-A3.2)
//
// The flux of Xi grad(eta) through side k of a cell is l_k d_k . grad(eta),
// d_k = Xi_k n_k.  Its tangential part d_{k,tau} = sigma_k t_k / l_k, with
// sigma_k = (Xi_k N_k) . t_k / (t_k . t_k) for the side vector t_k and
// N_k = l_k n_k, is written on the scaled outward normals N_a, N_b of the two
// other sides (co-normal decomposition); by Cramer's rule, with
// D = t_a x t_b (twice the area),
//   l_k d_{k,tau} = (-sigma_k (t_k . t_b) / D) N_a + (sigma_k (t_a . t_k) / D) N_b.
// Each normal derivative N_a . grad(eta) / l_a is the difference quotient
// (v_a - eta) / d_a, d_a = l_a / T_a, so the cell's estimate of
// l_k d_{k,tau} . grad(eta) is sum_a coef_a * T_a * (v_a - eta).  The side's
// term averages the two cells' estimates with opposite signs (each built on
// its own outward normal), which makes it continuous across the side and
// exact for linear eta and constant Xi.
// ---------------------------------------------------------------------------

// Renumbered copies of Xi and of the first solve's eta (cell order in).
__global__ void k_cross_prep(int n, const int* __restrict__ perm, const double* __restrict__ eps,
                             const double* __restrict__ logk, const double* __restrict__ chi,
                             const double* __restrict__ g11, const double* __restrict__ g12,
                             const double* __restrict__ g22, double nu, double dt,
                             const double* __restrict__ eta, double* __restrict__ X11,
                             double* __restrict__ X12, double* __restrict__ X22,
                             double* __restrict__ eta_r, int32_t* err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int o = perm[i];
  const double v = eta[o];
  if (!isfinite(v)) atomicExch(err, PM_NONFINITE);
  eta_r[i] = v;
  double e, K11, K12, K22, x11, x12, x22;
  if (!cell_xi(o, eps, logk, chi, g11, g12, g22, nu, dt, e, K11, K12, K22, x11, x12, x22, err))
    return;
  X11[i] = x11;
  X12[i] = x12;
  X22[i] = x22;
}

// F[k][i] = l_k times cell i's estimate of d_{k,tau} . grad(eta) for its side
// k, or 0 where the estimate would need a Neumann side (bit k of avail clear).
__global__ void __launch_bounds__(256)
k_cross_est(int n, const int* __restrict__ perm, const int* __restrict__ nb,
            const int8_t* __restrict__ tag, const uint8_t* __restrict__ avail,
            const double* __restrict__ T, const double* __restrict__ tx,
            const double* __restrict__ ty, const double* __restrict__ X11,
            const double* __restrict__ X12, const double* __restrict__ X22,
            const double* __restrict__ eta_r, const double* __restrict__ g,
            double* __restrict__ F) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const unsigned av = avail[i];
  const double e = eta_r[i];
  const double x11 = X11[i], x12 = X12[i], x22 = X22[i];
  double sx[3], sy[3], q[3], y11[3], y12[3], y22[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const size_t s = (size_t)k * n + i;
    const int o = nb[s];
    sx[k] = tx[s];
    sy[k] = ty[s];
    double v = 0.0;
    if (o >= 0) {
      v = eta_r[o];
      y11[k] = 0.5 * (x11 + X11[o]);
      y12[k] = 0.5 * (x12 + X12[o]);
      y22[k] = 0.5 * (x22 + X22[o]);
    } else {
      if ((tag[s] & 2) && g) v = g[3 * (size_t)perm[i] + k];
      y11[k] = x11;
      y12[k] = x12;
      y22[k] = x22;
    }
    q[k] = T[s] * (v - e);
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int a = k == 2 ? 0 : k + 1, b = k == 0 ? 2 : k - 1;
    double f = 0.0;
    if (av & (1u << k)) {
      const double Nx = sy[k], Ny = -sx[k];
      const double XNx = y11[k] * Nx + y12[k] * Ny, XNy = y12[k] * Nx + y22[k] * Ny;
      const double sigma = (XNx * sx[k] + XNy * sy[k]) / (sx[k] * sx[k] + sy[k] * sy[k]);
      const double D = sx[a] * sy[b] - sy[a] * sx[b];
      const double ca = -sigma * (sx[k] * sx[b] + sy[k] * sy[b]) / D;
      const double cb = sigma * (sx[a] * sx[k] + sy[a] * sy[k]) / D;
      f = ca * q[a] + cb * q[b];
    }
    F[(size_t)k * n + i] = f;
  }
}

// b_out = b_in + sum_k l_k T_k: the side term is half the difference of the
// two cells' estimates, the one available estimate alone, or (boundary) the
// cell's own estimate on CP2 Dirichlet sides and nothing on Neumann sides.
__global__ void __launch_bounds__(256)
k_cross_rhs(int n, const int* __restrict__ perm, const int* __restrict__ nb,
            const int8_t* __restrict__ nbs, const int8_t* __restrict__ tag,
            const uint8_t* __restrict__ avail, const double* __restrict__ F,
            const double* b_in, double* b_out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const unsigned av = avail[i];
  double t[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const size_t s = (size_t)k * n + i;
    const int o = nb[s];
    const bool mine = (av >> k) & 1u;
    const double f = F[s];
    if (o >= 0) {
      const int kp = nbs[s];
      const bool theirs = (avail[o] >> kp) & 1u;
      const double fo = F[(size_t)kp * n + o];
      t[k] = mine && theirs ? 0.5 * (f - fo) : (mine ? f : (theirs ? -fo : 0.0));
    } else {
      t[k] = mine && (tag[s] & 2) ? f : 0.0;
    }
  }
  const int old = perm[i];
  b_out[old] = b_in[old] + ((t[0] + t[1]) + t[2]);
}

// ---------------------------------------------------------------------------
// Averaged side fluxes after CP1 and the RT0 velocity at the end of the step
// (Sec. 3.2.2, eq. flux_k_+_2/3; Sec. 3.2.3, eq. eta_flux; App. A, eq. RT0)
// ---------------------------------------------------------------------------

// Outward unit normal of the CCW side vector t.
__device__ __forceinline__ void unit_normal(double tx, double ty, double& nx, double& ny,
                                            double& l) {
  l = sqrt(tx * tx + ty * ty);
  nx = ty / l;
  ny = -tx / l;
}

// fbar[e][k]: an interior side carries the two cells' normal fluxes averaged
// with the other cell's area as weight, (u_e.n A_ep + u_ep.n A_e) / (A_e +
// A_ep) l (n the outward normal of e); a side with a prescribed velocity (CP1
// Dirichlet bit) carries (g.n) l, any other boundary side (u_e.n) l.  The
// expression gives bitwise opposite values from the two cells.  b1[e] is the
// sum of the three.
__global__ void k_flux_avg(int n, const int* __restrict__ perm, const int* __restrict__ nb,
                           const int8_t* __restrict__ tag, const double* __restrict__ tx,
                           const double* __restrict__ ty, const double* __restrict__ area,
                           const double* __restrict__ u, const double* __restrict__ v,
                           const double* __restrict__ gu, const double* __restrict__ gv,
                           double* __restrict__ fbar, double* __restrict__ b1) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int old = perm[i];
  const double ue = u[old], ve = v[old], Ae = area[i];
  double f[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const size_t s = (size_t)k * n + i;
    double nx, ny, l;
    unit_normal(tx[s], ty[s], nx, ny, l);
    const double une = ue * nx + ve * ny;
    const int o = nb[s];
    if (o >= 0) {
      const int oo = perm[o];
      const double Ao = area[o];
      const double unp = u[oo] * nx + v[oo] * ny;
      f[k] = (une * Ao + unp * Ae) / (Ae + Ao) * l;
    } else if (tag[s] & 1) {
      const double gx = gu ? gu[3 * (size_t)old + k] : 0.0;
      const double gy = gv ? gv[3 * (size_t)old + k] : 0.0;
      f[k] = (gx * nx + gy * ny) * l;
    } else {
      f[k] = une * l;
    }
    fbar[3 * (size_t)old + k] = f[k];
  }
  if (b1) b1[old] = (f[0] + f[1]) + f[2];
}

// Renumbered copy of a cell-order vector.
__global__ void k_gather(int n, const int* __restrict__ perm, const double* __restrict__ src,
                         double* __restrict__ dst, int32_t* err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double x = src[perm[i]];
  if (!isfinite(x)) atomicExch(err, PM_NONFINITE);
  dst[i] = x;
}

// Q = fbar + Fl^eta per side, with Fl^eta the two-point flux of eta (the
// CP2 matrix weight times the difference; on a CP2 Dirichlet side the
// boundary weight times g - eta) plus the tangential term of the cross
// estimates F of eta~ (as in k_cross_rhs); then the RT0 field
// u(x) = sum_k Q_k (x - x_k) / (2 A) at the centroid, where centroid - x_k
// = (t_{k+2} - t_{k+1}) / 3 in side vectors.
__global__ void __launch_bounds__(256)
k_rt0(int n, const int* __restrict__ perm, const int* __restrict__ nb,
      const int8_t* __restrict__ nbs, const int8_t* __restrict__ tag,
      const uint8_t* __restrict__ avail, const double* __restrict__ T,
      const double* __restrict__ tx, const double* __restrict__ ty,
      const double* __restrict__ area, const double* __restrict__ X11,
      const double* __restrict__ X12, const double* __restrict__ X22,
      const double* __restrict__ eta_r, const double* __restrict__ F,
      const double* __restrict__ g, const double* __restrict__ fbar,
      double* __restrict__ u_out, double* __restrict__ v_out, double* __restrict__ q_out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int old = perm[i];
  const unsigned av = avail[i];
  const double e = eta_r[i];
  const double x11 = X11[i], x12 = X12[i], x22 = X22[i];
  double Q[3], sx[3], sy[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const size_t s = (size_t)k * n + i;
    const int o = nb[s];
    sx[k] = tx[s];
    sy[k] = ty[s];
    const bool mine = (av >> k) & 1u;
    const double f = F[s];
    double normal = 0.0, tang = 0.0;
    if (o >= 0) {
      const double a11 = 0.5 * (x11 + X11[o]);
      const double a12 = 0.5 * (x12 + X12[o]);
      const double a22 = 0.5 * (x22 + X22[o]);
      const double w = T[s] * normal_quadratic(sx[k], sy[k], a11, a12, a22);
      normal = w * (eta_r[o] - e);
      const int kp = nbs[s];
      const bool theirs = (avail[o] >> kp) & 1u;
      const double fo = F[(size_t)kp * n + o];
      tang = mine && theirs ? 0.5 * (f - fo) : (mine ? f : (theirs ? -fo : 0.0));
    } else if (tag[s] & 2) {
      const double w = T[s] * normal_quadratic(sx[k], sy[k], x11, x12, x22);
      normal = w * ((g ? g[3 * (size_t)old + k] : 0.0) - e);
      tang = mine ? f : 0.0;
    }
    Q[k] = (fbar[3 * (size_t)old + k] + normal) + tang;
    if (q_out) q_out[3 * (size_t)old + k] = Q[k];
  }
  double ux = 0.0, uy = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int a = k == 2 ? 0 : k + 1, b = k == 0 ? 2 : k - 1;
    ux += Q[k] * (sx[b] - sx[a]);
    uy += Q[k] * (sy[b] - sy[a]);
  }
  const double c = 1.0 / (6.0 * area[i]);
  u_out[old] = ux * c;
  v_out[old] = uy * c;
}

// ---------------------------------------------------------------------------
// Coupled CP1 (Sec. 3.2.2, eq. cs1_sys2 and eq. CS1_sys_coeff; App. B,
// eq. A1): with anisotropic permeability M12 = nu eps Kfrak_12 couples the x
// and y systems through the cell term M12 A_e.  The loop of App. B solves
// both scalar systems, then repeatedly re-solves them with the coupling
// evaluated at the other component's previous iterate.  Vectors of the pair
// are packed [x | y] in cell order.
// ---------------------------------------------------------------------------

// m_e = M12_e A_e in cell order (one thread per renumbered cell).
__global__ void k_cp1_mass(int n, const int* __restrict__ perm, const double* __restrict__ eps,
                           const double* __restrict__ logk, const double* __restrict__ chi,
                           const double* __restrict__ g11, const double* __restrict__ g12,
                           const double* __restrict__ g22, double nu, double dt,
                           const double* __restrict__ area, double* __restrict__ mA,
                           int32_t* err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int o = perm[i];
  double e, K11, K12, K22, x11, x12, x22;
  if (!cell_xi(o, eps, logk, chi, g11, g12, g22, nu, dt, e, K11, K12, K22, x11, x12, x22, err))
    return;
  mA[o] = (nu * e * K12) * area[i];
}

// Right-hand sides of a coupled pass from the previous iterate xp = [u | v]:
// [b_x - m v | b_y - m u]; the iterate is kept in prev for the change test.
__global__ void k_cp1_couple(int n, const double* __restrict__ mA, const double* __restrict__ bx,
                             const double* __restrict__ by, const double* __restrict__ xp,
                             double* __restrict__ bp, double* __restrict__ prev) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const double u = xp[e], v = xp[(size_t)n + e], m = mA[e];
  bp[e] = bx[e] - m * v;
  bp[(size_t)n + e] = by[e] - m * u;
  prev[e] = u;
  prev[(size_t)n + e] = v;
}

// Per-block partial sums of |u' - u|^2, |u|^2, |v' - v|^2, |v|^2 (new
// iterate xp, previous prev), grid-stride, written to part[block][4].
__global__ void __launch_bounds__(256)
k_cp1_change(int n, const double* __restrict__ xp, const double* __restrict__ prev,
             double* __restrict__ part) {
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
    const double u0 = prev[e], v0 = prev[(size_t)n + e];
    const double du = xp[e] - u0, dv = xp[(size_t)n + e] - v0;
    acc[0] += du * du;
    acc[1] += u0 * u0;
    acc[2] += dv * dv;
    acc[3] += v0 * v0;
  }
  block_partial<4>(acc, part + 4 * (size_t)blockIdx.x);
}

}  // namespace pm

using namespace pm;

namespace {

// The three kernels of cp2_cross_rhs, each bracketed by an event pair when ev
// is given (ev[0..5]).
void launch_cross(pm_mesh* m, const pm_cell_params* prm, double nu, double dt, const double* g,
                  const double* eta, const double* b_in, double* b_out, hipStream_t s,
                  hipEvent_t* ev) {
  const int nbk = blocks_for(m->n, 256);
  if (ev) (void)hipEventRecord(ev[0], s);
  k_cross_prep<<<nbk, 256, 0, s>>>(m->n, m->perm, prm->eps, prm->logk, prm->chi, prm->g11,
                                   prm->g12, prm->g22, nu, dt, eta, m->X11, m->X12, m->X22,
                                   m->eta_r, m->asm_err);
  if (ev) (void)hipEventRecord(ev[1], s);
  if (ev) (void)hipEventRecord(ev[2], s);
  k_cross_est<<<nbk, 256, 0, s>>>(m->n, m->perm, m->nb, m->tag, m->avail, m->T, m->tx, m->ty,
                                  m->X11, m->X12, m->X22, m->eta_r, g, m->F);
  if (ev) (void)hipEventRecord(ev[3], s);
  if (ev) (void)hipEventRecord(ev[4], s);
  k_cross_rhs<<<nbk, 256, 0, s>>>(m->n, m->perm, m->nb, m->nbs, m->tag, m->avail, m->F, b_in,
                                  b_out);
  if (ev) (void)hipEventRecord(ev[5], s);
}

int cross_args_ok(const pm_mesh* m, const pm_cell_params* prm, double nu, double dt,
                  const double* eta, const double* b_in, const double* b_out, const char* who) {
  if (!m || !prm || !prm->eps || !prm->logk || !eta || !b_in || !b_out || !(dt > 0.0) ||
      !(nu >= 0.0) || !std::isfinite(nu) || !std::isfinite(dt)) {
    set_error(PM_INVALID_ARG, std::string(who) + ": invalid argument");
    return PM_INVALID_ARG;
  }
  return PM_OK;
}

}  // namespace

extern "C" {

int cp2_cross_rhs(pm_mesh* m, const pm_cell_params* prm, double nu, double dt, const double* g,
                  const double* eta_tilde, const double* b_in, double* b_out, hipStream_t s) {
  if (int r = cross_args_ok(m, prm, nu, dt, eta_tilde, b_in, b_out, "cp2_cross_rhs")) return r;
  PM_HIP(hipMemsetAsync(m->asm_err, 0, sizeof(int32_t), s));
  launch_cross(m, prm, nu, dt, g, eta_tilde, b_in, b_out, s, nullptr);
  PM_HIP(hipGetLastError());
  PM_HIP(hipMemcpyAsync(m->h_err, m->asm_err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  PM_HIP(hipStreamSynchronize(s));
  if (*m->h_err) {
    set_error(*m->h_err, "cp2_cross_rhs: invalid or non-finite cell parameters or eta");
    return *m->h_err;
  }
  return PM_OK;
}

int cp2_solve_two_step(pm_mesh* m, const double* val64, const pm_cell_params* prm, double nu,
                       double dt, const double* g, const double* b, double* eta_tilde, double* eta,
                       const pm_opts* opts, pm_info* info, hipStream_t s) {
  if (!m || !val64 || !b || !eta_tilde || !eta || eta == eta_tilde || eta == b ||
      eta_tilde == b) {
    set_error(PM_INVALID_ARG, "cp2_solve_two_step: null or aliased vectors");
    return PM_INVALID_ARG;
  }
  if (int r = cross_args_ok(m, prm, nu, dt, eta_tilde, b, eta, "cp2_solve_two_step")) return r;
  pm_opts o;
  pm_opts_default(&o);
  if (opts) o = *opts;
  o.x0_is_zero = 1;
  const int st1 = pcg_solve(m, val64, b, eta_tilde, &o, info, s);
  if (st1 < 0) return st1;
  if (int r = cp2_cross_rhs(m, prm, nu, dt, g, eta_tilde, b, m->b2, s)) return r;
  PM_HIP(hipMemcpyAsync(eta, eta_tilde, sizeof(double) * (size_t)m->n, hipMemcpyDeviceToDevice, s));
  o.x0_is_zero = 0;
  const int st2 = pcg_solve(m, val64, m->b2, eta, &o, info ? info + 1 : nullptr, s);
  if (st2 < 0) return st2;
  return st1 != PM_OK ? st1 : st2;
}

}  // extern "C"

namespace {

constexpr int kChangeBlocks = 512;

// The pair batch and its workspace, on first use.
int ensure_pair(pm_mesh* m) {
  if (m->pair) return PM_OK;
  pm_mesh* two[2] = {m, m};
  pm_batch* b = nullptr;
  if (int r = pm_batch_create(2, two, &b)) return r;
  const size_t n = m->n;
  int r = PM_OK;
  if ((r = dalloc(m, &m->pv, 2 * (size_t)m->nnz)) || (r = dalloc(m, &m->pb, 2 * n)) ||
      (r = dalloc(m, &m->px, 2 * n)) || (r = dalloc(m, &m->pprev, 2 * n)) ||
      (!m->mA && (r = dalloc(m, &m->mA, n))) ||
      (r = dalloc(m, &m->ppart, 4 * (size_t)kChangeBlocks))) {
    pm_batch_destroy(b);
    return r;
  }
  hipError_t e = hipHostMalloc((void**)&m->h_part, sizeof(double) * 4 * kChangeBlocks,
                               hipHostMallocDefault);
  if (e != hipSuccess) {
    pm_batch_destroy(b);
    set_error(PM_HIP_ERROR, std::string("hipHostMalloc: ") + hipGetErrorString(e));
    return PM_HIP_ERROR;
  }
  m->pair = b;
  return PM_OK;
}

// The coupled-CG workspace of one precision (and the shared part), on first
// use.
int ensure_coupled(pm_mesh* m, int precision) {
  CoupledWork& w = m->cw;
  const size_t n = m->n;
  int r = PM_OK;
  if (!w.ready) {
    w.tile_rows = kCoupledTile;
    w.n_tiles = coupled_tiles(m->n);
    if ((!m->mA && (r = dalloc(m, &m->mA, n))) || (r = dalloc(m, &w.w64, 3 * n)) ||
        (r = dalloc(m, &w.dm64, 3 * n)) || (r = dalloc(m, &w.b, n)) ||
        (r = dalloc(m, &w.x, n)) || (r = dalloc(m, &w.part, 4 * (size_t)w.n_tiles)) ||
        (r = dalloc(m, &w.scal, 2)) || (r = dalloc(m, &w.flag, 1)))
      return r;
    hipError_t e = hipHostMalloc((void**)&w.h_part, sizeof(double) * (w.n_tiles + 1),
                                 hipHostMallocDefault);
    if (e != hipSuccess) {
      w.h_part = nullptr;
      set_error(PM_HIP_ERROR, std::string("hipHostMalloc: ") + hipGetErrorString(e));
      return PM_HIP_ERROR;
    }
    w.ready = true;
  }
  if (precision == PM_FP64 && !w.ready64) {
    if ((r = dalloc(m, &w.inv64, 3 * n)) || (r = dalloc(m, &w.r, n)) || (r = dalloc(m, &w.z, n)) ||
        (r = dalloc(m, &w.q, n)) || (r = dalloc(m, &w.p[0], n)) || (r = dalloc(m, &w.p[1], n)))
      return r;
    w.ready64 = true;
  }
  if (precision == PM_MIXED && !w.ready32) {
    if ((r = dalloc(m, &w.w32, 3 * n)) || (r = dalloc(m, &w.dm32, 3 * n)) ||
        (r = dalloc(m, &w.inv32, 3 * n)) || (r = dalloc(m, &w.r32, n)) ||
        (r = dalloc(m, &w.z32, n)) || (r = dalloc(m, &w.q32, n)) ||
        (r = dalloc(m, &w.p32[0], n)) || (r = dalloc(m, &w.p32[1], n)))
      return r;
    w.ready32 = true;
  }
  return PM_OK;
}

// Adds the per-system iteration counts of a batched pair solve to info.
void add_infos(pm_info* acc, const pm_info* last) {
  for (int c = 0; c < 2; ++c) {
    const int32_t it = acc[c].iters + last[c].iters;
    const int32_t st = acc[c].status != PM_OK ? acc[c].status : last[c].status;
    acc[c] = last[c];
    acc[c].iters = it;
    acc[c].status = st;
  }
}

}  // namespace

extern "C" {

int cp1_solve_coupled(pm_mesh* m, const pm_cell_params* prm, double nu, double dt,
                      const double* val_x, const double* val_y, const double* b_x,
                      const double* b_y, double* u, double* v, double toll, int32_t max_outer,
                      const pm_opts* opts, pm_info* info, int32_t* n_outer, double* err,
                      hipStream_t s) {
  if (!m || !prm || !prm->eps || !prm->logk || !val_x || !val_y || !b_x || !b_y || !u || !v ||
      u == v || !(toll >= 0.0) || max_outer < 0 || !(dt > 0.0) || !(nu >= 0.0) ||
      !std::isfinite(nu) || !std::isfinite(dt)) {
    set_error(PM_INVALID_ARG, "cp1_solve_coupled: invalid argument");
    return PM_INVALID_ARG;
  }
  pm_opts o;
  pm_opts_default(&o);
  if (opts) o = *opts;
  if (int r = check_opts(o)) return r;
  if (int r = ensure_pair(m)) return r;
  const size_t n = m->n, nnz = m->nnz;
  const int nbk = blocks_for(m->n, 256);
  PM_HIP(hipMemsetAsync(m->asm_err, 0, sizeof(int32_t), s));
  k_cp1_mass<<<nbk, 256, 0, s>>>(m->n, m->perm, prm->eps, prm->logk, prm->chi, prm->g11,
                                 prm->g12, prm->g22, nu, dt, m->area, m->mA, m->asm_err);
  PM_HIP(hipGetLastError());
  PM_HIP(hipMemcpyAsync(m->pv, val_x, sizeof(double) * nnz, hipMemcpyDeviceToDevice, s));
  PM_HIP(hipMemcpyAsync(m->pv + nnz, val_y, sizeof(double) * nnz, hipMemcpyDeviceToDevice, s));
  PM_HIP(hipMemcpyAsync(m->pb, b_x, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  PM_HIP(hipMemcpyAsync(m->pb + n, b_y, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  PM_HIP(hipMemcpyAsync(m->h_err, m->asm_err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  PM_HIP(hipStreamSynchronize(s));
  if (*m->h_err) {
    set_error(*m->h_err, "cp1_solve_coupled: invalid or non-finite cell parameters");
    return *m->h_err;
  }
  pm_info acc[2] = {}, last[2] = {};
  // uncoupled first pass (App. B: the coupling term starts at zero)
  o.x0_is_zero = 1;
  int st = pcg_solve_batched(m->pair, m->pv, m->pb, m->px, &o, last, s);
  add_infos(acc, last);
  if (st < 0) {
    if (info) std::memcpy(info, acc, sizeof(acc));
    return st;
  }
  o.x0_is_zero = 0;
  int pass = 0;
  double e_min = INFINITY;
  bool met = false;
  while (pass < max_outer) {
    k_cp1_couple<<<nbk, 256, 0, s>>>(m->n, m->mA, b_x, b_y, m->px, m->pb, m->pprev);
    PM_HIP(hipGetLastError());
    st = pcg_solve_batched(m->pair, m->pv, m->pb, m->px, &o, last, s);
    add_infos(acc, last);
    ++pass;
    if (st < 0) break;
    k_cp1_change<<<kChangeBlocks, 256, 0, s>>>(m->n, m->px, m->pprev, m->ppart);
    PM_HIP(hipGetLastError());
    PM_HIP(hipMemcpyAsync(m->h_part, m->ppart, sizeof(double) * 4 * kChangeBlocks,
                          hipMemcpyDeviceToHost, s));
    PM_HIP(hipStreamSynchronize(s));
    double sum[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = 0; b < kChangeBlocks; ++b)
      for (int k = 0; k < 4; ++k) sum[k] += m->h_part[4 * b + k];
    // err_c = sqrt(||c' - c||) / sqrt(||c||), a zero iterate settled only if unchanged
    auto comp = [](double d2, double o2) {
      if (o2 == 0.0) return d2 == 0.0 ? 0.0 : (double)INFINITY;
      return std::sqrt(std::sqrt(d2)) / std::sqrt(std::sqrt(o2));
    };
    e_min = std::min(comp(sum[0], sum[1]), comp(sum[2], sum[3]));
    if (e_min <= toll) {
      met = true;
      break;
    }
  }
  PM_HIP(hipMemcpyAsync(u, m->px, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  PM_HIP(hipMemcpyAsync(v, m->px + n, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  PM_HIP(hipStreamSynchronize(s));
  if (info) std::memcpy(info, acc, sizeof(acc));
  if (n_outer) *n_outer = pass;
  if (err) *err = pass > 0 ? e_min : INFINITY;
  if (st < 0) return st;
  if (st != PM_OK) return st;
  return met || max_outer == 0 ? PM_OK : PM_MAXIT;
}

int cp1_solve_coupled_pcg(pm_mesh* m, const pm_cell_params* prm, double nu, double dt,
                          const double* val_x, const double* val_y, const double* b_x,
                          const double* b_y, double* u, double* v, const pm_opts* opts,
                          pm_info* info, hipStream_t s) {
  if (!m || !prm || !prm->eps || !prm->logk || !val_x || !val_y || !b_x || !b_y || !u || !v ||
      u == v || !(dt > 0.0) || !(nu >= 0.0) || !std::isfinite(nu) || !std::isfinite(dt)) {
    set_error(PM_INVALID_ARG, "cp1_solve_coupled_pcg: invalid argument");
    return PM_INVALID_ARG;
  }
  pm_opts o;
  pm_opts_default(&o);
  if (opts) o = *opts;
  if (int r = check_opts(o)) return r;
  if (int r = ensure_coupled(m, o.precision)) return r;
  PM_HIP(hipMemsetAsync(m->asm_err, 0, sizeof(int32_t), s));
  k_cp1_mass<<<blocks_for(m->n, 256), 256, 0, s>>>(m->n, m->perm, prm->eps, prm->logk, prm->chi,
                                                   prm->g11, prm->g12, prm->g22, nu, dt, m->area,
                                                   m->mA, m->asm_err);
  PM_HIP(hipGetLastError());
  PM_HIP(hipMemcpyAsync(m->h_err, m->asm_err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  PM_HIP(hipStreamSynchronize(s));
  if (*m->h_err) {
    set_error(*m->h_err, "cp1_solve_coupled_pcg: invalid or non-finite cell parameters");
    return *m->h_err;
  }
  CoupledIn in;
  in.n = m->n;
  in.perm = m->perm;
  in.nb = m->nb;
  in.pos = m->pos;
  in.diagpos = m->diagpos;
  in.val_x = val_x;
  in.val_y = val_y;
  in.mA = m->mA;
  in.b_x = b_x;
  in.b_y = b_y;
  in.u = u;
  in.v = v;
  return coupled_pcg(in, m->cw, o.precision, o.tol, o.max_it, o.replace_every, info, s);
}

int flux_average(pm_mesh* m, const double* u, const double* v, const double* g_u,
                 const double* g_v, double* fbar, double* b1, hipStream_t s) {
  if (!m || !u || !v || !fbar) {
    set_error(PM_INVALID_ARG, "flux_average: invalid argument");
    return PM_INVALID_ARG;
  }
  k_flux_avg<<<blocks_for(m->n, 256), 256, 0, s>>>(m->n, m->perm, m->nb, m->tag, m->tx, m->ty,
                                                   m->area, u, v, g_u, g_v, fbar, b1);
  PM_HIP(hipGetLastError());
  return PM_OK;
}

int rt0_update(pm_mesh* m, const pm_cell_params* prm, double nu, double dt, const double* g,
               const double* eta_tilde, const double* eta, const double* fbar, double* u_out,
               double* v_out, double* q_out, hipStream_t s) {
  if (int r = cross_args_ok(m, prm, nu, dt, eta_tilde, fbar, u_out, "rt0_update")) return r;
  if (!eta || !v_out || u_out == v_out) {
    set_error(PM_INVALID_ARG, "rt0_update: invalid argument");
    return PM_INVALID_ARG;
  }
  const int nbk = blocks_for(m->n, 256);
  PM_HIP(hipMemsetAsync(m->asm_err, 0, sizeof(int32_t), s));
  k_cross_prep<<<nbk, 256, 0, s>>>(m->n, m->perm, prm->eps, prm->logk, prm->chi, prm->g11,
                                   prm->g12, prm->g22, nu, dt, eta_tilde, m->X11, m->X12, m->X22,
                                   m->eta_r, m->asm_err);
  k_cross_est<<<nbk, 256, 0, s>>>(m->n, m->perm, m->nb, m->tag, m->avail, m->T, m->tx, m->ty,
                                  m->X11, m->X12, m->X22, m->eta_r, g, m->F);
  k_gather<<<nbk, 256, 0, s>>>(m->n, m->perm, eta, m->eta2_r, m->asm_err);
  k_rt0<<<nbk, 256, 0, s>>>(m->n, m->perm, m->nb, m->nbs, m->tag, m->avail, m->T, m->tx, m->ty,
                            m->area, m->X11, m->X12, m->X22, m->eta2_r, m->F, g, fbar, u_out,
                            v_out, q_out);
  PM_HIP(hipGetLastError());
  PM_HIP(hipMemcpyAsync(m->h_err, m->asm_err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  PM_HIP(hipStreamSynchronize(s));
  if (*m->h_err) {
    set_error(*m->h_err, "rt0_update: invalid or non-finite cell parameters, eta or eta~");
    return *m->h_err;
  }
  return PM_OK;
}

int pm_time_cross(pm_mesh* m, const pm_cell_params* prm, double nu, double dt, const double* g,
                  const double* eta_tilde, const double* b_in, double* b_out, int32_t n_launch,
                  hipStream_t s, double* ms, double* bytes) {
  if (int r = cross_args_ok(m, prm, nu, dt, eta_tilde, b_in, b_out, "pm_time_cross")) return r;
  if (n_launch < 1 || !ms || b_in == b_out) {
    set_error(PM_INVALID_ARG, "pm_time_cross: n_launch < 1, ms null or b_in == b_out");
    return PM_INVALID_ARG;
  }
  hipEvent_t ev[6];
  for (auto& e : ev) PM_HIP(hipEventCreate(&e));
  double acc[3] = {0.0, 0.0, 0.0};
  PM_HIP(hipMemsetAsync(m->asm_err, 0, sizeof(int32_t), s));
  launch_cross(m, prm, nu, dt, g, eta_tilde, b_in, b_out, s, nullptr);  // warm-up
  int st = PM_OK;
  for (int it = 0; it < n_launch && st == PM_OK; ++it) {
    launch_cross(m, prm, nu, dt, g, eta_tilde, b_in, b_out, s, ev);
    if (hipEventSynchronize(ev[5]) != hipSuccess) st = PM_HIP_ERROR;
    for (int k = 0; k < 3 && st == PM_OK; ++k) {
      float t = 0.0f;
      if (hipEventElapsedTime(&t, ev[2 * k], ev[2 * k + 1]) != hipSuccess) st = PM_HIP_ERROR;
      acc[k] += t;
    }
  }
  for (auto& e : ev) (void)hipEventDestroy(e);
  if (st != PM_OK) {
    set_error(st, "pm_time_cross: event timing failed");
    return st;
  }
  PM_HIP(hipMemcpyAsync(m->h_err, m->asm_err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  PM_HIP(hipStreamSynchronize(s));
  if (*m->h_err) {
    set_error(*m->h_err, "pm_time_cross: invalid or non-finite cell parameters or eta");
    return *m->h_err;
  }
  for (int k = 0; k < 3; ++k) ms[k] = acc[k] / n_launch;
  if (bytes) {
    // Algorithmic bytes (every array element read or written once):
    //   prep  perm, eta, eps, logk (+ chi, g11, g12, g22 when given) in; Xi (3) and eta out
    //   est   avail, eta, Xi (3), per side nb, tag, T, tx, ty in; F (3 per cell) out
    //   rhs   perm, avail, F (3), per side nb, nbs, tag, b_in in; b_out out
    // (Dirichlet values g are read on boundary sides only and not counted.)
    const double n = m->n;
    const int given = (prm->chi != nullptr) + (prm->g11 != nullptr) + (prm->g12 != nullptr) +
                      (prm->g22 != nullptr);
    bytes[0] = n * (4 + 8 + 16 + 8.0 * given + 24 + 8);
    bytes[1] = n * (1 + 8 + 24 + 3 * (4 + 1 + 8 + 8 + 8) + 24);
    bytes[2] = n * (4 + 1 + 24 + 3 * (4 + 1 + 1) + 8 + 8);
  }
  return PM_OK;
}

}  // extern "C"
