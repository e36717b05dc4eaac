/*
 * pmcorr — corrector-system PCG for the mesoscopic one-domain
 * Navier-Stokes-Brinkman solver of Arico, Helmig, Puleo and Schneider
 * (arXiv 2309.03543), on AMD Instinct MI355X (gfx950).
 *
 * The two corrector problems of the fractional time step (Sec. 3.1, eq. cs1
 * and eq. cs2) reduce, per time step, to sparse symmetric positive definite
 * M-matrix systems on an unstructured Delaunay triangulation, one unknown per
 * triangle (Sec. 3.2.2, eq. CS1_sys_coeff; Sec. 3.2.3, eq. CS2_sys_coeff).
 * This library builds their sparsity once per mesh, assembles their values
 * from per-cell porosity and permeability on the GPU, and solves them with
 * Jacobi- or Chebyshev-polynomial-preconditioned conjugate gradients on the
 * GPU (single systems or batches of systems of uneven size).  Around the
 * solves it provides
 *   - a hand-written adjoint for gradients with respect to the cell
 *     parameters;
 *   - the co-normal cross terms that form the right-hand side of the second
 *     CP2 solve, and that two-solve sequence;
 *   - the coupled anisotropic CP1 (the paper's loop, or conjugate gradients
 *     on both components);
 *   - the averaged side fluxes that feed the CP2 and the RT0 velocity after
 *     it.
 *
 * Conventions shared by every entry point
 *   - Triangles are given counter-clockwise; side j of triangle e is the side
 *     opposite node j, i.e. from node (j+1)%3 to node (j+2)%3 (Appendix A).
 *   - side_tag[e*3+j] is a bit mask for boundary sides: bit 0 marks a Dirichlet
 *     side of CP1, bit 1 a Dirichlet side of CP2.  Untagged boundary sides are
 *     Neumann (no matrix term).  Tags on interior sides are ignored.
 *   - Public vectors (right-hand sides, solutions, per-cell parameters,
 *     gradients) are indexed by the caller's cell order.  Matrices are CSR
 *     with rows and columns in the library's reverse Cuthill-McKee order,
 *     which pm_mesh_export / pm_structure_host reveal (perm[new] = old).
 *   - Device pointers are owned by the caller; the library never frees them.
 *     Handles (pm_mesh, pm_batch) own their device workspace, freed by the
 *     matching *_destroy.  Calls on one handle must not overlap in time.
 *   - Every call returns a status (PM_OK = 0, > 0 warnings, < 0 errors) and
 *     never throws.  Work is ordered on the caller's HIP stream; calls that
 *     report solver information (pcg_*) block the host until it is known.
 */
#ifndef PMCORR_H
#define PMCORR_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define PM_OK 0
#define PM_MAXIT 1          /* iteration limit reached before the tolerance */
#define PM_STAGNATED 2      /* the true residual stopped decreasing near the float64
                               rounding floor of the system, which lies above tol */
#define PM_INVALID_ARG (-1) /* bad sizes, null pointers, out-of-range indices or tags */
#define PM_BAD_MESH (-2)    /* clockwise/degenerate triangle, repeated node, non-manifold side */
#define PM_NOT_DELAUNAY (-3) /* interior side with d <= 0, or Dirichlet side whose
                                circumcenter-to-side distance is <= 0 */
#define PM_SINGULAR (-4)    /* CP2 on a mesh component without a CP2 Dirichlet side */
#define PM_NONFINITE (-5)   /* NaN/Inf in coordinates, parameters, matrix or right-hand side */
#define PM_BREAKDOWN (-6)   /* p.Ap <= 0 or not finite during PCG */
#define PM_HIP_ERROR (-7)   /* a HIP runtime call failed (message via pm_last_error) */

/* corrector kinds */
#define PM_CP1X 0 /* eq. CS1_sys_coeff, x component: diagonal M11*A_e + nu*sum l/d */
#define PM_CP1Y 1 /* eq. CS1_sys_coeff, y component: diagonal M22*A_e + nu*sum l/d */
#define PM_CP2 2  /* eq. CS2_sys_coeff: coefficients (l/d) * (Xi_j n_j).n_j */

/* precisions */
#define PM_FP64 0  /* all vectors and the matrix in float64 */
#define PM_MIXED 1 /* float32 matrix and Krylov vectors; float64 solution,
                      residual replacement and convergence test */

/* preconditioners (both fully data-parallel; the paper's incomplete Cholesky
   needs sequential triangular sweeps) */
#define PM_PREC_JACOBI 0    /* z = D^-1 r */
#define PM_PREC_CHEBYSHEV 1 /* z = p(D^-1 A) D^-1 r: cheb_degree steps of Chebyshev
                               acceleration of the Jacobi iteration for A z = r from
                               z = 0 on [2/30, 2]; 2 bounds the spectrum of D^-1 A
                               (Gershgorin on a weakly diagonally dominant M-matrix) */

typedef struct pm_mesh pm_mesh;
typedef struct pm_batch pm_batch;

typedef struct {
  int32_t n_cells;
  int32_t n_nodes;
  int32_t nnz;              /* n_cells + 2 * n_interior_sides */
  int32_t n_interior_sides;
  int32_t n_boundary_sides;
  int32_t bandwidth;        /* max |row - col| in the renumbered matrix */
  int32_t n_components;     /* connected components of the cell graph */
  int32_t index_bits;       /* 16 or 32: width of the column offsets the solver streams */
  double max_T;             /* largest transmissibility l/d */
  double min_cot_sum;       /* smallest cot(t_e)+cot(t_ep) over interior sides */
} pm_mesh_stats;

/*
 * Per-cell coefficients, device pointers of length n_cells in cell order.
 *   eps   porosity (> 0)
 *   logk  s = ln K, natural log of the permeability scale
 *   chi   transition factor in [0,1] multiplying the inverse permeability;
 *         NULL means 1
 *   g11, g12, g22  normalised inverse-shape tensor G (symmetric positive
 *         definite); NULL means identity.  Inverse permeability
 *         Kfrak = chi * exp(-s) * G (Sec. 2: Kfrak = K^{-1}; eq. aniso gives
 *         G = R diag(beta,1) R^T).
 */
typedef struct {
  const double* eps;
  const double* logk;
  const double* chi;
  const double* g11;
  const double* g12;
  const double* g22;
} pm_cell_params;

typedef struct {
  double tol;            /* stop when ||b - A x||_2 <= tol * ||b||_2 (default 1e-10) */
  int32_t max_it;        /* iteration limit (default 200000) */
  int32_t precision;     /* PM_FP64 or PM_MIXED */
  int32_t replace_every; /* true-residual replacement period m (default 50); the
                            stopping test runs at these points */
  int32_t x0_is_zero;    /* 1: ignore x on entry and start from 0 */
  int32_t block;         /* threads per block of the iteration kernels when
                            tile_rows is given (0 = 256; rounded down to a
                            multiple of 64, at most 512) */
  int32_t tile_rows;     /* rows per work tile (one block each; >= 256); 0 = tile,
                            block and rows per thread chosen by the built-in
                            tuner, which times the fused iteration kernel on the
                            first solve of a problem shape and precision */
  int32_t stag_checks;   /* PM_STAGNATED once the best true residual is within
                            100x of the rounding floor u*|| |A||x| || and has
                            not halved for max(stag_checks * replace_every,
                            k_best) iterations, k_best being the iteration of
                            the last halving (default 40) */
  int32_t precond;       /* PM_PREC_JACOBI (default) or PM_PREC_CHEBYSHEV */
  int32_t cheb_degree;   /* Chebyshev polynomial degree, 2..16 (default 4): each
                            application costs degree - 1 products with A */
  int32_t iter_shape;    /* with tile_rows: the iteration schedule, -1 split
                            (update kernel, then product kernel), 1 or 2 the
                            fused kernel with that many rows per thread and
                            trip (0 = 1), 3 the fused kernel with the tile's
                            column window staged in LDS (PM_INVALID_ARG if it
                            does not fit), 4 the resident chunk kernel: one
                            launch runs the m - 1 fused iterations of a chunk
                            with every tile's rows held on chip and a grid
                            barrier between iterations (one system whose
                            tiles all fit the device at once, tile_rows at
                            most 8 x block; else PM_INVALID_ARG; pcg_solve
                            only).  Each barrier wait is bounded; if one
                            gives up (the grid was not all resident, e.g.
                            compute units held by another process), the
                            solve restarts on schedule 3 (or 1) with the
                            same tiles, which computes bitwise the same
                            iterations, and pm_last_launch reports that
                            schedule.  The environment variable
                            PMCORR_RESIDENT_SPINS sets the bound in polls
                            (default 2^20, about a second).  5 the resident
                            window kernel: the same, for operators too large
                            to hold on chip (one tile per compute unit):
                            only each tile's column window of p and z stays
                            in LDS, the matrix rows, x_acc and q~ are read
                            every iteration.  Ignored when the tuner
                            decides */
} pm_opts;

typedef struct {
  int32_t iters;         /* PCG iterations performed */
  int32_t status;        /* PM_OK, PM_MAXIT, PM_STAGNATED or an error */
  double rel_res_true;   /* ||b - A x||_2 / ||b||_2 of the returned x, residual
                            evaluated with error-free transformations (exact
                            up to the final rounding) */
  double bnorm;          /* ||b||_2 */
} pm_info;

/* Defaults for pm_opts (tol 1e-10, FP64, m = 50, x0 = 0, tuned launch). */
void pm_opts_default(pm_opts* opts);

/* Human-readable name of a status code. */
const char* pm_status_string(int status);

/* Copies the message of the last failing call on this thread into buf
 * (NUL-terminated, truncated to len) and returns its status. */
int pm_last_error(char* buf, int32_t len);

/*
 * Host-only mesh analysis (no GPU needed): validation, per-side
 * transmissibilities, reverse Cuthill-McKee order and the CSR pattern.
 *   xy       [n_nodes][2] host float64 node coordinates
 *   tri      [n_cells][3] host int32 CCW node indices
 *   side_tag [n_cells][3] host int8 boundary bit masks (see above)
 *   perm     [n_cells] out: perm[new] = old
 *   row_ptr  [n_cells+1] out, col [col_capacity] out (needs nnz <= col_capacity;
 *            4*n_cells always suffices)
 *   T        [n_cells][3] out, nullable: l/d per side in cell order (interior:
 *            2/(cot t_e + cot t_ep); boundary: 2/cot t; 0 where cot t <= 0)
 *   stats    out, nullable
 * Geometry follows Sec. 3.2.2 (eq. cs1_discr, d = signed circumcenter
 * distance) using the identity d = (l/2)(cot t_e + cot t_ep).
 * Errors: PM_INVALID_ARG, PM_NONFINITE, PM_BAD_MESH, PM_NOT_DELAUNAY.
 */
int pm_structure_host(int32_t n_nodes, const double* xy, int32_t n_cells, const int32_t* tri,
                      const int8_t* side_tag, int32_t* perm, int32_t* row_ptr, int32_t* col,
                      int32_t col_capacity, double* T, pm_mesh_stats* stats);

/*
 * Builds the mesh structure (as pm_structure_host) and uploads it with the
 * solver workspace to the current HIP device.  Inputs are host arrays and
 * are not retained.  *out receives a handle owned by the caller.
 */
int pm_mesh_create(int32_t n_nodes, const double* xy, int32_t n_cells, const int32_t* tri,
                   const int8_t* side_tag, pm_mesh** out);
void pm_mesh_destroy(pm_mesh* mesh);
int pm_mesh_get_stats(const pm_mesh* mesh, pm_mesh_stats* stats);
/*
 * Sets the width of the column offsets the solver streams for this mesh's
 * single-system solves: 32 always works; 16, the default whenever it fits,
 * needs an RCM bandwidth of at most 32767.  Wider offsets cost 6 bytes more
 * per row and iteration; the call lets the 32-bit path run on meshes of any
 * size (test it, or compare).  It resets the mesh's solver workspace;
 * pm_mesh_get_stats reports the width in use.  Errors: PM_INVALID_ARG.
 */
int pm_mesh_set_index_bits(pm_mesh* mesh, int32_t bits);
/* Host copies of the ordering and the CSR pattern (sizes n_cells, n_cells+1, nnz). */
int pm_mesh_export(const pm_mesh* mesh, int32_t* perm, int32_t* row_ptr, int32_t* col);

/*
 * Assembles a corrector matrix on the GPU (eq. CS1_sys_coeff for PM_CP1X /
 * PM_CP1Y, eq. CS2_sys_coeff for PM_CP2), with
 *   M = I/dt + nu*eps*Kfrak            (Sec. 3.1: M0 = I + m dt, M = M0/dt)
 *   Xi = eps * M^{-1}                  (eq. Cs2_4)
 *   CP1 side weight  w = nu * T
 *   CP2 side weight  w = T * n.((Xi_e + Xi_ep)/2).n   (boundary side: Xi_e)
 *   a(e,ep) = -w;  a(e,e) = sum of side weights + Dirichlet weights
 *                            + (CP1x: M11*A_e | CP1y: M22*A_e | CP2: 0).
 * Dirichlet sides of the kind contribute T-weighted terms to the diagonal and
 * w * g to b_lift; Neumann sides contribute nothing.
 *   params       device, cell order (see pm_cell_params)
 *   g_dirichlet  device [n_cells][3] Dirichlet values per side, cell order;
 *                nullable (= 0)
 *   val64        device [nnz] out, CSR values in the mesh's renumbered order
 *   val32        device [nnz] out, nullable: val64 rounded to float32
 *   dinv         device [n_cells] out, nullable: 1/diagonal, renumbered order
 *   b_lift       device [n_cells] out, nullable: Dirichlet right-hand side, cell order
 * Errors: PM_INVALID_ARG, PM_SINGULAR (CP2 with a component lacking a CP2
 * Dirichlet side), PM_NONFINITE (non-finite or non-positive eps, non-finite
 * parameters; checked on the device, reported after a stream sync).
 */
int assemble_corrector(pm_mesh* mesh, int32_t kind, const pm_cell_params* params, double nu,
                       double dt, const double* g_dirichlet, double* val64, float* val32,
                       double* dinv, double* b_lift, hipStream_t stream);

/*
 * Solves A x = b with Jacobi-preconditioned CG (Sec. 3.2.2 / 3.2.3 solve the
 * corrector systems by PCG; the diagonal preconditioner replaces the paper's
 * incomplete Cholesky).  The stopping test is the true residual
 * ||b - A x||_2 <= tol ||b||_2, evaluated every replace_every iterations, where
 * the recursive residual is also replaced by it and the accumulated increments
 * are folded into x (group update).  x is carried as a double-double sum
 * x_hi + x_lo between replacement points; the returned x is x_hi and the
 * stopping test is the exact residual of that float64 vector.  PM_MIXED runs
 * the Krylov recurrence on float32 copies with the same float64 solution,
 * residual and test.
 *   val64  device [nnz], CSR values on the mesh's pattern (renumbered order),
 *          e.g. from assemble_corrector
 *   b      device [n_cells], cell order
 *   x      device [n_cells], cell order; initial guess in (unless
 *          opts->x0_is_zero), solution out
 *   opts   host, nullable (defaults); info host out, nullable
 * Returns info->status (PM_OK, PM_MAXIT, PM_STAGNATED, PM_BREAKDOWN) or an
 * error.  PM_OK always means the float64 test passed.  A breakdown
 * (p.Ap <= 0 or not finite) whose returned x passes the test is PM_OK.  CG
 * ends within n iterations, so on a system of a few rows p.Ap reaches zero
 * before the next test.  A recurrence that reaches an exactly zero residual,
 * or breaks down after progress, while the test fails (float32 storage on
 * such a system) goes on from the returned x, at most four more passes;
 * info->iters counts all of them.
 */
int pcg_solve(pm_mesh* mesh, const double* val64, const double* b, double* x, const pm_opts* opts,
              pm_info* info, hipStream_t stream);

/*
 * Groups several meshes (for instance permeability realisations on meshes of
 * different sizes) for one batched solve.  The meshes must outlive the batch.
 */
int pm_batch_create(int32_t n_sys, pm_mesh* const* meshes, pm_batch** out);
void pm_batch_destroy(pm_batch* batch);
/* Offsets of system s in packed value and vector arrays: val_off[n_sys+1], vec_off[n_sys+1]. */
int pm_batch_offsets(const pm_batch* batch, int64_t* val_off, int64_t* vec_off);

/*
 * Solves all systems of the batch together with the algorithm and stopping
 * rule of pcg_solve: every launch of an iteration kernel covers the row tiles
 * of all systems still running, each system with its own scalars, test and
 * stop flag (a converged system is masked out of later launches); one replay
 * of the captured HIP graph advances the whole batch by replace_every
 * iterations.
 *   val64  device, packed: system s occupies [val_off[s], val_off[s+1])
 *   b, x   device, packed by vec_off, cell order within each system
 *   infos  host [n_sys] out, nullable
 * Returns PM_OK if every system converged, else the first non-OK status.
 */
int pcg_solve_batched(pm_batch* batch, const double* val64, const double* b, double* x,
                      const pm_opts* opts, pm_info* infos, hipStream_t stream);

/*
 * Adjoint of x = A(theta)^{-1} (b + b_lift(theta)) for a loss L(x): solves
 * A lambda = dL/dx with pcg_solve's algorithm (A is symmetric), then forms
 *   dL/dtheta_c = lambda . (d b_lift/dtheta_c - (dA/dtheta_c) x)
 * for theta = ln K and eps of every cell with one cell-wise gather kernel.
 *   params, nu, dt, g_dirichlet  as given to assemble_corrector
 *   val64      device [nnz], the assembled matrix
 *   eta        device [n_cells], the forward solution, cell order
 *   grad_eta   device [n_cells], dL/d eta, cell order
 *   lambda     device [n_cells] out (= dL/db), cell order
 *   grad_logk, grad_eps  device [n_cells] out, cell order
 */
int pcg_adjoint(pm_mesh* mesh, int32_t kind, const pm_cell_params* params, double nu, double dt,
                const double* g_dirichlet, const double* val64, const double* eta,
                const double* grad_eta, double* lambda, double* grad_logk, double* grad_eps,
                const pm_opts* opts, pm_info* info, hipStream_t stream);

/*
 * Right-hand side of the second CP2 solve (Sec. 3.2.3, eq. Cs2_7 and
 * eq. eta_flux; App. C, eq. A3.1-A3.2).  On a non-K-orthogonal mesh the flux
 * of Xi grad(eta) through a side has, beside the two-point normal part of the
 * matrix, a tangential part d_{j,tau} . grad(eta), d_j = Xi_j n_j.  Each cell
 * writes d_{j,tau} on the outward normals of its two other sides (co-normal
 * decomposition) and estimates each normal derivative by the circumcenter
 * difference quotient used by the matrix; the side's term is half the
 * difference of the two cells' estimates (each built on its own outward
 * normal), so it is continuous across the side and exact for linear eta and
 * constant Xi.  With eta~ the solution of A eta~ = b_in (eq. Cs2_7, first
 * system) this computes
 *   b_out = b_in + sum_j l_j T_j(eta~)
 * and A eta = b_out is the second system.  Boundary sides: a CP2 Dirichlet
 * side takes its g_dirichlet value in place of a neighbour's eta and carries
 * its own cell's estimate; an estimate that would need a Neumann side is
 * dropped (an interior side then takes the other cell's estimate alone);
 * Neumann sides carry no tangential term.  Isotropic Xi gives b_out = b_in.
 *   params, nu, dt, g_dirichlet  as given to assemble_corrector for PM_CP2
 *   eta_tilde  device [n_cells], cell order
 *   b_in       device [n_cells], cell order: the first system's right-hand side
 *   b_out      device [n_cells] out, cell order; may equal b_in
 * Errors: PM_INVALID_ARG, PM_NONFINITE (non-finite parameters or eta_tilde;
 * checked on the device, reported after a stream sync).  Uses the mesh's
 * workspace: calls on one mesh must not overlap in time.
 */
int cp2_cross_rhs(pm_mesh* mesh, const pm_cell_params* params, double nu, double dt,
                  const double* g_dirichlet, const double* eta_tilde, const double* b_in,
                  double* b_out, hipStream_t stream);

/*
 * The CP2 sequence of eq. Cs2_7 with one matrix: eta~ from A eta~ = b (zero
 * initial guess), then eta from A eta = cp2_cross_rhs(eta~, b), starting from
 * eta~.  Both solves use pcg_solve with opts (x0_is_zero is ignored).
 *   val64            device [nnz], the PM_CP2 matrix of assemble_corrector
 *   params .. g      as given to assemble_corrector for PM_CP2
 *   b                device [n_cells], cell order: B_1 plus the Dirichlet lift
 *   eta_tilde, eta   device [n_cells] out, cell order; distinct from b and
 *                    from each other
 *   info             host [2] out, nullable: the two solves
 * Returns the first negative status, else the first non-OK one, else PM_OK.
 * The sequence is one step of the fixed-point iteration
 * eta <- A^{-1}(b + C eta) for the full flux (C: the cross terms); it moves
 * eta~ towards the full solution when that iteration contracts, which holds
 * for mild anisotropy of Xi but not for eigenvalue ratios of Xi above about
 * eight on the meshes tested.
 */
int cp2_solve_two_step(pm_mesh* mesh, const double* val64, const pm_cell_params* params, double nu,
                       double dt, const double* g_dirichlet, const double* b, double* eta_tilde,
                       double* eta, const pm_opts* opts, pm_info* info, hipStream_t stream);

/*
 * Coupled CP1 velocity correction for anisotropic permeability (Sec. 3.2.2,
 * eq. cs1_sys2 and eq. CS1_sys_coeff; App. B, eq. A1).  The mass tensor's
 * off-diagonal M12 = nu eps Kfrak_12 couples the two components through the
 * cell term m_e = M12_e A_e:
 *   A_x u + m v = b_x,   m u + A_y v = b_y.
 * Following App. B, both scalar systems are solved without the coupling
 * (zero initial guess), then up to max_outer passes re-solve both with the
 * coupling taken from the other component's previous iterate (both from
 * the same iterate), each solve warm-started at that component's previous
 * iterate, until
 *   err = min(err_x, err_y) <= toll,  err_x = sqrt(||u' - u||_2) / sqrt(||u||_2)
 * (likewise y; the square roots are as printed, so err <= toll bounds a
 * relative change by toll^2; a zero iterate counts as settled only if it
 * stays zero).  The two systems of a pass are solved together as a batch of
 * two with pcg_solve_batched's algorithm and opts (x0_is_zero is ignored).
 *   params, nu, dt  as given to assemble_corrector
 *   val_x, val_y    device [nnz]: the PM_CP1X and PM_CP1Y matrices
 *   b_x, b_y        device [n_cells], cell order (Dirichlet lifts included)
 *   u, v            device [n_cells] out, cell order; distinct
 *   toll            >= 0 (the paper uses 1e-4 to 1e-3)
 *   info            host [2] out, nullable: per component, iters summed
 *                   over all passes, the first non-OK status, and the last
 *                   solve's residual
 *   n_outer         host out, nullable: coupled passes run
 *   err             host out, nullable: err of the last pass (+inf if none)
 * Returns PM_OK when the test was met (or max_outer is 0), PM_MAXIT when
 * max_outer passes did not meet it, else the first non-OK solve status.  The
 * first call on a mesh creates a two-system batch of it (with its own solver
 * workspace) and 2 nnz + 7 n doubles more, kept until pm_mesh_destroy.  The loop is block Jacobi
 * on the coupled system, which is symmetric positive definite, so it
 * converges to the coupled solution.
 */
int cp1_solve_coupled(pm_mesh* mesh, const pm_cell_params* params, double nu, double dt,
                      const double* val_x, const double* val_y, const double* b_x,
                      const double* b_y, double* u, double* v, double toll, int32_t max_outer,
                      const pm_opts* opts, pm_info* info, int32_t* n_outer, double* err,
                      hipStream_t stream);

/*
 * The coupled CP1 system of cp1_solve_coupled,
 *   A_x u + m v = b_x,   m u + A_y v = b_y,   m_e = M12_e A_e,
 * solved directly by conjugate gradients on both components together, with
 * the inverse of each cell's 2x2 diagonal block [[A_x,ee, m_e], [m_e, A_y,ee]]
 * as preconditioner.  This is not the paper's procedure (App. B iterates over
 * the two scalar systems); the system is symmetric positive definite (nu
 * times the Laplacian on each component, plus each cell's SPD mass tensor
 * times A_e, plus the Dirichlet terms), and one solve reaches the limit of
 * that iteration.  Starting from zero, every opts.replace_every iterations
 * the true residual ||b - C x||_2 (float64) is evaluated and the solve stops
 * once it is <= opts.tol ||b||_2.  PM_FP64: every value is float64 and the
 * recursive residual is not replaced.  PM_MIXED: the Krylov vectors and the
 * per-iteration copies of the weights, diagonal blocks and block inverses are
 * stored in float32 (arithmetic in float64); x, b and the residual check stay
 * float64, and every check replaces the recursive residual by the true one
 * (the direction restarts when the replaced r.z exceeds the recursive one a
 * hundredfold).
 *   params, nu, dt  as given to assemble_corrector (for m)
 *   val_x, val_y    device [nnz]: the PM_CP1X and PM_CP1Y matrices; their
 *                   off-diagonals must agree (both are -nu T)
 *   b_x, b_y        device [n_cells], cell order (Dirichlet lifts included)
 *   u, v            device [n_cells] out, cell order; distinct
 *   opts            tol, max_it, replace_every and precision apply; the other
 *                   fields are ignored
 *   info            host out, nullable: iterations, status, the true
 *                   relative residual of (u, v) and ||b||
 * Errors: PM_INVALID_ARG (arguments, off-diagonals that differ, a cell
 * block that is not positive definite), PM_NONFINITE, PM_BREAKDOWN.  A
 * breakdown (p.q <= 0) after (u, v) met the tolerance is PM_OK.  With
 * PM_MIXED on a mesh of a few cells, the float32 recurrence can reach
 * p.q = 0 before the float64 test passes.  There is no restart, so that
 * case is PM_BREAKDOWN.  The first call on a mesh allocates a workspace of 13 n doubles, and the first
 * call of each precision 13 n doubles (float64) or 19 n floats (mixed) more,
 * kept until pm_mesh_destroy.
 */
int cp1_solve_coupled_pcg(pm_mesh* mesh, const pm_cell_params* params, double nu, double dt,
                          const double* val_x, const double* val_y, const double* b_x,
                          const double* b_y, double* u, double* v, const pm_opts* opts,
                          pm_info* info, hipStream_t stream);

/*
 * Side fluxes after CP1 (Sec. 3.2.2, eq. flux_k_+_2/3): for cell velocities
 * (u, v), an interior side j of e carries the two cells' normal fluxes
 * averaged with the other cell's area as weight,
 *   fbar = (u_e . n_j A_ep + u_ep . n_j A_e) / (A_e + A_ep) l_j
 * (n_j the outward normal of e), the same value with opposite sign from ep.
 * A boundary side with the CP1 Dirichlet bit carries (g . n_j) l_j with g
 * = (g_u, g_v) the prescribed velocity of that side; any other boundary side
 * carries (u_e . n_j) l_j.  b1 = sum_j fbar_j is the CP2 source B_1 of
 * eq. CS2_sys_coeff.
 *   u, v        device [n_cells], cell order
 *   g_u, g_v    device [n_cells][3], cell order, nullable (= 0)
 *   fbar        device [n_cells][3] out, cell order
 *   b1          device [n_cells] out, cell order, nullable
 * Asynchronous on the stream; PM_INVALID_ARG for null arguments.
 */
int flux_average(pm_mesh* mesh, const double* u, const double* v, const double* g_u,
                 const double* g_v, double* fbar, double* b1, hipStream_t stream);

/*
 * Velocity at the end of the step (Sec. 3.2.3, eq. eta_flux and the RT0
 * reconstruction after it; App. A, eq. RT0).  Per side
 *   Q_j = fbar_j + Fl_j^eta,
 * Fl^eta the flux of Xi grad(eta): the two-point part of eta with the CP2
 * matrix's weights (interior: w (eta_ep - eta_e); CP2 Dirichlet side:
 * w_b (g - eta_e); Neumann: 0) plus the tangential cross term of eta~ (as in
 * cp2_cross_rhs).  The cell sums of Q are the residual b_out - A eta of the
 * second CP2 system, so they vanish when it is solved.  The velocity is the
 * RT0 field u(x) = sum_j Q_j (x - x_j) / (2 A_e) (x_j the node opposite side
 * j) at the centroid: its constant value when the sums vanish.
 *   params .. g     as given to assemble_corrector for PM_CP2
 *   eta_tilde, eta  device [n_cells], cell order: the two CP2 solutions
 *   fbar            device [n_cells][3], cell order (flux_average)
 *   u_out, v_out    device [n_cells] out, cell order
 *   q_out           device [n_cells][3] out, cell order, nullable
 * Errors: PM_INVALID_ARG, PM_NONFINITE (parameters, eta or eta~; reported
 * after a stream sync).  Uses the mesh's workspace: calls on one mesh must
 * not overlap in time.
 */
int rt0_update(pm_mesh* mesh, const pm_cell_params* params, double nu, double dt,
               const double* g_dirichlet, const double* eta_tilde, const double* eta,
               const double* fbar, double* u_out, double* v_out, double* q_out,
               hipStream_t stream);

/*
 * Measurement hook for cp2_cross_rhs: runs it n_launch times (after one
 * warm-up) with HIP events around each of its three kernels and returns the
 * mean durations in ms (ms[3]: per-cell preparation of Xi and eta~, the
 * estimates, the right-hand side) and the bytes each must move (bytes[3],
 * nullable), counting every array element once: n (60 + 8 g) with g the
 * number of the optional chi, g11, g12, g22 given; n (57 + 3 (4 + 1 + 24)) =
 * 144 n; n (29 + 3 * 6 + 16) = 63 n.  Dirichlet values are not counted.
 * b_in and b_out must differ here (b_out is overwritten n_launch + 1 times).
 */
int pm_time_cross(pm_mesh* mesh, const pm_cell_params* params, double nu, double dt,
                  const double* g_dirichlet, const double* eta_tilde, const double* b_in,
                  double* b_out, int32_t n_launch, hipStream_t stream, double* ms,
                  double* bytes);

/*
 * Measurement hook: runs one of the solver's iteration kernels n_launch times
 * on the state left by the last pcg_solve of this mesh (same precision and
 * launch shape) between two HIP events on `stream`, and returns the mean
 * duration in milliseconds and the bytes one launch must move.
 *   which  0: plain matrix-vector product with fused dot products (opens
 *             each chunk of m iterations)
 *          1: one iteration of the schedule in use: the fused kernel
 *             (update of x, z, p and the product of the new direction with
 *             its dot products in one launch), or on the split schedule the
 *             update kernel followed by the product; timed with zero step
 *             lengths, so the state does not change.  On the resident
 *             schedule n_launch launches of m - 1 iterations each are timed
 *             (m = replace_every of the last solve) and the time per
 *             iteration is returned
 *          2: true-residual kernel (float64 CSR, compensated)
 * Bytes per launch, n rows, vector/weight/index widths sv/sw/si:
 *   0: n (4 sw + 3 si + 3 sv)
 *   1: n (4 sw + 3 si + 8 sv) fused, n (4 sw + 3 si + 10 sv) split
 *   2: 12 nnz + 4 (n + 1) + 24 n
 */
int pm_time_kernel(pm_mesh* mesh, int32_t which, int32_t n_launch, hipStream_t stream,
                   double* ms_per_launch, double* bytes_per_launch);

/*
 * Launch shape of the last pcg_solve on this mesh: rows per tile, threads per
 * block and the iteration schedule (pm_opts.iter_shape encoding: 1, 2, 3 or -1),
 * as chosen by the tuner or given in pm_opts.  Returns PM_INVALID_ARG before
 * the first solve.
 */
int pm_last_launch(const pm_mesh* mesh, int32_t* tile_rows, int32_t* block, int32_t* iter_shape);

#ifdef __cplusplus
}
#endif
#endif /* PMCORR_H */
