/*
 * invdft.h — C ABI of the MI355X (gfx950) inverse-DFT hot path.
 *
 * The library solves the discrete problems of finite-element inverse DFT:
 * the standard-form Kohn-Sham eigenproblem H~ psi~ = eps psi~ (Eq. 19), the
 * adjoint equations (H~ - eps_i) q_i = b_i with q_i orthogonal to the occupied
 * orbitals (Eqs. 7, 10, 20 and the null-space treatment of Sec. 3.2.2), the
 * density and loss (Eqs. 1, 4) and the gradient with respect to the nodal
 * exchange-correlation potential (Eqs. 11, 22).
 *
 * Discretisation: box [-L, L]^3 with n x n x n hexahedral cells of order-p
 * spectral elements (tensor-product Lagrange polynomials on Gauss-Lobatto-
 * Legendre nodes, Eq. 12, Sec. 3.2.1). Homogeneous Dirichlet boundary; the
 * unknowns are the N_f = (p n - 1)^3 interior nodes, numbered
 *     a = (gx - 1) + n1 * ((gy - 1) + n1 * (gz - 1)),  n1 = p n - 1,
 * with 1-D global node g = e p + j of cell e. The stiffness is integrated
 * exactly, the overlap M is lumped by GLL quadrature into W = diag(W_a), and
 * the potential is collocated at the nodes, so
 *     H~ = (1/2) W^{-1/2} K W^{-1/2} + diag(v).
 *
 * Layout ("node-major", Sec. 3.2.3 and Fig. 4a): a block X of nv vectors is
 * stored as X[a * ld + j], a in [0, N_f), j in [0, nv), ld >= nv: all
 * coefficients of one basis function are contiguous.
 *
 * Pointers: every array argument is DEVICE memory unless its name ends in _h
 * (host memory). The caller owns every buffer it passes; the library keeps no
 * pointer after a call returns. The library owns only the mesh handle and the
 * small device tables inside it (fe_mesh_destroy frees them). Buffers must be
 * 16-byte aligned.
 *
 * Streams: all device work is enqueued on `stream` (a hipStream_t, NULL for
 * the default stream). Calls that return host results (names ending in _h)
 * synchronise that stream before returning. A mesh is immutable after
 * creation, so calls on different streams with separate work buffers may run
 * concurrently.
 *
 * Precision: FE_F64 -> double blocks and FP64 arithmetic. FE_F32 -> float
 * blocks, FP32 arithmetic. FE_BF16 -> bfloat16 blocks (2 bytes per element:
 * the upper 16 bits of an IEEE binary32), widened to FP32 on load, FP32
 * arithmetic and accumulation, rounded to nearest (ties to even) on store;
 * taken by ks_apply, cheb_filter and ks_eigensolve on uniform and graded
 * meshes (the sum-factorised apply has no matrix-core shape, so it runs on
 * the vector ALU like FP32). Every other call returns FE_EINVAL for it.
 * Potentials, weights, densities, Gram matrices, eigenvalues and every
 * reduction are always FP64.
 *
 * Errors: a non-zero fe_status never aborts the process; fe_last_error()
 * returns a thread-local message describing the last failure of this thread.
 * On error, outputs are undefined except where stated for FE_ENOCONV,
 * FE_ENOTPD and FE_EGAP.
 */
#ifndef INVDFT_H
#define INVDFT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fe_mesh_s* fe_mesh;
typedef struct vxc_mesh_s* vxc_mesh;

typedef enum {
  FE_OK = 0,
  FE_EINVAL = 1,   /* invalid argument (sizes, null or misaligned pointers, unknown op) */
  FE_ENOMEM = 2,   /* device or host allocation failed */
  FE_EDEVICE = 3,  /* HIP runtime error (message in fe_last_error) */
  FE_ENOCONV = 4,  /* iteration limit reached; outputs hold the last iterate */
  FE_ENOTPD = 5,   /* Cholesky of an overlap matrix failed; block left unchanged */
  FE_EGAP = 6,     /* no gap at the Fermi level: eps[nocc] - eps[nocc-1] < 1e-6 Ha */
  FE_ESTATES = 7   /* too few states for the Fermi tail: the highest one passed is occupied */
} fe_status;

typedef enum { FE_F64 = 0, FE_F32 = 1, FE_BF16 = 2 } fe_prec;

/* Operation codes for fe_workspace_bytes. */
typedef enum {
  FE_OP_KS_APPLY = 0,
  FE_OP_CHEB_FILTER = 1,
  FE_OP_RAYLEIGH_RITZ = 2,
  FE_OP_ADJOINT_SOLVE = 3,
  FE_OP_LOSS_GRAD = 4,
  FE_OP_EIGENSOLVE = 5,
  FE_OP_ALONG_PSI = 6,
  FE_OP_POISSON = 7,
  FE_OP_ADJOINT_DEFLATED = 8
} fe_op;

/* ------------------------------------------------------------------ mesh --
 * Build the mesh tables (Eq. 12 Lagrange basis on GLL nodes; exact-Gauss
 * element stiffness and mass of Eq. 17; GLL-lumped W of Sec. 3.2.1) and
 * upload them to the current device.
 *   p in [1, 8] (order), n_cells_per_dim >= 1, half_width > 0 (bohr).
 * The kinetic bound (fe_mesh_info) is Fried's element bound,
 * lambda_max(K~/2) <= (1/2) lambda_max(W_e^{-1/2} K_e W_e^{-1/2}).
 * Errors: FE_EINVAL (bad p, n, L or out == NULL), FE_ENOMEM, FE_EDEVICE. */
fe_status fe_mesh_create(int p, int n_cells_per_dim, double half_width, fe_mesh* out);

/* A graded tensor mesh (cells of different widths, Fig. 6 and the mesh parameters
 * of Sec. 4): the same n cells on every axis, cell e spanning
 * [breaks_h[e], breaks_h[e+1]] (n + 1 strictly increasing host doubles). Every
 * cell is a product of 1-D cells, so the operator keeps its Kronecker form with
 * 1-D factors assembled from per-cell element matrices K_e = (2/h_e) K^,
 * M_e = (h_e/2) M^, W_e = (h_e/2) w^; the apply carries the per-cell factors.
 * The kinetic bound uses the smallest cell. Everything else is as fe_mesh_create.
 * Errors: FE_EINVAL (NULL pointers, p outside [1, 8], n < 1, boundaries not
 * strictly increasing), FE_ENOMEM, FE_EDEVICE. */
fe_status fe_mesh_create_graded(int p, int n_cells_per_dim, const double* breaks_h, fe_mesh* out);

/* Mapped mesh (per-cell element matrices: Sec. 3.2.3's batched dense cell products;
 * the curved, non-tensor cells of adaptive meshes, Sec. 4 and Fig. 6): the uniform
 * mesh's GLL nodes moved by the smooth map of the box onto itself
 *   Phi_d(xi) = xi_d + amp (L/pi) sin(pi xi_d / L) sin(pi xi_{d+1} / L), d+1 cyclic,
 * with isoparametric cells (a cell's shape is the order-p interpolant of its nodes).
 * Every cell gets its own dense element stiffness (Eq. 17) by Gauss quadrature with
 * ceil((3p+1)/2) points per axis (exact for linear fields: the patch test), the
 * overlap is GLL-lumped with |det J| at the nodes (Sec. 3.2.1), and the library
 * stores K~_e = (1/2) W^{-1/2} K_e W^{-1/2} per cell in FP64 and FP32 (at p = 5:
 * 14 x 54 x 64 doubles per cell, 387 KB). Same free-node numbering as the uniform
 * mesh. p in [1, 5], |amp| < 1; FE_EINVAL if the map inverts a cell. Every operator
 * call accepts the handle; poisson_solve, xc_initial_guess and vxc_mesh_create
 * return FE_EINVAL for it. Set-up runs on the device (the element matrices on the
 * FP64 matrix cores) and synchronises the device. */
fe_status fe_mesh_create_mapped(int p, int n_cells_per_dim, double half_width, double amp, fe_mesh* out);

/* Sizes and the kinetic spectral bound; any output pointer may be NULL. */
fe_status fe_mesh_info(fe_mesh mesh, int64_t* n_free_h, int64_t* n_cells_h,
                       int* nodes_per_cell_h, double* kin_bound_h);

/* Free-node coordinates xyz (N_f x 3, row-major, x fastest over nodes) and the
 * lumped weights w (N_f). Either pointer may be NULL. */
fe_status fe_mesh_nodes(fe_mesh mesh, double* xyz, double* w, void* stream);

/* Diagonal of the kinetic part K~/2 at the free nodes (N_f doubles): the
 * Jacobi preconditioner of the adjoint solve (Sec. 3.2.2). */
fe_status fe_mesh_kinetic_diag(fe_mesh mesh, double* d, void* stream);

fe_status fe_mesh_destroy(fe_mesh mesh);

/* Bytes of device work buffer an operation needs for a block of nv columns
 * (nv = nocc for FE_OP_ADJOINT_SOLVE and FE_OP_LOSS_GRAD, nv = n for
 * FE_OP_ALONG_PSI, nv = 1 for FE_OP_POISSON, nv = nocc + nbuf for
 * FE_OP_ADJOINT_DEFLATED, FP64 only). For FE_OP_CHEB_FILTER,
 * FE_OP_RAYLEIGH_RITZ and FE_OP_EIGENSOLVE the work blocks share the caller's
 * row pitch, so pass the block's leading dimension ld (>= its column count) as
 * nv. 0 on bad input. */
size_t fe_workspace_bytes(fe_mesh mesh, int op, int nv, fe_prec prec);

const char* fe_last_error(void);

/* ------------------------------------------------------------- ks_apply --
 * Y = H~ X - X diag(shift):  Y = (1/2) W^{-1/2} K W^{-1/2} X + v .* X - shift_j X_j
 * (Eqs. 17, 19; the matrix-free product of Sec. 3.2.3). The kinetic part is
 * computed cell by cell and assembled without atomics, so the result is
 * bitwise reproducible.
 *   v: N_f doubles (always FP64). shift_h: nv host doubles or NULL (no shift),
 *   at most 256 columns when given. X, Y: N_f x ld blocks of the precision's
 *   type; Y must not alias X.
 * prec: FE_F64, FE_F32, or FE_BF16 (uniform and graded meshes); FE_EINVAL
 * otherwise. */
fe_status ks_apply(fe_mesh mesh, const double* v, const double* shift_h, const void* X, void* Y,
                   int nv, int ld, fe_prec prec, void* stream);

/* ---------------------------------------------------------- cheb_filter --
 * X <- p_m(H~) X with the scaled degree-m Chebyshev filter of ChFSI
 * (Sec. 3.2.2; Zhou and Saad 2007): with c = (a+b)/2, e = (b-a)/2,
 *   p_m(lambda) = T_m((lambda - c)/e) / T_m((a0 - c)/e),
 * which damps [a, b] and keeps the columns O(1) near a0 < a.
 *   degree >= 1, a < b, a0 < a. work: fe_workspace_bytes(FE_OP_CHEB_FILTER, ld).
 * prec: FE_F64, FE_F32 or FE_BF16 (X's type follows prec; every step of the
 * recurrence is rounded to it; FE_EINVAL otherwise). */
fe_status cheb_filter(fe_mesh mesh, const double* v, int degree, double a, double b, double a0,
                      void* X, int nv, int ld, fe_prec prec, void* work, void* stream);

/* -------------------------------------------------------- rayleigh_ritz --
 * Rayleigh-Ritz on span(X) (Eqs. 23-24), FP64: S = X^T X = L L^T,
 * H_X = X^T H~ X, eigen-decomposition of L^{-1} H_X L^{-T} = V diag(eig) V^T,
 * X <- X L^{-T} V (orthonormal Ritz vectors, ascending Ritz values in eig_h),
 * resnorm_h[i] = || H~ x_i - eig_i x_i ||_2 (nullable). Any nv: above 64
 * columns the rotations go through a second N_f x ld block in work.
 * On FE_ENOTPD (S not positive definite) X is left unchanged.
 * work: fe_workspace_bytes(FE_OP_RAYLEIGH_RITZ, ld). Synchronises the stream. */
fe_status rayleigh_ritz(fe_mesh mesh, const double* v, double* X, double* eig_h, double* resnorm_h,
                        int nv, int ld, void* work, void* stream);

/* ------------------------------------------------------- ks_eigensolve --
 * Chebyshev-filtered subspace iteration (Sec. 3.2.2) for the nocc lowest
 * eigenpairs: repeat { cheb_filter(degree) ; rayleigh_ritz } on the nv-column
 * block X (nv > nocc; start from a random or warm block) until
 * max_{i < nocc} ||H~ x_i - eig_i x_i|| <= tol or maxpass passes. The filter
 * bounds are b = kinetic bound + max(v), a = largest Ritz value, a0 = smallest.
 * prec selects the filter precision (FE_F64 / FE_F32 / FE_BF16; FE_EINVAL
 * otherwise); with a reduced precision the passes switch to FP64 once the
 * residual is below `switch_tol` (or stops falling), so the final accuracy is
 * FP64's. FE_BF16 (uniform and graded meshes) starts a stage lower: bf16 passes
 * (the block rounded to nearest even) until the residual stops halving or is
 * below switch_tol, then FP32 passes as above, then FP64. Rayleigh-Ritz
 * is FP64. Locking: a pass filters only the columns from the first leading Ritz
 * pair whose residual is above tol (rounded down to a multiple of 8); the pairs
 * before it are left as they are (also in FP64 during a reduced-precision pass)
 * and still enter the Rayleigh-Ritz of the whole block. A reduced-precision pass
 * locks against max(tol, switch_tol) instead of tol.
 *   eig_h: nv host doubles (Ritz values); resnorm_h: nv host doubles.
 *   passes_h: number of passes done (nullable); stage_passes_h: 3 host ints
 *   (nullable), the passes done in bf16, FP32 and FP64.
 * Returns FE_ENOCONV if maxpass was reached (X, eig_h, resnorm_h valid).
 * work: fe_workspace_bytes(FE_OP_EIGENSOLVE, ld, prec). */
fe_status ks_eigensolve(fe_mesh mesh, const double* v, double* X, int nv, int ld, int nocc,
                        int degree, double tol, int maxpass, fe_prec prec, double switch_tol,
                        double* eig_h, double* resnorm_h, int* passes_h, int* stage_passes_h, void* work,
                        void* stream);

/* --------------------------------------------------------- adjoint_solve --
 * Solves, for all i < nocc together, (H~ - eps_i) q_i = b_i with Psi^T q_i = 0
 * (Eq. 20, Sec. 3.2.2) by preconditioned MINRES (Paige and Saunders 1975),
 * one Krylov space per column, all columns advanced in lockstep so that each
 * iteration makes one ks_apply with per-column shifts. The operator and the
 * preconditioner T = P diag(K~_aa/2)^{-1} P (P = I - Psi Psi^T, the inverse
 * kinetic diagonal) are both restricted to the complement of the occupied
 * orbitals. MINRES stops a column on its residual estimate in the
 * preconditioner's norm (relative to b, <= tol); in FP64 every column is then
 * held to the Euclidean bar ||b_i - (H~ - eps_i) q_i||_2 <= 2 tol ||b_i||_2:
 * columns above it are refined on their true residual (at most three rounds).
 *   Psi: N_f x nocc orthonormal occupied orbitals (ld = nocc), eps_h: nocc
 *   host doubles, B: right-hand sides (N_f x nocc, orthogonal to Psi), Q: out.
 *   iters_h (nocc ints) and relres_h (nocc doubles: true ||b - A q|| / ||b||,
 *   nullable) are filled on return.
 * prec: FE_F64, or FE_F32 = FP32 inner MINRES (relative tolerance
 * max(tol, 1e-4)) with FP64 iterative refinement (residuals and updates of Q in
 * FP64). nocc <= 256 in FP64, nocc <= 64 with FE_F32. Above 64 orbitals the
 * shifts are solved in groups of at most 64 columns, each against all of Psi
 * (the first 64 orbitals inside the fused MINRES sweeps, the others by separate
 * projection sweeps); iters_h and relres_h keep the column order. Columns that
 * have converged are dropped from the batch.
 * Psi, B, Q and work must be 16-byte aligned (FE_EINVAL otherwise).
 * maxit bounds the whole FP64 solve (first solve and refinement rounds
 * together, counted in iterations of the slowest column). Returns FE_ENOCONV
 * when some column misses the bar within maxit (Q, iters_h, relres_h filled).
 * work: fe_workspace_bytes(FE_OP_ADJOINT_SOLVE, nocc, prec). Synchronises. */
fe_status adjoint_solve(fe_mesh mesh, const double* v, const double* Psi, const double* eps_h,
                        int nocc, const double* B, double* Q, double tol, int maxit, int* iters_h,
                        double* relres_h, fe_prec prec, void* work, void* stream);

/* ------------------------------------------------ adjoint_solve_deflated --
 * The same solve as adjoint_solve in FP64 (same system, Eq. 20 of Sec. 3.2.2,
 * same solution up to tol), with a preconditioner that also inverts the shifted
 * operator on nbuf further approximate eigenvectors U whose Rayleigh quotients
 * theta lie above every shift:
 *   M_i = P_V D^{-1} P_V + U diag(1 / (theta_j - eps_i)) U^T,  P_V = I - V V^T,
 *   V = [Psi U], D = diag(K~_aa/2).
 * M_i is symmetric positive definite on the complement of Psi for any U, so the
 * solution does not depend on U; only the iteration count does. The columns
 * whose shift lies closest to the rest of the spectrum (smallest gap) gain
 * the most. The paper's solver uses the plain diagonal preconditioner; this is
 * an addition on the same path, not a change of the method.
 *   U: N_f x nbuf (ld = nbuf), orthonormal columns orthogonal to Psi, e.g. the
 *   Ritz vectors of the eigensolve above the occupied ones (a copy of U with
 *   Psi projected out is used, the caller's U is not modified);
 *   theta_h: nbuf host doubles, each strictly greater than every eps_h[i].
 * Other arguments as adjoint_solve. 1 <= nocc <= 64, 1 <= nbuf <= 64. When
 * nocc + nbuf > 64 the fused MINRES sweeps take the first 64 columns of V and
 * the remaining deflation vectors are applied by separate Gram and update
 * sweeps (the same preconditioner).
 * The result is held to the same Euclidean bar as adjoint_solve (FP64):
 * ||b_i - (H~ - eps_i) q_i||_2 <= 2 tol ||b_i||_2 for every column. Since the
 * preconditioner's norm weighs the U directions by 1 / (theta_j - eps_i), the
 * first solve stops at tol / 6 and columns still above the bar are refined.
 * FE_EINVAL on bad sizes, NULL or unaligned pointers, or theta not above every
 * shift; FE_ENOCONV when some column misses the bar within maxit iterations
 * (one budget for the first solve and the refinement rounds; Q, iters_h and
 * relres_h are filled all the same).
 * work: fe_workspace_bytes(FE_OP_ADJOINT_DEFLATED, nocc + nbuf, FE_F64).
 * Synchronises the stream. */
fe_status adjoint_solve_deflated(fe_mesh mesh, const double* v, const double* Psi,
                                 const double* eps_h, int nocc, const double* U,
                                 const double* theta_h, int nbuf, const double* B, double* Q,
                                 double tol, int maxit, int* iters_h, double* relres_h,
                                 void* work, void* stream);

/* ------------------------------------------------------------- loss_grad --
 * Phase 1 (Q == NULL): rho_a = sum_i f_i psi_{a,i}^2 / W_a (Eq. 4),
 *   loss = sum_a W_a (rho_data,a - rho_a)^2 (Eq. 1, w = 1), and the adjoint
 *   right-hand sides B = -(I - Psi Psi^T) R with r_i = 4 f_i (rho - rho_data) psi_i
 *   (Eqs. 7, 10, 20). Any of rho, B, loss_h may be NULL.
 * Phase 2 (Q != NULL): grad_b = sum_i psi_{b,i} q_{b,i} (Eqs. 11, 22), then
 *   grad_b = 0 where rho_data,b < tau_bc when tau_bc > 0 (Sec. 3.1.2).
 *   Psi: N_f x nocc (ld = nocc), 1 <= nocc <= 256; occ_h: nocc host doubles (f_i);
 *   loss_h also returns the loss in phase 2 when rho is given.
 * Synchronises the stream when loss_h != NULL. work: FE_OP_LOSS_GRAD bytes. */
fe_status loss_grad(fe_mesh mesh, const double* Psi, const double* occ_h, int nocc,
                    const double* rho_data, const double* Q, double tau_bc, double* rho, double* B,
                    double* grad, double* loss_h, void* work, void* stream);

/* --------------------------------------------------------- vxc_mesh ------
 * The exchange-correlation potential on its own linear finite-element mesh
 * (Eq. 14: first-order elements, uniform in an inner cuboid and coarsening
 * outwards, Sec. 4) and the transfer to the orbital mesh. The linear mesh is the
 * tensor product of three 1-D vertex lists t^x (mx + 1 strictly increasing
 * host doubles), t^y, t^z with trilinear hat functions N_b; the unknowns are the
 * (mx+1)(my+1)(mz+1) vertex values, b = ix + (mx+1)(iy + (my+1) iz). The lists
 * must cover every free node of the orbital mesh.
 * With the orbital mesh's GLL quadrature the potential enters H~ through its
 * nodal values v_a = sum_b N_b(x_a) u_b = (P u)_a, and the gradient with respect
 * to u is f = P^T g for the nodal gradient g of loss_grad (Eq. 22).
 * vxc_mesh_create copies the tables to the current device and allocates the
 * restriction's two intermediate arrays, n1^2 (mx+1) and n1 (my+1)(mx+1) doubles
 * with n1 the free nodes per axis (the mesh handle is not retained). Errors: FE_EINVAL (NULL pointers, fewer than one cell on an
 * axis, vertices not increasing, nodes not covered), FE_ENOMEM, FE_EDEVICE. */
fe_status vxc_mesh_create(fe_mesh mesh, int mx, const double* tx_h, int my, const double* ty_h, int mz,
                          const double* tz_h, vxc_mesh* out);
/* Number of linear-mesh unknowns and vertices per axis (3 ints); either may be NULL. */
fe_status vxc_mesh_info(vxc_mesh vm, int64_t* n_vertices_h, int* vertices_per_axis_h);
fe_status vxc_mesh_destroy(vxc_mesh vm);
/* v = base + P u over the N_f free nodes (base may be NULL: v = P u). u: the
 * vertex values; u must not alias v or base (base may alias v). Asynchronous. */
fe_status vxc_prolong(vxc_mesh vm, const double* u, const double* base, double* v, void* stream);
/* f = P^T g: g over the N_f free nodes, f over the vertices (f must not alias g).
 * Three 1-D passes, each summing a support in a fixed order (bitwise
 * reproducible). The passes use two intermediate arrays owned by the handle, so
 * calls on one handle must not overlap (one stream at a time). Asynchronous. */
fe_status vxc_restrict(vxc_mesh vm, const double* g, double* f, void* stream);

/* --------------------------------------------------------- poisson_solve --
 * The Hartree potential v_H = int rho(r') / |r - r'| dr' of a density (part of the
 * Hamiltonian of Sec. 2; its Fermi-Amaldi scaling enters Eq. 25), from
 * -lap phi = 4 pi rho on the orbital mesh with zero values on the box and the
 * GLL-lumped right-hand side: (K~/2) phi~ = 2 pi W^{1/2} rho', phi = W^{-1/2} phi~.
 * With sigma > 0 the monopole is split off: Q = sum_a W_a rho_a, c its centroid,
 * rho' = rho - Q g_sigma(r - c) (normalised Gaussian), and the Gaussian's potential
 * Q erf(|r - c| / (sqrt(2) sigma)) / |r - c| is added in closed form (rho' has no
 * charge and no dipole about c). sigma = 0 solves for rho itself.
 * Conjugate gradients with the kinetic diagonal as preconditioner, each product
 * one ks_apply of the same stiffness with a zero potential; stops when
 * ||b - A x|| <= tol ||b|| or after maxit products.
 *   rho, phi: N_f device doubles (phi written, also on FE_ENOCONV). iters_h,
 *   relres_h, charge_h (Q): host outputs, each nullable.
 * work: fe_workspace_bytes(FE_OP_POISSON, 1). Synchronises the stream.
 * Errors: FE_EINVAL (NULL pointers, tol <= 0, maxit < 1, sigma < 0), FE_ENOCONV. */
fe_status poisson_solve(fe_mesh mesh, const double* rho, double sigma, double* phi, double tol, int maxit,
                        int* iters_h, double* relres_h, double* charge_h, void* work, void* stream);

/* ------------------------------------------------------ xc_initial_guess --
 * Eq. 25: v = f v0 + (1 - f) alpha v_FA at the free nodes, f = rho / (rho + tau),
 * v_FA = -v_H / n_elec (Fermi-Amaldi), v0 = exchange + Perdew-Wang 1992
 * correlation of the unpolarised gas (v0 = 0 where rho <= 1e-30). Exchange
 * (the paper's two choices): FE_XC_SLATER, -(3 rho / pi)^{1/3}; FE_XC_LB94,
 * Slater - beta rho_s^{1/3} x^2 / (1 + 3 beta x asinh x), rho_s = rho / 2,
 * x = |grad rho_s| / rho_s^{4/3}, beta = 0.05, with the gradient of the order-p
 * interpolant of the nodal density (per axis the GLL Lagrange derivative in the
 * node's cell, the two one-sided values averaged at a shared vertex).
 *   rho, v_h, v: N_f device doubles. work: n_cells_per_dim doubles (LB94 only,
 *   else may be NULL). Asynchronous for Slater; synchronises the stream for LB94.
 * Errors: FE_EINVAL (NULL pointers, n_elec <= 0, tau <= 0, unknown exchange). */
typedef enum { FE_XC_SLATER = 0, FE_XC_LB94 = 1 } fe_xc_exchange;
fe_status xc_initial_guess(fe_mesh mesh, const double* rho, const double* v_h, double n_elec, double tau,
                           double alpha, int exchange, double* v, void* work, void* stream);

/* ----------------------------------------------------- fermi_occupations --
 * Finite-temperature occupations (Eq. 4's Fermi-Dirac occupancy, Eq. 5):
 *   f_i = smax / (1 + exp((eig_i - mu) / kT)), mu such that sum_i f_i = n_elec,
 * found by bisection to the last bit (sum_i f_i increases with mu). smax is the
 * occupancy of a full orbital: 2 for spin-restricted orbitals, 1 for the paper's
 * per-orbital form. Host-only: no device work, no stream.
 *   eig_h: n ascending host doubles (the lowest n eigenvalues of H~).
 *   occ_h: out, n host doubles f_i. dfde_h (nullable): out, d f_i / d eig_i.
 *   mu_h (nullable): out, mu. n_incl_h (nullable): out, the number of leading
 *   states with f_i > occ_cut * smax, extended over Ritz values closer than
 *   1e-6 Ha so that no degenerate group is split: the orbitals to pass on.
 * Errors: FE_EINVAL (kT <= 0, smax <= 0, occ_cut outside [0, 1), n < 1,
 * n_elec outside (0, smax n), eigenvalues not ascending); FE_ESTATES when the
 * highest state passed holds more than occ_cut * smax (all outputs are written:
 * compute more states). */
fe_status fermi_occupations(const double* eig_h, int n, double n_elec, double kT, double smax,
                            double occ_cut, double* occ_h, double* dfde_h, double* mu_h, int* n_incl_h);

/* ----------------------------------------------------- adjoint_along_psi --
 * The component of the adjoint functions along the included orbitals at
 * finite temperature (Eqs. 8, 9 and the in-span part of Eq. 7), added to the
 * MINRES solution Q of adjoint_solve (which is orthogonal to all n orbitals):
 *   M = Psi^T diag(2 (rho - rho_data)) Psi                 (n x n, FP64 MFMA)
 *   etabar = sum_i f'_i M_ii / sum_i f'_i                  (eta of Eq. 9 = -etabar)
 *   C_ii = f'_i (M_ii - etabar),  C_ij = M_ij (f_i - f_j) / (eps_i - eps_j)
 *   Q <- Q + Psi C
 * with f_i, f'_i = d f_i / d eps_i from (mu, kT, smax) as in fermi_occupations
 * (the divided difference is evaluated without cancellation and tends to f'_i
 * as eps_j -> eps_i, so degenerate groups need no special treatment). Then
 * loss_grad phase 2 with this Q gives the gradient of Eq. 10. Over each
 * degenerate group the diagonal block of C is Eq. 8's overlap; between groups
 * the coupling is split symmetrically, which changes the individual adjoint
 * functions but not the gradient.
 *   Psi: N_f x n (ld = n), n <= 256; eps_h: n host doubles; rho, rho_data: N_f;
 *   Q: N_f x n (ld = n), in/out. eta_h (nullable): out, eta of Eq. 9.
 *   C_h (nullable): out, n x n host doubles (row-major).
 * Psi, Q and work must be 16-byte aligned. work: fe_workspace_bytes(
 * FE_OP_ALONG_PSI, n). Synchronises the stream.
 * Errors: FE_EINVAL (NULL or misaligned pointers, n outside [1, 256], kT <= 0). */
fe_status adjoint_along_psi(fe_mesh mesh, const double* Psi, int n, const double* eps_h, double mu, double kT,
                            double smax, const double* rho, const double* rho_data, double* Q, double* eta_h,
                            double* C_h, void* work, void* stream);

/* ---------------------------------------------------- loss_grad_noalloc --
 * For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): loss_grad with no
 * work argument. Same arguments, phases, results and errors as loss_grad,
 * except:
 *   - phase 1 (Q == NULL) requires rho (the caller's N_f density output);
 *     loss_grad can keep the density in its work buffer, this call cannot;
 *   - the scratch (the loss partial sums and the Gram partials of the
 *     projection of B) is a fixed device array of this library,
 *     loss_grad_noalloc_max_bytes() bytes (34 MiB), one copy per GPU, held
 *     until the process ends. A call whose scratch would exceed it returns
 *     FE_EINVAL (cannot happen for nocc <= 256 on any mesh);
 *   - the current device must be the one the mesh was created on (FE_EINVAL).
 * It calls no hipMalloc, hipFree or allocating library routine. Every call on
 * one GPU uses that GPU's single array: calls that overlap in time on one GPU
 * (two host threads, or two streams without ordering) race and give wrong
 * results; calls ordered on one stream are safe. Nothing in the array needs
 * to start at zero: every partial sum is written before it is read. */
size_t loss_grad_noalloc_max_bytes(void);
fe_status loss_grad_noalloc(fe_mesh mesh, const double* Psi, const double* occ_h, int nocc,
                            const double* rho_data, const double* Q, double tau_bc, double* rho, double* B,
                            double* grad, double* loss_h, void* stream);

/* --------------------------------------------------------- block helpers --
 * Small FP64 vector kernels used by the host-side L-BFGS driver (Eq. 21):
 * fe_dot returns sum_a x_a y_a over n entries (deterministic reduction);
 * fe_axpby computes y <- alpha x + beta y (n = 0: nothing, x and y may be NULL).
 * work: at least 64 KiB. */
fe_status fe_dot(const double* x, const double* y, int64_t n, double* out_h, void* work, void* stream);
fe_status fe_axpby(double alpha, const double* x, double beta, double* y, int64_t n, void* stream);

/* ------------------------------------------------------- apply timing ----
 * Measurement aid for the operator apply and the MINRES row sweeps (not part
 * of the method): while enabled, every operator launch (ks_apply and the
 * applies inside cheb_filter, ks_eigensolve and adjoint_solve) and every
 * fused MINRES pass of adjoint_solve (Sec. 3.2.2) is bracketed by two HIP
 * events on the stream it is launched on, so that its duration is measured
 * without synchronising the caller.
 * fe_apply_timing(enable): 1 starts a new measurement (clears the record),
 *   0 stops recording (the record is kept). Host-side, process-wide; not
 *   thread-safe while launches are in flight.
 * fe_apply_timing_read(prec, launches, ms, bytes, columns): waits for the
 *   recorded events and returns, for launches in precision prec (FE_F64,
 *   FE_F32 or FE_BF16), their count, summed duration in milliseconds, summed
 *   algorithmic bytes (X read, Y written, Z read when the Chebyshev term is
 *   present, v read: (2 or 3) N_f nv s + 8 N_f per launch, s = 8, 4 or 2 bytes
 *   per element; on a mapped mesh also the
 *   per-cell matrices of that precision) and summed column counts nv. Any
 *   output may be NULL.
 * fe_sweep_timing_read(pass, launches, ms, bytes, columns): the same for the
 *   MINRES passes, pass 0 = A (Psi^T y and the two column dots), 1 = B (the new
 *   residual, the preconditioned u, Psi^T u), 2 = C (the projected direction,
 *   the w recurrence and the solution update); a pass's launch includes its
 *   small fixed-order reduction. Algorithmic bytes per launch, N rows, k active
 *   columns, k0 = nocc, s = 8 or 4: A N s (k0 + 3k), B N (s (k0 + 5k) + 8),
 *   C N s (k0 + 8k); one iteration is N s (3 k0 + 16 k) + 8 N. columns sums k.
 * Errors: FE_EINVAL for another prec or pass, FE_EDEVICE for a failed event
 * call. */
fe_status fe_apply_timing(int enable);
fe_status fe_apply_timing_read(fe_prec prec, int64_t* launches, double* ms, double* bytes, double* columns);
fe_status fe_sweep_timing_read(int pass, int64_t* launches, double* ms, double* bytes, double* columns);

#ifdef __cplusplus
}
#endif
#endif /* INVDFT_H */
