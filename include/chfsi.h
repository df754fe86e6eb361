/*
 * chfsi.h -- C ABI of the MI355X ChFSI library.
 *
 * Chebyshev-filtered subspace iteration on two-component complex spinor
 * blocks under the finite-element Kohn-Sham Hamiltonian with noncollinear
 * exchange field and spin-orbit nonlocal projectors (arXiv 2410.02754,
 * Sec. III.A-B and Sec. IV.B).  The library applies the symmetrically scaled
 * operator
 *
 *     H_hat^k = M_D^{-1/2} H^k M_D^{-1/2}                       (Sec. III.B.2)
 *
 * where H^k = H^{k,loc} + H^{k,nloc} is the FE matrix of eqn:FEHloc and
 * eqn:FEHnloc (projectors eqn:CMat, coefficients Delta_{2chi+a,2chi'+b} =
 * D^{chi chi'}_{ab}) and M_D is the diagonal GLL (lumped) overlap.  H_hat^k has
 * the spectrum of M_D^{-1} H^k; a block Y of H_hat^k corresponds to the FE
 * coefficients U = M_D^{-1/2} Y.
 *
 * Conventions shared by every call
 *  - Memory: pointers named *_d and all multivector arguments (X, Y, work,
 *    v0) are DEVICE pointers owned by the caller; *_h pointers are host
 *    memory owned by the caller.  The library never frees caller memory.  The
 *    context owns everything it builds (cell matrices, projector tables,
 *    internal scratch) and frees it in chfsi_destroy.
 *  - Multivector layout: row-major [2M][ld] complex numbers, interleaved
 *    (re, im).  Row r = 2 I + alpha is node I, spin alpha (eqn:GHEP); the n_vec
 *    columns of a row are contiguous.  n_vec >= 1 (an empty block is
 *    CHFSI_EINVAL) and ld >= n_vec; pointers 16-byte aligned.  complex128 everywhere
 *    (mixed precision converts internally).  A block of a wider array is
 *    passed as (pointer to its first column, n_vec, ld of the wide array).
 *  - Streams: all device work is enqueued on the HIP stream given to
 *    chfsi_create.  Calls that return host data (ritz_h, resid_h, bad_col,
 *    lo, hi) synchronise that stream before returning; the others are
 *    asynchronous with respect to the host.
 *  - Errors: every call returns CHFSI_OK (0) or a negative status; arguments
 *    are validated before any launch.  chfsi_last_error(ctx) returns a text
 *    description of the most recent failure.  No C++ exception crosses the
 *    ABI.  A context is not thread-safe.
 */
#ifndef CHFSI_H
#define CHFSI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct chfsi_ctx chfsi_ctx;

enum chfsi_status {
  CHFSI_OK = 0,
  CHFSI_EINVAL = -1,      /* invalid argument (null pointer, size, range)        */
  CHFSI_ENOMEM = -2,      /* device or host allocation failed                     */
  CHFSI_EHIP = -3,        /* a HIP runtime call or kernel launch failed           */
  CHFSI_ENOTPD = -4,      /* Gram matrix not positive definite (chol_gs)          */
  CHFSI_ENONHERM = -5,    /* a Delta override is not Hermitian                    */
  CHFSI_ENONFINITE = -6,  /* NaN/Inf in an input field or a reduced matrix        */
  CHFSI_ESTATE = -7       /* call out of order (e.g. apply before set_local)      */
};

enum chfsi_quad { CHFSI_QUAD_GL = 0, CHFSI_QUAD_GLL = 1 };
enum chfsi_prec { CHFSI_PREC_FP64 = 0, CHFSI_PREC_MIXED = 1 };

/* Mesh of an orthorhombic periodic box (Sec. III.A).
 *   n_cells[d] >= 2 hexahedral cells per direction, box[d] > 0 bohr,
 *   p in 1..8: degree of the GLL Lagrange basis (n_p = p+1 nodes per direction),
 *   quad: CHFSI_QUAD_GL = tensor Gauss-Legendre rule with n_q points per
 *         direction for all cell integrals (eqn:cellIntegrals), 1 <= n_q <= 12;
 *         CHFSI_QUAD_GLL = collocation at the GLL nodes (n_q ignored, = p+1),
 *   n_k >= 1 k-points kpts[n_k][3] (host, Cartesian, 1/bohr); k enters through
 *   the Bloch form of the operator (eqn:HnlocPeriodic and the k-terms of
 *   eqn:FEHloc). */
typedef struct {
  int n_cells[3];
  double box[3];
  int p;
  int quad;
  int n_q;
  int n_k;
  const double* kpts;
} chfsi_mesh_desc;

/* One pseudo-atom with Gaussian real-harmonic projectors (stand-in for the
 * ONCV projectors of eqn:nlOP):
 *   p_lm(r) = c_l r^l Y_lm(r_hat) exp(-r^2/(2 sigma^2)) for r < rcut, else 0,
 *   c_l^2 = 2/(Gamma(l+3/2) sigma^(2l+3)); real harmonics ordered
 *   l=0; l=1 (x,y,z); l=2 (xy, yz, 3z^2-r^2, xz, x^2-y^2); l = 0..lmax <= 2.
 *   Delta (index 2 chi + alpha) = D0_l within each shell + dso L.S, S = sigma/2.
 *   delta_override: NULL, or host [2 n_pj][2 n_pj] complex128 (interleaved,
 *   row-major) replacing Delta; must be Hermitian (else CHFSI_ENONHERM). */
typedef struct {
  double pos[3];
  int lmax;
  double sigma;
  double rcut;
  double d0[3];
  double dso;
  const double* delta_override;
} chfsi_atom_desc;

/* Build the mesh: numbering, cell colouring, reference-cell tables, lumped
 * mass (Sec. III.A; Sec. III.B.2).  hip_stream: a hipStream_t (NULL = default
 * stream).  On success *out owns the context. */
int chfsi_create(const chfsi_mesh_desc* desc, void* hip_stream, chfsi_ctx** out);

/* Free everything the context owns.  ctx may be NULL. */
int chfsi_destroy(chfsi_ctx* ctx);

/* Sizes: number of global nodes M, spinor dofs 2M, cells E, quadrature points
 * per cell, cell colours of the scatter-add assembly.  Any pointer may be NULL. */
int chfsi_sizes(const chfsi_ctx* ctx, int64_t* n_nodes, int64_t* n_dof, int* n_cells,
                int* nq3, int* n_colours);

/* Physical quadrature points, host [E][nq^3][3], cell e = cx + nx (cy + ny cz),
 * point q = qx + nq (qy + nq qz).  The fields of chfsi_set_local are sampled
 * at exactly these points. */
int chfsi_quad_points(const chfsi_ctx* ctx, double* xyz_h);

/* Local fields at the quadrature points (eqn:FEHloc, eqn:FEHlocEl): veff_d
 * [E][nq^3] and bxc_d [E][nq^3][3] (device, float64).  Cell-matrix form
 * (default): builds every cell operator for every k-point (FP64, plus the FP32
 * copy for mixed precision); matrix-free form: stores w_q J (V, B) per point.
 * CHFSI_ENONFINITE if a value is NaN/Inf. */
int chfsi_set_local(chfsi_ctx* ctx, const double* veff_d, const double* bxc_d);

enum chfsi_form { CHFSI_FORM_CELL_MATRIX = 0, CHFSI_FORM_MATRIX_FREE = 1 };

/* Form of the local (cell) part of H_hat used by every apply of this context.
 * CHFSI_FORM_CELL_MATRIX (default): the cell operators are formed and stored
 * and applied as batched dense products (Sec. IV.B), FP64 or FP32.
 * CHFSI_FORM_MATRIX_FREE: the tensor-structured product that the paper leaves
 * to future work (Sec. VI): per cell and column, values at the quadrature
 * points by sum factorisation, collocation derivatives there, the terms of
 * eqn:FEHlocEl applied pointwise, and the transposed contractions back to the
 * nodes.  Only w_q J (V, B) per quadrature point is stored (32 B per point
 * instead of about 4 (2 n_p^3)^2 x 8 B of matrices per cell).  Same quadrature,
 * so the result equals the cell-matrix product up to rounding.  Needs
 * n_q = p + 1 (GL with n_q = p + 1, or GLL).  CHFSI_PREC_MIXED runs the same
 * contractions in FP32 (tables, quadrature data and fields in FP32, rows
 * converted on gather and added into the FP64 output).  In a batch (below),
 * tasks of this form run their own per-colour launches.  The call clears the local operator (CHFSI_ESTATE until
 * the next chfsi_set_local builds it in the chosen form).  CHFSI_EINVAL for an
 * unknown form or unsupported mesh. */
int chfsi_set_apply_form(chfsi_ctx* ctx, int form);

/* Replace the set of pseudo-atoms (eqn:FEHnloc, eqn:CMat).  Builds the
 * Bloch-phased, image-summed and M_D^{-1/2}-scaled projector tables for every
 * k-point.  n_atoms may be 0. */
int chfsi_set_atoms(chfsi_ctx* ctx, int n_atoms, const chfsi_atom_desc* atoms);

/* Y = H_hat^k X for k-point ik (Sec. IV.B: extraction, cell products, nonlocal
 * projector terms, assembly).  X_d, Y_d: [2M][ldx], [2M][ldy] complex128,
 * distinct.  prec: CHFSI_PREC_FP64, or CHFSI_PREC_MIXED (cell products and
 * projector products in FP32 with FP32 accumulation, converted on load/store). */
int chfsi_apply_H(chfsi_ctx* ctx, int ik, const void* X_d, int64_t ldx, void* Y_d, int64_t ldy,
                  int n_vec, int prec);

/* Degree-m Chebyshev filter (eqn:chebfilt) damping [a, b] and amplifying the
 * spectrum below a, in the scaled three-term form: e=(b-a)/2, c=(b+a)/2,
 * sigma_1 = e/(a0-c), Y_1 = (sigma_1/e)(H - c)X, sigma_{k+1} = 1/(2/sigma_1 -
 * sigma_k), Y_{k+1} = (2 sigma_{k+1}/e)(H - c)Y_k - sigma_k sigma_{k+1} Y_{k-1}.
 * In place on X_d [2M][ldx]; work_d [2M][ldw] (ldw >= n_vec) is overwritten.
 * Requires a0 < a < b and degree >= 1 (else CHFSI_EINVAL).  prec_mode
 * CHFSI_PREC_MIXED runs applies 1..m-1 in FP32 and apply m in FP64; the
 * recurrence itself is always FP64. */
int chfsi_cheb_filter(chfsi_ctx* ctx, int ik, void* X_d, int64_t ldx, void* work_d, int64_t ldw,
                      int n_vec, int degree, double a, double b, double a0, int prec_mode);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * filter as chfsi_cheb_filter, with the same arguments and the same result
 * (each column's arithmetic is unchanged), but the nonlocal coefficient
 * scratch of every apply lives in a fixed device array of
 * CHFSI_NOALLOC_SCRATCH_BYTES bytes inside the library instead of the
 * context's growable buffer.  The call issues no hipMalloc/hipFree and no
 * allocating library routine; X_d and work_d are the caller's as before.
 * Every context on a device shares that device's one array (held until the
 * process ends; its address is looked up once per device in chfsi_create):
 * calls that overlap on one device race, and each call leaves the array's
 * last contents (nothing in it needs to start at zero).  When the coefficient
 * arrays and one column of contraction partials do not fit,
 *   n_chunks * 2 max_pj * 16 + 2 n_atoms * 2 max_pj * n_vec * 16 bytes
 *   > CHFSI_NOALLOC_SCRATCH_BYTES,
 * it returns CHFSI_EINVAL before any launch; otherwise the contraction runs
 * over as many columns per launch as fit.  Stage timers do not record this
 * call.  Errors as chfsi_cheb_filter. */
#define CHFSI_NOALLOC_SCRATCH_BYTES (64u << 20)
int chfsi_cheb_filter_noalloc(chfsi_ctx* ctx, int ik, void* X_d, int64_t ldx, void* work_d, int64_t ldw,
                              int n_vec, int degree, double a, double b, double a0, int prec_mode);

/* Ritz residuals in place: W_d[:, i] <- W_d[:, i] - theta_h[i] X_d[:, i] for
 * i < n_vec.  After chfsi_rayleigh_ritz with resid_h non-NULL, work_d holds
 * H_hat X for the rotated X, so this turns it into R = H_hat X - X diag(theta). */
int chfsi_ritz_residual(chfsi_ctx* ctx, const void* X_d, int64_t ldx, void* W_d, int64_t ldw, int n_vec,
                        const double* theta_h);

/* Residual form of the filter (Sec. III.B.2: the Hamiltonian-times-residual
 * reformulation that allows lower-precision products near convergence).  X_d
 * holds Ritz vectors with Ritz values theta_h (host) and residuals R_d
 * (= H_hat X - X diag(theta), from chfsi_ritz_residual).  With p_k the scaled
 * Chebyshev polynomials of chfsi_cheb_filter, Y_k = X p_k(Theta) + Z_k where
 *   Z_0 = 0, Z_1 = alpha_1 R,
 *   Z_{k+1} = alpha_{k+1} (H_hat - c) Z_k + beta_{k+1} Z_{k-1} + alpha_{k+1} R p_k(Theta),
 * so only the correction Z passes through operator products.  On return X_d
 * holds Y_m = p_m(H_hat) X (the same result as chfsi_cheb_filter).  prec_mode
 * CHFSI_PREC_MIXED runs every product H_hat Z_k in FP32 (Z is small when the
 * residuals are); the recurrence and the final combination are FP64.
 * work_d [2M][ldw] with ldw >= 2 n_vec (two Z blocks side by side). */
int chfsi_cheb_filter_resid(chfsi_ctx* ctx, int ik, void* X_d, int64_t ldx, const void* R_d, int64_t ldr,
                            const double* theta_h, void* work_d, int64_t ldw, int n_vec, int degree, double a,
                            double b, double a0, int prec_mode);

/* Cholesky-Gram-Schmidt: S = X^H X (FP64), S = L L^H, X <- X L^{-H}, so that
 * the columns become orthonormal with the same span (the orthonormalisation
 * before the Rayleigh-Ritz step, Sec. III.B.2).  The factorisation runs on the
 * unit-diagonal D S D, D = diag(S)^{-1/2} (same result in exact arithmetic).  On CHFSI_ENOTPD *bad_col (if
 * non-NULL) is the first column whose pivot is not positive and X is left
 * unchanged. */
int chfsi_chol_gs(chfsi_ctx* ctx, void* X_d, int64_t ldx, int n_vec, int* bad_col);

/* Rayleigh-Ritz on an orthonormal block (Sec. III.B.2): W = H_hat^k X,
 * H_p = X^H W, H_p = Q diag(theta) Q^H (ascending), X <- X Q.  ritz_h[n_vec]
 * receives theta; if resid_h is non-NULL it receives ||H_hat x_i - theta_i x_i||
 * and work_d holds H_hat X for the rotated X on return (the input of
 * chfsi_ritz_residual).  work_d [2M][ldw] (ldw >= n_vec) is overwritten.  FP64
 * throughout. */
int chfsi_rayleigh_ritz(chfsi_ctx* ctx, int ik, void* X_d, int64_t ldx, void* work_d, int64_t ldw,
                        int n_vec, double* ritz_h, double* resid_h);

/* Overlap S = X^H Y of two blocks [2M][ldx], [2M][ldy] of n_vec columns (FP64
 * MFMA Gram, fixed-order reduction): S_h host [n_vec][n_vec] complex128, row-major
 * (S_h[i][j] = x_i^H y_j).  Synchronises the stream.  For checks such as the
 * orthonormality ||X^H X - I|| after chfsi_chol_gs. */
int chfsi_overlap(chfsi_ctx* ctx, const void* X_d, int64_t ldx, const void* Y_d, int64_t ldy, int n_vec,
                  double* S_h);

/* Device memory the library itself holds for one call of the given kind on a
 * block of n_vec columns at k-point ik (its growable scratch, the rotation panel,
 * partial sums), excluding the caller's buffers (X, work, the backward
 * workspace): the peak of the call, in bytes; 0 for invalid arguments. */
enum chfsi_op { CHFSI_OP_APPLY = 0, CHFSI_OP_FILTER = 1, CHFSI_OP_CHOL_GS = 2, CHFSI_OP_RAYLEIGH_RITZ = 3,
                CHFSI_OP_DENSITY = 4 };
size_t chfsi_workspace_bytes(const chfsi_ctx* ctx, int ik, int n_vec, int op);

/* Spectral bounds by `steps` Lanczos steps on H_hat^k from v0_d [2M]
 * (complex128, device, not modified): *lo = smallest Ritz value of the
 * tridiagonal, *hi = largest Ritz value + ||f_steps|| (an upper bound of the
 * spectrum, Sec. III.B.2).  In the cell-matrix form (when n_q = p + 1) the
 * single-column applies run the matrix-free product of the same operator, which
 * does not stream the cell matrices for one column. */
int chfsi_lanczos_bounds(chfsi_ctx* ctx, int ik, int steps, const void* v0_d, double* lo,
                         double* hi);

/* ---- Adjoint (gradients of a real loss L through the operator and the filter).
 * Convention: for a complex block Z the gradient is Zbar = 2 dL/d conj(Z)
 * (the PyTorch convention), so that dL = Re <Zbar, dZ>, <a,b> = sum conj(a) b.
 * The operator depends linearly on the fields at the quadrature points
 * (eqn:FEHlocEl); for blocks L, Y its derivatives pair as
 *   Re <L, dH_hat/dV(e,q) Y>   = w_q J Re sum_n l_n(q)^H y_n(q),
 *   Re <L, dH_hat/dB_d(e,q) Y> = w_q J Re sum_n l_n(q)^H sigma_d y_n(q),
 * where z(q) = sum_i N_i(r_q) (M_D^{-1/2} Z)_i is the unscaled field at r_q.
 * For L = sum_n Re <x_n|H_hat|x_n> these are w_q J times the density and the
 * magnetisation of eqn:rho and eqn:mag. */

/* Adjoint of chfsi_apply_H (Y = H_hat X): Xbar_d [2M][ldxb] = H_hat Ybar; ADDS
 * dL/dV into dV_d [E][nq^3] and dL/dB_d into dB_d [E][nq^3][3] (device, float64;
 * the caller zeroes them).  FP64.  Requires n_q <= 10. */
int chfsi_apply_H_backward(chfsi_ctx* ctx, int ik, const void* X_d, int64_t ldx, const void* Ybar_d,
                           int64_t ldyb, void* Xbar_d, int64_t ldxb, int n_vec, double* dV_d,
                           double* dB_d);

/* Workspace bytes needed by chfsi_cheb_filter_backward for these sizes. */
size_t chfsi_filter_backward_workspace(const chfsi_ctx* ctx, int n_vec, int degree, int ckpt_every);

/* Adjoint of chfsi_cheb_filter (same degree and bounds, FP64): with the forward
 * states Y_0 = X, ..., Y_m and Ybar = 2 dL/d conj(Y_m), runs the reverse
 * recurrence Lam_m = Ybar, Lam_{k-1} = alpha_k (H_hat - c) Lam_k + beta_{k+1} Lam_{k+1}
 * (the same operator chain: H_hat is Hermitian and the coefficients real), sets
 * Xbar_d = Lam_0 and ADDS sum_k alpha_k (dV, dB)(Lam_k, Y_{k-1}) into dV_d, dB_d.
 * Forward states are recomputed segment by segment from checkpoint pairs
 * (Y_{jc}, Y_{jc+1}), c = ckpt_every >= 1, kept in work_d (device, caller-owned,
 * at least chfsi_filter_backward_workspace bytes).  X_d is not modified. */
int chfsi_cheb_filter_backward(chfsi_ctx* ctx, int ik, const void* X_d, int64_t ldx, const void* Ybar_d,
                               int64_t ldyb, void* Xbar_d, int64_t ldxb, int n_vec, int degree, double a,
                               double b, double a0, int ckpt_every, void* work_d, size_t work_bytes,
                               double* dV_d, double* dB_d);

/* ---- Densities from the Rayleigh-Ritz output (eqn:rho, eqn:mag), with
 * Fermi-Dirac occupations at the smearing temperature of Sec. V and the entropy
 * term of the free energy in Sec. II.B. */

/* Fermi-Dirac occupations of n levels (host, float64): occ_h[i] =
 * 1 / (1 + exp((eps_h[i] - mu) / kT)) with mu chosen by bisection so that
 * sum_i w_h[i] occ_h[i] = n_electrons (w_h NULL: all weights 1; a weight is the
 * k-point weight of the level's k-point).  Writes mu to *mu_h and
 * E_ent = kT sum_i w_i [f_i ln f_i + (1 - f_i) ln(1 - f_i)] to *e_ent_h (each may
 * be NULL).  kT in Ha (500 K = 1.5834e-3 Ha).  CHFSI_EINVAL unless kT > 0,
 * every w_i >= 0, every eps finite and 0 < n_electrons < sum_i w_i.  Needs no
 * context and no GPU; its errors are read with chfsi_last_error(NULL). */
int chfsi_fermi_dirac(int n, const double* eps_h, const double* w_h, double n_electrons, double kT,
                      double* occ_h, double* mu_h, double* e_ent_h);

/* ADDS the occupation-weighted density and magnetisation of one block into
 * rho_d [E][nq^3] and mag_d [E][nq^3][3] (device, float64, cell-major as the
 * fields of chfsi_set_local; the caller zeroes them before the first block):
 *   rho(e,q)   += sum_n occ_h[n] u_n(q)^H u_n(q),
 *   mag_d(e,q) += sum_n occ_h[n] u_n(q)^H sigma_d u_n(q),
 * where u_n(q) = sum_i N_i(r_q) (M_D^{-1/2} x_n)_i is the spinor field of column n
 * of X_d [2M][ldx] at the quadrature point.  With psi = exp(ik.r) u the densities
 * depend on u only, so a k-point grid calls this once per k-point with
 * occ_h[n] = w_k f_nk (host, n_vec values, read before the call returns).  FP64;
 * needs the mesh only (not chfsi_set_local).  Requires n_q <= 10.  The sums over
 * n run in a fixed order: repeated calls give identical results. */
int chfsi_density(chfsi_ctx* ctx, const void* X_d, int64_t ldx, int n_vec, const double* occ_h,
                  double* rho_d, double* mag_d);

/* ---- Self-consistent field loop (Sec. III.B, eqn:fixedpointmap; Sec. IV.A).
 * Fields are at the cell quadrature points: scalar fields [E][nq^3] and vector
 * fields [E][nq^3][3] float64 device arrays in the order of chfsi_quad_points.
 * The paper's map needs electrostatics and an exchange-correlation functional;
 * these calls provide stand-ins of the same structure, solved in the FE space
 * of the context (K_s = int grad N_I . grad N_J, M_c = int N_I N_J with the
 * cell quadrature; Jacobi-preconditioned conjugate gradients to relative
 * residual tol, at most max_iter steps; *iters (if non-NULL) receives the step
 * count, negative when tol was not reached).  All synchronise the stream. */

/* eqn:innerPdt: *out = (1/2)(int r1 r2 + int m1 . m2) (cell quadrature); m1_d,
 * m2_d both NULL drops the magnetisation part. */
int chfsi_field_inner(chfsi_ctx* ctx, const double* r1_d, const double* m1_d, const double* r2_d,
                      const double* m2_d, double* out);

/* Hartree potential with a uniform compensating background (standing in for
 * the smeared nuclear charges of eqn:poissonEl): -lap V_H = 4 pi (rho - rho_bar)
 * on the periodic box, V_H of zero mean under the lumped mass M_D, written at
 * the quadrature points to vh_d (may alias rho_d). */
int chfsi_hartree(chfsi_ctx* ctx, const double* rho_d, double* vh_d, double tol, int max_iter, int* iters);

/* Kerker preconditioner of a charge residual: out = f - k0^2 w with
 * (k0^2 - lap) w = f (Fourier factor G^2/(G^2 + k0^2)); k0 = 0 copies f. */
int chfsi_kerker(chfsi_ctx* ctx, double k0, const double* f_d, double* out_d, double tol, int max_iter,
                 int* iters);

/* LSDA (Dirac) exchange under the locally collinear substitution of Sec. II.B,
 * rho_up,dn = (rho +- |m|)/2 (clamped at 0), v_s = -(6/pi)^(1/3) rho_s^(1/3):
 * vx_d = (v_up + v_dn)/2, bx_d = (v_up - v_dn)/2 m/|m| (0 where m = 0). */
int chfsi_exchange(chfsi_ctx* ctx, const double* rho_d, const double* m_d, double* vx_d, double* bx_d);

/* Two-grid transfer (Sec. IV.A, eqn:FEWfnsCMesh): the degree-(p-1) spinor fields
 * of the scaled block Yc_d [2M_c][ldc] on the coarse context, evaluated at the
 * degree-p nodes of the same cells and written, M_D-scaled, to Yf_d [2M_f][ldf]
 * of the fine context (fine p = coarse p + 1, same cells and box, same stream). */
int chfsi_interpolate_block(chfsi_ctx* coarse, chfsi_ctx* fine, const void* Yc_d, int64_t ldc, void* Yf_d,
                            int64_t ldf, int n_vec);

typedef struct {
  int n_vec;            /* block width N (all states, one electron each at most)     */
  int degree;           /* Chebyshev degree                                          */
  int passes_first;     /* ChFSI passes in the first SCF iteration of the first grid */
  int passes;           /* ChFSI passes in every other iteration                     */
  int depth;            /* Anderson history length, 1..16 (1 = linear mixing)        */
  int max_iter;         /* SCF iterations in total                                   */
  int max_coarse;       /* iterations on the coarse grid at most                     */
  int lanczos_steps;    /* Lanczos steps for the upper bound, every iteration        */
  int field_max_iter;   /* conjugate-gradient steps per field solve at most          */
  int prec_mode;        /* CHFSI_PREC_FP64, or CHFSI_PREC_MIXED: the residual form of
                           the filter (chfsi_cheb_filter_resid, FP32 products on the
                           residuals; R formed in FP64 at the start of every iteration
                           and after every Rayleigh-Ritz), which converges as far as
                           FP64 where FP32 products on the whole block stall        */
  double n_electrons;   /* 0 < N_e < n_vec                                           */
  double kT;            /* Fermi-Dirac smearing, Ha                                  */
  double alpha;         /* mixing parameter                                          */
  double k0;            /* Kerker wave number, 1/bohr (0: no preconditioning)        */
  double tol;           /* stop when the residual norm < tol on the fine grid        */
  double tol_coarse;    /* leave the coarse grid when the residual norm < tol_coarse */
  double field_tol;     /* relative residual of the field solves                     */
  uint64_t seed;        /* start block: SplitMix64 stream of chfsi_fill_random       */
  uint64_t lanczos_seed;/* Lanczos start vector stream                               */
  const double* bounds_h;/* host [n_bounds]: the filter's upper bound b of iteration i
                          at k-point ik in entry i n_k + ik (a known bound of the
                          spectrum; the Lanczos run is skipped), or NULL: b from
                          lanczos_steps Lanczos steps every iteration            */
  int n_bounds;         /* entries of bounds_h (iterations past them use Lanczos)    */
  const double* kweights_h;/* host [n_k]: zone-average weights of the context's k-points
                          (>= 0, summing to 1), or NULL: equal weights           */
  int start_given;      /* 1: X_d holds the start blocks (a restart; no coarse grid),
                          0: the seeded start blocks                             */
} chfsi_scf_params;

typedef struct {
  int p;                /* degree of the grid of this iteration                      */
  double resid;         /* || F(x) - x || in the norm of eqn:innerPdt                */
  double mu;            /* chemical potential, Ha                                    */
  double band_energy;   /* sum_k w_k sum_n f_nk theta_nk, Ha                         */
  double theta0;        /* lowest Ritz value over the k-points, Ha                   */
  int hartree_iters;    /* conjugate-gradient steps of this iteration's Hartree solve */
  double b;             /* the filter's upper bound in this iteration (k-point 0), Ha */
} chfsi_scf_record;

/* The SCF loop.  Each iteration: V_eff = vext + V_H[rho] + V_x, B_xc = bext + B_x
 * (chfsi_hartree, chfsi_exchange) set on the grid's context; a Lanczos bound;
 * on the first iteration of a grid a CholGS + Rayleigh-Ritz prologue; ChFSI
 * passes (filter with a = max theta, a0 = min theta of the previous RR);
 * Fermi-Dirac occupations; output densities (chfsi_density) scaled to hold
 * exactly N_e electrons; residual f = F(x) - x; Anderson mixing: b_j with
 * sum b_j = 1 minimise || sum b_j f_j || over the last `depth` iterations, and
 * the next input is sum b_j x_j + alpha (K f_rho, f_m), K = chfsi_kerker.
 * With coarse non-NULL (degree p-1, same cells, quadrature and stream) the loop
 * starts there, leaves it when the residual is below tol_coarse (or after
 * max_coarse iterations), moves the block with chfsi_interpolate_block and
 * clears the Anderson history; the densities carry over.  Both contexts need
 * their atoms set.
 * Brillouin-zone sampling (Sec. II.C): every k-point of the fine context (the
 * coarse one must have the same k-points) carries its own block, Lanczos bound
 * and ChFSI passes (start: the seeded block, or the caller's block in X_d with
 * start_given, which the first iteration orthonormalises before its
 * Rayleigh-Ritz); the occupations f_nk have one Fermi level for all (n, k)
 * with sum_k w_k sum_n f_nk = N_e (chfsi_fermi_dirac with weights w_k), and the
 * output densities are sum_k w_k sum_n f_nk |u_nk|^2 (likewise m).  The start
 * block of k-point ik is the chfsi_fill_random stream of seed + 7919 ik.
 * The host eigensolve of each k-point's last Rayleigh-Ritz runs on a helper
 * thread while the next k-point's work is issued (the results are those of
 * the plain order); the call returns after that thread has finished.
 * In/out: rho_d, m_d hold the initial input densities and, on return, the last
 * input; rho_out_d, m_out_d the last output; X_d (fine grid) the last Ritz
 * blocks, block ik [2M][ldx] at X_d + ik 2M ldx complex entries; theta_h and
 * occ_h [n_k][n_vec] (host, may be NULL) their Ritz values and occupations;
 * hist_h[max_hist] one record per iteration, *n_hist the count; *converged 1 if
 * the fine-grid residual fell below tol within max_iter. */
int chfsi_scf_run(chfsi_ctx* fine, chfsi_ctx* coarse, const chfsi_scf_params* params, const double* vext_d,
                  const double* bext_d, double* rho_d, double* m_d, double* rho_out_d, double* m_out_d, void* X_d,
                  int64_t ldx, double* theta_h, double* occ_h, chfsi_scf_record* hist_h, int max_hist, int* n_hist,
                  int* converged);

/* ---- Batched filtering of independent operators (the k-points of a grid and
 * independent systems: the eigenproblems of different k are independent,
 * Sec. III.B).  One task = one (context, k-point, block): X_d [2M][ldx] is
 * filtered in place with work_d [2M][ldw].  Per recurrence step the projector
 * terms run per task and the cell products of all tasks run as one persistent
 * launch per colour phase (per tile width and k-term variant).  Tasks may share
 * a context (k-points of one mesh) but not X or work buffers. */
typedef struct chfsi_batch chfsi_batch;
typedef struct {
  chfsi_ctx* ctx;
  int ik;
  void* X_d;
  int64_t ldx;
  void* work_d;
  int64_t ldw;
  int n_vec;
} chfsi_batch_task;
enum chfsi_batch_flags {
  CHFSI_BATCH_AUTOTUNE = 1,  /* time column tile widths 128/64/32 per task at create and keep the
                                fastest (a narrower width must win by more than 1 %); without it the
                                widest width <= n_vec is used */
  CHFSI_BATCH_GRAPH = 2      /* capture the whole filter into a hipGraph on the first chfsi_batch_filter
                                and replay that graph on every later call, whatever the bounds (needs a
                                non-default stream) */
};

/* Build a batch of n_tasks tasks for a degree-m filter in precision prec_mode.
 * All contexts must share one stream and have their fields set.  Buffers are
 * bound at creation.  With CHFSI_BATCH_AUTOTUNE the work buffers are used as
 * scratch during creation.  The batch owns the device memory its kernels use
 * besides the task buffers (projector partial sums, recurrence coefficient
 * tables), so other calls on the same contexts (chfsi_chol_gs,
 * chfsi_rayleigh_ritz, ...) may run between filters. */
int chfsi_batch_create(int n_tasks, const chfsi_batch_task* tasks, int degree, int prec_mode, int flags,
                       chfsi_batch** out);

/* Filter every task's block with its own bounds a[t], b[t], a0[t] (host arrays,
 * a0 < a < b): the same scaled recurrence as chfsi_cheb_filter, bitwise equal to
 * filtering the tasks one by one.  The recurrence coefficients of all tasks are
 * copied into a device table before the filter's kernels (which read them from
 * there), so a captured graph is replayed with new bounds without capturing
 * again.  Asynchronous.  CHFSI_ESTATE if a task's context has been rebuilt
 * (chfsi_set_local, chfsi_set_atoms, chfsi_set_apply_form) since
 * chfsi_batch_create: the batch holds that context's device pointers. */
int chfsi_batch_filter(chfsi_batch* batch, const double* a, const double* b, const double* a0);

/* Graph statistics of a CHFSI_BATCH_GRAPH batch: number of captures and of
 * replays, and the accumulated host milliseconds of stream capture and of
 * graph instantiation.  Any pointer may be NULL. */
int chfsi_batch_graph_info(const chfsi_batch* batch, int* n_captures, int* n_replays, double* capture_ms,
                           double* instantiate_ms);

/* Chosen column tile width per task (cols_out[n_tasks]; 0 for a task whose
 * context uses the matrix-free form, which runs its own per-colour launches) and,
 * if tune_ms is not NULL, the timed cell-stage milliseconds for widths 32, 64,
 * 128 (-1 = not run). */
int chfsi_batch_tiles(const chfsi_batch* batch, int* cols_out, double* tune_ms);

/* Free the batch (not the contexts or buffers).  batch may be NULL. */
int chfsi_batch_destroy(chfsi_batch* batch);

/* Text of the batch's most recent error. */
const char* chfsi_batch_last_error(const chfsi_batch* batch);

/* Fill rows [row0, row0+n_rows) x columns [col0, col0+n_vec) of a seeded
 * [..][n_total_cols] multivector into X_d [n_rows][ld]:
 * X[r][n] = u(2j) + i u(2j+1), j = r * n_total_cols + n, u(i) = 2 w - 1 with w
 * the top 53 bits of the i-th SplitMix64 output for `seed` (Steele et al. 2014). */
int chfsi_fill_random(chfsi_ctx* ctx, void* X_d, int64_t n_rows, int n_vec, int64_t ld,
                      uint64_t seed, int64_t row0, int col0, int64_t n_total_cols);

/* Per-stage timing (HIP events recorded on the context's stream around each
 * launch of a stage; off by default).  Stages: */
enum chfsi_stage {
  CHFSI_STAGE_CELL_FP64 = 0,  /* gather + FP64 cell products + scatter-add, one launch per colour */
  CHFSI_STAGE_CELL_FP32 = 1,  /* the same in FP32 (mixed precision)                              */
  CHFSI_STAGE_NONLOCAL = 2,   /* projector contraction, coupling and back-product                 */
  CHFSI_STAGE_AXPY = 3,       /* recurrence initialisation / element-wise passes                  */
  CHFSI_STAGE_GRAM = 4,       /* X^H Y overlap and projected-Hamiltonian products                 */
  CHFSI_STAGE_ROTATE = 5,     /* in-place subspace rotations X <- X Q                             */
  CHFSI_STAGE_HOST_DENSE = 6, /* host Cholesky / inverse / Hermitian eigensolver (wall time)      */
  CHFSI_N_STAGES = 7
};
/* Accumulated totals of one stage since the last reset.  flops: algorithmic
 * count (a complex multiply-add = 8 real flops; for the cell products
 * 8 (2 n_p^3)^2 N per cell); exec_flops: MFMA flops actually issued (padded
 * tiles, Pauli form); bytes: algorithmic HBM bytes (operator entries read
 * once, vector rows gathered / read-added-written once). */
typedef struct {
  int64_t launches;
  double ms;
  double flops;
  double exec_flops;
  double bytes;
} chfsi_stage_stats;

/* Enable (1) or disable (0) stage timing. */
int chfsi_stats_enable(chfsi_ctx* ctx, int enable);

/* Synchronise the stream and write the totals of all CHFSI_N_STAGES stages
 * into out[CHFSI_N_STAGES] (host). */
int chfsi_stats_read(chfsi_ctx* ctx, chfsi_stage_stats* out);

/* Zero the totals. */
int chfsi_stats_reset(chfsi_ctx* ctx);

/* Block until all work enqueued by the context has finished. */
int chfsi_sync(chfsi_ctx* ctx);

/* Text of the most recent error on ctx (or of the last failed create when ctx
 * is NULL).  Valid until the next call on the same context. */
const char* chfsi_last_error(const chfsi_ctx* ctx);

/* Library version string. */
const char* chfsi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* CHFSI_H */
