/*
 * cclr.h — C ABI of the MI355X CCSD linear-response library (libcclr.so).
 *
 * The method is relativistic (complex, spin-orbital) coupled-cluster linear
 * response of arXiv:2307.14296.  The library applies the CCSD Jacobian
 * A = <mu-bar|[H0, tau_nu]|CC> (Table 1) from the right and from the left,
 * shifted by a complex frequency z = omega + i*gamma, solves the damped
 * response equations (A - z) t = -xi (eq. "LR response equation_cpp") and the
 * Lambda equation lambda A = -eta (theory section, eq. "Lambda") with a
 * Davidson-type subspace solver (SI, "Davidson scheme"), and assembles the
 * symmetric CC-CC response function <<X;Y>> (eq. "CC-CC response function").
 * The contractions follow the SI working equations for the sigma vectors,
 * the Hbar intermediates, xi^X, eta^X and the Hessian product t^X F.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - o occupied and v virtual spin orbitals, n = o + v, occupied first.
 * - Complex numbers are interleaved double pairs (cclr_c64), identical in
 *   layout to C99 double _Complex and numpy/torch complex128.
 * - Tensors are row-major and C-contiguous:
 *     f[p][q]              n x n Fock matrix, f[p][q] = <p|f|q>
 *     blocks of <pq||rs>   oooo[o][o][o][o], ooov[o][o][o][v], oovv[o][o][v][v],
 *                          ovov[o][v][o][v], ovvv[o][v][v][v], vvvv[v][v][v][v]
 *                          (all other blocks follow from antisymmetry and
 *                          <pq||rs> = conj(<rs||pq>))
 *     t1[i][a] = t^a_i, t2[i][j][a][b] = t^ab_ij (antisymmetric in ij and ab)
 *     right vectors r1[i][a], r2[i][j][a][b]; left vectors l1[i][a] = l^i_a,
 *     l2[i][j][a][b] = l^ij_ab; perturbations X[p][q] = <p|X|q> (n x n).
 *   Only the unique doubles (i > j, a > b) of an input vector are read; the
 *   doubles of an output vector are written in full antisymmetric form.
 *   With nvec > 1 the vectors are stacked along a leading dimension.
 * - Tensor arguments are DEVICE pointers (HIP device memory, e.g. the
 *   data_ptr() of a torch tensor on the GPU).  Scalars and arrays of
 *   frequencies, and the response-function output, are HOST pointers.
 * - Work is enqueued on options.hip_stream (NULL = the null stream); every
 *   call returns after that stream has completed the call's work.
 * - The caller owns every buffer it passes; the context keeps its own device
 *   copies of f, the integral blocks, t, lambda and the intermediates and
 *   retains no caller pointer after a call returns.  A context is used by one
 *   host thread at a time; distinct contexts are independent.
 * - Return codes: CCLR_OK (0); CCLR_ENOTCONV (> 0: result written, solver
 *   did not reach the tolerance, see cclr_solve_info); negative codes are
 *   errors, with cclr_last_error() describing them.  Inputs containing
 *   NaN/Inf are rejected with CCLR_EINVAL.
 */
#ifndef CCLR_H
#define CCLR_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { double re, im; } cclr_c64;
typedef struct cclr_ctx cclr_ctx;

enum {
  CCLR_OK = 0,
  CCLR_ENOTCONV = 1,
  CCLR_EINVAL = -1,
  CCLR_ENOMEM = -2,
  CCLR_EHIP = -3,
  CCLR_ESTATE = -4
};

/* arithmetic of the bulk contractions (solver, residuals and dot products
 * are always FP64): FP64; FP32 MFMA; split-BF16 MFMA with FP32 accumulation,
 * both operands split hi + lo and three bf16 products per real product
 * (BF16X3), or the trial-vector operand split and the Jacobian's operator
 * rounded to bf16, two bf16 products per real product (BF16X2).  The reduced
 * precisions run inside an FP64 iterative refinement, so the results meet
 * the same tolerance. */
enum { CCLR_FP64 = 0, CCLR_FP32 = 1, CCLR_BF16X3 = 2, CCLR_BF16X2 = 3 };

enum { CCLR_RIGHT = 0, CCLR_LEFT = 1 };

typedef struct {
  int prec;              /* CCLR_FP64 (default)                               */
  double tol;            /* solver stop: ||R|| <= tol * ||rhs|| (1e-10)       */
  int maxiter;           /* sigma applications per right-hand side (500)      */
  int max_subspace;      /* subspace size before a restart (48)               */
  size_t device_mem_cap; /* bytes the context may allocate, 0 = unlimited     */
  void* hip_stream;      /* hipStream_t; NULL = null stream                   */
} cclr_options;

typedef struct {
  int iters;        /* Davidson iterations (max over right-hand sides)        */
  int converged;    /* 1 if every right-hand side met the tolerance           */
  double resnorm;   /* max relative residual norm ||R||/||rhs|| at exit       */
  double time_ms;   /* wall time of the call                                  */
  long nsigma;      /* number of single-vector Jacobian transforms applied    */
  double kappa;     /* conditioning estimate of the damped solves: the largest
                       over right-hand sides of max|theta|/min|theta|, theta
                       the Ritz values of (A - z) on the final subspace (the
                       eigenvalues of the projected matrix G'); 0 if none    */
  double ritz_min;  /* the smallest such |theta|: an estimate of the distance
                       from z to the spectrum of A (0 if none)               */
} cclr_solve_info;

/* Fill *opt with the defaults listed above. */
int cclr_default_options(cclr_options* opt);

/* New context for o >= 2 occupied and v >= 2 virtual spin orbitals.
 * opt may be NULL (defaults).  On success *out owns device resources until
 * cclr_destroy. */
int cclr_create(int o, int v, const cclr_options* opt, cclr_ctx** out);
int cclr_destroy(cclr_ctx* ctx);

/* Copy f and the six canonical blocks of <pq||rs> (device pointers, layouts
 * above) into the context.  Invalidates amplitudes, intermediates and lambda. */
int cclr_set_hamiltonian(cclr_ctx* ctx, const cclr_c64* f,
                         const cclr_c64* oooo, const cclr_c64* ooov, const cclr_c64* oovv,
                         const cclr_c64* ovov, const cclr_c64* ovvv, const cclr_c64* vvvv);

/* Form the six canonical <pq||rs> blocks from Cholesky vectors of the
 * Coulomb integrals, as the paper does for every integral class
 * (computational details), and copy f.  L: DEVICE array nchol x n x n,
 * L[P][p][q] Hermitian in (p, q) for each P, with the Mulliken integrals
 * (pq|rs) = sum_P L[P][p][q] L[P][r][s], so
 *   <pq||rs> = sum_P ( L[P][p][r] L[P][q][s] - L[P][p][s] L[P][q][r] ).
 * The blocks are built on the device (products over P) and kept in the
 * layouts of cclr_set_hamiltonian; L is not retained.  Invalidates
 * amplitudes, intermediates and lambda.  CCLR_EINVAL for nchol < 1 or
 * non-finite input. */
int cclr_set_hamiltonian_cholesky(cclr_ctx* ctx, const cclr_c64* f, int nchol, const cclr_c64* L);

/* The CCSD residual Omega_mu = <mu| e^-T H_N e^T |R> for amplitudes t1
 * [o][v], t2 [o][o][v][v] (antisymmetric; DEVICE), written to o1, o2 in the
 * same layouts (DEVICE), and the correlation energy
 * f_ia t^a_i + 1/4 <ij||ab> tau^ab_ij to *energy (HOST, may be NULL).  The
 * ground-state equations that the implementation section solves first (not
 * printed in the paper; spin-orbital CCSD in the intermediate form of
 * Stanton and Gauss, J. Chem. Phys. 94, 4334 (1991)).  Needs
 * cclr_set_hamiltonian; does not change the context's amplitudes. */
int cclr_ccsd_residual(cclr_ctx* ctx, const cclr_c64* t1, const cclr_c64* t2, cclr_c64* o1, cclr_c64* o2,
                       cclr_c64* energy);

/* Solve Omega(t) = 0 by CROP (conjugate residual with optimal trial
 * vectors; Ziolkowski et al., J. Chem. Phys. 128, 204105 (2008)), the
 * ground-state solver the implementation section names.  t1, t2 (DEVICE,
 * layouts of cclr_ccsd_residual) hold the start on entry and the solution
 * on return; each iteration takes a Jacobi step with the Fock diagonal from
 * the current optimal vector, evaluates the residual there, and combines
 * the last nsub - 1 optimal vectors and the new one with weights summing to
 * one that minimize the norm of the combined residual (nsub in [2, 8];
 * 3 is the usual CROP).  Converged when the residual's 2-norm over unique
 * amplitudes is <= tol.  The solution becomes the context's amplitudes
 * (as by cclr_set_amplitudes).  energy (HOST, may be NULL) receives the
 * correlation energy.  info: iters, converged, resnorm, nsigma = residual
 * evaluations.  Returns CCLR_ENOTCONV (results written) after maxiter
 * iterations without convergence, and without writing anything if the
 * iteration diverges to non-finite values. */
int cclr_solve_ccsd(cclr_ctx* ctx, double tol, int maxiter, int nsub, cclr_c64* t1, cclr_c64* t2,
                    cclr_c64* energy, cclr_solve_info* info);

/* Copy t1 and t2 and build the property-independent Hbar intermediates
 * F^i_m, F^a_e, F^m_e, W^ij_mn, W^mb_ej, W^ie_mn, W^ef_am, W^ef_ab, W^mn_ie,
 * W^am_ef (SI, eqs. F_im ... W_amef).  Needs cclr_set_hamiltonian first
 * (CCLR_ESTATE otherwise).  Invalidates lambda. */
int cclr_set_amplitudes(cclr_ctx* ctx, const cclr_c64* t1, const cclr_c64* t2);

/* s = (A - z_k) r_k for k < nvec, z_k = omega[k] + i*gamma[k]  (right
 * EOM-EE sigma vector, SI eqs. sigma_sin-ee and sigma_double-ee).
 * nvec = 0 returns CCLR_OK and reads or writes nothing (any pointer may
 * be null); nvec < 0 is CCLR_EINVAL. */
int cclr_jacobian_right(cclr_ctx* ctx, int nvec, const double* omega, const double* gamma,
                        const cclr_c64* r1, const cclr_c64* r2, cclr_c64* s1, cclr_c64* s2);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * transform and arguments as cclr_jacobian_right, with every temporary taken
 * from a fixed 256 MiB work space that the library holds on each GPU it runs
 * on until the process ends.  The call makes no hipMalloc or hipFree and
 * starts no GEMM timing run (a product shape not yet timed in this context
 * uses the untimed kernel choice).  FP64 transforms only (CCLR_EINVAL when a
 * test hook forces another precision).  Sizes whose temporaries do not fit
 * are rejected with CCLR_ENOMEM and nothing is written; about six full
 * doubles tensors (16*o*o*v*v bytes each) per vector and three per call must
 * fit, e.g. four vectors at o=10, v=80.  Every call on one GPU uses that GPU's one work
 * space, which keeps the last call's contents: calls overlapping in time on
 * one GPU would race, so the library serializes them (a second host thread
 * waits).  The call returns after its stream has drained. */
int cclr_jacobian_right_noalloc(cclr_ctx* ctx, int nvec, const double* omega, const double* gamma,
                                const cclr_c64* r1, const cclr_c64* r2, cclr_c64* s1, cclr_c64* s2);

/* s = l_k (A - z_k)  (left sigma vector, SI eqs. sigma_sin-ee-left and
 * sigma_double-ee-left; the transposed transform of the Lambda and left
 * response equations).  nvec = 0 as for cclr_jacobian_right. */
int cclr_jacobian_left(cclr_ctx* ctx, int nvec, const double* omega, const double* gamma,
                       const cclr_c64* l1, const cclr_c64* l2, cclr_c64* s1, cclr_c64* s2);

/* Right transforms of several independent problems (contexts of any sizes
 * o, v) in one call: for context i, s_i = (A_i - z_ik) r_ik for k < nvec[i],
 * with the arrays of context i at omega[i], gamma[i], r1[i], r2[i], s1[i],
 * s2[i] (layouts as for cclr_jacobian_right).  The ring and particle-
 * particle ladder products of all contexts (SI, eq. sigma_double-ee) run
 * as one persistent launch each, with the tile shape timed once per set of
 * shapes.  The contexts must be distinct, share one hip_stream and use FP64
 * transforms; errors are reported on ctx[0]. */
int cclr_jacobian_right_multi(int nctx, cclr_ctx* const* ctx, const int* nvec, const double* const* omega,
                              const double* const* gamma, const cclr_c64* const* r1, const cclr_c64* const* r2,
                              cclr_c64* const* s1, cclr_c64* const* s2);

/* Damped linear systems, one per right-hand side k < nrhs:
 *   side == CCLR_RIGHT:  (A - z_k) x_k = -b_k
 *   side == CCLR_LEFT :  x_k (A - z_k) = -b_k
 * Davidson subspace iteration (SI, "Davidson scheme"): pivoted unit start
 * vector, projected system G'beta = -C', preconditioner (z - D)^-1 with D the
 * Fock-like diagonal, antisymmetry kept by packed (i>j, a>b) storage,
 * classical Gram-Schmidt applied twice.  info may be NULL. */
int cclr_solve_damped(cclr_ctx* ctx, int side, int nrhs, const double* omega, const double* gamma,
                      const cclr_c64* b1, const cclr_c64* b2, cclr_c64* x1, cclr_c64* x2,
                      cclr_solve_info* info);

/* The nroots lowest EOM-EE excitation energies (smallest real part) and
 * their eigenvectors: side == CCLR_RIGHT: A x_k = w_k x_k; CCLR_LEFT:
 * x_k A = w_k x_k.  These are the poles of the response function (theory
 * section, poles of the linear response function at the EOM-EE excitation
 * energies; SI, "EOM-EE sigma-vectors").  Davidson's method for a few
 * eigenpairs of a non-Hermitian matrix: one subspace shared by the roots,
 * start vectors on the smallest Fock-like diagonal entries, corrections
 * (w_k - D)^-1 r_k, restart from the Ritz vectors when the subspace is full.
 * Stops when every residual ||A x_k - w_k x_k|| <= tol (x_k of unit norm).
 * omega: HOST array of nroots complex values (written); x1[k][o][v] and
 * x2[k][o][o][v][v]: DEVICE outputs (both may be NULL to skip them).
 * 1 <= nroots <= 30; options.maxiter bounds the iterations. */
int cclr_eom_ee(cclr_ctx* ctx, int side, int nroots, double tol, cclr_c64* omega, cclr_c64* x1, cclr_c64* x2,
                cclr_solve_info* info);

/* Solve lambda A = -eta0 (eta0 singles F^i_a, doubles <ij||ab>) and keep
 * lambda in the context.  Needs cclr_set_amplitudes. */
int cclr_solve_lambda(cclr_ctx* ctx, cclr_solve_info* info);

/* Copy the context's lambda (l1[o][v], l2[o][o][v][v], device pointers). */
int cclr_get_lambda(const cclr_ctx* ctx, cclr_c64* l1, cclr_c64* l2);

/* Symmetric CC-CC linear response function for every pair of the nx
 * perturbations X[p] (host array of device pointers to n x n matrices) at
 * each of nfreq complex frequencies z = omega[w] + i*gamma[w]:
 *   out[w][p][q] = <<X_p; X_q>>_z = 1/2 [ g_pq(z) + conj g_pq(-conj z) ],
 *   g_pq(z) = eta^p t^q(z) + eta^q t^p(-z) + F t^p(-z) t^q(z),
 * with xi, eta, t^X F from the SI working equations and t^X from
 * cclr_solve_damped.  Solves lambda first if the context has none.  out is a
 * HOST array of nfreq*nx*nx complex values.  The polarizability is
 * alpha = -<<mu;mu>>. */
int cclr_response_function(cclr_ctx* ctx, int nx, const cclr_c64* const* X,
                           int nfreq, const double* omega, const double* gamma,
                           cclr_c64* out, cclr_solve_info* info);

/* The CC-CI (EOM-CC) response function (eq. CC-CI response function) with
 * the same conventions as cclr_response_function:
 *   out[w][p][q] = 1/2 [ h_pq(z) + conj h_pq(-conj z) ],
 *   h_pq(z) = Eeta^p t^q(z) + Eeta^q t^p(-z)
 *             - (lambda . t^p(-z)) (lambda . xi^q) - (lambda . t^q(z)) (lambda . xi^p),
 * with the EOM eta vector Eeta^X (SI: the singles of eta^X plus
 * lambda^ij_ab xi^X_jb, the doubles of eta^X) and "." the sum over unique
 * excitations.  The response solves are those of the CC-CC form; no Hessian
 * product is needed. */
int cclr_response_function_ci(cclr_ctx* ctx, int nx, const cclr_c64* const* X, int nfreq, const double* omega,
                              const double* gamma, cclr_c64* out, cclr_solve_info* info);

/* The CC-CC response function in the asymmetric form (the eq. following the
 * CC-CI response function): for nx operators X and ny operators Y,
 *   out[w][p][q] = <<X_p; Y_q>>_z = 1/2 [ a_pq(z) + conj a_pq(-conj z) ],
 *   a_pq(f) = eta^{X_p} . t^{Y_q}(f) + tbar^{Y_q}(f) . xi^{X_p},
 * with the multiplier responses tbar^Y(f) (A + f) = -(eta^Y + F t^Y(f)).
 * Response equations are solved for the Y operators only (right and left,
 * at z and -conj z), which pays off when ny << nx.  Equal to
 * cclr_response_function for X = Y.  out: HOST array nfreq*nx*ny. */
int cclr_response_function_asym(cclr_ctx* ctx, int nx, const cclr_c64* const* X, int ny, const cclr_c64* const* Y,
                                int nfreq, const double* omega, const double* gamma, cclr_c64* out,
                                cclr_solve_info* info);

/* Gradient of the response function (adjoint of cclr_response_function).
 * For the real scalar
 *   L = Re sum_{w,p,q} conj(G[w][p][q]) * out[w][p][q]
 * (G: HOST array nfreq*nx*nx, e.g. the output gradient handed down by an
 * autograd engine) it writes gradients in the convention
 * dL/dRe x + i dL/dIm x for every complex input entry x:
 *   dX[r]  (array of nx DEVICE n x n matrices, or NULL): with respect to the
 *          perturbation matrices, every entry of X_r treated as independent;
 *   df     (DEVICE n x n, or NULL) and dV (array of 6 DEVICE blocks in the
 *          layouts of cclr_set_hamiltonian: oooo, ooov, oovv, ovov, ovvv,
 *          vvvv; or NULL): with respect to the Fock matrix and the
 *          antisymmetrized integrals, projected onto changes that keep the
 *          symmetries of the inputs (f Hermitian; <pq||rs> antisymmetric in
 *          pq and in rs, and equal to conj <rs||pq>), so that for every such
 *          change dL = Re sum conj(grad) * change.  df and dV are given
 *          together or both NULL.  The amplitudes t are held fixed.
 * All outputs are overwritten.
 * X enters through xi^X and eta^X, linear in X (SI, "Linear response"); the
 * adjoint of the damped solves is the left transform, so the gradient needs
 * one left damped solve x (A - f) = -u per perturbation and frequency f in
 * {z, -z, z*, -z*} (eq. "LR response equation_cpp", transposed) followed by
 * transition densities of xi^X and eta^X.  The Hamiltonian enters through
 * the Hbar intermediates, the Jacobian, the Hessian product t^X F and the
 * Lambda equation (theory section, eq. "Lambda"), all linear in it at fixed
 * t; its gradient adds one right solve A x = -lambda-bar and the transposed
 * products of the intermediates, sigma and t^X F.  Intermediates and
 * solutions are recomputed, not stored by the forward call. */
int cclr_response_backward(cclr_ctx* ctx, int nx, const cclr_c64* const* X, int nfreq, const double* omega,
                           const double* gamma, const cclr_c64* G, cclr_c64* const* dX, cclr_c64* df,
                           cclr_c64* const* dV, cclr_solve_info* info);

/* Message describing the last error on ctx (or a creation error if ctx is
 * NULL); valid until the next call on the same context. */
const char* cclr_last_error(const cclr_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* CCLR_H */
