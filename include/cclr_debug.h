/*
 * cclr_debug.h — internal test hooks of libcclr (not part of the public ABI).
 *
 * Used by the test suite to check single building blocks of the library on
 * the GPU: the complex GEMM kernel, the contraction engine and the Hbar
 * intermediates.  All tensor pointers are device pointers to complex128
 * data; dims/strides are host arrays of element counts.
 */
#ifndef CCLR_DEBUG_H
#define CCLR_DEBUG_H
#include "cclr.h"
#ifdef __cplusplus
extern "C" {
#endif

/* C[b][m][n] (+)= alpha * sum_k op(A)[b][m][k] op(B)[b][k][n] with element strides;
 * op = complex conjugate when conjA/conjB is set; beta 0 overwrites, 1 accumulates. */
int cclr_dbg_zgemm(int M, int N, int K, int batch, const cclr_c64* A, long long sAb, long long sAm, long long sAk,
                   int conjA, const cclr_c64* B, long long sBb, long long sBk, long long sBn, int conjB, cclr_c64* C,
                   long long sCb, long long sCm, long long sCn, double alpha_re, double alpha_im, int beta);

/* C[b] (+)= alpha * op(A[b]) op(B[b]) for b < batch with one FP64 kernel
 * variant (0: simple; 1..4: MFMA tiles 128x64 / 64x64 with three or four
 * real products per complex block; 4 + k: variant k in the XCD-grouped tile
 * order; 9, 10 and 11, 12: 64x64 and 128x64 four-product tiles with one LDS
 * buffer, plain and grouped order; 13, 14: 128x128 tiles, operands staged
 * through registers; 15, 16: 128x128 tiles with direct global-to-LDS operand
 * loads; 17, 18: 64x256 direct-load tiles; plain and grouped order; 19: 128x32
 * tiles with one LDS buffer, 20: 64x32 tiles, for outputs at most 32 wide;
 * 100 + v: variant v on the transposed product C^T = B^T A^T).
 * All pointers are device memory; strides in elements.  For tests
 * of every variant (the autotuner otherwise runs only the fastest). */
int cclr_dbg_zgemm_f64(int variant, int batch, int M, int N, int K, const cclr_c64* A, long long sAb, long long sAm,
                       long long sAk, int conjA, const cclr_c64* B, long long sBb, long long sBk, long long sBn,
                       int conjB, cclr_c64* C, long long sCb, long long sCm, long long sCn, double ar, double ai,
                       int beta);

/* The engine's strided copy: for every index (i_0 .. i_{nd-1}) < dim,
 * dst[sum i_d sd[d]] = (acc ? dst : 0) + alpha * op(src[sum i_d ss[d]]), op
 * the conjugate when conj; alpha = 0 writes zeros without reading src.
 * nd <= 6; device pointers; strides in elements.  For tests of its forms
 * (merged indices, 32-bit index path, LDS-tiled transpose). */
int cclr_dbg_tcopy(int nd, const long long* dim, const long long* sd, const long long* ss, cclr_c64* dst,
                   const cclr_c64* src, double ar, double ai, int conj, int acc);

/* Split-K form of one FP64 MFMA variant (1 .. 20): the partial products
 * W[s][m][n] = sum over k in chunk s (k = s kchunk .. min(K, (s+1) kchunk) - 1)
 * of A(m, k) B(k, n), for s < ceil(K / kchunk); A(m, k) = A[m sAm + k sAk],
 * B(k, n) = B[k sBk + n sBn]; device pointers.  For tests of the chunk
 * bounds that the split-K products of the engine rely on. */
int cclr_dbg_zgemm_f64_splitk(int variant, int M, int N, int K, int kchunk, const cclr_c64* A, long long sAm,
                              long long sAk, const cclr_c64* B, long long sBk, long long sBn, cclr_c64* W);

/* Several independent products C[p] = A[p] B[p] (A[p] row-major M[p] x K[p];
 * B[p] row-major K[p] x N[p], or N[p] x K[p] when btrans; C[p] row-major
 * M[p] x N[p]; all device pointers) in the one persistent grouped launch of
 * FP64 variant 1, 2, 3, 4, 13 or 15 (the tile shapes that have a grouped form). */
int cclr_dbg_zgemm_group_f64(int variant, int nprob, const int* M, const int* N, const int* K,
                             const cclr_c64* const* A, const cclr_c64* const* B, int btrans, cclr_c64* const* C);

/* The same product (device pointers, the context's stream) through the
 * context's GEMM dispatch: the short-reduction vector-ALU kernel, the
 * short-output vector-ALU kernels (at most 16 columns with the long operand
 * contiguous in m, at most 8 with it contiguous in k), split-K, or the
 * autotuned MFMA kernels (a product with at most 32 rows and more columns
 * runs transposed), chosen by shape as for the contractions of a transform. */
int cclr_dbg_run_gemm(cclr_ctx* ctx, int M, int N, int K, int batch, const cclr_c64* A, long long sAb, long long sAm,
                      long long sAk, int conjA, const cclr_c64* B, long long sBb, long long sBk, long long sBn,
                      int conjB, cclr_c64* C, long long sCb, long long sCm, long long sCn, double alpha_re,
                      double alpha_im, int beta);

/* The same dispatch with a two-level batch: batch entry b = b1 nb2 + b2
 * (b1 < nb1, 1 < nb2) of X starts at b1 sXb + b2 sXb2; no conjugation. */
int cclr_dbg_run_gemm_b2(cclr_ctx* ctx, int M, int N, int K, int nb1, int nb2, const cclr_c64* A, long long sAb,
                         long long sAb2, long long sAm, long long sAk, const cclr_c64* B, long long sBb,
                         long long sBb2, long long sBk, long long sBn, cclr_c64* C, long long sCb, long long sCb2,
                         long long sCm, long long sCn, double alpha_re, double alpha_im, int beta);

/* The same product (batch 1) in reduced arithmetic on pre-split operands, the
 * form of the transforms' ladder and ring products: prec = CCLR_FP32 (FP32
 * MFMA, three real products per complex block), CCLR_BF16X3 or CCLR_BF16X2
 * (split-BF16 MFMA, FP32 accumulation); prec = 16: the engine's FP32 kernel
 * of the other products (complex128 operands converted in the kernel).
 * Operands and C stay complex128. */
int cclr_dbg_zgemm_lowp(int prec, int M, int N, int K, const cclr_c64* A, long long sAm, long long sAk, int conjA,
                        const cclr_c64* B, long long sBk, long long sBn, int conjB, cclr_c64* C, long long sCm,
                        long long sCn, double alpha_re, double alpha_im, int beta);

/* C[lc] += alpha * sum A[la] B[lb] through the contraction engine; A, B, C are
 * contiguous row-major tensors with the given dims (nd = strlen of labels). */
int cclr_dbg_contract(cclr_ctx* ctx, double alpha_re, double alpha_im, const cclr_c64* A, const char* la,
                      const long long* adims, const cclr_c64* B, const char* lb, const long long* bdims, cclr_c64* C,
                      const char* lc, const long long* cdims);

/* Copy the named intermediate (Foo, Fvv, Fov, Woooo, Wovvo, Wbar, Wooov, Wvovv,
 * Wovoo, Wvvvo, Wvvvv, Wp, diag) into dst; *count receives its element count
 * (dst may be NULL to query the count only). */
int cclr_dbg_get(cclr_ctx* ctx, const char* name, cclr_c64* dst, long long* count);

/* Enable (1) or disable (0) event timing of the particle-particle ladder
 * GEMM launches; enabling clears earlier records. */
int cclr_dbg_profile(cclr_ctx* ctx, int enable);

/* Launch count, summed duration (ms, from HIP events on the context's
 * stream) and summed algorithmic flops (8 per complex multiply-add) of the
 * ladder GEMM launches recorded since profiling was enabled, those in
 * arithmetic prec only (CCLR_FP64 ...; -1: all); with largest_only, only the
 * launches of the largest such product (most flops).  A split-BF16 launch
 * includes the split of the trial vectors. */
int cclr_dbg_profile_read(cclr_ctx* ctx, int largest_only, int prec, long long* launches, double* ms,
                          double* flops);

/* Arithmetic of the ladder and ring products used by subsequent
 * cclr_jacobian_right/left calls on ctx (CCLR_FP64, CCLR_FP32, CCLR_BF16X3,
 * CCLR_BF16X2); the solvers set it themselves. */
int cclr_dbg_set_sigma_prec(cclr_ctx* ctx, int prec);

/* Relative residual at which a reduced-precision inner solve hands over to
 * an FP64 refinement step (0: the default of the context's precision). */
int cclr_dbg_set_inner_tol(cclr_ctx* ctx, double tol);

/* Per-product timing of the contraction engine's GEMMs: writes up to cap
 * bytes of the record so far, one line per product: "MxNxK bB sA(m,k)
 * sB(k,n) sC(m,n) sb(A,B,C) beta E form F ms TFLOP/s" (sb: the batch
 * strides; E: 1 when the product accumulates into C; F: FP64 variant >= 0
 * (100 + v: variant v on the transposed product),
 * -1 short-reduction VALU
 * kernel, -2 split-K, -3 reduced precision, -4 short-output VALU kernel, -5
 * reduced precision on pre-split FP32 planes, -6 short-output VALU kernel on
 * a long operand contiguous in k);
 * then, for enable >= 0, clears the record and switches timing on (1) or
 * off (0).  Timing synchronizes the stream after every product. */
int cclr_dbg_gemm_trace(cclr_ctx* ctx, int enable, char* buf, long long cap);

/* Run (1) or do not run (0) the ring and ladder products of FP64 right
 * transforms on a second stream, concurrently with the other products. */
int cclr_dbg_set_overlap(cclr_ctx* ctx, int enable);

/* Size-dependent blocking, for tests of the paths that large problems take
 * (0 restores the natural choice):
 *   wp_block  > 0: the packed W^ef_ab build of later cclr_set_amplitudes calls
 *              forms the term -P(ef) t^e_m V^mf_ab in column blocks of wp_block
 *              AB pairs (naturally at most 2 GiB of temporary per block, so
 *              only v >= 129 takes more than one block);
 *   rhs_group > 0: lockstep solves and Hessian products take at most
 *              rhs_group right-hand sides per group (naturally as many as fit
 *              in free device memory under the context's cap).
 * Negative values are CCLR_EINVAL. */
int cclr_dbg_set_blocking(cclr_ctx* ctx, long long wp_block, int rhs_group);

/* Hessian products (t^X F) of nvec response vectors with the context's
 * amplitudes and lambda (cclr_solve_lambda first; CCLR_ESTATE otherwise):
 * x1 [nvec][o][v], x2 [nvec][o][o][v][v] in (only unique doubles read), s1,
 * s2 the same layouts out (full antisymmetric doubles); device pointers. */
int cclr_dbg_hessian(cclr_ctx* ctx, int nvec, const cclr_c64* x1, const cclr_c64* x2, cclr_c64* s1, cclr_c64* s2);

/* Bytes of the fixed work space that the context's last
 * cclr_jacobian_right_noalloc call took at most (0 before the first). */
int cclr_dbg_fixed_ws_peak(const cclr_ctx* ctx, long long* bytes);

/* The GPU eigensolver of the EOM-EE Davidson subspace (Householder
 * reduction, shifted QR, back substitution; one workgroup) on a host matrix
 * H (n x n row-major, 1 <= n <= 120): all eigenvalues in w[n] (in the order
 * of the Schur form), the nroots eigenvalues of smallest real part (ties by
 * index) in theta and their unit-norm right eigenvectors in vecs[nroots][n].
 * Host pointers.  CCLR_ENOTCONV if the QR iteration does not converge. */
int cclr_dbg_small_eig(int n, const cclr_c64* H, int nroots, cclr_c64* w, cclr_c64* theta, cclr_c64* vecs);

/* Autotuner record: writes up to cap bytes of text, one line per tuned
 * GEMM shape class: "MxNxK bB layoutL timed mxNxK bb: variant=ms ... -> chosen"
 * (the product's shape, then the part of it that was timed: at most 8192 rows
 * and 16 batch entries, so the times are those of the timed part; chosen is
 * the variant in use: within 2% of the fastest, the grouped tile order, then
 * larger tiles, are preferred; 100 + v is variant v on the transposed product
 * C^T = B^T A^T, timed for the 32-column variants when the row count is one
 * they pad less than 64-row tiles would).
 * enable >= 0 switches tuning of new shape classes on (1) or off (0) for
 * later products; with tuning off a product of a class not yet timed takes
 * the untimed choice, and the classes already timed keep theirs. */
int cclr_dbg_tuning(cclr_ctx* ctx, int enable, char* buf, long long cap);

#ifdef __cplusplus
}
#endif
#endif
