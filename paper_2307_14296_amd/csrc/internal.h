// Internal declarations of libcclr: context, device buffers, tensor views,
// the contraction engine and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <algorithm>
#include <complex>
#include <map>
#include <tuple>
#include <vector>
#include <stdexcept>

#include "../../include/cclr.h"

typedef double2 cplx;
typedef long long i64;

// ------------------------------------------------------------------ errors
struct CclrError : public std::runtime_error {
  int code;
  CclrError(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define HIPCHK(expr)                                                                  \
  do {                                                                                \
    hipError_t e__ = (expr);                                                          \
    if (e__ != hipSuccess)                                                            \
      throw CclrError(CCLR_EHIP, std::string(#expr) + ": " + hipGetErrorString(e__)); \
  } while (0)

#define REQUIRE(cond, code, msg) \
  do {                           \
    if (!(cond)) throw CclrError(code, msg); \
  } while (0)

// ------------------------------------------------------- device memory
struct cclr_ctx;

// RAII device allocation accounted against the context's cap.
struct DevBuf {
  cclr_ctx* ctx = nullptr;
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void alloc(cclr_ctx* c, size_t nbytes);
  void release();
  cplx* c() const { return (cplx*)p; }
};

// Bump allocator for temporaries.  Chunks are kept for reuse after a reset
// (device allocation is slow and synchronizing); trim() releases the unused
// ones at a quiet point.
struct Arena {
  cclr_ctx* ctx = nullptr;
  std::vector<DevBuf*> chunks;
  std::vector<size_t> used;
  size_t cur = 0;
  size_t chunk_bytes = size_t(256) << 20;
  // while hold > 0, reset() keeps everything: memory handed to work queued on
  // another stream stays untouched until that stream has been joined
  int hold = 0;
  // external mode: while ext is set, get() carves from [ext, ext + ext_bytes)
  // and never allocates; a request beyond the region throws CCLR_ENOMEM
  char* ext = nullptr;
  size_t ext_bytes = 0, ext_used = 0, ext_peak = 0;
  ~Arena();
  void* get(size_t bytes);
  struct Mark { size_t chunk, top; };
  Mark mark() const;
  void reset(Mark m);
  void trim();
};

// ----------------------------------------------------------- tensor views
// A strided complex tensor (up to 6 dims).  When read, an element is
// scale * (conj ? conj(x) : x).
struct Ten {
  cplx* p = nullptr;
  int nd = 0;
  i64 dim[6] = {0, 0, 0, 0, 0, 0};
  i64 st[6] = {0, 0, 0, 0, 0, 0};
  bool conj = false;
  double sr = 1.0, si = 0.0;
  i64 size() const {
    i64 s = 1;
    for (int d = 0; d < nd; ++d) s *= dim[d];
    return s;
  }
};

Ten ten(cplx* p, std::initializer_list<i64> dims);      // contiguous row-major
Ten ten(const DevBuf& b, std::initializer_list<i64> dims);
// Reorder the axes of a view: `from` names the axes of t, `to` the new order.
Ten reorder(const Ten& t, const char* from, const char* to);
Ten scaled(const Ten& t, double re, double im = 0.0);
Ten conjugated(const Ten& t);

// ------------------------------------------------------------- kernels
struct GemmArgs {
  int M, N, K, batch;
  const cplx* A; i64 sAb, sAm, sAk; int conjA;
  const cplx* B; i64 sBb, sBk, sBn; int conjB;
  cplx* C; i64 sCb, sCm, sCn;
  double ar, ai;   // alpha
  int beta;        // 0: C = alpha*AB, 1: C += alpha*AB
  int kchunk;      // > 0: K split in chunks of kchunk; batch then counts (batch index, chunk) pairs,
                   // chunk fastest, and C is the [batch][chunk][M][N] workspace (single batch index)
  // optional second batch index: with nb2 > 1, batch b = b1 * nb2 + b2 and the
  // operands are offset by b1 * s?b + b2 * s?b2
  int nb2;
  i64 sAb2, sBb2, sCb2;
};
void launch_zgemm(const GemmArgs& g, hipStream_t s);
// FP64 kernel variants (tile shape, three or four real products per complex
// block); variants 4 + k run variant k (k = 1..4) in the XCD-grouped tile
// order; 9, 10: the 64x64 four-product tile with one LDS buffer (three
// waves per SIMD), plain and grouped order; 11, 12: the same for 128x64
// tiles (two waves per SIMD); 13, 14: 128x128 four-product tiles with
// double-buffered LDS and eight waves (two per SIMD, one workgroup per CU);
// 15, 16: the same tile with direct global-to-LDS operand loads; 17, 18: 64x256
// direct-load tiles (eight waves in one row), for products with few rows;
// 19, 20: 128x32 (one LDS buffer) and 64x32 four-product tiles, for products
// with at most 32 output columns (a 64-column tile would be mostly padding)
enum {
  GEMM_SIMPLE = 0, GEMM_128x64_G3 = 1, GEMM_64x64_G3 = 2, GEMM_128x64_G4 = 3, GEMM_64x64_G4 = 4,
  GEMM_64x64_G4_SB = 9, GEMM_64x64_G4_SB_GROUPED = 10, GEMM_128x64_G4_SB = 11, GEMM_128x64_G4_SB_GROUPED = 12,
  GEMM_128x128_G4 = 13, GEMM_128x128_G4_GROUPED = 14, GEMM_128x128_DMA = 15,
  GEMM_128x128_DMA_GROUPED = 16, GEMM_64x256_DMA = 17, GEMM_64x256_DMA_GROUPED = 18, GEMM_128x32_G4_SB = 19,
  GEMM_64x32_G4 = 20, GEMM_NVAR = 21
};
// the narrow variants (19, 20): timed by the autotuner for outputs at most this
// wide (and for wider ones up to 512 that 64-column tiles pad much more)
constexpr int kNarrowMaxN = 64;
bool gemm_variant_grouped(int variant);
bool gemm_variant_narrow(int variant);
// an autotuner choice: an FP64 variant v, or kTransposedChoice + v for variant
// v on the transposed product C^T = B^T A^T
constexpr int kTransposedChoice = 100;
void launch_gemm_choice(const GemmArgs& g, int choice, hipStream_t s);
void launch_zgemm_variant(const GemmArgs& g, int variant, hipStream_t s);
int gemm_default_variant(const GemmArgs& g);
// Several products (same operand layouts: ak = unit-stride k in A, bn = unit-
// stride n in B; batch 1 or batched, no K splitting) in one persistent launch.
// probs / tstart are DEVICE arrays: problem p owns tiles [tstart[p], tstart[p+1])
// of the variant's tile shape (gemm_tile_rows(variant) x gemm_tile_cols(variant)).
void launch_zgemm_group(const GemmArgs* probs, const int* tstart, int nprob, int total, int variant, bool ak, bool bn,
                        hipStream_t s);
int gemm_tile_rows(int variant);
int gemm_tile_cols(int variant);
// the same product with FP32 (prec = CCLR_FP32) or split-BF16 (CCLR_BF16X3)
// MFMA arithmetic and FP32 accumulation; operands and C stay complex128 in memory
void launch_zgemm_lowp(const GemmArgs& g, int prec, hipStream_t s);
// Products on pre-split operands (gemm_split.hip): split-BF16 with three (X3:
// both operands split hi + lo) or two (X2: the B operand hi only) bf16
// products per real product, and FP32 Gauss planes (three real products per
// complex block).
enum { BF16_X3 = 0, BF16_X2 = 1, F32_G3 = 2 };
bool split_form_valid(int form);
int split_form_of(int prec);  // prec CCLR_FP32, CCLR_BF16X3 or CCLR_BF16X2
// A split operand of one form and side (0: A, the rows of C; 1: B, the
// columns): a rows x K complex matrix as [K/kstep][rows_pad][chunks] 16-byte
// chunks of planes (bf16: kstep 32, codes in planes[]; FP32: kstep 16, three
// planes), position-permuted within a row, zero padded.
struct SplitMat {
  const void* p = nullptr;
  int rows = 0, K = 0, rows_pad = 0, nkc = 0;
  int form = 0, side = 0, nplanes = 0, chunks = 0;
  int planes[4] = {0, 0, 0, 0};
};
SplitMat split_shape(int rows, int K, int form, int side);
size_t split_bytes(int rows, int K, int form, int side);
// dst <- split of op(src)[r][k] = src[r*sR + k*sK] (conjugated if conj)
SplitMat launch_split(int rows, int K, const cplx* src, i64 sR, i64 sK, int conj, void* dst, int form, int side,
                      hipStream_t s);
// C[m][n] (+)= alpha * sum_k A[m][k] B[n][k] on operands split for one form, FP32 accumulation
void launch_split_gemm(const SplitMat& A, const SplitMat& B, cplx* C, i64 sCm, i64 sCn, double ar, double ai,
                       int beta, hipStream_t s);
// Eigenpairs of a small dense complex matrix on the GPU (one workgroup):
// H(i, j) = Hu[j ld + i] for i <= j and Hl[i ld + j] for i > j, n <= kSmallEigMax;
// work holds small_eig_work_elems(n) elements.  Writes theta[r] and the unit-norm
// right eigenvector coef[r ldc + i] of the nroots eigenvalues of smallest real
// part (ties by index), coef2 = -theta coef, all eigenvalues in wall (if not
// null), and status[0] = 1, or 0 if the QR iteration did not converge.
constexpr int kSmallEigMax = 120;
size_t small_eig_work_elems(int n);
void launch_small_eig(int n, const cplx* Hu, const cplx* Hl, int ld, cplx* work, int nroots, cplx* coef, cplx* coef2,
                      int ldc, cplx* theta, cplx* wall, int* status, hipStream_t st);
// products with K <= 32 on the vector ALU (returns false if the form does not apply)
bool launch_zgemm_smallk(const GemmArgs& g, hipStream_t s);
// C[b][m][n] = (beta ? C : 0) + alpha * sum_s W[b][s][m][n]
// products with at most 16 output columns (after transposing, if the unit-stride output index is n):
// skinny_plan fills g (possibly the transposed product), the chunk length kc and the chunk count S,
// or returns false; S > 1 needs a workspace W of batch*S*M*N elements (the launch also sums it into C)
bool skinny_plan(const GemmArgs& g0, GemmArgs& g, int& kc, int& S);
void launch_zgemm_skinny(const GemmArgs& g, int kc, int S, cplx* W, hipStream_t s);
// products with at most 8 output columns whose long operand has unit stride in k
// (sAk = 1): chunk length kc and chunk count S (a workspace of batch*S*M*N
// elements when S > 1)
bool rowdot_plan(const GemmArgs& g, int& kc, int& S);
void launch_zgemm_rowdot(const GemmArgs& g, int kc, int S, cplx* W, hipStream_t s);
void launch_splitk_reduce(int nb, int S, int M, int N, const cplx* W, cplx* C, i64 sCb, i64 sCm, i64 sCn, double ar,
                          double ai, int beta, hipStream_t s);
// GEMM with automatic K splitting when the output has too few tiles to fill the GPU
void run_gemm(cclr_ctx* c, const GemmArgs& g);
// FP64 GEMM through the autotuner (large products: variant timed once per shape class)
int tuned_gemm(cclr_ctx* c, const GemmArgs& g);  // returns the variant launched
// extent rounded up to the autotuner's quarter-octave and octave shape classes
int shape_bucket(int x);
int octave_bucket(int x);

struct CopyArgs {
  int nd;
  i64 dim[6], sd[6], ss[6];
  cplx* dst;
  const cplx* src;
  double ar, ai;
  int conj;
  int acc;
  i64 total;
};
void launch_tcopy(const CopyArgs& a, hipStream_t s);
void launch_fill(cplx* p, i64 n, cplx val, hipStream_t s);

// packed excitation-vector sets: singles s[k][o*v], doubles d[k][O2][V2]
struct VecSet {
  cplx* s = nullptr;
  cplx* d = nullptr;
  int n = 0;
};

void launch_unpack(int nvec, int o, int v, const cplx* s, const cplx* d, cplx* r1, cplx* r2, hipStream_t st);
// packed doubles -> ring layout rr[k][i][a][m][e] = r^ae_im
void launch_unpack_ring(int nvec, int o, int v, const cplx* d, cplx* rr, hipStream_t st);
void launch_pack_full(int nvec, int o, int v, const cplx* r1, const cplx* r2, cplx* s, cplx* d, hipStream_t st);
// pair packing of the last two indices: dst[r][AB] = src[r][a][b] (a > b)
// X[P][Q] += alpha (d(p1,q1) F[p2][q2] - d(p1,q2) F[p2][q1] - d(p2,q1) F[p1][q2] + d(p2,q2) F[p1][q1])
// for pairs P = (p1 > p2), Q = (q1 > q2) of n indices; X is [n(n-1)/2][n(n-1)/2], F is n x n
void launch_pair_fold(int n, const cplx* F, cplx* X, double alpha, hipStream_t s);
// W[a][m][pair(a,x)] += (a > x ? 1 : -1) F[m][x] for x != a (W [v][o][v(v-1)/2], F [o][v])
void launch_fold_ov(int o, int v, const cplx* F, cplx* W, hipStream_t s);
// dst[b][P][x] = src[b][p1][p2][x] for P = (p1 > p2) (src [nb][n][n][rest] -> dst [nb][n(n-1)/2][rest])
void launch_pack_first_pair(i64 nb, int n, i64 rest, const cplx* src, cplx* dst, hipStream_t s);
// the inverse for antisymmetric data: dst[b][i][j][x] = +-src[b][pair(i,j)][x], 0 on i == j
void launch_unpack_first_pair(i64 nb, int n, i64 rest, const cplx* src, cplx* dst, hipStream_t s);
struct cclr_ctx;
// adds (sign = +1) or removes (sign = -1) the doubles' one-body term P(ab) F^b_e r^ae_ij
// folded into the packed particle-ladder operator c->Wp
void fold_vv(cclr_ctx* c, double sign);
void launch_pack_pairs(i64 rows, int v, const cplx* src, cplx* dst, hipStream_t s);
// dst[r][a][b] += alpha src[r][AB], dst[r][b][a] -= alpha src[r][AB]
void launch_unpack_pairs_acc(i64 rows, int v, const cplx* src, cplx* dst, double alpha, hipStream_t s);
// W[EF][X] += alpha (Y[e][f][X] - Y[f][e][X]), e > f, X < nc; W row stride ldw
void launch_pair_antisym_acc(int v, int nc, const cplx* Y, cplx* W, i64 ldw, double alpha, hipStream_t s);
// dst[e][f][a][b] = W^ef_ab from Wp[EF][AB]
void launch_unpack_vvvv(int v, const cplx* Wp, cplx* dst, hipStream_t s);
void launch_pack_vvvv(int v, const cplx* W, cplx* Wp, hipStream_t s);
// out(packed) += X0 + P(ab)Xa + P(ij)Xi + P(ab)P(ij)Xai  (any X may be null),
// singles out += S1; then out -= z_k * r_k  (z may be null).  X0, Xa, Xi are
// [k][i][j][a][b]; Xai is [k][i][j][a][b], or [k][i][a][j][b] if xai_ring; Xa
// is [k][IJ][a][b] (pairs i > j only) if xa_half; Xi is [k][i][j][AB] (pairs
// a > b only) if xi_vpacked.
void launch_pack_sigma(int nvec, int o, int v, const cplx* X0, const cplx* Xa, const cplx* Xi, const cplx* Xai,
                       const cplx* S1, cplx* outs, cplx* outd, const cplx* zk, const cplx* rs, const cplx* rd,
                       hipStream_t st, bool xai_ring = false, bool xa_half = false, bool xi_vpacked = false);

// ------------------------------------------------------------ context
struct cclr_ctx {
  int o = 0, v = 0;
  cclr_options opt{};
  hipStream_t stream = nullptr;
  std::string err;
  size_t allocated = 0;
  int device = 0;

  // inputs
  DevBuf f, Voooo, Vooov, Voovv, Vovov, Vovvv, Vvvvv, t1, t2;
  bool have_H = false, have_t = false, have_lam = false;
  // intermediates (unpacked, W[p][q][r][s] = W^pq_rs)
  DevBuf Foo, Fvv, Fov, Woooo, Wovvo, Wbar, Wooov, Wvovv, Wovoo, Wvvvo;
  DevBuf Wp;         // packed particle-ladder operator, [V2][V2], a>b, e>f: W^ab_ef with the
                     // doubles' F^b_e term folded in (see fold_vv; the only copy of W^ab_ef)
  // operators of the right transform with one index pair packed, so that the
  // products over that pair run on it once: VoovvH[MN][e][f] = V^mn_ef (m>n),
  // VoovvP[m][n][EF] = V^mn_ef (e>f), WvovvP[a][m][EF] = W^am_ef (e>f) with the
  // singles term -F^m_e r^ea_im folded in
  DevBuf VoovvH, VoovvP, WvovvP;
  // the operands of the P(ab)-only doubles terms with the occupied pair packed
  // (their output is needed for i > j only): WovooH[m][b][IJ] = W^mb_ij,
  // WooovH[IJ][m][b] = W^ij_mb, t2H[IJ][a][f] = t^af_ij
  DevBuf WovooH, WooovH, t2H;
  DevBuf t2P;        // t2P[i][n][AB] = t^ab_in (a > b), for the P(ij)-only right doubles term
  DevBuf Wop;        // packed hole-ladder operator, [O2][O2], m>n (rows), i>j (columns): W^mn_ij with
                     // the doubles' F^m_j term folded in
  DevBuf WR, WL;     // ring operators: WR[j][b][m][e] = W^mb_ej, WL[m][e][j][b] = W^je_bm
  DevBuf WvvvoTP;    // WvvvoTP[j][e][AB] = W^ab_ej (a > b), for the right doubles term P(ij) W^ab_ej r^e_i
  DevBuf WvvvoLP, WvovvL;  // WvvvoLP[a][m][EF] = W^ef_am (e > f), WvovvL[i][a][f][e] = W^ei_fa (left transform)
  // split-BF16 copies of the ladder and ring operators, made on first use in
  // that precision (in the form of the products): right ladder, left ladder,
  // right ring, left ring
  DevBuf wsplit[4];
  SplitMat wsplit_m[4];
  DevBuf diag;       // Fock-like diagonal for preconditioning: singles then doubles (packed)
  DevBuf lam_s, lam_d;  // lambda, packed
  DevBuf Vpk;         // packed <ab||ef> (a>b, e>f) of the ground-state residual, made on first use
  Arena arena;
  // arithmetic of the ladder and ring products in the transforms being applied
  // (CCLR_FP64 for the FP64 path and every true residual; opt.prec inside the
  // low-precision inner solves)
  int sigma_prec = CCLR_FP64;
  // relative residual at which a reduced-precision inner solve is refined (0: default)
  double inner_tol = 0.0;
  // GEMM autotuner: best FP64 kernel variant per shape class, and a record of
  // the timings that decided it (variant -> ms)
  std::map<std::tuple<int, int, int, int, int>, int> gemm_choice;
  struct TuneRecord {
    std::string shape;
    std::vector<std::pair<int, double>> ms;  // (variant, ms) of every timed variant
    int chosen;
  };
  std::vector<TuneRecord> gemm_tuning_log;
  bool autotune = true;
  // no new timing runs (they create events and take scratch outputs); cached
  // choices are still used
  bool no_timing = false;
  // this device's copy of the library's fixed work space (see capi.hip)
  void* fixed_ws = nullptr;
  size_t fixed_ws_peak = 0;  // bytes of it the last such call took at most
  // kernel variant of grouped multi-context launches, per set of product shapes
  std::map<std::string, int> group_choice;
  // the ring and ladder products of an FP64 right transform run on a second
  // stream of default priority (`side`, created on first use) while the other
  // products run on `stream`; joined before the result is packed
  bool overlap = false;
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // optional per-product timing of run_gemm (shape, kernel form, ms), for diagnostics
  bool gemm_trace = false;
  std::vector<std::string> gemm_trace_log;
  // test overrides of size-dependent blocking (0 = natural): the column block
  // of the packed W^ef_ab build (AB pairs per block) and the number of
  // right-hand sides a memory-bounded group may hold
  i64 dbg_wp_block = 0;
  int dbg_rhs_group = 0;
  // optional timing of the particle-particle ladder GEMM launches
  bool prof = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_events;
  std::vector<double> prof_flops;
  std::vector<int> prof_prec;  // arithmetic of each recorded launch

  i64 O2() const { return (i64)o * (o - 1) / 2; }
  i64 V2() const { return (i64)v * (v - 1) / 2; }
  i64 ns() const { return (i64)o * v; }
  i64 nd() const { return O2() * V2(); }
};

// integral block views (any kinds string, e.g. "vovv"), derived by symmetry
Ten Vblk(cclr_ctx* c, const char* kinds);
Ten fblk(cclr_ctx* c, const char* kinds);

// ------------------------------------------------------ contraction engine
// C[lc] (+)= alpha * sum A[la] B[lb]  (labels: one char per axis)
void contract(cclr_ctx* c, cplx alpha, const Ten& A, const char* la, const Ten& B, const char* lb,
              const Ten& C, const char* lc, bool accumulate = true);
// dst[ld] (+)= alpha * src[ls]   (ls a permutation of ld)
void tcopy(cclr_ctx* c, const Ten& dst, const char* ld, const Ten& src, const char* ls, cplx alpha,
           bool accumulate = true);
void tzero(cclr_ctx* c, const Ten& t);
Ten tmp(cclr_ctx* c, std::initializer_list<i64> dims);

inline cplx cx(double r, double i = 0.0) { return make_double2(r, i); }

// ------------------------------------------------------------ schedule
void build_intermediates(cclr_ctx* c);
// runs f with the plain W^ab_ef in c->Wp (the one-body term taken out and put back afterwards)
template <class F>
void with_plain_wp(cclr_ctx* c, F&& f) {
  fold_vv(c, -1.0);
  try {
    f();
  } catch (...) {
    try {
      fold_vv(c, 1.0);
    } catch (...) {
    }
    throw;
  }
  fold_vv(c, 1.0);
}
// sigma for nvec packed vectors in `in` -> `out` (packed); z per vector (may be null)
void sigma_right(cclr_ctx* c, const VecSet& in, const VecSet& out, const cplx* z_dev);
// The right sigma in two halves around its two large products, so that the
// products of several contexts can be launched together: begin runs every
// other term and returns the ring and ladder products (not yet launched);
// finish adds the hole ladder and packs the result once both have run.
struct SigmaAcc {
  Ten X0, Xa, Xi, Xai, S1, R1, R2;
};
struct SigmaWork {
  Arena::Mark mk;
  SigmaAcc a;
  GemmArgs ring, ladder;
};
SigmaWork sigma_right_begin(cclr_ctx* c, const VecSet& in, const VecSet& out);
void sigma_finish(cclr_ctx* c, SigmaWork& w, const VecSet& in, const VecSet& out, const cplx* z_dev);
void sigma_left(cclr_ctx* c, const VecSet& in, const VecSet& out, const cplx* z_dev);

// ------------------------------------------------- solver and response pieces
void launch_check_finite(const cplx* p, i64 n, int* flag, hipStream_t s);
void launch_bdot(int npair, const cplx* const* xs, const cplx* const* xd, const cplx* const* ys,
                 const cplx* const* yd, i64 ov, i64 nd, cplx* partial, cplx* out, hipStream_t s, bool conjx = false);
void launch_caxpy(i64 n, cplx a, const cplx* x, cplx* y, hipStream_t s);
void launch_conj_inplace(i64 n, cplx* x, hipStream_t s);
// (A - z_k) x_k = -rhs_k (right) or x_k (A - z_k) = -rhs_k (left) in the context's precision
int solve_system(cclr_ctx* c, int side, int nr, const cplx* zh, const VecSet& rhs, const VecSet& xout,
                 cclr_solve_info* info);
// folds the conditioning estimates of src into dst (largest kappa, smallest nonzero Ritz value)
void merge_conditioning(cclr_solve_info& dst, const cclr_solve_info& src);
// nvec packed vectors from the arena
VecSet packed_buf(cclr_ctx* c, int n);
// how many of n vectors with the given working memory each fit in free device memory (>= 1)
int fit_vectors(cclr_ctx* c, double bytes_per_vec, int n);
void build_xi(cclr_ctx* c, const cplx* X, const VecSet& out);
void build_eta(cclr_ctx* c, const cplx* X, const VecSet& out);
void hessian_product(cclr_ctx* c, const VecSet& xin, const VecSet& out);
void density_xi(cclr_ctx* c, const VecSet& y, cplx* D, cplx alpha);
void density_eta(cclr_ctx* c, const VecSet& y, cplx* D, cplx alpha);
// gradient with respect to f and the integral blocks (see adjoint.hip)
void hamiltonian_adjoint(cclr_ctx* c, int nx, const cplx* Xs, const VecSet& sol, const VecSet& xl, const VecSet& Y,
                         const VecSet& PA, const VecSet& PB, cplx* df, cplx* const* dV, cclr_solve_info* info);
// CCSD ground state (ground.hip): residual of one packed amplitude vector
// (returns the correlation energy), the CROP solve (t: start in, solution
// out), and the integral blocks from Cholesky vectors L[nchol][n][n]
std::complex<double> ccsd_residual(cclr_ctx* c, const VecSet& t, const VecSet& out);
int ccsd_crop(cclr_ctx* c, double tol, int maxit, int nsub, const VecSet& t, std::complex<double>* energy,
              cclr_solve_info* info);
void integrals_from_cholesky(cclr_ctx* c, int nchol, const cplx* L);
// lowest EOM-EE eigenpairs (right: A x = w x, left: x A = w x); omega by increasing real part
int eom_davidson(cclr_ctx* c, int side, int nroots, double tol, int maxit, std::vector<cplx>& omega,
                 const VecSet& xout, cclr_solve_info* info);
