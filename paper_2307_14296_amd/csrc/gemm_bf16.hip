// Split-BF16 complex GEMM for the low-precision inner solves.
//
// Every real component x of a complex128 operand is split into two bf16
// numbers, hi = bf16(x) and lo = bf16(x - hi), so x = hi + lo to about 2^-17
// relative.  A real product is then formed from three bf16 MFMA products,
// hi*hi + hi*lo + lo*hi (the lo*lo term is below the split's own error),
// accumulated in FP32 on v_mfma_f32_16x16x32_bf16.  A complex block takes
// four real products (Re = ArBr - AiBi, Im = ArBi + AiBr), so twelve bf16
// MFMAs; the negated Ai planes are made in registers by flipping sign bits.
//
// Operands are stored pre-split ("split layout"): a rows x K complex matrix
// becomes [K/32][rows_pad][4 planes][32] bf16 with planes re_hi, re_lo,
// im_hi, im_lo, rows padded to the 128-row tile and K to the MFMA's 32 with
// zeros.  One (row, 32-k chunk) is 256 contiguous bytes, one 128-row tile of
// a k step is 32 KiB contiguous, so the GEMM streams both operands with
// plain 16-byte coalesced loads and no bounds checks.  The Jacobian's ladder
// and ring operators are split once per set of amplitudes and kept; the
// trial vectors are split per product.
#include "internal.h"

namespace {
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned u4v __attribute__((ext_vector_type(4)));

constexpr int TB = 128;  // tile rows of both operands
constexpr int RS = 17;   // LDS row stride in 16-byte units (16 + 1 pad: conflict-free row-parallel reads)

// round-to-nearest-even bf16 bits of a finite float
__device__ __forceinline__ unsigned bf16_bits(float x) {
  const unsigned u = __float_as_uint(x);
  return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}

__device__ __forceinline__ void split2(double x, unsigned& hi, unsigned& lo) {
  hi = bf16_bits((float)x);
  lo = bf16_bits((float)(x - (double)__uint_as_float(hi << 16)));
}

// One thread writes the 8 k values [kc*32 + g*8, +8) of one row in all four
// planes.  rows_fast selects the thread order that keeps the source reads
// coalesced (rows contiguous in memory) versus k contiguous.
__global__ __launch_bounds__(256) void k_split_bf16(int rows, int K, const cplx* __restrict__ src, i64 sR, i64 sK,
                                                    int conj, u4v* __restrict__ dst, int rows_pad, int nkc,
                                                    int rows_fast) {
  const i64 units = (i64)rows_pad * nkc * 4;
  const double si = conj ? -1.0 : 1.0;
  for (i64 u = blockIdx.x * (i64)blockDim.x + threadIdx.x; u < units; u += (i64)gridDim.x * blockDim.x) {
    i64 r, g, kc;
    if (rows_fast) {
      r = u % rows_pad;
      const i64 q = u / rows_pad;
      g = q & 3;
      kc = q >> 2;
    } else {
      g = u & 3;
      const i64 q = u >> 2;
      r = q % rows_pad;
      kc = q / rows_pad;
    }
    u4v w[4];
#pragma unroll
    for (int e = 0; e < 8; e += 2) {
      unsigned h[2][4];  // [element][plane]
#pragma unroll
      for (int d = 0; d < 2; ++d) {
        const i64 k = kc * 32 + g * 8 + e + d;
        cplx x = make_double2(0.0, 0.0);
        if (r < rows && k < K) x = src[r * sR + k * sK];
        split2(x.x, h[d][0], h[d][1]);
        split2(si * x.y, h[d][2], h[d][3]);
      }
#pragma unroll
      for (int p = 0; p < 4; ++p) w[p][e >> 1] = h[0][p] | (h[1][p] << 16);
    }
    u4v* o = dst + (kc * rows_pad + r) * 16 + g;
#pragma unroll
    for (int p = 0; p < 4; ++p) o[p * 4] = w[p];
  }
}

__device__ __forceinline__ bf8 as_bf8(u4v x) { return __builtin_bit_cast(bf8, x); }
__device__ __forceinline__ bf8 neg_bf8(u4v x) { return __builtin_bit_cast(bf8, x ^ 0x80008000u); }

#define MF(a, b, c) __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0)

// C[m][n] (+)= alpha * sum_k A[m][k] B[n][k] on split operands.  128x128
// tile per workgroup, NWM x NWN waves each owning a (128/NWM) x (128/NWN)
// sub-tile of 16x16 MFMA blocks, double-buffered LDS fed from registers.
// Workgroups are numbered so that each XCD (workgroups are dealt to the 8
// XCDs round-robin) walks a contiguous range of tiles, m fastest: the B tile
// of a step is shared by the workgroups of one XCD and its L2.
template <int NWM, int NWN>
__global__ __launch_bounds__(64 * NWM * NWN) void k_cgemm_bf16x3(const u4v* __restrict__ As, const u4v* __restrict__ Bs,
                                                                 int Mpad, int Npad, int nkc, int M, int N,
                                                                 cplx* __restrict__ C, i64 sCm, i64 sCn, double ar,
                                                                 double ai, int beta, int Mt, int T) {
  constexpr int NT = 64 * NWM * NWN;       // threads
  constexpr int WM = TB / NWM, WN = TB / NWN;
  constexpr int FM = WM / 16, FN = WN / 16;
  constexpr int LQ = TB * 16 / NT;          // 16-byte chunks per thread per operand and k step
  __shared__ u4v sA[2][TB * RS];
  __shared__ u4v sB[2][TB * RS];
  const int per = gridDim.x >> 3;
  const int t = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
  if (t >= T) return;
  const int m0 = (t % Mt) * TB, n0 = (t / Mt) * TB;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave % NWM) * WM, wn = (wave / NWM) * WN;
  const int rr = lane & 15, g = lane >> 4;
  u4v pa[LQ], pb[LQ];
  auto gload = [&](int kc) {
    const u4v* a = As + ((i64)kc * Mpad + m0) * 16;
    const u4v* b = Bs + ((i64)kc * Npad + n0) * 16;
#pragma unroll
    for (int q = 0; q < LQ; ++q) {
      pa[q] = a[tid + q * NT];
      pb[q] = b[tid + q * NT];
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int q = 0; q < LQ; ++q) {
      const int e = tid + q * NT;
      sA[buf][(e >> 4) * RS + (e & 15)] = pa[q];
      sB[buf][(e >> 4) * RS + (e & 15)] = pb[q];
    }
  };
  f4 cr[FM][FN], ci[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      cr[i][j] = f4{0.f, 0.f, 0.f, 0.f};
      ci[i][j] = f4{0.f, 0.f, 0.f, 0.f};
    }
  gload(0);
  sstore(0);
  __syncthreads();
  int buf = 0;
  for (int kc = 0; kc < nkc; ++kc) {
    const bool more = kc + 1 < nkc;
    if (more) gload(kc + 1);
    bf8 b[FN][4];  // [j][plane]
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int p = 0; p < 4; ++p) b[j][p] = as_bf8(sB[buf][(wn + 16 * j + rr) * RS + p * 4 + g]);
#pragma unroll
    for (int i = 0; i < FM; ++i) {
      u4v a[4];
#pragma unroll
      for (int p = 0; p < 4; ++p) a[p] = sA[buf][(wm + 16 * i + rr) * RS + p * 4 + g];
      const bf8 arh = as_bf8(a[0]), arl = as_bf8(a[1]), aih = as_bf8(a[2]), ail = as_bf8(a[3]);
      const bf8 naih = neg_bf8(a[2]), nail = neg_bf8(a[3]);
      // small terms first
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        cr[i][j] = MF(arl, b[j][0], cr[i][j]);
        ci[i][j] = MF(arl, b[j][2], ci[i][j]);
      }
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        cr[i][j] = MF(arh, b[j][1], cr[i][j]);
        ci[i][j] = MF(arh, b[j][3], ci[i][j]);
      }
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        cr[i][j] = MF(nail, b[j][2], cr[i][j]);
        ci[i][j] = MF(ail, b[j][0], ci[i][j]);
      }
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        cr[i][j] = MF(naih, b[j][3], cr[i][j]);
        ci[i][j] = MF(aih, b[j][1], ci[i][j]);
      }
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        cr[i][j] = MF(arh, b[j][0], cr[i][j]);
        ci[i][j] = MF(arh, b[j][2], ci[i][j]);
      }
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        cr[i][j] = MF(naih, b[j][2], cr[i][j]);
        ci[i][j] = MF(aih, b[j][0], ci[i][j]);
      }
    }
    if (more) sstore(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  // output block (i, j): row 16i + 4*(lane/16) + r, column 16j + lane%16
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm + 16 * i + 4 * g + r;
        const int n = n0 + wn + 16 * j + rr;
        if (m < M && n < N) {
          const double xr = (double)cr[i][j][r], xi = (double)ci[i][j][r];
          cplx y = make_double2(ar * xr - ai * xi, ar * xi + ai * xr);
          cplx* dst = C + (i64)m * sCm + (i64)n * sCn;
          if (beta) {
            const cplx o = *dst;
            y.x += o.x;
            y.y += o.y;
          }
          *dst = y;
        }
      }
}
#undef MF
}  // namespace

SplitMat split_shape(int rows, int K) {
  SplitMat s;
  s.rows = rows;
  s.K = K;
  s.rows_pad = (rows + TB - 1) / TB * TB;
  s.nkc = (K + 31) / 32;
  return s;
}

size_t split_bytes(int rows, int K) {
  const SplitMat s = split_shape(rows, K);
  return (size_t)s.rows_pad * (size_t)s.nkc * 256;
}

SplitMat launch_split_bf16(int rows, int K, const cplx* src, i64 sR, i64 sK, int conj, void* dst, hipStream_t st) {
  REQUIRE(rows > 0 && K > 0, CCLR_EINVAL, "split: empty operand");
  SplitMat s = split_shape(rows, K);
  s.p = dst;
  const i64 units = (i64)s.rows_pad * s.nkc * 4;
  i64 grid = (units + 255) / 256;
  if (grid > 65536) grid = 65536;
  hipLaunchKernelGGL(k_split_bf16, dim3((unsigned)grid), dim3(256), 0, st, rows, K, src, sR, sK, conj, (u4v*)dst,
                     s.rows_pad, s.nkc, sR == 1 ? 1 : 0);
  HIPCHK(hipGetLastError());
  return s;
}

void launch_cgemm_bf16x3(const SplitMat& A, const SplitMat& B, cplx* C, i64 sCm, i64 sCn, double ar, double ai,
                         int beta, hipStream_t st, int variant) {
  REQUIRE(A.K == B.K && A.nkc == B.nkc, CCLR_EINVAL, "split GEMM: operands differ in K");
  REQUIRE(A.p && B.p, CCLR_EINVAL, "split GEMM: operand not split");
  const int Mt = A.rows_pad / TB, Nt = B.rows_pad / TB;
  const i64 T = (i64)Mt * Nt;
  REQUIRE(T < (i64)1 << 30, CCLR_EINVAL, "split GEMM: too many tiles");
  const i64 grid = (T + 7) / 8 * 8;
  if (variant == 1)
    hipLaunchKernelGGL((k_cgemm_bf16x3<2, 4>), dim3((unsigned)grid), dim3(512), 0, st, (const u4v*)A.p,
                       (const u4v*)B.p, A.rows_pad, B.rows_pad, A.nkc, A.rows, B.rows, C, sCm, sCn, ar, ai, beta, Mt,
                       (int)T);
  else
    hipLaunchKernelGGL((k_cgemm_bf16x3<2, 2>), dim3((unsigned)grid), dim3(256), 0, st, (const u4v*)A.p,
                       (const u4v*)B.p, A.rows_pad, B.rows_pad, A.nkc, A.rows, B.rows, C, sCm, sCn, ar, ai, beta, Mt,
                       (int)T);
  HIPCHK(hipGetLastError());
}
