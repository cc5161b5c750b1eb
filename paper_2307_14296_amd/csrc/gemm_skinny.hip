// Complex products with a short output side (at most 16 columns) on FP64
// VALU.  The MFMA tiles of the GEMM kernels are 64 or 128 columns wide, so
// a product with 1 or 12 columns executes several times its work
// on padding; here one thread owns one row of C and keeps all of its columns
// in registers, so every element of the long operand is read from HBM once
// and used for every column.  The short operand is staged through LDS in
// K-tiles and read back as a broadcast.  Rows run along the unit-stride
// index of the long operand (the product is transposed when that index is
// n), so the loads of a wave are contiguous.  Long
// reductions are split into chunks whose partial sums go to a workspace
// that a second kernel sums in a fixed order.  A second kernel covers the
// other layout of the long operand (rows contiguous in k, at most 8 output
// columns): the threads of a workgroup run along k and their partial sums
// are added at the end.  At 20 columns the broadcast
// reads of the short operand from LDS already cost more than the padding of
// the MFMA tiles (measured), so products wider than 16 stay on MFMA.
#include <algorithm>

#include "internal.h"

namespace {
constexpr int SN_THREADS = 256;
constexpr int SN_KT = 16;      // K values per LDS tile (and A values in flight per thread)
constexpr int SN_MAXN = 16;

__device__ __forceinline__ i64 skn_off(const GemmArgs& g, i64 bz, i64 s1, i64 s2) {
  if (g.nb2 <= 1) return bz * s1;
  return (bz / g.nb2) * s1 + (bz % g.nb2) * s2;
}

// C[m][n] (+)= alpha * sum_k op(A)[m][k] op(B)[k][n] for n < N <= NS, with
// sAm = 1.  blockIdx = (row block, K chunk q, batch).  With S > 1 chunk
// q of kc reduction indices writes its raw sums to W[(b*S + q)][m][n].
template <int NS>
__global__ __launch_bounds__(SN_THREADS) void k_zgemm_skinny(GemmArgs g, int kc, int S, cplx* W) {
  __shared__ cplx sB[SN_KT][NS];
  const i64 bz = blockIdx.z;
  const int q = blockIdx.y;
  const int m = blockIdx.x * SN_THREADS + threadIdx.x;
  const bool live = m < g.M;
  const cplx* __restrict__ A = g.A + skn_off(g, bz, g.sAb, g.sAb2) + (live ? m : 0);
  const cplx* __restrict__ B = g.B + skn_off(g, bz, g.sBb, g.sBb2);
  const double sa = g.conjA ? -1.0 : 1.0, sb = g.conjB ? -1.0 : 1.0;
  const int k0 = q * kc, k1 = min(g.K, k0 + kc);
  double accr[NS], acci[NS];
#pragma unroll
  for (int n = 0; n < NS; ++n) accr[n] = acci[n] = 0.0;
  for (int kb = k0; kb < k1; kb += SN_KT) {
    const int kt = min(SN_KT, k1 - kb);
    // this thread's A values of the tile, issued before the barrier so they are in flight meanwhile
    cplx a[SN_KT];
#pragma unroll
    for (int kk = 0; kk < SN_KT; ++kk) {
      a[kk] = make_double2(0.0, 0.0);
      if (live && kk < kt) a[kk] = A[(i64)(kb + kk) * g.sAk];
    }
    __syncthreads();  // the previous tile of sB has been consumed
    for (int e = threadIdx.x; e < SN_KT * NS; e += SN_THREADS) {
      const int kk = e / NS, n = e % NS;
      cplx x = make_double2(0.0, 0.0);
      if (kk < kt && n < g.N) {
        x = B[(i64)(kb + kk) * g.sBk + (i64)n * g.sBn];
        x.y *= sb;
      }
      sB[kk][n] = x;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < SN_KT; ++kk) {
      const double ar = a[kk].x, ai = sa * a[kk].y;
#pragma unroll
      for (int n = 0; n < NS; ++n) {
        const cplx b = sB[kk][n];
        accr[n] += ar * b.x - ai * b.y;
        acci[n] += ar * b.y + ai * b.x;
      }
    }
  }
  if (!live) return;
  if (S > 1) {
    cplx* w = W + ((bz * S + q) * (i64)g.M + m) * g.N;
#pragma unroll
    for (int n = 0; n < NS; ++n)
      if (n < g.N) w[n] = make_double2(accr[n], acci[n]);
    return;
  }
  cplx* C = g.C + skn_off(g, bz, g.sCb, g.sCb2) + (i64)m * g.sCm;
#pragma unroll
  for (int n = 0; n < NS; ++n) {
    if (n >= g.N) break;
    cplx y = make_double2(g.ar * accr[n] - g.ai * acci[n], g.ar * acci[n] + g.ai * accr[n]);
    cplx* dst = C + (i64)n * g.sCn;
    if (g.beta) {
      const cplx o = *dst;
      y.x += o.x;
      y.y += o.y;
    }
    *dst = y;
  }
}
// C[m][n] (+)= alpha * sum_k op(A)[m][k] op(B)[k][n] for n < N <= NS, with
// sAk = 1 (the long operand's rows are contiguous in k).  A workgroup owns R
// rows (and, with S > 1, chunk q of kc reduction indices, raw sums to
// W[(b*S + q)][m][n]); thread t sums k = k0 + t, k0 + t + 256, ..., so each
// load of A by a wave is 1 KiB contiguous and every element of A is read
// once; the NS values of B at k are read once for the R rows.  The 256
// partial sums of each (row, column) are added across the lanes of each wave
// and then across the four waves through LDS.
template <int NS, int R>
__global__ __launch_bounds__(256) void k_zgemm_rowdot(GemmArgs g, int kc, int S, cplx* W) {
  __shared__ cplx red[4][R][NS];
  const i64 bz = blockIdx.z;
  const int q = blockIdx.y;
  const int m0 = blockIdx.x * R;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const cplx* __restrict__ A = g.A + skn_off(g, bz, g.sAb, g.sAb2);
  const cplx* __restrict__ B = g.B + skn_off(g, bz, g.sBb, g.sBb2);
  const double sa = g.conjA ? -1.0 : 1.0, sb = g.conjB ? -1.0 : 1.0;
  const int k0 = q * kc, k1 = min(g.K, k0 + kc);
  // rows past the end read the last row (always in bounds) and are not stored
  const cplx* __restrict__ arow[R];
#pragma unroll
  for (int r = 0; r < R; ++r) arow[r] = A + (i64)min(m0 + r, g.M - 1) * g.sAm;
  double accr[R][NS], acci[R][NS];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int n = 0; n < NS; ++n) accr[r][n] = acci[r][n] = 0.0;
  for (int k = k0 + tid; k < k1; k += 256) {
    cplx a[R], b[NS];
#pragma unroll
    for (int r = 0; r < R; ++r) a[r] = arow[r][k];
#pragma unroll
    for (int n = 0; n < NS; ++n) b[n] = n < g.N ? B[(i64)k * g.sBk + (i64)n * g.sBn] : make_double2(0.0, 0.0);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const double xr = a[r].x, xi = sa * a[r].y;
#pragma unroll
      for (int n = 0; n < NS; ++n) {
        const double yr = b[n].x, yi = sb * b[n].y;
        accr[r][n] += xr * yr - xi * yi;
        acci[r][n] += xr * yi + xi * yr;
      }
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int n = 0; n < NS; ++n) {
      double xr = accr[r][n], xi = acci[r][n];
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) {
        xr += __shfl_xor(xr, off, 64);
        xi += __shfl_xor(xi, off, 64);
      }
      if (lane == 0) red[wave][r][n] = make_double2(xr, xi);
    }
  __syncthreads();
  if (tid >= R * NS) return;
  const int r = tid / NS, n = tid % NS, m = m0 + r;
  if (m >= g.M || n >= g.N) return;
  double xr = 0.0, xi = 0.0;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    xr += red[w][r][n].x;
    xi += red[w][r][n].y;
  }
  if (S > 1) {
    W[((bz * S + q) * (i64)g.M + m) * g.N + n] = make_double2(xr, xi);
    return;
  }
  cplx y = make_double2(g.ar * xr - g.ai * xi, g.ar * xi + g.ai * xr);
  cplx* dst = g.C + skn_off(g, bz, g.sCb, g.sCb2) + (i64)m * g.sCm + (i64)n * g.sCn;
  if (g.beta) {
    const cplx o = *dst;
    y.x += o.x;
    y.y += o.y;
  }
  *dst = y;
}

// C = alpha * (sum of the S chunk sums in W) (+ C): one element per thread, chunks in order
__global__ __launch_bounds__(256) void k_skinny_reduce(GemmArgs g, int S, const cplx* __restrict__ W) {
  const i64 mn = (i64)g.M * g.N, total = mn * g.batch, stride = (i64)gridDim.x * blockDim.x;
  for (i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
    const i64 b = e / mn, r = e % mn;
    double sr = 0.0, si = 0.0;
    for (int q = 0; q < S; ++q) {
      const cplx w = W[(b * S + q) * mn + r];
      sr += w.x;
      si += w.y;
    }
    const i64 m = r / g.N, n = r % g.N;
    cplx y = make_double2(g.ar * sr - g.ai * si, g.ar * si + g.ai * sr);
    cplx* dst = g.C + skn_off(g, b, g.sCb, g.sCb2) + m * g.sCm + n * g.sCn;
    if (g.beta) {
      const cplx o = *dst;
      y.x += o.x;
      y.y += o.y;
    }
    *dst = y;
  }
}
}  // namespace

bool skinny_plan(const GemmArgs& g0, GemmArgs& g, int& kc, int& S) {
  if (g0.kchunk > 0 || g0.M <= 0 || g0.N <= 0 || g0.K <= 0 || g0.batch <= 0) return false;
  // (the stores of C are coalesced when its unit stride is m; otherwise they
  // are a small part of the traffic next to the long operand's loads)
  if (g0.N <= SN_MAXN && g0.M >= 64 && g0.sAm == 1) {
    g = g0;
  } else if (g0.M <= SN_MAXN && g0.N >= 64 && g0.sBn == 1) {
    // C^T = B^T A^T: rows along n
    g = g0;
    g.M = g0.N; g.N = g0.M;
    g.A = g0.B; g.sAb = g0.sBb; g.sAb2 = g0.sBb2; g.sAm = g0.sBn; g.sAk = g0.sBk; g.conjA = g0.conjB;
    g.B = g0.A; g.sBb = g0.sAb; g.sBb2 = g0.sAb2; g.sBk = g0.sAk; g.sBn = g0.sAm; g.conjB = g0.conjA;
    g.sCm = g0.sCn; g.sCn = g0.sCm;
  } else {
    return false;
  }
  const i64 rb = (g.M + SN_THREADS - 1) / SN_THREADS;
  if (rb >= (1ll << 31) || g.batch >= 65536) return false;
  // enough workgroups to keep every CU streaming: split the reduction when the rows alone give too few
  i64 s = 1;
  const i64 blocks = rb * g.batch;
  if (blocks < 2048 && g.K >= 8 * SN_KT)
    s = std::min<i64>((3072 + blocks - 1) / blocks, g.K / (4 * SN_KT));
  // workspace of the partial sums at most 256 MB
  s = std::min<i64>(s, std::max<i64>(1, (i64(1) << 28) / ((i64)sizeof(cplx) * g.batch * g.M * g.N)));
  s = std::max<i64>(s, 1);
  i64 c = (g.K + s - 1) / s;
  c = (c + SN_KT - 1) / SN_KT * SN_KT;
  s = (g.K + c - 1) / c;
  if (s >= 65536) return false;
  kc = (int)c;
  S = (int)s;
  return true;
}

constexpr int RD_MAXN = 8;

bool rowdot_plan(const GemmArgs& g, int& kc, int& S) {
  if (g.kchunk > 0 || g.M < 64 || g.N <= 0 || g.N > RD_MAXN || g.K < 256 || g.batch <= 0 || g.sAk != 1) return false;
  const int R = g.N <= 2 ? 8 : 4;
  const i64 rb = (g.M + R - 1) / R;
  if (rb >= (1ll << 31) || g.batch >= 65536) return false;
  // split the reduction when the row blocks alone give fewer than 1024 workgroups
  const i64 blocks = rb * g.batch;
  i64 s = 1;
  if (blocks < 1024) s = std::min<i64>((1024 + blocks - 1) / blocks, g.K / 1024);
  s = std::min<i64>(s, std::max<i64>(1, (i64(1) << 28) / ((i64)sizeof(cplx) * g.batch * g.M * g.N)));
  s = std::max<i64>(s, 1);
  i64 c = (g.K + s - 1) / s;
  c = (c + 255) / 256 * 256;
  s = (g.K + c - 1) / c;
  if (s >= 65536) return false;
  kc = (int)c;
  S = (int)s;
  return true;
}

void launch_zgemm_rowdot(const GemmArgs& g, int kc, int S, cplx* W, hipStream_t s) {
  REQUIRE(g.N >= 1 && g.N <= RD_MAXN && g.sAk == 1 && g.M >= 1 && S >= 1 && (S == 1 || W != nullptr) &&
              (i64)kc * S >= g.K,
          CCLR_EINVAL, "row-dot product: arguments outside the kernel's contract");
  const int R = g.N <= 2 ? 8 : 4;
  const dim3 grid((unsigned)((g.M + R - 1) / R), (unsigned)S, (unsigned)g.batch);
  if (g.N <= 1) hipLaunchKernelGGL((k_zgemm_rowdot<1, 8>), grid, dim3(256), 0, s, g, kc, S, W);
  else if (g.N <= 2) hipLaunchKernelGGL((k_zgemm_rowdot<2, 8>), grid, dim3(256), 0, s, g, kc, S, W);
  else if (g.N <= 4) hipLaunchKernelGGL((k_zgemm_rowdot<4, 4>), grid, dim3(256), 0, s, g, kc, S, W);
  else hipLaunchKernelGGL((k_zgemm_rowdot<8, 4>), grid, dim3(256), 0, s, g, kc, S, W);
  HIPCHK(hipGetLastError());
  if (S == 1) return;
  const i64 total = (i64)g.batch * g.M * g.N;
  const unsigned rgrid = (unsigned)std::min<i64>((total + 255) / 256, 65536);
  hipLaunchKernelGGL(k_skinny_reduce, dim3(rgrid), dim3(256), 0, s, g, S, W);
  HIPCHK(hipGetLastError());
}

void launch_zgemm_skinny(const GemmArgs& g, int kc, int S, cplx* W, hipStream_t s) {
  REQUIRE(g.N >= 1 && g.N <= SN_MAXN && g.sAm == 1 && S >= 1 && (S == 1 || W != nullptr) &&
              (i64)kc * S >= g.K,
          CCLR_EINVAL, "skinny product: arguments outside the kernel's contract");
  const dim3 grid((unsigned)((g.M + SN_THREADS - 1) / SN_THREADS), (unsigned)S, (unsigned)g.batch);
  // the column count rounded up to an instantiated width (the padding columns cost LDS reads and FMAs)
  if (g.N <= 1) hipLaunchKernelGGL(k_zgemm_skinny<1>, grid, dim3(SN_THREADS), 0, s, g, kc, S, W);
  else if (g.N <= 2) hipLaunchKernelGGL(k_zgemm_skinny<2>, grid, dim3(SN_THREADS), 0, s, g, kc, S, W);
  else if (g.N <= 4) hipLaunchKernelGGL(k_zgemm_skinny<4>, grid, dim3(SN_THREADS), 0, s, g, kc, S, W);
  else if (g.N <= 8) hipLaunchKernelGGL(k_zgemm_skinny<8>, grid, dim3(SN_THREADS), 0, s, g, kc, S, W);
  else if (g.N <= 12) hipLaunchKernelGGL(k_zgemm_skinny<12>, grid, dim3(SN_THREADS), 0, s, g, kc, S, W);
  else hipLaunchKernelGGL(k_zgemm_skinny<16>, grid, dim3(SN_THREADS), 0, s, g, kc, S, W);
  HIPCHK(hipGetLastError());
  if (S == 1) return;
  const i64 total = (i64)g.batch * g.M * g.N;
  const unsigned rgrid = (unsigned)std::min<i64>((total + 255) / 256, 65536);
  hipLaunchKernelGGL(k_skinny_reduce, dim3(rgrid), dim3(256), 0, s, g, S, W);
  HIPCHK(hipGetLastError());
}
