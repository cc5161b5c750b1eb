// Complex GEMM kernels of libcclr for gfx950: FP64 MFMA (three or four real
// products per complex block), FP32 MFMA, the short-reduction VALU form and the split-K reduction.
#include "internal.h"

typedef double d4 __attribute__((ext_vector_type(4)));
// last operand of the FP64 MFMA builtin: on CDNA3/CDNA4 its bits are the
// DGEMM negate modifiers of the A, B and C operands; 1 negates A
constexpr int kNegA = 1;
// output row of v_mfma_f32_16x16x4_f32 for (lane, register)
#define F32_ROW(lane, r) (4 * ((lane) >> 4) + (r))

// --------------------------------------------------------------------------
// Complex GEMM  C[b][m][n] (+)= alpha * sum_k A[b][m][k] * B[b][k][n]
// with arbitrary element strides, lowered to four real FP64 MFMA products
// per 16x16x4 complex block (Re*Re - Im*Im, Re*Im + Im*Re).
// Workgroup tile 64x64 (complex), k-step 16; four waves, each owning a 32x32
// sub-tile as 2x2 MFMA blocks.  v_mfma_f64_16x16x4_f64 operand layout:
// A[i][k] in lane i + 16k, B[k][j] in lane j + 16k, D[i][j] in lane
// j + 16*(i%4), register i/4 (measured on gfx950).
// --------------------------------------------------------------------------
namespace {
constexpr int GBM = 64, GBN = 64, GBK = 16, GPAD = 1;

// complex value with the sign bit of its imaginary part xor-ed with sgn
// (0 or 0x80000000): the conjugate, or the value itself, without arithmetic
__device__ __forceinline__ cplx flip_im(cplx v, unsigned sgn) {
  v.y = __hiloint2double(__double2hiint(v.y) ^ (int)sgn, __double2loint(v.y));
  return v;
}
// element offset of batch bz (one or two batch indices)
__device__ __forceinline__ i64 boff(const GemmArgs& g, i64 bz, i64 s1, i64 s2) {
  if (g.nb2 <= 1) return bz * s1;
  return (bz / g.nb2) * s1 + (bz % g.nb2) * s2;
}

__global__ __launch_bounds__(256) void k_zgemm(GemmArgs g) {
  __shared__ double sAr[GBK][GBM + GPAD], sAi[GBK][GBM + GPAD];
  __shared__ double sBr[GBK][GBN + GPAD], sBi[GBK][GBN + GPAD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.x * GBM, n0 = blockIdx.y * GBN;
  const i64 bz = blockIdx.z;
  int kbeg = 0, kend = g.K;
  i64 bb = bz;  // batch index of the operands (the K chunk is folded into bz when splitting)
  if (g.kchunk > 0) {
    const int ns = (g.K + g.kchunk - 1) / g.kchunk;
    kbeg = (int)(bz % ns) * g.kchunk;
    kend = min(g.K, kbeg + g.kchunk);
    bb = bz / ns;
  }
  const cplx* __restrict__ A = g.A + boff(g, bb, g.sAb, g.sAb2);
  const cplx* __restrict__ B = g.B + boff(g, bb, g.sBb, g.sBb2);
  const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
  const bool a_kfast = (g.sAk == 1);
  const bool b_nfast = (g.sBn == 1);

  d4 accR[2][2], accI[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      accR[i][j] = d4{0, 0, 0, 0};
      accI[i][j] = d4{0, 0, 0, 0};
    }

  for (int k0 = kbeg; k0 < kend; k0 += GBK) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int e = tid + r * 256;
      int mm, kk;
      if (a_kfast) { kk = e % GBK; mm = e / GBK; }
      else { mm = e % GBM; kk = e / GBM; }
      const int gm = m0 + mm, gk = k0 + kk;
      cplx x = make_double2(0.0, 0.0);
      if (gm < g.M && gk < kend) x = A[(i64)gm * g.sAm + (i64)gk * g.sAk];
      sAr[kk][mm] = x.x;
      sAi[kk][mm] = g.conjA ? -x.y : x.y;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int e = tid + r * 256;
      int nn, kk;
      if (b_nfast) { nn = e % GBN; kk = e / GBN; }
      else { kk = e % GBK; nn = e / GBK; }
      const int gn = n0 + nn, gk = k0 + kk;
      cplx x = make_double2(0.0, 0.0);
      if (gn < g.N && gk < kend) x = B[(i64)gk * g.sBk + (i64)gn * g.sBn];
      sBr[kk][nn] = x.x;
      sBi[kk][nn] = g.conjB ? -x.y : x.y;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < GBK; ks += 4) {
      const int kk = ks + (lane >> 4);
      double ar[2], ai[2], br[2], bi[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        ar[i] = sAr[kk][wm + i * 16 + (lane & 15)];
        ai[i] = sAi[kk][wm + i * 16 + (lane & 15)];
        br[i] = sBr[kk][wn + i * 16 + (lane & 15)];
        bi[i] = sBi[kk][wn + i * 16 + (lane & 15)];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          accR[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], br[j], accR[i][j], 0, 0, 0);
          accR[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai[i], bi[j], accR[i][j], 0, 0, 0);
          accI[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], bi[j], accI[i][j], 0, 0, 0);
          accI[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[i], br[j], accI[i][j], 0, 0, 0);
        }
    }
    __syncthreads();
  }
  cplx* __restrict__ C = g.C + boff(g, bz, g.sCb, g.sCb2);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm + i * 16 + 4 * r + (lane >> 4);
        const int n = n0 + wn + j * 16 + (lane & 15);
        if (m < g.M && n < g.N) {
          const double cr = accR[i][j][r], ci = accI[i][j][r];
          cplx y = make_double2(g.ar * cr - g.ai * ci, g.ar * ci + g.ai * cr);
          cplx* dst = C + (i64)m * g.sCm + (i64)n * g.sCn;
          if (g.beta) {
            cplx o = *dst;
            y.x += o.x;
            y.y += o.y;
          }
          *dst = y;
        }
      }
}

// W[b][s][m][n] summed over s in a fixed order into C[b][m][n]
__global__ __launch_bounds__(256) void k_splitk_reduce(int nb, int S, int M, int N, const cplx* __restrict__ W,
                                                       cplx* __restrict__ C, i64 sCb, i64 sCm, i64 sCn, double ar,
                                                       double ai, int beta) {
  const i64 mn = (i64)M * N, total = mn * nb, stride = (i64)gridDim.x * blockDim.x;
  for (i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
    const i64 b = e / mn, r = e % mn;
    double sr = 0.0, si = 0.0;
    for (int q = 0; q < S; ++q) {
      const cplx w = W[(b * S + q) * mn + r];
      sr += w.x;
      si += w.y;
    }
    const i64 m = r / N, n = r % N;
    cplx y = make_double2(ar * sr - ai * si, ar * si + ai * sr);
    cplx* dst = C + b * sCb + m * sCm + n * sCn;
    if (beta) {
      const cplx o = *dst;
      y.x += o.x;
      y.y += o.y;
    }
    *dst = y;
  }
}

// --------------------------------------------------------------------------
// Short reductions (K <= 32): memory-bound products such as the o-index
// terms of the doubles.  FP64 on the vector ALU: the threads of a workgroup
// run along n (coalesced B and C), each keeps its column of B in registers
// and sweeps a block of 32 rows of A held in LDS, four rows at a time, so
// every element of B and C moves once.
// --------------------------------------------------------------------------
constexpr int SK_MAX = 32, SK_MB = 32;

template <int KM>  // an upper bound of K, a multiple of 4 up to 32
__global__ __launch_bounds__(256) void k_zgemm_smallk(GemmArgs g) {
  __shared__ cplx sA[SK_MB][KM];
  const i64 bz = blockIdx.z;
  const int n = blockIdx.x * 256 + threadIdx.x;
  const int m0 = blockIdx.y * SK_MB;
  const cplx* __restrict__ A = g.A + boff(g, bz, g.sAb, g.sAb2);
  const cplx* __restrict__ B = g.B + boff(g, bz, g.sBb, g.sBb2);
  cplx* __restrict__ C = g.C + boff(g, bz, g.sCb, g.sCb2);
  const double sa = g.conjA ? -1.0 : 1.0, sb = g.conjB ? -1.0 : 1.0;
  for (int e = threadIdx.x; e < SK_MB * KM; e += 256) {
    const int mm = e / KM, kk = e % KM;
    cplx x = make_double2(0.0, 0.0);
    if (m0 + mm < g.M && kk < g.K) {
      x = A[(i64)(m0 + mm) * g.sAm + (i64)kk * g.sAk];
      x.y *= sa;
    }
    sA[mm][kk] = x;
  }
  __syncthreads();
  if (n >= g.N) return;
  cplx b[KM];
#pragma unroll
  for (int k = 0; k < KM; ++k) {
    b[k] = make_double2(0.0, 0.0);
    if (k < g.K) {
      b[k] = B[(i64)k * g.sBk + (i64)n * g.sBn];
      b[k].y *= sb;
    }
  }
  // four rows at a time: their C loads are in flight together
  constexpr int R = 4;
  const int mend = min(SK_MB, g.M - m0);
  for (int mm0 = 0; mm0 < mend; mm0 += R) {
    cplx o[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      o[r] = make_double2(0.0, 0.0);
      if (g.beta && mm0 + r < mend) o[r] = C[(i64)(m0 + mm0 + r) * g.sCm + (i64)n * g.sCn];
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (mm0 + r >= mend) break;
      double xr = 0.0, xi = 0.0;
#pragma unroll
      for (int k = 0; k < KM; ++k) {
        const cplx a = sA[mm0 + r][k];
        xr += a.x * b[k].x - a.y * b[k].y;
        xi += a.x * b[k].y + a.y * b[k].x;
      }
      const cplx y = make_double2(g.ar * xr - g.ai * xi + o[r].x, g.ar * xi + g.ai * xr + o[r].y);
      C[(i64)(m0 + mm0 + r) * g.sCm + (i64)n * g.sCn] = y;
    }
  }
}

// --------------------------------------------------------------------------
// Pipelined complex GEMM with three real products per complex block (Gauss):
//   k1 = (Ar + Ai) Br,  k2 = Ar (Bi - Br),  k3 = Ai (Br + Bi),
//   Re C = k1 - k3,     Im C = k1 + k2.
// Same contract as k_zgemm; specialised on the operand layouts (which index
// is unit-stride in A and in B).  The LDS holds the three planes of each
// operand; the next K-tile is fetched into registers while the MFMAs consume
// the current one, and LDS is double buffered so each K-tile costs one
// barrier.  Four waves in a 2x2 arrangement, each owning a (BM/2)x(BN/2)
// sub-tile.
// --------------------------------------------------------------------------
template <int BM, int BN, bool AK, bool BNF, bool G3, bool SB = false>
__device__ __forceinline__ void zgemm_tile(const GemmArgs& g, const int m0, const int n0, const i64 bz) {
  constexpr int BK = 16;
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int FM = WM / 16, FN = WN / 16;
  constexpr int LA = BM * BK / 256, LB = BN * BK / 256;
  // three products: planes Ar, Ai, Ar + Ai and Br, Bi - Br, Br + Bi; four
  // products: interleaved (re, im) pairs, read as one 16-byte LDS access
  constexpr int NP = G3 ? 3 : 1;
  constexpr int EW = G3 ? 1 : 2;  // doubles per LDS element
  // SB: one LDS buffer (two barriers per K-tile) for a smaller footprint and more resident workgroups
  constexpr int NB = SB ? 1 : 2;
  __shared__ double sA[NB][NP][BK][(BM + 1) * EW];
  __shared__ double sB[NB][NP][BK][(BN + 1) * EW];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int kbeg = 0, kend = g.K;
  i64 bb = bz;  // batch index of the operands (the K chunk is folded into bz when splitting)
  if (g.kchunk > 0) {
    const int ns = (g.K + g.kchunk - 1) / g.kchunk;
    kbeg = (int)(bz % ns) * g.kchunk;
    kend = min(g.K, kbeg + g.kchunk);
    bb = bz / ns;
  }
  const cplx* __restrict__ A = g.A + boff(g, bb, g.sAb, g.sAb2);
  const cplx* __restrict__ B = g.B + boff(g, bb, g.sBb, g.sBb2);
  const int wm = (wave & 1) * WM, wn = (wave >> 1) * WN;
  const double sa = g.conjA ? -1.0 : 1.0, sb = g.conjB ? -1.0 : 1.0;
  const unsigned sgnA = g.conjA ? 0x80000000u : 0u, sgnB = g.conjB ? 0x80000000u : 0u;
  const i64 sAk = AK ? 1 : g.sAk, sBn = BNF ? 1 : g.sBn;
  // element r of this thread's share of a K-tile: A row mA + r*dmA, column kA + r*dkA (and alike for B)
  const int mA = AK ? tid / BK : tid % BM, kA = AK ? tid % BK : tid / BM;
  const int dmA = AK ? 256 / BK : 0, dkA = AK ? 0 : 256 / BM;
  const int nB = BNF ? tid % BN : tid / BK, kB = BNF ? tid / BN : tid % BK;
  const int dnB = BNF ? 0 : 256 / BK, dkB = BNF ? 256 / BN : 0;
  const cplx* __restrict__ pA = A + (i64)(m0 + mA) * g.sAm + (i64)kA * sAk;
  const cplx* __restrict__ pB = B + (i64)kB * g.sBk + (i64)(n0 + nB) * sBn;
  const i64 stA = (i64)dmA * g.sAm + (i64)dkA * sAk, stB = (i64)dkB * g.sBk + (i64)dnB * sBn;

  cplx ra[LA], rb[LB];
  auto gload = [&](int k0) {
#pragma unroll
    for (int r = 0; r < LA; ++r) {
      const int gm = m0 + mA + r * dmA, gk = k0 + kA + r * dkA;
      ra[r] = (gm < g.M && gk < kend) ? pA[r * stA + (i64)k0 * sAk] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int r = 0; r < LB; ++r) {
      const int gn = n0 + nB + r * dnB, gk = k0 + kB + r * dkB;
      rb[r] = (gn < g.N && gk < kend) ? pB[r * stB + (i64)k0 * g.sBk] : make_double2(0.0, 0.0);
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int r = 0; r < LA; ++r) {
      const int mm = mA + r * dmA, kk = kA + r * dkA;
      const double re = ra[r].x, im = sa * ra[r].y;
      if (G3) {
        sA[buf][0][kk][mm] = re;
        sA[buf][G3 ? 1 : 0][kk][mm] = im;
        sA[buf][G3 ? 2 : 0][kk][mm] = re + im;
      } else {
        *(double2*)&sA[buf][0][kk][2 * mm] = flip_im(ra[r], sgnA);
      }
    }
#pragma unroll
    for (int r = 0; r < LB; ++r) {
      const int nn = nB + r * dnB, kk = kB + r * dkB;
      const double re = rb[r].x, im = sb * rb[r].y;
      if (G3) {
        sB[buf][0][kk][nn] = re;
        sB[buf][G3 ? 1 : 0][kk][nn] = im - re;
        sB[buf][G3 ? 2 : 0][kk][nn] = re + im;
      } else {
        *(double2*)&sB[buf][0][kk][2 * nn] = flip_im(rb[r], sgnB);
      }
    }
  };

  d4 k1[FM][FN], k2[FM][FN], k3[G3 ? FM : 1][G3 ? FN : 1];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      k1[i][j] = d4{0, 0, 0, 0};
      k2[i][j] = d4{0, 0, 0, 0};
      if (G3) k3[G3 ? i : 0][G3 ? j : 0] = d4{0, 0, 0, 0};
    }

  gload(kbeg);
  sstore(0);
  __syncthreads();
  int buf = 0;
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    const bool more = k0 + BK < kend;
    if (more) gload(k0 + BK);
#pragma unroll(SB ? 2 : 4)
    for (int ks = 0; ks < BK; ks += 4) {
      const int kk = ks + (lane >> 4);
      double ar[FM], ai[FM], as[FM], br[FN], bd[FN], bs[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) {
        const int mm = wm + i * 16 + (lane & 15);
        if (G3) {
          ar[i] = sA[buf][0][kk][mm];
          ai[i] = sA[buf][G3 ? 1 : 0][kk][mm];
          as[i] = sA[buf][G3 ? 2 : 0][kk][mm];
        } else {
          const double2 x = *(const double2*)&sA[buf][0][kk][2 * mm];
          ar[i] = x.x, ai[i] = x.y, as[i] = 0.0;
        }
      }
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const int nn = wn + j * 16 + (lane & 15);
        if (G3) {
          br[j] = sB[buf][0][kk][nn];
          bd[j] = sB[buf][G3 ? 1 : 0][kk][nn];
          bs[j] = sB[buf][G3 ? 2 : 0][kk][nn];
        } else {
          const double2 x = *(const double2*)&sB[buf][0][kk][2 * nn];
          br[j] = x.x, bd[j] = x.y, bs[j] = 0.0;
        }
      }
      if (G3) {
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) {
            k1[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(as[i], br[j], k1[i][j], 0, 0, 0);
            k2[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], bd[j], k2[i][j], 0, 0, 0);
            k3[G3 ? i : 0][G3 ? j : 0] =
                __builtin_amdgcn_mfma_f64_16x16x4f64(ai[i], bs[j], k3[G3 ? i : 0][G3 ? j : 0], 0, 0, 0);
          }
      } else {
        // four products: k1 = Re, k2 = Im  (bd holds Bi here)
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) {
            k1[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], br[j], k1[i][j], 0, 0, 0);
            k2[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], bd[j], k2[i][j], 0, 0, 0);
          }
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) {
            k1[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[i], bd[j], k1[i][j], 0, 0, kNegA);
            k2[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[i], br[j], k2[i][j], 0, 0, 0);
          }
      }
    }
    if (SB) {
      if (more) {
        __syncthreads();  // every wave is done reading the buffer
        sstore(0);
        __syncthreads();
      }
    } else {
      if (more) sstore(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    }
  }
  cplx* __restrict__ C = g.C + boff(g, bz, g.sCb, g.sCb2);
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm + i * 16 + 4 * r + (lane >> 4);
        const int n = n0 + wn + j * 16 + (lane & 15);
        if (m < g.M && n < g.N) {
          const double cr = G3 ? k1[i][j][r] - k3[G3 ? i : 0][G3 ? j : 0][r] : k1[i][j][r];
          const double ci = G3 ? k1[i][j][r] + k2[i][j][r] : k2[i][j][r];
          cplx y = make_double2(g.ar * cr - g.ai * ci, g.ar * ci + g.ai * cr);
          cplx* dst = C + (i64)m * g.sCm + (i64)n * g.sCn;
          if (g.beta) {
            const cplx o = *dst;
            y.x += o.x;
            y.y += o.y;
          }
          *dst = y;
        }
      }
}

// Tile order of the one-dimensional launch.  The hardware deals workgroups
// round-robin over the 8 XCDs (each with its own L2), so workgroup w is
// mapped to a contiguous run of the tile sequence on XCD w % 8.  In the
// sequence the batch index is slowest; inside a batch, groups of gm M-tiles
// sweep the N-tiles with M fastest, so the tiles that run together on one
// XCD share both their B column panels (gm of them per panel) and their A
// row panels (across the N-tiles in flight).
// With xcd = 0 and gm = tm this is the plain order (M fastest, then N, then
// the batch index) in which consecutive tiles land on different XCDs.
__device__ __forceinline__ void tile_of(int w, int T, int tm, int tn, int gm, int xcd, int& mi, int& ni, int& bz) {
  const int x = w & 7, l = w >> 3, per = T >> 3, rem = T & 7;
  const int t = xcd ? (x < rem ? x * (per + 1) : rem * (per + 1) + (x - rem) * per) + l : w;
  const int per_b = tm * tn;
  bz = t / per_b;
  const int r = t - bz * per_b;
  const int grp = r / (gm * tn), within = r - grp * gm * tn;
  const int gme = min(gm, tm - grp * gm);
  mi = grp * gm + within % gme;
  ni = within / gme;
}

template <int BM, int BN, bool AK, bool BNF, bool G3>
__global__ __launch_bounds__(256) void k_zgemm_p(GemmArgs g, int tm, int tn, int gm, int xcd) {
  int mi, ni, bz;
  tile_of((int)blockIdx.x, (int)gridDim.x, tm, tn, gm, xcd, mi, ni, bz);
  zgemm_tile<BM, BN, AK, BNF, G3>(g, mi * BM, ni * BN, bz);
}

// single-buffered LDS, registers capped for three (64-row tiles) or two
// (128-row tiles) waves per SIMD
template <int BM, int BN, bool AK, bool BNF, bool G3>
__global__ __launch_bounds__(256, BM == 64 ? 3 : 2) void k_zgemm_p1(GemmArgs g, int tm, int tn, int gm, int xcd) {
  int mi, ni, bz;
  tile_of((int)blockIdx.x, (int)gridDim.x, tm, tn, gm, xcd, mi, ni, bz);
  zgemm_tile<BM, BN, AK, BNF, G3, true>(g, mi * BM, ni * BN, bz);
}

// --------------------------------------------------------------------------
// Large-tile form: 128x128 tiles, four real products, double-buffered LDS
// (132 KB, so one workgroup per CU) and eight waves (two per SIMD), each
// owning a 64x32 complex sub-tile.  One barrier per K-tile; the operand
// fragments of the next 4-deep K step are read from LDS while the MFMAs of
// the current one run, and the next K-tile is fetched into registers during
// the whole tile.
// --------------------------------------------------------------------------
template <bool AK, bool BNF>
__device__ __forceinline__ void zgemm_tile_w1(const GemmArgs& g, const int m0, const int n0, const i64 bz) {
  constexpr int BM = 128, BN = 128, BK = 16;
  constexpr int NT = 512, WM = 64, WN = 32, FM = WM / 16, FN = WN / 16;
  constexpr int LA = BM * BK / NT, LB = BN * BK / NT;
  __shared__ double sA[2][BK][(BM + 1) * 2];
  __shared__ double sB[2][BK][(BN + 1) * 2];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int kbeg = 0, kend = g.K;
  i64 bb = bz;
  if (g.kchunk > 0) {
    const int ns = (g.K + g.kchunk - 1) / g.kchunk;
    kbeg = (int)(bz % ns) * g.kchunk;
    kend = min(g.K, kbeg + g.kchunk);
    bb = bz / ns;
  }
  const cplx* __restrict__ A = g.A + boff(g, bb, g.sAb, g.sAb2);
  const cplx* __restrict__ B = g.B + boff(g, bb, g.sBb, g.sBb2);
  const int wm = (wave & 1) * WM, wn = (wave >> 1) * WN;
  const unsigned sgnA = g.conjA ? 0x80000000u : 0u, sgnB = g.conjB ? 0x80000000u : 0u;
  const i64 sAk = AK ? 1 : g.sAk, sBn = BNF ? 1 : g.sBn;
  // element r of this thread's share of a K-tile: A row mA + r*dmA, column kA + r*dkA (and alike for B)
  const int mA = AK ? tid / BK : tid % BM, kA = AK ? tid % BK : tid / BM;
  const int dmA = AK ? NT / BK : 0, dkA = AK ? 0 : NT / BM;
  const int nB = BNF ? tid % BN : tid / BK, kB = BNF ? tid / BN : tid % BK;
  const int dnB = BNF ? 0 : NT / BK, dkB = BNF ? NT / BN : 0;
  const cplx* __restrict__ pA = A + (i64)(m0 + mA) * g.sAm + (i64)kA * sAk;
  const cplx* __restrict__ pB = B + (i64)kB * g.sBk + (i64)(n0 + nB) * sBn;
  const i64 stA = (i64)dmA * g.sAm + (i64)dkA * sAk, stB = (i64)dkB * g.sBk + (i64)dnB * sBn;

  cplx ra[LA], rb[LB];
  auto gload = [&](int k0) {
#pragma unroll
    for (int r = 0; r < LA; ++r) {
      const int gm = m0 + mA + r * dmA, gk = k0 + kA + r * dkA;
      ra[r] = (gm < g.M && gk < kend) ? pA[r * stA + (i64)k0 * sAk] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int r = 0; r < LB; ++r) {
      const int gn = n0 + nB + r * dnB, gk = k0 + kB + r * dkB;
      rb[r] = (gn < g.N && gk < kend) ? pB[r * stB + (i64)k0 * g.sBk] : make_double2(0.0, 0.0);
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int r = 0; r < LA; ++r)
      *(double2*)&sA[buf][kA + r * dkA][2 * (mA + r * dmA)] = flip_im(ra[r], sgnA);
#pragma unroll
    for (int r = 0; r < LB; ++r)
      *(double2*)&sB[buf][kB + r * dkB][2 * (nB + r * dnB)] = flip_im(rb[r], sgnB);
  };
  double2 fa[2][FM], fb[2][FN];
  auto fread = [&](int buf, int ks, int s) {
    const int kk = ks + (lane >> 4);
#pragma unroll
    for (int i = 0; i < FM; ++i) fa[s][i] = *(const double2*)&sA[buf][kk][2 * (wm + i * 16 + (lane & 15))];
#pragma unroll
    for (int j = 0; j < FN; ++j) fb[s][j] = *(const double2*)&sB[buf][kk][2 * (wn + j * 16 + (lane & 15))];
  };

  d4 cr[FM][FN], ci[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      cr[i][j] = d4{0, 0, 0, 0};
      ci[i][j] = d4{0, 0, 0, 0};
    }

  gload(kbeg);
  sstore(0);
  __syncthreads();
  int buf = 0;
  fread(0, 0, 0);
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    const bool more = k0 + BK < kend;
    if (more) gload(k0 + BK);
#pragma unroll
    for (int q = 0; q < BK / 4; ++q) {
      const int s = q & 1;
      if (q + 1 < BK / 4) fread(buf, 4 * (q + 1), s ^ 1);
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          cr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[s][i].x, fb[s][j].x, cr[i][j], 0, 0, 0);
          ci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[s][i].x, fb[s][j].y, ci[i][j], 0, 0, 0);
        }
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          cr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[s][i].y, fb[s][j].y, cr[i][j], 0, 0, kNegA);
          ci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[s][i].y, fb[s][j].x, ci[i][j], 0, 0, 0);
        }
    }
    if (more) sstore(buf ^ 1);
    __syncthreads();
    buf ^= 1;
    if (more) fread(buf, 0, 0);
  }
  cplx* __restrict__ C = g.C + boff(g, bz, g.sCb, g.sCb2);
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm + i * 16 + 4 * r + (lane >> 4);
        const int n = n0 + wn + j * 16 + (lane & 15);
        if (m < g.M && n < g.N) {
          const double xr = cr[i][j][r], xi = ci[i][j][r];
          cplx y = make_double2(g.ar * xr - g.ai * xi, g.ar * xi + g.ai * xr);
          cplx* dst = C + (i64)m * g.sCm + (i64)n * g.sCn;
          if (g.beta) {
            const cplx o = *dst;
            y.x += o.x;
            y.y += o.y;
          }
          *dst = y;
        }
      }
}

template <bool AK, bool BNF>
__global__ __launch_bounds__(512, 2) void k_zgemm_w1(GemmArgs g, int tm, int tn, int gm, int xcd) {
  int mi, ni, bz;
  tile_of((int)blockIdx.x, (int)gridDim.x, tm, tn, gm, xcd, mi, ni, bz);
  zgemm_tile_w1<AK, BNF>(g, mi * 128, ni * 128, bz);
}

// grouped persistent form of the 128x128 tile (one workgroup per CU)
template <bool AK, bool BNF>
__global__ __launch_bounds__(512, 2) void k_zgemm_group_w1(const GemmArgs* __restrict__ probs,
                                                          const int* __restrict__ tstart, int nprob, int total) {
  for (int t = blockIdx.x; t < total; t += gridDim.x) {
    int p = 0;
    while (p + 1 < nprob && t >= tstart[p + 1]) ++p;
    const GemmArgs g = probs[p];
    const int lt = t - tstart[p];
    const int tm = (g.M + 127) / 128, tn = (g.N + 127) / 128;
    const int mi = lt % tm, rest = lt / tm;
    zgemm_tile_w1<AK, BNF>(g, mi * 128, (rest % tn) * 128, rest / tn);
  }
}

// --------------------------------------------------------------------------
// 128x128 (or 64x256) four-product tile whose operand tiles go from HBM to LDS by direct
// loads (global_load_lds_dwordx4: each lane names one 16-byte complex element,
// the wave's 64 elements land as one contiguous KiB of LDS), so no register
// staging, no LDS stores and no wait for the global loads sit in the K loop.
// Each 16-deep K tile of an operand is 32 KiB in one of two layouts:
//  * unit-stride k (the operand rows hold consecutive k): [row][16 slots],
//    element k of a row in slot k ^ (row mod 16), so the 16 lanes that read
//    one k of 16 consecutive rows hit 16 different bank groups and the 16
//    lanes that load a row read its 256 contiguous bytes;
//  * unit-stride rows: [k][128 rows], rows contiguous in both places.
// Two stages in separate LDS arrays (128 KiB, one workgroup per CU, eight
// waves of 64x32): each K tile first requests the next tile's loads into the
// idle stage, then runs its MFMAs; the wait for the loads and the barrier sit
// before its last K step.
// Rows beyond the operand are clamped to its last row (their outputs are not
// stored); a K remainder below 16 goes through registers with zero fill.
// Conjugation flips the sign of the imaginary part of each operand fragment
// (a separate instantiation, so products without it carry no flips).
// --------------------------------------------------------------------------
// row and k of this lane's element of 1 KiB chunk c of an operand tile of R rows
template <bool KC, int R>
__device__ __forceinline__ int dma_row(int c, int lane) {
  return KC ? 4 * c + (lane >> 4) : (c % (R / 64)) * 64 + lane;
}
template <bool KC, int R>
__device__ __forceinline__ int dma_k(int c, int lane) {
  return KC ? (lane & 15) ^ ((4 * c + (lane >> 4)) & 15) : c / (R / 64);
}
__device__ __forceinline__ void dma16(const cplx* src, cplx* lds) {
  __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)src,
                                   (__attribute__((address_space(3))) void*)lds, 16, 0, 0);
}

// tile shapes: BM x BN with eight waves of 64 x 32 (BM = 128: 2 x 4 waves,
// BN = 128; BM = 64: 1 x 8 waves, BN = 256, for products with few rows)
template <int BM>
struct DmaShape {
  static constexpr int WAVES_M = BM / 64, WAVES_N = 8 / WAVES_M, BN = WAVES_N * 32;
  static constexpr int TA = BM * 16, TB = BN * 16;  // complex elements per operand tile and stage
};

template <int BM, bool AK, bool BNF, bool CJ>
__device__ __forceinline__ void zgemm_tile_dma(const GemmArgs& g, const int m0, const int n0, const i64 bz,
                                               cplx* sA0, cplx* sA1, cplx* sB0, cplx* sB1) {
  using SH = DmaShape<BM>;
  constexpr int BN = SH::BN, BK = 16, WM = 64, WN = 32, FM = WM / 16, FN = WN / 16;
  constexpr int JA = BM / 32, JB = BN / 32;  // 1 KiB chunks per wave and stage (of BM / 4 and BN / 4)
  constexpr bool KCA = AK, KCB = !BNF;  // which operands have unit-stride k
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int kbeg = 0, kend = g.K;
  i64 bb = bz;
  if (g.kchunk > 0) {
    const int ns = (g.K + g.kchunk - 1) / g.kchunk;
    kbeg = (int)(bz % ns) * g.kchunk;
    kend = min(g.K, kbeg + g.kchunk);
    bb = bz / ns;
  }
  const cplx* __restrict__ A = g.A + boff(g, bb, g.sAb, g.sAb2);
  const cplx* __restrict__ B = g.B + boff(g, bb, g.sBb, g.sBb2);
  const int wm = (wave % SH::WAVES_M) * WM, wn = (wave / SH::WAVES_M) * WN;
  const unsigned sgnA = g.conjA ? 0x80000000u : 0u, sgnB = g.conjB ? 0x80000000u : 0u;
  const int nfull = (kend - kbeg) / BK, tail = kend - kbeg - nfull * BK;
  // this lane's element of each of its 1 KiB chunks (chunk c = 8 j + wave) of a K tile
  const cplx* pa[JA];
  const cplx* pb[JB];
#pragma unroll
  for (int j = 0; j < JA; ++j) {
    const int c = 8 * j + wave;
    const int ra = min(m0 + dma_row<KCA, BM>(c, lane), g.M - 1);
    pa[j] = A + (i64)ra * g.sAm + (i64)(kbeg + dma_k<KCA, BM>(c, lane)) * g.sAk;
  }
#pragma unroll
  for (int j = 0; j < JB; ++j) {
    const int c = 8 * j + wave;
    const int rb = min(n0 + dma_row<KCB, BN>(c, lane), g.N - 1);
    pb[j] = B + (i64)rb * g.sBn + (i64)(kbeg + dma_k<KCB, BN>(c, lane)) * g.sBk;
  }
  const i64 dA = (i64)BK * g.sAk, dB = (i64)BK * g.sBk;
  auto fetch = [&](int t, cplx* la, cplx* lb) {
#pragma unroll
    for (int j = 0; j < JA; ++j) dma16(pa[j] + t * dA, la + 64 * (8 * j + wave));
#pragma unroll
    for (int j = 0; j < JB; ++j) dma16(pb[j] + t * dB, lb + 64 * (8 * j + wave));
  };
  // LDS element of this lane's fragment of K step q (k = 4q + lane/16) in block i (A) or j (B)
  const int rr = lane & 15, gq = lane >> 4;
  auto offa = [&](int q, int i) {
    return KCA ? (wm + 16 * i + rr) * BK + ((4 * q + gq) ^ rr) : (4 * q + gq) * BM + wm + 16 * i + rr;
  };
  auto offb = [&](int q, int j) {
    return KCB ? (wn + 16 * j + rr) * BK + ((4 * q + gq) ^ rr) : (4 * q + gq) * BN + wn + 16 * j + rr;
  };
  d4 cr[FM][FN], ci[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      cr[i][j] = d4{0, 0, 0, 0};
      ci[i][j] = d4{0, 0, 0, 0};
    }
  double2 fa[2][FM], fb[2][FN];
  auto fread = [&](const cplx* la, const cplx* lb, int q, int s) {
#pragma unroll
    for (int i = 0; i < FM; ++i) fa[s][i] = CJ ? flip_im(la[offa(q, i)], sgnA) : la[offa(q, i)];
#pragma unroll
    for (int j = 0; j < FN; ++j) fb[s][j] = CJ ? flip_im(lb[offb(q, j)], sgnB) : lb[offb(q, j)];
  };
  // the 32 MFMAs of one 4-deep K step on the fragments in slot s
  auto mfma_q = [&](int s) {
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        cr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[s][i].x, fb[s][j].x, cr[i][j], 0, 0, 0);
        ci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[s][i].x, fb[s][j].y, ci[i][j], 0, 0, 0);
      }
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        cr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[s][i].y, fb[s][j].y, cr[i][j], 0, 0, kNegA);
        ci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[s][i].y, fb[s][j].x, ci[i][j], 0, 0, 0);
      }
  };
  // a whole K tile on one stage, its first fragments read here
  auto compute = [&](const cplx* la, const cplx* lb) {
    fread(la, lb, 0, 0);
#pragma unroll
    for (int q = 0; q < BK / 4; ++q) {
      const int s = q & 1;
      if (q + 1 < BK / 4) fread(la, lb, q + 1, s ^ 1);
      mfma_q(s);
    }
  };
  // one K tile on stage (ca, cb) while tile t + 1 loads into (na, nb); the
  // last tile reloads itself into the idle stage (no branch around the loads).
  // The tile's first fragments are already in slot 0.  The wait for the loads
  // and the barrier come once the last K step's fragments are in registers,
  // so the next tile's first fragments are read while that step's MFMAs run
  // (2% faster than a barrier after the last MFMA).
  auto step = [&](int t, const cplx* ca, const cplx* cb, cplx* na, cplx* nb) {
    fetch(t + 1 < nfull ? t + 1 : t, na, nb);
    __builtin_amdgcn_sched_barrier(0);
    fread(ca, cb, 1, 1);
    mfma_q(0);
    fread(ca, cb, 2, 0);
    mfma_q(1);
    fread(ca, cb, 3, 1);
    mfma_q(0);
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    fread(na, nb, 0, 0);
    mfma_q(1);
  };
  if (nfull > 0) {
    fetch(0, sA0, sB0);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    fread(sA0, sB0, 0, 0);
    for (int t = 0; t < nfull; t += 2) {
      step(t, sA0, sB0, sA1, sB1);
      if (t + 1 < nfull) step(t + 1, sA1, sB1, sA0, sB0);
    }
    __syncthreads();  // every wave is done reading the stages before the remainder overwrites one
  }
  if (tail > 0) {  // K remainder: through registers, zero beyond kend (both stages are idle here)
    const cplx z = make_double2(0.0, 0.0);
#pragma unroll
    for (int j = 0; j < JA; ++j) {
      const int c = 8 * j + wave;
      sA0[64 * c + lane] = dma_k<KCA, BM>(c, lane) < tail ? pa[j][nfull * dA] : z;
    }
#pragma unroll
    for (int j = 0; j < JB; ++j) {
      const int c = 8 * j + wave;
      sB0[64 * c + lane] = dma_k<KCB, BN>(c, lane) < tail ? pb[j][nfull * dB] : z;
    }
    __syncthreads();
    compute(sA0, sB0);
  }
  cplx* __restrict__ C = g.C + boff(g, bz, g.sCb, g.sCb2);
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm + i * 16 + 4 * r + (lane >> 4);
        const int n = n0 + wn + j * 16 + (lane & 15);
        if (m < g.M && n < g.N) {
          const double xr = cr[i][j][r], xi = ci[i][j][r];
          cplx y = make_double2(g.ar * xr - g.ai * xi, g.ar * xi + g.ai * xr);
          cplx* dst = C + (i64)m * g.sCm + (i64)n * g.sCn;
          if (g.beta) {
            const cplx o = *dst;
            y.x += o.x;
            y.y += o.y;
          }
          *dst = y;
        }
      }
}

template <int BM, bool AK, bool BNF>
__global__ __launch_bounds__(512, 2) void k_zgemm_dma(GemmArgs g, int tm, int tn, int gm, int xcd) {
  using SH = DmaShape<BM>;
  int mi, ni, bz;
  // the two stages of each operand are separate arrays, so the compiler knows
  // that reads of one stage do not depend on the direct loads into the other
  __shared__ cplx sA0[SH::TA], sA1[SH::TA], sB0[SH::TB], sB1[SH::TB];
  tile_of((int)blockIdx.x, (int)gridDim.x, tm, tn, gm, xcd, mi, ni, bz);
  if (g.conjA || g.conjB) zgemm_tile_dma<BM, AK, BNF, true>(g, mi * BM, ni * SH::BN, bz, sA0, sA1, sB0, sB1);
  else zgemm_tile_dma<BM, AK, BNF, false>(g, mi * BM, ni * SH::BN, bz, sA0, sA1, sB0, sB1);
}

// grouped persistent form of the direct-load tile (one workgroup per CU); the
// barrier ahead of each tile keeps its first loads from overwriting a stage
// that another wave still reads for the previous tile
template <bool AK, bool BNF>
__global__ __launch_bounds__(512, 2) void k_zgemm_group_dma(const GemmArgs* __restrict__ probs,
                                                           const int* __restrict__ tstart, int nprob, int total) {
  __shared__ cplx sA0[DmaShape<128>::TA], sA1[DmaShape<128>::TA], sB0[DmaShape<128>::TB], sB1[DmaShape<128>::TB];
  for (int t = blockIdx.x; t < total; t += gridDim.x) {
    int p = 0;
    while (p + 1 < nprob && t >= tstart[p + 1]) ++p;
    const GemmArgs g = probs[p];
    const int lt = t - tstart[p];
    const int tm = (g.M + 127) / 128, tn = (g.N + 127) / 128;
    const int mi = lt % tm, rest = lt / tm;
    __syncthreads();
    if (g.conjA || g.conjB)
      zgemm_tile_dma<128, AK, BNF, true>(g, mi * 128, (rest % tn) * 128, rest / tn, sA0, sA1, sB0, sB1);
    else
      zgemm_tile_dma<128, AK, BNF, false>(g, mi * 128, (rest % tn) * 128, rest / tn, sA0, sA1, sB0, sB1);
  }
}

// Grouped persistent form: one launch walks the tiles of several products
// (problem p owns tiles [tstart[p], tstart[p+1])), each workgroup taking
// every gridDim.x-th tile.  The LDS of a tile is released by the barrier
// that ends its last K step, so consecutive tiles reuse it safely.
template <int BM, int BN, bool AK, bool BNF, bool G3>
__global__ __launch_bounds__(256) void k_zgemm_group(const GemmArgs* __restrict__ probs, const int* __restrict__ tstart,
                                                     int nprob, int total) {
  for (int t = blockIdx.x; t < total; t += gridDim.x) {
    int p = 0;
    while (p + 1 < nprob && t >= tstart[p + 1]) ++p;
    const GemmArgs g = probs[p];
    const int lt = t - tstart[p];
    const int tm = (g.M + BM - 1) / BM, tn = (g.N + BN - 1) / BN;
    const int mi = lt % tm, rest = lt / tm;
    zgemm_tile<BM, BN, AK, BNF, G3>(g, mi * BM, (rest % tn) * BN, rest / tn);
  }
}

// --------------------------------------------------------------------------
// Low-precision complex GEMM: operands and C are complex128 in memory, the
// products run on FP32 MFMA (v_mfma_f32_16x16x4_f32) with FP32 accumulation,
// three real products per complex block as in k_zgemm_p.  Used for the
// ladder and ring products inside the inner solves of the mixed-precision
// path; residuals are always re-formed with the FP64 kernels.
// --------------------------------------------------------------------------
typedef float f4 __attribute__((ext_vector_type(4)));

// row of the 16x16 f32 MFMA output held by lane `lane` in register r
__device__ __forceinline__ int f32_out_row(int lane, int r) { return F32_ROW(lane, r); }

template <int BM, int BN, bool AK, bool BNF>
__global__ __launch_bounds__(256) void k_cgemm_f32(GemmArgs g) {
  constexpr int BK = 16;
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int FM = WM / 16, FN = WN / 16;
  constexpr int LA = BM * BK / 256, LB = BN * BK / 256;
  __shared__ float sA[2][3][BK][BM + 1];
  __shared__ float sB[2][3][BK][BN + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
  const i64 bz = blockIdx.z;
  int kbeg = 0, kend = g.K;
  i64 bb = bz;  // batch index of the operands (the K chunk is folded into bz when splitting)
  if (g.kchunk > 0) {
    const int ns = (g.K + g.kchunk - 1) / g.kchunk;
    kbeg = (int)(bz % ns) * g.kchunk;
    kend = min(g.K, kbeg + g.kchunk);
    bb = bz / ns;
  }
  const cplx* __restrict__ A = g.A + boff(g, bb, g.sAb, g.sAb2);
  const cplx* __restrict__ B = g.B + boff(g, bb, g.sBb, g.sBb2);
  const int wm = (wave & 1) * WM, wn = (wave >> 1) * WN;
  const float sa = g.conjA ? -1.f : 1.f, sb = g.conjB ? -1.f : 1.f;
  cplx ra[LA], rb[LB];
  auto gload = [&](int k0) {
#pragma unroll
    for (int r = 0; r < LA; ++r) {
      const int e = tid + r * 256;
      const int mm = AK ? e / BK : e % BM;
      const int kk = AK ? e % BK : e / BM;
      const int gm = m0 + mm, gk = k0 + kk;
      ra[r] = (gm < g.M && gk < kend) ? A[(i64)gm * g.sAm + (i64)gk * g.sAk] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int r = 0; r < LB; ++r) {
      const int e = tid + r * 256;
      const int nn = BNF ? e % BN : e / BK;
      const int kk = BNF ? e / BN : e % BK;
      const int gn = n0 + nn, gk = k0 + kk;
      rb[r] = (gn < g.N && gk < kend) ? B[(i64)gk * g.sBk + (i64)gn * g.sBn] : make_double2(0.0, 0.0);
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int r = 0; r < LA; ++r) {
      const int e = tid + r * 256;
      const int mm = AK ? e / BK : e % BM;
      const int kk = AK ? e % BK : e / BM;
      const float re = (float)ra[r].x, im = sa * (float)ra[r].y;
      sA[buf][0][kk][mm] = re;
      sA[buf][1][kk][mm] = im;
      sA[buf][2][kk][mm] = (float)(ra[r].x + (double)sa * ra[r].y);
    }
#pragma unroll
    for (int r = 0; r < LB; ++r) {
      const int e = tid + r * 256;
      const int nn = BNF ? e % BN : e / BK;
      const int kk = BNF ? e / BN : e % BK;
      const double re = rb[r].x, im = (double)sb * rb[r].y;
      sB[buf][0][kk][nn] = (float)re;
      sB[buf][1][kk][nn] = (float)(im - re);
      sB[buf][2][kk][nn] = (float)(re + im);
    }
  };
  f4 k1[FM][FN], k2[FM][FN], k3[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      k1[i][j] = f4{0, 0, 0, 0};
      k2[i][j] = f4{0, 0, 0, 0};
      k3[i][j] = f4{0, 0, 0, 0};
    }
  gload(kbeg);
  sstore(0);
  __syncthreads();
  int buf = 0;
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    const bool more = k0 + BK < kend;
    if (more) gload(k0 + BK);
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      const int kk = ks + (lane >> 4);
      float ar[FM], ai[FM], as[FM], br[FN], bd[FN], bs[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) {
        const int mm = wm + i * 16 + (lane & 15);
        ar[i] = sA[buf][0][kk][mm];
        ai[i] = sA[buf][1][kk][mm];
        as[i] = sA[buf][2][kk][mm];
      }
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const int nn = wn + j * 16 + (lane & 15);
        br[j] = sB[buf][0][kk][nn];
        bd[j] = sB[buf][1][kk][nn];
        bs[j] = sB[buf][2][kk][nn];
      }
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          k1[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(as[i], br[j], k1[i][j], 0, 0, 0);
          k2[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[i], bd[j], k2[i][j], 0, 0, 0);
          k3[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai[i], bs[j], k3[i][j], 0, 0, 0);
        }
    }
    if (more) sstore(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  cplx* __restrict__ C = g.C + boff(g, bz, g.sCb, g.sCb2);
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm + i * 16 + f32_out_row(lane, r);
        const int n = n0 + wn + j * 16 + (lane & 15);
        if (m < g.M && n < g.N) {
          const double cr = (double)k1[i][j][r] - (double)k3[i][j][r];
          const double ci = (double)k1[i][j][r] + (double)k2[i][j][r];
          cplx y = make_double2(g.ar * cr - g.ai * ci, g.ar * ci + g.ai * cr);
          cplx* dst = C + (i64)m * g.sCm + (i64)n * g.sCn;
          if (g.beta) {
            const cplx o = *dst;
            y.x += o.x;
            y.y += o.y;
          }
          *dst = y;
        }
      }
}

// 128x128 form of the FP32 kernel (three products, FP32 planes in LDS),
// with the structure of the FP64 128x128 tile: eight waves of 64x32, LDS
// double-buffered (99 KB), the next K-tile fetched into registers during the
// tile and the fragments of the next 4-deep K step read during the MFMAs of
// the current one.  XCD-grouped tile order.
template <bool AK, bool BNF>
__global__ __launch_bounds__(512, 2) void k_cgemm_f32w(GemmArgs g, int tm, int tn, int gm) {
  constexpr int BM = 128, BN = 128, BK = 16, NT = 512, WM = 64, WN = 32, FM = WM / 16, FN = WN / 16;
  constexpr int LA = BM * BK / NT, LB = BN * BK / NT;
  __shared__ float sA[2][3][BK][BM + 1];
  __shared__ float sB[2][3][BK][BN + 1];
  int mi, ni, bz;
  tile_of((int)blockIdx.x, (int)gridDim.x, tm, tn, gm, 1, mi, ni, bz);
  const int m0 = mi * BM, n0 = ni * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const cplx* __restrict__ A = g.A + boff(g, bz, g.sAb, g.sAb2);
  const cplx* __restrict__ B = g.B + boff(g, bz, g.sBb, g.sBb2);
  const int wm = (wave & 1) * WM, wn = (wave >> 1) * WN;
  const float sa = g.conjA ? -1.f : 1.f;
  const double sb = g.conjB ? -1.0 : 1.0;
  const i64 sAk = AK ? 1 : g.sAk, sBn = BNF ? 1 : g.sBn;
  const int mA = AK ? tid / BK : tid % BM, kA = AK ? tid % BK : tid / BM;
  const int dmA = AK ? NT / BK : 0, dkA = AK ? 0 : NT / BM;
  const int nB = BNF ? tid % BN : tid / BK, kB = BNF ? tid / BN : tid % BK;
  const int dnB = BNF ? 0 : NT / BK, dkB = BNF ? NT / BN : 0;
  const cplx* __restrict__ pA = A + (i64)(m0 + mA) * g.sAm + (i64)kA * sAk;
  const cplx* __restrict__ pB = B + (i64)kB * g.sBk + (i64)(n0 + nB) * sBn;
  const i64 stA = (i64)dmA * g.sAm + (i64)dkA * sAk, stB = (i64)dkB * g.sBk + (i64)dnB * sBn;
  const int kend = g.K;
  cplx ra[LA], rb[LB];
  auto gload = [&](int k0) {
#pragma unroll
    for (int r = 0; r < LA; ++r) {
      const int gm = m0 + mA + r * dmA, gk = k0 + kA + r * dkA;
      ra[r] = (gm < g.M && gk < kend) ? pA[r * stA + (i64)k0 * sAk] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int r = 0; r < LB; ++r) {
      const int gn = n0 + nB + r * dnB, gk = k0 + kB + r * dkB;
      rb[r] = (gn < g.N && gk < kend) ? pB[r * stB + (i64)k0 * g.sBk] : make_double2(0.0, 0.0);
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int r = 0; r < LA; ++r) {
      const int mm = mA + r * dmA, kk = kA + r * dkA;
      sA[buf][0][kk][mm] = (float)ra[r].x;
      sA[buf][1][kk][mm] = sa * (float)ra[r].y;
      sA[buf][2][kk][mm] = (float)(ra[r].x + (double)sa * ra[r].y);
    }
#pragma unroll
    for (int r = 0; r < LB; ++r) {
      const int nn = nB + r * dnB, kk = kB + r * dkB;
      const double re = rb[r].x, im = sb * rb[r].y;
      sB[buf][0][kk][nn] = (float)re;
      sB[buf][1][kk][nn] = (float)(im - re);
      sB[buf][2][kk][nn] = (float)(re + im);
    }
  };
  float fa[2][3][FM], fb[2][3][FN];
  auto fread = [&](int buf, int ks, int s) {
    const int kk = ks + (lane >> 4);
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int p = 0; p < 3; ++p) fa[s][p][i] = sA[buf][p][kk][wm + i * 16 + (lane & 15)];
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int p = 0; p < 3; ++p) fb[s][p][j] = sB[buf][p][kk][wn + j * 16 + (lane & 15)];
  };
  f4 k1[FM][FN], k2[FM][FN], k3[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      k1[i][j] = f4{0, 0, 0, 0};
      k2[i][j] = f4{0, 0, 0, 0};
      k3[i][j] = f4{0, 0, 0, 0};
    }
  gload(0);
  sstore(0);
  __syncthreads();
  int buf = 0;
  fread(0, 0, 0);
  for (int k0 = 0; k0 < kend; k0 += BK) {
    const bool more = k0 + BK < kend;
    if (more) gload(k0 + BK);
#pragma unroll
    for (int q = 0; q < BK / 4; ++q) {
      const int s = q & 1;
      if (q + 1 < BK / 4) fread(buf, 4 * (q + 1), s ^ 1);
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          // k1 = (Ar + Ai) Br, k2 = Ar (Bi - Br), k3 = Ai (Br + Bi)
          k1[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[s][2][i], fb[s][0][j], k1[i][j], 0, 0, 0);
          k2[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[s][0][i], fb[s][1][j], k2[i][j], 0, 0, 0);
          k3[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[s][1][i], fb[s][2][j], k3[i][j], 0, 0, 0);
        }
    }
    if (more) sstore(buf ^ 1);
    __syncthreads();
    buf ^= 1;
    if (more) fread(buf, 0, 0);
  }
  cplx* __restrict__ C = g.C + boff(g, bz, g.sCb, g.sCb2);
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm + i * 16 + f32_out_row(lane, r);
        const int n = n0 + wn + j * 16 + (lane & 15);
        if (m < g.M && n < g.N) {
          const double cr = (double)k1[i][j][r] - (double)k3[i][j][r];
          const double ci = (double)k1[i][j][r] + (double)k2[i][j][r];
          cplx y = make_double2(g.ar * cr - g.ai * ci, g.ar * ci + g.ai * cr);
          cplx* dst = C + (i64)m * g.sCm + (i64)n * g.sCn;
          if (g.beta) {
            const cplx o = *dst;
            y.x += o.x;
            y.y += o.y;
          }
          *dst = y;
        }
      }
}

inline unsigned grid_for(i64 total) {
  i64 g = (total + 255) / 256;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (unsigned)g;
}
}  // namespace

// FP64 GEMM variants: tile 128x64 or 64x64, three or four real products
// (M-tiles per group of the tile order)
constexpr int kGroupM = 8;
template <int BM, int BN, bool G3>
static void launch_p(const GemmArgs& g, bool grouped, hipStream_t s) {
  const bool ak = g.sAk == 1, bn = g.sBn == 1;
  const int tm = (g.M + BM - 1) / BM, tn = (g.N + BN - 1) / BN, gm = grouped ? std::min(tm, kGroupM) : tm;
  const int xcd = grouped ? 1 : 0;
  const i64 total = (i64)tm * tn * g.batch;
  REQUIRE(total >= 1 && total < (1ll << 31), CCLR_EINVAL, "GEMM launch has too many tiles");
  dim3 grid((unsigned)total);
  if (ak && bn) hipLaunchKernelGGL((k_zgemm_p<BM, BN, true, true, G3>), grid, dim3(256), 0, s, g, tm, tn, gm, xcd);
  else if (ak) hipLaunchKernelGGL((k_zgemm_p<BM, BN, true, false, G3>), grid, dim3(256), 0, s, g, tm, tn, gm, xcd);
  else if (bn) hipLaunchKernelGGL((k_zgemm_p<BM, BN, false, true, G3>), grid, dim3(256), 0, s, g, tm, tn, gm, xcd);
  else hipLaunchKernelGGL((k_zgemm_p<BM, BN, false, false, G3>), grid, dim3(256), 0, s, g, tm, tn, gm, xcd);
}

template <int BM, int BN = 64>
static void launch_p1(const GemmArgs& g, bool grouped, hipStream_t s) {
  const bool ak = g.sAk == 1, bn = g.sBn == 1;
  const int tm = (g.M + BM - 1) / BM, tn = (g.N + BN - 1) / BN, gm = grouped ? std::min(tm, kGroupM) : tm;
  const int xcd = grouped ? 1 : 0;
  const i64 total = (i64)tm * tn * g.batch;
  REQUIRE(total >= 1 && total < (1ll << 31), CCLR_EINVAL, "GEMM launch has too many tiles");
  dim3 grid((unsigned)total);
  if (ak && bn) hipLaunchKernelGGL((k_zgemm_p1<BM, BN, true, true, false>), grid, dim3(256), 0, s, g, tm, tn, gm, xcd);
  else if (ak) hipLaunchKernelGGL((k_zgemm_p1<BM, BN, true, false, false>), grid, dim3(256), 0, s, g, tm, tn, gm, xcd);
  else if (bn) hipLaunchKernelGGL((k_zgemm_p1<BM, BN, false, true, false>), grid, dim3(256), 0, s, g, tm, tn, gm, xcd);
  else hipLaunchKernelGGL((k_zgemm_p1<BM, BN, false, false, false>), grid, dim3(256), 0, s, g, tm, tn, gm, xcd);
}

static void launch_w1(const GemmArgs& g, bool grouped, hipStream_t s) {
  const bool ak = g.sAk == 1, bn = g.sBn == 1;
  const int tm = (g.M + 127) / 128, tn = (g.N + 127) / 128, gm = grouped ? std::min(tm, kGroupM) : tm;
  const int xcd = grouped ? 1 : 0;
  const i64 total = (i64)tm * tn * g.batch;
  REQUIRE(total >= 1 && total < (1ll << 31), CCLR_EINVAL, "GEMM launch has too many tiles");
  dim3 grid((unsigned)total);
  if (ak && bn) hipLaunchKernelGGL((k_zgemm_w1<true, true>), grid, dim3(512), 0, s, g, tm, tn, gm, xcd);
  else if (ak) hipLaunchKernelGGL((k_zgemm_w1<true, false>), grid, dim3(512), 0, s, g, tm, tn, gm, xcd);
  else if (bn) hipLaunchKernelGGL((k_zgemm_w1<false, true>), grid, dim3(512), 0, s, g, tm, tn, gm, xcd);
  else hipLaunchKernelGGL((k_zgemm_w1<false, false>), grid, dim3(512), 0, s, g, tm, tn, gm, xcd);
}

template <int BM>
static void launch_dma(const GemmArgs& g, bool grouped, hipStream_t s) {
  constexpr int BN = DmaShape<BM>::BN;
  const bool ak = g.sAk == 1, bn = g.sBn == 1;
  const int tm = (g.M + BM - 1) / BM, tn = (g.N + BN - 1) / BN, gm = grouped ? std::min(tm, kGroupM) : tm;
  const int xcd = grouped ? 1 : 0;
  const i64 total = (i64)tm * tn * g.batch;
  REQUIRE(total >= 1 && total < (1ll << 31), CCLR_EINVAL, "GEMM launch has too many tiles");
  dim3 grid((unsigned)total);
  if (ak && bn) hipLaunchKernelGGL((k_zgemm_dma<BM, true, true>), grid, dim3(512), 0, s, g, tm, tn, gm, xcd);
  else if (ak) hipLaunchKernelGGL((k_zgemm_dma<BM, true, false>), grid, dim3(512), 0, s, g, tm, tn, gm, xcd);
  else if (bn) hipLaunchKernelGGL((k_zgemm_dma<BM, false, true>), grid, dim3(512), 0, s, g, tm, tn, gm, xcd);
  else hipLaunchKernelGGL((k_zgemm_dma<BM, false, false>), grid, dim3(512), 0, s, g, tm, tn, gm, xcd);
}

void launch_zgemm_variant(const GemmArgs& g, int variant, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0 || g.batch <= 0 || g.K <= 0) return;
  if (variant == GEMM_64x256_DMA || variant == GEMM_64x256_DMA_GROUPED) {
    launch_dma<64>(g, variant == GEMM_64x256_DMA_GROUPED, s);
    HIPCHK(hipGetLastError());
    return;
  }
  if (variant == GEMM_128x128_DMA || variant == GEMM_128x128_DMA_GROUPED) {
    launch_dma<128>(g, variant == GEMM_128x128_DMA_GROUPED, s);
    HIPCHK(hipGetLastError());
    return;
  }
  if (variant == GEMM_128x32_G4_SB) {
    launch_p1<128, 32>(g, false, s);
    HIPCHK(hipGetLastError());
    return;
  }
  if (variant == GEMM_64x32_G4) {
    launch_p<64, 32, false>(g, false, s);
    HIPCHK(hipGetLastError());
    return;
  }
  if (variant == GEMM_128x128_G4 || variant == GEMM_128x128_G4_GROUPED) {
    launch_w1(g, variant == GEMM_128x128_G4_GROUPED, s);
    HIPCHK(hipGetLastError());
    return;
  }
  if (variant == GEMM_64x64_G4_SB || variant == GEMM_64x64_G4_SB_GROUPED) {
    launch_p1<64>(g, variant == GEMM_64x64_G4_SB_GROUPED, s);
    HIPCHK(hipGetLastError());
    return;
  }
  if (variant == GEMM_128x64_G4_SB || variant == GEMM_128x64_G4_SB_GROUPED) {
    launch_p1<128>(g, variant == GEMM_128x64_G4_SB_GROUPED, s);
    HIPCHK(hipGetLastError());
    return;
  }
  const bool grouped = variant > GEMM_64x64_G4;
  switch (grouped ? variant - GEMM_64x64_G4 : variant) {
    case GEMM_128x64_G3: launch_p<128, 64, true>(g, grouped, s); break;
    case GEMM_64x64_G3: launch_p<64, 64, true>(g, grouped, s); break;
    case GEMM_128x64_G4: launch_p<128, 64, false>(g, grouped, s); break;
    case GEMM_64x64_G4: launch_p<64, 64, false>(g, grouped, s); break;
    default: {
      dim3 grid((g.M + GBM - 1) / GBM, (g.N + GBN - 1) / GBN, g.batch);
      hipLaunchKernelGGL(k_zgemm, grid, dim3(256), 0, s, g);
    }
  }
  HIPCHK(hipGetLastError());
}

template <int BM, int BN, bool G3>
static void launch_group(const GemmArgs* probs, const int* tstart, int nprob, int total, bool ak, bool bn,
                         hipStream_t s) {
  // persistent grid: as many workgroups as fit on the 256 CUs at once (LDS bound)
  constexpr int NP = G3 ? 3 : 2;
  constexpr int lds = 2 * NP * 16 * (BM + 1 + BN + 1) * 8;
  const int per_cu = (160 * 1024) / lds;
  const int grid = std::min(total, 256 * std::max(1, per_cu));
  if (ak && bn) hipLaunchKernelGGL((k_zgemm_group<BM, BN, true, true, G3>), dim3(grid), dim3(256), 0, s, probs, tstart, nprob, total);
  else if (ak) hipLaunchKernelGGL((k_zgemm_group<BM, BN, true, false, G3>), dim3(grid), dim3(256), 0, s, probs, tstart, nprob, total);
  else if (bn) hipLaunchKernelGGL((k_zgemm_group<BM, BN, false, true, G3>), dim3(grid), dim3(256), 0, s, probs, tstart, nprob, total);
  else hipLaunchKernelGGL((k_zgemm_group<BM, BN, false, false, G3>), dim3(grid), dim3(256), 0, s, probs, tstart, nprob, total);
}

int gemm_tile_rows(int variant) {
  return (variant == GEMM_128x64_G3 || variant == GEMM_128x64_G4 || variant == GEMM_128x128_G4 ||
          variant == GEMM_128x128_DMA || variant == GEMM_128x32_G4_SB)
             ? 128
             : 64;
}
int gemm_tile_cols(int variant) {
  if (variant == GEMM_128x32_G4_SB || variant == GEMM_64x32_G4) return 32;
  return (variant == GEMM_128x128_G4 || variant == GEMM_128x128_DMA) ? 128 : 64;
}

void launch_zgemm_group(const GemmArgs* probs, const int* tstart, int nprob, int total, int variant, bool ak, bool bn,
                        hipStream_t s) {
  if (total <= 0) return;
  if (variant == GEMM_128x128_DMA) {
    const int grid = std::min(total, 256);
    if (ak && bn) hipLaunchKernelGGL((k_zgemm_group_dma<true, true>), dim3(grid), dim3(512), 0, s, probs, tstart, nprob, total);
    else if (ak) hipLaunchKernelGGL((k_zgemm_group_dma<true, false>), dim3(grid), dim3(512), 0, s, probs, tstart, nprob, total);
    else if (bn) hipLaunchKernelGGL((k_zgemm_group_dma<false, true>), dim3(grid), dim3(512), 0, s, probs, tstart, nprob, total);
    else hipLaunchKernelGGL((k_zgemm_group_dma<false, false>), dim3(grid), dim3(512), 0, s, probs, tstart, nprob, total);
    HIPCHK(hipGetLastError());
    return;
  }
  if (variant == GEMM_128x128_G4) {
    const int grid = std::min(total, 256);
    if (ak && bn) hipLaunchKernelGGL((k_zgemm_group_w1<true, true>), dim3(grid), dim3(512), 0, s, probs, tstart, nprob, total);
    else if (ak) hipLaunchKernelGGL((k_zgemm_group_w1<true, false>), dim3(grid), dim3(512), 0, s, probs, tstart, nprob, total);
    else if (bn) hipLaunchKernelGGL((k_zgemm_group_w1<false, true>), dim3(grid), dim3(512), 0, s, probs, tstart, nprob, total);
    else hipLaunchKernelGGL((k_zgemm_group_w1<false, false>), dim3(grid), dim3(512), 0, s, probs, tstart, nprob, total);
    HIPCHK(hipGetLastError());
    return;
  }
  switch (variant) {
    case GEMM_128x64_G3: launch_group<128, 64, true>(probs, tstart, nprob, total, ak, bn, s); break;
    case GEMM_64x64_G3: launch_group<64, 64, true>(probs, tstart, nprob, total, ak, bn, s); break;
    case GEMM_128x64_G4: launch_group<128, 64, false>(probs, tstart, nprob, total, ak, bn, s); break;
    default: launch_group<64, 64, false>(probs, tstart, nprob, total, ak, bn, s); break;
  }
  HIPCHK(hipGetLastError());
}

int gemm_default_variant(const GemmArgs& g) {
  return (i64)g.M * g.N * g.batch >= (i64)128 * 64 * 1024 ? GEMM_128x64_G4 : GEMM_64x64_G4;
}

void launch_zgemm(const GemmArgs& g, hipStream_t s) { launch_zgemm_variant(g, gemm_default_variant(g), s); }

void launch_zgemm_lowp(const GemmArgs& g, int prec, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0 || g.batch <= 0 || g.K <= 0) return;
  REQUIRE(prec == CCLR_FP32, CCLR_EINVAL, "low-precision GEMM: only CCLR_FP32 is available");
  const bool ak = g.sAk == 1, bn = g.sBn == 1;
  if (g.kchunk == 0 && g.M >= 512 && g.N >= 512) {
    // large products: 128x128 tiles in the XCD-grouped order
    const int tm = (g.M + 127) / 128, tn = (g.N + 127) / 128, gm = std::min(tm, kGroupM);
    const i64 total = (i64)tm * tn * g.batch;
    REQUIRE(total < (1ll << 31), CCLR_EINVAL, "GEMM launch has too many tiles");
    dim3 grid((unsigned)total);
    if (ak && bn) hipLaunchKernelGGL((k_cgemm_f32w<true, true>), grid, dim3(512), 0, s, g, tm, tn, gm);
    else if (ak) hipLaunchKernelGGL((k_cgemm_f32w<true, false>), grid, dim3(512), 0, s, g, tm, tn, gm);
    else if (bn) hipLaunchKernelGGL((k_cgemm_f32w<false, true>), grid, dim3(512), 0, s, g, tm, tn, gm);
    else hipLaunchKernelGGL((k_cgemm_f32w<false, false>), grid, dim3(512), 0, s, g, tm, tn, gm);
    HIPCHK(hipGetLastError());
    return;
  }
  const int p32 = (g.N + 31) / 32 * 32, p64 = (g.N + 63) / 64 * 64;
  if (g.N <= 32 || (g.N <= 512 && 8 * (p64 - p32) >= p32)) {
    // at most 32 output columns (the o index): 32-column tiles pad half as much as
    // 64-column ones; also outputs up to 512 wide that 64-column tiles pad by a
    // further eighth or more (200: 224 columns against 256)
    dim3 grid((g.M + 127) / 128, (g.N + 31) / 32, g.batch);
    if (ak && bn) hipLaunchKernelGGL((k_cgemm_f32<128, 32, true, true>), grid, dim3(256), 0, s, g);
    else if (ak) hipLaunchKernelGGL((k_cgemm_f32<128, 32, true, false>), grid, dim3(256), 0, s, g);
    else if (bn) hipLaunchKernelGGL((k_cgemm_f32<128, 32, false, true>), grid, dim3(256), 0, s, g);
    else hipLaunchKernelGGL((k_cgemm_f32<128, 32, false, false>), grid, dim3(256), 0, s, g);
    HIPCHK(hipGetLastError());
    return;
  }
  dim3 grid((g.M + 127) / 128, (g.N + 63) / 64, g.batch);
  if (ak && bn) hipLaunchKernelGGL((k_cgemm_f32<128, 64, true, true>), grid, dim3(256), 0, s, g);
  else if (ak) hipLaunchKernelGGL((k_cgemm_f32<128, 64, true, false>), grid, dim3(256), 0, s, g);
  else if (bn) hipLaunchKernelGGL((k_cgemm_f32<128, 64, false, true>), grid, dim3(256), 0, s, g);
  else hipLaunchKernelGGL((k_cgemm_f32<128, 64, false, false>), grid, dim3(256), 0, s, g);
  HIPCHK(hipGetLastError());
}

bool launch_zgemm_smallk(const GemmArgs& g0, hipStream_t s) {
  if (g0.K > SK_MAX || g0.kchunk > 0 || g0.M <= 0 || g0.N <= 0 || g0.batch <= 0 || g0.K <= 0) return false;
  GemmArgs g = g0;
  // run the threads along the unit-stride index of C (transpose the product if that is m)
  if (g0.sCn != 1 && g0.sCm == 1) {
    g.M = g0.N; g.N = g0.M;
    g.A = g0.B; g.sAb = g0.sBb; g.sAb2 = g0.sBb2; g.sAm = g0.sBn; g.sAk = g0.sBk; g.conjA = g0.conjB;
    g.B = g0.A; g.sBb = g0.sAb; g.sBb2 = g0.sAb2; g.sBk = g0.sAk; g.sBn = g0.sAm; g.conjB = g0.conjA;
    g.sCm = g0.sCn; g.sCn = g0.sCm;
  }
  if (g.batch >= 65536 || (g.M + SK_MB - 1) / SK_MB >= 65536) return false;
  dim3 grid((g.N + 255) / 256, (g.M + SK_MB - 1) / SK_MB, g.batch);
  // the reduction length rounded up to a multiple of 4: the padding terms cost
  // LDS reads and FMAs like real ones (K = 20 on the 32-term kernel took
  // 20-28% longer than on the 20-term one)
  switch ((g.K + 3) / 4) {
    case 1: hipLaunchKernelGGL(k_zgemm_smallk<4>, grid, dim3(256), 0, s, g); break;
    case 2: hipLaunchKernelGGL(k_zgemm_smallk<8>, grid, dim3(256), 0, s, g); break;
    case 3: hipLaunchKernelGGL(k_zgemm_smallk<12>, grid, dim3(256), 0, s, g); break;
    case 4: hipLaunchKernelGGL(k_zgemm_smallk<16>, grid, dim3(256), 0, s, g); break;
    case 5: hipLaunchKernelGGL(k_zgemm_smallk<20>, grid, dim3(256), 0, s, g); break;
    case 6: hipLaunchKernelGGL(k_zgemm_smallk<24>, grid, dim3(256), 0, s, g); break;
    case 7: hipLaunchKernelGGL(k_zgemm_smallk<28>, grid, dim3(256), 0, s, g); break;
    default: hipLaunchKernelGGL(k_zgemm_smallk<32>, grid, dim3(256), 0, s, g); break;
  }
  HIPCHK(hipGetLastError());
  return true;
}

void launch_zgemm_simple(const GemmArgs& g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0 || g.batch <= 0 || g.K <= 0) return;
  dim3 grid((g.M + GBM - 1) / GBM, (g.N + GBN - 1) / GBN, g.batch);
  hipLaunchKernelGGL(k_zgemm, grid, dim3(256), 0, s, g);
  HIPCHK(hipGetLastError());
}

void launch_splitk_reduce(int nb, int S, int M, int N, const cplx* W, cplx* C, i64 sCb, i64 sCm, i64 sCn, double ar,
                          double ai, int beta, hipStream_t s) {
  hipLaunchKernelGGL(k_splitk_reduce, dim3(grid_for((i64)M * N * nb)), dim3(256), 0, s, nb, S, M, N, W, C, sCb, sCm,
                     sCn, ar, ai, beta);
  HIPCHK(hipGetLastError());
}
