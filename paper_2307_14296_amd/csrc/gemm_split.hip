// Complex GEMMs on pre-split operands for the reduced-precision inner
// solves: split-BF16 (below) and FP32 Gauss planes (after it).
//
// Split-BF16.
// Every real component x of a complex128 operand is split into bf16 numbers,
// hi = bf16(x) and lo = bf16(x - hi), so x = hi + lo to about 2^-17
// relative.  A real product of two split operands is formed from three bf16
// MFMA products, hi*hi + hi*lo + lo*hi (the lo*lo term is below the split's
// own error; CCLR_BF16X3), or, with the second operand kept as hi only, from
// two, hi*hi + lo*hi (CCLR_BF16X2: the second operand then carries bf16
// rounding, about 2^-9 relative, which the FP64 refinement of the solver
// absorbs).  Products accumulate in FP32 on v_mfma_f32_16x16x32_bf16.
//
// A complex block takes three accumulators holding Ar Br, Ai Bi and
// Ar Bi + Ai Br, so Re = acc0 - acc1 and Im = acc2: twelve (X3) or eight (X2)
// bf16 MFMAs per complex block.  (Gauss's three-product form would save a
// quarter of the MFMAs but needs the (re + im) planes too, 1.5 times the
// operand traffic through LDS, which the kernel cannot afford: LDS reads and
// the direct loads already take about half of the MFMA time.)
//
// Operands are stored pre-split: a rows x K complex matrix becomes
// [K/32][rows_pad][4P] 16-byte chunks for P planes (re_hi, re_lo, im_hi,
// im_lo, or re_hi, im_hi).  Logical chunk c = 4p + g of row r holds the eight
// bf16 values k = 32 kc + 8 g ... + 7 of plane p and is stored at position
// c ^ sw(r) of the row, sw(r) = r mod 16 (P = 4) or (r / 2) mod 8 (P = 2):
// the MFMA operand reads (one chunk of 16 consecutive rows per 16 lanes) then
// fall in 16 different 16-byte bank groups.  Rows are padded to the 128-row
// tile and K to the MFMA's 32 with zeros.  One tile of one k step is
// contiguous and a multiple of 256 chunks, so it is copied into LDS by
// direct global-to-LDS loads, every lane active (no registers, no LDS store
// instructions, no branches in the loop).  The Jacobian's ladder and ring
// operators are split once per set of amplitudes and kept; the trial vectors
// are split per product.
#include "internal.h"

namespace {
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned u4v __attribute__((ext_vector_type(4)));

constexpr int TM = 128;  // tile rows of both operands (and row padding of every split operand)

// plane codes of a split operand
enum { P_RH = 0, P_RL, P_IH, P_IL };

// The two kernel forms: planes of the A and B operands and the MFMA list
// (A plane, B plane, accumulator), small terms first, ordered so that
// consecutive MFMAs go to different accumulators.
struct FormDesc {
  int pa, pb;  // planes per operand
  int planes_a[4], planes_b[4];
  int nprod;
  int prod[12][3];
};
constexpr FormDesc kForms[2] = {
    // X3: both operands split, 12 MFMAs per complex block
    {4, 4, {P_RH, P_RL, P_IH, P_IL}, {P_RH, P_RL, P_IH, P_IL}, 12,
     {{1, 0, 0}, {3, 2, 1}, {1, 2, 2}, {0, 1, 0}, {2, 3, 1}, {3, 0, 2},
      {0, 0, 0}, {2, 2, 1}, {0, 3, 2}, {0, 2, 2}, {2, 1, 2}, {2, 0, 2}}},
    // X2: B planes re_hi, im_hi; 8 MFMAs per complex block
    {4, 2, {P_RH, P_RL, P_IH, P_IL}, {P_RH, P_IH}, 8,
     {{1, 0, 0}, {3, 1, 1}, {1, 1, 2}, {0, 0, 0}, {2, 1, 1}, {3, 0, 2}, {0, 1, 2}, {2, 0, 2}}},
};

// position of logical chunk c in row r of a split operand with P planes
__host__ __device__ constexpr int swz(int P, int r, int c) { return c ^ (P == 4 ? (r & 15) : ((r >> 1) & 7)); }

// round-to-nearest-even bf16 bits of a finite float
__device__ __forceinline__ unsigned bf16_bits(float x) {
  const unsigned u = __float_as_uint(x);
  return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}

// bits of plane `code` of the complex value (re, im)
__device__ __forceinline__ unsigned plane_bits(int code, double re, double im) {
  const double x = code < P_IH ? re : im;
  const unsigned hi = bf16_bits((float)x);
  if (!(code & 1)) return hi;
  return bf16_bits((float)(x - (double)__uint_as_float(hi << 16)));
}

// One thread reads eight k values of one row and writes their chunk in every
// plane.  Threads run along k when the source's unit stride is k, along rows
// otherwise, so the reads coalesce.
template <int P>
__global__ __launch_bounds__(256) void k_split(int rows, int K, const cplx* __restrict__ src, i64 sR, i64 sK,
                                               int conj, u4v* __restrict__ dst, int rows_pad, int nkc, int p0, int p1,
                                               int p2, int p3, int rows_fast) {
  const int code[4] = {p0, p1, p2, p3};
  const i64 units = (i64)rows_pad * nkc * 4;
  const double si = conj ? -1.0 : 1.0;
  for (i64 u = blockIdx.x * (i64)blockDim.x + threadIdx.x; u < units; u += (i64)gridDim.x * blockDim.x) {
    i64 r, kc;
    int g;
    if (rows_fast) {
      r = u % rows_pad;
      const i64 q = u / rows_pad;
      g = (int)(q & 3);
      kc = q >> 2;
    } else {
      g = (int)(u & 3);
      const i64 q = u >> 2;
      r = q % rows_pad;
      kc = q / rows_pad;
    }
    cplx x[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const i64 k = kc * 32 + g * 8 + e;
      x[e] = (r < rows && k < K) ? src[r * sR + k * sK] : make_double2(0.0, 0.0);
      x[e].y *= si;
    }
    u4v* o = dst + (kc * rows_pad + r) * (4 * P);
#pragma unroll
    for (int p = 0; p < P; ++p) {
      u4v w;
#pragma unroll
      for (int e = 0; e < 8; e += 2)
        w[e >> 1] = plane_bits(code[p], x[e].x, x[e].y) | (plane_bits(code[p], x[e + 1].x, x[e + 1].y) << 16);
      o[swz(P, (int)r, 4 * p + g)] = w;
    }
  }
}

__device__ __forceinline__ bf8 as_bf8(u4v x) { return __builtin_bit_cast(bf8, x); }

#define MF(a, b, c) __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0)

// Copy CH contiguous 16-byte chunks (a multiple of NT) from global memory
// into LDS with direct loads; each wave instruction moves 64 consecutive chunks.
template <int NT, int CH>
__device__ __forceinline__ void dma_tile(const u4v* __restrict__ g, u4v* lds, int tid) {
  static_assert(CH % NT == 0, "tile must be a whole number of rounds");
#pragma unroll
  for (int e0 = 0; e0 < CH; e0 += NT)
    __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(g + e0 + tid),
                                     (__attribute__((address_space(3))) void*)(lds + e0 + (tid & ~63)), 16, 0, 0);
}

// C[m][n] (+)= alpha * sum_k A[m][k] B[n][k] on split operands.  128 x 128
// tile per workgroup of eight waves (2 x 4, each 64 x 32 in 16x16 MFMA
// blocks; two waves per SIMD, which hide each other's LDS and barrier
// waits: about 1.2 times faster than four waves of 64 x 64 with one wave per
// SIMD), double-buffered LDS filled by direct loads one k step ahead: each
// step requests the next step's tiles into the other stage, then reads its
// operand fragments and runs its MFMAs while the loads are in flight; the
// wait for the loads and the barrier come before the MFMAs of its last row
// block, whose time covers the reads of the next step's first fragments
// (3-5% faster than a barrier after the last MFMA).  The
// stages are separate LDS arrays, so the compiler does not make the reads of
// one wait for the direct loads into the other.  Workgroups are numbered so
// that each XCD (workgroups are dealt to the 8 XCDs round-robin) walks a
// contiguous range of tiles, m fastest: the B tile of a step is shared by
// the workgroups of one XCD and its L2.
template <int F>
__global__ __launch_bounds__(512) void k_cgemm_bf16s(const u4v* __restrict__ As, const u4v* __restrict__ Bs,
                                                     int Mpad, int Npad, int nkc, int M, int N, cplx* __restrict__ C,
                                                     i64 sCm, i64 sCn, double ar, double ai, int beta, int Mt, int T) {
  constexpr FormDesc D = kForms[F];
  constexpr int PA = D.pa, PB = D.pb;
  constexpr int RSA = 4 * PA, RSB = 4 * PB;  // chunks per row
  constexpr int NT = 512;  // eight waves: two along m, four along n
  constexpr int WM = TM / 2, WN = TM / 4;
  constexpr int FM = WM / 16, FN = WN / 16;
  constexpr int CA = TM * RSA, CB = TM * RSB;  // chunks per tile and k step
  // the two stages in separate arrays, so the compiler can tell a read of
  // one stage from the direct loads into the other and does not make the
  // reads wait for the loads
  __shared__ u4v sA0[CA], sA1[CA];
  __shared__ u4v sB0[CB], sB1[CB];
  const int per = gridDim.x >> 3;
  const int t = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
  if (t >= T) return;
  const int m0 = (t % Mt) * TM, n0 = (t / Mt) * TM;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave & 1) * WM, wn = (wave >> 1) * WN;
  static_assert(CA % NT == 0 && CB % NT == 0, "tiles must be whole rounds of direct loads");
  const int rr = lane & 15, g = lane >> 4;
  auto fetch = [&](int kc, u4v* la, u4v* lb) {
    dma_tile<NT, CA>(As + ((i64)kc * Mpad + m0) * RSA, la, tid);
    dma_tile<NT, CB>(Bs + ((i64)kc * Npad + n0) * RSB, lb, tid);
  };
  // LDS offsets of this lane's fragments (rows wm + 16 i + rr, wn + 16 j + rr;
  // the swizzle depends on the row only through rr)
  int offa[PA], offb[PB];
#pragma unroll
  for (int p = 0; p < PA; ++p) offa[p] = (wm + rr) * RSA + swz(PA, rr, 4 * p + g);
#pragma unroll
  for (int p = 0; p < PB; ++p) offb[p] = (wn + rr) * RSB + swz(PB, rr, 4 * p + g);
  f4 acc[3][FM][FN];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) acc[a][i][j] = f4{0.f, 0.f, 0.f, 0.f};
  auto mfma_i = [&](int i, const bf8 (&a)[PA], const bf8 (&b)[FN][PB]) {
#pragma unroll
    for (int q = 0; q < D.nprod; ++q)
#pragma unroll
      for (int j = 0; j < FN; ++j)
        acc[D.prod[q][2]][i][j] = MF(a[D.prod[q][0]], b[j][D.prod[q][1]], acc[D.prod[q][2]][i][j]);
  };
  auto read_b = [&](const u4v* cb, bf8 (&b)[FN][PB]) {
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int p = 0; p < PB; ++p) b[j][p] = as_bf8(cb[offb[p] + 16 * j * RSB]);
  };
  auto read_a = [&](const u4v* ca, int i, bf8 (&a)[PA]) {
#pragma unroll
    for (int p = 0; p < PA; ++p) a[p] = as_bf8(ca[offa[p] + 16 * i * RSA]);
  };
  bf8 bq[FN][PB], aq[PA];  // the first fragments of the next step, read ahead
  // one k step on the stage (ca, cb) while the next step's tiles load into (na, nb)
  auto step = [&](int kc, const u4v* ca, const u4v* cb, u4v* na, u4v* nb) {
    // the last step reloads its own tiles into the idle stage (no branch)
    fetch(kc + 1 < nkc ? kc + 1 : kc, na, nb);
    __builtin_amdgcn_sched_barrier(0);  // the loads are requested first, not scheduled between the MFMAs
    // the wait and the barrier come once the last fragments of this stage
    // are read; the next stage's first fragments are read while the MFMAs
    // of the last row block run
#pragma unroll
    for (int i = 0; i < FM; ++i) {
      bf8 a[PA];
      if (i == 0) {
#pragma unroll
        for (int p = 0; p < PA; ++p) a[p] = aq[p];
      } else {
        read_a(ca, i, a);
      }
      if (i + 1 < FM) {
        mfma_i(i, a, bq);
      } else {
        bf8 bn[FN][PB], an[PA];
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        read_b(nb, bn);
        read_a(na, 0, an);
        mfma_i(i, a, bq);
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
          for (int p = 0; p < PB; ++p) bq[j][p] = bn[j][p];
#pragma unroll
        for (int p = 0; p < PA; ++p) aq[p] = an[p];
      }
    }
  };
  fetch(0, sA0, sB0);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  read_b(sB0, bq);
  read_a(sA0, 0, aq);
  for (int kc = 0; kc < nkc; kc += 2) {
    step(kc, sA0, sB0, sA1, sB1);
    if (kc + 1 < nkc) step(kc + 1, sA1, sB1, sA0, sB0);
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
          const double xr = (double)acc[0][i][j][r] - (double)acc[1][i][j][r], xi = (double)acc[2][i][j][r];
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

// ---------------------------------------------------------------- FP32 form
// Three real products per complex block (Gauss): k1 = (Ar + Ai) Br,
// k2 = Ar (Bi - Br), k3 = Ai (Br + Bi), Re = k1 - k3, Im = k1 + k2, on
// v_mfma_f32_16x16x4f32 with FP32 accumulation.  Split layout: [K/16][rows_pad]
// [12] 16-byte chunks; logical chunk c = 4p + g of a row holds the four FP32
// values k = 16 kb + 4g ... + 3 of plane p (A: Ar + Ai, Ar, Ai; B: Br,
// Bi - Br, Br + Bi), stored at position (c + (r / 4) mod 4) mod 12, which
// puts one chunk of 16 consecutive rows in 16 different bank groups.  A lane
// reads its four k values with one 16-byte read and feeds them to the four
// MFMAs of the k-step (lane group g takes k = 4g + s in MFMA s: the k order
// within the step is the same on both operands, so the sum is unchanged).
__host__ __device__ constexpr int f32pos(int r, int c) { return (c + ((r >> 2) & 3)) % 12; }

__global__ __launch_bounds__(256) void k_split_f32(int rows, int K, const cplx* __restrict__ src, i64 sR, i64 sK,
                                                   int conj, int side, u4v* __restrict__ dst, int rows_pad, int nkb,
                                                   int rows_fast) {
  const i64 units = (i64)rows_pad * nkb * 4;
  const double si = conj ? -1.0 : 1.0;
  for (i64 u = blockIdx.x * (i64)blockDim.x + threadIdx.x; u < units; u += (i64)gridDim.x * blockDim.x) {
    i64 r, kb;
    int g;
    if (rows_fast) {
      r = u % rows_pad;
      const i64 q = u / rows_pad;
      g = (int)(q & 3);
      kb = q >> 2;
    } else {
      g = (int)(u & 3);
      const i64 q = u >> 2;
      r = q % rows_pad;
      kb = q / rows_pad;
    }
    float pl[3][4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const i64 k = kb * 16 + g * 4 + e;
      cplx x = (r < rows && k < K) ? src[r * sR + k * sK] : make_double2(0.0, 0.0);
      const double re = x.x, im = si * x.y;
      if (side == 0) {
        pl[0][e] = (float)(re + im);
        pl[1][e] = (float)re;
        pl[2][e] = (float)im;
      } else {
        pl[0][e] = (float)re;
        pl[1][e] = (float)(im - re);
        pl[2][e] = (float)(re + im);
      }
    }
    u4v* o = dst + (kb * rows_pad + r) * 12;
#pragma unroll
    for (int p = 0; p < 3; ++p)
      o[f32pos((int)r, 4 * p + g)] =
          u4v{__float_as_uint(pl[p][0]), __float_as_uint(pl[p][1]), __float_as_uint(pl[p][2]), __float_as_uint(pl[p][3])};
  }
}

// C[m][n] (+)= alpha * sum_k A[m][k] B[n][k] on FP32 split operands: the
// pipeline of k_cgemm_bf16s (128 x 128 tiles of eight 64 x 32 waves, direct
// loads one 16-deep k step ahead into the other of two LDS stages).
__global__ __launch_bounds__(512) void k_cgemm_f32s(const u4v* __restrict__ As, const u4v* __restrict__ Bs, int Mpad,
                                                    int Npad, int nkb, int M, int N, cplx* __restrict__ C, i64 sCm,
                                                    i64 sCn, double ar, double ai, int beta, int Mt, int T) {
  constexpr int RS = 12, NT = 512, WM = TM / 2, WN = TM / 4, FM = WM / 16, FN = WN / 16;
  constexpr int CH = TM * RS;  // chunks per tile and k step
  static_assert(CH % NT == 0, "tiles must be whole rounds of direct loads");
  __shared__ u4v sA0[CH], sA1[CH];
  __shared__ u4v sB0[CH], sB1[CH];
  const int per = gridDim.x >> 3;
  const int t = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
  if (t >= T) return;
  const int m0 = (t % Mt) * TM, n0 = (t / Mt) * TM;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave & 1) * WM, wn = (wave >> 1) * WN;
  const int rr = lane & 15, g = lane >> 4;
  auto fetch = [&](int kb, u4v* la, u4v* lb) {
    dma_tile<NT, CH>(As + ((i64)kb * Mpad + m0) * RS, la, tid);
    dma_tile<NT, CH>(Bs + ((i64)kb * Npad + n0) * RS, lb, tid);
  };
  // the rotation depends on the row only through rr (wm, wn and 16 i are multiples of 16)
  int off[3];
#pragma unroll
  for (int p = 0; p < 3; ++p) off[p] = rr * RS + f32pos(rr, 4 * p + g);
  f4 acc[3][FM][FN];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) acc[a][i][j] = f4{0.f, 0.f, 0.f, 0.f};
  auto mfma_i = [&](int i, const f4 (&a)[3], const f4 (&b)[FN][3]) {
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          acc[p][i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[p][s], b[j][p][s], acc[p][i][j], 0, 0, 0);
  };
  auto read_b = [&](const u4v* cb, f4 (&b)[FN][3]) {
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int p = 0; p < 3; ++p) b[j][p] = __builtin_bit_cast(f4, cb[(wn + 16 * j) * RS + off[p]]);
  };
  auto read_a = [&](const u4v* ca, int i, f4 (&a)[3]) {
#pragma unroll
    for (int p = 0; p < 3; ++p) a[p] = __builtin_bit_cast(f4, ca[(wm + 16 * i) * RS + off[p]]);
  };
  f4 bq[FN][3], aq[3];  // the first fragments of the next step, read ahead
  auto step = [&](int kb, const u4v* ca, const u4v* cb, u4v* na, u4v* nb) {
    fetch(kb + 1 < nkb ? kb + 1 : kb, na, nb);
    __builtin_amdgcn_sched_barrier(0);  // the loads are requested first, not scheduled between the MFMAs
    // as in the split-BF16 kernel: wait and barrier before the last row block's MFMAs
#pragma unroll
    for (int i = 0; i < FM; ++i) {
      f4 a[3];
      if (i == 0) {
#pragma unroll
        for (int p = 0; p < 3; ++p) a[p] = aq[p];
      } else {
        read_a(ca, i, a);
      }
      if (i + 1 < FM) {
        mfma_i(i, a, bq);
      } else {
        f4 bn[FN][3], an[3];
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        read_b(nb, bn);
        read_a(na, 0, an);
        mfma_i(i, a, bq);
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
          for (int p = 0; p < 3; ++p) bq[j][p] = bn[j][p];
#pragma unroll
        for (int p = 0; p < 3; ++p) aq[p] = an[p];
      }
    }
  };
  fetch(0, sA0, sB0);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  read_b(sB0, bq);
  read_a(sA0, 0, aq);
  for (int kb = 0; kb < nkb; kb += 2) {
    step(kb, sA0, sB0, sA1, sB1);
    if (kb + 1 < nkb) step(kb + 1, sA1, sB1, sA0, sB0);
  }
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm + 16 * i + 4 * g + r;
        const int n = n0 + wn + 16 * j + rr;
        if (m < M && n < N) {
          const double k1 = acc[0][i][j][r], k2 = acc[1][i][j][r], k3 = acc[2][i][j][r];
          const double xr = k1 - k3, xi = k1 + k2;
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

template <int P>
void launch_split_p(const SplitMat& s, const cplx* src, i64 sR, i64 sK, int conj, hipStream_t st) {
  const i64 units = (i64)s.rows_pad * s.nkc * 4;
  i64 grid = (units + 255) / 256;
  if (grid > 65536) grid = 65536;
  const int* c = s.planes;
  hipLaunchKernelGGL(k_split<P>, dim3((unsigned)grid), dim3(256), 0, st, s.rows, s.K, src, sR, sK, conj,
                     (u4v*)s.p, s.rows_pad, s.nkc, c[0], c[1], c[2], c[3], sR == 1 ? 1 : 0);
}
}  // namespace

bool split_form_valid(int form) { return form == BF16_X3 || form == BF16_X2 || form == F32_G3; }

int split_form_of(int prec) { return prec == CCLR_FP32 ? F32_G3 : prec == CCLR_BF16X2 ? BF16_X2 : BF16_X3; }

SplitMat split_shape(int rows, int K, int form, int side) {
  REQUIRE(split_form_valid(form), CCLR_EINVAL, "split: unknown form");
  SplitMat s;
  s.rows = rows;
  s.K = K;
  s.rows_pad = (rows + TM - 1) / TM * TM;
  s.form = form;
  s.side = side;
  if (form == F32_G3) {
    s.nkc = (K + 15) / 16;
    s.nplanes = 3;
    s.chunks = 12;
    return s;
  }
  const FormDesc& d = kForms[form];
  s.nkc = (K + 31) / 32;
  s.nplanes = side == 0 ? d.pa : d.pb;
  s.chunks = 4 * s.nplanes;
  for (int p = 0; p < 4; ++p) s.planes[p] = p < s.nplanes ? (side == 0 ? d.planes_a[p] : d.planes_b[p]) : 0;
  return s;
}

size_t split_bytes(int rows, int K, int form, int side) {
  const SplitMat s = split_shape(rows, K, form, side);
  return (size_t)s.rows_pad * (size_t)s.nkc * (size_t)s.chunks * 16;
}

SplitMat launch_split(int rows, int K, const cplx* src, i64 sR, i64 sK, int conj, void* dst, int form, int side,
                      hipStream_t st) {
  REQUIRE(rows > 0 && K > 0, CCLR_EINVAL, "split: empty operand");
  SplitMat s = split_shape(rows, K, form, side);
  s.p = dst;
  if (form == F32_G3) {
    const i64 units = (i64)s.rows_pad * s.nkc * 4;
    i64 grid = (units + 255) / 256;
    if (grid > 65536) grid = 65536;
    hipLaunchKernelGGL(k_split_f32, dim3((unsigned)grid), dim3(256), 0, st, rows, K, src, sR, sK, conj, side,
                       (u4v*)dst, s.rows_pad, s.nkc, sR == 1 ? 1 : 0);
  } else if (s.nplanes == 4) {
    launch_split_p<4>(s, src, sR, sK, conj, st);
  } else {
    launch_split_p<2>(s, src, sR, sK, conj, st);
  }
  HIPCHK(hipGetLastError());
  return s;
}

void launch_split_gemm(const SplitMat& A, const SplitMat& B, cplx* C, i64 sCm, i64 sCn, double ar, double ai,
                       int beta, hipStream_t st) {
  REQUIRE(A.p && B.p, CCLR_EINVAL, "split GEMM: operand not split");
  REQUIRE(A.form == B.form && A.side == 0 && B.side == 1, CCLR_EINVAL, "split GEMM: operands of different forms");
  REQUIRE(A.K == B.K && A.nkc == B.nkc && A.nkc > 0, CCLR_EINVAL, "split GEMM: operands differ in K");
  const int Mt = A.rows_pad / TM, Nt = B.rows_pad / TM;
  const i64 T = (i64)Mt * Nt;
  REQUIRE(T < (i64)1 << 30, CCLR_EINVAL, "split GEMM: too many tiles");
  const i64 grid = (T + 7) / 8 * 8;
  if (A.form == F32_G3)
    hipLaunchKernelGGL(k_cgemm_f32s, dim3((unsigned)grid), dim3(512), 0, st, (const u4v*)A.p, (const u4v*)B.p,
                       A.rows_pad, B.rows_pad, A.nkc, A.rows, B.rows, C, sCm, sCn, ar, ai, beta, Mt, (int)T);
  else if (A.form == BF16_X2)
    hipLaunchKernelGGL((k_cgemm_bf16s<BF16_X2>), dim3((unsigned)grid), dim3(512), 0, st, (const u4v*)A.p,
                       (const u4v*)B.p, A.rows_pad, B.rows_pad, A.nkc, A.rows, B.rows, C, sCm, sCn, ar, ai, beta, Mt,
                       (int)T);
  else
    hipLaunchKernelGGL((k_cgemm_bf16s<BF16_X3>), dim3((unsigned)grid), dim3(512), 0, st, (const u4v*)A.p,
                       (const u4v*)B.p, A.rows_pad, B.rows_pad, A.nkc, A.rows, B.rows, C, sCm, sCn, ar, ai, beta, Mt,
                       (int)T);
  HIPCHK(hipGetLastError());
}
