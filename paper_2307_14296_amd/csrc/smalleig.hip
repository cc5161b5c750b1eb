// Eigenpairs of the small projected matrix of the EOM-EE Davidson solver, on
// the GPU in one workgroup of one wave: Householder reduction to upper
// Hessenberg form, shifted QR iteration (Wilkinson shift, Givens rotations,
// deflation on small subdiagonals) to the Schur form T = Q^H H Q, then the
// eigenvectors of T for the selected eigenvalues by back substitution, mapped
// back with Q and normalized (Golub and Van Loan, "Matrix Computations",
// ch. 7).  The Hessenberg matrix lives in LDS, packed by rows (row i holds
// columns max(0, i - 1) .. n - 1); the Householder reduction runs on the full
// matrix in LDS as well when it fits (n <= 96), else in a global work area;
// Q lives in the global work area.  Within the one wave, LDS and global accesses of one lane are seen by
// the others after a barrier, and the barriers separate every step whose
// reads depend on another lane's writes.
#include "internal.h"

namespace {
constexpr int kT = 64;                                      // one wave
constexpr int kPacked = (kSmallEigMax * kSmallEigMax + 3 * kSmallEigMax) / 2;  // >= packed Hessenberg size
constexpr int kFullLds = 96;                                 // largest n reduced in LDS
constexpr int kLds = kFullLds * kFullLds > kPacked ? kFullLds * kFullLds : kPacked;

__device__ __forceinline__ cplx cz(double re, double im = 0.0) { return make_double2(re, im); }
__device__ __forceinline__ cplx cadd(cplx a, cplx b) { return cz(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ cplx csub(cplx a, cplx b) { return cz(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ cplx cmul(cplx a, cplx b) { return cz(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ __forceinline__ cplx cjmul(cplx a, cplx b) { return cz(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x); }  // conj(a) b
__device__ __forceinline__ cplx cscale(cplx a, double s) { return cz(a.x * s, a.y * s); }
__device__ __forceinline__ cplx cconj(cplx a) { return cz(a.x, -a.y); }
__device__ __forceinline__ double cnorm(cplx a) { return a.x * a.x + a.y * a.y; }
__device__ __forceinline__ double cabsv(cplx a) { return hypot(a.x, a.y); }
// a / b by Smith's method (no overflow in |b|^2)
__device__ __forceinline__ cplx cdiv(cplx a, cplx b) {
  if (fabs(b.x) >= fabs(b.y)) {
    const double r = b.y / b.x, d = b.x + b.y * r;
    return cz((a.x + a.y * r) / d, (a.y - a.x * r) / d);
  }
  const double r = b.x / b.y, d = b.y + b.x * r;
  return cz((a.x * r + a.y) / d, (a.y * r - a.x) / d);
}
// principal square root
__device__ __forceinline__ cplx csqrtv(cplx z) {
  const double r = hypot(z.x, z.y);
  if (r == 0.0) return cz(0.0);
  const double t = sqrt(0.5 * (r + fabs(z.x)));
  if (z.x >= 0.0) return cz(t, z.y / (2.0 * t));
  return cz(fabs(z.y) / (2.0 * t), copysign(t, z.y));
}
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kT);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kT));
  return v;
}

// H(i, j) = Hu[j ld + i] for i <= j, Hl[i ld + j] for i > j; A and Q are
// n x n row-major work areas.  Outputs: theta[r] and coef[r ldc + i] (unit
// norm eigenvector) for the nroots eigenvalues of smallest real part (ties by
// index), coef2 = -theta coef, all n eigenvalues in wall (if not null), and
// status[0] = 1 (0: the QR iteration did not converge).
__global__ __launch_bounds__(kT) void k_small_eig(int n, const cplx* __restrict__ Hu, const cplx* __restrict__ Hl,
                                                  int ld, cplx* __restrict__ A, cplx* __restrict__ Q, int nroots,
                                                  cplx* __restrict__ coef, cplx* __restrict__ coef2, int ldc,
                                                  cplx* __restrict__ theta, cplx* __restrict__ wall,
                                                  int* __restrict__ status) {
  __shared__ cplx T[kLds];
  __shared__ cplx cs[kSmallEigMax], sn[kSmallEigMax], vv[kSmallEigMax];
  __shared__ int sel[kSmallEigMax];
  const int t = threadIdx.x;
  auto off = [&](int i) { return i == 0 ? 0 : n + (i - 1) * (n + 1) - ((i - 1) * i) / 2; };
  auto h = [&](int i, int j) -> cplx& { return T[off(i) + j - (i > 0 ? i - 1 : 0)]; };

  // the matrix being reduced: in LDS when it fits (generic pointer: LDS or global)
  const bool in_lds = n <= kFullLds;
  cplx* Am = in_lds ? T : A;
  for (int e = t; e < n * n; e += kT) {
    const int i = e / n, j = e - i * n;
    Am[e] = i <= j ? Hu[(i64)j * ld + i] : Hl[(i64)i * ld + j];
    Q[e] = cz(i == j ? 1.0 : 0.0);
  }
  __syncthreads();
  // ---- Householder reduction: A <- P A P, Q <- Q P, P = I - 2 v v^H
  for (int k = 0; k + 2 < n; ++k) {
    double s2 = 0.0;
    for (int i = k + 1 + t; i < n; i += kT) s2 += cnorm(Am[(i64)i * n + k]);
    s2 = wave_sum(s2);
    if (s2 == 0.0) continue;
    const double xn = sqrt(s2);
    const cplx x0 = Am[(i64)(k + 1) * n + k];
    const double ax0 = cabsv(x0);
    const cplx ph = ax0 > 0.0 ? cscale(x0, 1.0 / ax0) : cz(1.0);
    const cplx alpha = cscale(ph, -xn);
    double v2 = 0.0;
    for (int i = k + 1 + t; i < n; i += kT) {
      cplx vi = Am[(i64)i * n + k];
      if (i == k + 1) vi = csub(vi, alpha);
      vv[i] = vi;
      v2 += cnorm(vi);
    }
    v2 = wave_sum(v2);
    if (v2 == 0.0) continue;
    const double inv = 1.0 / sqrt(v2);
    for (int i = k + 1 + t; i < n; i += kT) vv[i] = cscale(vv[i], inv);
    __syncthreads();
    for (int j = t; j < n; j += kT) {  // columns of A
      cplx s = cz(0.0);
#pragma unroll 4
      for (int i = k + 1; i < n; ++i) s = cadd(s, cjmul(vv[i], Am[(i64)i * n + j]));
      for (int i = k + 1; i < n; ++i) Am[(i64)i * n + j] = csub(Am[(i64)i * n + j], cscale(cmul(vv[i], s), 2.0));
    }
    __syncthreads();
    for (int i = t; i < n; i += kT) {  // rows of A and Q
      cplx s = cz(0.0), u = cz(0.0);
#pragma unroll 4
      for (int j = k + 1; j < n; ++j) {
        s = cadd(s, cmul(Am[(i64)i * n + j], vv[j]));
        u = cadd(u, cmul(Q[(i64)i * n + j], vv[j]));
      }
      for (int j = k + 1; j < n; ++j) {
        const cplx cv = cconj(vv[j]);
        Am[(i64)i * n + j] = csub(Am[(i64)i * n + j], cscale(cmul(s, cv), 2.0));
        Q[(i64)i * n + j] = csub(Q[(i64)i * n + j], cscale(cmul(u, cv), 2.0));
      }
    }
    __syncthreads();
  }
  // pack the Hessenberg part by rows; in LDS in place (row i's packed range
  // starts at or before its full range and ends before row i + 1's), one
  // row at a time: every lane reads its entries of the row before any writes
  for (int i = 0; i < n; ++i) {
    const int j0 = i > 0 ? i - 1 : 0;
    cplx x[(kSmallEigMax + kT - 1) / kT];
#pragma unroll
    for (int q = 0; q < (kSmallEigMax + kT - 1) / kT; ++q) {
      const int j = j0 + t + q * kT;
      if (j < n) x[q] = Am[(i64)i * n + j];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < (kSmallEigMax + kT - 1) / kT; ++q) {
      const int j = j0 + t + q * kT;
      if (j < n) h(i, j) = x[q];
    }
    __syncthreads();
  }

  // ---- shifted QR iteration on the Hessenberg matrix
  const double eps = 2.220446049250313e-16;
  int hi = n - 1, iter = 0, total = 0, ok = 1;
  while (hi > 0) {
    int l = hi;
    for (; l > 0; --l) {
      const double s = cabsv(h(l - 1, l - 1)) + cabsv(h(l, l));
      if (cabsv(h(l, l - 1)) <= eps * (s > 0.0 ? s : 1.0)) break;
    }
    __syncthreads();
    if (l > 0 && t == 0) h(l, l - 1) = cz(0.0);
    __syncthreads();
    if (l == hi) {  // one eigenvalue converged
      --hi;
      iter = 0;
      continue;
    }
    if (++total > 100 * n) {
      ok = 0;
      break;
    }
    ++iter;
    // Wilkinson shift from the trailing 2x2 block of the active window
    const cplx a = h(hi - 1, hi - 1), b = h(hi - 1, hi), c = h(hi, hi - 1), d = h(hi, hi);
    const cplx tr = cadd(a, d), det = csub(cmul(a, d), cmul(b, c));
    const cplx disc = csqrtv(csub(cscale(cmul(tr, tr), 0.25), det));
    const cplx m1 = cadd(cscale(tr, 0.5), disc), m2 = csub(cscale(tr, 0.5), disc);
    cplx mu = cabsv(csub(m1, d)) < cabsv(csub(m2, d)) ? m1 : m2;
    if (iter % 11 == 10) mu = cadd(d, cz(cabsv(c)));  // exceptional shift
    __syncthreads();
    for (int k = l + t; k <= hi; k += kT) h(k, k) = csub(h(k, k), mu);
    __syncthreads();
    // H - mu I = G R: rotations from the left, each zeroing one subdiagonal entry
    for (int k = l; k < hi; ++k) {
      const cplx x = h(k, k), y = h(k + 1, k);
      const double r = sqrt(cnorm(x) + cnorm(y));
      cplx cc = cz(1.0), ss = cz(0.0);
      if (r > 0.0) cc = cscale(x, 1.0 / r), ss = cscale(y, 1.0 / r);
      __syncthreads();
      if (t == 0) cs[k - l] = cc, sn[k - l] = ss;
      for (int j = k + t; j < n; j += kT) {
        const cplx u = h(k, j), w = h(k + 1, j);
        h(k, j) = cadd(cjmul(cc, u), cjmul(ss, w));
        h(k + 1, j) = csub(cmul(cc, w), cmul(ss, u));
      }
      __syncthreads();
    }
    // R G + mu I: each lane applies the rotations in order to its own rows
    // (row i takes part in rotation k for i <= k + 1: R is upper triangular)
    for (int i = t; i <= hi; i += kT)
      for (int k = (i > l + 1 ? i - 1 : l); k < hi; ++k) {
        const cplx cc = cs[k - l], ss = sn[k - l];
        const cplx u = h(i, k), w = h(i, k + 1);
        h(i, k) = cadd(cmul(u, cc), cmul(w, ss));
        h(i, k + 1) = csub(cmul(w, cconj(cc)), cmul(u, cconj(ss)));
      }
    for (int i = t; i < n; i += kT) {  // Q <- Q G, row by row
      cplx x = Q[(i64)i * n + l];
      for (int k = l; k < hi; ++k) {
        const cplx cc = cs[k - l], ss = sn[k - l], y = Q[(i64)i * n + k + 1];
        Q[(i64)i * n + k] = cadd(cmul(x, cc), cmul(y, ss));
        x = csub(cmul(y, cconj(cc)), cmul(x, cconj(ss)));
      }
      Q[(i64)i * n + hi] = x;
    }
    __syncthreads();
    for (int k = l + t; k <= hi; k += kT) h(k, k) = cadd(h(k, k), mu);
    __syncthreads();
  }
  if (t == 0) status[0] = ok;
  if (!ok) return;

  // ---- selection: the nroots eigenvalues of smallest real part (ties by index)
  for (int k = t; k < n; k += kT) {
    const double wk = h(k, k).x;
    if (wall) wall[k] = h(k, k);
    int r = 0;
    for (int j = 0; j < n; ++j) {
      const double wj = h(j, j).x;
      r += (wj < wk || (wj == wk && j < k)) ? 1 : 0;
    }
    if (r < nroots) sel[r] = k;
  }
  double tm = 0.0;
  for (int i = t; i < n; i += kT)
    for (int j = i; j < n; ++j) tm = fmax(tm, cabsv(h(i, j)));
  tm = wave_max(tm);
  const double small = eps * (tm > 0.0 ? tm : 1.0);
  __syncthreads();
  // ---- eigenvectors of T (one lane per selected root): y_k = 1, back substitution; y in A's rows
  if (t < nroots) {
    const int k = sel[t];
    const cplx wk = h(k, k);
    cplx* y = A + (i64)t * n;
    y[k] = cz(1.0);
    for (int j = k - 1; j >= 0; --j) {
      cplx s = cz(0.0);
      for (int m = j + 1; m <= k; ++m) s = cadd(s, cmul(h(j, m), y[m]));
      cplx den = csub(h(j, j), wk);
      if (cabsv(den) < small) den = cz(small);
      y[j] = cdiv(cscale(s, -1.0), den);
    }
  }
  __syncthreads();
  // ---- x = Q y, normalized
  for (int r = 0; r < nroots; ++r) {
    const int k = sel[r];
    const cplx* y = A + (i64)r * n;
    double nr = 0.0;
    for (int i = t; i < n; i += kT) {
      cplx s = cz(0.0);
      for (int m = 0; m <= k; ++m) s = cadd(s, cmul(Q[(i64)i * n + m], y[m]));
      coef[(i64)r * ldc + i] = s;
      nr += cnorm(s);
    }
    nr = wave_sum(nr);
    const double inv = nr > 0.0 ? 1.0 / sqrt(nr) : 1.0;
    const cplx th = h(k, k);
    for (int i = t; i < n; i += kT) {
      const cplx x = cscale(coef[(i64)r * ldc + i], inv);
      coef[(i64)r * ldc + i] = x;
      coef2[(i64)r * ldc + i] = cscale(cmul(th, x), -1.0);
    }
    if (t == 0) theta[r] = th;
  }
}
}  // namespace

size_t small_eig_work_elems(int n) { return 2 * (size_t)n * n; }

void launch_small_eig(int n, const cplx* Hu, const cplx* Hl, int ld, cplx* work, int nroots, cplx* coef, cplx* coef2,
                      int ldc, cplx* theta, cplx* wall, int* status, hipStream_t st) {
  REQUIRE(n >= 1 && n <= kSmallEigMax, CCLR_EINVAL, "projected matrix larger than the small eigensolver takes");
  REQUIRE(nroots >= 1 && nroots <= n && ldc >= n, CCLR_EINVAL, "small eigensolver: bad root count or stride");
  hipLaunchKernelGGL(k_small_eig, dim3(1), dim3(kT), 0, st, n, Hu, Hl, ld, work, work + (size_t)n * n, nroots, coef,
                     coef2, ldc, theta, wall, status);
  HIPCHK(hipGetLastError());
}
