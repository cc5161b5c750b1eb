// Pair packing helpers for the packed particle-particle operator: packing
// and unpacking of the last index pair (a > b, pair index a(a-1)/2 + b),
// the antisymmetrizing accumulate used while building W^ef_ab in packed
// form, and the unpacked view of the packed operator.
#include "internal.h"

namespace {
__device__ __forceinline__ i64 pair_index(int hi, int lo) { return (i64)hi * (hi - 1) / 2 + lo; }

__device__ __forceinline__ void unpair(i64 P, int& hi, int& lo) {
  int h = (int)((1.0 + sqrt(1.0 + 8.0 * (double)P)) * 0.5);
  while ((i64)h * (h - 1) / 2 > P) --h;
  while ((i64)(h + 1) * h / 2 <= P) ++h;
  hi = h;
  lo = (int)(P - (i64)h * (h - 1) / 2);
}

inline unsigned grid_for(i64 total) {
  i64 g = (total + 255) / 256;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (unsigned)g;
}

// dst[r][AB] = src[r][a][b] for a > b (the last two indices of rows x v x v packed)
__global__ __launch_bounds__(256) void k_pack_pairs(i64 rows, int v, const cplx* __restrict__ src, cplx* __restrict__ dst) {
  const i64 V2 = (i64)v * (v - 1) / 2, total = rows * V2;
  for (i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (i64)gridDim.x * blockDim.x) {
    const i64 r = e / V2, AB = e % V2;
    int a, b;
    unpair(AB, a, b);
    dst[e] = src[(r * v + a) * v + b];
  }
}

// dst[r][a][b] += alpha src[r][AB], dst[r][b][a] -= alpha src[r][AB] for a > b
__global__ __launch_bounds__(256) void k_unpack_pairs_acc(i64 rows, int v, const cplx* __restrict__ src,
                                                          cplx* __restrict__ dst, double alpha) {
  const i64 V2 = (i64)v * (v - 1) / 2, total = rows * V2;
  for (i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (i64)gridDim.x * blockDim.x) {
    const i64 r = e / V2, AB = e % V2;
    int a, b;
    unpair(AB, a, b);
    const cplx x = src[e];
    cplx* p = dst + (r * v + a) * v + b;
    cplx* q = dst + (r * v + b) * v + a;
    p->x += alpha * x.x, p->y += alpha * x.y;
    q->x -= alpha * x.x, q->y -= alpha * x.y;
  }
}

// W[EF][X] += alpha (Y[e][f][X] - Y[f][e][X]) for e > f, X < nc (W row stride ldw)
__global__ __launch_bounds__(256) void k_pair_antisym_acc(int v, int nc, const cplx* __restrict__ Y,
                                                          cplx* __restrict__ W, i64 ldw, double alpha) {
  const i64 V2 = (i64)v * (v - 1) / 2, total = V2 * nc;
  for (i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (i64)gridDim.x * blockDim.x) {
    const i64 EF = e / nc, X = e % nc;
    int a, b;
    unpair(EF, a, b);
    const cplx y1 = Y[((i64)a * v + b) * nc + X], y2 = Y[((i64)b * v + a) * nc + X];
    cplx* w = W + EF * ldw + X;
    w->x += alpha * (y1.x - y2.x);
    w->y += alpha * (y1.y - y2.y);
  }
}

// dst[e][f][a][b] = W^ef_ab from the packed Wp[EF][AB] (zero on e == f or a == b)
__global__ __launch_bounds__(256) void k_unpack_vvvv(int v, const cplx* __restrict__ Wp, cplx* __restrict__ dst) {
  const i64 V2 = (i64)v * (v - 1) / 2, total = (i64)v * v * v * v;
  for (i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (i64)gridDim.x * blockDim.x) {
    const int b = (int)(e % v), a = (int)(e / v % v), f = (int)(e / ((i64)v * v) % v), ee = (int)(e / ((i64)v * v * v));
    cplx y = make_double2(0.0, 0.0);
    if (ee != f && a != b) {
      const double sg = ((ee > f) == (a > b)) ? 1.0 : -1.0;
      const i64 EF = ee > f ? pair_index(ee, f) : pair_index(f, ee), AB = a > b ? pair_index(a, b) : pair_index(b, a);
      const cplx x = Wp[EF * V2 + AB];
      y = make_double2(sg * x.x, sg * x.y);
    }
    dst[e] = y;
  }
}

// One-body operator folded into a packed pair operator:
//   X[P][Q] += s (d(p1,q1) F[p2][q2] - d(p1,q2) F[p2][q1] - d(p2,q1) F[p1][q2] + d(p2,q2) F[p1][q1])
// for pairs P = (p1 > p2), Q = (q1 > q2) of n indices, X row-major [n2][n2].
// Thread (P, x) updates the pairs Q = {p1, x} (x != p1) and Q = {p2, x}
// (x != p1, p2), which are all the Q that share an index with P, once each.
__global__ __launch_bounds__(256) void k_pair_fold(int n, const cplx* __restrict__ F, cplx* __restrict__ X, double s) {
  const i64 n2 = (i64)n * (n - 1) / 2, total = n2 * n;
  for (i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (i64)gridDim.x * blockDim.x) {
    const i64 P = e / n;
    const int x = (int)(e % n);
    int p1, p2;
    unpair(P, p1, p2);
    auto add = [&](int y, int z) {
      const int q1 = y > z ? y : z, q2 = y > z ? z : y;
      double tr = 0.0, ti = 0.0;
      if (p1 == q1) tr += F[p2 * n + q2].x, ti += F[p2 * n + q2].y;
      if (p1 == q2) tr -= F[p2 * n + q1].x, ti -= F[p2 * n + q1].y;
      if (p2 == q1) tr -= F[p1 * n + q2].x, ti -= F[p1 * n + q2].y;
      if (p2 == q2) tr += F[p1 * n + q1].x, ti += F[p1 * n + q1].y;
      cplx& dst = X[P * n2 + pair_index(q1, q2)];
      dst.x += s * tr;
      dst.y += s * ti;
    };
    if (x != p1) add(p1, x);
    if (x != p1 && x != p2) add(p2, x);
  }
}

// dst[b][P][x] = src[b][p1][p2][x] for P = (p1 > p2): the rows of a leading
// antisymmetric index pair kept once (src [nb][n][n][rest], dst [nb][n2][rest])
__global__ __launch_bounds__(256) void k_pack_first_pair(i64 nb, int n, i64 rest, const cplx* __restrict__ src,
                                                         cplx* __restrict__ dst) {
  const i64 n2 = (i64)n * (n - 1) / 2, total = nb * n2 * rest;
  for (i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (i64)gridDim.x * blockDim.x) {
    const i64 x = e % rest, P = e / rest % n2, b = e / (rest * n2);
    int p1, p2;
    unpair(P, p1, p2);
    dst[e] = src[((b * n + p1) * n + p2) * rest + x];
  }
}

// dst[b][i][j][x] = src[b][IJ][x] (i > j), -src[b][JI][x] (i < j), 0 (i == j):
// a leading packed pair unpacked (src [nb][n2][rest], dst [nb][n][n][rest])
__global__ __launch_bounds__(256) void k_unpack_first_pair(i64 nb, int n, i64 rest, const cplx* __restrict__ src,
                                                           cplx* __restrict__ dst) {
  const i64 n2 = (i64)n * (n - 1) / 2, total = nb * n * n * rest;
  for (i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (i64)gridDim.x * blockDim.x) {
    const i64 x = e % rest, ij = e / rest % ((i64)n * n), b = e / (rest * n * n);
    const int i = (int)(ij / n), j = (int)(ij % n);
    cplx y = make_double2(0.0, 0.0);
    if (i > j) y = src[(b * n2 + pair_index(i, j)) * rest + x];
    else if (i < j) {
      const cplx t = src[(b * n2 + pair_index(j, i)) * rest + x];
      y = make_double2(-t.x, -t.y);
    }
    dst[e] = y;
  }
}

// W[a][m][pair(a,x)] += (a > x ? 1 : -1) F[m][x] for x != a (W [v][o][V2], F [o][v]):
// the singles term -sum_me F^m_e r^ea_im as a v-pair operator, added to the
// pair-packed W^am_ef of the term 1/2 W^am_ef r^ef_im
__global__ __launch_bounds__(256) void k_fold_ov(int o, int v, const cplx* __restrict__ F, cplx* __restrict__ W) {
  const i64 V2 = (i64)v * (v - 1) / 2, total = (i64)v * o * v;
  for (i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (i64)gridDim.x * blockDim.x) {
    const int x = (int)(e % v), m = (int)(e / v % o), a = (int)(e / ((i64)v * o));
    if (x == a) continue;
    const cplx f = F[(i64)m * v + x];
    const double sg = a > x ? 1.0 : -1.0;
    cplx& dst = W[((i64)a * o + m) * V2 + (a > x ? pair_index(a, x) : pair_index(x, a))];
    dst.x += sg * f.x;
    dst.y += sg * f.y;
  }
}
}  // namespace

void launch_fold_ov(int o, int v, const cplx* F, cplx* W, hipStream_t s) {
  const i64 total = (i64)v * o * v;
  if (total <= 0 || v < 2) return;
  hipLaunchKernelGGL(k_fold_ov, dim3(grid_for(total)), dim3(256), 0, s, o, v, F, W);
  HIPCHK(hipGetLastError());
}

void launch_pack_first_pair(i64 nb, int n, i64 rest, const cplx* src, cplx* dst, hipStream_t s) {
  const i64 total = nb * ((i64)n * (n - 1) / 2) * rest;
  if (total <= 0) return;
  hipLaunchKernelGGL(k_pack_first_pair, dim3(grid_for(total)), dim3(256), 0, s, nb, n, rest, src, dst);
  HIPCHK(hipGetLastError());
}

void launch_unpack_first_pair(i64 nb, int n, i64 rest, const cplx* src, cplx* dst, hipStream_t s) {
  const i64 total = nb * n * (i64)n * rest;
  if (total <= 0) return;
  hipLaunchKernelGGL(k_unpack_first_pair, dim3(grid_for(total)), dim3(256), 0, s, nb, n, rest, src, dst);
  HIPCHK(hipGetLastError());
}

void launch_pair_fold(int n, const cplx* F, cplx* X, double alpha, hipStream_t s) {
  const i64 total = (i64)n * (n - 1) / 2 * n;
  if (total <= 0) return;
  hipLaunchKernelGGL(k_pair_fold, dim3(grid_for(total)), dim3(256), 0, s, n, F, X, alpha);
  HIPCHK(hipGetLastError());
}

void launch_pack_pairs(i64 rows, int v, const cplx* src, cplx* dst, hipStream_t s) {
  const i64 total = rows * ((i64)v * (v - 1) / 2);
  if (total <= 0) return;
  hipLaunchKernelGGL(k_pack_pairs, dim3(grid_for(total)), dim3(256), 0, s, rows, v, src, dst);
  HIPCHK(hipGetLastError());
}

void launch_unpack_pairs_acc(i64 rows, int v, const cplx* src, cplx* dst, double alpha, hipStream_t s) {
  const i64 total = rows * ((i64)v * (v - 1) / 2);
  if (total <= 0) return;
  hipLaunchKernelGGL(k_unpack_pairs_acc, dim3(grid_for(total)), dim3(256), 0, s, rows, v, src, dst, alpha);
  HIPCHK(hipGetLastError());
}

void launch_pair_antisym_acc(int v, int nc, const cplx* Y, cplx* W, i64 ldw, double alpha, hipStream_t s) {
  const i64 total = ((i64)v * (v - 1) / 2) * nc;
  if (total <= 0) return;
  hipLaunchKernelGGL(k_pair_antisym_acc, dim3(grid_for(total)), dim3(256), 0, s, v, nc, Y, W, ldw, alpha);
  HIPCHK(hipGetLastError());
}

void launch_unpack_vvvv(int v, const cplx* Wp, cplx* dst, hipStream_t s) {
  const i64 total = (i64)v * v * v * v;
  hipLaunchKernelGGL(k_unpack_vvvv, dim3(grid_for(total)), dim3(256), 0, s, v, Wp, dst);
  HIPCHK(hipGetLastError());
}

