// Device kernels of libcclr for gfx950: strided tensor copies, the packed
// (i>j, a>b) excitation-vector kernels and small helpers of the solver.
#include "internal.h"

namespace {
// --------------------------------------------------------------------------
// Strided tensor copy / accumulate: dst[idx] (+)= alpha * op(src[idx]).
// --------------------------------------------------------------------------
template <typename IT>
__global__ __launch_bounds__(256) void k_tcopy(CopyArgs a) {
  // IT: the index type of the element number and its decomposition (32-bit
  // when the count fits: integer division is several times cheaper)
  const i64 stride = (i64)gridDim.x * blockDim.x;
  for (i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x; e < a.total; e += stride) {
    IT r = (IT)e;
    i64 od = 0, os = 0;
    for (int d = a.nd - 1; d >= 0; --d) {
      const IT n = (IT)a.dim[d], q = r / n, i = r - q * n;
      r = q;
      od += (i64)i * a.sd[d];
      os += (i64)i * a.ss[d];
    }
    cplx y = make_double2(0.0, 0.0);
    if (a.ar != 0.0 || a.ai != 0.0) {  // alpha = 0 writes zeros without reading src
      cplx x = a.src[os];
      if (a.conj) x.y = -x.y;
      y = make_double2(a.ar * x.x - a.ai * x.y, a.ar * x.y + a.ai * x.x);
    }
    if (a.acc) {
      const cplx o = a.dst[od];
      y.x += o.x;
      y.y += o.y;
    }
    a.dst[od] = y;
  }
}

// Transposing form: the source's unit-stride index d0 and the destination's
// unit-stride index d1 are tiled 32 x 32 through LDS, so both the reads and
// the writes are unit-stride runs of 32 elements; the other indices (at most
// four, in a.dim/sd/ss[0 .. a.nd - 1]) are the batch, one per blockIdx.y.
struct TransArgs {
  CopyArgs a;     // batch indices only
  i64 n0, n1;     // extents of d0 and d1
  i64 sd0, ss1;   // destination stride of d0, source stride of d1
  i64 nbatch;
};
__global__ __launch_bounds__(256) void k_tcopy_t(TransArgs t) {
  __shared__ cplx tile[32][33];
  const CopyArgs& a = t.a;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const i64 t0n = (t.n0 + 31) / 32;
  const i64 t0 = blockIdx.x % t0n, t1 = blockIdx.x / t0n;
  const bool rd = a.ar != 0.0 || a.ai != 0.0;
  for (i64 b = blockIdx.y; b < t.nbatch; b += gridDim.y) {
    i64 r = b, od = 0, os = 0;
    for (int d = a.nd - 1; d >= 0; --d) {
      const i64 i = r % a.dim[d];
      r /= a.dim[d];
      od += i * a.sd[d];
      os += i * a.ss[d];
    }
    __syncthreads();  // the previous batch entry's tile has been written out
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const i64 i0 = t0 * 32 + tx, i1 = t1 * 32 + ty + 8 * k;
      cplx x = make_double2(0.0, 0.0);
      if (rd && i0 < t.n0 && i1 < t.n1) x = a.src[os + i0 + i1 * t.ss1];
      tile[ty + 8 * k][tx] = x;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const i64 i1 = t1 * 32 + tx, i0 = t0 * 32 + ty + 8 * k;
      if (i0 >= t.n0 || i1 >= t.n1) continue;
      cplx x = tile[tx][ty + 8 * k];
      if (a.conj) x.y = -x.y;
      cplx y = make_double2(a.ar * x.x - a.ai * x.y, a.ar * x.y + a.ai * x.x);
      cplx* p = a.dst + od + i1 + i0 * t.sd0;
      if (a.acc) {
        const cplx o = *p;
        y.x += o.x;
        y.y += o.y;
      }
      *p = y;
    }
  }
}

__global__ __launch_bounds__(256) void k_fill(cplx* p, i64 n, cplx val) {
  const i64 stride = (i64)gridDim.x * blockDim.x;
  for (i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) p[e] = val;
}

__device__ __forceinline__ i64 pair_index(int hi, int lo) { return (i64)hi * (hi - 1) / 2 + lo; }

// --------------------------------------------------------------------------
// Antisymmetry-aware permutations of packed doubles, tiled through LDS.
// A workgroup takes one occupied pair (i > j) of one vector and one pair of
// 32x32 tiles (A tile >= B tile) of the virtual indices: it reads the packed
// entries of the tile (a > b: row segments a(a-1)/2 + b, unit stride in b)
// once, and writes the four images (i,j,a,b), (j,i,a,b), (i,j,b,a),
// (j,i,b,a) with unit-stride stores, the transposed ones read back from LDS.
// Extra workgroups (y >= O2) write the zero blocks i == j.
// --------------------------------------------------------------------------
constexpr int PT = 32;

__device__ __forceinline__ void tile_pair(int p, int& ta, int& tb) {
  int t = (int)((sqrt(8.0 * p + 1.0) - 1.0) * 0.5);
  while (t * (t + 1) / 2 > p) --t;
  while ((t + 1) * (t + 2) / 2 <= p) ++t;
  ta = t;
  tb = p - t * (t + 1) / 2;
}

__device__ __forceinline__ void occ_pair(i64 P, int& hi, int& lo) {
  int h = (int)((1.0 + sqrt(1.0 + 8.0 * (double)P)) * 0.5);
  while ((i64)h * (h - 1) / 2 > P) --h;
  while ((i64)(h + 1) * h / 2 <= P) ++h;
  hi = h;
  lo = (int)(P - (i64)h * (h - 1) / 2);
}

__device__ __forceinline__ cplx cneg(cplx x) { return make_double2(-x.x, -x.y); }

// RING = false: out[k][p][q][a][b] (full r2); RING = true: out[k][p][a][q][b] (ring layout rr)
template <bool RING>
__global__ __launch_bounds__(256) void k_unpack_t(int o, int v, const cplx* __restrict__ d, cplx* __restrict__ out) {
  __shared__ cplx s[PT][PT + 1];
  const i64 O2 = (i64)o * (o - 1) / 2, V2 = (i64)v * (v - 1) / 2;
  const int k = blockIdx.z, y = blockIdx.y, tid = threadIdx.x;
  int ta, tb;
  tile_pair(blockIdx.x, ta, tb);
  const int a0 = ta * PT, b0 = tb * PT;
  auto off = [&](int p, int q, int a, int b) -> i64 {
    return RING ? ((((i64)k * o + p) * v + a) * o + q) * v + b : ((((i64)k * o + p) * o + q) * v + a) * v + b;
  };
  const cplx zero = make_double2(0.0, 0.0);
  if (y >= O2) {  // i == j: zeros on the tile and its transpose
    const int i = (int)(y - O2);
    for (int e = tid; e < PT * PT; e += 256) {
      const int r = e / PT, c = e % PT;
      if (a0 + r < v && b0 + c < v) out[off(i, i, a0 + r, b0 + c)] = zero;
      if (ta != tb && b0 + r < v && a0 + c < v) out[off(i, i, b0 + r, a0 + c)] = zero;
    }
    return;
  }
  int i, j;
  occ_pair(y, i, j);
  const cplx* __restrict__ dr = d + ((i64)k * O2 + y) * V2;
  for (int e = tid; e < PT * PT; e += 256) {
    const int r = e / PT, c = e % PT, a = a0 + r, b = b0 + c;
    s[r][c] = (a < v && b < v && a > b) ? dr[pair_index(a, b)] : zero;
  }
  __syncthreads();
  for (int e = tid; e < PT * PT; e += 256) {
    const int r = e / PT, c = e % PT, a = a0 + r, b = b0 + c;
    if (a >= v || b >= v) continue;
    // a < b only on a diagonal tile, where s[c][r] holds the entry (b, a)
    const cplx x = a > b ? s[r][c] : (a < b ? cneg(s[c][r]) : zero);
    out[off(i, j, a, b)] = x;
    out[off(j, i, a, b)] = cneg(x);
  }
  if (ta != tb) {
    for (int e = tid; e < PT * PT; e += 256) {
      const int r = e / PT, c = e % PT, b = b0 + r, a = a0 + c;
      if (a >= v || b >= v) continue;
      const cplx x = cneg(s[c][r]);  // entry (b, a) = -(a, b)
      out[off(i, j, b, a)] = x;
      out[off(j, i, b, a)] = cneg(x);
    }
  }
}

// full -> packed (takes the i>j, a>b entries)
__global__ __launch_bounds__(256) void k_pack_full(int nvec, int o, int v, const cplx* __restrict__ r1,
                                                   const cplx* __restrict__ r2, cplx* __restrict__ s,
                                                   cplx* __restrict__ d) {
  const i64 ov = (i64)o * v, O2 = (i64)o * (o - 1) / 2, V2 = (i64)v * (v - 1) / 2;
  const i64 nd = O2 * V2;
  const i64 total = (i64)nvec * (ov + nd);
  const i64 stride = (i64)gridDim.x * blockDim.x;
  for (i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
    const i64 k = e / (ov + nd), q = e % (ov + nd);
    if (q < ov) {
      s[k * ov + q] = r1[k * ov + q];
    } else {
      const i64 p = q - ov, IJ = p / V2, AB = p % V2;
      // invert the pair index
      int i = (int)((1.0 + sqrt(1.0 + 8.0 * (double)IJ)) * 0.5);
      while ((i64)i * (i - 1) / 2 > IJ) --i;
      while ((i64)(i + 1) * i / 2 <= IJ) ++i;
      const int j = (int)(IJ - (i64)i * (i - 1) / 2);
      int a = (int)((1.0 + sqrt(1.0 + 8.0 * (double)AB)) * 0.5);
      while ((i64)a * (a - 1) / 2 > AB) --a;
      while ((i64)(a + 1) * a / 2 <= AB) ++a;
      const int b = (int)(AB - (i64)a * (a - 1) / 2);
      d[k * nd + p] = r2[(((k * o + i) * o + j) * v + a) * v + b];
    }
  }
}

// packed sigma assembly with the antisymmetrizers applied on the fly:
// out += X0 + P(ab) Xa + P(ij) Xi + P(ab)P(ij) Xai - z r (Xa, having no P(ij),
// may hold the pairs i > j only: xa_half, layout [k][IJ][a][b]; Xi, having no
// P(ab), the pairs a > b only: xi_vpacked, layout [k][i][j][AB]).  Doubles: one
// workgroup per (vector, occupied pair i > j, tile pair); the images with
// exchanged virtual indices are read with unit stride along a into LDS.
__global__ __launch_bounds__(256) void k_pack_sigma_t(int o, int v, const cplx* __restrict__ X0,
                                                      const cplx* __restrict__ Xa, const cplx* __restrict__ Xi,
                                                      const cplx* __restrict__ Xai, cplx* __restrict__ outd,
                                                      const cplx* __restrict__ zk, const cplx* __restrict__ rd,
                                                      int xai_ring, int xa_half, int xi_vpacked) {
  __shared__ cplx s[PT][PT + 1];
  const i64 O2 = (i64)o * (o - 1) / 2, V2 = (i64)v * (v - 1) / 2;
  const int k = blockIdx.z, y = blockIdx.y, tid = threadIdx.x;
  int ta, tb, i, j;
  tile_pair(blockIdx.x, ta, tb);
  occ_pair(y, i, j);
  const int a0 = ta * PT, b0 = tb * PT;
  const i64 base = (i64)k * o * o * v * v;
  auto at = [&](int ii, int jj, int aa, int bb) -> i64 { return base + (((i64)ii * o + jj) * v + aa) * v + bb; };
  auto ar = [&](int ii, int jj, int aa, int bb) -> i64 {
    return xai_ring ? base + (((i64)ii * v + aa) * o + jj) * v + bb : at(ii, jj, aa, bb);
  };
  // Xa of the pair i > j only ([k][IJ][a][b]) or full
  auto ah = [&](int aa, int bb) -> i64 {
    return xa_half ? (((i64)k * O2 + y) * v + aa) * v + bb : at(i, j, aa, bb);
  };
  // exchanged-virtual images on rows b, columns a: -Xa(i,j,b,a) - Xai(i,j,b,a) + Xai(j,i,b,a)
  for (int e = tid; e < PT * PT; e += 256) {
    const int r = e / PT, c = e % PT, b = b0 + r, a = a0 + c;
    double tr = 0.0, ti = 0.0;
    if (a < v && b < v) {
      if (Xa) { const cplx u = Xa[ah(b, a)]; tr -= u.x; ti -= u.y; }
      if (Xai) {
        const cplx u = Xai[ar(i, j, b, a)], w = Xai[ar(j, i, b, a)];
        tr += w.x - u.x; ti += w.y - u.y;
      }
    }
    s[r][c] = make_double2(tr, ti);
  }
  __syncthreads();
  const cplx z = zk ? zk[k] : make_double2(0.0, 0.0);
  for (int e = tid; e < PT * PT; e += 256) {
    const int r = e / PT, c = e % PT, a = a0 + r, b = b0 + c;
    if (a >= v || b >= v || a <= b) continue;
    const i64 q = ((i64)k * O2 + y) * V2 + pair_index(a, b);
    cplx t = outd[q];
    const cplx sx = s[c][r];
    t.x += sx.x; t.y += sx.y;
    if (X0) { const cplx u = X0[at(i, j, a, b)]; t.x += u.x; t.y += u.y; }
    if (Xa) { const cplx u = Xa[ah(a, b)]; t.x += u.x; t.y += u.y; }
    if (Xi) {
      const i64 AB = pair_index(a, b);
      const cplx u = xi_vpacked ? Xi[(((i64)k * o + i) * o + j) * V2 + AB] : Xi[at(i, j, a, b)];
      const cplx w = xi_vpacked ? Xi[(((i64)k * o + j) * o + i) * V2 + AB] : Xi[at(j, i, a, b)];
      t.x += u.x - w.x; t.y += u.y - w.y;
    }
    if (Xai) {
      const cplx u = Xai[ar(i, j, a, b)], w = Xai[ar(j, i, a, b)];
      t.x += u.x - w.x; t.y += u.y - w.y;
    }
    if (zk) {
      const cplx x = rd[q];
      t.x -= z.x * x.x - z.y * x.y;
      t.y -= z.x * x.y + z.y * x.x;
    }
    outd[q] = t;
  }
}

// singles: outs += S1 - z r
__global__ __launch_bounds__(256) void k_pack_sigma_s(int nvec, i64 ov, const cplx* __restrict__ S1,
                                                      cplx* __restrict__ outs, const cplx* __restrict__ zk,
                                                      const cplx* __restrict__ rs) {
  const i64 total = (i64)nvec * ov;
  for (i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (i64)gridDim.x * blockDim.x) {
    cplx y = outs[e];
    if (S1) { y.x += S1[e].x; y.y += S1[e].y; }
    if (zk) {
      const cplx z = zk[e / ov], x = rs[e];
      y.x -= z.x * x.x - z.y * x.y;
      y.y -= z.x * x.y + z.y * x.x;
    }
    outs[e] = y;
  }
}

inline unsigned grid_for(i64 total) {
  i64 g = (total + 255) / 256;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (unsigned)g;
}
}  // namespace

void launch_tcopy(const CopyArgs& a0, hipStream_t s) {
  if (a0.total <= 0) return;
  // drop unit extents and merge neighbouring indices that are contiguous in
  // both tensors (fewer divisions per element)
  CopyArgs a = a0;
  a.nd = 0;
  for (int d = 0; d < a0.nd; ++d) {
    if (a0.dim[d] == 1) continue;
    const int k = a.nd - 1;
    if (k >= 0 && a.sd[k] == a0.sd[d] * a0.dim[d] && a.ss[k] == a0.ss[d] * a0.dim[d]) {
      a.dim[k] *= a0.dim[d];
      a.sd[k] = a0.sd[d];
      a.ss[k] = a0.ss[d];
      continue;
    }
    a.dim[a.nd] = a0.dim[d];
    a.sd[a.nd] = a0.sd[d];
    a.ss[a.nd] = a0.ss[d];
    ++a.nd;
  }
  if (a.nd == 0) {  // a single element
    a.nd = 1;
    a.dim[0] = 1;
    a.sd[0] = a.ss[0] = 1;
  }
  // a transpose: the source and the destination have their unit strides on different indices
  int d0 = -1, d1 = -1;
  const bool rd = a.ar != 0.0 || a.ai != 0.0;
  for (int d = 0; d < a.nd; ++d) {
    if (a.ss[d] == 1 && a.dim[d] >= 16) d0 = d;
    if (a.sd[d] == 1 && a.dim[d] >= 16) d1 = d;
  }
  if (rd && d0 >= 0 && d1 >= 0 && d0 != d1) {
    TransArgs t{};
    t.a = a;
    t.a.nd = 0;
    t.nbatch = 1;
    for (int d = 0; d < a.nd; ++d) {
      if (d == d0 || d == d1) continue;
      t.a.dim[t.a.nd] = a.dim[d];
      t.a.sd[t.a.nd] = a.sd[d];
      t.a.ss[t.a.nd] = a.ss[d];
      t.nbatch *= a.dim[d];
      ++t.a.nd;
    }
    t.n0 = a.dim[d0];
    t.n1 = a.dim[d1];
    t.sd0 = a.sd[d0];
    t.ss1 = a.ss[d1];
    const i64 tiles = ((t.n0 + 31) / 32) * ((t.n1 + 31) / 32);
    if (tiles < (1ll << 31)) {
      hipLaunchKernelGGL(k_tcopy_t, dim3((unsigned)tiles, (unsigned)std::min<i64>(t.nbatch, 65535)), dim3(256), 0, s,
                         t);
      HIPCHK(hipGetLastError());
      return;
    }
  }
  if (a.total < (1ll << 31))
    hipLaunchKernelGGL(k_tcopy<unsigned>, dim3(grid_for(a.total)), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(k_tcopy<i64>, dim3(grid_for(a.total)), dim3(256), 0, s, a);
  HIPCHK(hipGetLastError());
}

void launch_fill(cplx* p, i64 n, cplx val, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(256), 0, s, p, n, val);
  HIPCHK(hipGetLastError());
}

static dim3 perm_grid(int nvec, int o, int v, bool diag) {
  const int nt = (v + PT - 1) / PT;
  const i64 rows = (i64)o * (o - 1) / 2 + (diag ? o : 0);
  REQUIRE(nvec <= 65535 && rows <= 65535, CCLR_EINVAL, "too many vectors or occupied pairs for one permutation launch");
  return dim3((unsigned)(nt * (nt + 1) / 2), (unsigned)rows, (unsigned)nvec);
}

void launch_unpack(int nvec, int o, int v, const cplx* s, const cplx* d, cplx* r1, cplx* r2, hipStream_t st) {
  if (nvec <= 0) return;
  if (r1) HIPCHK(hipMemcpyAsync(r1, s, sizeof(cplx) * (size_t)nvec * o * v, hipMemcpyDeviceToDevice, st));
  hipLaunchKernelGGL(k_unpack_t<false>, perm_grid(nvec, o, v, true), dim3(256), 0, st, o, v, d, r2);
  HIPCHK(hipGetLastError());
}

void launch_pack_full(int nvec, int o, int v, const cplx* r1, const cplx* r2, cplx* s, cplx* d, hipStream_t st) {
  const i64 total = (i64)nvec * ((i64)o * v + (i64)o * (o - 1) / 2 * ((i64)v * (v - 1) / 2));
  hipLaunchKernelGGL(k_pack_full, dim3(grid_for(total)), dim3(256), 0, st, nvec, o, v, r1, r2, s, d);
  HIPCHK(hipGetLastError());
}

void launch_pack_sigma(int nvec, int o, int v, const cplx* X0, const cplx* Xa, const cplx* Xi, const cplx* Xai,
                       const cplx* S1, cplx* outs, cplx* outd, const cplx* zk, const cplx* rs, const cplx* rd,
                       hipStream_t st, bool xai_ring, bool xa_half, bool xi_vpacked) {
  if (nvec <= 0) return;
  const i64 ov = (i64)o * v;
  hipLaunchKernelGGL(k_pack_sigma_s, dim3(grid_for((i64)nvec * ov)), dim3(256), 0, st, nvec, ov, S1, outs, zk, rs);
  hipLaunchKernelGGL(k_pack_sigma_t, perm_grid(nvec, o, v, false), dim3(256), 0, st, o, v, X0, Xa, Xi, Xai, outd, zk,
                     rd, xai_ring ? 1 : 0, xa_half ? 1 : 0, xi_vpacked ? 1 : 0);
  HIPCHK(hipGetLastError());
}

void launch_unpack_ring(int nvec, int o, int v, const cplx* d, cplx* rr, hipStream_t st) {
  if (nvec <= 0) return;
  hipLaunchKernelGGL(k_unpack_t<true>, perm_grid(nvec, o, v, true), dim3(256), 0, st, o, v, d, rr);
  HIPCHK(hipGetLastError());
}

// --------------------------------------------------------------------------
// small helpers for the intermediates, the solver and the C ABI
// --------------------------------------------------------------------------
namespace {
__device__ __forceinline__ void unpair(i64 P, int& hi, int& lo) {
  int h = (int)((1.0 + sqrt(1.0 + 8.0 * (double)P)) * 0.5);
  while ((i64)h * (h - 1) / 2 > P) --h;
  while ((i64)(h + 1) * h / 2 <= P) ++h;
  hi = h;
  lo = (int)(P - (i64)h * (h - 1) / 2);
}

// Wp[AB][EF] = W[a][b][e][f], a>b, e>f
__global__ __launch_bounds__(256) void k_pack_vvvv(int v, const cplx* __restrict__ W, cplx* __restrict__ Wp) {
  const i64 V2 = (i64)v * (v - 1) / 2, total = V2 * V2;
  const i64 stride = (i64)gridDim.x * blockDim.x;
  for (i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
    const i64 AB = e / V2, EF = e % V2;
    int a, b, ee, f;
    unpair(AB, a, b);
    unpair(EF, ee, f);
    Wp[e] = W[(((i64)a * v + b) * v + ee) * v + f];
  }
}

__global__ __launch_bounds__(256) void k_diag(int o, int v, const cplx* __restrict__ Foo, const cplx* __restrict__ Fvv,
                                              cplx* __restrict__ diag) {
  const i64 ov = (i64)o * v, O2 = (i64)o * (o - 1) / 2, V2 = (i64)v * (v - 1) / 2;
  const i64 total = ov + O2 * V2;
  const i64 stride = (i64)gridDim.x * blockDim.x;
  for (i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
    cplx y;
    if (e < ov) {
      const int i = (int)(e / v), a = (int)(e % v);
      y = make_double2(Fvv[(i64)a * v + a].x - Foo[(i64)i * o + i].x, Fvv[(i64)a * v + a].y - Foo[(i64)i * o + i].y);
    } else {
      const i64 p = e - ov;
      int i, j, a, b;
      unpair(p / V2, i, j);
      unpair(p % V2, a, b);
      y = make_double2(Fvv[(i64)a * v + a].x + Fvv[(i64)b * v + b].x - Foo[(i64)i * o + i].x - Foo[(i64)j * o + j].x,
                       Fvv[(i64)a * v + a].y + Fvv[(i64)b * v + b].y - Foo[(i64)i * o + i].y - Foo[(i64)j * o + j].y);
    }
    diag[e] = y;
  }
}

__global__ __launch_bounds__(256) void k_check_finite(const cplx* __restrict__ p, i64 n, int* flag) {
  const i64 stride = (i64)gridDim.x * blockDim.x;
  int bad = 0;
  for (i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
    const cplx x = p[e];
    if (!isfinite(x.x) || !isfinite(x.y)) bad = 1;
  }
  if (bad) atomicOr(flag, 1);
}

constexpr int kDotChunks = 256;
// partial[p][chunk] = sum over chunk of x_p * y_p (bilinear, packed vectors; x conjugated if conjx)
__global__ __launch_bounds__(256) void k_bdot(const cplx* const* xs, const cplx* const* xd, const cplx* const* ys,
                                              const cplx* const* yd, i64 ov, i64 nd, cplx* partial, int conjx) {
  const int p = blockIdx.y, chunk = blockIdx.x;
  const i64 n = ov + nd;
  const i64 per = (n + kDotChunks - 1) / kDotChunks;
  const i64 lo = chunk * per, hi = min(n, lo + per);
  double ar = 0.0, ai = 0.0;
  for (i64 e = lo + threadIdx.x; e < hi; e += 256) {
    cplx x = e < ov ? xs[p][e] : xd[p][e - ov];
    const cplx y = e < ov ? ys[p][e] : yd[p][e - ov];
    if (conjx) x.y = -x.y;
    ar += x.x * y.x - x.y * y.y;
    ai += x.x * y.y + x.y * y.x;
  }
  __shared__ double sr[256], si[256];
  sr[threadIdx.x] = ar;
  si[threadIdx.x] = ai;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      sr[threadIdx.x] += sr[threadIdx.x + s];
      si[threadIdx.x] += si[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[(i64)p * kDotChunks + chunk] = make_double2(sr[0], si[0]);
}

__global__ __launch_bounds__(256) void k_bdot_reduce(const cplx* partial, cplx* out) {
  const int p = blockIdx.x;
  double ar = 0.0, ai = 0.0;
  for (int k = threadIdx.x; k < kDotChunks; k += 256) {
    ar += partial[(i64)p * kDotChunks + k].x;
    ai += partial[(i64)p * kDotChunks + k].y;
  }
  __shared__ double sr[256], si[256];
  sr[threadIdx.x] = ar;
  si[threadIdx.x] = ai;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      sr[threadIdx.x] += sr[threadIdx.x + s];
      si[threadIdx.x] += si[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[p] = make_double2(sr[0], si[0]);
}
}  // namespace

void launch_pack_vvvv(int v, const cplx* W, cplx* Wp, hipStream_t s) {
  const i64 V2 = (i64)v * (v - 1) / 2;
  hipLaunchKernelGGL(k_pack_vvvv, dim3(grid_for(V2 * V2)), dim3(256), 0, s, v, W, Wp);
  HIPCHK(hipGetLastError());
}

void launch_diag(int o, int v, const cplx* Foo, const cplx* Fvv, cplx* diag, hipStream_t s) {
  const i64 total = (i64)o * v + (i64)o * (o - 1) / 2 * ((i64)v * (v - 1) / 2);
  hipLaunchKernelGGL(k_diag, dim3(grid_for(total)), dim3(256), 0, s, o, v, Foo, Fvv, diag);
  HIPCHK(hipGetLastError());
}

void launch_check_finite(const cplx* p, i64 n, int* flag, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_check_finite, dim3(grid_for(n)), dim3(256), 0, s, p, n, flag);
  HIPCHK(hipGetLastError());
}

// out[p] = sum x_p y_p for npair packed-vector pairs given by device pointer arrays
void launch_bdot(int npair, const cplx* const* xs, const cplx* const* xd, const cplx* const* ys,
                 const cplx* const* yd, i64 ov, i64 nd, cplx* partial, cplx* out, hipStream_t s, bool conjx) {
  if (npair <= 0) return;
  hipLaunchKernelGGL(k_bdot, dim3(kDotChunks, npair), dim3(256), 0, s, xs, xd, ys, yd, ov, nd, partial, (int)conjx);
  hipLaunchKernelGGL(k_bdot_reduce, dim3(npair), dim3(256), 0, s, partial, out);
  HIPCHK(hipGetLastError());
}

namespace {
__global__ __launch_bounds__(256) void k_caxpy(i64 n, cplx a, const cplx* __restrict__ x, cplx* __restrict__ y) {
  for (i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (i64)gridDim.x * blockDim.x) {
    const cplx u = x[e];
    y[e].x += a.x * u.x - a.y * u.y;
    y[e].y += a.x * u.y + a.y * u.x;
  }
}
__global__ __launch_bounds__(256) void k_conj(i64 n, cplx* x) {
  for (i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (i64)gridDim.x * blockDim.x) x[e].y = -x[e].y;
}
}  // namespace

void launch_caxpy(i64 n, cplx a, const cplx* x, cplx* y, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_caxpy, dim3(grid_for(n)), dim3(256), 0, s, n, a, x, y);
  HIPCHK(hipGetLastError());
}

void launch_conj_inplace(i64 n, cplx* x, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_conj, dim3(grid_for(n)), dim3(256), 0, s, n, x);
  HIPCHK(hipGetLastError());
}
