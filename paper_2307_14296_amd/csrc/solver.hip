// Davidson-type subspace solver for the damped response and Lambda
// equations (SI, "Davidson scheme for solving first-order response
// equation"), device resident in FP64.
//
// Per right-hand side: orthonormal trial vectors b_j and their transforms
// s_j = (A - z) b_j (or b_j (A - z) for the left problem).  The projected
// system G' beta = -C' with G'_ij = <b_i, s_j>, C'_j = <b_j, xi> is solved by
// LU with partial pivoting on the device; the residual is
// R = sum_j beta_j s_j + xi; the correction (z - D)^-1 R is orthogonalized
// against {b} by classical Gram-Schmidt (a second pass where the first
// removed more than half of its squared norm) and appended.  The
// start vector is the unit vector on the largest |xi| component.  When the
// subspace is full it restarts from the current solution.  All right-hand
// sides advance in lockstep so each Jacobian transform is batched.
#include <algorithm>
#include <chrono>
#include <cmath>

#include "internal.h"
#include "eigen_small.h"

namespace {
constexpr int kThreads = 256;
constexpr int kChunks = 512;

// vector (r, j) of a set with R slots per right-hand side
struct VS {
  cplx* s;
  cplx* d;
  int R;
};

__device__ __forceinline__ const cplx* vs_s(const VS& v, int r, int j, i64 ov) { return v.s + ((i64)r * v.R + j) * ov; }
__device__ __forceinline__ const cplx* vs_d(const VS& v, int r, int j, i64 nd) { return v.d + ((i64)r * v.R + j) * nd; }

__device__ __forceinline__ cplx cmul(cplx a, cplx b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ __forceinline__ cplx cconjmul(cplx a, cplx b) { return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x); }

__device__ cplx block_sum(cplx v) {
  __shared__ double sr[kThreads], si[kThreads];
  sr[threadIdx.x] = v.x;
  si[threadIdx.x] = v.y;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      sr[threadIdx.x] += sr[threadIdx.x + s];
      si[threadIdx.x] += si[threadIdx.x + s];
    }
    __syncthreads();
  }
  cplx out = make_double2(sr[0], si[0]);
  __syncthreads();
  return out;
}

// partial[(a*nj + j)*kChunks + chunk] = sum over chunk of conj(X[r][xj0+j]) * Y[r][yj],  r = act[a].
// One block takes kGramJ consecutive j, so each element of Y is read once for up to kGramJ vectors of X.
constexpr int kGramJ = 4;
__global__ __launch_bounds__(kThreads) void k_gram(VS X, int xj0, int nj, VS Y, int yj, const int* act, i64 ov, i64 nd,
                                                   cplx* partial) {
  const int a = blockIdx.z, j0 = blockIdx.y * kGramJ, chunk = blockIdx.x;
  const int cnt = min(kGramJ, nj - j0);
  const int r = act[a];
  const cplx* xs[kGramJ];
  const cplx* xd[kGramJ];
  for (int q = 0; q < kGramJ; ++q) {
    const int j = xj0 + j0 + min(q, cnt - 1);
    xs[q] = vs_s(X, r, j, ov);
    xd[q] = vs_d(X, r, j, nd);
  }
  const cplx* ys = vs_s(Y, r, yj, ov);
  const cplx* yd = vs_d(Y, r, yj, nd);
  const i64 n = ov + nd;
  const i64 per = (n + kChunks - 1) / kChunks;
  const i64 lo = chunk * per, hi = min(n, lo + per);
  double accr[kGramJ], acci[kGramJ];
  for (int q = 0; q < kGramJ; ++q) accr[q] = acci[q] = 0.0;
  for (i64 e = lo + threadIdx.x; e < hi; e += kThreads) {
    const bool single = e < ov;
    const cplx y = single ? ys[e] : yd[e - ov];
#pragma unroll
    for (int q = 0; q < kGramJ; ++q) {
      if (q < cnt) {
        const cplx x = single ? xs[q][e] : xd[q][e - ov];
        const cplx p = cconjmul(x, y);
        accr[q] += p.x;
        acci[q] += p.y;
      }
    }
  }
  // wave sums by lane exchange, then the four waves through LDS
  __shared__ double ws[kThreads / 64][2 * kGramJ];
#pragma unroll
  for (int q = 0; q < kGramJ; ++q) {
    for (int off = 32; off > 0; off >>= 1) {
      accr[q] += __shfl_xor(accr[q], off, 64);
      acci[q] += __shfl_xor(acci[q], off, 64);
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    for (int q = 0; q < kGramJ; ++q) {
      ws[wave][2 * q] = accr[q];
      ws[wave][2 * q + 1] = acci[q];
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < cnt) {
    const int q = threadIdx.x;
    cplx t = make_double2(0.0, 0.0);
    for (int w = 0; w < kThreads / 64; ++w) {
      t.x += ws[w][2 * q];
      t.y += ws[w][2 * q + 1];
    }
    partial[((i64)a * nj + j0 + q) * kChunks + chunk] = t;
  }
}

// out[r*ld + col0 + j] = sum of the chunk partials (conjugated if cj)
__global__ __launch_bounds__(kThreads) void k_reduce(const cplx* partial, int nj, const int* act, cplx* out, int ld,
                                                     int col0, int cj) {
  const int p = blockIdx.x;
  cplx acc = make_double2(0.0, 0.0);
  for (int k = threadIdx.x; k < kChunks; k += kThreads) {
    acc.x += partial[(i64)p * kChunks + k].x;
    acc.y += partial[(i64)p * kChunks + k].y;
  }
  acc = block_sum(acc);
  if (threadIdx.x == 0) {
    const int a = p / nj, j = p % nj;
    if (cj) acc.y = -acc.y;
    out[(i64)act[a] * ld + col0 + j] = acc;
  }
}

// out[r][oj] = (acc ? out : 0) + sign * sum_j coef[r][j] X[r][xj0 + j] + (use_y ? Y[r][yj] : 0)
__global__ __launch_bounds__(kThreads) void k_lincomb(VS out, int oj, VS X, int xj0, int nj, const cplx* coef, int ldc,
                                                      double sign, VS Y, int yj, int use_y, int acc_out,
                                                      const int* act, i64 ov, i64 nd) {
  __shared__ cplx c[128];
  const int a = blockIdx.y, r = act[a];
  for (int j = threadIdx.x; j < nj; j += kThreads) {
    const cplx t = coef[(i64)r * ldc + j];
    c[j] = make_double2(sign * t.x, sign * t.y);
  }
  __syncthreads();
  const i64 n = ov + nd;
  cplx* os = (cplx*)vs_s(out, r, oj, ov);
  cplx* od = (cplx*)vs_d(out, r, oj, nd);
  for (i64 e = (i64)blockIdx.x * kThreads + threadIdx.x; e < n; e += (i64)gridDim.x * kThreads) {
    cplx y = make_double2(0.0, 0.0);
    if (acc_out) y = e < ov ? os[e] : od[e - ov];
    // four loads in flight per thread (the loop is latency-bound otherwise)
#pragma unroll 4
    for (int j = 0; j < nj; ++j) {
      const cplx x = e < ov ? vs_s(X, r, xj0 + j, ov)[e] : vs_d(X, r, xj0 + j, nd)[e - ov];
      const cplx p = cmul(c[j], x);
      y.x += p.x;
      y.y += p.y;
    }
    if (use_y) {
      const cplx x = e < ov ? vs_s(Y, r, yj, ov)[e] : vs_d(Y, r, yj, nd)[e - ov];
      y.x += x.x;
      y.y += x.y;
    }
    if (e < ov) os[e] = y;
    else od[e - ov] = y;
  }
}

// out[r][oj] = X[r][xj] * f,  f = 1/(z_r - D) (mode 0) or 1/sqrt(Re nrm2[r]) (mode 1)
__global__ __launch_bounds__(kThreads) void k_scale(VS out, int oj, VS X, int xj, const cplx* z, const cplx* diag,
                                                    const cplx* nrm2, int mode, const int* act, i64 ov, i64 nd) {
  const int a = blockIdx.y, r = act[a];
  const i64 n = ov + nd;
  cplx* os = (cplx*)vs_s(out, r, oj, ov);
  cplx* od = (cplx*)vs_d(out, r, oj, nd);
  const cplx* xs = vs_s(X, r, xj, ov);
  const cplx* xd = vs_d(X, r, xj, nd);
  const double f = mode == 1 ? 1.0 / sqrt(nrm2[r].x) : 0.0;
  for (i64 e = (i64)blockIdx.x * kThreads + threadIdx.x; e < n; e += (i64)gridDim.x * kThreads) {
    const cplx x = e < ov ? xs[e] : xd[e - ov];
    cplx y;
    if (mode == 0) {
      const cplx dd = diag[e];
      const cplx w = make_double2(z[r].x - dd.x, z[r].y - dd.y);
      const double den = w.x * w.x + w.y * w.y;
      y = make_double2((x.x * w.x + x.y * w.y) / den, (x.y * w.x - x.x * w.y) / den);
    } else {
      y = make_double2(x.x * f, x.y * f);
    }
    if (e < ov) os[e] = y;
    else od[e - ov] = y;
  }
}

// unit vector on the largest |X[r]| entry (first index on ties); one block per right-hand side
__global__ __launch_bounds__(kThreads) void k_pivot(VS out, VS X, const int* act, i64 ov, i64 nd) {
  const int a = blockIdx.x, r = act[a];
  const cplx* xs = vs_s(X, r, 0, ov);
  const cplx* xd = vs_d(X, r, 0, nd);
  const i64 n = ov + nd;
  double best = -1.0;
  i64 bi = 0;
  for (i64 e = threadIdx.x; e < n; e += kThreads) {
    const cplx x = e < ov ? xs[e] : xd[e - ov];
    const double m = x.x * x.x + x.y * x.y;
    if (m > best) { best = m; bi = e; }
  }
  __shared__ double sb[kThreads];
  __shared__ i64 si[kThreads];
  sb[threadIdx.x] = best;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      const double ob = sb[threadIdx.x + s];
      const i64 oi = si[threadIdx.x + s];
      if (ob > sb[threadIdx.x] || (ob == sb[threadIdx.x] && oi < si[threadIdx.x])) {
        sb[threadIdx.x] = ob;
        si[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  const i64 p = si[0];
  cplx* os = (cplx*)vs_s(out, r, 0, ov);
  cplx* od = (cplx*)vs_d(out, r, 0, nd);
  for (i64 e = threadIdx.x; e < n; e += kThreads) {
    const cplx y = make_double2(e == p ? 1.0 : 0.0, 0.0);
    if (e < ov) os[e] = y;
    else od[e - ov] = y;
  }
}

// Solve G[r] beta[r] = -C[r] (order m, leading dim ld) by Gaussian
// elimination with partial pivoting; one block per active right-hand side.
// W is scratch [nact][ld][ld+1].
__global__ __launch_bounds__(kThreads) void k_small_solve(const cplx* G, const cplx* C, int m, int ld, cplx* W,
                                                          cplx* beta, int* singular, const int* act) {
  const int a = blockIdx.x, r = act[a];
  const int lw = ld + 1;
  cplx* M = W + (i64)a * ld * lw;
  for (int e = threadIdx.x; e < m * (m + 1); e += kThreads) {
    const int i = e / (m + 1), j = e % (m + 1);
    cplx x = j < m ? G[((i64)r * ld + i) * ld + j] : C[(i64)r * ld + i];
    if (j == m) { x.x = -x.x; x.y = -x.y; }
    M[i * lw + j] = x;
  }
  __syncthreads();
  __shared__ int piv;
  for (int k = 0; k < m; ++k) {
    if (threadIdx.x == 0) {
      double best = -1.0;
      int bi = k;
      for (int i = k; i < m; ++i) {
        const cplx x = M[i * lw + k];
        const double mag = x.x * x.x + x.y * x.y;
        if (mag > best) { best = mag; bi = i; }
      }
      piv = bi;
      if (best == 0.0) singular[r] = 1;
    }
    __syncthreads();
    const int p = piv;
    if (p != k)
      for (int j = threadIdx.x; j <= m; j += kThreads) {
        const cplx t = M[k * lw + j];
        M[k * lw + j] = M[p * lw + j];
        M[p * lw + j] = t;
      }
    __syncthreads();
    const cplx d = M[k * lw + k];
    const double den = d.x * d.x + d.y * d.y;
    const int w = m - k;  // columns k+1 .. m (m = right-hand side column)
    for (int e = threadIdx.x; e < (m - k - 1) * w; e += kThreads) {
      const int i = k + 1 + e / w, j = k + 1 + e % w;
      const cplx lik = M[i * lw + k];
      const cplx f = make_double2((lik.x * d.x + lik.y * d.y) / den, (lik.y * d.x - lik.x * d.y) / den);
      const cplx mkj = M[k * lw + j];
      M[i * lw + j].x -= f.x * mkj.x - f.y * mkj.y;
      M[i * lw + j].y -= f.x * mkj.y + f.y * mkj.x;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    for (int i = m - 1; i >= 0; --i) {
      cplx s = M[i * lw + m];
      for (int j = i + 1; j < m; ++j) {
        const cplx b = beta[(i64)r * ld + j];
        const cplx g = M[i * lw + j];
        s.x -= g.x * b.x - g.y * b.y;
        s.y -= g.x * b.y + g.y * b.x;
      }
      const cplx d = M[i * lw + i];
      const double den = d.x * d.x + d.y * d.y;
      beta[(i64)r * ld + i] = make_double2((s.x * d.x + s.y * d.y) / den, (s.y * d.x - s.x * d.y) / den);
    }
  }
}

// G[r][row q][j] = vals[r][j] (as_row) or G[r][j][col q] = vals[r][j]
__global__ void k_put(const cplx* vals, int nj, cplx* G, int ld, int q, int as_row, const int* act) {
  const int r = act[blockIdx.x];
  for (int j = threadIdx.x; j < nj; j += blockDim.x) {
    const cplx x = vals[(i64)r * ld + j];
    if (as_row) G[((i64)r * ld + q) * ld + j] = x;
    else G[((i64)r * ld + j) * ld + q] = x;
  }
}

unsigned vgrid(i64 n) {
  i64 g = (n + kThreads - 1) / kThreads;
  if (g > 2048) g = 2048;
  return (unsigned)std::max<i64>(g, 1);
}
}  // namespace

// --------------------------------------------------------------- driver
// Davidson solve of (A - z_r) x_r = -rhs_r (right) or x_r (A - z_r) = -rhs_r
// (left) for nr right-hand sides in lockstep.
//
// lowp != CCLR_FP64 selects iterative refinement with subspace recycling:
// the trial vectors are transformed with reduced-precision ladder and ring
// products; when a right-hand side's projected residual falls below
// inner_tol relative to its current right-hand side, its solution is
// accumulated, the true residual R = (A - z) x + rhs is formed with FP64
// transforms, and if ||R|| > tol ||rhs|| the same subspace continues on the
// correction equation with right-hand side R (only the projected right-hand
// side C' is recomputed).  Residual norms, orthogonalisation and the
// projected system are FP64 throughout.
int davidson(cclr_ctx* c, int side, int nr, const cplx* zh, const VecSet& rhs, const VecSet& xout,
             cclr_solve_info* info, double tol, int maxit_in, int lowp, double inner_tol) {
  auto t0 = std::chrono::steady_clock::now();
  const bool refine = lowp != CCLR_FP64;
  const i64 ov = c->ns(), nd = c->nd(), n = ov + nd;
  const int ms = std::max(4, std::min(c->opt.max_subspace, 120));
  hipStream_t st = c->stream;
  Arena::Mark mk = c->arena.mark();
  auto vbuf = [&](int nvec) {
    VecSet v;
    v.s = (cplx*)c->arena.get(sizeof(cplx) * (size_t)(nvec * ov));
    v.d = (cplx*)c->arena.get(sizeof(cplx) * (size_t)(nvec * nd));
    v.n = nvec;
    return v;
  };
  VecSet Bv = vbuf(nr * ms), Sv = vbuf(nr * ms), Rv = vbuf(nr), Ev = vbuf(nr), Xin = vbuf(nr), Xout = vbuf(nr);
  VecSet Yv = vbuf(nr);                      // restart scratch
  VecSet RCv = refine ? vbuf(nr) : rhs;      // current right-hand side (the true residual after refinement)
  const VS B{Bv.s, Bv.d, ms}, S{Sv.s, Sv.d, ms}, R{Rv.s, Rv.d, 1}, E{Ev.s, Ev.d, 1};
  const VS XI{RCv.s, RCv.d, 1}, X0{rhs.s, rhs.d, 1}, XO{xout.s, xout.d, 1}, T{Xout.s, Xout.d, 1};
  const VS YT{Yv.s, Yv.d, 1};
  if (refine) {
    HIPCHK(hipMemcpyAsync(RCv.s, rhs.s, sizeof(cplx) * (size_t)nr * ov, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(RCv.d, rhs.d, sizeof(cplx) * (size_t)nr * nd, hipMemcpyDeviceToDevice, st));
  }
  cplx* G = (cplx*)c->arena.get(sizeof(cplx) * (size_t)nr * ms * ms);
  cplx* Cp = (cplx*)c->arena.get(sizeof(cplx) * (size_t)nr * ms);
  cplx* beta = (cplx*)c->arena.get(sizeof(cplx) * (size_t)nr * ms);
  cplx* coef = (cplx*)c->arena.get(sizeof(cplx) * (size_t)nr * ms);
  cplx* tmpv = (cplx*)c->arena.get(sizeof(cplx) * (size_t)nr * ms);
  cplx* W = (cplx*)c->arena.get(sizeof(cplx) * (size_t)nr * ms * (ms + 1));
  cplx* partial = (cplx*)c->arena.get(sizeof(cplx) * (size_t)nr * ms * kChunks);
  int* act_d = (int*)c->arena.get(sizeof(int) * nr);
  int* sing_d = (int*)c->arena.get(sizeof(int) * nr);
  cplx* z_d = (cplx*)c->arena.get(sizeof(cplx) * nr);     // by right-hand side
  cplx* za_d = (cplx*)c->arena.get(sizeof(cplx) * nr);    // by active position (for the transform)
  launch_fill(G, (i64)nr * ms * ms, cx(0.0), st);
  HIPCHK(hipMemsetAsync(sing_d, 0, sizeof(int) * nr, st));
  HIPCHK(hipMemcpyAsync(z_d, zh, sizeof(cplx) * nr, hipMemcpyHostToDevice, st));

  int na = 0;
  // out[r*ld + col0 + j] = <X[r][xj0+j], Y[r][yj]> for active r
  auto gram = [&](VS X, int xj0, int nj, VS Y, int yj, cplx* out, int ld, int col0, int cj) {
    if (nj <= 0 || na <= 0) return;
    hipLaunchKernelGGL(k_gram, dim3(kChunks, (nj + kGramJ - 1) / kGramJ, na), dim3(kThreads), 0, st, X, xj0, nj, Y,
                       yj, act_d, ov, nd, partial);
    hipLaunchKernelGGL(k_reduce, dim3(na * nj), dim3(kThreads), 0, st, partial, nj, act_d, out, ld, col0, cj);
  };
  auto lincomb = [&](VS out, int oj, VS X, int xj0, int nj, const cplx* cf, int ldc, double sign, VS Y, int yj,
                     int use_y, int acc) {
    hipLaunchKernelGGL(k_lincomb, dim3(vgrid(n), na), dim3(kThreads), 0, st, out, oj, X, xj0, nj, cf, ldc, sign, Y,
                       yj, use_y, acc, act_d, ov, nd);
  };
  auto scale = [&](VS out, int oj, VS X, int xj, const cplx* nrm2, int mode) {
    hipLaunchKernelGGL(k_scale, dim3(vgrid(n), na), dim3(kThreads), 0, st, out, oj, X, xj, z_d, c->diag.c(), nrm2,
                       mode, act_d, ov, nd);
  };
  auto fetch = [&](const cplx* src, std::vector<cplx>& h, int ld) {
    h.resize((size_t)nr * ld);
    HIPCHK(hipMemcpyAsync(h.data(), src, sizeof(cplx) * (size_t)nr * ld, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
  };
  std::vector<int> act;
  auto set_active = [&](const std::vector<int>& a2) {
    act = a2;
    na = (int)act.size();
    if (!na) return;
    HIPCHK(hipMemcpyAsync(act_d, act.data(), sizeof(int) * na, hipMemcpyHostToDevice, st));
    std::vector<cplx> za(na);
    for (int a = 0; a < na; ++a) za[a] = zh[act[a]];
    HIPCHK(hipMemcpyAsync(za_d, za.data(), sizeof(cplx) * na, hipMemcpyHostToDevice, st));
  };

  std::vector<int> all(nr);
  for (int r = 0; r < nr; ++r) all[r] = r;
  set_active(all);
  std::vector<cplx> hv;
  gram(XI, 0, 1, XI, 0, tmpv, 1, 0, 0);
  fetch(tmpv, hv, 1);
  std::vector<double> xinorm(nr), rcnorm(nr), res(nr, 0.0);
  std::vector<int> msub(nr, 0), done(nr, 0), outer(nr, 0), accumulated(nr, 0);
  for (int r = 0; r < nr; ++r) {
    xinorm[r] = rcnorm[r] = std::sqrt(hv[r].x);
    if (xinorm[r] == 0.0) done[r] = 1, accumulated[r] = 1;  // x = 0
  }
  const int max_outer = 12;
  launch_fill(xout.s, (i64)nr * ov, cx(0.0), st);
  launch_fill(xout.d, (i64)nr * nd, cx(0.0), st);
  {
    std::vector<int> a2;
    for (int r = 0; r < nr; ++r)
      if (!done[r]) a2.push_back(r);
    set_active(a2);
  }
  if (na) hipLaunchKernelGGL(k_pivot, dim3(na), dim3(kThreads), 0, st, B, XI, act_d, ov, nd);

  int j = 0;  // slot of the newest trial vector, shared by the active right-hand sides
  int iters = 0;
  long nsigma = 0;
  auto sigma = (side == CCLR_RIGHT) ? sigma_right : sigma_left;
  const int maxit = std::max(1, maxit_in);
  c->sigma_prec = lowp;
  // projected solve and residual R = sum_i beta_i s_i + rhs_cur for the active set; returns the
  // relative residual of each active right-hand side (by rhs index)
  auto project = [&](int m) {
    hipLaunchKernelGGL(k_small_solve, dim3(na), dim3(kThreads), 0, st, G, Cp, m, ms, W, beta, sing_d, act_d);
    lincomb(R, 0, S, 0, m, beta, ms, 1.0, XI, 0, 1, 0);
    gram(R, 0, 1, R, 0, tmpv, 1, 0, 0);
    fetch(tmpv, hv, 1);
  };
  // x += sum beta b, then the FP64 true residual into the current right-hand side
  auto refine_step = [&](const std::vector<int>& cand, int m) {
    set_active(cand);
    lincomb(XO, 0, B, 0, m, beta, ms, 1.0, XO, 0, 0, 1);
    for (int a = 0; a < na; ++a) {
      const int r = act[a];
      HIPCHK(hipMemcpyAsync(Xin.s + a * ov, xout.s + (i64)r * ov, sizeof(cplx) * ov, hipMemcpyDeviceToDevice, st));
      HIPCHK(hipMemcpyAsync(Xin.d + a * nd, xout.d + (i64)r * nd, sizeof(cplx) * nd, hipMemcpyDeviceToDevice, st));
    }
    VecSet vin = Xin, vout = Xout;
    vin.n = vout.n = na;
    c->sigma_prec = CCLR_FP64;
    sigma(c, vin, vout, za_d);
    c->sigma_prec = lowp;
    nsigma += na;
    for (int a = 0; a < na; ++a) {
      const int r = act[a];
      HIPCHK(hipMemcpyAsync(RCv.s + (i64)r * ov, Xout.s + a * ov, sizeof(cplx) * ov, hipMemcpyDeviceToDevice, st));
      HIPCHK(hipMemcpyAsync(RCv.d + (i64)r * nd, Xout.d + a * nd, sizeof(cplx) * nd, hipMemcpyDeviceToDevice, st));
    }
    lincomb(XI, 0, B, 0, 0, beta, ms, 1.0, X0, 0, 1, 1);  // rhs_cur = (A - z) x + rhs
    gram(XI, 0, 1, XI, 0, tmpv, 1, 0, 0);
    fetch(tmpv, hv, 1);
  };
  while (na > 0) {
    // batched transform of the newest trial vectors
    for (int a = 0; a < na; ++a) {
      const int r = act[a];
      HIPCHK(hipMemcpyAsync(Xin.s + a * ov, Bv.s + ((i64)r * ms + j) * ov, sizeof(cplx) * ov, hipMemcpyDeviceToDevice, st));
      HIPCHK(hipMemcpyAsync(Xin.d + a * nd, Bv.d + ((i64)r * ms + j) * nd, sizeof(cplx) * nd, hipMemcpyDeviceToDevice, st));
    }
    VecSet vin = Xin, vout = Xout;
    vin.n = vout.n = na;
    sigma(c, vin, vout, za_d);
    nsigma += na;
    for (int a = 0; a < na; ++a) {
      const int r = act[a];
      HIPCHK(hipMemcpyAsync(Sv.s + ((i64)r * ms + j) * ov, Xout.s + a * ov, sizeof(cplx) * ov, hipMemcpyDeviceToDevice, st));
      HIPCHK(hipMemcpyAsync(Sv.d + ((i64)r * ms + j) * nd, Xout.d + a * nd, sizeof(cplx) * nd, hipMemcpyDeviceToDevice, st));
    }
    ++iters;
    // extend the projected matrix by column j, row j and C'_j
    gram(B, 0, j + 1, S, j, tmpv, ms, 0, 0);  // <b_i, s_j>
    hipLaunchKernelGGL(k_put, dim3(na), dim3(128), 0, st, tmpv, j + 1, G, ms, j, 0, act_d);
    if (j > 0) {
      gram(S, 0, j, B, j, tmpv, ms, 0, 1);    // conj <s_i, b_j> = <b_j, s_i>
      hipLaunchKernelGGL(k_put, dim3(na), dim3(128), 0, st, tmpv, j, G, ms, j, 1, act_d);
    }
    gram(B, j, 1, XI, 0, Cp, ms, j, 0);       // C'_j = <b_j, rhs_cur>
    const int m = j + 1;
    project(m);
    std::vector<int> still, cand;
    for (int a = 0; a < na; ++a) {
      const int r = act[a];
      const double rin = std::sqrt(std::max(hv[r].x, 0.0)) / rcnorm[r];
      res[r] = rin * rcnorm[r] / xinorm[r];
      msub[r] = m;
      if (!std::isfinite(res[r])) done[r] = 1;
      else if (!refine && res[r] <= tol) done[r] = 1;
      else if (refine && (rin <= inner_tol || res[r] <= tol)) cand.push_back(r);
      else still.push_back(r);
    }
    // refinement: accumulate, FP64 residual, continue on the correction equation in the same subspace
    while (!cand.empty()) {
      refine_step(cand, m);
      std::vector<int> again;
      for (int r : cand) {
        const double tn = std::sqrt(std::max(hv[r].x, 0.0));
        res[r] = tn / xinorm[r];
        ++outer[r];
        if (res[r] <= tol || !std::isfinite(res[r]) || outer[r] >= max_outer) {
          done[r] = 1;
          accumulated[r] = 1;
        } else {
          rcnorm[r] = tn;
          again.push_back(r);
        }
      }
      if (again.empty()) break;
      set_active(again);
      gram(B, 0, m, XI, 0, Cp, ms, 0, 0);     // C' for the new right-hand side
      project(m);
      cand.clear();
      for (int r : again) {
        const double rin = std::sqrt(std::max(hv[r].x, 0.0)) / rcnorm[r];
        if (rin <= inner_tol) cand.push_back(r);
        else still.push_back(r);
      }
    }
    if (still.empty() || iters >= maxit) break;
    std::sort(still.begin(), still.end());
    set_active(still);
    // correction (z - D)^-1 R
    scale(E, 0, R, 0, nullptr, 0);
    int nj = m;
    if (m == ms) {
      // restart from the current solution: b0 = x/|x|, s0 = (sum beta s)/|x|
      lincomb(YT, 0, B, 0, m, beta, ms, 1.0, YT, 0, 0, 0);
      lincomb(T, 0, S, 0, m, beta, ms, 1.0, T, 0, 0, 0);
      gram(YT, 0, 1, YT, 0, tmpv, 1, 0, 0);
      scale(B, 0, YT, 0, tmpv, 1);
      scale(S, 0, T, 0, tmpv, 1);
      gram(B, 0, 1, S, 0, tmpv, ms, 0, 0);
      hipLaunchKernelGGL(k_put, dim3(na), dim3(128), 0, st, tmpv, 1, G, ms, 0, 0, act_d);
      gram(B, 0, 1, XI, 0, Cp, ms, 0, 0);
      nj = 1;
    }
    // classical Gram-Schmidt against the orthonormal subspace, with a second
    // pass only for the right-hand sides whose correction lost more than half
    // of its squared norm in the first (|e'|^2 = |e|^2 - sum |c_i|^2): a
    // vector that is not nearly inside the subspace is orthogonal to working
    // accuracy after one pass (Daniel, Gragg, Kaufman and Stewart's criterion)
    gram(E, 0, 1, E, 0, tmpv, 1, 0, 0);
    gram(B, 0, nj, E, 0, coef, ms, 0, 0);
    lincomb(E, 0, B, 0, nj, coef, ms, -1.0, E, 0, 0, 1);
    {
      std::vector<cplx> ch((size_t)nr * ms), nh(nr);
      HIPCHK(hipMemcpyAsync(ch.data(), coef, sizeof(cplx) * ch.size(), hipMemcpyDeviceToHost, st));
      HIPCHK(hipMemcpyAsync(nh.data(), tmpv, sizeof(cplx) * nr, hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      std::vector<int> again;
      for (int r : act) {
        double p = 0.0;
        for (int i = 0; i < nj; ++i) {
          const cplx x = ch[(size_t)r * ms + i];
          p += x.x * x.x + x.y * x.y;
        }
        if (!(p <= 0.5 * nh[r].x)) again.push_back(r);
      }
      if (!again.empty()) {
        const std::vector<int> keep = act;
        set_active(again);
        gram(B, 0, nj, E, 0, coef, ms, 0, 0);
        lincomb(E, 0, B, 0, nj, coef, ms, -1.0, E, 0, 0, 1);
        set_active(keep);
      }
    }
    gram(E, 0, 1, E, 0, tmpv, 1, 0, 0);
    j = nj;
    scale(B, j, E, 0, tmpv, 1);
  }
  // solutions x_r = sum_i beta_i b_i over each right-hand side's final subspace
  // (added to the accumulated solution when refining)
  for (int r = 0; r < nr; ++r) {
    if (msub[r] == 0 || accumulated[r]) continue;
    std::vector<int> one{r};
    set_active(one);
    lincomb(XO, 0, B, 0, msub[r], beta, ms, 1.0, XO, 0, 0, refine ? 1 : 0);
  }
  c->sigma_prec = CCLR_FP64;
  // conditioning estimate: Ritz values of (A - z) on each final subspace
  double kappa = 0.0, ritz_min = 0.0;
  {
    std::vector<cplx> Gh((size_t)nr * ms * ms);
    HIPCHK(hipMemcpyAsync(Gh.data(), G, sizeof(cplx) * Gh.size(), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int r = 0; r < nr; ++r) {
      const int m = msub[r];
      if (m < 1) continue;
      std::vector<eigsmall::zc> A((size_t)m * m), w, V;
      for (int i = 0; i < m; ++i)
        for (int jj = 0; jj < m; ++jj) {
          const cplx g = Gh[((size_t)r * ms + i) * ms + jj];
          A[(size_t)i * m + jj] = eigsmall::zc(g.x, g.y);
        }
      if (!eigsmall::eig(m, A, w, V)) continue;
      double lo = 1e300, hi = 0.0;
      for (const auto& x : w) lo = std::min(lo, std::abs(x)), hi = std::max(hi, std::abs(x));
      if (!(lo > 0.0) || !std::isfinite(hi)) continue;
      kappa = std::max(kappa, hi / lo);
      ritz_min = ritz_min > 0.0 ? std::min(ritz_min, lo) : lo;
    }
  }
  HIPCHK(hipStreamSynchronize(st));
  c->arena.reset(mk);
  int conv = 1;
  double mx = 0.0;
  for (int r = 0; r < nr; ++r) {
    mx = std::max(mx, res[r]);
    if (!(res[r] <= tol)) conv = 0;
  }
  if (info) {
    info->iters = iters;
    info->resnorm = mx;
    info->converged = conv;
    info->nsigma = nsigma;
    info->time_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    info->kappa = kappa;
    info->ritz_min = ritz_min;
  }
  return conv ? CCLR_OK : CCLR_ENOTCONV;
}

void merge_conditioning(cclr_solve_info& dst, const cclr_solve_info& src) {
  dst.kappa = std::max(dst.kappa, src.kappa);
  if (src.ritz_min > 0.0) dst.ritz_min = dst.ritz_min > 0.0 ? std::min(dst.ritz_min, src.ritz_min) : src.ritz_min;
}

// ------------------------------------------------------- precision driver
// Solve with the context's precision.  FP64: one Davidson solve.  FP32 /
// split-BF16: the Davidson solve with iterative refinement and subspace
// recycling (see davidson): reduced-precision ladder and ring products for
// the trial vectors, FP64 true residuals, until ||R|| <= tol ||b||.
// Right-hand sides advance in lockstep; when the subspaces and transform
// temporaries of all of them do not fit in free device memory they are
// solved in consecutive groups that do.
int solve_system(cclr_ctx* c, int side, int nr, const cplx* zh, const VecSet& rhs, const VecSet& xout,
                 cclr_solve_info* info) {
  const double tol = c->opt.tol;
  const int lowp = c->opt.prec;
  // inner accuracy: what the reduced-precision products can deliver
  // (split-BF16 with the operator rounded to bf16: about 2^-9 of the operator)
  const double inner = lowp == CCLR_FP64      ? 0.0
                       : c->inner_tol > 0.0   ? c->inner_tol
                       : lowp == CCLR_FP32    ? 1e-6
                       : lowp == CCLR_BF16X3  ? 1e-4
                                              : 1e-3;
  if (lowp == CCLR_FP64) c->sigma_prec = CCLR_FP64;
  const i64 ov = c->ns(), nd = c->nd(), oovv = (i64)c->o * c->o * c->v * c->v;
  const int ms = std::max(4, std::min(c->opt.max_subspace, 120));
  const double per = (2.0 * ms + 10.0) * (double)(ov + nd) * sizeof(cplx) + 10.0 * (double)oovv * sizeof(cplx);
  const int chunk = fit_vectors(c, per, nr);
  if (chunk >= nr) return davidson(c, side, nr, zh, rhs, xout, info, tol, c->opt.maxiter, lowp, inner);
  cclr_solve_info all{};
  all.converged = 1;
  int rc = CCLR_OK;
  auto t0 = std::chrono::steady_clock::now();
  for (int k0 = 0; k0 < nr; k0 += chunk) {
    const int n = std::min(chunk, nr - k0);
    const VecSet r{rhs.s + k0 * ov, rhs.d + k0 * nd, n}, x{xout.s + k0 * ov, xout.d + k0 * nd, n};
    cclr_solve_info part{};
    const int pr = davidson(c, side, n, zh + k0, r, x, &part, tol, c->opt.maxiter, lowp, inner);
    if (pr == CCLR_ENOTCONV) rc = CCLR_ENOTCONV;
    all.iters = std::max(all.iters, part.iters);
    all.converged = all.converged && part.converged;
    all.resnorm = std::max(all.resnorm, part.resnorm);
    all.nsigma += part.nsigma;
    merge_conditioning(all, part);
  }
  all.time_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (info) *info = all;
  return rc;
}

// ------------------------------------------------------------ EOM-EE roots
// Lowest eigenpairs of the Jacobian (right: A x = w x; left: x A = w x), the
// EOM-EE excitation energies that are the poles of the response function
// (SI, "EOM-EE sigma-vectors"; Davidson's method for a few eigenpairs of a
// non-Hermitian matrix).  One subspace shared by all roots: orthonormal b_i,
// s_i = A b_i, projected matrix H = B^H S (built and solved on the GPU: the
// Gram products write its new rows and columns in place, the small
// eigensolver writes the Ritz coefficients straight into the combinations),
// Ritz pairs (theta_k, x_k = B y_k), residuals r_k = S y_k - theta_k x_k,
// corrections (theta_k - D)^-1 r_k orthogonalized twice against the
// subspace.  When the subspace is full it restarts from the Ritz vectors.

int eom_davidson(cclr_ctx* c, int side, int nroots, double tol, int maxit_in, std::vector<cplx>& omega,
                 const VecSet& xout, cclr_solve_info* info) {
  auto t0 = std::chrono::steady_clock::now();
  const i64 ov = c->ns(), nd = c->nd(), n = ov + nd;
  const int ms = std::max(std::min(120, std::max(c->opt.max_subspace, 4 * nroots)), 2 * nroots + 2);
  REQUIRE(nroots >= 1 && nroots <= 30 && nroots <= n, CCLR_EINVAL, "nroots must be in [1, 30] and not above the dimension");
  hipStream_t st = c->stream;
  Arena::Mark mk = c->arena.mark();
  auto vbuf = [&](int nvec) {
    VecSet v;
    v.s = (cplx*)c->arena.get(sizeof(cplx) * (size_t)(nvec * ov));
    v.d = (cplx*)c->arena.get(sizeof(cplx) * (size_t)(nvec * nd));
    v.n = nvec;
    return v;
  };
  VecSet Bv = vbuf(ms), Sv = vbuf(ms), Rv = vbuf(nroots), Ev = vbuf(nroots);
  const VS B{Bv.s, Bv.d, 0}, S{Sv.s, Sv.d, 0};  // shared by every root (slot stride 0)
  const VS R{Rv.s, Rv.d, 1}, E{Ev.s, Ev.d, 1}, X{xout.s, xout.d, 1};
  cplx* tmpv = (cplx*)c->arena.get(sizeof(cplx) * (size_t)nroots * ms);
  cplx* coef = (cplx*)c->arena.get(sizeof(cplx) * (size_t)nroots * ms);
  cplx* coef2 = (cplx*)c->arena.get(sizeof(cplx) * (size_t)nroots * ms);
  // projected matrix: Hu[j ms + i] = H[i][j] (i <= j), Hl[j ms + i] = H[j][i] (i < j)
  cplx* Hu = (cplx*)c->arena.get(sizeof(cplx) * (size_t)ms * ms);
  cplx* Hl = (cplx*)c->arena.get(sizeof(cplx) * (size_t)ms * ms);
  cplx* eigw = (cplx*)c->arena.get(sizeof(cplx) * small_eig_work_elems(ms));
  int* eig_status = (int*)c->arena.get(sizeof(int));
  cplx* partial = (cplx*)c->arena.get(sizeof(cplx) * (size_t)nroots * ms * kChunks);
  int* act_d = (int*)c->arena.get(sizeof(int) * nroots);
  cplx* z_d = (cplx*)c->arena.get(sizeof(cplx) * nroots);
  int na = 0;
  auto set_active = [&](const std::vector<int>& a) {
    na = (int)a.size();
    if (na) HIPCHK(hipMemcpyAsync(act_d, a.data(), sizeof(int) * na, hipMemcpyHostToDevice, st));
  };
  auto gram = [&](VS Xs, int xj0, int nj, VS Ys, int yj, cplx* out, int ld, int col0, int cj) {
    if (nj <= 0 || na <= 0) return;
    hipLaunchKernelGGL(k_gram, dim3(kChunks, (nj + kGramJ - 1) / kGramJ, na), dim3(kThreads), 0, st, Xs, xj0, nj,
                       Ys, yj, act_d, ov, nd, partial);
    hipLaunchKernelGGL(k_reduce, dim3(na * nj), dim3(kThreads), 0, st, partial, nj, act_d, out, ld, col0, cj);
  };
  auto lincomb = [&](VS out, int oj, VS Xs, int xj0, int nj, const cplx* cf, int ldc, int acc) {
    hipLaunchKernelGGL(k_lincomb, dim3(vgrid(n), na), dim3(kThreads), 0, st, out, oj, Xs, xj0, nj, cf, ldc, 1.0, Xs, 0,
                       0, acc, act_d, ov, nd);
  };
  auto fetch = [&](const cplx* src, std::vector<cplx>& h, size_t count) {
    h.resize(count);
    HIPCHK(hipMemcpyAsync(h.data(), src, sizeof(cplx) * count, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
  };
  auto sigma = (side == CCLR_RIGHT) ? sigma_right : sigma_left;
  // transforms s_j = A b_j for j in [j0, j1)
  long nsigma = 0;
  auto transform = [&](int j0, int j1) {
    VecSet in{Bv.s + (i64)j0 * ov, Bv.d + (i64)j0 * nd, j1 - j0}, out{Sv.s + (i64)j0 * ov, Sv.d + (i64)j0 * nd, j1 - j0};
    sigma(c, in, out, nullptr);
    nsigma += j1 - j0;
  };
  // orthonormalize E[k] against b_0..b_{m-1} (classical Gram-Schmidt twice) and store it as b_m;
  // returns false if nothing new is left
  auto append = [&](int k, int m) {
    std::vector<int> one{k};
    set_active(one);
    std::vector<cplx> hv;
    gram(E, 0, 1, E, 0, tmpv, 1, 0, 0);  // |e_k|^2 at tmpv[k]
    fetch(tmpv + k, hv, 1);
    const double n0 = std::sqrt(std::max(hv[0].x, 0.0));
    for (int pass = 0; pass < 2 && m > 0; ++pass) {
      gram(B, 0, m, E, 0, coef, ms, 0, 0);
      hipLaunchKernelGGL(k_lincomb, dim3(vgrid(n), 1), dim3(kThreads), 0, st, E, 0, B, 0, m, coef, ms, -1.0, E, 0, 0, 1,
                         act_d, ov, nd);
    }
    gram(E, 0, 1, E, 0, tmpv, 1, 0, 0);
    fetch(tmpv + k, hv, 1);
    const double n1 = std::sqrt(std::max(hv[0].x, 0.0));
    if (!(n1 > 1e-3 * n0) || !(n1 > 0.0)) return false;
    hipLaunchKernelGGL(k_scale, dim3(vgrid(n), 1), dim3(kThreads), 0, st, B, m, E, 0, z_d, c->diag.c(), tmpv, 1, act_d,
                       ov, nd);
    return true;
  };
  // ---- start: unit vectors on the smallest Re D
  std::vector<cplx> dh;
  fetch(c->diag.c(), dh, (size_t)n);
  std::vector<i64> idx(n);
  for (i64 e = 0; e < n; ++e) idx[e] = e;
  const int nstart = std::min<i64>(n, std::min(ms / 2, 2 * nroots));
  std::partial_sort(idx.begin(), idx.begin() + nstart, idx.end(),
                    [&](i64 a, i64 b) { return dh[a].x < dh[b].x || (dh[a].x == dh[b].x && a < b); });
  launch_fill(Bv.s, (i64)ms * ov, cx(0.0), st);
  launch_fill(Bv.d, (i64)ms * nd, cx(0.0), st);
  const cplx one_c = cx(1.0);
  for (int j = 0; j < nstart; ++j) {
    const i64 e = idx[j];
    cplx* p = e < ov ? Bv.s + (i64)j * ov + e : Bv.d + (i64)j * nd + (e - ov);
    HIPCHK(hipMemcpyAsync(p, &one_c, sizeof(cplx), hipMemcpyHostToDevice, st));
  }
  HIPCHK(hipStreamSynchronize(st));
  int m = nstart;
  transform(0, m);
  auto update_H = [&](int j0, int j1) {  // rows and columns of H for the new vectors j0..j1-1
    std::vector<int> zero{0};
    set_active(zero);
    for (int j = j0; j < j1; ++j) {
      gram(B, 0, j + 1, S, j, Hu, 0, j * ms, 0);  // H[i][j] = <b_i, s_j>, i <= j
      if (j > 0) gram(S, 0, j, B, j, Hl, 0, j * ms, 1);  // H[j][i] = <b_j, s_i>, i < j
    }
  };
  update_H(0, m);
  const int maxit = std::max(1, maxit_in);
  int iters = 0;
  std::vector<double> res(nroots, 1e300);
  omega.assign(nroots, cx(0.0));
  bool conv = false;
  std::vector<int> roots(nroots);
  for (int k = 0; k < nroots; ++k) roots[k] = k;
  while (true) {
    ++iters;
    // Ritz pairs of the projected matrix (on the GPU): theta_k in z_d, y_k in coef, -theta_k y_k in coef2
    launch_small_eig(m, Hu, Hl, ms, eigw, nroots, coef, coef2, ms, z_d, nullptr, eig_status, st);
    set_active(roots);
    lincomb(X, 0, B, 0, m, coef, ms, 0);   // x_k = B y_k
    lincomb(R, 0, S, 0, m, coef, ms, 0);   // r_k = S y_k ...
    lincomb(R, 0, B, 0, m, coef2, ms, 1);  // ... - theta_k B y_k
    gram(R, 0, 1, R, 0, tmpv, 1, 0, 0);
    std::vector<cplx> hv((size_t)nroots);
    int eig_ok = 0;
    HIPCHK(hipMemcpyAsync(hv.data(), tmpv, sizeof(cplx) * nroots, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(omega.data(), z_d, sizeof(cplx) * nroots, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(&eig_ok, eig_status, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    REQUIRE(eig_ok == 1, CCLR_ENOTCONV, "projected eigenproblem did not converge");
    std::vector<int> open;
    for (int k = 0; k < nroots; ++k) {
      res[k] = std::sqrt(std::max(hv[k].x, 0.0));
      if (!(res[k] <= tol)) open.push_back(k);
    }
    if (open.empty()) {
      conv = true;
      break;
    }
    if (iters >= maxit) break;
    // corrections (theta_k - D)^-1 r_k
    set_active(open);
    hipLaunchKernelGGL(k_scale, dim3(vgrid(n), na), dim3(kThreads), 0, st, E, 0, R, 0, z_d, c->diag.c(), nullptr, 0,
                       act_d, ov, nd);
    if (m + (int)open.size() > ms) {
      // restart from the Ritz vectors: b = orthonormalized x_k, s = A b
      int m2 = 0;
      for (int k = 0; k < nroots; ++k) {
        HIPCHK(hipMemcpyAsync(Ev.s + (i64)k * ov, xout.s + (i64)k * ov, sizeof(cplx) * ov, hipMemcpyDeviceToDevice, st));
        HIPCHK(hipMemcpyAsync(Ev.d + (i64)k * nd, xout.d + (i64)k * nd, sizeof(cplx) * nd, hipMemcpyDeviceToDevice, st));
        if (append(k, m2)) ++m2;
      }
      m = m2;
      transform(0, m);
      update_H(0, m);
      continue;
    }
    const int m0 = m;
    for (int k : open)
      if (append(k, m)) ++m;
    if (m == m0) break;  // no new directions
    transform(m0, m);
    update_H(m0, m);
  }
  HIPCHK(hipStreamSynchronize(st));
  c->arena.reset(mk);
  double mx = 0.0;
  for (double r : res) mx = std::max(mx, r);
  if (info) {
    info->iters = iters;
    info->converged = conv ? 1 : 0;
    info->resnorm = mx;
    info->nsigma = nsigma;
    info->time_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    info->kappa = info->ritz_min = 0.0;
  }
  return conv ? CCLR_OK : CCLR_ENOTCONV;
}
