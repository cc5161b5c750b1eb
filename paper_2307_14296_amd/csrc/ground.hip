// CCSD ground state on the device: the residual Omega(t), its solution by
// CROP, and the six integral blocks formed from Cholesky vectors.
//
// The amplitude equations are not printed in the paper (its implementation
// section takes the converged t as the first step); they are the standard
// spin-orbital CCSD equations in the intermediate form of Stanton and Gauss
// (J. Chem. Phys. 94, 4334 (1991)), with the diagonal Fock terms kept in F so
// that the result is the residual.  The two 1/4 tau <mn||ef> pieces of the
// hole and particle ladders are carried together by the hole-ladder
// intermediate (1/2 tau there), and the particle ladder 1/2 tau^ef_ij W^ab_ef
// is split into the packed-pair product with <ab||ef> (the large GEMM, the
// same shape as the transforms' ladder) and -1/2 P(ab) t^b_m Z^am_ij with
// Z^am_ij = <am||ef> tau^ef_ij, so that no t-dependent v^4 tensor is built.
//
// CROP (conjugate residual with optimal trial vectors; Ziolkowski et al.,
// J. Chem. Phys. 128, 204105 (2008)) is the ground-state solver the
// implementation section names: a Jacobi step from the current optimal
// vector, the true residual there, then the affine combination (weights
// summing to one) of the kept optimal vectors and the new one whose residual
// combination has the least norm.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <vector>

#include "internal.h"

void launch_pack_vvvv(int v, const cplx* W, cplx* Wp, hipStream_t s);
void launch_diag(int o, int v, const cplx* Foo, const cplx* Fvv, cplx* diag, hipStream_t s);

namespace {

constexpr int kMaxComb = 8;
struct Ptrs {
  const cplx* p[kMaxComb];
};
struct Coefs {
  cplx c[kMaxComb];
};

__global__ __launch_bounds__(256) void k_comb(i64 n, int m, Ptrs x, Coefs w, cplx* __restrict__ out) {
  for (i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (i64)gridDim.x * blockDim.x) {
    double yr = 0.0, yi = 0.0;
    for (int k = 0; k < m; ++k) {
      const cplx a = x.p[k][e], c = w.c[k];
      yr += c.x * a.x - c.y * a.y;
      yi += c.x * a.y + c.y * a.x;
    }
    out[e] = make_double2(yr, yi);
  }
}

// out = x - r / D
__global__ __launch_bounds__(256) void k_jacobi(i64 n, const cplx* __restrict__ x, const cplx* __restrict__ r,
                                                const cplx* __restrict__ D, cplx* __restrict__ out) {
  for (i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (i64)gridDim.x * blockDim.x) {
    const cplx d = D[e], q = r[e];
    const double den = d.x * d.x + d.y * d.y;
    out[e] = make_double2(x[e].x - (q.x * d.x + q.y * d.y) / den, x[e].y - (q.y * d.x - q.x * d.y) / den);
  }
}

unsigned grid1(i64 n) {
  const i64 b = (n + 255) / 256;
  return (unsigned)std::max<i64>(1, std::min<i64>(b, 8192));
}

// out = sum_k w_k x_k over packed vectors (out may not alias any x_k)
void combine(cclr_ctx* c, int m, const VecSet* x, const cplx* w, const VecSet& out) {
  REQUIRE(m >= 1 && m <= kMaxComb, CCLR_EINVAL, "too many vectors in a combination");
  Ptrs ps{}, pd{};
  Coefs cw{};
  for (int k = 0; k < m; ++k) ps.p[k] = x[k].s, pd.p[k] = x[k].d, cw.c[k] = w[k];
  const i64 ov = c->ns(), nd = c->nd();
  hipLaunchKernelGGL(k_comb, dim3(grid1(ov)), dim3(256), 0, c->stream, ov, m, ps, cw, out.s);
  hipLaunchKernelGGL(k_comb, dim3(grid1(nd)), dim3(256), 0, c->stream, nd, m, pd, cw, out.d);
  HIPCHK(hipGetLastError());
}

// sum over unique amplitudes of (conj x if conjx) * y for several pairs, to the host
std::vector<std::complex<double>> dots(cclr_ctx* c, const std::vector<std::pair<VecSet, VecSet>>& pairs, bool conjx) {
  const int np = (int)pairs.size();
  std::vector<std::complex<double>> out(np);
  if (!np) return out;
  Arena::Mark mk = c->arena.mark();
  std::vector<const cplx*> h(4 * np);
  for (int p = 0; p < np; ++p) {
    h[p] = pairs[p].first.s;
    h[np + p] = pairs[p].first.d;
    h[2 * np + p] = pairs[p].second.s;
    h[3 * np + p] = pairs[p].second.d;
  }
  const cplx** pd = (const cplx**)c->arena.get(sizeof(cplx*) * 4 * np);
  HIPCHK(hipMemcpyAsync(pd, h.data(), sizeof(cplx*) * 4 * np, hipMemcpyHostToDevice, c->stream));
  cplx* partial = (cplx*)c->arena.get(sizeof(cplx) * (size_t)np * 256);
  cplx* res = (cplx*)c->arena.get(sizeof(cplx) * np);
  launch_bdot(np, pd, pd + np, pd + 2 * np, pd + 3 * np, c->ns(), c->nd(), partial, res, c->stream, conjx);
  std::vector<cplx> hr(np);
  HIPCHK(hipMemcpyAsync(hr.data(), res, sizeof(cplx) * np, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  for (int p = 0; p < np; ++p) out[p] = std::complex<double>(hr[p].x, hr[p].y);
  c->arena.reset(mk);
  return out;
}

// the packed <ab||ef> (a>b, e>f) used by the residual's particle ladder; made once per Hamiltonian
const cplx* packed_vvvv(cclr_ctx* c) {
  if (!c->Vpk.p) {
    c->Vpk.alloc(c, sizeof(cplx) * (size_t)(c->V2() * c->V2()));
    launch_pack_vvvv(c->v, c->Vvvvv.c(), c->Vpk.c(), c->stream);
  }
  return c->Vpk.c();
}

// solve a small complex system A x = b (n x n, row-major) by Gaussian
// elimination with partial pivoting; false if a pivot vanishes
bool small_solve(int n, std::vector<std::complex<double>> A, std::vector<std::complex<double>>& b) {
  for (int k = 0; k < n; ++k) {
    int p = k;
    for (int i = k + 1; i < n; ++i)
      if (std::abs(A[(size_t)i * n + k]) > std::abs(A[(size_t)p * n + k])) p = i;
    if (std::abs(A[(size_t)p * n + k]) == 0.0) return false;
    if (p != k) {
      for (int j = 0; j < n; ++j) std::swap(A[(size_t)k * n + j], A[(size_t)p * n + j]);
      std::swap(b[k], b[p]);
    }
    for (int i = k + 1; i < n; ++i) {
      const std::complex<double> f = A[(size_t)i * n + k] / A[(size_t)k * n + k];
      for (int j = k; j < n; ++j) A[(size_t)i * n + j] -= f * A[(size_t)k * n + j];
      b[i] -= f * b[k];
    }
  }
  for (int k = n - 1; k >= 0; --k) {
    std::complex<double> s = b[k];
    for (int j = k + 1; j < n; ++j) s -= A[(size_t)k * n + j] * b[j];
    b[k] = s / A[(size_t)k * n + k];
  }
  return true;
}

}  // namespace

// Omega(t) for one packed amplitude vector; out packed.  Returns the
// correlation energy f_ia t^a_i + 1/4 <ij||ab> tau^ab_ij.
std::complex<double> ccsd_residual(cclr_ctx* c, const VecSet& t, const VecSet& out) {
  const i64 o = c->o, v = c->v;
  const cplx one = cx(1.0), mone = cx(-1.0), half = cx(0.5), mhalf = cx(-0.5);
  const cplx* Vp = packed_vvvv(c);
  Arena::Mark mk = c->arena.mark();
  Ten T1 = ten(t.s, {o, v});
  Ten T2 = tmp(c, {o, o, v, v});
  launch_unpack(1, (int)o, (int)v, t.s, t.d, nullptr, T2.p, c->stream);
  // tau = t2 + t1 t1 - t1 t1 ; tau-tilde with half the singles products
  Ten tau = tmp(c, {o, o, v, v}), taut = tmp(c, {o, o, v, v});
  tcopy(c, tau, "ijab", T2, "ijab", one, false);
  contract(c, one, T1, "ia", T1, "jb", tau, "ijab");
  contract(c, mone, T1, "ib", T1, "ja", tau, "ijab");
  tcopy(c, taut, "ijab", T2, "ijab", one, false);
  contract(c, half, T1, "ia", T1, "jb", taut, "ijab");
  contract(c, mhalf, T1, "ib", T1, "ja", taut, "ijab");
  Ten Voovv = Vblk(c, "oovv");
  // one-body intermediates
  Ten Fae = tmp(c, {v, v}), Fmi = tmp(c, {o, o}), Fme = tmp(c, {o, v});
  tcopy(c, Fae, "ae", fblk(c, "vv"), "ae", one, false);
  contract(c, mhalf, fblk(c, "ov"), "me", T1, "ma", Fae, "ae");
  contract(c, one, T1, "mf", Vblk(c, "ovvv"), "mafe", Fae, "ae");
  contract(c, mhalf, taut, "mnaf", Voovv, "mnef", Fae, "ae");
  tcopy(c, Fmi, "mi", fblk(c, "oo"), "mi", one, false);
  contract(c, half, T1, "ie", fblk(c, "ov"), "me", Fmi, "mi");
  contract(c, one, T1, "ne", Vblk(c, "ooov"), "mnie", Fmi, "mi");
  contract(c, half, taut, "inef", Voovv, "mnef", Fmi, "mi");
  tcopy(c, Fme, "me", fblk(c, "ov"), "me", one, false);
  contract(c, one, T1, "nf", Voovv, "mnef", Fme, "me");
  // hole ladder W^mn_ij (1/2 tau: both ladders' tau tau pieces)
  Ten Wmnij = tmp(c, {o, o, o, o});
  {
    tcopy(c, Wmnij, "mnij", Vblk(c, "oooo"), "mnij", one, false);
    Ten w = tmp(c, {o, o, o, o});
    contract(c, one, T1, "je", Vblk(c, "ooov"), "mnie", w, "mnij", false);
    tcopy(c, Wmnij, "mnij", w, "mnij", one);
    tcopy(c, Wmnij, "mnij", w, "mnji", mone);
    contract(c, half, tau, "ijef", Voovv, "mnef", Wmnij, "mnij");
  }
  // ring W^mb_ej
  Ten Wmbej = tmp(c, {o, v, v, o});
  {
    tcopy(c, Wmbej, "mbej", Vblk(c, "ovvo"), "mbej", one, false);
    contract(c, one, T1, "jf", Vblk(c, "ovvv"), "mbef", Wmbej, "mbej");
    contract(c, mone, T1, "nb", Vblk(c, "oovo"), "mnej", Wmbej, "mbej");
    Ten Y = tmp(c, {o, o, v, v});
    tcopy(c, Y, "jnfb", T2, "jnfb", half, false);
    contract(c, one, T1, "jf", T1, "nb", Y, "jnfb");
    contract(c, mone, Y, "jnfb", Voovv, "mnef", Wmbej, "mbej");
  }
  // singles
  Ten S1 = tmp(c, {o, v});
  tcopy(c, S1, "ia", fblk(c, "vo"), "ai", one, false);
  contract(c, one, T1, "ie", Fae, "ae", S1, "ia");
  contract(c, mone, T1, "ma", Fmi, "mi", S1, "ia");
  contract(c, one, T2, "imae", Fme, "me", S1, "ia");
  contract(c, mone, T1, "nf", Vblk(c, "ovov"), "naif", S1, "ia");
  contract(c, mhalf, T2, "imef", Vblk(c, "ovvv"), "maef", S1, "ia");
  contract(c, mhalf, T2, "mnae", Vblk(c, "oovo"), "nmei", S1, "ia");
  // doubles, grouped by the antisymmetrizer they take
  Ten X0 = tmp(c, {o, o, v, v}), Xa = tmp(c, {o, o, v, v}), Xi = tmp(c, {o, o, v, v}), Xai = tmp(c, {o, o, v, v});
  tcopy(c, X0, "ijab", Vblk(c, "vvoo"), "abij", one, false);
  contract(c, half, tau, "mnab", Wmnij, "mnij", X0, "ijab");
  {
    Ten Fbe = tmp(c, {v, v});
    tcopy(c, Fbe, "be", Fae, "be", one, false);
    contract(c, mhalf, T1, "mb", Fme, "me", Fbe, "be");
    contract(c, one, T2, "ijae", Fbe, "be", Xa, "ijab", false);
    Ten Fmj = tmp(c, {o, o});
    tcopy(c, Fmj, "mj", Fmi, "mj", one, false);
    contract(c, half, T1, "je", Fme, "me", Fmj, "mj");
    contract(c, mone, T2, "imab", Fmj, "mj", Xi, "ijab", false);
  }
  {
    Ten Z = tmp(c, {v, o, o, o});
    contract(c, one, Vblk(c, "vovv"), "amef", tau, "ijef", Z, "amij", false);
    contract(c, mhalf, T1, "mb", Z, "amij", Xa, "ijab");
  }
  contract(c, mone, T1, "ma", Vblk(c, "ovoo"), "mbij", Xa, "ijab");
  contract(c, one, T1, "ie", Vblk(c, "vvvo"), "abej", Xi, "ijab");
  contract(c, one, T2, "imae", Wmbej, "mbej", Xai, "ijab", false);
  {
    Ten Rt = tmp(c, {o, v, o, o});
    contract(c, one, T1, "ie", Vblk(c, "ovvo"), "mbej", Rt, "mbij", false);
    contract(c, mone, T1, "ma", Rt, "mbij", Xai, "ijab");
  }
  // packed tau (singles slot carries t1) for the particle ladder and the energy
  const i64 V2 = c->V2(), O2 = c->O2();
  VecSet taup = packed_buf(c, 1);
  launch_pack_full(1, (int)o, (int)v, T1.p, tau.p, taup.s, taup.d, c->stream);
  {
    GemmArgs g{};
    g.M = (int)O2;
    g.N = (int)V2;
    g.K = (int)V2;
    g.batch = 1;
    g.A = taup.d; g.sAm = V2; g.sAk = 1;
    g.B = Vp; g.sBk = 1; g.sBn = V2;
    g.C = out.d; g.sCm = V2; g.sCn = 1;
    g.ar = 1.0; g.ai = 0.0; g.beta = 0;
    tuned_gemm(c, g);
  }
  launch_fill(out.s, o * v, cx(0.0), c->stream);
  launch_pack_sigma(1, (int)o, (int)v, X0.p, Xa.p, Xi.p, Xai.p, S1.p, out.s, out.d, nullptr, nullptr, nullptr,
                    c->stream, false);
  // energy: sum f_ia t^a_i + sum_(i>j,a>b) <ij||ab> tau^ab_ij
  VecSet e0 = packed_buf(c, 1);
  Ten fov = tmp(c, {o, v});
  tcopy(c, fov, "ia", fblk(c, "ov"), "ia", one, false);
  launch_pack_full(1, (int)o, (int)v, fov.p, c->Voovv.c(), e0.s, e0.d, c->stream);
  const std::complex<double> E = dots(c, {{e0, taup}}, false)[0];
  c->arena.reset(mk);
  return E;
}

int ccsd_crop(cclr_ctx* c, double tol, int maxit, int nsub, const VecSet& t, std::complex<double>* energy,
              cclr_solve_info* info) {
  REQUIRE(nsub >= 2 && nsub <= kMaxComb, CCLR_EINVAL, "CROP subspace size must be in [2, 8]");
  REQUIRE(tol > 0.0 && maxit >= 1, CCLR_EINVAL, "need tol > 0 and maxiter >= 1");
  const auto t0 = std::chrono::steady_clock::now();
  const i64 o = c->o, v = c->v, ov = c->ns(), nd = c->nd();
  Arena::Mark mk = c->arena.mark();
  // Fock diagonal of the Jacobi step
  cplx* D = (cplx*)c->arena.get(sizeof(cplx) * (size_t)(ov + nd));
  {
    Arena::Mark m2 = c->arena.mark();
    Ten Foo = tmp(c, {o, o}), Fvv = tmp(c, {v, v});
    tcopy(c, Foo, "ij", fblk(c, "oo"), "ij", cx(1.0), false);
    tcopy(c, Fvv, "ab", fblk(c, "vv"), "ab", cx(1.0), false);
    launch_diag((int)o, (int)v, Foo.p, Fvv.p, D, c->stream);
    HIPCHK(hipStreamSynchronize(c->stream));
    c->arena.reset(m2);
  }
  // nsub optimal-vector slots (nsub - 1 live, one spare) and the trial pair
  std::vector<VecSet> X(nsub), R(nsub);
  for (int k = 0; k < nsub; ++k) X[k] = packed_buf(c, 1), R[k] = packed_buf(c, 1);
  VecSet xt = packed_buf(c, 1), rt = packed_buf(c, 1);
  auto norm = [&](const VecSet& r) { return std::sqrt(std::max(0.0, dots(c, {{r, r}}, true)[0].real())); };
  auto copy = [&](const VecSet& dst, const VecSet& src) {
    HIPCHK(hipMemcpyAsync(dst.s, src.s, sizeof(cplx) * ov, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(dst.d, src.d, sizeof(cplx) * nd, hipMemcpyDeviceToDevice, c->stream));
  };
  std::vector<int> live;  // slots of the kept optimal vectors, oldest first
  copy(X[0], t);
  std::complex<double> E = ccsd_residual(c, X[0], R[0]);
  long nres = 1;
  double rn = norm(R[0]);
  int it = 0;
  bool conv = rn <= tol;
  if (conv) copy(xt, X[0]);
  live.push_back(0);
  while (!conv && it < maxit) {
    ++it;
    const int last = live.back();
    hipLaunchKernelGGL(k_jacobi, dim3(grid1(ov)), dim3(256), 0, c->stream, ov, X[last].s, R[last].s, D, xt.s);
    hipLaunchKernelGGL(k_jacobi, dim3(grid1(nd)), dim3(256), 0, c->stream, nd, X[last].d, R[last].d, D + ov, xt.d);
    HIPCHK(hipGetLastError());
    E = ccsd_residual(c, xt, rt);
    ++nres;
    rn = norm(rt);
    if (!std::isfinite(rn)) throw CclrError(CCLR_ENOTCONV, "CCSD residual is not finite (diverged)");
    if (rn <= tol) {
      conv = true;
      break;
    }
    // subspace: the kept optimal vectors and the trial one
    std::vector<VecSet> xs, rs;
    for (int k : live) xs.push_back(X[k]), rs.push_back(R[k]);
    xs.push_back(xt);
    rs.push_back(rt);
    int m = (int)rs.size();
    std::vector<std::complex<double>> coef;
    for (;;) {
      std::vector<std::pair<VecSet, VecSet>> pairs;
      for (int a = 0; a < m; ++a)
        for (int b = a; b < m; ++b) pairs.push_back({rs[a], rs[b]});
      const auto g = dots(c, pairs, true);
      std::vector<std::complex<double>> A((size_t)(m + 1) * (m + 1), 0.0), b(m + 1, 0.0);
      int q = 0;
      for (int a = 0; a < m; ++a)
        for (int bb = a; bb < m; ++bb, ++q) {
          A[(size_t)a * (m + 1) + bb] = g[q];
          A[(size_t)bb * (m + 1) + a] = std::conj(g[q]);
        }
      for (int a = 0; a < m; ++a) A[(size_t)a * (m + 1) + m] = A[(size_t)m * (m + 1) + a] = 1.0;
      b[m] = 1.0;
      if (small_solve(m + 1, A, b)) {
        coef.assign(b.begin(), b.begin() + m);
        break;
      }
      // singular (linearly dependent residuals): drop the oldest kept vector
      REQUIRE(m > 1, CCLR_ENOTCONV, "CROP subspace collapsed");
      xs.erase(xs.begin());
      rs.erase(rs.begin());
      live.erase(live.begin());
      --m;
    }
    // the new optimal vector goes to a free slot
    int slot = -1;
    for (int k = 0; k < nsub && slot < 0; ++k)
      if (std::find(live.begin(), live.end(), k) == live.end()) slot = k;
    std::vector<cplx> w(m);
    for (int k = 0; k < m; ++k) w[k] = cx(coef[k].real(), coef[k].imag());
    combine(c, m, xs.data(), w.data(), X[slot]);
    combine(c, m, rs.data(), w.data(), R[slot]);
    live.push_back(slot);
    while ((int)live.size() > nsub - 1) live.erase(live.begin());
  }
  copy(t, xt);
  HIPCHK(hipStreamSynchronize(c->stream));
  c->arena.reset(mk);
  if (energy) *energy = E;
  if (info) {
    info->iters = it;
    info->converged = conv ? 1 : 0;
    info->resnorm = rn;
    info->nsigma = nres;
    info->kappa = info->ritz_min = 0.0;
    info->time_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  return conv ? CCLR_OK : CCLR_ENOTCONV;
}

// the six canonical <pq||rs> blocks from Cholesky vectors L[P][n][n]:
// <pq||rs> = sum_P (L[P][p][r] L[P][q][s] - L[P][p][s] L[P][q][r])
void integrals_from_cholesky(cclr_ctx* c, int nchol, const cplx* L) {
  const i64 o = c->o, v = c->v, n = o + v;
  auto sz = [&](char k) { return k == 'o' ? o : v; };
  auto lv = [&](char a, char b) {
    Ten t;
    t.p = (cplx*)L + (a == 'o' ? 0 : o) * n + (b == 'o' ? 0 : o);
    t.nd = 3;
    t.dim[0] = nchol, t.dim[1] = sz(a), t.dim[2] = sz(b);
    t.st[0] = n * n, t.st[1] = n, t.st[2] = 1;
    return t;
  };
  struct B {
    const char* k;
    DevBuf* buf;
  } blocks[] = {{"oooo", &c->Voooo}, {"ooov", &c->Vooov}, {"oovv", &c->Voovv},
                {"ovov", &c->Vovov}, {"ovvv", &c->Vovvv}, {"vvvv", &c->Vvvvv}};
  for (const B& b : blocks) {
    const char* k = b.k;
    b.buf->alloc(c, sizeof(cplx) * (size_t)(sz(k[0]) * sz(k[1]) * sz(k[2]) * sz(k[3])));
    Ten V = ten(*b.buf, {sz(k[0]), sz(k[1]), sz(k[2]), sz(k[3])});
    Arena::Mark mk = c->arena.mark();
    contract(c, cx(1.0), lv(k[0], k[2]), "Ppr", lv(k[1], k[3]), "Pqs", V, "pqrs", false);
    contract(c, cx(-1.0), lv(k[0], k[3]), "Pps", lv(k[1], k[2]), "Pqr", V, "pqrs");
    c->arena.reset(mk);
  }
}
