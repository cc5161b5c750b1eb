// Internal test hooks (include/cclr_debug.h).
#include <algorithm>
#include <cstring>
#include <vector>

#include "../../include/cclr_debug.h"
#include "internal.h"

extern "C" {

int cclr_dbg_zgemm(int M, int N, int K, int batch, const cclr_c64* A, long long sAb, long long sAm, long long sAk,
                   int conjA, const cclr_c64* B, long long sBb, long long sBk, long long sBn, int conjB, cclr_c64* C,
                   long long sCb, long long sCm, long long sCn, double ar, double ai, int beta) {
  try {
    GemmArgs g{};
    g.M = M; g.N = N; g.K = K; g.batch = batch;
    g.A = (const cplx*)A; g.sAb = sAb; g.sAm = sAm; g.sAk = sAk; g.conjA = conjA;
    g.B = (const cplx*)B; g.sBb = sBb; g.sBk = sBk; g.sBn = sBn; g.conjB = conjB;
    g.C = (cplx*)C; g.sCb = sCb; g.sCm = sCm; g.sCn = sCn;
    g.ar = ar; g.ai = ai; g.beta = beta;
    launch_zgemm(g, nullptr);
    HIPCHK(hipDeviceSynchronize());
    return CCLR_OK;
  } catch (const CclrError& e) {
    return e.code;
  }
}

int cclr_dbg_run_gemm_b2(cclr_ctx* c, int M, int N, int K, int nb1, int nb2, const cclr_c64* A, long long sAb,
                         long long sAb2, long long sAm, long long sAk, const cclr_c64* B, long long sBb, long long sBb2,
                         long long sBk, long long sBn, cclr_c64* C, long long sCb, long long sCb2, long long sCm,
                         long long sCn, double ar, double ai, int beta) {
  if (!c) return CCLR_EINVAL;
  try {
    REQUIRE(M > 0 && N > 0 && K > 0 && nb1 > 0 && nb2 > 1 && (long long)nb1 * nb2 < 65536, CCLR_EINVAL,
            "two-level batch: empty product or batch out of range");
    GemmArgs g{};
    g.M = M; g.N = N; g.K = K; g.batch = nb1 * nb2; g.nb2 = nb2;
    g.A = (const cplx*)A; g.sAb = sAb; g.sAb2 = sAb2; g.sAm = sAm; g.sAk = sAk;
    g.B = (const cplx*)B; g.sBb = sBb; g.sBb2 = sBb2; g.sBk = sBk; g.sBn = sBn;
    g.C = (cplx*)C; g.sCb = sCb; g.sCb2 = sCb2; g.sCm = sCm; g.sCn = sCn;
    g.ar = ar; g.ai = ai; g.beta = beta;
    run_gemm(c, g);
    HIPCHK(hipStreamSynchronize(c->stream));
  } catch (const CclrError& e) {
    return e.code;
  }
  return CCLR_OK;
}

int cclr_dbg_run_gemm(cclr_ctx* c, int M, int N, int K, int batch, const cclr_c64* A, long long sAb, long long sAm,
                      long long sAk, int conjA, const cclr_c64* B, long long sBb, long long sBk, long long sBn,
                      int conjB, cclr_c64* C, long long sCb, long long sCm, long long sCn, double ar, double ai,
                      int beta) {
  if (!c) return CCLR_EINVAL;
  try {
    REQUIRE(M > 0 && N > 0 && K > 0 && batch > 0, CCLR_EINVAL, "empty product");
    GemmArgs g{};
    g.M = M; g.N = N; g.K = K; g.batch = batch;
    g.A = (const cplx*)A; g.sAb = sAb; g.sAm = sAm; g.sAk = sAk; g.conjA = conjA;
    g.B = (const cplx*)B; g.sBb = sBb; g.sBk = sBk; g.sBn = sBn; g.conjB = conjB;
    g.C = (cplx*)C; g.sCb = sCb; g.sCm = sCm; g.sCn = sCn;
    g.ar = ar; g.ai = ai; g.beta = beta;
    run_gemm(c, g);
    HIPCHK(hipStreamSynchronize(c->stream));
  } catch (const CclrError& e) {
    return e.code;
  }
  return CCLR_OK;
}

int cclr_dbg_zgemm_f64(int variant, int batch, int M, int N, int K, const cclr_c64* A, long long sAb, long long sAm,
                       long long sAk, int conjA, const cclr_c64* B, long long sBb, long long sBk, long long sBn,
                       int conjB, cclr_c64* C, long long sCb, long long sCm, long long sCn, double ar, double ai,
                       int beta) {
  try {
    REQUIRE((variant >= 0 && variant < GEMM_NVAR) ||
                (variant > kTransposedChoice && variant < kTransposedChoice + GEMM_NVAR),
            CCLR_EINVAL, "no such GEMM variant");
    REQUIRE(M > 0 && N > 0 && K > 0 && batch > 0, CCLR_EINVAL, "empty product");
    GemmArgs g{};
    g.M = M; g.N = N; g.K = K; g.batch = batch;
    g.A = (const cplx*)A; g.sAb = sAb; g.sAm = sAm; g.sAk = sAk; g.conjA = conjA;
    g.B = (const cplx*)B; g.sBb = sBb; g.sBk = sBk; g.sBn = sBn; g.conjB = conjB;
    g.C = (cplx*)C; g.sCb = sCb; g.sCm = sCm; g.sCn = sCn;
    g.ar = ar; g.ai = ai; g.beta = beta;
    launch_gemm_choice(g, variant, nullptr);
    HIPCHK(hipDeviceSynchronize());
  } catch (const CclrError& e) {
    return e.code;
  }
  return CCLR_OK;
}

int cclr_dbg_tcopy(int nd, const long long* dim, const long long* sd, const long long* ss, cclr_c64* dst,
                   const cclr_c64* src, double ar, double ai, int conj, int acc) {
  try {
    REQUIRE(nd >= 1 && nd <= 6 && dim && sd && ss && dst && src, CCLR_EINVAL, "tcopy: bad arguments");
    CopyArgs a{};
    a.nd = nd;
    a.total = 1;
    for (int d = 0; d < nd; ++d) {
      REQUIRE(dim[d] >= 1, CCLR_EINVAL, "tcopy: empty extent");
      a.dim[d] = dim[d];
      a.sd[d] = sd[d];
      a.ss[d] = ss[d];
      a.total *= dim[d];
    }
    a.dst = (cplx*)dst;
    a.src = (const cplx*)src;
    a.ar = ar;
    a.ai = ai;
    a.conj = conj;
    a.acc = acc;
    launch_tcopy(a, nullptr);
    HIPCHK(hipDeviceSynchronize());
  } catch (const CclrError& e) {
    return e.code;
  }
  return CCLR_OK;
}

int cclr_dbg_zgemm_f64_splitk(int variant, int M, int N, int K, int kchunk, const cclr_c64* A, long long sAm,
                              long long sAk, const cclr_c64* B, long long sBk, long long sBn, cclr_c64* W) {
  try {
    REQUIRE(variant >= 1 && variant < GEMM_NVAR, CCLR_EINVAL, "no such MFMA GEMM variant");
    REQUIRE(M > 0 && N > 0 && K > 0 && kchunk > 0, CCLR_EINVAL, "empty product");
    GemmArgs g{};
    g.M = M; g.N = N; g.K = K; g.kchunk = kchunk;
    g.batch = (K + kchunk - 1) / kchunk;  // one batch entry per K chunk
    g.A = (const cplx*)A; g.sAm = sAm; g.sAk = sAk;
    g.B = (const cplx*)B; g.sBk = sBk; g.sBn = sBn;
    g.C = (cplx*)W; g.sCb = (i64)M * N; g.sCm = N; g.sCn = 1;
    g.ar = 1.0; g.ai = 0.0; g.beta = 0;
    launch_zgemm_variant(g, variant, nullptr);
    HIPCHK(hipDeviceSynchronize());
  } catch (const CclrError& e) {
    return e.code;
  }
  return CCLR_OK;
}

int cclr_dbg_zgemm_group_f64(int variant, int nprob, const int* M, const int* N, const int* K,
                             const cclr_c64* const* A, const cclr_c64* const* B, int btrans, cclr_c64* const* C) {
  void* dev = nullptr;
  int rc = CCLR_OK;
  try {
    REQUIRE(variant == GEMM_128x64_G3 || variant == GEMM_64x64_G3 || variant == GEMM_128x64_G4 ||
                variant == GEMM_64x64_G4 || variant == GEMM_128x128_G4 || variant == GEMM_128x128_DMA,
            CCLR_EINVAL, "no grouped form of this GEMM variant");
    REQUIRE(nprob > 0 && M && N && K && A && B && C, CCLR_EINVAL, "grouped GEMM: missing arguments");
    std::vector<GemmArgs> g(nprob);
    std::vector<int> ts(nprob + 1, 0);
    const int bm = gemm_tile_rows(variant), bn = gemm_tile_cols(variant);
    for (int p = 0; p < nprob; ++p) {
      REQUIRE(M[p] > 0 && N[p] > 0 && K[p] > 0, CCLR_EINVAL, "grouped GEMM: empty product");
      GemmArgs& x = g[p];
      x = GemmArgs{};
      x.M = M[p]; x.N = N[p]; x.K = K[p]; x.batch = 1;
      x.A = (const cplx*)A[p]; x.sAm = K[p]; x.sAk = 1;
      x.B = (const cplx*)B[p];
      if (btrans) x.sBk = 1, x.sBn = K[p];
      else x.sBk = N[p], x.sBn = 1;
      x.C = (cplx*)C[p]; x.sCm = N[p]; x.sCn = 1;
      x.ar = 1.0; x.ai = 0.0; x.beta = 0;
      const long long tiles = (long long)((M[p] + bm - 1) / bm) * ((N[p] + bn - 1) / bn);
      REQUIRE(ts[p] + tiles < (1ll << 31), CCLR_EINVAL, "grouped GEMM: too many tiles");
      ts[p + 1] = ts[p] + (int)tiles;
    }
    const size_t bytes = sizeof(GemmArgs) * nprob + sizeof(int) * (nprob + 1);
    HIPCHK(hipMalloc(&dev, bytes));
    GemmArgs* pd = (GemmArgs*)dev;
    int* td = (int*)((char*)dev + sizeof(GemmArgs) * nprob);
    HIPCHK(hipMemcpy(pd, g.data(), sizeof(GemmArgs) * nprob, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(td, ts.data(), sizeof(int) * (nprob + 1), hipMemcpyHostToDevice));
    launch_zgemm_group(pd, td, nprob, ts.back(), variant, true, !btrans, nullptr);
    HIPCHK(hipDeviceSynchronize());
  } catch (const CclrError& e) {
    rc = e.code;
  }
  if (dev) (void)hipFree(dev);
  return rc;
}

int cclr_dbg_zgemm_lowp(int prec, int M, int N, int K, const cclr_c64* A, long long sAm, long long sAk, int conjA,
                        const cclr_c64* B, long long sBk, long long sBn, int conjB, cclr_c64* C, long long sCm,
                        long long sCn, double ar, double ai, int beta) {
  void* wa = nullptr;
  void* wb = nullptr;
  int rc = CCLR_OK;
  try {
    REQUIRE(M > 0 && N > 0 && K > 0, CCLR_EINVAL, "empty product");
    GemmArgs g{};
    g.M = M; g.N = N; g.K = K; g.batch = 1;
    g.A = (const cplx*)A; g.sAm = sAm; g.sAk = sAk; g.conjA = conjA;
    g.B = (const cplx*)B; g.sBk = sBk; g.sBn = sBn; g.conjB = conjB;
    g.C = (cplx*)C; g.sCm = sCm; g.sCn = sCn;
    g.ar = ar; g.ai = ai; g.beta = beta;
    if (prec == CCLR_FP32 || prec == CCLR_BF16X3 || prec == CCLR_BF16X2) {
      const int form = split_form_of(prec);
      HIPCHK(hipMalloc(&wa, split_bytes(M, K, form, 0)));
      HIPCHK(hipMalloc(&wb, split_bytes(N, K, form, 1)));
      const SplitMat sa = launch_split(M, K, g.A, sAm, sAk, conjA, wa, form, 0, nullptr);
      const SplitMat sb = launch_split(N, K, g.B, sBn, sBk, conjB, wb, form, 1, nullptr);
      launch_split_gemm(sa, sb, g.C, sCm, sCn, ar, ai, beta, nullptr);
    } else {
      REQUIRE(prec == 16, CCLR_EINVAL, "unknown arithmetic");
      launch_zgemm_lowp(g, CCLR_FP32, nullptr);
    }
    HIPCHK(hipDeviceSynchronize());
  } catch (const CclrError& e) {
    rc = e.code;
  }
  if (wa) (void)hipFree(wa);
  if (wb) (void)hipFree(wb);
  return rc;
}

static Ten dten(const cclr_c64* p, const char* l, const long long* dims) {
  Ten t;
  t.p = (cplx*)p;
  t.nd = (int)strlen(l);
  i64 s = 1;
  for (int d = t.nd - 1; d >= 0; --d) {
    t.dim[d] = dims[d];
    t.st[d] = s;
    s *= dims[d];
  }
  return t;
}

int cclr_dbg_contract(cclr_ctx* c, double ar, double ai, const cclr_c64* A, const char* la, const long long* adims,
                      const cclr_c64* B, const char* lb, const long long* bdims, cclr_c64* C, const char* lc,
                      const long long* cdims) {
  if (!c) return CCLR_EINVAL;
  try {
    contract(c, cx(ar, ai), dten(A, la, adims), la, dten(B, lb, bdims), lb, dten(C, lc, cdims), lc, true);
    HIPCHK(hipStreamSynchronize(c->stream));
    return CCLR_OK;
  } catch (const CclrError& e) {
    c->err = e.what();
    return e.code;
  }
}

int cclr_dbg_get(cclr_ctx* c, const char* name, cclr_c64* dst, long long* count) {
  if (!c || !name) return CCLR_EINVAL;
  DevBuf* b = nullptr;
  const std::string n(name);
  if (n == "Foo") b = &c->Foo;
  else if (n == "Fvv") b = &c->Fvv;
  else if (n == "Fov") b = &c->Fov;
  else if (n == "Woooo") b = &c->Woooo;
  else if (n == "Wovvo") b = &c->Wovvo;
  else if (n == "Wbar") b = &c->Wbar;
  else if (n == "Wooov") b = &c->Wooov;
  else if (n == "Wvovv") b = &c->Wvovv;
  else if (n == "Wovoo") b = &c->Wovoo;
  else if (n == "Wvvvo") b = &c->Wvvvo;
  else if (n == "Wvvvv") {
    // unpacked on request from the packed operator
    const i64 v = c->v;
    if (count) *count = (long long)(v * v * v * v);
    if (dst && c->Wp.p) {
      try {
        with_plain_wp(c, [&]() { launch_unpack_vvvv(c->v, c->Wp.c(), (cplx*)dst, c->stream); });
        HIPCHK(hipStreamSynchronize(c->stream));
      } catch (const CclrError& e) {
        c->err = e.what();
        return e.code;
      }
    }
    return CCLR_OK;
  } else if (n == "Wp") b = &c->Wp;
  else if (n == "diag") b = &c->diag;
  if (!b) {
    c->err = "unknown intermediate " + n;
    return CCLR_EINVAL;
  }
  if (count) *count = (long long)(b->bytes / sizeof(cplx));
  if (dst && b->p) {
    if (hipMemcpy(dst, b->p, b->bytes, hipMemcpyDeviceToDevice) != hipSuccess) return CCLR_EHIP;
  }
  return CCLR_OK;
}

static void clear_prof(cclr_ctx* c) {
  for (auto& e : c->prof_events) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  c->prof_events.clear();
  c->prof_flops.clear();
  c->prof_prec.clear();
}

int cclr_dbg_profile(cclr_ctx* c, int enable) {
  if (!c) return CCLR_EINVAL;
  (void)hipStreamSynchronize(c->stream);
  clear_prof(c);
  c->prof = enable != 0;
  return CCLR_OK;
}

int cclr_dbg_profile_read(cclr_ctx* c, int largest_only, int prec, long long* launches, double* ms, double* flops) {
  if (!c) return CCLR_EINVAL;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return CCLR_EHIP;
  double t = 0.0, f = 0.0, fmax = 0.0;
  long long n = 0;
  for (size_t k = 0; k < c->prof_events.size(); ++k)
    if (prec < 0 || c->prof_prec[k] == prec) fmax = std::max(fmax, c->prof_flops[k]);
  for (size_t k = 0; k < c->prof_events.size(); ++k) {
    if (prec >= 0 && c->prof_prec[k] != prec) continue;
    if (largest_only && c->prof_flops[k] < fmax) continue;
    float x = 0.f;
    if (hipEventElapsedTime(&x, c->prof_events[k].first, c->prof_events[k].second) != hipSuccess) return CCLR_EHIP;
    t += x;
    f += c->prof_flops[k];
    ++n;
  }
  if (launches) *launches = n;
  if (ms) *ms = t;
  if (flops) *flops = f;
  return CCLR_OK;
}

int cclr_dbg_set_sigma_prec(cclr_ctx* c, int prec) {
  if (!c || (prec != CCLR_FP64 && prec != CCLR_FP32 && prec != CCLR_BF16X3 && prec != CCLR_BF16X2)) return CCLR_EINVAL;
  c->sigma_prec = prec;
  return CCLR_OK;
}

int cclr_dbg_set_inner_tol(cclr_ctx* c, double tol) {
  if (!c || !(tol >= 0.0) || tol >= 1.0) return CCLR_EINVAL;
  c->inner_tol = tol;
  return CCLR_OK;
}

int cclr_dbg_gemm_trace(cclr_ctx* c, int enable, char* buf, long long cap) {
  if (!c) return CCLR_EINVAL;
  std::string out;
  for (const auto& l : c->gemm_trace_log) out += l + "\n";
  if (buf && cap > 0) {
    const size_t n = std::min<size_t>(out.size(), (size_t)cap - 1);
    memcpy(buf, out.data(), n);
    buf[n] = 0;
  }
  if (enable >= 0) {
    c->gemm_trace = enable != 0;
    c->gemm_trace_log.clear();
  }
  return CCLR_OK;
}

int cclr_dbg_set_overlap(cclr_ctx* c, int enable) {
  if (!c) return CCLR_EINVAL;
  c->overlap = enable != 0;
  return CCLR_OK;
}

int cclr_dbg_set_blocking(cclr_ctx* c, long long wp_block, int rhs_group) {
  if (!c || wp_block < 0 || rhs_group < 0) return CCLR_EINVAL;
  c->dbg_wp_block = wp_block;
  c->dbg_rhs_group = rhs_group;
  return CCLR_OK;
}

int cclr_dbg_hessian(cclr_ctx* c, int nvec, const cclr_c64* x1, const cclr_c64* x2, cclr_c64* s1, cclr_c64* s2) {
  if (!c || nvec < 1 || !x1 || !x2 || !s1 || !s2) return CCLR_EINVAL;
  if (!c->have_t || !c->have_lam) return CCLR_ESTATE;
  try {
    HIPCHK(hipSetDevice(c->device));
    Arena::Mark mk = c->arena.mark();
    VecSet in = packed_buf(c, nvec), out = packed_buf(c, nvec);
    launch_pack_full(nvec, c->o, c->v, (const cplx*)x1, (const cplx*)x2, in.s, in.d, c->stream);
    hessian_product(c, in, out);
    launch_unpack(nvec, c->o, c->v, out.s, out.d, (cplx*)s1, (cplx*)s2, c->stream);
    HIPCHK(hipStreamSynchronize(c->stream));
    c->arena.reset(mk);
  } catch (const CclrError& e) {
    c->err = e.what();
    return e.code;
  }
  return CCLR_OK;
}

int cclr_dbg_fixed_ws_peak(const cclr_ctx* c, long long* bytes) {
  if (!c || !bytes) return CCLR_EINVAL;
  *bytes = (long long)c->fixed_ws_peak;
  return CCLR_OK;
}

int cclr_dbg_small_eig(int n, const cclr_c64* H, int nroots, cclr_c64* w, cclr_c64* theta, cclr_c64* vecs) {
  void* dev = nullptr;
  int rc = CCLR_OK;
  try {
    REQUIRE(H && w && theta && vecs, CCLR_EINVAL, "small eigensolver: null argument");
    REQUIRE(n >= 1 && n <= kSmallEigMax && nroots >= 1 && nroots <= n, CCLR_EINVAL, "small eigensolver: bad size");
    const size_t nn = (size_t)n * n;
    // device: Hu (column-major copy), Hl (row-major), work, coef, coef2, theta, w, status
    const size_t elems = 2 * nn + small_eig_work_elems(n) + 2 * (size_t)nroots * n + nroots + n;
    HIPCHK(hipMalloc(&dev, sizeof(cplx) * elems + 256));
    cplx* Hu = (cplx*)dev;
    cplx* Hl = Hu + nn;
    cplx* work = Hl + nn;
    cplx* coef = work + small_eig_work_elems(n);
    cplx* coef2 = coef + (size_t)nroots * n;
    cplx* th = coef2 + (size_t)nroots * n;
    cplx* wall = th + nroots;
    int* status = (int*)(wall + n);
    std::vector<cplx> hu(nn), hl(nn);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        const cplx x = make_double2(H[(size_t)i * n + j].re, H[(size_t)i * n + j].im);
        hu[(size_t)j * n + i] = x;
        hl[(size_t)i * n + j] = x;
      }
    HIPCHK(hipMemcpy(Hu, hu.data(), sizeof(cplx) * nn, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(Hl, hl.data(), sizeof(cplx) * nn, hipMemcpyHostToDevice));
    launch_small_eig(n, Hu, Hl, n, work, nroots, coef, coef2, n, th, wall, status, nullptr);
    int ok = 0;
    HIPCHK(hipMemcpy(&ok, status, sizeof(int), hipMemcpyDeviceToHost));
    REQUIRE(ok == 1, CCLR_ENOTCONV, "small eigensolver: QR iteration did not converge");
    HIPCHK(hipMemcpy(w, wall, sizeof(cplx) * n, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(theta, th, sizeof(cplx) * nroots, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(vecs, coef, sizeof(cplx) * (size_t)nroots * n, hipMemcpyDeviceToHost));
  } catch (const CclrError& e) {
    rc = e.code;
  }
  if (dev) (void)hipFree(dev);
  return rc;
}

int cclr_dbg_tuning(cclr_ctx* c, int enable, char* buf, long long cap) {
  if (!c) return CCLR_EINVAL;
  if (enable >= 0) c->autotune = enable != 0;
  std::string out;
  for (const auto& r : c->gemm_tuning_log) {
    out += r.shape + ":";
    for (const auto& vm : r.ms) out += " " + std::to_string(vm.first) + "=" + std::to_string(vm.second);
    out += " -> " + std::to_string(r.chosen) + "\n";
  }
  if (buf && cap > 0) {
    const size_t n = std::min<size_t>(out.size(), (size_t)cap - 1);
    memcpy(buf, out.data(), n);
    buf[n] = 0;
  }
  return CCLR_OK;
}
}
