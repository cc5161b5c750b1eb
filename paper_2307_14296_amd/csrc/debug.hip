// Internal test hooks (include/cclr_debug.h).
#include <algorithm>
#include <cstring>

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

int cclr_dbg_zgemm_f64(int variant, int batch, int M, int N, int K, const cclr_c64* A, long long sAb, long long sAm,
                       long long sAk, int conjA, const cclr_c64* B, long long sBb, long long sBk, long long sBn,
                       int conjB, cclr_c64* C, long long sCb, long long sCm, long long sCn, double ar, double ai,
                       int beta) {
  try {
    REQUIRE(variant >= 0 && variant < GEMM_NVAR, CCLR_EINVAL, "no such GEMM variant");
    REQUIRE(M > 0 && N > 0 && K > 0 && batch > 0, CCLR_EINVAL, "empty product");
    GemmArgs g{};
    g.M = M; g.N = N; g.K = K; g.batch = batch;
    g.A = (const cplx*)A; g.sAb = sAb; g.sAm = sAm; g.sAk = sAk; g.conjA = conjA;
    g.B = (const cplx*)B; g.sBb = sBb; g.sBk = sBk; g.sBn = sBn; g.conjB = conjB;
    g.C = (cplx*)C; g.sCb = sCb; g.sCm = sCm; g.sCn = sCn;
    g.ar = ar; g.ai = ai; g.beta = beta;
    launch_zgemm_variant(g, variant, nullptr);
    HIPCHK(hipDeviceSynchronize());
  } catch (const CclrError& e) {
    return e.code;
  }
  return CCLR_OK;
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
    if (prec == CCLR_BF16X3) {
      HIPCHK(hipMalloc(&wa, split_bytes(M, K)));
      HIPCHK(hipMalloc(&wb, split_bytes(N, K)));
      const SplitMat sa = launch_split_bf16(M, K, g.A, sAm, sAk, conjA, wa, nullptr);
      const SplitMat sb = launch_split_bf16(N, K, g.B, sBn, sBk, conjB, wb, nullptr);
      launch_cgemm_bf16x3(sa, sb, g.C, sCm, sCn, ar, ai, beta, nullptr);
    } else {
      launch_zgemm_lowp(g, prec, nullptr);
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
        launch_unpack_vvvv(c->v, c->Wp.c(), (cplx*)dst, c->stream);
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
}

int cclr_dbg_profile(cclr_ctx* c, int enable) {
  if (!c) return CCLR_EINVAL;
  (void)hipStreamSynchronize(c->stream);
  clear_prof(c);
  c->prof = enable != 0;
  return CCLR_OK;
}

int cclr_dbg_profile_read(cclr_ctx* c, int largest_only, long long* launches, double* ms, double* flops) {
  if (!c) return CCLR_EINVAL;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return CCLR_EHIP;
  double t = 0.0, f = 0.0, fmax = 0.0;
  long long n = 0;
  for (double x : c->prof_flops) fmax = std::max(fmax, x);
  for (size_t k = 0; k < c->prof_events.size(); ++k) {
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
  if (!c || (prec != CCLR_FP64 && prec != CCLR_FP32 && prec != CCLR_BF16X3)) return CCLR_EINVAL;
  c->sigma_prec = prec;
  return CCLR_OK;
}

int cclr_dbg_set_inner_tol(cclr_ctx* c, double tol) {
  if (!c || !(tol >= 0.0) || tol >= 1.0) return CCLR_EINVAL;
  c->inner_tol = tol;
  return CCLR_OK;
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
