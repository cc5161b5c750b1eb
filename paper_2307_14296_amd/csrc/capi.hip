// C ABI of libcclr (declared in include/cclr.h).
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <algorithm>
#include <map>
#include <mutex>

#include "internal.h"

VecSet packed_buf(cclr_ctx* c, int n) {
  VecSet v;
  v.s = (cplx*)c->arena.get(sizeof(cplx) * (size_t)(n * c->ns()));
  v.d = (cplx*)c->arena.get(sizeof(cplx) * (size_t)(n * c->nd()));
  v.n = n;
  return v;
}

static thread_local std::string g_create_error;

// The library's fixed work space, for cclr_jacobian_right_noalloc: a file-scope
// device array that every GPU the library runs on holds until the process
// ends.  In host code `scratch` names a host-side stand-in, not a device
// address, so the kernels only ever see the address hipGetSymbolAddress gives
// for the current device, looked up once per device when a context is created.
constexpr size_t kFixedWsBytes = size_t(256) << 20;
static __device__ __align__(256) char scratch[kFixedWsBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_ws_mutex;                 // guards g_ws_ptr
void* g_ws_ptr[kMaxDevices] = {};      // this device's address of `scratch`
std::mutex g_ws_busy[kMaxDevices];     // one no-alloc call per device at a time

// the device's address of the work space (device current); called from cclr_create
void* fixed_ws_address(int dev) {
  REQUIRE(dev >= 0 && dev < kMaxDevices, CCLR_EHIP, "device index out of range for the fixed work space");
  std::lock_guard<std::mutex> lk(g_ws_mutex);
  if (!g_ws_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      throw CclrError(CCLR_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    }
    g_ws_ptr[dev] = p;
  }
  return g_ws_ptr[dev];
}
}  // namespace

namespace {
template <class F>
int guarded(cclr_ctx* c, F&& f) {
  try {
    if (c) {
      c->err.clear();
      HIPCHK(hipSetDevice(c->device));
    }
    return f();
  } catch (const CclrError& e) {
    if (c) c->err = e.what();
    else g_create_error = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    if (c) c->err = "host allocation failed";
    return CCLR_ENOMEM;
  } catch (const std::exception& e) {
    if (c) c->err = e.what();
    return CCLR_EHIP;
  }
}

void check_ptr(const void* p, const char* what) {
  REQUIRE(p != nullptr, CCLR_EINVAL, std::string("null pointer: ") + what);
  hipPointerAttribute_t attr;
  hipError_t e = hipPointerGetAttributes(&attr, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw CclrError(CCLR_EINVAL, std::string(what) + " is not a HIP device pointer");
  }
  REQUIRE(attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged, CCLR_EINVAL,
          std::string(what) + " must point to device memory");
}

void check_finite(cclr_ctx* c, const cplx* p, i64 n, const char* what) {
  int* flag = (int*)c->arena.get(sizeof(int));
  HIPCHK(hipMemsetAsync(flag, 0, sizeof(int), c->stream));
  launch_check_finite(p, n, flag, c->stream);
  int h = 0;
  HIPCHK(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  REQUIRE(!h, CCLR_EINVAL, std::string("non-finite value in ") + what);
}

void copy_in(cclr_ctx* c, DevBuf& dst, const cclr_c64* src, i64 n, const char* what) {
  check_ptr(src, what);
  dst.alloc(c, sizeof(cplx) * (size_t)n);
  HIPCHK(hipMemcpyAsync(dst.p, src, sizeof(cplx) * (size_t)n, hipMemcpyDeviceToDevice, c->stream));
  Arena::Mark mk = c->arena.mark();
  check_finite(c, dst.c(), n, what);
  c->arena.reset(mk);
}

void check_freqs(int n, const double* omega, const double* gamma) {
  REQUIRE(n >= 0, CCLR_EINVAL, "negative count");
  if (n == 0) return;
  REQUIRE(omega && gamma, CCLR_EINVAL, "null frequency array");
  for (int k = 0; k < n; ++k) {
    REQUIRE(std::isfinite(omega[k]) && std::isfinite(gamma[k]), CCLR_EINVAL, "non-finite frequency");
    REQUIRE(gamma[k] >= 0.0, CCLR_EINVAL, "negative damping gamma");
  }
}

// full (r1[n][o][v], r2[n][o][o][v][v]) -> packed
void pack_in(cclr_ctx* c, int n, const cclr_c64* r1, const cclr_c64* r2, const VecSet& out, const char* what) {
  check_ptr(r1, what);
  check_ptr(r2, what);
  const i64 oovv = (i64)c->o * c->o * c->v * c->v;
  launch_pack_full(n, c->o, c->v, (const cplx*)r1, (const cplx*)r2, out.s, out.d, c->stream);
  check_finite(c, out.s, n * c->ns(), what);
  check_finite(c, out.d, n * c->nd(), what);
  (void)oovv;
}

void unpack_out(cclr_ctx* c, const VecSet& in, cclr_c64* s1, cclr_c64* s2, const char* what) {
  check_ptr(s1, what);
  check_ptr(s2, what);
  launch_unpack(in.n, c->o, c->v, in.s, in.d, (cplx*)s1, (cplx*)s2, c->stream);
}

void require_t(cclr_ctx* c) {
  REQUIRE(c->have_H, CCLR_ESTATE, "cclr_set_hamiltonian has not been called");
  REQUIRE(c->have_t, CCLR_ESTATE, "cclr_set_amplitudes has not been called");
}

int solve_lambda_impl(cclr_ctx* c, cclr_solve_info* info) {
  require_t(c);
  Arena::Mark mk = c->arena.mark();
  VecSet rhs = packed_buf(c, 1);
  // eta0: singles F^i_a, doubles <ij||ab>
  HIPCHK(hipMemcpyAsync(rhs.s, c->Fov.p, sizeof(cplx) * (size_t)c->ns(), hipMemcpyDeviceToDevice, c->stream));
  launch_pack_full(1, c->o, c->v, c->Fov.c(), c->Voovv.c(), rhs.s, rhs.d, c->stream);
  c->lam_s.alloc(c, sizeof(cplx) * (size_t)c->ns());
  c->lam_d.alloc(c, sizeof(cplx) * (size_t)c->nd());
  VecSet x{c->lam_s.c(), c->lam_d.c(), 1};
  const cplx z0 = cx(0.0);
  const int rc = solve_system(c, CCLR_LEFT, 1, &z0, rhs, x, info);
  c->arena.reset(mk);
  c->have_lam = true;
  return rc;
}
}  // namespace

extern "C" {

int cclr_default_options(cclr_options* opt) {
  if (!opt) return CCLR_EINVAL;
  opt->prec = CCLR_FP64;
  opt->tol = 1e-10;
  opt->maxiter = 500;
  opt->max_subspace = 48;
  opt->device_mem_cap = 0;
  opt->hip_stream = nullptr;
  return CCLR_OK;
}

int cclr_create(int o, int v, const cclr_options* opt, cclr_ctx** out) {
  return guarded(nullptr, [&]() -> int {
    REQUIRE(out, CCLR_EINVAL, "null output pointer");
    *out = nullptr;
    REQUIRE(o >= 2 && v >= 2, CCLR_EINVAL, "need o >= 2 and v >= 2");
    REQUIRE((i64)o * o * v * v < (1ll << 40), CCLR_EINVAL, "problem too large");
    cclr_ctx* c = new cclr_ctx();
    c->o = o;
    c->v = v;
    if (opt) c->opt = *opt;
    else cclr_default_options(&c->opt);
    if (c->opt.prec != CCLR_FP64 && c->opt.prec != CCLR_FP32 && c->opt.prec != CCLR_BF16X3 &&
        c->opt.prec != CCLR_BF16X2) {
      delete c;
      throw CclrError(CCLR_EINVAL, "prec must be CCLR_FP64, CCLR_FP32, CCLR_BF16X3 or CCLR_BF16X2");
    }
    if (!(c->opt.tol > 0.0) || c->opt.maxiter < 1 || c->opt.max_subspace < 4 || c->opt.max_subspace > 120) {
      delete c;
      throw CclrError(CCLR_EINVAL, "invalid options (tol > 0, maxiter >= 1, 4 <= max_subspace <= 120)");
    }
    c->stream = (hipStream_t)c->opt.hip_stream;
    hipError_t e = hipGetDevice(&c->device);
    if (e != hipSuccess) {
      delete c;
      throw CclrError(CCLR_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    }
    c->arena.ctx = c;
    try {
      c->fixed_ws = fixed_ws_address(c->device);
    } catch (...) {
      delete c;
      throw;
    }
    *out = c;
    return CCLR_OK;
  });
}

int cclr_destroy(cclr_ctx* c) {
  if (!c) return CCLR_OK;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  if (c->side) {
    (void)hipStreamSynchronize(c->side);
    (void)hipStreamDestroy(c->side);
  }
  if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
  if (c->ev_join) (void)hipEventDestroy(c->ev_join);
  delete c;
  return CCLR_OK;
}

const char* cclr_last_error(const cclr_ctx* c) { return c ? c->err.c_str() : g_create_error.c_str(); }

int cclr_set_hamiltonian(cclr_ctx* c, const cclr_c64* f, const cclr_c64* oooo, const cclr_c64* ooov,
                         const cclr_c64* oovv, const cclr_c64* ovov, const cclr_c64* ovvv, const cclr_c64* vvvv) {
  if (!c) return CCLR_EINVAL;
  return guarded(c, [&]() -> int {
    const i64 o = c->o, v = c->v, n = o + v;
    c->have_H = c->have_t = c->have_lam = false;
    c->Vpk.release();
    copy_in(c, c->f, f, n * n, "f");
    copy_in(c, c->Voooo, oooo, o * o * o * o, "oooo");
    copy_in(c, c->Vooov, ooov, o * o * o * v, "ooov");
    copy_in(c, c->Voovv, oovv, o * o * v * v, "oovv");
    copy_in(c, c->Vovov, ovov, o * v * o * v, "ovov");
    copy_in(c, c->Vovvv, ovvv, o * v * v * v, "ovvv");
    copy_in(c, c->Vvvvv, vvvv, v * v * v * v, "vvvv");
    HIPCHK(hipStreamSynchronize(c->stream));
    c->have_H = true;
    return CCLR_OK;
  });
}

int cclr_set_hamiltonian_cholesky(cclr_ctx* c, const cclr_c64* f, int nchol, const cclr_c64* L) {
  if (!c) return CCLR_EINVAL;
  return guarded(c, [&]() -> int {
    const i64 o = c->o, v = c->v, n = o + v;
    REQUIRE(nchol >= 1, CCLR_EINVAL, "need nchol >= 1");
    c->have_H = c->have_t = c->have_lam = false;
    c->Vpk.release();
    copy_in(c, c->f, f, n * n, "f");
    check_ptr(L, "L");
    {
      Arena::Mark mk = c->arena.mark();
      check_finite(c, (const cplx*)L, (i64)nchol * n * n, "L");
      c->arena.reset(mk);
    }
    integrals_from_cholesky(c, nchol, (const cplx*)L);
    HIPCHK(hipStreamSynchronize(c->stream));
    c->have_H = true;
    return CCLR_OK;
  });
}

int cclr_ccsd_residual(cclr_ctx* c, const cclr_c64* t1, const cclr_c64* t2, cclr_c64* o1, cclr_c64* o2,
                       cclr_c64* energy) {
  if (!c) return CCLR_EINVAL;
  return guarded(c, [&]() -> int {
    REQUIRE(c->have_H, CCLR_ESTATE, "cclr_set_hamiltonian has not been called");
    Arena::Mark mk = c->arena.mark();
    VecSet t = packed_buf(c, 1), out = packed_buf(c, 1);
    pack_in(c, 1, t1, t2, t, "t");
    const std::complex<double> E = ccsd_residual(c, t, out);
    unpack_out(c, out, o1, o2, "output");
    HIPCHK(hipStreamSynchronize(c->stream));
    c->arena.reset(mk);
    if (energy) *energy = cclr_c64{E.real(), E.imag()};
    return CCLR_OK;
  });
}

int cclr_solve_ccsd(cclr_ctx* c, double tol, int maxiter, int nsub, cclr_c64* t1, cclr_c64* t2, cclr_c64* energy,
                    cclr_solve_info* info) {
  if (!c) return CCLR_EINVAL;
  return guarded(c, [&]() -> int {
    REQUIRE(c->have_H, CCLR_ESTATE, "cclr_set_hamiltonian has not been called");
    const i64 o = c->o, v = c->v;
    Arena::Mark mk = c->arena.mark();
    VecSet t = packed_buf(c, 1);
    pack_in(c, 1, t1, t2, t, "t");
    std::complex<double> E;
    const int rc = ccsd_crop(c, tol, maxiter, nsub, t, &E, info);
    unpack_out(c, t, t1, t2, "t");
    c->arena.reset(mk);
    // the solution becomes the context's amplitudes
    c->have_t = c->have_lam = false;
    copy_in(c, c->t1, t1, o * v, "t1");
    copy_in(c, c->t2, t2, o * o * v * v, "t2");
    build_intermediates(c);
    HIPCHK(hipStreamSynchronize(c->stream));
    c->have_t = true;
    if (energy) *energy = cclr_c64{E.real(), E.imag()};
    return rc;
  });
}

int cclr_set_amplitudes(cclr_ctx* c, const cclr_c64* t1, const cclr_c64* t2) {
  if (!c) return CCLR_EINVAL;
  return guarded(c, [&]() -> int {
    REQUIRE(c->have_H, CCLR_ESTATE, "cclr_set_hamiltonian has not been called");
    const i64 o = c->o, v = c->v;
    c->have_t = c->have_lam = false;
    copy_in(c, c->t1, t1, o * v, "t1");
    copy_in(c, c->t2, t2, o * o * v * v, "t2");
    build_intermediates(c);
    c->have_t = true;
    return CCLR_OK;
  });
}

static int jacobian(cclr_ctx* c, int side, int nvec, const double* omega, const double* gamma, const cclr_c64* r1,
                    const cclr_c64* r2, cclr_c64* s1, cclr_c64* s2) {
  return guarded(c, [&]() -> int {
    require_t(c);
    check_freqs(nvec, omega, gamma);
    if (nvec == 0) return CCLR_OK;
    Arena::Mark mk = c->arena.mark();
    VecSet in = packed_buf(c, nvec), out = packed_buf(c, nvec);
    pack_in(c, nvec, r1, r2, in, side == CCLR_RIGHT ? "r" : "l");
    std::vector<cplx> z(nvec);
    for (int k = 0; k < nvec; ++k) z[k] = cx(omega[k], gamma[k]);
    cplx* zd = (cplx*)c->arena.get(sizeof(cplx) * nvec);
    HIPCHK(hipMemcpyAsync(zd, z.data(), sizeof(cplx) * nvec, hipMemcpyHostToDevice, c->stream));
    if (side == CCLR_RIGHT) sigma_right(c, in, out, zd);
    else sigma_left(c, in, out, zd);
    unpack_out(c, out, s1, s2, "output");
    HIPCHK(hipStreamSynchronize(c->stream));
    c->arena.reset(mk);
    return CCLR_OK;
  });
}

int cclr_jacobian_right(cclr_ctx* c, int nvec, const double* omega, const double* gamma, const cclr_c64* r1,
                        const cclr_c64* r2, cclr_c64* s1, cclr_c64* s2) {
  if (!c) return CCLR_EINVAL;
  return jacobian(c, CCLR_RIGHT, nvec, omega, gamma, r1, r2, s1, s2);
}

int cclr_jacobian_right_noalloc(cclr_ctx* c, int nvec, const double* omega, const double* gamma,
                                const cclr_c64* r1, const cclr_c64* r2, cclr_c64* s1, cclr_c64* s2) {
  if (!c) return CCLR_EINVAL;
  return guarded(c, [&]() -> int {
    require_t(c);
    check_freqs(nvec, omega, gamma);
    if (nvec == 0) return CCLR_OK;
    REQUIRE(c->sigma_prec == CCLR_FP64, CCLR_EINVAL,
            "cclr_jacobian_right_noalloc: FP64 transforms only (a reduced-precision operator copy is allocated)");
    REQUIRE(c->fixed_ws, CCLR_ESTATE, "the fixed work space was not set up for this context");
    // the packed input and output vectors, the full doubles layout and the
    // ring layout are the least the transform takes; the arena's own bound
    // check catches the rest before anything is written beyond the region
    const double need = 16.0 * nvec * (2.0 * (c->ns() + c->nd()) + 2.0 * c->o * c->o * (double)c->v * c->v);
    REQUIRE(need <= (double)kFixedWsBytes, CCLR_ENOMEM,
            "cclr_jacobian_right_noalloc: " + std::to_string(nvec) + " vectors at o=" + std::to_string(c->o) +
                ", v=" + std::to_string(c->v) + " need more than the fixed work space of " +
                std::to_string(kFixedWsBytes) + " bytes; use cclr_jacobian_right");
    std::lock_guard<std::mutex> busy(g_ws_busy[c->device]);
    // route every temporary of this call into the work space, take no new
    // timing runs, and keep the transform on the context's stream
    struct Scope {
      cclr_ctx* c;
      bool overlap, prof;
      Scope(cclr_ctx* c_) : c(c_), overlap(c_->overlap), prof(c_->prof) {
        c->arena.ext = (char*)c->fixed_ws;
        c->arena.ext_bytes = kFixedWsBytes;
        c->arena.ext_used = c->arena.ext_peak = 0;
        c->no_timing = true;
        c->overlap = false;
        c->prof = false;
      }
      ~Scope() {
        // the work queued on the region must end before another call reuses it
        (void)hipStreamSynchronize(c->stream);
        c->fixed_ws_peak = c->arena.ext_peak;
        c->arena.ext = nullptr;
        c->arena.ext_bytes = c->arena.ext_used = 0;
        c->no_timing = false;
        c->overlap = overlap;
        c->prof = prof;
      }
    } scope(c);
    return jacobian(c, CCLR_RIGHT, nvec, omega, gamma, r1, r2, s1, s2);
  });
}

namespace {
// One persistent launch for products of several contexts that share operand
// layouts; the kernel variant is timed once per set of shapes and kept.
void grouped_products(cclr_ctx* c0, std::vector<GemmArgs> g) {
  g.erase(std::remove_if(g.begin(), g.end(), [](const GemmArgs& x) { return x.M <= 0 || x.N <= 0 || x.K <= 0; }),
          g.end());
  if (g.empty()) return;
  const bool ak = g[0].sAk == 1, bn = g[0].sBn == 1;
  for (const GemmArgs& x : g)
    REQUIRE((x.sAk == 1) == ak && (x.sBn == 1) == bn && x.kchunk == 0, CCLR_EINVAL, "grouped products: layouts differ");
  // longest reductions first: the tiles are dealt round-robin to the workgroups
  std::stable_sort(g.begin(), g.end(), [](const GemmArgs& a, const GemmArgs& b) { return a.K > b.K; });
  std::string key = ak ? "A1" : "A0";
  key += bn ? "B1" : "B0";
  for (const GemmArgs& x : g) key += ":" + std::to_string(x.M) + "x" + std::to_string(x.N) + "x" + std::to_string(x.K);
  Arena::Mark mk = c0->arena.mark();
  GemmArgs* pd = (GemmArgs*)c0->arena.get(sizeof(GemmArgs) * g.size());
  int* td = (int*)c0->arena.get(sizeof(int) * (g.size() + 1));
  HIPCHK(hipMemcpyAsync(pd, g.data(), sizeof(GemmArgs) * g.size(), hipMemcpyHostToDevice, c0->stream));
  auto launch = [&](int variant) {
    std::vector<int> ts(g.size() + 1, 0);
    const int bm = gemm_tile_rows(variant), bn_ = gemm_tile_cols(variant);
    for (size_t p = 0; p < g.size(); ++p) {
      const i64 tiles = (i64)((g[p].M + bm - 1) / bm) * ((g[p].N + bn_ - 1) / bn_) * g[p].batch;
      REQUIRE(ts[p] + tiles < (1ll << 31), CCLR_EINVAL, "grouped products: too many tiles");
      ts[p + 1] = ts[p] + (int)tiles;
    }
    HIPCHK(hipMemcpyAsync(td, ts.data(), sizeof(int) * ts.size(), hipMemcpyHostToDevice, c0->stream));
    launch_zgemm_group(pd, td, (int)g.size(), ts.back(), variant, ak, bn, c0->stream);
  };
  auto it = c0->group_choice.find(key);
  if (it == c0->group_choice.end()) {
    int best = GEMM_128x64_G4;
    double best_ms = -1;
    std::vector<std::pair<int, double>> ms_all;
    for (int var : {GEMM_128x64_G3, GEMM_64x64_G3, GEMM_128x64_G4, GEMM_64x64_G4, GEMM_128x128_G4, GEMM_128x128_DMA}) {
      hipEvent_t e0, e1;
      HIPCHK(hipEventCreate(&e0));
      HIPCHK(hipEventCreate(&e1));
      HIPCHK(hipEventRecord(e0, c0->stream));
      launch(var);
      HIPCHK(hipEventRecord(e1, c0->stream));
      HIPCHK(hipEventSynchronize(e1));
      float ms = 0;
      HIPCHK(hipEventElapsedTime(&ms, e0, e1));
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      ms_all.push_back({var, ms});
      if (best_ms < 0 || ms < best_ms) best_ms = ms, best = var;
    }
    c0->group_choice[key] = best;
    c0->gemm_tuning_log.push_back({"group " + key, ms_all, best});
    it = c0->group_choice.find(key);
  }
  launch(it->second);
  c0->arena.reset(mk);
}
}  // namespace

int cclr_jacobian_right_multi(int nctx, cclr_ctx* const* ctx, const int* nvec, const double* const* omega,
                              const double* const* gamma, const cclr_c64* const* r1, const cclr_c64* const* r2,
                              cclr_c64* const* s1, cclr_c64* const* s2) {
  if (nctx < 1 || !ctx || !ctx[0]) return CCLR_EINVAL;
  cclr_ctx* c0 = ctx[0];
  std::vector<Arena::Mark> marks(nctx);
  std::vector<bool> marked(nctx, false);
  const int rc = guarded(c0, [&]() -> int {
    REQUIRE(nvec && omega && gamma && r1 && r2 && s1 && s2, CCLR_EINVAL, "null argument array");
    for (int i = 0; i < nctx; ++i) {
      REQUIRE(ctx[i], CCLR_EINVAL, "null context");
      for (int j = 0; j < i; ++j) REQUIRE(ctx[j] != ctx[i], CCLR_EINVAL, "a context appears twice");
      require_t(ctx[i]);
      REQUIRE(ctx[i]->stream == c0->stream, CCLR_EINVAL, "contexts must share one stream");
      REQUIRE(ctx[i]->sigma_prec == CCLR_FP64, CCLR_EINVAL, "grouped transforms are FP64");
      check_freqs(nvec[i], omega[i], gamma[i]);
    }
    std::vector<VecSet> in(nctx), out(nctx);
    std::vector<cplx*> zd(nctx, nullptr);
    std::vector<SigmaWork> w(nctx);
    std::vector<GemmArgs> rings, ladders;
    for (int i = 0; i < nctx; ++i) {
      cclr_ctx* c = ctx[i];
      if (nvec[i] == 0) continue;
      marks[i] = c->arena.mark();
      marked[i] = true;
      in[i] = packed_buf(c, nvec[i]);
      out[i] = packed_buf(c, nvec[i]);
      pack_in(c, nvec[i], r1[i], r2[i], in[i], "r");
      std::vector<cplx> z(nvec[i]);
      for (int k = 0; k < nvec[i]; ++k) z[k] = cx(omega[i][k], gamma[i][k]);
      zd[i] = (cplx*)c->arena.get(sizeof(cplx) * nvec[i]);
      HIPCHK(hipMemcpyAsync(zd[i], z.data(), sizeof(cplx) * nvec[i], hipMemcpyHostToDevice, c->stream));
      w[i] = sigma_right_begin(c, in[i], out[i]);
      rings.push_back(w[i].ring);
      ladders.push_back(w[i].ladder);
    }
    grouped_products(c0, rings);
    grouped_products(c0, ladders);
    for (int i = 0; i < nctx; ++i) {
      if (nvec[i] == 0) continue;
      sigma_finish(ctx[i], w[i], in[i], out[i], zd[i]);
      unpack_out(ctx[i], out[i], s1[i], s2[i], "output");
    }
    HIPCHK(hipStreamSynchronize(c0->stream));
    return CCLR_OK;
  });
  for (int i = 0; i < nctx; ++i)
    if (marked[i]) ctx[i]->arena.reset(marks[i]);
  return rc;
}

int cclr_jacobian_left(cclr_ctx* c, int nvec, const double* omega, const double* gamma, const cclr_c64* l1,
                       const cclr_c64* l2, cclr_c64* s1, cclr_c64* s2) {
  if (!c) return CCLR_EINVAL;
  return jacobian(c, CCLR_LEFT, nvec, omega, gamma, l1, l2, s1, s2);
}

int cclr_solve_damped(cclr_ctx* c, int side, int nrhs, const double* omega, const double* gamma, const cclr_c64* b1,
                      const cclr_c64* b2, cclr_c64* x1, cclr_c64* x2, cclr_solve_info* info) {
  if (!c) return CCLR_EINVAL;
  return guarded(c, [&]() -> int {
    require_t(c);
    REQUIRE(side == CCLR_RIGHT || side == CCLR_LEFT, CCLR_EINVAL, "side must be CCLR_RIGHT or CCLR_LEFT");
    check_freqs(nrhs, omega, gamma);
    if (nrhs == 0) return CCLR_OK;
    Arena::Mark mk = c->arena.mark();
    VecSet rhs = packed_buf(c, nrhs), x = packed_buf(c, nrhs);
    pack_in(c, nrhs, b1, b2, rhs, "b");
    std::vector<cplx> z(nrhs);
    for (int k = 0; k < nrhs; ++k) z[k] = cx(omega[k], gamma[k]);
    const int rc = solve_system(c, side, nrhs, z.data(), rhs, x, info);
    unpack_out(c, x, x1, x2, "x");
    HIPCHK(hipStreamSynchronize(c->stream));
    c->arena.reset(mk);
    return rc;
  });
}

int cclr_eom_ee(cclr_ctx* c, int side, int nroots, double tol, cclr_c64* omega, cclr_c64* x1, cclr_c64* x2,
                cclr_solve_info* info) {
  if (!c) return CCLR_EINVAL;
  return guarded(c, [&]() -> int {
    require_t(c);
    REQUIRE(side == CCLR_RIGHT || side == CCLR_LEFT, CCLR_EINVAL, "side must be CCLR_RIGHT or CCLR_LEFT");
    REQUIRE(omega, CCLR_EINVAL, "null omega");
    REQUIRE(std::isfinite(tol) && tol > 0.0, CCLR_EINVAL, "tol must be positive");
    Arena::Mark mk = c->arena.mark();
    VecSet x = packed_buf(c, std::max(nroots, 1));
    std::vector<cplx> w;
    const int rc = eom_davidson(c, side, nroots, tol, c->opt.maxiter, w, x, info);
    for (int k = 0; k < nroots; ++k) omega[k] = cclr_c64{w[k].x, w[k].y};
    if (x1 || x2) unpack_out(c, x, x1, x2, "eigenvectors");
    HIPCHK(hipStreamSynchronize(c->stream));
    c->arena.reset(mk);
    return rc;
  });
}

int cclr_solve_lambda(cclr_ctx* c, cclr_solve_info* info) {
  if (!c) return CCLR_EINVAL;
  return guarded(c, [&]() -> int { return solve_lambda_impl(c, info); });
}

int cclr_get_lambda(const cclr_ctx* cc, cclr_c64* l1, cclr_c64* l2) {
  cclr_ctx* c = const_cast<cclr_ctx*>(cc);
  if (!c) return CCLR_EINVAL;
  return guarded(c, [&]() -> int {
    REQUIRE(c->have_lam, CCLR_ESTATE, "no lambda in the context");
    VecSet l{c->lam_s.c(), c->lam_d.c(), 1};
    unpack_out(c, l, l1, l2, "lambda");
    HIPCHK(hipStreamSynchronize(c->stream));
    return CCLR_OK;
  });
}

// model 0: CC-CC (eq. CC-CC response function); model 1: CC-CI (eq. CC-CI
// response function, EOM eta vector)
static int response_impl(cclr_ctx* c, int model, int nx, const cclr_c64* const* X, int nfreq, const double* omega,
                         const double* gamma, cclr_c64* out, cclr_solve_info* info) {
  if (!c) return CCLR_EINVAL;
  return guarded(c, [&]() -> int {
    auto t0 = std::chrono::steady_clock::now();
    require_t(c);
    REQUIRE(nx >= 1 && X && out, CCLR_EINVAL, "need nx >= 1 perturbations and an output array");
    check_freqs(nfreq, omega, gamma);
    const i64 n = c->o + c->v, ov = c->ns(), nd = c->nd();
    for (int p = 0; p < nx; ++p) {
      check_ptr(X[p], "X");
      Arena::Mark mk = c->arena.mark();
      check_finite(c, (const cplx*)X[p], n * n, "X");
      c->arena.reset(mk);
    }
    cclr_solve_info linfo{};
    long nsig = 0;
    int rc = CCLR_OK;
    if (!c->have_lam) {
      rc = solve_lambda_impl(c, &linfo);
      nsig += linfo.nsigma;
      if (rc < 0) return rc;
    }
    Arena::Mark mk = c->arena.mark();
    // property vectors
    VecSet xi = packed_buf(c, nx), eta = packed_buf(c, nx);
    for (int p = 0; p < nx; ++p) {
      VecSet a{xi.s + p * ov, xi.d + p * nd, 1}, b{eta.s + p * ov, eta.d + p * nd, 1};
      build_xi(c, (const cplx*)X[p], a);
      build_eta(c, (const cplx*)X[p], b);
    }
    if (model == 1) {  // EOM eta: singles + lambda^ij_ab xi^X_jb
      const i64 o = c->o, v = c->v;
      Ten l2 = tmp(c, {o, o, v, v});
      launch_unpack(1, (int)o, (int)v, c->lam_s.c(), c->lam_d.c(), nullptr, l2.p, c->stream);
      contract(c, cx(1.0), l2, "ijab", ten(xi.s, {(i64)nx, o, v}), "Zjb", ten(eta.s, {(i64)nx, o, v}), "Zia");
    }
    // distinct solve frequencies: z, -z, conj z, -conj z for every requested z
    std::vector<std::complex<double>> fr;
    auto fid = [&](std::complex<double> w) {
      for (size_t k = 0; k < fr.size(); ++k)
        if (fr[k] == w) return (int)k;
      fr.push_back(w);
      return (int)fr.size() - 1;
    };
    std::vector<int> idz(nfreq), idmz(nfreq), idcz(nfreq), idmcz(nfreq);
    for (int w = 0; w < nfreq; ++w) {
      const std::complex<double> z(omega[w], gamma[w]);
      idz[w] = fid(z);
      idmz[w] = fid(-z);
      idcz[w] = fid(std::conj(z));
      idmcz[w] = fid(-std::conj(z));
    }
    const int nf = (int)fr.size();
    const int nr = nf * nx;  // right-hand side (f, p) at index f*nx + p
    VecSet rhs = packed_buf(c, nr), sol = packed_buf(c, nr);
    std::vector<cplx> zr(nr);
    for (int f = 0; f < nf; ++f)
      for (int p = 0; p < nx; ++p) {
        const int r = f * nx + p;
        zr[r] = cx(fr[f].real(), fr[f].imag());
        HIPCHK(hipMemcpyAsync(rhs.s + r * ov, xi.s + p * ov, sizeof(cplx) * ov, hipMemcpyDeviceToDevice, c->stream));
        HIPCHK(hipMemcpyAsync(rhs.d + r * nd, xi.d + p * nd, sizeof(cplx) * nd, hipMemcpyDeviceToDevice, c->stream));
      }
    cclr_solve_info sinfo{};
    const int rs = solve_system(c, CCLR_RIGHT, nr, zr.data(), rhs, sol, &sinfo);
    nsig += sinfo.nsigma;
    // Hessian products of the X-side solutions only: t^p(-z) and t^p(z*)
    std::vector<int> xside_f;
    for (int w = 0; w < nfreq; ++w)
      for (int f : {idmz[w], idcz[w]})
        if (std::find(xside_f.begin(), xside_f.end(), f) == xside_f.end()) xside_f.push_back(f);
    if (model == 1) xside_f.clear();  // no Hessian term in the CC-CI form
    const int ntf = (int)xside_f.size() * nx;
    VecSet tfin = packed_buf(c, ntf), tfo = packed_buf(c, ntf);
    std::map<int, int> tf_slot;  // solution index r -> Hessian-product slot
    for (size_t q = 0; q < xside_f.size(); ++q)
      for (int p = 0; p < nx; ++p) {
        const int r = xside_f[q] * nx + p, k = (int)q * nx + p;
        tf_slot[r] = k;
        HIPCHK(hipMemcpyAsync(tfin.s + k * ov, sol.s + r * ov, sizeof(cplx) * ov, hipMemcpyDeviceToDevice, c->stream));
        HIPCHK(hipMemcpyAsync(tfin.d + k * nd, sol.d + r * nd, sizeof(cplx) * nd, hipMemcpyDeviceToDevice, c->stream));
      }
    if (ntf > 0) hessian_product(c, tfin, tfo);
    // bilinear products
    auto vs = [&](const VecSet& s, int k) { return std::make_pair(s.s + k * ov, s.d + k * nd); };
    std::vector<const cplx*> hx_s, hx_d, hy_s, hy_d;
    auto add = [&](std::pair<cplx*, cplx*> a, std::pair<cplx*, cplx*> b) {
      hx_s.push_back(a.first), hx_d.push_back(a.second), hy_s.push_back(b.first), hy_d.push_back(b.second);
      return (int)hx_s.size() - 1;
    };
    std::map<std::pair<int, int>, int> eta_t, tf_t;  // (p, r) -> pair index
    for (int p = 0; p < nx; ++p)
      for (int r = 0; r < nr; ++r) eta_t[{p, r}] = add(vs(eta, p), vs(sol, r));
    for (const auto& kv : tf_slot)
      for (int r2 = 0; r2 < nr; ++r2) tf_t[{kv.first, r2}] = add(vs(tfo, kv.second), vs(sol, r2));
    std::vector<int> lam_t(nr), lam_xi(nx);  // lambda . t_r and lambda . xi_p
    if (model == 1) {
      const auto lam = std::make_pair(c->lam_s.c(), c->lam_d.c());
      for (int r = 0; r < nr; ++r) lam_t[r] = add(lam, vs(sol, r));
      for (int p = 0; p < nx; ++p) lam_xi[p] = add(lam, vs(xi, p));
    }
    const int np = (int)hx_s.size();
    const cplx** pd = (const cplx**)c->arena.get(sizeof(cplx*) * 4 * np);
    std::vector<const cplx*> all;
    all.insert(all.end(), hx_s.begin(), hx_s.end());
    all.insert(all.end(), hx_d.begin(), hx_d.end());
    all.insert(all.end(), hy_s.begin(), hy_s.end());
    all.insert(all.end(), hy_d.begin(), hy_d.end());
    HIPCHK(hipMemcpyAsync(pd, all.data(), sizeof(cplx*) * 4 * np, hipMemcpyHostToDevice, c->stream));
    cplx* partial = (cplx*)c->arena.get(sizeof(cplx) * (size_t)np * 256);
    cplx* dots = (cplx*)c->arena.get(sizeof(cplx) * np);
    launch_bdot(np, pd, pd + np, pd + 2 * np, pd + 3 * np, ov, nd, partial, dots, c->stream);
    std::vector<cplx> hd(np);
    HIPCHK(hipMemcpyAsync(hd.data(), dots, sizeof(cplx) * np, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    auto C = [&](int k) { return std::complex<double>(hd[k].x, hd[k].y); };
    // g_pq(z) = eta^p t^q(z) + eta^q t^p(-z) + F t^p(-z) t^q(z)
    // CC-CI: h_pq(z) = Eeta^p t^q(z) + Eeta^q t^p(-z) - (lambda t^p(-z))(lambda xi^q) - (lambda t^q(z))(lambda xi^p)
    auto g = [&](int p, int q, int fz, int fmz) {
      const int rq = fz * nx + q, rpm = fmz * nx + p;
      if (model == 1)
        return C(eta_t[{p, rq}]) + C(eta_t[{q, rpm}]) - C(lam_t[rpm]) * C(lam_xi[q]) - C(lam_t[rq]) * C(lam_xi[p]);
      return C(eta_t[{p, rq}]) + C(eta_t[{q, rpm}]) + C(tf_t[{rpm, rq}]);
    };
    for (int w = 0; w < nfreq; ++w)
      for (int p = 0; p < nx; ++p)
        for (int q = 0; q < nx; ++q) {
          const std::complex<double> val = 0.5 * (g(p, q, idz[w], idmz[w]) + std::conj(g(p, q, idmcz[w], idcz[w])));
          out[((i64)w * nx + p) * nx + q] = cclr_c64{val.real(), val.imag()};
        }
    c->arena.reset(mk);
    if (info) {
      info->iters = std::max(sinfo.iters, linfo.iters);
      info->converged = sinfo.converged && (linfo.iters == 0 || linfo.converged);
      info->resnorm = std::max(sinfo.resnorm, linfo.resnorm);
      info->nsigma = nsig;
      info->kappa = info->ritz_min = 0.0;
      merge_conditioning(*info, sinfo);
      merge_conditioning(*info, linfo);
      info->time_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    if (rc == CCLR_ENOTCONV || rs == CCLR_ENOTCONV) return CCLR_ENOTCONV;
    return CCLR_OK;
  });
}

int cclr_response_function(cclr_ctx* c, int nx, const cclr_c64* const* X, int nfreq, const double* omega,
                           const double* gamma, cclr_c64* out, cclr_solve_info* info) {
  return response_impl(c, 0, nx, X, nfreq, omega, gamma, out, info);
}

int cclr_response_function_ci(cclr_ctx* c, int nx, const cclr_c64* const* X, int nfreq, const double* omega,
                              const double* gamma, cclr_c64* out, cclr_solve_info* info) {
  return response_impl(c, 1, nx, X, nfreq, omega, gamma, out, info);
}

int cclr_response_function_asym(cclr_ctx* c, int nx, const cclr_c64* const* X, int ny, const cclr_c64* const* Y,
                                int nfreq, const double* omega, const double* gamma, cclr_c64* out,
                                cclr_solve_info* info) {
  if (!c) return CCLR_EINVAL;
  return guarded(c, [&]() -> int {
    auto t0 = std::chrono::steady_clock::now();
    require_t(c);
    REQUIRE(nx >= 1 && ny >= 1 && X && Y && out, CCLR_EINVAL, "need nx, ny >= 1 perturbations and an output array");
    check_freqs(nfreq, omega, gamma);
    const i64 n = c->o + c->v, ov = c->ns(), nd = c->nd();
    for (int p = 0; p < nx; ++p) check_ptr(X[p], "X");
    for (int q = 0; q < ny; ++q) check_ptr(Y[q], "Y");
    for (int p = 0; p < nx + ny; ++p) {
      Arena::Mark mk = c->arena.mark();
      check_finite(c, (const cplx*)(p < nx ? X[p] : Y[p - nx]), n * n, "X/Y");
      c->arena.reset(mk);
    }
    cclr_solve_info linfo{}, rinfo{}, minfo{};
    long nsig = 0;
    int rc = CCLR_OK;
    if (!c->have_lam) {
      rc = solve_lambda_impl(c, &linfo);
      nsig += linfo.nsigma;
      if (rc < 0) return rc;
    }
    Arena::Mark mk = c->arena.mark();
    VecSet xiX = packed_buf(c, nx), etX = packed_buf(c, nx), xiY = packed_buf(c, ny), etY = packed_buf(c, ny);
    for (int p = 0; p < nx; ++p) {
      build_xi(c, (const cplx*)X[p], VecSet{xiX.s + p * ov, xiX.d + p * nd, 1});
      build_eta(c, (const cplx*)X[p], VecSet{etX.s + p * ov, etX.d + p * nd, 1});
    }
    for (int q = 0; q < ny; ++q) {
      build_xi(c, (const cplx*)Y[q], VecSet{xiY.s + q * ov, xiY.d + q * nd, 1});
      build_eta(c, (const cplx*)Y[q], VecSet{etY.s + q * ov, etY.d + q * nd, 1});
    }
    // frequencies z and -conj z of every request
    std::vector<std::complex<double>> fr;
    auto fid = [&](std::complex<double> w) {
      for (size_t k = 0; k < fr.size(); ++k)
        if (fr[k] == w) return (int)k;
      fr.push_back(w);
      return (int)fr.size() - 1;
    };
    std::vector<int> idz(nfreq), idmcz(nfreq);
    for (int w = 0; w < nfreq; ++w) {
      const std::complex<double> z(omega[w], gamma[w]);
      idz[w] = fid(z);
      idmcz[w] = fid(-std::conj(z));
    }
    const int nf = (int)fr.size(), nr = nf * ny;  // (f, q) at f*ny + q
    VecSet rhs = packed_buf(c, nr), sol = packed_buf(c, nr), tf = packed_buf(c, nr), tb = packed_buf(c, nr);
    std::vector<cplx> zr(nr), zl(nr);
    for (int f = 0; f < nf; ++f)
      for (int q = 0; q < ny; ++q) {
        const int r = f * ny + q;
        zr[r] = cx(fr[f].real(), fr[f].imag());
        zl[r] = cx(-fr[f].real(), -fr[f].imag());
        HIPCHK(hipMemcpyAsync(rhs.s + r * ov, xiY.s + q * ov, sizeof(cplx) * ov, hipMemcpyDeviceToDevice, c->stream));
        HIPCHK(hipMemcpyAsync(rhs.d + r * nd, xiY.d + q * nd, sizeof(cplx) * nd, hipMemcpyDeviceToDevice, c->stream));
      }
    const int rs = solve_system(c, CCLR_RIGHT, nr, zr.data(), rhs, sol, &rinfo);
    nsig += rinfo.nsigma;
    // multiplier responses: tbar (A + f) = -(eta^Y + F t^Y(f))
    hessian_product(c, sol, tf);
    for (int f = 0; f < nf; ++f)
      for (int q = 0; q < ny; ++q) {
        const int r = f * ny + q;
        launch_caxpy(ov, cx(1.0), etY.s + q * ov, tf.s + r * ov, c->stream);
        launch_caxpy(nd, cx(1.0), etY.d + q * nd, tf.d + r * nd, c->stream);
      }
    const int ls = solve_system(c, CCLR_LEFT, nr, zl.data(), tf, tb, &minfo);
    nsig += minfo.nsigma;
    // a_pq(f) = eta^p . t^q(f) + tbar^q(f) . xi^p
    std::vector<const cplx*> hx_s, hx_d, hy_s, hy_d;
    for (int r = 0; r < nr; ++r)
      for (int p = 0; p < nx; ++p) {
        hx_s.push_back(etX.s + p * ov), hx_d.push_back(etX.d + p * nd);
        hy_s.push_back(sol.s + r * ov), hy_d.push_back(sol.d + r * nd);
        hx_s.push_back(tb.s + r * ov), hx_d.push_back(tb.d + r * nd);
        hy_s.push_back(xiX.s + p * ov), hy_d.push_back(xiX.d + p * nd);
      }
    const int np = (int)hx_s.size();
    const cplx** pd = (const cplx**)c->arena.get(sizeof(cplx*) * 4 * np);
    std::vector<const cplx*> all;
    all.insert(all.end(), hx_s.begin(), hx_s.end());
    all.insert(all.end(), hx_d.begin(), hx_d.end());
    all.insert(all.end(), hy_s.begin(), hy_s.end());
    all.insert(all.end(), hy_d.begin(), hy_d.end());
    HIPCHK(hipMemcpyAsync(pd, all.data(), sizeof(cplx*) * 4 * np, hipMemcpyHostToDevice, c->stream));
    cplx* partial = (cplx*)c->arena.get(sizeof(cplx) * (size_t)np * 256);
    cplx* dots = (cplx*)c->arena.get(sizeof(cplx) * np);
    launch_bdot(np, pd, pd + np, pd + 2 * np, pd + 3 * np, ov, nd, partial, dots, c->stream);
    std::vector<cplx> hd(np);
    HIPCHK(hipMemcpyAsync(hd.data(), dots, sizeof(cplx) * np, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    auto a = [&](int f, int p, int q) {
      const int k = 2 * ((f * ny + q) * nx + p);
      return std::complex<double>(hd[k].x, hd[k].y) + std::complex<double>(hd[k + 1].x, hd[k + 1].y);
    };
    for (int w = 0; w < nfreq; ++w)
      for (int p = 0; p < nx; ++p)
        for (int q = 0; q < ny; ++q) {
          const std::complex<double> val = 0.5 * (a(idz[w], p, q) + std::conj(a(idmcz[w], p, q)));
          out[((i64)w * nx + p) * ny + q] = cclr_c64{val.real(), val.imag()};
        }
    c->arena.reset(mk);
    if (info) {
      info->iters = std::max(std::max(rinfo.iters, minfo.iters), linfo.iters);
      info->converged = rinfo.converged && minfo.converged && (linfo.iters == 0 || linfo.converged);
      info->resnorm = std::max(std::max(rinfo.resnorm, minfo.resnorm), linfo.resnorm);
      info->nsigma = nsig;
      info->kappa = info->ritz_min = 0.0;
      for (const cclr_solve_info* x : {&rinfo, &minfo, &linfo}) merge_conditioning(*info, *x);
      info->time_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    if (rc == CCLR_ENOTCONV || rs == CCLR_ENOTCONV || ls == CCLR_ENOTCONV) return CCLR_ENOTCONV;
    return CCLR_OK;
  });
}

int cclr_response_backward(cclr_ctx* c, int nx, const cclr_c64* const* X, int nfreq, const double* omega,
                           const double* gamma, const cclr_c64* Gh, cclr_c64* const* dX, cclr_c64* df,
                           cclr_c64* const* dV, cclr_solve_info* info) {
  if (!c) return CCLR_EINVAL;
  return guarded(c, [&]() -> int {
    auto t0 = std::chrono::steady_clock::now();
    require_t(c);
    REQUIRE(nx >= 1 && X && Gh, CCLR_EINVAL, "need perturbations and G");
    REQUIRE((df == nullptr) == (dV == nullptr), CCLR_EINVAL, "df and dV are given together or not at all");
    REQUIRE(dX || df, CCLR_EINVAL, "no gradient requested (dX, df and dV are NULL)");
    check_freqs(nfreq, omega, gamma);
    const i64 n = c->o + c->v, ov = c->ns(), nd = c->nd();
    for (int p = 0; p < nx; ++p) {
      check_ptr(X[p], "X");
      if (dX) check_ptr(dX[p], "dX");
    }
    if (df) {
      check_ptr(df, "df");
      for (int b = 0; b < 6; ++b) check_ptr(dV[b], "dV");
    }
    for (int k = 0; k < nfreq * nx * nx; ++k)
      REQUIRE(std::isfinite(Gh[k].re) && std::isfinite(Gh[k].im), CCLR_EINVAL, "non-finite G");
    cclr_solve_info linfo{}, sinfo{}, ainfo{};
    long nsig = 0;
    int rc = CCLR_OK;
    if (!c->have_lam) {
      rc = solve_lambda_impl(c, &linfo);
      nsig += linfo.nsigma;
      if (rc < 0) return rc;
    }
    Arena::Mark mk = c->arena.mark();
    VecSet xi = packed_buf(c, nx), eta = packed_buf(c, nx);
    for (int p = 0; p < nx; ++p) {
      build_xi(c, (const cplx*)X[p], VecSet{xi.s + p * ov, xi.d + p * nd, 1});
      build_eta(c, (const cplx*)X[p], VecSet{eta.s + p * ov, eta.d + p * nd, 1});
    }
    std::vector<std::complex<double>> fr;
    auto fid = [&](std::complex<double> w) {
      for (size_t k = 0; k < fr.size(); ++k)
        if (fr[k] == w) return (int)k;
      fr.push_back(w);
      return (int)fr.size() - 1;
    };
    for (int w = 0; w < nfreq; ++w) {
      const std::complex<double> z(omega[w], gamma[w]);
      fid(z), fid(-z), fid(std::conj(z)), fid(-std::conj(z));
    }
    const int nf = (int)fr.size(), nr = nf * nx;
    VecSet rhs = packed_buf(c, nr), sol = packed_buf(c, nr), tf = packed_buf(c, nr);
    std::vector<cplx> zr(nr);
    for (int f = 0; f < nf; ++f)
      for (int p = 0; p < nx; ++p) {
        const int r = f * nx + p;
        zr[r] = cx(fr[f].real(), fr[f].imag());
        HIPCHK(hipMemcpyAsync(rhs.s + r * ov, xi.s + p * ov, sizeof(cplx) * ov, hipMemcpyDeviceToDevice, c->stream));
        HIPCHK(hipMemcpyAsync(rhs.d + r * nd, xi.d + p * nd, sizeof(cplx) * nd, hipMemcpyDeviceToDevice, c->stream));
      }
    const int rs = solve_system(c, CCLR_RIGHT, nr, zr.data(), rhs, sol, &sinfo);
    nsig += sinfo.nsigma;
    hessian_product(c, sol, tf);
    // adjoint right-hand sides u[f][r] (left solves) and density vectors y[r] (eta densities)
    VecSet U = packed_buf(c, nr), Y = packed_buf(c, nx);
    // Hessian pairings (F PA_r) . t_r for the Hamiltonian gradient: PA_r = sum cf t^p(-s), r = (s, q)
    VecSet PA = df ? packed_buf(c, nr) : VecSet{};
    if (df) {
      launch_fill(PA.s, nr * ov, cx(0.0), c->stream);
      launch_fill(PA.d, nr * nd, cx(0.0), c->stream);
    }
    launch_fill(U.s, nr * ov, cx(0.0), c->stream);
    launch_fill(U.d, nr * nd, cx(0.0), c->stream);
    launch_fill(Y.s, nx * ov, cx(0.0), c->stream);
    launch_fill(Y.d, nx * nd, cx(0.0), c->stream);
    auto axpy = [&](const VecSet& dst, int kd, const VecSet& src, int ks, std::complex<double> a) {
      if (a == 0.0) return;
      launch_caxpy(ov, cx(a.real(), a.imag()), src.s + ks * ov, dst.s + kd * ov, c->stream);
      launch_caxpy(nd, cx(a.real(), a.imag()), src.d + ks * nd, dst.d + kd * nd, c->stream);
    };
    // L = Re sum conj(G) out, out = 1/2 [g(z) + conj g(-z*)]  =>  L = Re h,
    // h = sum c1 g(z) + c2 g(-z*),  c1 = conj(G)/2,  c2 = G/2  (h holomorphic in X)
    // g_pq(s) = eta^p t^q(s) + eta^q t^p(-s) + (F t^p(-s)) t^q(s)
    for (int w = 0; w < nfreq; ++w) {
      const std::complex<double> z(omega[w], gamma[w]);
      for (int part = 0; part < 2; ++part) {
        const std::complex<double> s_ = part == 0 ? z : -std::conj(z);
        const int fs = fid(s_), fms = fid(-s_);
        for (int p = 0; p < nx; ++p)
          for (int q = 0; q < nx; ++q) {
            const cclr_c64 g = Gh[((i64)w * nx + p) * nx + q];
            const std::complex<double> cf = part == 0 ? 0.5 * std::complex<double>(g.re, -g.im)
                                                      : 0.5 * std::complex<double>(g.re, g.im);
            // eta^p . t^q(s): density of eta in X_p with vector t^q(s)
            axpy(Y, p, sol, fs * nx + q, cf);
            // eta^q . t^p(-s): density of eta in X_q with t^p(-s)
            axpy(Y, q, sol, fms * nx + p, cf);
            // t^q(s) = -(A - s)^-1 xi^q with coefficient vector eta^p + F t^p(-s): left solve at s for X_q
            axpy(U, fs * nx + q, eta, p, cf);
            axpy(U, fs * nx + q, tf, fms * nx + p, cf);
            // t^p(-s) with coefficient vector eta^q + F t^q(s): left solve at -s for X_p
            axpy(U, fms * nx + p, eta, q, cf);
            axpy(U, fms * nx + p, tf, fs * nx + q, cf);
            if (df) axpy(PA, fs * nx + q, sol, fms * nx + p, cf);
          }
      }
    }
    // left solves x (A - f) = -u  =>  u . t^X(f) = x . xi^X
    VecSet xl = packed_buf(c, nr);
    const int ra = solve_system(c, CCLR_LEFT, nr, zr.data(), U, xl, &ainfo);
    nsig += ainfo.nsigma;
    if (dX) {
      for (int r = 0; r < nx; ++r) launch_fill((cplx*)dX[r], n * n, cx(0.0), c->stream);
      for (int f = 0; f < nf; ++f)
        for (int r = 0; r < nx; ++r)
          density_xi(c, VecSet{xl.s + (f * nx + r) * ov, xl.d + (f * nx + r) * nd, 1}, (cplx*)dX[r], cx(1.0));
      for (int r = 0; r < nx; ++r)
        density_eta(c, VecSet{Y.s + r * ov, Y.d + r * nd, 1}, (cplx*)dX[r], cx(1.0));
      // dL/dRe X + i dL/dIm X = conj(dh/dX)
      for (int r = 0; r < nx; ++r) launch_conj_inplace(n * n, (cplx*)dX[r], c->stream);
    }
    cclr_solve_info hinfo{};
    if (df) {
      cplx* Xs = (cplx*)c->arena.get(sizeof(cplx) * (size_t)(nx * n * n));
      for (int p = 0; p < nx; ++p)
        HIPCHK(hipMemcpyAsync(Xs + p * n * n, X[p], sizeof(cplx) * n * n, hipMemcpyDeviceToDevice, c->stream));
      hamiltonian_adjoint(c, nx, Xs, sol, xl, Y, PA, sol, (cplx*)df, (cplx* const*)dV, &hinfo);
      nsig += hinfo.nsigma;
    }
    HIPCHK(hipStreamSynchronize(c->stream));
    c->arena.reset(mk);
    if (info) {
      info->iters = std::max(std::max(sinfo.iters, ainfo.iters), linfo.iters);
      info->converged = sinfo.converged && ainfo.converged && (linfo.iters == 0 || linfo.converged) &&
                        (!df || hinfo.converged);
      info->resnorm = std::max(std::max(std::max(sinfo.resnorm, ainfo.resnorm), linfo.resnorm), hinfo.resnorm);
      info->nsigma = nsig;
      info->kappa = info->ritz_min = 0.0;
      for (const cclr_solve_info* x : {&sinfo, &ainfo, &linfo, &hinfo}) merge_conditioning(*info, *x);
      info->time_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    if (rc == CCLR_ENOTCONV || rs == CCLR_ENOTCONV || ra == CCLR_ENOTCONV || (df && !hinfo.converged))
      return CCLR_ENOTCONV;
    return CCLR_OK;
  });
}

}  // extern "C"
