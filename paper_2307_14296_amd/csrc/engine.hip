// Device memory management, tensor views and the contraction engine.
//
// contract() evaluates C[lc] += alpha * sum A[la] B[lb] by classifying the
// labels (batch: in A, B and C; M: A and C; N: B and C; K: A and B), viewing
// each operand as a strided [batch][M][K] / [batch][K][N] / [batch][M][N]
// matrix when its axes can be merged, and copying it into a packed
// temporary otherwise.  The product itself runs on the FP64-MFMA complex
// GEMM kernel.
#include <algorithm>
#include <cstring>

#include <cmath>

#include "internal.h"

// ------------------------------------------------------------ allocation
void DevBuf::alloc(cclr_ctx* c, size_t nbytes) {
  if (p && nbytes == bytes && ctx == c) return;  // same size: keep the allocation
  release();
  if (nbytes == 0) return;
  if (c->opt.device_mem_cap && c->allocated + nbytes > c->opt.device_mem_cap)
    throw CclrError(CCLR_ENOMEM, "device memory cap exceeded (" + std::to_string(c->allocated + nbytes) +
                                     " > " + std::to_string(c->opt.device_mem_cap) + " bytes)");
  hipError_t e = hipMalloc(&p, nbytes);
  if (e != hipSuccess) {
    p = nullptr;
    (void)hipGetLastError();
    throw CclrError(CCLR_ENOMEM, "hipMalloc of " + std::to_string(nbytes) + " bytes failed");
  }
  ctx = c;
  bytes = nbytes;
  c->allocated += nbytes;
}

void DevBuf::release() {
  if (p) {
    (void)hipFree(p);
    if (ctx) ctx->allocated -= bytes;
  }
  p = nullptr;
  bytes = 0;
}

Arena::~Arena() {
  for (auto* b : chunks) delete b;
}

void* Arena::get(size_t bytes) {
  bytes = (bytes + 255) & ~size_t(255);
  if (ext) {
    if (bytes > ext_bytes - ext_used)
      throw CclrError(CCLR_ENOMEM, "work space of " + std::to_string(ext_bytes) + " bytes exhausted (" +
                                       std::to_string(ext_used + bytes) + " bytes needed so far)");
    void* p = ext + ext_used;
    ext_used += bytes;
    ext_peak = std::max(ext_peak, ext_used);
    return p;
  }
  while (cur < chunks.size()) {
    if (used[cur] + bytes <= chunks[cur]->bytes) {
      void* p = (char*)chunks[cur]->p + used[cur];
      used[cur] += bytes;
      return p;
    }
    if (cur + 1 < chunks.size()) ++cur;
    else break;
  }
  DevBuf* b = new DevBuf();
  try {
    b->alloc(ctx, std::max(bytes, chunk_bytes));
  } catch (...) {
    delete b;
    throw;
  }
  chunks.push_back(b);
  used.push_back(bytes);
  cur = chunks.size() - 1;
  return b->p;
}

Arena::Mark Arena::mark() const {
  if (ext) return {size_t(-1), ext_used};
  return {cur, chunks.empty() ? 0 : used[cur]};
}

void Arena::reset(Mark m) {
  if (hold > 0) return;
  if (ext) {
    if (m.chunk == size_t(-1)) ext_used = m.top;
    return;
  }
  if (m.chunk == size_t(-1)) return;  // a mark of the external region
  for (size_t k = m.chunk + 1; k < chunks.size(); ++k) used[k] = 0;
  if (!chunks.empty()) used[m.chunk] = m.top;
  cur = m.chunk;
}

void Arena::trim() {
  // free every chunk after the active one that holds nothing
  (void)hipDeviceSynchronize();
  while (chunks.size() > cur + 1 && used.back() == 0) {
    delete chunks.back();
    chunks.pop_back();
    used.pop_back();
  }
}

// How many of n vectors, each needing bytes_per_vec of working memory, fit
// in the device memory that is still free (and under the context's cap).
// Unused arena chunks are released first so that they count as free.
int fit_vectors(cclr_ctx* c, double bytes_per_vec, int n) {
  if (n <= 1) return n;
  c->arena.trim();
  size_t fr = 0, tot = 0;
  HIPCHK(hipMemGetInfo(&fr, &tot));
  double budget = 0.8 * (double)fr;
  if (c->opt.device_mem_cap) {
    const double left = c->opt.device_mem_cap > c->allocated ? (double)(c->opt.device_mem_cap - c->allocated) : 0.0;
    budget = std::min(budget, left);
  }
  const double k = budget / std::max(bytes_per_vec, 1.0);
  const int fit = (int)std::max(1.0, std::min((double)n, std::floor(k)));
  return c->dbg_rhs_group > 0 ? std::min(fit, c->dbg_rhs_group) : fit;
}

// ------------------------------------------------------------------ views
Ten ten(cplx* p, std::initializer_list<i64> dims) {
  Ten t;
  t.p = p;
  t.nd = (int)dims.size();
  int d = 0;
  for (i64 x : dims) t.dim[d++] = x;
  i64 s = 1;
  for (d = t.nd - 1; d >= 0; --d) {
    t.st[d] = s;
    s *= t.dim[d];
  }
  return t;
}

Ten ten(const DevBuf& b, std::initializer_list<i64> dims) { return ten(b.c(), dims); }

Ten reorder(const Ten& t, const char* from, const char* to) {
  Ten r = t;
  const int n = t.nd;
  REQUIRE((int)strlen(from) == n && (int)strlen(to) == n, CCLR_EINVAL, "reorder: label count");
  for (int d = 0; d < n; ++d) {
    const char* q = strchr(from, to[d]);
    REQUIRE(q, CCLR_EINVAL, "reorder: unknown label");
    const int s = (int)(q - from);
    r.dim[d] = t.dim[s];
    r.st[d] = t.st[s];
  }
  return r;
}

Ten scaled(const Ten& t, double re, double im) {
  Ten r = t;
  const double nr = t.sr * re - t.si * im, ni = t.sr * im + t.si * re;
  r.sr = nr;
  r.si = ni;
  return r;
}

Ten conjugated(const Ten& t) {
  // conj(s * conj?(x)) = conj(s) * conj(conj?(x))
  Ten r = t;
  r.conj = !t.conj;
  r.si = -t.si;
  return r;
}

Ten tmp(cclr_ctx* c, std::initializer_list<i64> dims) {
  i64 n = 1;
  for (i64 x : dims) n *= x;
  cplx* p = (cplx*)c->arena.get(sizeof(cplx) * (size_t)std::max<i64>(n, 1));
  return ten(p, dims);
}

void tzero(cclr_ctx* c, const Ten& t) {
  // only contiguous tensors are zeroed in one sweep
  i64 n = t.size();
  bool contig = true;
  i64 s = 1;
  for (int d = t.nd - 1; d >= 0; --d) {
    if (t.dim[d] != 1 && t.st[d] != s) contig = false;
    s *= t.dim[d];
  }
  if (contig) {
    launch_fill(t.p, n, cx(0.0), c->stream);
    return;
  }
  CopyArgs a{};
  a.nd = t.nd;
  for (int d = 0; d < t.nd; ++d) {
    a.dim[d] = t.dim[d];
    a.sd[d] = t.st[d];
    a.ss[d] = 0;
  }
  // alpha = 0 writes zeros without reading the source
  a.dst = t.p;
  a.src = t.p;
  a.ar = 0.0;
  a.ai = 0.0;
  a.conj = 0;
  a.acc = 0;
  a.total = n;
  launch_tcopy(a, c->stream);
}

// -------------------------------------------------------- copy / permute
static int lpos(const char* l, char ch) {
  const char* q = strchr(l, ch);
  return q ? (int)(q - l) : -1;
}

void tcopy(cclr_ctx* c, const Ten& dst, const char* ld, const Ten& src, const char* ls, cplx alpha,
           bool accumulate) {
  const int n = dst.nd;
  REQUIRE((int)strlen(ld) == n && (int)strlen(ls) == src.nd && src.nd == n, CCLR_EINVAL, "tcopy: labels");
  REQUIRE(!dst.conj && dst.sr == 1.0 && dst.si == 0.0, CCLR_EINVAL, "tcopy: scaled destination");
  CopyArgs a{};
  a.nd = n;
  i64 total = 1;
  for (int d = 0; d < n; ++d) {
    const int s = lpos(ls, ld[d]);
    REQUIRE(s >= 0 && src.dim[s] == dst.dim[d], CCLR_EINVAL, std::string("tcopy: label/dim mismatch ") + ld + " <- " + ls);
    a.dim[d] = dst.dim[d];
    a.sd[d] = dst.st[d];
    a.ss[d] = src.st[s];
    total *= dst.dim[d];
  }
  // alpha * s * op(x)
  a.ar = alpha.x * src.sr - alpha.y * src.si;
  a.ai = alpha.x * src.si + alpha.y * src.sr;
  a.conj = src.conj ? 1 : 0;
  a.acc = accumulate ? 1 : 0;
  a.dst = dst.p;
  a.src = src.p;
  a.total = total;
  launch_tcopy(a, c->stream);
}

// ---------------------------------------------------------------- engine
namespace {
struct Group {
  std::string labels;
  i64 size = 1;
  i64 stride = 0;
  bool ok = true;
};

// View the axes `g` (in this order) of tensor t with labels l as one merged
// axis.  Succeeds if consecutive axes are nested with matching strides.
Group merge(const Ten& t, const char* l, const std::string& g) {
  Group r;
  r.labels = g;
  if (g.empty()) return r;
  i64 size = 1;
  i64 expect = -1;
  for (int q = (int)g.size() - 1; q >= 0; --q) {
    const int d = lpos(l, g[q]);
    const i64 dim = t.dim[d], st = t.st[d];
    if (dim == 1) continue;
    if (expect < 0) {
      r.stride = st;
    } else if (st != expect) {
      r.ok = false;
    }
    expect = st * dim;
    size *= dim;
  }
  r.size = size;
  if (expect < 0) r.stride = 0;
  return r;
}

i64 labsize(const Ten& t, const char* l, char ch) { return t.dim[lpos(l, ch)]; }
}  // namespace

void contract(cclr_ctx* c, cplx alpha, const Ten& A, const char* la, const Ten& B, const char* lb, const Ten& C,
              const char* lc, bool accumulate) {
  REQUIRE((int)strlen(la) == A.nd && (int)strlen(lb) == B.nd && (int)strlen(lc) == C.nd, CCLR_EINVAL,
          std::string("contract: label count ") + la + "," + lb + "->" + lc);
  REQUIRE(!C.conj && C.sr == 1.0 && C.si == 0.0, CCLR_EINVAL, "contract: scaled output");
  std::string Lb, Lm, Ln, Lk;
  for (const char* p = lc; *p; ++p) {
    const bool inA = lpos(la, *p) >= 0, inB = lpos(lb, *p) >= 0;
    REQUIRE(inA || inB, CCLR_EINVAL, std::string("contract: output label not in inputs: ") + lc);
    if (inA && inB) Lb += *p;
    else if (inA) Lm += *p;
    else Ln += *p;
  }
  for (const char* p = la; *p; ++p) {
    if (lpos(lc, *p) < 0) {
      REQUIRE(lpos(lb, *p) >= 0, CCLR_EINVAL, std::string("contract: unsummed label ") + la);
      Lk += *p;
    }
  }
  for (const char* p = lb; *p; ++p)
    if (lpos(lc, *p) < 0) REQUIRE(lpos(la, *p) >= 0, CCLR_EINVAL, std::string("contract: unsummed label ") + lb);
  // sizes must agree
  auto chk = [&](const std::string& g) {
    for (char ch : g) {
      i64 s = -1;
      if (lpos(la, ch) >= 0) s = labsize(A, la, ch);
      if (lpos(lb, ch) >= 0) REQUIRE(s < 0 || labsize(B, lb, ch) == s, CCLR_EINVAL, "contract: size mismatch");
      if (lpos(lc, ch) >= 0 && s >= 0) REQUIRE(labsize(C, lc, ch) == s, CCLR_EINVAL, "contract: size mismatch");
    }
  };
  chk(Lb), chk(Lm), chk(Ln), chk(Lk);

  // Without shared batch labels, output labels of one operand that break the
  // nesting of the M (or N) group can become a batch index of their own (the
  // other operand gets stride 0), which avoids copying large operands.  A
  // small operand may be copied into the order the plan wants.
  if (Lb.empty()) {
    const i64 small = (i64)1 << 22;
    struct Plan {
      std::string sm, rm, sn, rn;
      bool ca = false, cb = false;
      double score = -1;
    } best;
    const int nm = (int)Lm.size(), nn = (int)Ln.size();
    const bool kshort = merge(A, la, Lk).size <= 32;
    for (int ca = 0; ca < 2; ++ca)
      for (int cbq = 0; cbq < 2; ++cbq) {
        if ((ca && A.size() > small) || (cbq && B.size() > small)) continue;
        if (best.score > 0 && (ca + cbq) > (int)best.ca + (int)best.cb) continue;  // fewer copies first
        for (int mm = 0; mm < (1 << nm); ++mm)
          for (int mn = 0; mn < (1 << nn); ++mn) {
            std::string sm, rm, sn, rn;
            for (int q = 0; q < nm; ++q) ((mm >> q) & 1 ? sm : rm) += Lm[q];
            for (int q = 0; q < nn; ++q) ((mn >> q) & 1 ? sn : rn) += Ln[q];
            const bool okA = ca || (merge(A, la, Lk).ok && merge(A, la, rm).ok && merge(A, la, sm).ok);
            const bool okB = cbq || (merge(B, lb, Lk).ok && merge(B, lb, rn).ok && merge(B, lb, sn).ok);
            if (!okA || !okB) continue;
            if (!(merge(C, lc, rm).ok && merge(C, lc, rn).ok && merge(C, lc, sm).ok && merge(C, lc, sn).ok)) continue;
            if (mm == 0 && mn == 0 && !ca && !cbq) continue;  // the plain plan below handles it
            const i64 nbat = merge(C, lc, sm).size * merge(C, lc, sn).size;
            if (nbat >= 65536) continue;
            double score = (double)merge(C, lc, rm).size * (double)merge(C, lc, rn).size;
            // a short reduction runs on the vector ALU and is bound by its output
            // traffic: prefer plans whose output has a unit-stride M or N index
            if (kshort) {
              const Group gm = merge(C, lc, rm), gn = merge(C, lc, rn);
              if ((gm.size > 1 && gm.stride == 1) || (gn.size > 1 && gn.stride == 1)) score *= 64.0;
            }
            const bool fewer = (ca + cbq) < (int)best.ca + (int)best.cb;
            if (best.score < 0 || fewer || score > best.score) best = Plan{sm, rm, sn, rn, ca != 0, cbq != 0, score};
          }
      }
    const bool okA0 = merge(A, la, Lk).ok && merge(A, la, Lm).ok, okB0 = merge(B, lb, Lk).ok && merge(B, lb, Ln).ok,
               okC0 = merge(C, lc, Lm).ok && merge(C, lc, Ln).ok;
    // bytes the plain path would copy
    const i64 copied = (okA0 ? 0 : A.size()) + (okB0 ? 0 : B.size()) + (okC0 ? 0 : 2 * C.size());
    if (!(okA0 && okB0 && okC0) && copied > small && best.score > 0) {
      Arena::Mark mk = c->arena.mark();
      Ten Aw = A, Bw = B;
      std::string law = la, lbw = lb;
      auto relayout = [&](const Ten& X, const char* lx, const std::string& order, Ten& out, std::string& lout) {
        i64 n = 1;
        for (char ch : order) n *= labsize(X, lx, ch);
        Ten T;
        T.p = (cplx*)c->arena.get(sizeof(cplx) * (size_t)std::max<i64>(n, 1));
        T.nd = (int)order.size();
        i64 st = 1;
        for (int d = T.nd - 1; d >= 0; --d) {
          T.dim[d] = labsize(X, lx, order[d]);
          T.st[d] = st;
          st *= T.dim[d];
        }
        tcopy(c, T, order.c_str(), X, lx, cx(1.0), false);
        out = T;
        lout = order;
      };
      if (best.ca) relayout(A, la, best.sm + best.rm + Lk, Aw, law);
      if (best.cb) relayout(B, lb, best.sn + Lk + best.rn, Bw, lbw);
      const Group Am2 = merge(Aw, law.c_str(), best.rm), Ak2 = merge(Aw, law.c_str(), Lk),
                  As = merge(Aw, law.c_str(), best.sm);
      const Group Bn2 = merge(Bw, lbw.c_str(), best.rn), Bk2 = merge(Bw, lbw.c_str(), Lk),
                  Bs = merge(Bw, lbw.c_str(), best.sn);
      const Group Cm2 = merge(C, lc, best.rm), Cn2 = merge(C, lc, best.rn), Cs1 = merge(C, lc, best.sn),
                  Cs2 = merge(C, lc, best.sm);
      // a copied operand already carries its scale and conjugation
      const double sr = Aw.sr * Bw.sr - Aw.si * Bw.si, si = Aw.sr * Bw.si + Aw.si * Bw.sr;
      GemmArgs g{};
      g.M = (int)Am2.size;
      g.N = (int)Bn2.size;
      g.K = (int)Ak2.size;
      g.nb2 = (int)Cs2.size;
      g.batch = (int)(Cs1.size * Cs2.size);
      g.A = Aw.p; g.sAb = 0; g.sAb2 = As.stride; g.sAm = Am2.stride; g.sAk = Ak2.stride; g.conjA = Aw.conj;
      g.B = Bw.p; g.sBb = Bs.stride; g.sBb2 = 0; g.sBk = Bk2.stride; g.sBn = Bn2.stride; g.conjB = Bw.conj;
      g.C = C.p; g.sCb = Cs1.stride; g.sCb2 = Cs2.stride; g.sCm = Cm2.stride; g.sCn = Cn2.stride;
      g.ar = alpha.x * sr - alpha.y * si;
      g.ai = alpha.x * si + alpha.y * sr;
      g.beta = accumulate ? 1 : 0;
      REQUIRE(Am2.size < (1ll << 31) && Bn2.size < (1ll << 31) && Ak2.size < (1ll << 31), CCLR_EINVAL,
              "contract: dimension too large for one GEMM");
      if (g.K == 0) {
        if (!accumulate) tzero(c, C);
      } else {
        run_gemm(c, g);
      }
      c->arena.reset(mk);
      return;
    }
  }
  Arena::Mark mk = c->arena.mark();
  // ---- A as [b][m][k]
  Group Ab = merge(A, la, Lb), Am = merge(A, la, Lm), Ak = merge(A, la, Lk);
  Ten Aw = A;
  std::string law = la;
  if (!(Ab.ok && Am.ok && Ak.ok)) {
    std::string nl = Lb + Lm + Lk;
    Ten T = tmp(c, {1});
    // allocate contiguous buffer
    i64 n = 1;
    for (char ch : nl) n *= labsize(A, la, ch);
    T.p = (cplx*)c->arena.get(sizeof(cplx) * (size_t)n);
    T.nd = (int)nl.size();
    i64 s = 1;
    for (int d = T.nd - 1; d >= 0; --d) {
      T.dim[d] = labsize(A, la, nl[d]);
      T.st[d] = s;
      s *= T.dim[d];
    }
    tcopy(c, T, nl.c_str(), A, la, cx(1.0), false);
    Aw = T;
    law = nl;
    Ab = merge(Aw, law.c_str(), Lb), Am = merge(Aw, law.c_str(), Lm), Ak = merge(Aw, law.c_str(), Lk);
  }
  // ---- B as [b][k][n]
  Group Bb = merge(B, lb, Lb), Bk = merge(B, lb, Lk), Bn = merge(B, lb, Ln);
  Ten Bw = B;
  std::string lbw = lb;
  if (!(Bb.ok && Bk.ok && Bn.ok)) {
    std::string nl = Lb + Lk + Ln;
    i64 n = 1;
    for (char ch : nl) n *= labsize(B, lb, ch);
    Ten T;
    T.p = (cplx*)c->arena.get(sizeof(cplx) * (size_t)n);
    T.nd = (int)nl.size();
    i64 s = 1;
    for (int d = T.nd - 1; d >= 0; --d) {
      T.dim[d] = labsize(B, lb, nl[d]);
      T.st[d] = s;
      s *= T.dim[d];
    }
    tcopy(c, T, nl.c_str(), B, lb, cx(1.0), false);
    Bw = T;
    lbw = nl;
    Bb = merge(Bw, lbw.c_str(), Lb), Bk = merge(Bw, lbw.c_str(), Lk), Bn = merge(Bw, lbw.c_str(), Ln);
  }
  // ---- C as [b][m][n]
  Group Cb = merge(C, lc, Lb), Cm = merge(C, lc, Lm), Cn = merge(C, lc, Ln);
  // a copied operand already carries its scale and conjugation
  const double sr = Aw.sr * Bw.sr - Aw.si * Bw.si, si = Aw.sr * Bw.si + Aw.si * Bw.sr;
  const cplx al = cx(alpha.x * sr - alpha.y * si, alpha.x * si + alpha.y * sr);

  GemmArgs g{};
  g.M = (int)Am.size;
  g.N = (int)Bn.size;
  g.K = (int)Ak.size;
  g.batch = (int)Ab.size;
  g.A = Aw.p; g.sAb = Ab.stride; g.sAm = Am.stride; g.sAk = Ak.stride; g.conjA = Aw.conj;
  g.B = Bw.p; g.sBb = Bb.stride; g.sBk = Bk.stride; g.sBn = Bn.stride; g.conjB = Bw.conj;
  REQUIRE(Am.size < (1ll << 31) && Bn.size < (1ll << 31) && Ak.size < (1ll << 31) && Ab.size < 65536, CCLR_EINVAL,
          "contract: dimension too large for one GEMM");

  if (Cb.ok && Cm.ok && Cn.ok) {
    g.C = C.p; g.sCb = Cb.stride; g.sCm = Cm.stride; g.sCn = Cn.stride;
    g.ar = al.x; g.ai = al.y; g.beta = accumulate ? 1 : 0;
    if (g.K == 0) {
      if (!accumulate) tzero(c, C);
    } else {
      run_gemm(c, g);
    }
  } else {
    std::string nl = Lb + Lm + Ln;
    i64 n = 1;
    for (char ch : nl) n *= labsize(C, lc, ch);
    Ten T;
    T.p = (cplx*)c->arena.get(sizeof(cplx) * (size_t)n);
    T.nd = (int)nl.size();
    i64 s = 1;
    for (int d = T.nd - 1; d >= 0; --d) {
      T.dim[d] = labsize(C, lc, nl[d]);
      T.st[d] = s;
      s *= T.dim[d];
    }
    g.C = T.p;
    g.sCb = g.M * (i64)g.N;
    g.sCm = g.N;
    g.sCn = 1;
    g.ar = al.x; g.ai = al.y; g.beta = 0;
    run_gemm(c, g);
    tcopy(c, C, lc, T, nl.c_str(), cx(1.0), accumulate);
  }
  c->arena.reset(mk);
}

// GEMM dispatch: products whose output covers too few 64x64 tiles to occupy
// the 256 compute units split the reduction into chunks that write partial
// products to a workspace, summed in a fixed order afterwards.
// form: the kernel that ran (FP64 variant >= 0, -1 short-reduction VALU
// kernel, -2 split-K with the default variant, -3 reduced precision, -4
// short-output VALU kernel, -5 reduced precision on pre-split FP32 planes, -6
// short-output VALU kernel on a long operand contiguous in k)
static void run_gemm_form(cclr_ctx* c, const GemmArgs& g, int& form);
void run_gemm(cclr_ctx* c, const GemmArgs& g) {
  if (g.M <= 0 || g.N <= 0 || g.batch <= 0 || g.K <= 0) return;
  int form = 0;
  if (!c->gemm_trace) {
    run_gemm_form(c, g, form);
    return;
  }
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  HIPCHK(hipEventRecord(e0, c->stream));
  run_gemm_form(c, g, form);
  HIPCHK(hipEventRecord(e1, c->stream));
  HIPCHK(hipEventSynchronize(e1));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  char line[384];
  snprintf(line, sizeof line,
           "%dx%dx%d b%d sA(%lld,%lld) sB(%lld,%lld) sC(%lld,%lld) sb(%lld,%lld,%lld) beta %d form %d %.4f ms "
           "%.2f TFLOP/s",
           g.M, g.N, g.K, g.batch, (long long)g.sAm, (long long)g.sAk, (long long)g.sBk, (long long)g.sBn,
           (long long)g.sCm, (long long)g.sCn, (long long)g.sAb, (long long)g.sBb, (long long)g.sCb, g.beta, form, ms,
           8.0 * g.M * (double)g.N * g.K * g.batch / (ms * 1e-3) / 1e12);
  c->gemm_trace_log.push_back(line);
}

// C^T = B^T A^T: the same product with the roles of m and n exchanged
static GemmArgs transposed(const GemmArgs& g0) {
  GemmArgs g = g0;
  g.M = g0.N; g.N = g0.M;
  g.A = g0.B; g.sAb = g0.sBb; g.sAb2 = g0.sBb2; g.sAm = g0.sBn; g.sAk = g0.sBk; g.conjA = g0.conjB;
  g.B = g0.A; g.sBb = g0.sAb; g.sBb2 = g0.sAb2; g.sBk = g0.sAk; g.sBn = g0.sAm; g.conjB = g0.conjA;
  g.sCm = g0.sCn; g.sCn = g0.sCm;
  return g;
}

// dst[b][e][r][q] (+)= src[b][e][r][q] between two strided 4-index views
// (b, e: the two levels of a GEMM batch)
static void copy4(cclr_ctx* c, const i64 (&dim)[4], cplx* dst, const i64 (&sd)[4], const cplx* src,
                  const i64 (&ss)[4], bool acc) {
  CopyArgs a{};
  a.nd = 4;
  a.total = 1;
  for (int d = 0; d < 4; ++d) {
    a.dim[d] = dim[d];
    a.sd[d] = sd[d];
    a.ss[d] = ss[d];
    a.total *= dim[d];
  }
  a.dst = dst;
  a.src = src;
  a.ar = 1.0;
  a.ai = 0.0;
  a.conj = 0;
  a.acc = acc ? 1 : 0;
  launch_tcopy(a, c->stream);
}

static void run_gemm_form(cclr_ctx* c, const GemmArgs& g0, int& form) {
  form = -1;
  // An operand or output whose unit stride is a batch index would have every
  // tile (or every thread's row) touch one element per cache line of it:
  // such tensors are copied to a batch-outermost layout first, and the
  // output is added back afterwards.
  if (g0.kchunk == 0 && g0.batch >= 8) {
    const i64 M = g0.M, N = g0.N, K = g0.K;
    const i64 n2 = g0.nb2 > 1 ? g0.nb2 : 1, n1 = g0.batch / n2;
    auto inner = [&](i64 s1, i64 s2, i64 sz) { return sz > 1 && ((n1 > 1 && s1 == 1) || (n2 > 1 && s2 == 1)); };
    const bool ca = inner(g0.sAb, g0.sAb2, M * K), cb = inner(g0.sBb, g0.sBb2, K * N),
               cc = inner(g0.sCb, g0.sCb2, M * N);
    const i64 big = (i64)g0.batch * std::max({ca ? M * K : 0, cb ? K * N : 0, cc ? M * N : 0});
    if ((ca || cb || cc) && big >= (i64(1) << 20)) {
      Arena::Mark mk = c->arena.mark();
      GemmArgs h = g0;
      const i64 s2b = n2 > 1 ? 1 : 0;  // the second batch level's stride factor in the copies
      if (ca) {
        cplx* t = (cplx*)c->arena.get(sizeof(cplx) * (size_t)(g0.batch * M * K));
        copy4(c, {n1, n2, M, K}, t, {n2 * M * K, M * K, K, 1}, g0.A, {g0.sAb, s2b * g0.sAb2, g0.sAm, g0.sAk}, false);
        h.A = t; h.sAb = n2 * M * K; h.sAb2 = M * K; h.sAm = K; h.sAk = 1;
      }
      if (cb) {
        cplx* t = (cplx*)c->arena.get(sizeof(cplx) * (size_t)(g0.batch * K * N));
        copy4(c, {n1, n2, K, N}, t, {n2 * K * N, K * N, N, 1}, g0.B, {g0.sBb, s2b * g0.sBb2, g0.sBk, g0.sBn}, false);
        h.B = t; h.sBb = n2 * K * N; h.sBb2 = K * N; h.sBk = N; h.sBn = 1;
      }
      if (cc) {
        cplx* t = (cplx*)c->arena.get(sizeof(cplx) * (size_t)(g0.batch * M * N));
        h.C = t; h.sCb = n2 * M * N; h.sCb2 = M * N; h.sCm = N; h.sCn = 1; h.beta = 0;
      }
      run_gemm_form(c, h, form);
      if (cc)
        copy4(c, {n1, n2, M, N}, g0.C, {g0.sCb, s2b * g0.sCb2, g0.sCm, g0.sCn}, h.C, {n2 * M * N, M * N, N, 1},
              g0.beta != 0);
      c->arena.reset(mk);
      return;
    }
  }
  if (g0.K <= 32 && launch_zgemm_smallk(g0, c->stream)) return;
  // the MFMA tiles are at least 32 columns but 64 (FP64) or 128 (FP32) rows
  // high: a product with a short m side (at most 32) and a long n side runs
  // transposed, so that its short side can take the 32-column tiles
  const GemmArgs g = (g0.M <= 32 && g0.N > 32) ? transposed(g0) : g0;
  {
    // at most 16 output columns: FP64 VALU rows instead of mostly empty MFMA tiles
    GemmArgs h;
    int kc = 0, S = 0;
    if (skinny_plan(g, h, kc, S)) {
      form = -4;
      if (S == 1) {
        launch_zgemm_skinny(h, kc, 1, nullptr, c->stream);
        return;
      }
      Arena::Mark mk = c->arena.mark();
      cplx* W = (cplx*)c->arena.get(sizeof(cplx) * (size_t)h.batch * S * h.M * (size_t)h.N);
      launch_zgemm_skinny(h, kc, S, W, c->stream);
      c->arena.reset(mk);
      return;
    }
    // at most 8 output columns, long operand contiguous in k: rows dotted along k
    if (rowdot_plan(g, kc, S)) {
      form = -6;
      if (S == 1) {
        launch_zgemm_rowdot(g, kc, 1, nullptr, c->stream);
        return;
      }
      Arena::Mark mk = c->arena.mark();
      cplx* W = (cplx*)c->arena.get(sizeof(cplx) * (size_t)g.batch * S * g.M * (size_t)g.N);
      launch_zgemm_rowdot(g, kc, S, W, c->stream);
      c->arena.reset(mk);
      return;
    }
  }
  // inside reduced-precision transforms the remaining products run on FP32 MFMA as well
  const bool lowp = c->sigma_prec != CCLR_FP64;
  const i64 tiles = (i64)((g.M + 63) / 64) * ((g.N + 63) / 64) * g.batch;
  if (g.nb2 <= 1 && tiles < 512 && g.K >= 512) {
    i64 S = std::min<i64>((1024 + tiles - 1) / tiles, g.K / 256);
    S = std::max<i64>(S, 2);
    i64 kc = (g.K + S - 1) / S;
    kc = (kc + 15) / 16 * 16;
    S = (g.K + kc - 1) / kc;
    if ((i64)g.batch * S < 65536) {
      Arena::Mark mk = c->arena.mark();
      cplx* W = (cplx*)c->arena.get(sizeof(cplx) * (size_t)(g.batch * S * g.M * (i64)g.N));
      GemmArgs h = g;
      h.kchunk = (int)kc;
      h.batch = (int)(g.batch * S);
      h.nb2 = 0;
      h.C = W;
      h.sCb = (i64)g.M * g.N;
      h.sCm = g.N;
      h.sCn = 1;
      h.ar = 1.0;
      h.ai = 0.0;
      h.beta = 0;
      form = lowp ? -3 : -2;
      if (lowp) launch_zgemm_lowp(h, CCLR_FP32, c->stream);
      else tuned_gemm(c, h);
      launch_splitk_reduce(g.batch, (int)S, g.M, g.N, W, g.C, g.sCb, g.sCm, g.sCn, g.ar, g.ai, g.beta, c->stream);
      c->arena.reset(mk);
      return;
    }
  }
  if (lowp) {
    form = -3;
    // large single products: each operand converted once to the three FP32
    // Gauss planes, then the direct-load split kernel (the conversion passes
    // cost less than the gain over converting inside the K loop once both
    // output sides are a few hundred long)
    if (g.batch == 1 && g.kchunk == 0 && g.nb2 <= 1 && g.M >= 512 && g.N >= 512 && g.K >= 256) {
      form = -5;
      Arena::Mark mk = c->arena.mark();
      void* wa = c->arena.get(split_bytes(g.M, g.K, F32_G3, 0));
      void* wb = c->arena.get(split_bytes(g.N, g.K, F32_G3, 1));
      const SplitMat A = launch_split(g.M, g.K, g.A, g.sAm, g.sAk, g.conjA, wa, F32_G3, 0, c->stream);
      const SplitMat B = launch_split(g.N, g.K, g.B, g.sBn, g.sBk, g.conjB, wb, F32_G3, 1, c->stream);
      launch_split_gemm(A, B, g.C, g.sCm, g.sCn, g.ar, g.ai, g.beta, c->stream);
      c->arena.reset(mk);
      return;
    }
    launch_zgemm_lowp(g, CCLR_FP32, c->stream);
  } else {
    form = tuned_gemm(c, g);
  }
}

// Autotuner.  The first time a large product of a given shape class (M, N,
// K, batch, operand layouts) is requested, every MFMA kernel variant is
// timed once with HIP events on a scratch output of the same strides, and
// the fastest is cached in the context.  Products under 1e10 flop use the
// untimed choice.
// The row count M and the batch count carry the number of vectors a
// transform is applied to, which changes from call to call (a lockstep
// solve whose active right-hand sides converge one by one): they are timed
// on at most kTuneRows rows and kTuneBatch batch entries and classed by
// octave; N and K are classed by quarter octave.  Split-K products (the
// partial products of run_gemm) are timed whole and classed by chunk length.
constexpr int kTuneRows = 8192, kTuneBatch = 16;
bool gemm_variant_grouped(int variant) {
  return (variant > GEMM_64x64_G4 && variant <= 2 * GEMM_64x64_G4) || variant == GEMM_64x64_G4_SB_GROUPED ||
         variant == GEMM_128x64_G4_SB_GROUPED || variant == GEMM_128x128_G4_GROUPED ||
         variant == GEMM_128x128_DMA_GROUPED || variant == GEMM_64x256_DMA_GROUPED;
}
int octave_bucket(int x) {
  int p = 1;
  while (p < x) p *= 2;
  return p;
}
int shape_bucket(int x) {
  if (x <= 64) return x;
  int p = 1;
  while (p * 2 <= x) p *= 2;
  const int q = p / 4;
  return ((x + q - 1) / q) * q;
}

bool gemm_variant_narrow(int variant) { return variant == GEMM_128x32_G4_SB || variant == GEMM_64x32_G4; }

// the 32-column tiles are worth timing for outputs at most kNarrowMaxN wide,
// and for outputs up to 512 wide that 64-column tiles would pad by a further
// eighth or more (200 columns: 224 against 256)
static bool narrow_may_pay(int N) {
  if (N <= kNarrowMaxN) return true;
  const int p32 = (N + 31) / 32 * 32, p64 = (N + 63) / 64 * 64;
  return N <= 512 && 8 * (p64 - p32) >= p32;
}

// the variant of a product that is not timed: 32-column tiles for outputs at
// most 32 wide, 64-row tiles when the output has at most 64 rows (a 128-row
// tile would be mostly empty)
static int untimed_variant(const GemmArgs& g) {
  if (g.N <= 32) return g.M <= 64 ? GEMM_64x32_G4 : GEMM_128x32_G4_SB;
  return g.M <= 64 ? GEMM_64x64_G4 : gemm_default_variant(g);
}

void launch_gemm_choice(const GemmArgs& g, int choice, hipStream_t s) {
  if (choice >= kTransposedChoice) launch_zgemm_variant(transposed(g), choice - kTransposedChoice, s);
  else launch_zgemm_variant(g, choice, s);
}
static void launch_choice(const GemmArgs& g, int choice, hipStream_t s) { launch_gemm_choice(g, choice, s); }

int tuned_gemm(cclr_ctx* c, const GemmArgs& g) {
  if (g.M <= 0 || g.N <= 0 || g.batch <= 0 || g.K <= 0) return -1;
  const double flops = 8.0 * g.M * (double)g.N * (g.kchunk > 0 ? g.kchunk : g.K) * g.batch;
  if (flops < 1e10) {
    const int v = untimed_variant(g);
    launch_zgemm_variant(g, v, c->stream);
    return v;
  }
  // a split-K product keeps its whole batch (it carries the parallelism of the launch)
  const int tmr = std::min(g.M, kTuneRows),
            tbt = (g.nb2 > 1 || g.kchunk > 0) ? g.batch : std::min(g.batch, kTuneBatch);
  // split-K products (kchunk > 0: the batch index carries the K chunk) are classed by the chunk length
  // (the transposed product runs on 32-column tiles only when its row count
  // is one that they pad less, which the row octave alone does not tell)
  const bool trans_narrow = g.M != g.N && narrow_may_pay(g.M);
  const auto key = std::make_tuple(octave_bucket(tmr), shape_bucket(g.N), shape_bucket(g.kchunk > 0 ? g.kchunk : g.K),
                                   octave_bucket(tbt),
                                   (g.sAk == 1 ? 1 : 0) + (g.sBn == 1 ? 2 : 0) + (g.nb2 > 1 ? 4 : 0) +
                                       (g.kchunk > 0 ? 8 : 0) + (trans_narrow ? 16 : 0));
  auto it = c->gemm_choice.find(key);
  if (it != c->gemm_choice.end()) {
    launch_choice(g, it->second, c->stream);
    return it->second;
  }
  if (c->no_timing || !c->autotune) {  // no new timing runs (a call that may not allocate, or tuning off)
    const int v = untimed_variant(g);
    launch_zgemm_variant(g, v, c->stream);
    return v;
  }
  // nothing else may run while the variants are timed: drain the side stream too
  HIPCHK(hipStreamSynchronize(c->stream));
  if (c->side) HIPCHK(hipStreamSynchronize(c->side));
  // the timed product: the leading rows and batch entries, on a scratch output covering their index range
  GemmArgs h = g;
  h.M = tmr;
  h.batch = tbt;
  const i64 nb2 = h.nb2 > 1 ? h.nb2 : 1, nb1 = h.batch / nb2;
  const i64 extent = (i64)(h.M - 1) * h.sCm + (i64)(h.N - 1) * h.sCn + (nb1 - 1) * h.sCb + (nb2 - 1) * h.sCb2 + 1;
  Arena::Mark mk = c->arena.mark();
  h.C = (cplx*)c->arena.get(sizeof(cplx) * (size_t)extent);
  h.beta = 0;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  // candidates: every variant (the 32-column ones only where they may pay) and,
  // when the rows are a count that 32-column tiles pad less, those tiles on the
  // transposed product
  std::vector<int> cand;
  for (int v = GEMM_128x64_G3; v < GEMM_NVAR; ++v)  // the simple kernel (variant 0) never competes
    if (!gemm_variant_narrow(v) || narrow_may_pay(g.N)) cand.push_back(v);
  if (trans_narrow)
    for (int v = GEMM_128x64_G3; v < GEMM_NVAR; ++v)
      if (gemm_variant_narrow(v)) cand.push_back(kTransposedChoice + v);
  std::vector<double> ms(cand.size(), 0.0);
  launch_zgemm_variant(h, gemm_default_variant(g), c->stream);  // warm caches and clocks
  int best = gemm_default_variant(g);
  double tbest = 1e300;
  for (size_t q = 0; q < cand.size(); ++q) {
    HIPCHK(hipEventRecord(e0, c->stream));
    launch_choice(h, cand[q], c->stream);
    HIPCHK(hipEventRecord(e1, c->stream));
    HIPCHK(hipEventSynchronize(e1));
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, e0, e1));
    ms[q] = t;
    if (t < tbest) {
      tbest = t;
      best = cand[q];
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  // within the timing noise (2%) of the fastest, prefer the variant that
  // re-reads its operands from HBM least for the same time: the XCD-grouped
  // tile order first, then tiles of 128 rows and of 128 or more columns, then the
  // faster one
  {
    auto rereads = [](int choice) {
      const int v = choice % kTransposedChoice;
      const int base = gemm_variant_grouped(v) && v <= 2 * GEMM_64x64_G4 ? v - GEMM_64x64_G4 : v;
      const bool rows128 = base == GEMM_128x64_G3 || base == GEMM_128x64_G4 || v == GEMM_128x64_G4_SB ||
                           v == GEMM_128x64_G4_SB_GROUPED || (v >= GEMM_128x128_G4 && v < GEMM_64x256_DMA) ||
                           v == GEMM_128x32_G4_SB;
      const bool cols128 = v >= GEMM_128x128_G4 && !gemm_variant_narrow(v);
      return (gemm_variant_grouped(v) ? 0 : 3) + (rows128 ? 0 : 1) + (cols128 ? 0 : 1);
    };
    size_t pick = 0;
    for (size_t q = 0; q < cand.size(); ++q)
      if (cand[q] == best) pick = q;
    for (size_t q = 0; q < cand.size(); ++q) {
      if (ms[q] > 1.02 * tbest) continue;
      if (rereads(cand[q]) < rereads(cand[pick]) || (rereads(cand[q]) == rereads(cand[pick]) && ms[q] < ms[pick]))
        pick = q;
    }
    best = cand[pick];
  }
  c->arena.reset(mk);
  c->gemm_choice[key] = best;
  std::vector<std::pair<int, double>> rec;
  for (size_t q = 0; q < cand.size(); ++q) rec.push_back({cand[q], ms[q]});
  // the product's shape, then the part that was timed (at most kTuneRows rows and kTuneBatch batch entries)
  c->gemm_tuning_log.push_back({std::to_string(g.M) + "x" + std::to_string(g.N) + "x" + std::to_string(g.K) + " b" +
                                    std::to_string(g.batch) + " layout" + std::to_string(std::get<4>(key)) +
                                    " timed " + std::to_string(tmr) + "x" + std::to_string(g.N) + "x" +
                                    std::to_string(g.K) + " b" + std::to_string(tbt),
                                rec, best});
  launch_choice(g, best, c->stream);
  return best;
}

// -------------------------------------------------------- integral views
Ten fblk(cclr_ctx* c, const char* kinds) {
  const int o = c->o, n = c->o + c->v;
  Ten t = ten(c->f.c(), {(i64)n, (i64)n});
  i64 off = (kinds[0] == 'o' ? 0 : o) * (i64)n + (kinds[1] == 'o' ? 0 : o);
  t.p += off;
  t.dim[0] = kinds[0] == 'o' ? o : c->v;
  t.dim[1] = kinds[1] == 'o' ? o : c->v;
  return t;
}

Ten Vblk(cclr_ctx* c, const char* kinds) {
  const i64 o = c->o, v = c->v;
  auto sz = [&](char k) { return k == 'o' ? o : v; };
  std::string bra(kinds, 2), ket(kinds + 2, 2);
  double sign = 1.0;
  // labels track axis identity: requested axes are "pqrs"
  std::string lab = "pqrs";
  if (bra == "vo") { bra = "ov"; sign = -sign; std::swap(lab[0], lab[1]); }
  if (ket == "vo") { ket = "ov"; sign = -sign; std::swap(lab[2], lab[3]); }
  auto rank = [](const std::string& s) { return s == "oo" ? 0 : (s == "ov" ? 1 : 2); };
  Ten base;
  std::string baselab;
  bool cj = false;
  auto blk = [&](const std::string& k) -> DevBuf& {
    if (k == "oooo") return c->Voooo;
    if (k == "ooov") return c->Vooov;
    if (k == "oovv") return c->Voovv;
    if (k == "ovov") return c->Vovov;
    if (k == "ovvv") return c->Vovvv;
    if (k == "vvvv") return c->Vvvvv;
    throw CclrError(CCLR_EINVAL, "Vblk: no block " + k);
  };
  if (rank(bra) <= rank(ket)) {
    std::string k = bra + ket;
    base = ten(blk(k), {sz(k[0]), sz(k[1]), sz(k[2]), sz(k[3])});
    baselab = lab;  // base axes carry labels lab[0..3]
  } else {
    std::string k = ket + bra;
    base = ten(blk(k), {sz(k[0]), sz(k[1]), sz(k[2]), sz(k[3])});
    // V[pqrs] = conj(Vbase[rspq]): base axes are (r, s, p, q) of the request
    baselab = std::string() + lab[2] + lab[3] + lab[0] + lab[1];
    cj = true;
  }
  Ten r = reorder(base, baselab.c_str(), "pqrs");
  r.conj = cj;
  r.sr = sign;
  r.si = 0.0;
  return r;
}
