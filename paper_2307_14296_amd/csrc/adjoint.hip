// Gradient of the response function with respect to the Fock matrix and the
// antisymmetrized integrals (the Hamiltonian part of cclr_response_backward).
//
// For fixed amplitudes t every Hbar element is linear in (f, <pq||rs>), and
// so are the Jacobian A, the Hessian product t^X F and eta^0 = (F^m_e, V^ij_ab).
// With the left solutions y of the adjoint systems (they carry the
// cotangents of the right solutions t^X) and the Lambda cotangent solved
// from A x = -lambda-bar, the derivative of the response function along a
// change dH is a sum of bilinear pairings, each linear in dH:
//   sum_k y_k (dA) t_k  +  lambda (dA) x  +  eta^0(dH) . x  +  sum_k (t^X F)(dH)[a_k] . b_k.
// The pairings are evaluated backwards through the same products that define
// sigma, t^X F and the intermediates (SI, "EOM-EE sigma-vectors and
// intermediates" and "Linear response"): every product term is listed once
// below as an einsum-style term, and its transposed contraction with the
// output cotangent is formed for each operand that depends on H.  The
// Lambda cotangent comes from the same terms of t^X F and of eta^X, which are
// linear in lambda.
//
// Conventions: the cotangents are holomorphic derivatives of
// h = sum c1 g(z) + c2 g(-z*) (see cclr_response_backward); an integral block
// read through a conjugated view contributes its conjugate.  The gradient of
// the real loss is conj(dh/dH), finally projected onto perturbations that
// keep the symmetries of the inputs (f Hermitian; <pq||rs> antisymmetric in
// each pair and equal to conj <rs||pq>).
#include <cstring>
#include <functional>

#include "internal.h"

namespace {
struct Op {
  const char* name;
  const char* lab;
};
struct Term {
  double coef;
  const char* out;
  const char* lo;
  Op ops[4];
};

// Hbar intermediates (SI, eqs. F_im ... W_efam) with the readings of the
// sigma equations: F^a_e with bra a, ket e; minus signs on F^i_f t^ef_mn in
// W_iemn and on P(ef) V^en_ag t^gf_mn in W_efam.  Permutation operators are
// written out as separate terms with exchanged output labels.
const Term H_TERMS[] = {
    {1.0, "Foo", "im", {{"f:oo", "im"}}},
    {1.0, "Foo", "im", {{"f:ov", "ie"}, {"t1", "me"}}},
    {1.0, "Foo", "im", {{"V:ooov", "inme"}, {"t1", "ne"}}},
    {0.5, "Foo", "im", {{"V:oovv", "inef"}, {"tau", "mnef"}}},
    {1.0, "Fvv", "ae", {{"f:vv", "ae"}}},
    {-1.0, "Fvv", "ae", {{"f:ov", "me"}, {"t1", "ma"}}},
    {1.0, "Fvv", "ae", {{"V:vovv", "amef"}, {"t1", "mf"}}},
    {-0.5, "Fvv", "ae", {{"V:oovv", "mnef"}, {"tau", "mnaf"}}},
    {1.0, "Fov", "me", {{"f:ov", "me"}}},
    {1.0, "Fov", "me", {{"V:oovv", "mnef"}, {"t1", "nf"}}},
    {1.0, "Woooo", "ijmn", {{"V:oooo", "ijmn"}}},
    {1.0, "Woooo", "ijmn", {{"V:oovo", "ijen"}, {"t1", "me"}}},
    {-1.0, "Woooo", "ijnm", {{"V:oovo", "ijen"}, {"t1", "me"}}},
    {0.5, "Woooo", "ijmn", {{"V:oovv", "ijef"}, {"tau", "mnef"}}},
    {1.0, "Wovvo", "mbej", {{"V:ovvo", "mbej"}}},
    {1.0, "Wovvo", "mbej", {{"V:ovvv", "mbef"}, {"t1", "jf"}}},
    {-1.0, "Wovvo", "mbej", {{"V:oovo", "mnej"}, {"t1", "nb"}}},
    {-1.0, "Wovvo", "mbej", {{"V:oovv", "mnef"}, {"tt2", "jnfb"}}},
    {1.0, "Wbar", "mbej", {{"V:ovvo", "mbej"}}},
    {-1.0, "Wbar", "mbej", {{"V:oovv", "mnef"}, {"t2", "njbf"}}},
    {1.0, "Wooov", "mnie", {{"V:ooov", "mnie"}}},
    {1.0, "Wooov", "mnie", {{"V:oovv", "mnfe"}, {"t1", "if"}}},
    {1.0, "Wvovv", "amef", {{"V:vovv", "amef"}}},
    {-1.0, "Wvovv", "amef", {{"V:oovv", "nmef"}, {"t1", "na"}}},
    {1.0, "Wvvvv", "efab", {{"V:vvvv", "efab"}}},
    {-1.0, "Wvvvv", "efab", {{"V:ovvv", "mfab"}, {"t1", "me"}}},
    {1.0, "Wvvvv", "feab", {{"V:ovvv", "mfab"}, {"t1", "me"}}},
    {0.5, "Wvvvv", "efab", {{"V:oovv", "mnab"}, {"tau", "mnef"}}},
    {1.0, "Wovoo", "iemn", {{"V:ovoo", "iemn"}}},
    {-1.0, "Wovoo", "iemn", {{"Fov", "if"}, {"t2", "mnef"}}},
    {-1.0, "Wovoo", "iemn", {{"Woooo", "iomn"}, {"t1", "oe"}}},
    {0.5, "Wovoo", "iemn", {{"V:ovvv", "iefg"}, {"tau", "mnfg"}}},
    {1.0, "Wovoo", "iemn", {{"Wbar", "iefn"}, {"t1", "mf"}}},
    {-1.0, "Wovoo", "ienm", {{"Wbar", "iefn"}, {"t1", "mf"}}},
    {1.0, "Wovoo", "iemn", {{"V:ooov", "iomf"}, {"t2", "noef"}}},
    {-1.0, "Wovoo", "ienm", {{"V:ooov", "iomf"}, {"t2", "noef"}}},
    {1.0, "Wvvvo", "efam", {{"V:vvvo", "efam"}}},
    {-1.0, "Wvvvo", "efam", {{"V:vovv", "enag"}, {"t2", "mngf"}}},
    {1.0, "Wvvvo", "feam", {{"V:vovv", "enag"}, {"t2", "mngf"}}},
    {1.0, "Wvvvo", "efam", {{"Wvvvv", "efag"}, {"t1", "mg"}}},
    {1.0, "Wvvvo", "efam", {{"Fov", "na"}, {"t2", "mnef"}}},
    {0.5, "Wvvvo", "efam", {{"V:oovo", "noam"}, {"tau", "noef"}}},
    {-1.0, "Wvvvo", "efam", {{"Wbar", "nfam"}, {"t1", "ne"}}},
    {1.0, "Wvvvo", "feam", {{"Wbar", "nfam"}, {"t1", "ne"}}},
};

// Right sigma (SI, eqs. sigma_sin-ee and sigma_double-ee; the right-singles
// ring element read as W^ma_ei), batched over Z.  Doubles go to groups
// S0 / Sa / Si / Sai that carry no permutation, P(ab), P(ij), P(ab)P(ij).
const Term SIGMA_TERMS[] = {
    {1.0, "S1", "Zia", {{"Fvv", "ae"}, {"x1", "Zie"}}},
    {-1.0, "S1", "Zia", {{"Foo", "mi"}, {"x1", "Zma"}}},
    {1.0, "S1", "Zia", {{"Fov", "me"}, {"x2", "Zmiea"}}},
    {1.0, "S1", "Zia", {{"Wovvo", "maei"}, {"x1", "Zme"}}},
    {0.5, "S1", "Zia", {{"Wvovv", "amef"}, {"x2", "Zimef"}}},
    {0.5, "S1", "Zia", {{"Wooov", "mnie"}, {"x2", "Zmnea"}}},
    {-1.0, "Sa", "Zijab", {{"Wovoo", "mbij"}, {"x1", "Zma"}}},
    {1.0, "Si", "Zijab", {{"Wvvvo", "abej"}, {"x1", "Zie"}}},
    {1.0, "Sa", "Zijab", {{"Wvovv", "bmfe"}, {"x1", "Zme"}, {"t2", "ijaf"}}},
    {-1.0, "Si", "Zijab", {{"Wooov", "nmje"}, {"x1", "Zme"}, {"t2", "inab"}}},
    {1.0, "Sa", "Zijab", {{"Fvv", "be"}, {"x2", "Zijae"}}},
    {-1.0, "Si", "Zijab", {{"Foo", "mj"}, {"x2", "Zimab"}}},
    {0.5, "S0", "Zijab", {{"Woooo", "mnij"}, {"x2", "Zmnab"}}},
    {1.0, "Sai", "Zijab", {{"Wovvo", "mbej"}, {"x2", "Zimae"}}},
    {-0.5, "Sa", "Zijab", {{"V:oovv", "nmfe"}, {"x2", "Zmnea"}, {"t2", "ijfb"}}},
    {-0.5, "Si", "Zijab", {{"V:oovv", "nmfe"}, {"x2", "Zimfe"}, {"t2", "jnba"}}},
    {0.5, "S0", "Zijab", {{"Wvvvv", "abef"}, {"x2", "Zijef"}}},
};

// Hessian product t^X F (SI, "(t^X F)^k_c" and "(t^X F)^kl_cd"), batched
// over Z; doubles groups as for sigma with P(ij) on (k,l), P(ab) on (c,d).
const Term TF_TERMS[] = {
    {1.0, "T1", "Zkc", {{"V:oovv", "kica"}, {"x1", "Zia"}}},
    {-1.0, "T1", "Zkc", {{"l1", "ic"}, {"Fov", "ka"}, {"x1", "Zia"}}},
    {-1.0, "T1", "Zkc", {{"l1", "ka"}, {"Fov", "ic"}, {"x1", "Zia"}}},
    {1.0, "T1", "Zkc", {{"l1", "ke"}, {"Wvovv", "eica"}, {"x1", "Zia"}}},
    {-1.0, "T1", "Zkc", {{"l1", "mc"}, {"Wooov", "kima"}, {"x1", "Zia"}}},
    {-1.0, "T1", "Zkc", {{"l1", "ma"}, {"Wooov", "ikmc"}, {"x1", "Zia"}}},
    {1.0, "T1", "Zkc", {{"l1", "ie"}, {"Wvovv", "ekac"}, {"x1", "Zia"}}},
    {-0.5, "T1", "Zkc", {{"l1", "ic"}, {"V:oovv", "kjab"}, {"x2", "Zijab"}}},
    {-0.5, "T1", "Zkc", {{"l1", "ka"}, {"V:oovv", "ijcb"}, {"x2", "Zijab"}}},
    {1.0, "T1", "Zkc", {{"l1", "ia"}, {"V:oovv", "jkbc"}, {"x2", "Zijab"}}},
    {1.0, "T1", "Zkc", {{"l2", "mkae"}, {"Wovvo", "iecm"}, {"x1", "Zia"}}},
    {1.0, "T1", "Zkc", {{"l2", "imec"}, {"Wovvo", "keam"}, {"x1", "Zia"}}},
    {0.5, "T1", "Zkc", {{"l2", "kief"}, {"Wvvvv", "efca"}, {"x1", "Zia"}}},
    {0.5, "T1", "Zkc", {{"l2", "mnca"}, {"Woooo", "kimn"}, {"x1", "Zia"}}},
    {-0.5, "T1", "Zkc", {{"l2", "mnec"}, {"t2", "mnef"}, {"V:oovv", "kifa"}, {"x1", "Zia"}}},
    {-0.5, "T1", "Zkc", {{"l2", "mkef"}, {"t2", "mnef"}, {"V:oovv", "nica"}, {"x1", "Zia"}}},
    {-0.5, "T1", "Zkc", {{"l2", "mnea"}, {"t2", "mnef"}, {"V:oovv", "ikfc"}, {"x1", "Zia"}}},
    {-0.5, "T1", "Zkc", {{"l2", "mief"}, {"t2", "mnef"}, {"V:oovv", "nkac"}, {"x1", "Zia"}}},
    {-0.5, "T1", "Zkc", {{"l2", "ijac"}, {"Fov", "kb"}, {"x2", "Zijab"}}},
    {-0.5, "T1", "Zkc", {{"l2", "ikab"}, {"Fov", "jc"}, {"x2", "Zijab"}}},
    {-1.0, "T1", "Zkc", {{"l2", "ikeb"}, {"Wvovv", "ejac"}, {"x2", "Zijab"}}},
    {1.0, "T1", "Zkc", {{"l2", "mjac"}, {"Wooov", "ikmb"}, {"x2", "Zijab"}}},
    {-0.25, "T1", "Zkc", {{"l2", "ijec"}, {"Wvovv", "ekab"}, {"x2", "Zijab"}}},
    {0.25, "T1", "Zkc", {{"l2", "mkab"}, {"Wooov", "ijmc"}, {"x2", "Zijab"}}},
    {0.5, "T1", "Zkc", {{"l2", "ijae"}, {"Wvovv", "ekbc"}, {"x2", "Zijab"}}},
    {-0.5, "T1", "Zkc", {{"l2", "imab"}, {"Wooov", "jkmc"}, {"x2", "Zijab"}}},
    {1.0, "Tai", "Zklcd", {{"l1", "kc"}, {"V:oovv", "lida"}, {"x1", "Zia"}}},
    {-1.0, "Ti", "Zklcd", {{"l1", "ka"}, {"V:oovv", "ilcd"}, {"x1", "Zia"}}},
    {-1.0, "Ta", "Zklcd", {{"l1", "ic"}, {"V:oovv", "klad"}, {"x1", "Zia"}}},
    {-1.0, "Ti", "Zklcd", {{"l2", "kicd"}, {"Fov", "la"}, {"x1", "Zia"}}},
    {-1.0, "Ta", "Zklcd", {{"l2", "klca"}, {"Fov", "id"}, {"x1", "Zia"}}},
    {1.0, "Ta", "Zklcd", {{"l2", "klce"}, {"Wvovv", "eida"}, {"x1", "Zia"}}},
    {-1.0, "Ti", "Zklcd", {{"l2", "kmcd"}, {"Wooov", "lima"}, {"x1", "Zia"}}},
    {1.0, "Tai", "Zklcd", {{"l2", "mlca"}, {"Wooov", "kimd"}, {"x1", "Zia"}}},
    {1.0, "T0", "Zklcd", {{"l2", "micd"}, {"Wooov", "klma"}, {"x1", "Zia"}}},
    {-1.0, "Tai", "Zklcd", {{"l2", "kied"}, {"Wvovv", "elca"}, {"x1", "Zia"}}},
    {-1.0, "T0", "Zklcd", {{"l2", "klea"}, {"Wvovv", "eicd"}, {"x1", "Zia"}}},
    {-0.5, "Ta", "Zklcd", {{"l2", "klca"}, {"V:oovv", "ijdb"}, {"x2", "Zijab"}}},
    {-0.5, "Ti", "Zklcd", {{"l2", "kicd"}, {"V:oovv", "ljab"}, {"x2", "Zijab"}}},
    {0.25, "T0", "Zklcd", {{"l2", "ijcd"}, {"V:oovv", "klab"}, {"x2", "Zijab"}}},
    {0.25, "T0", "Zklcd", {{"l2", "klab"}, {"V:oovv", "ijcd"}, {"x2", "Zijab"}}},
    {1.0, "Tai", "Zklcd", {{"l2", "kjcb"}, {"V:oovv", "lida"}, {"x2", "Zijab"}}},
    {-0.5, "Ti", "Zklcd", {{"l2", "ikab"}, {"V:oovv", "jlcd"}, {"x2", "Zijab"}}},
    {-0.5, "Ta", "Zklcd", {{"l2", "ijac"}, {"V:oovv", "klbd"}, {"x2", "Zijab"}}},
};

// The lambda-dependent terms of eta^X (SI, eq. eta-equation, programmable
// form), batched over the perturbations Z.
const Term ETA_TERMS[] = {
    {1.0, "E1", "Zia", {{"X:vv", "Zea"}, {"l1", "ie"}}},
    {-1.0, "E1", "Zia", {{"X:oo", "Zim"}, {"l1", "ma"}}},
    {-1.0, "E1", "Zia", {{"X:ov", "Zma"}, {"t1", "me"}, {"l1", "ie"}}},
    {-1.0, "E1", "Zia", {{"X:ov", "Zie"}, {"t1", "me"}, {"l1", "ma"}}},
    {-0.5, "E1", "Zia", {{"t2", "mnfe"}, {"l2", "mife"}, {"X:ov", "Zna"}}},
    {-0.5, "E1", "Zia", {{"t2", "nmfe"}, {"l2", "nmfa"}, {"X:ov", "Zie"}}},
    {1.0, "Eai", "Zijab", {{"l1", "ia"}, {"X:ov", "Zjb"}}},
    {1.0, "Ea", "Zijab", {{"l2", "ijae"}, {"X:vv", "Zeb"}}},
    {-1.0, "Ei", "Zijab", {{"l2", "imab"}, {"X:oo", "Zjm"}}},
    {-1.0, "Ea", "Zijab", {{"t1", "me"}, {"l2", "ijae"}, {"X:ov", "Zmb"}}},
    {-1.0, "Ei", "Zijab", {{"t1", "me"}, {"l2", "imab"}, {"X:ov", "Zje"}}},
};

int nops(const Term& t) {
  int n = 0;
  while (n < 4 && t.ops[n].name) ++n;
  return n;
}

bool is_hbar(const std::string& n) {
  static const char* names[] = {"Foo", "Fvv", "Fov", "Woooo", "Wovvo", "Wbar", "Wooov", "Wvovv", "Wvvvv", "Wovoo",
                                "Wvvvo"};
  for (const char* s : names)
    if (n == s) return true;
  return false;
}
bool is_h(const std::string& n) { return n.rfind("V:", 0) == 0 || n.rfind("f:", 0) == 0 || is_hbar(n); }
bool is_lam(const std::string& n) { return n == "l1" || n == "l2"; }

struct Opnd {
  Ten t;
  std::string lab;
};

i64 labsz(const std::vector<Opnd>& ops, char ch) {
  for (const Opnd& o : ops) {
    const size_t p = o.lab.find(ch);
    if (p != std::string::npos) return o.t.dim[p];
  }
  return 1;
}

// C[lc] += alpha * prod of the operands (einsum), contracted pairwise,
// smallest intermediate first.
void einsum_acc(cclr_ctx* c, cplx alpha, std::vector<Opnd> ops, const Ten& C, const std::string& lc) {
  Arena::Mark mk = c->arena.mark();
  while (ops.size() > 2) {
    size_t bi = 0, bj = 1;
    double best = -1;
    std::string bkeep;
    for (size_t i = 0; i < ops.size(); ++i)
      for (size_t j = i + 1; j < ops.size(); ++j) {
        std::string keep;
        const std::string u = ops[i].lab + ops[j].lab;
        for (char ch : u) {
          if (keep.find(ch) != std::string::npos) continue;
          bool needed = lc.find(ch) != std::string::npos;
          for (size_t k = 0; k < ops.size() && !needed; ++k)
            if (k != i && k != j && ops[k].lab.find(ch) != std::string::npos) needed = true;
          if (needed) keep += ch;
        }
        double sz = 1;
        for (char ch : keep) sz *= (double)labsz(ops, ch);
        if (best < 0 || sz < best) best = sz, bi = i, bj = j, bkeep = keep;
      }
    Ten T;
    i64 n = 1;
    for (char ch : bkeep) n *= labsz(ops, ch);
    T.p = (cplx*)c->arena.get(sizeof(cplx) * (size_t)std::max<i64>(n, 1));
    T.nd = (int)bkeep.size();
    i64 s = 1;
    for (int d = T.nd - 1; d >= 0; --d) {
      T.dim[d] = labsz(ops, bkeep[d]);
      T.st[d] = s;
      s *= T.dim[d];
    }
    contract(c, cx(1.0), ops[bi].t, ops[bi].lab.c_str(), ops[bj].t, ops[bj].lab.c_str(), T, bkeep.c_str(), false);
    ops.erase(ops.begin() + bj);
    ops[bi] = Opnd{T, bkeep};
  }
  if (ops.size() == 2)
    contract(c, alpha, ops[0].t, ops[0].lab.c_str(), ops[1].t, ops[1].lab.c_str(), C, lc.c_str(), true);
  else
    tcopy(c, C, lc.c_str(), ops[0].t, ops[0].lab.c_str(), alpha, true);
  c->arena.reset(mk);
}

struct Env {
  cclr_ctx* c = nullptr;
  std::map<std::string, Ten> val;  // values of the operands that are not integral views
  std::map<std::string, Ten> cot;  // cotangents
  cplx* gf = nullptr;              // holomorphic cotangent of f (n x n)
  std::map<std::string, cplx*> gv; // ... and of each canonical integral block
  // W^ef_ab exists only packed.  Its cotangent is accumulated directly in the
  // vvvv block of the integral gradient (W^ef_ab = V^ef_ab + ..., so that
  // block receives exactly this cotangent), and the one product that needs
  // its value (the lambda cotangent of the t^X F ladder term) runs on the
  // packed operator.
  bool w4_in_gv = false;
};

Ten value(Env& e, const std::string& n) {
  if (n.rfind("V:", 0) == 0) return Vblk(e.c, n.c_str() + 2);
  if (n.rfind("f:", 0) == 0) return fblk(e.c, n.c_str() + 2);
  auto it = e.val.find(n);
  REQUIRE(it != e.val.end(), CCLR_EINVAL, "adjoint: no value for " + n);
  return it->second;
}

const char* canonical_block(const cclr_ctx* c, const cplx* p) {
  if (p >= c->Voooo.c() && p < c->Voooo.c() + c->Voooo.bytes / sizeof(cplx)) return "oooo";
  if (p >= c->Vooov.c() && p < c->Vooov.c() + c->Vooov.bytes / sizeof(cplx)) return "ooov";
  if (p >= c->Voovv.c() && p < c->Voovv.c() + c->Voovv.bytes / sizeof(cplx)) return "oovv";
  if (p >= c->Vovov.c() && p < c->Vovov.c() + c->Vovov.bytes / sizeof(cplx)) return "ovov";
  if (p >= c->Vovvv.c() && p < c->Vovvv.c() + c->Vovvv.bytes / sizeof(cplx)) return "ovvv";
  if (p >= c->Vvvvv.c() && p < c->Vvvvv.c() + c->Vvvvv.bytes / sizeof(cplx)) return "vvvv";
  throw CclrError(CCLR_EINVAL, "adjoint: view outside the integral blocks");
}

const DevBuf& block_buf(const cclr_ctx* c, const std::string& k) {
  if (k == "oooo") return c->Voooo;
  if (k == "ooov") return c->Vooov;
  if (k == "oovv") return c->Voovv;
  if (k == "ovov") return c->Vovov;
  if (k == "ovvv") return c->Vovvv;
  return c->Vvvvv;
}

// Accumulate alpha * prod(ops) into the cotangent of operand `name`
// (labels `la`).  An integral view v = s * op(block) sends s * (.) to the
// block's cotangent, conjugated when op is a conjugation.
void add_cot(Env& e, const std::string& name, const std::string& la, cplx alpha, std::vector<Opnd> ops) {
  cclr_ctx* c = e.c;
  Ten tgt;
  bool cj = false;
  if (name.rfind("V:", 0) == 0 || name.rfind("f:", 0) == 0) {
    const Ten v = value(e, name);
    if (name[0] == 'V') {
      const std::string blk = canonical_block(c, v.p);
      tgt = v;
      tgt.p = e.gv.at(blk) + (v.p - block_buf(c, blk).c());
    } else {
      tgt = v;
      tgt.p = e.gf + (v.p - c->f.c());
    }
    cj = v.conj;
    REQUIRE(v.si == 0.0, CCLR_EINVAL, "adjoint: complex-scaled integral view");
    alpha = cx(alpha.x * v.sr, alpha.y * v.sr);
    tgt.conj = false;
    tgt.sr = 1.0;
    tgt.si = 0.0;
  } else {
    auto it = e.cot.find(name);
    if (it == e.cot.end() && name == "Wvvvv") {
      const i64 v = c->v;
      REQUIRE(e.gv.count("vvvv"), CCLR_EINVAL, "adjoint: W^ef_ab cotangent needs the integral gradient");
      it = e.cot.emplace(name, ten(e.gv.at("vvvv"), {v, v, v, v})).first;
      e.w4_in_gv = true;
    }
    if (it == e.cot.end()) {
      const Ten v = value(e, name);
      i64 n = v.size();
      std::vector<i64> dims(v.dim, v.dim + v.nd);
      Ten z;
      z.p = (cplx*)c->arena.get(sizeof(cplx) * (size_t)std::max<i64>(n, 1));
      z.nd = v.nd;
      i64 s = 1;
      for (int d = v.nd - 1; d >= 0; --d) {
        z.dim[d] = v.dim[d];
        z.st[d] = s;
        s *= v.dim[d];
      }
      launch_fill(z.p, n, cx(0.0), c->stream);
      it = e.cot.emplace(name, z).first;
    }
    tgt = it->second;
  }
  if (cj) {
    alpha = cx(alpha.x, -alpha.y);
    for (Opnd& o : ops) o.t = conjugated(o.t);
  }
  einsum_acc(c, alpha, ops, tgt, la);
}

// cot(l2)_kief += coef sum_(Z,c,a) cot(out)_Zkc W^ef_ca x1_Zia on the packed
// operator: U_kica = sum_Z cot_Zkc x1_Zia, antisymmetrized and packed in
// (c,a), times Wp[EF][CA], unpacked with antisymmetry in (e,f).
void ladder_lambda_cot(Env& e, const Term& t, const Ten& cot_out);

// Backward pass through a term table: for every term whose output has a
// cotangent, the cotangent of each operand selected by `want`.
void reverse(Env& e, const Term* terms, int nt, const std::function<bool(const std::string&)>& want) {
  for (int ti = nt - 1; ti >= 0; --ti) {
    const Term& t = terms[ti];
    auto co = e.cot.find(t.out);
    if (co == e.cot.end()) continue;
    const int no = nops(t);
    for (int j = 0; j < no; ++j) {
      if (!want(t.ops[j].name)) continue;
      // W^ef_ab = V^ef_ab + ...: the vvvv gradient block already holds the cotangent
      if (e.w4_in_gv && std::string(t.out) == "Wvvvv" && std::string(t.ops[j].name) == "V:vvvv") continue;
      bool w4_value = false;
      for (int k = 0; k < no; ++k)
        if (k != j && std::string(t.ops[k].name) == "Wvvvv") w4_value = true;
      if (w4_value) {
        REQUIRE(std::string(t.ops[j].name) == "l2", CCLR_EINVAL, "adjoint: unsupported use of W^ef_ab");
        ladder_lambda_cot(e, t, co->second);
        continue;
      }
      std::vector<Opnd> ops;
      ops.push_back(Opnd{co->second, t.lo});
      for (int k = 0; k < no; ++k)
        if (k != j) ops.push_back(Opnd{value(e, t.ops[k].name), t.ops[k].lab});
      add_cot(e, t.ops[j].name, t.ops[j].lab, cx(t.coef), ops);
    }
  }
}

void ladder_lambda_cot(Env& e, const Term& t, const Ten& cot_out) {
  cclr_ctx* c = e.c;
  const i64 o = c->o, v = c->v, V2 = c->V2();
  REQUIRE(nops(t) == 3 && std::string(t.lo) == "Zkc" && std::string(t.ops[0].lab) == "kief" &&
              std::string(t.ops[1].lab) == "efca" && std::string(t.ops[2].name) == "x1" &&
              std::string(t.ops[2].lab) == "Zia",
          CCLR_EINVAL, "adjoint: unexpected form of the ladder term");
  auto it = e.cot.find("l2");
  if (it == e.cot.end()) {
    Ten z = tmp(c, {o, o, v, v});
    launch_fill(z.p, z.size(), cx(0.0), c->stream);
    it = e.cot.emplace("l2", z).first;
  }
  Arena::Mark mk = c->arena.mark();
  Ten U = tmp(c, {o, o, v, v});
  contract(c, cx(1.0), cot_out, "Zkc", value(e, "x1"), "Zia", U, "kica", false);
  Ten Ua = tmp(c, {o, o, v, v});
  tcopy(c, Ua, "kica", U, "kica", cx(1.0), false);
  tcopy(c, Ua, "kica", U, "kiac", cx(-1.0), true);
  cplx* Up = (cplx*)c->arena.get(sizeof(cplx) * (size_t)(o * o * V2));
  launch_pack_pairs(o * o, (int)v, Ua.p, Up, c->stream);
  cplx* R = (cplx*)c->arena.get(sizeof(cplx) * (size_t)(o * o * V2));
  GemmArgs g{};
  g.M = (int)(o * o); g.N = (int)V2; g.K = (int)V2; g.batch = 1;
  g.A = Up; g.sAm = V2; g.sAk = 1;
  g.B = c->Wp.c(); g.sBk = 1; g.sBn = V2;
  g.C = R; g.sCm = V2; g.sCn = 1;
  g.ar = 1.0; g.ai = 0.0; g.beta = 0;
  with_plain_wp(c, [&]() { run_gemm(c, g); });
  launch_unpack_pairs_acc(o * o, (int)v, R, it->second.p, t.coef, c->stream);
  c->arena.reset(mk);
}

// group cotangents of a doubles output paired with the antisymmetric y2
void set_groups(Env& e, const char* g1, const char* g0, const char* ga, const char* gi, const char* gai,
                const Ten& y1, const Ten& y2) {
  e.cot[g1] = y1;
  e.cot[g0] = scaled(y2, 0.25);
  e.cot[ga] = scaled(y2, 0.5);
  e.cot[gi] = scaled(y2, 0.5);
  e.cot[gai] = y2;
}

// in-place projection of a 4-index block gradient onto the symmetric
// perturbations: average over the group generated by the enabled symmetries
// (1: antisymmetry in axes 0,1; 2: in axes 2,3; 4: exchange of the pairs
// with complex conjugation)
__global__ __launch_bounds__(256) void k_symmetrize4(cplx* g, int d0, int d1, int d2, int d3, int flags) {
  const i64 total = (i64)d0 * d1 * d2 * d3;
  for (i64 e = blockIdx.x * (i64)blockDim.x + threadIdx.x; e < total; e += (i64)gridDim.x * blockDim.x) {
    const int i3 = (int)(e % d3), i2 = (int)(e / d3 % d2), i1 = (int)(e / ((i64)d3 * d2) % d1),
              i0 = (int)(e / ((i64)d3 * d2 * d1));
    i64 idx[8];
    double sg[8];
    bool cj[8];
    int ng = 0;
    i64 mn = e;
    for (int m = 0; m < 8; ++m) {
      if (m & ~flags) continue;
      int a = i0, b = i1, cc = i2, d = i3;
      double s = 1.0;
      bool conj = false;
      if (m & 1) { const int t = a; a = b; b = t; s = -s; }
      if (m & 2) { const int t = cc; cc = d; d = t; s = -s; }
      if (m & 4) { int t = a; a = cc; cc = t; t = b; b = d; d = t; conj = true; }
      idx[ng] = (((i64)a * d1 + b) * d2 + cc) * d3 + d;
      sg[ng] = s;
      cj[ng] = conj;
      if (idx[ng] < mn) mn = idx[ng];
      ++ng;
    }
    if (mn != e) continue;  // one thread per orbit: its smallest element
    double ar = 0, ai = 0;
    for (int k = 0; k < ng; ++k) {
      const cplx x = g[idx[k]];
      ar += sg[k] * x.x;
      ai += sg[k] * (cj[k] ? -x.y : x.y);
    }
    ar /= ng, ai /= ng;
    for (int k = 0; k < ng; ++k) g[idx[k]] = make_double2(sg[k] * ar, sg[k] * (cj[k] ? -ai : ai));
  }
}

unsigned grid_of(i64 n) {
  i64 g = (n + 255) / 256;
  if (g > 65536) g = 65536;
  return (unsigned)std::max<i64>(g, 1);
}

void symmetrize4(cclr_ctx* c, cplx* g, int d0, int d1, int d2, int d3, int flags) {
  hipLaunchKernelGGL(k_symmetrize4, dim3(grid_of((i64)d0 * d1 * d2 * d3)), dim3(256), 0, c->stream, g, d0, d1, d2,
                     d3, flags);
  HIPCHK(hipGetLastError());
}

Ten dense(cclr_ctx* c, std::initializer_list<i64> dims) { return tmp(c, dims); }
}  // namespace

// Inputs of the Hamiltonian adjoint, prepared by cclr_response_backward.
//   Xs        nx perturbations stacked [nx][n][n] (device)
//   sol, xl   the nr right solutions and their left (adjoint) solutions
//   Y         eta cotangents per perturbation (right vectors, nx)
//   PA, PB    Hessian pairings (t^X F)(PA_k) . PB_k  (npair each)
//   df, dV    outputs: n x n and the six canonical blocks (overwritten)
void hamiltonian_adjoint(cclr_ctx* c, int nx, const cplx* Xs, const VecSet& sol, const VecSet& xl, const VecSet& Y,
                         const VecSet& PA, const VecSet& PB, cplx* df, cplx* const* dV, cclr_solve_info* info) {
  const i64 o = c->o, v = c->v, n = o + v;
  Arena::Mark mk = c->arena.mark();
  Env e;
  e.c = c;
  // outputs double as the holomorphic cotangent accumulators
  const char* blocks[6] = {"oooo", "ooov", "oovv", "ovov", "ovvv", "vvvv"};
  const i64 bsz[6] = {o * o * o * o, o * o * o * v, o * o * v * v, o * v * o * v, o * v * v * v, v * v * v * v};
  e.gf = df;
  launch_fill(df, n * n, cx(0.0), c->stream);
  for (int b = 0; b < 6; ++b) {
    e.gv[blocks[b]] = dV[b];
    launch_fill(dV[b], bsz[b], cx(0.0), c->stream);
  }
  // values
  e.val["t1"] = ten(c->t1, {o, v});
  e.val["t2"] = ten(c->t2, {o, o, v, v});
  {
    Ten tau = dense(c, {o, o, v, v}), tt2 = dense(c, {o, o, v, v});
    tcopy(c, tau, "ijab", e.val["t2"], "ijab", cx(1.0), false);
    contract(c, cx(1.0), e.val["t1"], "ia", e.val["t1"], "jb", tau, "ijab");
    contract(c, cx(-1.0), e.val["t1"], "ib", e.val["t1"], "ja", tau, "ijab");
    tcopy(c, tt2, "jnfb", e.val["t2"], "jnfb", cx(1.0), false);
    contract(c, cx(1.0), e.val["t1"], "jf", e.val["t1"], "nb", tt2, "jnfb");
    e.val["tau"] = tau;
    e.val["tt2"] = tt2;
  }
  e.val["Foo"] = ten(c->Foo, {o, o});
  e.val["Fvv"] = ten(c->Fvv, {v, v});
  e.val["Fov"] = ten(c->Fov, {o, v});
  e.val["Woooo"] = ten(c->Woooo, {o, o, o, o});
  e.val["Wovvo"] = ten(c->Wovvo, {o, v, v, o});
  e.val["Wbar"] = ten(c->Wbar, {o, v, v, o});
  e.val["Wooov"] = ten(c->Wooov, {o, o, o, v});
  e.val["Wvovv"] = ten(c->Wvovv, {v, o, v, v});
  e.val["Wovoo"] = ten(c->Wovoo, {o, v, o, o});
  e.val["Wvvvo"] = ten(c->Wvvvo, {v, v, v, o});
  Ten l1 = dense(c, {o, v}), l2 = dense(c, {o, o, v, v});
  launch_unpack(1, (int)o, (int)v, c->lam_s.c(), c->lam_d.c(), l1.p, l2.p, c->stream);
  e.val["l1"] = l1;
  e.val["l2"] = l2;
  auto unpacked = [&](const VecSet& s, Ten& u1, Ten& u2) {
    u1 = dense(c, {(i64)s.n, o, v});
    u2 = dense(c, {(i64)s.n, o, o, v, v});
    launch_unpack(s.n, (int)o, (int)v, s.s, s.d, u1.p, u2.p, c->stream);
  };
  {
    Ten Xall = ten((cplx*)Xs, {(i64)nx, n, n});
    Ten Xoo = Xall, Xov = Xall, Xvv = Xall;
    Xoo.dim[1] = o, Xoo.dim[2] = o;
    Xov.p += o, Xov.dim[1] = o, Xov.dim[2] = v;
    Xvv.p += o * n + o, Xvv.dim[1] = v, Xvv.dim[2] = v;
    e.val["X:oo"] = Xoo;
    e.val["X:ov"] = Xov;
    e.val["X:vv"] = Xvv;
  }
  // ---- Lambda cotangent: eta^X terms paired with Y, Hessian terms paired with PB
  Ten y1, y2, a1, a2, b1, b2;
  unpacked(Y, y1, y2);
  set_groups(e, "E1", "E0", "Ea", "Ei", "Eai", y1, y2);
  reverse(e, ETA_TERMS, (int)(sizeof(ETA_TERMS) / sizeof(Term)), is_lam);
  unpacked(PA, a1, a2);
  unpacked(PB, b1, b2);
  e.val["x1"] = a1;
  e.val["x2"] = a2;
  set_groups(e, "T1", "T0", "Ta", "Ti", "Tai", b1, b2);
  reverse(e, TF_TERMS, (int)(sizeof(TF_TERMS) / sizeof(Term)), is_lam);
  // unique-amplitude cotangent of lambda: singles, and the four images of each doubles entry
  VecSet lb = packed_buf(c, 1), xt = packed_buf(c, 1);
  {
    Ten R1 = dense(c, {o, v}), R2 = dense(c, {o, o, v, v});
    launch_fill(R1.p, o * v, cx(0.0), c->stream);
    launch_fill(R2.p, o * o * v * v, cx(0.0), c->stream);
    if (e.cot.count("l1")) tcopy(c, R1, "ia", e.cot["l1"], "ia", cx(1.0), true);
    if (e.cot.count("l2")) {
      const Ten& L = e.cot["l2"];
      tcopy(c, R2, "ijab", L, "ijab", cx(1.0), true);
      tcopy(c, R2, "ijab", L, "jiab", cx(-1.0), true);
      tcopy(c, R2, "ijab", L, "ijba", cx(-1.0), true);
      tcopy(c, R2, "ijab", L, "jiba", cx(1.0), true);
    }
    launch_pack_full(1, (int)o, (int)v, R1.p, R2.p, lb.s, lb.d, c->stream);
  }
  // xt = -A^-1 lambda-bar  (A xt = -lambda-bar)
  const cplx z0 = cx(0.0);
  solve_system(c, CCLR_RIGHT, 1, &z0, lb, xt, info);
  e.cot.clear();
  // ---- H cotangents
  // sigma pairings y_k . A x_k: (left solution, right solution) and (lambda, xt)
  {
    const int np = sol.n + 1;
    Ten sx1 = dense(c, {(i64)np, o, v}), sx2 = dense(c, {(i64)np, o, o, v, v});
    Ten sy1 = dense(c, {(i64)np, o, v}), sy2 = dense(c, {(i64)np, o, o, v, v});
    const i64 s1n = o * v, s2n = o * o * v * v;
    launch_unpack(sol.n, (int)o, (int)v, sol.s, sol.d, sx1.p, sx2.p, c->stream);
    launch_unpack(1, (int)o, (int)v, xt.s, xt.d, sx1.p + sol.n * s1n, sx2.p + sol.n * s2n, c->stream);
    launch_unpack(xl.n, (int)o, (int)v, xl.s, xl.d, sy1.p, sy2.p, c->stream);
    launch_unpack(1, (int)o, (int)v, c->lam_s.c(), c->lam_d.c(), sy1.p + xl.n * s1n, sy2.p + xl.n * s2n, c->stream);
    e.val["x1"] = sx1;
    e.val["x2"] = sx2;
    set_groups(e, "S1", "S0", "Sa", "Si", "Sai", sy1, sy2);
    reverse(e, SIGMA_TERMS, (int)(sizeof(SIGMA_TERMS) / sizeof(Term)), is_h);
    for (const char* g : {"S1", "S0", "Sa", "Si", "Sai"}) e.cot.erase(g);
  }
  // Hessian pairings at fixed lambda
  e.val["x1"] = a1;
  e.val["x2"] = a2;
  set_groups(e, "T1", "T0", "Ta", "Ti", "Tai", b1, b2);
  reverse(e, TF_TERMS, (int)(sizeof(TF_TERMS) / sizeof(Term)), is_h);
  for (const char* g : {"T1", "T0", "Ta", "Ti", "Tai"}) e.cot.erase(g);
  // eta^0 . xt:  eta^0 = (F^m_e, V^ij_ab), doubles weighted 1/4 on full tensors
  {
    Ten x1 = dense(c, {o, v}), x2 = dense(c, {o, o, v, v});
    launch_unpack(1, (int)o, (int)v, xt.s, xt.d, x1.p, x2.p, c->stream);
    add_cot(e, "Fov", "me", cx(1.0), {Opnd{x1, "me"}});
    add_cot(e, "V:oovv", "ijab", cx(0.25), {Opnd{x2, "ijab"}});
  }
  // through the intermediates to f and the integral blocks
  reverse(e, H_TERMS, (int)(sizeof(H_TERMS) / sizeof(Term)), is_h);
  // gradient of the real loss: conj of the holomorphic cotangent, projected
  launch_conj_inplace(n * n, df, c->stream);
  symmetrize4(c, df, 1, (int)n, 1, (int)n, 4);  // f Hermitian: treated as pairs (0,1) <-> (2,3) with unit axes
  const int dims[6][4] = {{(int)o, (int)o, (int)o, (int)o}, {(int)o, (int)o, (int)o, (int)v},
                          {(int)o, (int)o, (int)v, (int)v}, {(int)o, (int)v, (int)o, (int)v},
                          {(int)o, (int)v, (int)v, (int)v}, {(int)v, (int)v, (int)v, (int)v}};
  const int flags[6] = {1 | 2 | 4, 1, 1 | 2, 4, 2, 1 | 2 | 4};
  for (int b = 0; b < 6; ++b) {
    launch_conj_inplace(bsz[b], dV[b], c->stream);
    symmetrize4(c, dV[b], dims[b][0], dims[b][1], dims[b][2], dims[b][3], flags[b]);
  }
  c->arena.reset(mk);
}
