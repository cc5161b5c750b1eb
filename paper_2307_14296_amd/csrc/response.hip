// Property vectors and the Hessian product for the linear response function
// (SI, "Linear response": xi^X, eta^X and (t^X F)), evaluated with the
// contraction engine on unpacked tensors and returned packed.  The
// contraction orders are chosen for cost (largest intermediate o^3 v^3 or
// o^2 v^3); the v^4 pieces go through the packed particle-particle ladder.
#include "internal.h"

namespace {
struct Groups {
  Ten X0, Xa, Xi, Xai, S1;
};

Groups groups(cclr_ctx* c, i64 nv) {
  const i64 o = c->o, v = c->v;
  Groups g;
  g.X0 = tmp(c, {nv, o, o, v, v});
  g.Xa = tmp(c, {nv, o, o, v, v});
  g.Xi = tmp(c, {nv, o, o, v, v});
  g.Xai = tmp(c, {nv, o, o, v, v});
  g.S1 = tmp(c, {nv, o, v});
  for (Ten* t : {&g.X0, &g.Xa, &g.Xi, &g.Xai, &g.S1}) launch_fill(t->p, t->size(), cx(0.0), c->stream);
  return g;
}

void finish(cclr_ctx* c, const Groups& g, i64 nv, const VecSet& out) {
  launch_fill(out.s, nv * c->ns(), cx(0.0), c->stream);
  launch_fill(out.d, nv * c->nd(), cx(0.0), c->stream);
  launch_pack_sigma((int)nv, c->o, c->v, g.X0.p, g.Xa.p, g.Xi.p, g.Xai.p, g.S1.p, out.s, out.d, nullptr, nullptr,
                    nullptr, c->stream);
}

Ten xblk(const cplx* X, cclr_ctx* c, const char* kinds) {
  const int o = c->o, n = c->o + c->v;
  Ten t = ten((cplx*)X, {(i64)n, (i64)n});
  t.p += (kinds[0] == 'o' ? 0 : o) * (i64)n + (kinds[1] == 'o' ? 0 : o);
  t.dim[0] = kinds[0] == 'o' ? o : c->v;
  t.dim[1] = kinds[1] == 'o' ? o : c->v;
  return t;
}
}  // namespace

// xi^X_mu = <mu-bar|X|CC> for one perturbation X (n x n, device) -> packed out (1 vector)
void build_xi(cclr_ctx* c, const cplx* X, const VecSet& out) {
  const i64 o = c->o, v = c->v;
  Arena::Mark mk = c->arena.mark();
  const cplx one = cx(1.0), mone = cx(-1.0);
  Ten t1 = ten(c->t1, {o, v}), t2 = ten(c->t2, {o, o, v, v});
  Ten Xoo = xblk(X, c, "oo"), Xov = xblk(X, c, "ov"), Xvo = xblk(X, c, "vo"), Xvv = xblk(X, c, "vv");
  Groups g = groups(c, 1);
  Ten S1 = ten(g.S1.p, {o, v});
  Ten Xa = ten(g.Xa.p, {o, o, v, v}), Xi = ten(g.Xi.p, {o, o, v, v});
  // singles: X^a_i + X^a_e t^e_i - X^m_i t^a_m - (X^m_e t^e_i) t^a_m + X^m_e t^ae_im
  tcopy(c, S1, "ia", Xvo, "ai", one);
  contract(c, one, Xvv, "ae", t1, "ie", S1, "ia");
  contract(c, mone, Xoo, "mi", t1, "ma", S1, "ia");
  Ten Y = tmp(c, {o, o});  // X^m_e t^e_i  -> [m][i]
  contract(c, one, Xov, "me", t1, "ie", Y, "mi", false);
  contract(c, mone, Y, "mi", t1, "ma", S1, "ia");
  contract(c, one, Xov, "me", t2, "imae", S1, "ia");
  // doubles: P(ab) X^b_f t^af_ij - P(ij) X^m_j t^ab_im - P(ij)(X^m_e t^e_i) t^ab_mj - P(ab)(X^m_f t^a_m) t^fb_ij
  contract(c, one, Xvv, "bf", t2, "ijaf", Xa, "ijab");
  contract(c, mone, Xoo, "mj", t2, "imab", Xi, "ijab");
  contract(c, mone, Y, "mi", t2, "mjab", Xi, "ijab");
  Ten Y2 = tmp(c, {v, v});  // X^m_f t^a_m -> [a][f]
  contract(c, one, Xov, "mf", t1, "ma", Y2, "af", false);
  contract(c, mone, Y2, "af", t2, "ijfb", Xa, "ijab");
  finish(c, g, 1, out);
  c->arena.reset(mk);
}

// eta^X_mu = <Lambda|[X, tau_mu]|CC> for one perturbation -> packed out
void build_eta(cclr_ctx* c, const cplx* X, const VecSet& out) {
  const i64 o = c->o, v = c->v;
  Arena::Mark mk = c->arena.mark();
  const cplx one = cx(1.0), mone = cx(-1.0), mhalf = cx(-0.5);
  Ten t1 = ten(c->t1, {o, v}), t2 = ten(c->t2, {o, o, v, v});
  Ten l1 = ten(c->lam_s, {o, v});
  Ten l2 = tmp(c, {o, o, v, v});
  launch_unpack(1, (int)o, (int)v, c->lam_s.c(), c->lam_d.c(), nullptr, l2.p, c->stream);
  Ten Xoo = xblk(X, c, "oo"), Xov = xblk(X, c, "ov"), Xvv = xblk(X, c, "vv");
  Groups g = groups(c, 1);
  Ten S1 = ten(g.S1.p, {o, v});
  Ten Xa = ten(g.Xa.p, {o, o, v, v}), Xi = ten(g.Xi.p, {o, o, v, v}), Xai = ten(g.Xai.p, {o, o, v, v});
  // singles
  tcopy(c, S1, "ia", Xov, "ia", one);
  contract(c, one, Xvv, "ea", l1, "ie", S1, "ia");
  contract(c, mone, Xoo, "im", l1, "ma", S1, "ia");
  Ten U = tmp(c, {o, o});  // t^e_m lambda^i_e -> [m][i]
  contract(c, one, t1, "me", l1, "ie", U, "mi", false);
  contract(c, mone, Xov, "ma", U, "mi", S1, "ia");
  Ten U2 = tmp(c, {o, o});  // X^i_e t^e_m -> [i][m]
  contract(c, one, Xov, "ie", t1, "me", U2, "im", false);
  contract(c, mone, U2, "im", l1, "ma", S1, "ia");
  Ten A = tmp(c, {o, o});  // t^fe_mn lambda^mi_fe -> [n][i]
  contract(c, one, t2, "mnfe", l2, "mife", A, "ni", false);
  contract(c, mhalf, A, "ni", Xov, "na", S1, "ia");
  Ten B = tmp(c, {v, v});  // t^fe_nm lambda^nm_fa -> [e][a]
  contract(c, one, t2, "nmfe", l2, "nmfa", B, "ea", false);
  contract(c, mhalf, B, "ea", Xov, "ie", S1, "ia");
  // doubles
  contract(c, one, l1, "ia", Xov, "jb", Xai, "ijab");
  contract(c, one, l2, "ijae", Xvv, "eb", Xa, "ijab");
  contract(c, mone, l2, "imab", Xoo, "jm", Xi, "ijab");
  Ten C = tmp(c, {o, v});  // t^e_m X^m_b... first (t^e_m lambda^ij_ae) then X^m_b
  Ten L3 = tmp(c, {o, o, v, o});  // t^e_m lambda^ij_ae -> [i][j][a][m]
  contract(c, one, t1, "me", l2, "ijae", L3, "ijam", false);
  contract(c, mone, L3, "ijam", Xov, "mb", Xa, "ijab");
  (void)C;
  Ten L4 = tmp(c, {o, o, v, v});  // X^j_e t^e_m -> U2[j][m]; then lambda^im_ab U2[j][m]
  (void)L4;
  contract(c, mone, l2, "imab", U2, "jm", Xi, "ijab");
  finish(c, g, 1, out);
  c->arena.reset(mk);
}

// lambda-only pieces of the Hessian product (recomputed whenever lambda changes)
struct HessPre {
  Ten LW;   // [k][i][c][a] = 1/2 lambda^ki_ef W^ef_ca + 1/2 W^ki_mn lambda^mn_ca
  Ten A1;   // [f][c] = lambda^mn_ec t^ef_mn
  Ten A2;   // [k][n] = lambda^mk_ef t^ef_mn
  Ten l2;   // lambda doubles unpacked
};

// (x F)_mu for nv packed response vectors x -> packed out  (SI, (t^X F)^k_c and (t^X F)^kl_cd)
static void hessian_block(cclr_ctx* c, const VecSet& xin, const VecSet& out);

// t^X F for several vectors, in groups whose temporaries fit in device memory
void hessian_product(cclr_ctx* c, const VecSet& xin, const VecSet& out) {
  const i64 ov = c->ns(), nd = c->nd(), oovv = (i64)c->o * c->o * c->v * c->v;
  // In the reduced-precision modes the bulk products of t^X F run on FP32 MFMA
  // (not split-BF16: the product enters the response function directly, with
  // no refinement after it, so it keeps about 1e-7 relative accuracy); the
  // FP64 mode stays FP64.
  struct Prec {
    cclr_ctx* c;
    int keep;
    Prec(cclr_ctx* c_) : c(c_), keep(c_->sigma_prec) {
      if (c->opt.prec != CCLR_FP64) c->sigma_prec = CCLR_FP32;
    }
    ~Prec() { c->sigma_prec = keep; }
  } prec(c);
  const int chunk = fit_vectors(c, 10.0 * (double)oovv * sizeof(cplx) + 2.0 * (ov + nd) * sizeof(cplx), xin.n);
  for (int k0 = 0; k0 < xin.n; k0 += chunk) {
    const int n = std::min(chunk, xin.n - k0);
    hessian_block(c, VecSet{xin.s + k0 * ov, xin.d + k0 * nd, n}, VecSet{out.s + k0 * ov, out.d + k0 * nd, n});
  }
}

static void hessian_block(cclr_ctx* c, const VecSet& xin, const VecSet& out) {
  const i64 o = c->o, v = c->v, nv = xin.n;
  Arena::Mark mk = c->arena.mark();
  const cplx one = cx(1.0), mone = cx(-1.0), half = cx(0.5), mhalf = cx(-0.5), qtr = cx(0.25);
  Ten t2 = ten(c->t2, {o, o, v, v});
  Ten Fov = ten(c->Fov, {o, v});
  Ten Woooo = ten(c->Woooo, {o, o, o, o}), Wovvo = ten(c->Wovvo, {o, v, v, o});
  Ten Wooov = ten(c->Wooov, {o, o, o, v}), Wvovv = ten(c->Wvovv, {v, o, v, v});
  Ten Vv = Vblk(c, "oovv");
  Ten l1 = ten(c->lam_s, {o, v});
  Ten l2 = tmp(c, {o, o, v, v});
  launch_unpack(1, (int)o, (int)v, c->lam_s.c(), c->lam_d.c(), nullptr, l2.p, c->stream);
  // operands of the products over unique pairs: lambda^IJ_ea for i > j ([IJ][e][a]),
  // W^ek_AB for a > b ([e][k][AB]) and the packed doubles of the vectors ([Z][IJ][AB])
  const i64 O2 = c->O2(), V2 = c->V2();
  Ten lamH = tmp(c, {O2, v, v});
  launch_pack_first_pair(1, (int)o, v * v, l2.p, lamH.p, c->stream);
  Ten WvP = tmp(c, {v, o, V2});
  launch_pack_pairs(v * o, (int)v, c->Wvovv.c(), WvP.p, c->stream);
  Ten xp2 = ten(xin.d, {nv, O2, V2});
  // lambda-only pieces
  Ten LW = tmp(c, {o, o, v, v});
  {
    VecSet lin{c->lam_s.c(), c->lam_d.c(), 1};
    VecSet lo;
    lo.s = (cplx*)c->arena.get(sizeof(cplx) * (size_t)c->ns());
    lo.d = (cplx*)c->arena.get(sizeof(cplx) * (size_t)c->nd());
    lo.n = 1;
    // packed left ladder: lo[KI][CA] = sum_EF lambda[KI][EF] W[EF][CA]  (= 1/2 lambda^ki_ef W^ef_ca)
    GemmArgs g{};
    const i64 V2 = c->V2(), O2 = c->O2();
    g.M = (int)O2; g.N = (int)V2; g.K = (int)V2; g.batch = 1;
    g.A = lin.d; g.sAm = V2; g.sAk = 1;
    g.B = c->Wp.c(); g.sBk = V2; g.sBn = 1;
    g.C = lo.d; g.sCm = V2; g.sCn = 1;
    g.ar = 1.0; g.ai = 0.0; g.beta = 0;
    with_plain_wp(c, [&]() { tuned_gemm(c, g); });
    launch_unpack(1, (int)o, (int)v, lo.s, lo.d, nullptr, LW.p, c->stream);
  }
  contract(c, half, Woooo, "kimn", l2, "mnca", LW, "kica");
  Ten A1 = tmp(c, {v, v}), A2 = tmp(c, {o, o});
  contract(c, one, l2, "mnec", t2, "mnef", A1, "fc", false);
  contract(c, one, l2, "mkef", t2, "mnef", A2, "kn", false);

  // unpack the response vectors
  Ten x1 = ten(xin.s, {nv, o, v});
  Ten x2 = tmp(c, {nv, o, o, v, v});
  launch_unpack((int)nv, (int)o, (int)v, xin.s, xin.d, nullptr, x2.p, c->stream);
  Groups G = groups(c, nv);
  Ten s = G.S1;
  // common x-dependent intermediates
  Ten Yik = tmp(c, {nv, o, o});   // [Z][i][k] = F^k_a x^a_i
  contract(c, one, Fov, "ka", x1, "Zia", Yik, "Zik", false);
  Ten Uki = tmp(c, {nv, o, o});   // [Z][k][i] = lambda^k_a x^a_i
  contract(c, one, l1, "ka", x1, "Zia", Uki, "Zki", false);
  Ten Qec = tmp(c, {nv, v, v});   // [Z][e][c] = W^ei_ca x^a_i
  contract(c, one, Wvovv, "eica", x1, "Zia", Qec, "Zec", false);
  Ten Qkm = tmp(c, {nv, o, o});   // [Z][k][m] = W^ki_ma x^a_i
  contract(c, one, Wooov, "kima", x1, "Zia", Qkm, "Zkm", false);
  Ten Uea = tmp(c, {nv, v, v});   // [Z][e][a] = lambda^i_e x^a_i
  contract(c, one, l1, "ie", x1, "Zia", Uea, "Zea", false);
  Ten Y2ki = tmp(c, {nv, o, o});  // [Z][k][i] = V^kj_ab x^ab_ij
  contract(c, one, Vv, "kjab", x2, "Zijab", Y2ki, "Zki", false);
  Ten Y3ca = tmp(c, {nv, v, v});  // [Z][c][a] = V^ij_cb x^ab_ij
  contract(c, one, Vv, "ijcb", x2, "Zijab", Y3ca, "Zca", false);
  Ten Y4jb = tmp(c, {nv, o, v});  // [Z][j][b] = lambda^i_a x^ab_ij
  contract(c, one, l1, "ia", x2, "Zijab", Y4jb, "Zjb", false);
  Ten Z2nc = tmp(c, {nv, o, v});  // [Z][n][c] = V^ni_ca x^a_i
  contract(c, one, Vv, "nica", x1, "Zia", Z2nc, "Znc", false);
  Ten Zkf = tmp(c, {nv, o, v});   // [Z][k][f] = V^ki_fa x^a_i  (= Z2 relabelled)
  (void)Zkf;
  Ten Z3cb = tmp(c, {nv, v, v});  // [Z][c][b] = lambda^ij_ac x^ab_ij
  contract(c, one, l2, "ijac", x2, "Zijab", Z3cb, "Zcb", false);
  Ten Z4kj = tmp(c, {nv, o, o});  // [Z][k][j] = lambda^ik_ab x^ab_ij
  contract(c, one, l2, "ikab", x2, "Zijab", Z4kj, "Zkj", false);

  // ---- singles (k, c)
  contract(c, one, Vv, "kica", x1, "Zia", s, "Zkc");                       // 1
  contract(c, mone, l1, "ic", Yik, "Zik", s, "Zkc");                       // 2
  contract(c, mone, Uki, "Zki", Fov, "ic", s, "Zkc");                      // 3
  contract(c, one, l1, "ke", Qec, "Zec", s, "Zkc");                        // 4
  contract(c, mone, Qkm, "Zkm", l1, "mc", s, "Zkc");                       // 5
  {
    Ten Umi = tmp(c, {nv, o, o});                                          // lambda^m_a x^a_i
    contract(c, one, l1, "ma", x1, "Zia", Umi, "Zmi", false);
    contract(c, mone, Umi, "Zmi", Wooov, "ikmc", s, "Zkc");                // 6
  }
  contract(c, one, Uea, "Zea", Wvovv, "ekac", s, "Zkc");                   // 7
  contract(c, mhalf, Y2ki, "Zki", l1, "ic", s, "Zkc");                     // 8
  contract(c, mhalf, l1, "ka", Y3ca, "Zca", s, "Zkc");                     // 9
  contract(c, one, Y4jb, "Zjb", Vv, "jkbc", s, "Zkc");                     // 10
  {
    Ten L = tmp(c, {nv, o, o, v, o});  // [Z][m][k][e][i] = lambda^mk_ae x^a_i
    contract(c, one, l2, "mkae", x1, "Zia", L, "Zmkei", false);
    contract(c, one, L, "Zmkei", Wovvo, "iecm", s, "Zkc");                 // 11 (W^ie_mc = -W^ie_cm)
    Ten Zm = tmp(c, {nv, o, v, o, o});  // [Z][k][e][m][i] = W^ke_am x^a_i
    contract(c, one, Wovvo, "keam", x1, "Zia", Zm, "Zkemi", false);
    contract(c, one, l2, "imec", Zm, "Zkemi", s, "Zkc");                   // 12 (W^ek_am = -W^ke_am)
  }
  contract(c, one, LW, "kica", x1, "Zia", s, "Zkc");                       // 13 + 14
  {
    Ten Zk = tmp(c, {nv, o, v});  // V^ki_fa x^a_i
    contract(c, one, Vv, "kifa", x1, "Zia", Zk, "Zkf", false);
    contract(c, mhalf, Zk, "Zkf", A1, "fc", s, "Zkc");                     // 15
  }
  contract(c, mhalf, A2, "kn", Z2nc, "Znc", s, "Zkc");                     // 16
  {
    Ten U = tmp(c, {nv, o, v});   // A1[f][a] x^a_i -> [i][f]
    contract(c, one, A1, "fa", x1, "Zia", U, "Zif", false);
    contract(c, mhalf, U, "Zif", Vv, "ikfc", s, "Zkc");                    // 17
    Ten U2 = tmp(c, {nv, o, v});  // A2[i][n] x^a_i -> [n][a]
    contract(c, one, A2, "in", x1, "Zia", U2, "Zna", false);
    contract(c, mhalf, U2, "Zna", Vv, "nkac", s, "Zkc");                   // 18
  }
  contract(c, mhalf, Fov, "kb", Z3cb, "Zcb", s, "Zkc");                    // 19
  contract(c, mhalf, Z4kj, "Zkj", Fov, "jc", s, "Zkc");                    // 20
  {
    Ten Z5 = tmp(c, {nv, o, v, o, v});  // [Z][k][e][j][a] = lambda^ik_eb x^ab_ij
    contract(c, one, l2, "ikeb", x2, "Zijab", Z5, "Zkeja", false);
    contract(c, mone, Z5, "Zkeja", Wvovv, "ejac", s, "Zkc");               // 21
    // lambda^mj_ac x^ab_ij = lambda^jm_ca x^ba_ji is the same array, read as [Z][m][c][i][b]
    contract(c, one, Z5, "Zmcib", Wooov, "ikmb", s, "Zkc");                // 22
    // -1/4 lambda^ij_ec W^ek_ab x^ab_ij over the unique pairs i > j, a > b (every factor
    // antisymmetric in them): Z7[Z][IJ][e][k] = sum_(a>b) W^ek_ab x^ab_ij
    Ten Z7 = tmp(c, {nv, O2, v, o});
    contract(c, one, WvP, "ekQ", xp2, "ZIQ", Z7, "ZIek", false);
    contract(c, mone, lamH, "Iec", Z7, "ZIek", s, "Zkc");                  // 23
    Ten Z8 = tmp(c, {nv, o, o, o, o});  // [Z][m][k][i][j] = lambda^mk_ab x^ab_ij
    contract(c, one, l2, "mkab", x2, "Zijab", Z8, "Zmkij", false);
    contract(c, qtr, Z8, "Zmkij", Wooov, "ijmc", s, "Zkc");                // 24
  }
  contract(c, half, Z3cb, "Zeb", Wvovv, "ekbc", s, "Zkc");                 // 25
  contract(c, mhalf, Z4kj, "Zmj", Wooov, "jkmc", s, "Zkc");                // 26

  // ---- doubles (k, l, c, d): Xi carries P(kl), Xa P(cd), Xai both
  Ten X0 = G.X0, Xa = G.Xa, Xi = G.Xi, Xai = G.Xai;
  contract(c, one, l1, "kc", Z2nc, "Zld", Xai, "Zklcd");                   // 1
  contract(c, mone, Uki, "Zki", Vv, "ilcd", Xi, "Zklcd");                  // 2
  contract(c, mone, Uea, "Zca", Vv, "klad", Xa, "Zklcd");                  // 3
  contract(c, mone, l2, "kicd", Yik, "Zil", Xi, "Zklcd");                  // 4
  {
    Ten Yad = tmp(c, {nv, v, v});  // F^i_d x^a_i -> [a][d]
    contract(c, one, Fov, "id", x1, "Zia", Yad, "Zad", false);
    contract(c, mone, l2, "klca", Yad, "Zad", Xa, "Zklcd");                // 5
  }
  contract(c, one, l2, "klce", Qec, "Zed", Xa, "Zklcd");                   // 6
  contract(c, mone, l2, "kmcd", Qkm, "Zlm", Xi, "Zklcd");                  // 7
  {
    Ten Zp = tmp(c, {nv, o, o, o, o});  // [Z][k][l][m][i] = W^kl_ma x^a_i
    contract(c, one, Wooov, "klma", x1, "Zia", Zp, "Zklmi", false);
    contract(c, one, l2, "micd", Zp, "Zklmi", X0, "Zklcd");                // 9
  }
  contract(c, mhalf, l2, "klca", Y3ca, "Zda", Xa, "Zklcd");                // 12
  contract(c, mhalf, l2, "kicd", Y2ki, "Zli", Xi, "Zklcd");                // 13
  {
    Ten M = tmp(c, {nv, o, o, o, o});  // [Z][k][l][i][j] = V^kl_ab x^ab_ij
    contract(c, one, Vv, "klab", x2, "Zijab", M, "Zklij", false);
    contract(c, qtr, M, "Zklij", l2, "ijcd", X0, "Zklcd");                 // 14
    Ten N = tmp(c, {nv, o, o, o, o});  // [Z][k][l][i][j] = lambda^kl_ab x^ab_ij
    contract(c, one, l2, "klab", x2, "Zijab", N, "Zklij", false);
    contract(c, qtr, N, "Zklij", Vv, "ijcd", X0, "Zklcd");                 // 15
    // terms 8, 10 and 16 under P(kl)P(cd) as one product lambda^ky_cw T[l][d][y][w]
    // (8 read with k and l exchanged, 10 with c and d exchanged, each a sign):
    //   T[l][d][y][w] = V^li_da x^aw_iy (16) + W^li_yd x^w_i (8) - W^wl_da x^a_y (10)
    Ten T = tmp(c, {nv, o, v, o, v});
    contract(c, one, Vv, "lida", x2, "Zijab", T, "Zldjb", false);          // 16: V^li_da x^ab_ij
    contract(c, one, Wooov, "liyd", x1, "Ziw", T, "Zldyw");                // 8
    contract(c, mone, Wvovv, "wlda", x1, "Zya", T, "Zldyw");               // 10
    contract(c, one, l2, "kycw", T, "Zldyw", Xai, "Zklcd");                // 8 + 10 + 16
  }
  contract(c, mhalf, Z4kj, "Zkj", Vv, "jlcd", Xi, "Zklcd");                // 17
  contract(c, mhalf, Z3cb, "Zcb", Vv, "klbd", Xa, "Zklcd");                // 18
  finish(c, G, nv, out);
  // term 11, -lambda^kl_ea x^a_i W^ei_cd, has no permutation operator: only its
  // unique pairs k > l, c > d enter the result, so it is added to the packed
  // doubles directly: out[KL][CD] -= sum_(e,i) Lp[KL][e][i] W^ei_CD
  {
    Ten Lp = tmp(c, {nv, O2, v, o});  // [Z][KL][e][i] = lambda^kl_ea x^a_i  (k > l)
    contract(c, one, lamH, "Kea", x1, "Zia", Lp, "ZKei", false);
    contract(c, mone, Lp, "ZKei", WvP, "eiC", ten(out.d, {nv, O2, V2}), "ZKC");  // 11
  }
  c->arena.reset(mk);
}

// --------------------------------------------------------------------------
// Adjoint pieces of the response function with respect to a perturbation X.
// xi^X and eta^X are linear in X, so for a vector y the scalars y.xi^X and
// eta^X.y are linear functionals of X; their gradients
//   Dxi(y)[p][q]  = d (y . xi^X)  / d X[p][q]
//   Deta(y)[p][q] = d (eta^X . y) / d X[p][q]
// are one-particle "transition densities", obtained term by term from the
// programmable expressions of xi^X and eta^X (SI, "Linear response").  Both
// accumulate alpha * D into the n x n matrix D (device).
// --------------------------------------------------------------------------
namespace {
Ten dblk(cplx* D, cclr_ctx* c, const char* kinds) { return xblk(D, c, kinds); }
}  // namespace

void density_xi(cclr_ctx* c, const VecSet& y, cplx* D, cplx alpha) {
  const i64 o = c->o, v = c->v;
  Arena::Mark mk = c->arena.mark();
  auto mul = [&](double s) { return cx(alpha.x * s, alpha.y * s); };
  Ten t1 = ten(c->t1, {o, v}), t2 = ten(c->t2, {o, o, v, v});
  Ten y1 = ten(y.s, {o, v});
  Ten y2 = tmp(c, {o, o, v, v});
  launch_unpack(1, (int)o, (int)v, y.s, y.d, nullptr, y2.p, c->stream);
  Ten Doo = dblk(D, c, "oo"), Dov = dblk(D, c, "ov"), Dvo = dblk(D, c, "vo"), Dvv = dblk(D, c, "vv");
  // singles: X^a_i + X^a_e t^e_i - X^m_i t^a_m - (X^m_e t^e_i) t^a_m + X^m_e t^ae_im
  tcopy(c, Dvo, "ai", y1, "ia", mul(1.0));
  Ten U = tmp(c, {v, v});  // y_i^a t^e_i -> [a][e]
  contract(c, cx(1.0), y1, "ia", t1, "ie", U, "ae", false);
  tcopy(c, Dvv, "ae", U, "ae", mul(1.0));
  contract(c, mul(-1.0), y1, "ia", t1, "ma", Doo, "mi");
  contract(c, mul(-1.0), t1, "ma", U, "ae", Dov, "me");
  contract(c, mul(1.0), y1, "ia", t2, "imae", Dov, "me");
  // doubles (1/4 sum over unrestricted indices; P() doubles each term on antisymmetric y)
  contract(c, mul(0.5), y2, "ijab", t2, "ijaf", Dvv, "bf");
  contract(c, mul(-0.5), y2, "ijab", t2, "imab", Doo, "mj");
  Ten W = tmp(c, {o, o});  // y^ij_ab t^ab_mj -> [i][m]
  contract(c, cx(1.0), y2, "ijab", t2, "mjab", W, "im", false);
  contract(c, mul(-0.5), W, "im", t1, "ie", Dov, "me");
  Ten Q = tmp(c, {v, v});  // y^ij_ab t^fb_ij -> [a][f]
  contract(c, cx(1.0), y2, "ijab", t2, "ijfb", Q, "af", false);
  contract(c, mul(-0.5), t1, "ma", Q, "af", Dov, "mf");
  c->arena.reset(mk);
}

void density_eta(cclr_ctx* c, const VecSet& y, cplx* D, cplx alpha) {
  const i64 o = c->o, v = c->v;
  Arena::Mark mk = c->arena.mark();
  auto mul = [&](double s) { return cx(alpha.x * s, alpha.y * s); };
  Ten t1 = ten(c->t1, {o, v}), t2 = ten(c->t2, {o, o, v, v});
  Ten l1 = ten(c->lam_s, {o, v});
  Ten l2 = tmp(c, {o, o, v, v});
  launch_unpack(1, (int)o, (int)v, c->lam_s.c(), c->lam_d.c(), nullptr, l2.p, c->stream);
  Ten y1 = ten(y.s, {o, v});
  Ten y2 = tmp(c, {o, o, v, v});
  launch_unpack(1, (int)o, (int)v, y.s, y.d, nullptr, y2.p, c->stream);
  Ten Doo = dblk(D, c, "oo"), Dov = dblk(D, c, "ov"), Dvv = dblk(D, c, "vv");
  // singles of eta^X
  tcopy(c, Dov, "ia", y1, "ia", mul(1.0));
  contract(c, mul(1.0), l1, "ie", y1, "ia", Dvv, "ea");
  contract(c, mul(-1.0), l1, "ma", y1, "ia", Doo, "im");
  Ten U = tmp(c, {o, o});  // t^e_m lambda^i_e -> [m][i]
  contract(c, cx(1.0), t1, "me", l1, "ie", U, "mi", false);
  contract(c, mul(-1.0), U, "mi", y1, "ia", Dov, "ma");
  Ten P = tmp(c, {v, v});  // t^e_m lambda^m_a -> [e][a]
  contract(c, cx(1.0), t1, "me", l1, "ma", P, "ea", false);
  contract(c, mul(-1.0), y1, "ia", P, "ea", Dov, "ie");
  Ten A = tmp(c, {o, o});  // t^fe_mn lambda^mi_fe -> [n][i]
  contract(c, cx(1.0), t2, "mnfe", l2, "mife", A, "ni", false);
  contract(c, mul(-0.5), A, "ni", y1, "ia", Dov, "na");
  Ten B = tmp(c, {v, v});  // t^fe_nm lambda^nm_fa -> [e][a]
  contract(c, cx(1.0), t2, "nmfe", l2, "nmfa", B, "ea", false);
  contract(c, mul(-0.5), B, "ea", y1, "ia", Dov, "ie");
  // doubles of eta^X
  contract(c, mul(1.0), y2, "ijab", l1, "ia", Dov, "jb");
  contract(c, mul(0.5), y2, "ijab", l2, "ijae", Dvv, "eb");
  Ten Y = tmp(c, {o, o});  // y^ij_ab lambda^im_ab -> [j][m]
  contract(c, cx(1.0), y2, "ijab", l2, "imab", Y, "jm", false);
  tcopy(c, Doo, "jm", Y, "jm", mul(-0.5));
  Ten L3 = tmp(c, {o, o, v, o});  // t^e_m lambda^ij_ae -> [i][j][a][m]
  contract(c, cx(1.0), t1, "me", l2, "ijae", L3, "ijam", false);
  contract(c, mul(-0.5), y2, "ijab", L3, "ijam", Dov, "mb");
  contract(c, mul(-0.5), Y, "jm", t1, "me", Dov, "je");
  c->arena.reset(mk);
}
