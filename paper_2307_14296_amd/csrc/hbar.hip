// Property-independent Hbar intermediates (SI, "EOM-EE sigma-vectors and
// intermediates": eqs. F_im, F_ea, F_me, W_ijmn, W_mbej, W_iemn, W_efam,
// W_efab, barW_mbej, W_mnie, W_amef and tau).  Stored unpacked with
// W[p][q][r][s] = W^pq_rs (bra pq, ket rs) and F[p][q] = F^p_q, except
// W^ef_ab, which is built and kept only packed (e>f, a>b) for the
// particle-particle ladder: no v^4 tensor is formed beyond the integrals.
//
// Sign/index readings of the printed equations (each decided by second-
// quantization brute force on random complex data): F^a_e is the Hbar
// element with bra a and ket e; W_iemn carries -F^i_f t^ef_mn; W_efam
// carries -P(ef) V^en_ag t^gf_mn.
#include "internal.h"

void launch_diag(int o, int v, const cplx* Foo, const cplx* Fvv, cplx* diag, hipStream_t s);

// The doubles term P(ab) F^b_e r^ae_ij of the transforms equals
// 1/2 sum_ef D^ab_ef r^ef_ij with the pair operator
//   D^ab_ef = d_ae F^b_f - d_af F^b_e - d_be F^a_f + d_bf F^a_e,
// so it is carried by the packed particle ladder when D is added to Wp[AB][EF];
// read as Wp[EF][AB] the same array gives the left-transform term P(ab) l^ae_ij F^e_b.
void fold_vv(cclr_ctx* c, double sign) {
  if (c->v < 2 || !c->Wp.p) return;
  launch_pair_fold((int)c->v, c->Fvv.c(), c->Wp.c(), sign, c->stream);
}

void build_intermediates(cclr_ctx* c) {
  const i64 o = c->o, v = c->v;
  for (int w = 0; w < 4; ++w) {  // split copies of the previous operators
    c->wsplit[w].release();
    c->wsplit_m[w] = SplitMat{};
  }
  Arena::Mark mk = c->arena.mark();
  const cplx one = cx(1.0), mone = cx(-1.0), half = cx(0.5), mhalf = cx(-0.5);
  Ten t1 = ten(c->t1, {o, v});
  Ten t2 = ten(c->t2, {o, o, v, v});
  // tau^ab_ij = t^ab_ij + t^a_i t^b_j - t^b_i t^a_j
  Ten tau = tmp(c, {o, o, v, v});
  tcopy(c, tau, "ijab", t2, "ijab", one, false);
  contract(c, one, t1, "ia", t1, "jb", tau, "ijab");
  contract(c, mone, t1, "ib", t1, "ja", tau, "ijab");

  auto alloc = [&](DevBuf& b, i64 n) {
    b.alloc(c, sizeof(cplx) * (size_t)n);
    launch_fill(b.c(), n, cx(0.0), c->stream);
  };
  alloc(c->Foo, o * o);
  alloc(c->Fvv, v * v);
  alloc(c->Fov, o * v);
  alloc(c->Woooo, o * o * o * o);
  alloc(c->Wovvo, o * v * v * o);
  alloc(c->Wbar, o * v * v * o);
  alloc(c->Wooov, o * o * o * v);
  alloc(c->Wvovv, v * o * v * v);
  alloc(c->Wovoo, o * v * o * o);
  alloc(c->Wvvvo, v * v * v * o);

  Ten Foo = ten(c->Foo, {o, o}), Fvv = ten(c->Fvv, {v, v}), Fov = ten(c->Fov, {o, v});
  Ten Woooo = ten(c->Woooo, {o, o, o, o}), Wovvo = ten(c->Wovvo, {o, v, v, o}), Wbar = ten(c->Wbar, {o, v, v, o});
  Ten Wooov = ten(c->Wooov, {o, o, o, v}), Wvovv = ten(c->Wvovv, {v, o, v, v});
  Ten Wovoo = ten(c->Wovoo, {o, v, o, o}), Wvvvo = ten(c->Wvvvo, {v, v, v, o});
  Ten Voovv = Vblk(c, "oovv");

  // F^i_m = f^i_m + f^i_e t^e_m + V^in_me t^e_n + 1/2 V^in_ef tau^ef_mn
  tcopy(c, Foo, "im", fblk(c, "oo"), "im", one);
  contract(c, one, fblk(c, "ov"), "ie", t1, "me", Foo, "im");
  contract(c, one, Vblk(c, "ooov"), "inme", t1, "ne", Foo, "im");
  contract(c, half, Voovv, "inef", tau, "mnef", Foo, "im");
  // F^a_e = f^a_e - f^m_e t^a_m + V^am_ef t^f_m - 1/2 V^mn_ef tau^af_mn
  tcopy(c, Fvv, "ae", fblk(c, "vv"), "ae", one);
  contract(c, mone, fblk(c, "ov"), "me", t1, "ma", Fvv, "ae");
  contract(c, one, Vblk(c, "vovv"), "amef", t1, "mf", Fvv, "ae");
  contract(c, mhalf, Voovv, "mnef", tau, "mnaf", Fvv, "ae");
  // F^m_e = f^m_e + V^mn_ef t^f_n
  tcopy(c, Fov, "me", fblk(c, "ov"), "me", one);
  contract(c, one, Voovv, "mnef", t1, "nf", Fov, "me");
  // W^ij_mn = V^ij_mn + P(mn) V^ij_en t^e_m + 1/2 V^ij_ef tau^ef_mn
  tcopy(c, Woooo, "ijmn", Vblk(c, "oooo"), "ijmn", one);
  {
    Ten w = tmp(c, {o, o, o, o});
    contract(c, one, Vblk(c, "oovo"), "ijen", t1, "me", w, "ijmn", false);
    tcopy(c, Woooo, "ijmn", w, "ijmn", one);
    tcopy(c, Woooo, "ijmn", w, "ijnm", mone);
  }
  contract(c, half, Voovv, "ijef", tau, "mnef", Woooo, "ijmn");
  // W^mb_ej = V^mb_ej + V^mb_ef t^f_j - V^mn_ej t^b_n - V^mn_ef (t^fb_jn + t^f_j t^b_n)
  tcopy(c, Wovvo, "mbej", Vblk(c, "ovvo"), "mbej", one);
  contract(c, one, Vblk(c, "ovvv"), "mbef", t1, "jf", Wovvo, "mbej");
  contract(c, mone, Vblk(c, "oovo"), "mnej", t1, "nb", Wovvo, "mbej");
  {
    Ten w = tmp(c, {o, o, v, v});  // t^fb_jn + t^f_j t^b_n, labels jnfb
    tcopy(c, w, "jnfb", t2, "jnfb", one, false);
    contract(c, one, t1, "jf", t1, "nb", w, "jnfb");
    contract(c, mone, Voovv, "mnef", w, "jnfb", Wovvo, "mbej");
  }
  // barW^mb_ej = V^mb_ej - V^mn_ef t^bf_nj
  tcopy(c, Wbar, "mbej", Vblk(c, "ovvo"), "mbej", one);
  contract(c, mone, Voovv, "mnef", t2, "njbf", Wbar, "mbej");
  // W^mn_ie = V^mn_ie + t^f_i V^mn_fe
  tcopy(c, Wooov, "mnie", Vblk(c, "ooov"), "mnie", one);
  contract(c, one, t1, "if", Voovv, "mnfe", Wooov, "mnie");
  // W^am_ef = V^am_ef - V^nm_ef t^a_n
  tcopy(c, Wvovv, "amef", Vblk(c, "vovv"), "amef", one);
  contract(c, mone, Voovv, "nmef", t1, "na", Wvovv, "amef");
  // W^ef_ab = V^ef_ab - P(ef) V^mf_ab t^e_m + 1/2 V^mn_ab tau^ef_mn, packed: Wp[EF][AB]
  {
    const i64 V2 = c->V2(), O2 = c->O2();
    c->Wp.alloc(c, sizeof(cplx) * (size_t)(V2 * V2));
    launch_pack_vvvv((int)v, c->Vvvvv.c(), c->Wp.c(), c->stream);
    Arena::Mark m2 = c->arena.mark();
    // - P(ef) t^e_m V^mf_ab: Y[e][f][AB] = t^e_m V^mf_ab over column blocks of AB
    cplx* P = (cplx*)c->arena.get(sizeof(cplx) * (size_t)(o * v * V2));  // P[m][f][AB] = V^mf_ab
    launch_pack_pairs(o * v, (int)v, c->Vovvv.c(), P, c->stream);
    i64 nc = std::max<i64>(1, std::min<i64>(V2, (i64)(size_t(1) << 27) / (v * v)));  // Y block <= 2 GiB
    if (c->dbg_wp_block > 0) nc = std::min<i64>(V2, c->dbg_wp_block);
    Ten Y = tmp(c, {v, v, nc});
    for (i64 c0 = 0; c0 < V2; c0 += nc) {
      const i64 n = std::min(nc, V2 - c0);
      Ten Pb;
      Pb.p = P + c0;
      Pb.nd = 3;
      Pb.dim[0] = o, Pb.dim[1] = v, Pb.dim[2] = n;
      Pb.st[0] = v * V2, Pb.st[1] = V2, Pb.st[2] = 1;
      Ten Yb = ten(Y.p, {v, v, n});
      contract(c, one, t1, "me", Pb, "mfX", Yb, "efX", false);
      launch_pair_antisym_acc((int)v, (int)n, Yb.p, c->Wp.c() + c0, V2, -1.0, c->stream);
    }
    // + sum_(m>n) tau^ef_mn V^mn_ab: packed product over the occupied pairs
    VecSet tp = packed_buf(c, 1), vp = packed_buf(c, 1);
    launch_pack_full(1, (int)o, (int)v, t1.p, tau.p, tp.s, tp.d, c->stream);
    launch_pack_full(1, (int)o, (int)v, t1.p, c->Voovv.c(), vp.s, vp.d, c->stream);
    GemmArgs g{};
    g.M = (int)V2; g.N = (int)V2; g.K = (int)O2; g.batch = 1;
    g.A = tp.d; g.sAm = 1; g.sAk = V2;
    g.B = vp.d; g.sBk = V2; g.sBn = 1;
    g.C = c->Wp.c(); g.sCm = V2; g.sCn = 1;
    g.ar = 1.0; g.ai = 0.0; g.beta = 1;
    tuned_gemm(c, g);
    c->arena.reset(m2);
  }
  // W^ie_mn = V^ie_mn - F^i_f t^ef_mn - W^io_mn t^e_o + 1/2 V^ie_fg tau^fg_mn
  //          + P(mn) barW^ie_fn t^f_m + P(mn) V^io_mf t^ef_no
  tcopy(c, Wovoo, "iemn", Vblk(c, "ovoo"), "iemn", one);
  contract(c, mone, Fov, "if", t2, "mnef", Wovoo, "iemn");
  contract(c, mone, Woooo, "iomn", t1, "oe", Wovoo, "iemn");
  contract(c, half, Vblk(c, "ovvv"), "iefg", tau, "mnfg", Wovoo, "iemn");
  {
    Ten w = tmp(c, {o, v, o, o});
    contract(c, one, Wbar, "iefn", t1, "mf", w, "iemn", false);
    contract(c, one, Vblk(c, "ooov"), "iomf", t2, "noef", w, "iemn");
    tcopy(c, Wovoo, "iemn", w, "iemn", one);
    tcopy(c, Wovoo, "iemn", w, "ienm", mone);
  }
  // W^ef_am = V^ef_am - P(ef) V^en_ag t^gf_mn + W^ef_ag t^g_m + F^n_a t^ef_mn
  //          + 1/2 V^no_am tau^ef_no - P(ef) barW^nf_am t^e_n
  tcopy(c, Wvvvo, "efam", Vblk(c, "vvvo"), "efam", one);
  // W^ef_ag t^g_m is formed from the pieces of W^ef_ag (no unpacked W^ef_ab):
  //   V^ef_ag t^g_m - P(ef) t^e_n (V^nf_ag t^g_m) + 1/2 tau^ef_no (V^no_ag t^g_m)
  {
    Ten w = tmp(c, {v, v, v, o});
    contract(c, mone, Vblk(c, "vovv"), "enag", t2, "mngf", w, "efam", false);
    contract(c, mone, Wbar, "nfam", t1, "ne", w, "efam");
    Ten Q = tmp(c, {o, v, v, o});
    contract(c, one, Vblk(c, "ovvv"), "nfag", t1, "mg", Q, "nfam", false);
    contract(c, mone, t1, "ne", Q, "nfam", w, "efam");
    tcopy(c, Wvvvo, "efam", w, "efam", one);
    tcopy(c, Wvvvo, "efam", w, "feam", mone);
  }
  contract(c, one, Vblk(c, "vvvv"), "efag", t1, "mg", Wvvvo, "efam");
  {
    Ten R = tmp(c, {o, o, v, o});
    contract(c, one, Voovv, "noag", t1, "mg", R, "noam", false);
    contract(c, half, tau, "noef", R, "noam", Wvvvo, "efam");
  }
  contract(c, one, Fov, "na", t2, "mnef", Wvvvo, "efam");
  contract(c, half, Vblk(c, "oovo"), "noam", tau, "noef", Wvvvo, "efam");

  // ring operators in GEMM-ready layouts
  c->WR.alloc(c, sizeof(cplx) * (size_t)(o * v * o * v));
  c->WL.alloc(c, sizeof(cplx) * (size_t)(o * v * o * v));
  tcopy(c, ten(c->WR, {o, v, o, v}), "jbme", Wovvo, "mbej", one, false);
  tcopy(c, ten(c->WL, {o, v, o, v}), "mejb", Wovvo, "jebm", one, false);
  // W^ab_ej as [j][e][a][b] for the right doubles term P(ij) W^ab_ej r^e_i (unit-stride ab)
  if (v >= 2) {
    // W^ab_ej as [j][e][AB] (a > b) for the right doubles term P(ij) W^ab_ej r^e_i
    Ten wt = tmp(c, {o, v, v, v});
    tcopy(c, wt, "jeab", Wvvvo, "abej", one, false);
    c->WvvvoTP.alloc(c, sizeof(cplx) * (size_t)(o * v * c->V2()));
    launch_pack_pairs(o * v, (int)v, wt.p, c->WvvvoTP.c(), c->stream);
  }
  // left-transform layouts with unit-stride reductions: W^ef_am as [a][m][e][f], W^ei_fa as [i][a][f][e]
  if (v >= 2) {
    // W^ef_am as [a][m][EF] (e > f) for the left singles term 1/2 l^im_ef W^ef_am
    Ten wl = tmp(c, {v, o, v, v});
    tcopy(c, wl, "amef", Wvvvo, "efam", one, false);
    c->WvvvoLP.alloc(c, sizeof(cplx) * (size_t)(v * o * c->V2()));
    launch_pack_pairs(v * o, (int)v, wl.p, c->WvvvoLP.c(), c->stream);
  }
  c->WvovvL.alloc(c, sizeof(cplx) * (size_t)(o * v * v * v));
  tcopy(c, ten(c->WvovvL, {o, v, v, v}), "iafe", Wvovv, "eifa", one, false);
  // pair-packed operators of the right transform's o^2 v^3 products
  if (o >= 2 && v >= 2) {
    const i64 O2 = c->O2(), V2 = c->V2();
    c->VoovvH.alloc(c, sizeof(cplx) * (size_t)(O2 * v * v));
    launch_pack_first_pair(1, (int)o, v * v, c->Voovv.c(), c->VoovvH.c(), c->stream);
    c->VoovvP.alloc(c, sizeof(cplx) * (size_t)(o * o * V2));
    launch_pack_pairs(o * o, (int)v, c->Voovv.c(), c->VoovvP.c(), c->stream);
    c->WvovvP.alloc(c, sizeof(cplx) * (size_t)(v * o * V2));
    launch_pack_pairs(v * o, (int)v, c->Wvovv.c(), c->WvovvP.c(), c->stream);
    // -sum_me F^m_e r^ea_im = sum_(m, e>f) X^am_ef r^ef_im with X^am_ef = d_ea F^m_f - d_fa F^m_e
    launch_fold_ov((int)o, (int)v, c->Fov.c(), c->WvovvP.c(), c->stream);
    c->WovooH.alloc(c, sizeof(cplx) * (size_t)(o * v * O2));
    launch_pack_pairs(o * v, (int)o, c->Wovoo.c(), c->WovooH.c(), c->stream);
    c->WooovH.alloc(c, sizeof(cplx) * (size_t)(O2 * o * v));
    launch_pack_first_pair(1, (int)o, o * v, c->Wooov.c(), c->WooovH.c(), c->stream);
    c->t2P.alloc(c, sizeof(cplx) * (size_t)(o * o * V2));
    launch_pack_pairs(o * o, (int)v, c->t2.c(), c->t2P.c(), c->stream);
    c->t2H.alloc(c, sizeof(cplx) * (size_t)(O2 * v * v));
    launch_pack_first_pair(1, (int)o, v * v, c->t2.c(), c->t2H.c(), c->stream);
  }
  // particle-ladder operator of the transforms: W^ab_ef plus the doubles term
  // P(ab) F^b_e r^ae_ij written as a pair operator (fold_vv)
  fold_vv(c, 1.0);
  // hole-ladder operator of the transforms on packed pairs: W^mn_ij plus the
  // doubles term -P(ij) F^m_j r^ab_im written as a pair operator,
  //   E^mn_ij = -(d_im F^n_j - d_in F^m_j - d_jm F^n_i + d_jn F^m_i),
  // so that 1/2 sum_mn (W + E)^mn_ij r^ab_mn carries both (the same array read
  // as [IJ][MN] gives the left-transform terms 1/2 l^mn_ab W^ij_mn - P(ij) l^im_ab F^j_m)
  if (o >= 2) {
    c->Wop.alloc(c, sizeof(cplx) * (size_t)(c->O2() * c->O2()));
    launch_pack_vvvv((int)o, c->Woooo.c(), c->Wop.c(), c->stream);
    launch_pair_fold((int)o, c->Foo.c(), c->Wop.c(), -1.0, c->stream);
  }
  // preconditioner diagonal
  c->diag.alloc(c, sizeof(cplx) * (size_t)(c->ns() + c->nd()));
  launch_diag((int)o, (int)v, c->Foo.c(), c->Fvv.c(), c->diag.c(), c->stream);
  HIPCHK(hipStreamSynchronize(c->stream));
  c->arena.reset(mk);
  c->arena.trim();  // the v^4 temporaries of the build are not needed again
}
