// Right and left EOM-EE sigma vectors (SI, eqs. sigma_sin-ee,
// sigma_double-ee, sigma_sin-ee-left, sigma_double-ee-left) on packed
// vector sets.
//
// The doubles of every term are accumulated unsymmetrized into four groups
// (no permutation operator, P(ab), P(ij), P(ab)P(ij)); the antisymmetrizers
// are applied once, while packing the i>j, a>b result.  The particle-
// particle ladder 1/2 W^ab_ef r^ef_ij is evaluated directly on packed pairs:
// sigma[IJ][AB] = sum_EF r[IJ][EF] W[AB][EF]  (right) and
// sigma[IJ][AB] = sum_EF l[IJ][EF] W[EF][AB]  (left), with e>f so the 1/2
// is absorbed; the doubles term P(ab) F^b_e r^ae_ij is folded into the same
// packed operator when the intermediates are built.  So is the hole ladder 1/2 W^mn_ij r^ab_mn together with the
// doubles term -P(ij) F^m_j r^ab_im (folded into one packed pair operator
// when the intermediates are built): sigma[IJ][AB] += sum_MN W[MN][IJ] r[MN][AB]
// (right; left: W[IJ][MN]).  Readings applied: the right-singles ring element is W^ma_ei;
// the left doubles carry -P(ab) l^m_a W^ij_mb, P(ij) l^i_e W^ej_ab and
// 1/2 l^ij_ef W^ef_ab.
#include "internal.h"

namespace {

// xi_vpacked: the P(ij) group only for the pairs a > b ([k][i][j][AB]; no P(ab) acts on it)
SigmaAcc prepare(cclr_ctx* c, const VecSet& in, bool xi_vpacked) {
  const i64 o = c->o, v = c->v, k = in.n;
  SigmaAcc a;
  a.R1 = ten(in.s, {k, o, v});
  a.R2 = tmp(c, {k, o, o, v, v});
  launch_unpack((int)k, (int)o, (int)v, in.s, in.d, nullptr, a.R2.p, c->stream);
  // no group without a permutation operator remains outside the packed ladders (X0 stays empty)
  // P(ab) group of the pairs i > j only ([k][IJ][a][b]): no P(ij) acts on it
  a.Xa = tmp(c, {k, c->O2(), v, v});
  a.Xi = xi_vpacked ? tmp(c, {k, o, o, c->V2()}) : tmp(c, {k, o, o, v, v});
  // P(ab)P(ij) group in the ring layout [k][i][a][j][b], seen through a kijab view
  a.Xai = reorder(tmp(c, {k, o, v, o, v}), "kiajb", "kijab");
  a.S1 = tmp(c, {k, o, v});
  for (Ten* t : {&a.Xa, &a.Xi, &a.S1}) launch_fill(t->p, t->size(), cx(0.0), c->stream);
  return a;
}

// Product with one of the Jacobian's large operators (B side of g: 0 right
// ladder, 1 left ladder, 2 right ring, 3 left ring) in the arithmetic of the
// transforms being applied.  FP32 and split-BF16 keep a split copy of the
// operator, made on first use; the trial-vector side is split per product.
void op_gemm(cclr_ctx* c, const GemmArgs& g, int which) {
  if (c->sigma_prec == CCLR_FP64) {
    if (which < 2) tuned_gemm(c, g);
    else run_gemm(c, g);
    return;
  }
  REQUIRE(g.batch == 1 && g.kchunk == 0, CCLR_EINVAL, "unsupported product form");
  const int form = split_form_of(c->sigma_prec);
  SplitMat& W = c->wsplit_m[which];
  if (!W.p || W.form != form) {
    c->wsplit_m[which] = SplitMat{};
    c->wsplit[which].release();
    c->wsplit[which].alloc(c, split_bytes(g.N, g.K, form, 1));
    W = launch_split(g.N, g.K, g.B, g.sBn, g.sBk, g.conjB, c->wsplit[which].p, form, 1, c->stream);
  }
  REQUIRE(W.rows == g.N && W.K == g.K, CCLR_EINVAL, "split operator has another shape");
  Arena::Mark mk = c->arena.mark();
  void* ws = c->arena.get(split_bytes(g.M, g.K, form, 0));
  const SplitMat A = launch_split(g.M, g.K, g.A, g.sAm, g.sAk, g.conjA, ws, form, 0, c->stream);
  launch_split_gemm(A, W, g.C, g.sCm, g.sCn, g.ar, g.ai, g.beta, c->stream);
  c->arena.reset(mk);
}

// Ring term  Z[(k,i,a),(j,b)] = sum_(m,e) R[(k,i,a),(m,e)] W[(m,e),(j,b)]  written into the
// [k][i][a][j][b] accumulator (first writer: overwrites).  Right: W^mb_ej r^ae_im;
// left: l^im_ae W^je_bm.  Unpacks the vectors into the ring layout (arena) and
// returns the product; the caller launches it.
GemmArgs ring_args(cclr_ctx* c, const VecSet& in, const Ten& Xai, bool right) {
  const i64 o = c->o, v = c->v, ov = o * v, nv = in.n;
  cplx* rr = (cplx*)c->arena.get(sizeof(cplx) * (size_t)(nv * ov * ov));
  launch_unpack_ring((int)nv, (int)o, (int)v, in.d, rr, c->stream);
  GemmArgs g{};
  g.M = (int)(nv * ov);
  g.N = (int)ov;
  g.K = (int)ov;
  g.batch = 1;
  g.A = rr; g.sAm = ov; g.sAk = 1;
  if (right) { g.B = c->WR.c(); g.sBk = 1; g.sBn = ov; }
  else { g.B = c->WL.c(); g.sBk = ov; g.sBn = 1; }
  g.C = Xai.p; g.sCm = ov; g.sCn = 1;
  g.ar = 1.0; g.ai = 0.0; g.beta = 0;
  return g;
}

// Particle-particle ladder on packed pairs (overwrites the packed doubles of out).
GemmArgs ladder_args(cclr_ctx* c, const VecSet& in, const VecSet& out, bool right) {
  const i64 V2 = c->V2(), O2 = c->O2();
  GemmArgs g{};
  g.M = (int)(O2 * in.n);
  g.N = (int)V2;
  g.K = (int)V2;
  g.batch = 1;
  g.A = in.d; g.sAb = 0; g.sAm = V2; g.sAk = 1; g.conjA = 0;
  g.B = c->Wp.c(); g.sBb = 0; g.conjB = 0;
  if (right) { g.sBk = 1; g.sBn = V2; }
  else { g.sBk = V2; g.sBn = 1; }
  g.C = out.d; g.sCb = 0; g.sCm = V2; g.sCn = 1;
  g.ar = 1.0; g.ai = 0.0; g.beta = 0;
  return g;
}

// Hole ladder on packed pairs, accumulated into the packed doubles of out
// (after the particle-particle ladder, which overwrites them):
// out[k][IJ][AB] += sum_MN Wop[MN][IJ] in[k][MN][AB] (right) or Wop[IJ][MN] (left).
void hole_ladder(cclr_ctx* c, const VecSet& in, const VecSet& out, bool right) {
  const i64 O2 = c->O2(), V2 = c->V2();
  if (O2 == 0 || V2 == 0 || in.n == 0) return;
  GemmArgs g{};
  g.M = (int)O2;
  g.N = (int)V2;
  g.K = (int)O2;
  g.batch = (int)in.n;
  g.A = c->Wop.c(); g.sAb = 0;
  if (right) { g.sAm = 1; g.sAk = O2; }
  else { g.sAm = O2; g.sAk = 1; }
  g.B = in.d; g.sBb = O2 * V2; g.sBk = V2; g.sBn = 1;
  g.C = out.d; g.sCb = O2 * V2; g.sCm = V2; g.sCn = 1;
  g.ar = 1.0; g.ai = 0.0; g.beta = 1;
  run_gemm(c, g);
}

// launch with optional event timing (the debug profile hook)
template <class F>
void timed(cclr_ctx* c, double flops, F&& launch) {
  if (!c->prof) {
    launch();
    return;
  }
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  HIPCHK(hipEventRecord(e0, c->stream));
  launch();
  HIPCHK(hipEventRecord(e1, c->stream));
  c->prof_events.push_back({e0, e1});
  c->prof_flops.push_back(flops);
  c->prof_prec.push_back(c->sigma_prec);
}

double gemm_flops(const GemmArgs& g) { return 8.0 * (double)g.M * (double)g.N * (double)g.K * (double)g.batch; }
}  // namespace

namespace {
// every term of the right transform except the ring and the two ladders
void right_terms(cclr_ctx* c, const VecSet& in, SigmaAcc& a) {
  const i64 o = c->o, v = c->v, nv = in.n;
  const cplx one = cx(1.0), mone = cx(-1.0);
  Ten Foo = ten(c->Foo, {o, o}), Fvv = ten(c->Fvv, {v, v}), Fov = ten(c->Fov, {o, v});
  Ten Wooov = ten(c->Wooov, {o, o, o, v}), Wvovv = ten(c->Wvovv, {v, o, v, v});
  Ten WR = ten(c->WR, {o, v, o, v});
  // singles
  contract(c, one, Fvv, "ae", a.R1, "kie", a.S1, "kia");
  contract(c, mone, Foo, "mi", a.R1, "kma", a.S1, "kia");
  // W^ma_ei read from the ring operator WR[i][a][m][e]
  contract(c, one, WR, "iame", a.R1, "kme", a.S1, "kia");
  // r^ef_im with (i, m) unpacked and (e, f) packed, and r^ea_mn on the rows m > n: the pair
  // sums below run over each antisymmetric pair once
  const bool pairs = o >= 2 && v >= 2;
  Ten R2v, R2h;
  if (pairs) {
    R2h = tmp(c, {nv, c->O2(), v, v});
    launch_pack_first_pair(nv, (int)o, v * v, a.R2.p, R2h.p, c->stream);
    R2v = tmp(c, {nv, o, o, c->V2()});
    launch_unpack_first_pair(nv, (int)o, c->V2(), in.d, R2v.p, c->stream);
    // 1/2 W^am_ef r^ef_im - F^m_e r^ea_im = sum_(m, e>f) (W + X)^am_ef r^ef_im (X folded into WvovvP)
    contract(c, one, ten(c->WvovvP, {v, o, c->V2()}), "amQ", R2v, "kimQ", a.S1, "kia");
  } else {
    contract(c, mone, Fov, "me", a.R2, "kimea", a.S1, "kia");
  }
  // 1/2 W^mn_ie r^ea_mn = sum_(m>n, e) W^mn_ie r^ea_mn
  if (pairs) contract(c, one, ten(c->WooovH, {c->O2(), o, v}), "Pie", R2h, "kPea", a.S1, "kia");
  // doubles (the P(ij) group Xi holds the pairs a > b only: [k][i][j][AB])
  const i64 O2 = c->O2();
  if (O2 > 0) contract(c, mone, ten(c->WovooH, {o, v, O2}), "mbP", a.R1, "kma", a.Xa, "kPab");
  if (pairs) contract(c, one, ten(c->WvvvoTP, {o, v, c->V2()}), "jeQ", a.R1, "kie", a.Xi, "kijQ");
  {
    // P(ab) [W^bm_fe r^e_m t^af_ij - 1/2 V^nm_fe r^ea_mn t^fb_ij] = P(ab) t^af_ij Y_bf with
    // Y_bf = W^bm_fe r^e_m - 1/2 V^nm_fe r^eb_mn, and likewise
    // -P(ij) [W^nm_je r^e_m t^ab_in + 1/2 V^nm_fe r^fe_im t^ba_jn] = -P(ij) t^ab_in Z_nj with
    // Z_nj = W^nm_je r^e_m + 1/2 V^nm_fe r^fe_jm  (antisymmetry of t relabels the second terms)
    Ten Y = tmp(c, {nv, v, v});
    // antisymmetry relabellings W^bm_fe = -W^bm_ef, V^nm_fe = V^mn_ef keep the reductions unit-stride
    contract(c, mone, Wvovv, "bmef", a.R1, "kme", Y, "kbf", false);
    // -1/2 V^mn_ef r^eb_mn = -sum_(m>n, e) V^mn_ef r^eb_mn on the (m>n) rows of r
    if (pairs) contract(c, mone, ten(c->VoovvH, {c->O2(), v, v}), "Pef", R2h, "kPeb", Y, "kbf");
    if (O2 > 0) contract(c, one, ten(c->t2H, {O2, v, v}), "Paf", Y, "kbf", a.Xa, "kPab");
    Ten Z = tmp(c, {nv, o, o});
    contract(c, one, Wooov, "nmje", a.R1, "kme", Z, "knj", false);
    // 1/2 V^nm_fe r^fe_jm = sum_(m, f>e) V^nm_fe r^fe_jm
    if (pairs) contract(c, one, ten(c->VoovvP, {o, o, c->V2()}), "nmQ", R2v, "kjmQ", Z, "knj");
    if (pairs) contract(c, mone, ten(c->t2P, {o, o, c->V2()}), "inQ", Z, "knj", a.Xi, "kijQ");
  }
}

// exchanges the context's stream with its side stream for the lifetime of the
// object; the arena keeps what the side-stream work takes until the join
struct SideStream {
  cclr_ctx* c;
  explicit SideStream(cclr_ctx* cc) : c(cc) {
    std::swap(c->stream, c->side);
    ++c->arena.hold;
  }
  ~SideStream() {
    --c->arena.hold;
    std::swap(c->stream, c->side);
  }
};
}  // namespace

SigmaWork sigma_right_begin(cclr_ctx* c, const VecSet& in, const VecSet& out) {
  SigmaWork w;
  w.mk = c->arena.mark();
  w.a = prepare(c, in, c->o >= 2 && c->v >= 2);
  right_terms(c, in, w.a);
  w.ring = ring_args(c, in, w.a.Xai, true);
  w.ladder = ladder_args(c, in, out, true);
  return w;
}

void sigma_finish(cclr_ctx* c, SigmaWork& w, const VecSet& in, const VecSet& out, const cplx* z) {
  const i64 o = c->o, v = c->v, nv = in.n;
  hole_ladder(c, in, out, true);
  launch_fill(out.s, nv * o * v, cx(0.0), c->stream);
  launch_pack_sigma((int)nv, (int)o, (int)v, w.a.X0.p, w.a.Xa.p, w.a.Xi.p, w.a.Xai.p, w.a.S1.p, out.s, out.d, z, in.s,
                    in.d, c->stream, true, true, o >= 2 && v >= 2);
  c->arena.reset(w.mk);
}

void sigma_right(cclr_ctx* c, const VecSet& in, const VecSet& out, const cplx* z) {
  if (!(c->overlap && c->sigma_prec == CCLR_FP64)) {
    SigmaWork w = sigma_right_begin(c, in, out);
    op_gemm(c, w.ring, 2);
    timed(c, gemm_flops(w.ladder), [&]() { op_gemm(c, w.ladder, 0); });
    sigma_finish(c, w, in, out, z);
    return;
  }
  // the ring and ladder products on the side stream, the other terms on the
  // context's stream meanwhile; their buffers are taken from the arena before
  // the other terms take theirs, and none is released before the join
  if (!c->side) {
    HIPCHK(hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming));
  }
  SigmaWork w;
  w.mk = c->arena.mark();
  w.a = prepare(c, in, c->o >= 2 && c->v >= 2);
  HIPCHK(hipEventRecord(c->ev_fork, c->stream));
  HIPCHK(hipStreamWaitEvent(c->side, c->ev_fork, 0));
  {
    SideStream on_side(c);
    w.ring = ring_args(c, in, w.a.Xai, true);
    op_gemm(c, w.ring, 2);
    w.ladder = ladder_args(c, in, out, true);
    timed(c, gemm_flops(w.ladder), [&]() { op_gemm(c, w.ladder, 0); });
    HIPCHK(hipEventRecord(c->ev_join, c->stream));
  }
  right_terms(c, in, w.a);
  HIPCHK(hipStreamWaitEvent(c->stream, c->ev_join, 0));
  sigma_finish(c, w, in, out, z);
}

void sigma_left(cclr_ctx* c, const VecSet& in, const VecSet& out, const cplx* z) {
  const i64 o = c->o, v = c->v, nv = in.n;
  Arena::Mark mk = c->arena.mark();
  const cplx one = cx(1.0), mone = cx(-1.0);
  SigmaAcc a = prepare(c, in, false);
  // l^ef_im with (e, f) packed and l^ea_mn on the rows m > n, as in the right transform
  const bool pairs = o >= 2 && v >= 2;
  Ten R2v, R2h;
  if (pairs) {
    R2v = tmp(c, {nv, o, o, c->V2()});
    launch_unpack_first_pair(nv, (int)o, c->V2(), in.d, R2v.p, c->stream);
    R2h = tmp(c, {nv, c->O2(), v, v});
    launch_pack_first_pair(nv, (int)o, v * v, a.R2.p, R2h.p, c->stream);
  }
  Ten Foo = ten(c->Foo, {o, o}), Fvv = ten(c->Fvv, {v, v}), Fov = ten(c->Fov, {o, v});
  Ten Wooov = ten(c->Wooov, {o, o, o, v}), Wvovv = ten(c->Wvovv, {v, o, v, v});
  Ten Voovv = Vblk(c, "oovv");
  Ten WL = ten(c->WL, {o, v, o, v});
  // G^e_a = -1/2 l^mn_af t^ef_mn ; G^i_m = 1/2 l^in_ef t^ef_mn  (SI, eqs. G_ea, G_mi)
  Ten Gvv = tmp(c, {nv, v, v}), Goo = tmp(c, {nv, o, o});
  // over the pairs once: -sum_(m>n, f) l^fa_mn t^fe_mn and sum_(n, e>f) l^ef_in t^ef_mn
  if (pairs) {
    contract(c, mone, R2h, "kPfa", ten(c->t2H, {c->O2(), v, v}), "Pfe", Gvv, "kea", false);
    contract(c, one, R2v, "kinQ", ten(c->t2P, {o, o, c->V2()}), "mnQ", Goo, "kim", false);
  } else {
    launch_fill(Gvv.p, Gvv.size(), cx(0.0), c->stream);
    launch_fill(Goo.p, Goo.size(), cx(0.0), c->stream);
  }
  // singles
  contract(c, one, a.R1, "kie", Fvv, "ea", a.S1, "kia");
  contract(c, mone, a.R1, "kma", Foo, "im", a.S1, "kia");
  if (pairs) {
    // 1/2 l^im_ef W^ef_am over e > f; 1/2 l^mn_ae W^ie_mn = 1/2 l^ea_mn W^ie_mn over m > n
    contract(c, one, R2v, "kimQ", ten(c->WvvvoLP, {v, o, c->V2()}), "amQ", a.S1, "kia");
    contract(c, one, R2h, "kPea", ten(c->WovooH, {o, v, c->O2()}), "ieP", a.S1, "kia");
  }
  contract(c, mone, Gvv, "kfe", ten(c->WvovvL, {o, v, v, v}), "iafe", a.S1, "kia");  // W^ei_fa as [i][a][f][e]
  contract(c, mone, Goo, "knm", Wooov, "mina", a.S1, "kia");
  contract(c, one, a.R1, "kme", WL, "meia", a.S1, "kia");  // W^ie_am = WL[m][e][i][a]
  // doubles
  op_gemm(c, ring_args(c, in, a.Xai, false), 3);
  if (c->O2() > 0) {
    contract(c, one, ten(c->VoovvH, {c->O2(), v, v}), "Pae", Gvv, "keb", a.Xa, "kPab");
    contract(c, mone, a.R1, "kma", ten(c->WooovH, {c->O2(), o, v}), "Pmb", a.Xa, "kPab");
  }
  contract(c, mone, Voovv, "imab", Goo, "kjm", a.Xi, "kijab");
  contract(c, one, a.R1, "kie", Wvovv, "ejab", a.Xi, "kijab");
  contract(c, one, a.R1, "kia", Fov, "jb", a.Xai, "kijab");
  {
    const GemmArgs g = ladder_args(c, in, out, false);
    timed(c, gemm_flops(g), [&]() { op_gemm(c, g, 1); });
  }
  hole_ladder(c, in, out, false);
  launch_fill(out.s, nv * o * v, cx(0.0), c->stream);
  launch_pack_sigma((int)nv, (int)o, (int)v, a.X0.p, a.Xa.p, a.Xi.p, a.Xai.p, a.S1.p, out.s, out.d, z, in.s, in.d,
                    c->stream, true, true);
  c->arena.reset(mk);
}
