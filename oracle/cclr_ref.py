"""Plain FP64 CPU oracle of CCSD linear response (TEST INFRASTRUCTURE ONLY).

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this module.  It shares no code with the GPU library.

What it computes (arXiv:2307.14296, "Formulation and Implementation of
Frequency-Dependent Linear Response Properties with Relativistic Coupled
Cluster Theory for GPU-accelerated Computer Architectures"):

* the property-independent Hbar intermediates (SI, "EOM-EE sigma-vectors and
  intermediates", eqs. F_im ... tau),
* right and left EOM-EE sigma vectors (SI, eqs. sigma_sin-ee, sigma_double-ee,
  sigma_sin-ee-left, sigma_double-ee-left),
* xi^X, eta^X and the Hessian product t^X F (SI, "Linear response"),
* eta^0 and the Lambda equation t0bar A = -eta (theory section, eq. Lambda),
* damped response solutions (A - (w + i g)) t^Y = -xi^Y (eq. LR response
  equation_cpp) by dense LU or by GMRES,
* the symmetric CC-CC response function (eq. CC-CC response function, with
  the permutation P and the conjugation symmetrizer C^{+-w}), and the CC-CI
  (EOM-CC) response function (eq. CC-CI response function, EOM eta vector),
  and the asymmetric CC-CC form with multiplier responses (eq. asymmetric
  form of the response function),
* the CCSD ground state that feeds all of the above (implementation section,
  first step): the residual Omega(t), the correlation energy, the CROP
  solver that section names, and the integral blocks formed from Cholesky
  vectors (computational details).

Conventions.  Indices i,j,k,l,m,n,o are occupied, a..g virtual; sums are
unrestricted (Einstein).  Arrays: t1[i,a] = t^a_i, t2[i,j,a,b] = t^ab_ij,
left vectors l1[i,a] = l^i_a, l2[i,j,a,b] = l^ij_ab; X[p,q] = <p|X|q>;
V[p,q,r,s] = <pq||rs> = V^pq_rs; one-body Hbar blocks F[p,q] = F^p_q (bra p,
ket q); two-body blocks W[p,q,r,s] = W^pq_rs (bra pq, ket rs).  The
excitation-space inner product sums over unique excitations:
<x, y> = sum_ia x1 y1 + 1/4 sum_ijab x2 y2 (bilinear).

Readings of the printed equations are listed where they are applied
("reading:" comments); each was decided by the formula-free second-
quantization pins in the test suite.
"""
from __future__ import annotations

import numpy as np

einsum = lambda *a: np.einsum(*a, optimize=True)  # noqa: E731


# ---------------------------------------------------------------- integrals
class Hamiltonian:
    """f (n x n) and the six canonical blocks of <pq||rs> (oooo, ooov, oovv,
    ovov, ovvv, vvvv).  Any other block follows from <pq||rs> = -<qp||rs> =
    -<pq||sr> = conj(<rs||pq>)."""

    _order = {"oo": 0, "ov": 1, "vv": 2}

    def __init__(self, o, v, f, blocks):
        self.o, self.v = o, v
        self.f = np.asarray(f, dtype=np.complex128)
        self.blocks = {k: np.asarray(b, dtype=np.complex128) for k, b in blocks.items()}
        self._cache = {}

    def fb(self, kinds):
        o = self.o
        sl = {"o": slice(0, o), "v": slice(o, None)}
        return self.f[sl[kinds[0]], sl[kinds[1]]]

    def V(self, kinds):
        if kinds in self._cache:
            return self._cache[kinds]
        bra, ket = kinds[:2], kinds[2:]
        sign = 1.0
        perm = [0, 1, 2, 3]
        if bra == "vo":
            bra, sign, perm = "ov", -sign, [perm[1], perm[0], perm[2], perm[3]]
        if ket == "vo":
            ket, sign, perm = "ov", -sign, [perm[0], perm[1], perm[3], perm[2]]
        if self._order[bra] <= self._order[ket]:
            base = self.blocks[bra + ket]
        else:
            base = self.blocks[ket + bra].conj().transpose(2, 3, 0, 1)
        # base has kinds (bra, ket) in canonical order; undo the swaps
        inv = np.argsort(perm)
        out = sign * base.transpose(inv)
        self._cache[kinds] = out
        return out


def Pij(x):
    """P_-(ij) on the first two axes: f(ij) - f(ji)."""
    return x - x.swapaxes(0, 1)


def Pab(x):
    """P_-(ab) on the last two axes."""
    return x - x.swapaxes(2, 3)


def tau(t1, t2):
    """tau^ab_ij = t^ab_ij + 1/2 P(ab) P(ij) t^a_i t^b_j  (SI, eq. tau)."""
    x = einsum("ia,jb->ijab", t1, t1)
    return t2 + 0.5 * Pij(Pab(x))


# ------------------------------------------------------------ intermediates
def hbar(H: Hamiltonian, t1, t2):
    """Hbar one- and two-body blocks (SI, eqs. F_im, F_ea, F_me, W_ijmn,
    W_mbej, W_iemn, W_efam, W_efab, barW_mbej, W_mnie, W_amef)."""
    V, f = H.V, H.fb
    tt = tau(t1, t2)
    hb = {}
    # F^i_m (eq. F_im)
    hb["Foo"] = (f("oo") + einsum("ie,me->im", f("ov"), t1) + einsum("inme,ne->im", V("ooov"), t1)
                 + 0.5 * einsum("inef,mnef->im", V("oovv"), tt))
    # F^a_e (eq. F_ea).  reading: Hbar element with bra a, ket e; the printed
    # t-dependent terms carry the transposed pair (e,a), the standard element
    # is  f^a_e - f^m_e t^a_m + V^am_ef t^f_m - 1/2 V^mn_ef tau^af_mn.
    hb["Fvv"] = (f("vv") - einsum("me,ma->ae", f("ov"), t1) + einsum("amef,mf->ae", V("vovv"), t1)
                 - 0.5 * einsum("mnef,mnaf->ae", V("oovv"), tt))
    # F^m_e (eq. F_me)
    hb["Fov"] = f("ov") + einsum("mnef,nf->me", V("oovv"), t1)
    # W^ij_mn (eq. W_ijmn)
    w = einsum("ijen,me->ijmn", V("oovo"), t1)
    hb["Woooo"] = V("oooo") + Pab(w) + 0.5 * einsum("ijef,mnef->ijmn", V("oovv"), tt)
    # W^mb_ej (eq. W_mbej)
    hb["Wovvo"] = (V("ovvo") + einsum("mbef,jf->mbej", V("ovvv"), t1) - einsum("mnej,nb->mbej", V("oovo"), t1)
                   - einsum("mnef,jnfb->mbej", V("oovv"), t2 + einsum("jf,nb->jnfb", t1, t1)))
    # barW^mb_ej (eq. barW_mbej)
    Wbar = V("ovvo") - einsum("mnef,njbf->mbej", V("oovv"), t2)
    hb["Wbar"] = Wbar
    # W^mn_ie (eq. W_mnie)
    hb["Wooov"] = V("ooov") + einsum("if,mnfe->mnie", t1, V("oovv"))
    # W^am_ef (eq. W_amef)
    hb["Wvovv"] = V("vovv") - einsum("nmef,na->amef", V("oovv"), t1)
    # W^ef_ab (eq. W_efab)
    w = einsum("mfab,me->efab", V("ovvv"), t1)
    hb["Wvvvv"] = V("vvvv") - (w - w.swapaxes(0, 1)) + 0.5 * einsum("mnab,mnef->efab", V("oovv"), tt)
    # W^ie_mn (eq. W_iemn).  reading: the F^i_f t^ef_mn term enters with a
    # minus sign (equivalently t^fe_mn).
    w1 = einsum("iefn,mf->iemn", Wbar, t1)
    w2 = einsum("iomf,noef->iemn", V("ooov"), t2)
    hb["Wovoo"] = (V("ovoo") - einsum("if,mnef->iemn", hb["Fov"], t2)
                   - einsum("iomn,oe->iemn", hb["Woooo"], t1)
                   + 0.5 * einsum("iefg,mnfg->iemn", V("ovvv"), tt) + Pab(w1) + Pab(w2))
    # W^ef_am (eq. W_efam).  reading: the P(ef) V^en_ag t^gf_mn term enters
    # with a minus sign (equivalently t^fg_mn).
    w1 = -einsum("enag,mngf->efam", V("vovv"), t2)
    w2 = einsum("nfam,ne->efam", Wbar, t1)
    hb["Wvvvo"] = (V("vvvo") + (w1 - w1.swapaxes(0, 1)) + einsum("efag,mg->efam", hb["Wvvvv"], t1)
                   + einsum("na,mnef->efam", hb["Fov"], t2) + 0.5 * einsum("noam,noef->efam", V("oovo"), tt)
                   - (w2 - w2.swapaxes(0, 1)))
    return hb


# ------------------------------------------------------------ sigma vectors
def sigma_right(H: Hamiltonian, hb, t1, t2, r1, r2):
    """(A r): right EOM-EE sigma vector (SI, eqs. sigma_sin-ee, sigma_double-ee)."""
    V = H.V
    F_vv, F_oo, F_ov = hb["Fvv"], hb["Foo"], hb["Fov"]
    s1 = (einsum("ae,ie->ia", F_vv, r1) - einsum("mi,ma->ia", F_oo, r1) + einsum("me,miea->ia", F_ov, r2)
          # reading: the ring element is W^ma_ei (printed with bra and ket exchanged)
          + einsum("maei,me->ia", hb["Wovvo"], r1)
          + 0.5 * einsum("amef,imef->ia", hb["Wvovv"], r2)
          + 0.5 * einsum("mnie,mnea->ia", hb["Wooov"], r2))
    s2 = -Pab(einsum("mbij,ma->ijab", hb["Wovoo"], r1))
    s2 = s2 + Pij(einsum("abej,ie->ijab", hb["Wvvvo"], r1))
    s2 = s2 + Pab(einsum("bmfe,me,ijaf->ijab", hb["Wvovv"], r1, t2))
    s2 = s2 - Pij(einsum("nmje,me,inab->ijab", hb["Wooov"], r1, t2))
    s2 = s2 + Pab(einsum("be,ijae->ijab", F_vv, r2))
    s2 = s2 - Pij(einsum("mj,imab->ijab", F_oo, r2))
    s2 = s2 + 0.5 * einsum("mnij,mnab->ijab", hb["Woooo"], r2)
    s2 = s2 + Pab(Pij(einsum("mbej,imae->ijab", hb["Wovvo"], r2)))
    s2 = s2 - 0.5 * Pab(einsum("nmfe,mnea,ijfb->ijab", V("oovv"), r2, t2))
    s2 = s2 - 0.5 * Pij(einsum("nmfe,imfe,jnba->ijab", V("oovv"), r2, t2))
    s2 = s2 + 0.5 * einsum("abef,ijef->ijab", hb["Wvvvv"], r2)
    return s1, s2


def G_intermediates(t2, l2):
    """G^e_a = -1/2 l^mn_af t^ef_mn ; G^i_m = 1/2 l^in_ef t^ef_mn  (SI, eqs. G_ea, G_mi)."""
    Gvv = -0.5 * einsum("mnaf,mnef->ea", l2, t2)
    Goo = 0.5 * einsum("inef,mnef->im", l2, t2)
    return Gvv, Goo


def sigma_left(H: Hamiltonian, hb, t1, t2, l1, l2):
    """(l A): left EOM-EE sigma vector (SI, eqs. sigma_sin-ee-left, sigma_double-ee-left)."""
    V = H.V
    F_vv, F_oo, F_ov = hb["Fvv"], hb["Foo"], hb["Fov"]
    Gvv, Goo = G_intermediates(t2, l2)
    s1 = (einsum("ie,ea->ia", l1, F_vv) - einsum("ma,im->ia", l1, F_oo)
          + 0.5 * einsum("imef,efam->ia", l2, hb["Wvvvo"])
          - 0.5 * einsum("mnae,iemn->ia", l2, hb["Wovoo"])
          - einsum("fe,eifa->ia", Gvv, hb["Wvovv"])
          - einsum("nm,mina->ia", Goo, hb["Wooov"])
          + einsum("me,ieam->ia", l1, hb["Wovvo"]))
    s2 = Pab(einsum("ijae,eb->ijab", l2, F_vv))
    s2 = s2 - Pij(einsum("imab,jm->ijab", l2, F_oo))
    s2 = s2 + 0.5 * einsum("mnab,ijmn->ijab", l2, hb["Woooo"])
    s2 = s2 + Pij(Pab(einsum("imae,jebm->ijab", l2, hb["Wovvo"])))
    s2 = s2 + Pab(einsum("ijae,eb->ijab", V("oovv"), Gvv))
    # reading: the l^m_a W^ij_mb term carries P(ab)
    s2 = s2 - Pab(einsum("ma,ijmb->ijab", l1, hb["Wooov"]))
    s2 = s2 - Pij(einsum("imab,jm->ijab", V("oovv"), Goo))
    # reading: the l^i_e term contracts the Hbar element W^ej_ab
    s2 = s2 + Pij(einsum("ie,ejab->ijab", l1, hb["Wvovv"]))
    s2 = s2 + Pij(Pab(einsum("ia,jb->ijab", l1, F_ov)))
    # reading: the last term is 1/2 l^ij_ef W^ef_ab (printed with W^ef_am)
    s2 = s2 + 0.5 * einsum("ijef,efab->ijab", l2, hb["Wvvvv"])
    return s1, s2


# ------------------------------------------------- property vectors, Hessian
def xi(H: Hamiltonian, X, t1, t2):
    """xi^X_mu = <mu-bar|X|CC>  (SI, eq. xi-equation and its programmable form)."""
    o = H.o
    Xoo, Xov, Xvo, Xvv = X[:o, :o], X[:o, o:], X[o:, :o], X[o:, o:]
    x1 = (Xvo.T + einsum("ae,ie->ia", Xvv, t1) - einsum("mi,ma->ia", Xoo, t1)
          - einsum("me,ie,ma->ia", Xov, t1, t1) + einsum("me,imae->ia", Xov, t2))
    x2 = (Pab(einsum("bf,ijaf->ijab", Xvv, t2)) - Pij(einsum("mj,imab->ijab", Xoo, t2))
          - Pij(einsum("me,ie,mjab->ijab", Xov, t1, t2)) - Pab(einsum("mf,ma,ijfb->ijab", Xov, t1, t2)))
    return x1, x2


def eta(H: Hamiltonian, X, t1, t2, lam1, lam2):
    """eta^X_mu = <Lambda|[X, tau_mu]|CC>  (SI, eq. eta-equation, programmable form)."""
    o = H.o
    Xoo, Xov, Xvv = X[:o, :o], X[:o, o:], X[o:, o:]
    e1 = (Xov + einsum("ea,ie->ia", Xvv, lam1) - einsum("im,ma->ia", Xoo, lam1)
          - einsum("ma,me,ie->ia", Xov, t1, lam1) - einsum("ie,me,ma->ia", Xov, t1, lam1)
          - 0.5 * einsum("mnfe,mife,na->ia", t2, lam2, Xov)
          - 0.5 * einsum("nmfe,nmfa,ie->ia", t2, lam2, Xov))
    e2 = (Pij(Pab(einsum("ia,jb->ijab", lam1, Xov))) + Pab(einsum("ijae,eb->ijab", lam2, Xvv))
          - Pij(einsum("imab,jm->ijab", lam2, Xoo))
          - Pab(einsum("me,ijae,mb->ijab", t1, lam2, Xov))
          - Pij(einsum("me,imab,je->ijab", t1, lam2, Xov)))
    return e1, e2


def eom_eta(H: Hamiltonian, X, t1, t2, lam1, lam2):
    """^EOM eta^X (SI, EOM eta vector): the singles of eta^X plus
    lambda^ij_ab xi^X_jb; the doubles are those of eta^X."""
    e1, e2 = eta(H, X, t1, t2, lam1, lam2)
    x1, _ = xi(H, X, t1, t2)
    return e1 + einsum("ijab,jb->ia", lam2, x1), e2


def eta0(H: Hamiltonian, hb):
    """eta^0_mu = <R|[H, tau_mu]|CC>, the right-hand side of the Lambda
    equation (theory section, eq. Lambda; Table 1 with X -> H0 and
    <Lambda| -> <R|): singles F^i_a, doubles V^ij_ab."""
    return hb["Fov"].copy(), H.V("oovv").copy()


def tF(H: Hamiltonian, hb, t1, t2, lam1, lam2, x1, x2):
    """(t^X F)_mu, the product of a response vector with the CC Hessian
    F_mu,nu = <Lambda|[[H0, tau_mu], tau_nu]|CC>  (SI, "(t^X F)^k_c" and
    "(t^X F)^kl_cd").  Output has left-vector index placement [k,c], [k,l,c,d]."""
    V = H.V
    Vv = V("oovv")
    Fov = hb["Fov"]
    Wvovv, Wooov, Wovvo, Woooo, Wvvvv = hb["Wvovv"], hb["Wooov"], hb["Wovvo"], hb["Woooo"], hb["Wvvvv"]
    l1, l2 = lam1, lam2
    # ---- singles, projected on (k, c)
    s = einsum("kica,ia->kc", Vv, x1)
    s = s - einsum("ic,ka,ia->kc", l1, Fov, x1)
    s = s - einsum("ka,ic,ia->kc", l1, Fov, x1)
    s = s + einsum("ke,eica,ia->kc", l1, Wvovv, x1)
    s = s - einsum("mc,kima,ia->kc", l1, Wooov, x1)
    s = s - einsum("ma,ikmc,ia->kc", l1, Wooov, x1)
    s = s + einsum("ie,ekac,ia->kc", l1, Wvovv, x1)
    s = s - 0.5 * einsum("ic,kjab,ijab->kc", l1, Vv, x2)
    s = s - 0.5 * einsum("ka,ijcb,ijab->kc", l1, Vv, x2)
    s = s + einsum("ia,jkbc,ijab->kc", l1, Vv, x2)
    # W^ie_mc = -W^ie_cm and W^ek_am = -W^ke_am (antisymmetry of the Hbar element)
    s = s + einsum("mkae,iecm,ia->kc", l2, Wovvo, x1)
    s = s + einsum("imec,keam,ia->kc", l2, Wovvo, x1)
    s = s + 0.5 * einsum("kief,efca,ia->kc", l2, Wvvvv, x1)
    s = s + 0.5 * einsum("mnca,kimn,ia->kc", l2, Woooo, x1)
    s = s - 0.5 * einsum("mnec,mnef,kifa,ia->kc", l2, t2, Vv, x1)
    s = s - 0.5 * einsum("mkef,mnef,nica,ia->kc", l2, t2, Vv, x1)
    s = s - 0.5 * einsum("mnea,mnef,ikfc,ia->kc", l2, t2, Vv, x1)
    s = s - 0.5 * einsum("mief,mnef,nkac,ia->kc", l2, t2, Vv, x1)
    s = s - 0.5 * einsum("ijac,kb,ijab->kc", l2, Fov, x2)
    s = s - 0.5 * einsum("ikab,jc,ijab->kc", l2, Fov, x2)
    s = s - einsum("ikeb,ejac,ijab->kc", l2, Wvovv, x2)
    s = s + einsum("mjac,ikmb,ijab->kc", l2, Wooov, x2)
    s = s - 0.25 * einsum("ijec,ekab,ijab->kc", l2, Wvovv, x2)
    s = s + 0.25 * einsum("mkab,ijmc,ijab->kc", l2, Wooov, x2)
    s = s + 0.5 * einsum("ijae,ekbc,ijab->kc", l2, Wvovv, x2)
    s = s - 0.5 * einsum("imab,jkmc,ijab->kc", l2, Wooov, x2)
    # ---- doubles, projected on (k, l, c, d); Pij acts on (k,l), Pab on (c,d)
    d = Pab(Pij(einsum("kc,lida,ia->klcd", l1, Vv, x1)))
    d = d - Pij(einsum("ka,ilcd,ia->klcd", l1, Vv, x1))
    d = d - Pab(einsum("ic,klad,ia->klcd", l1, Vv, x1))
    d = d - Pij(einsum("kicd,la,ia->klcd", l2, Fov, x1))
    d = d - Pab(einsum("klca,id,ia->klcd", l2, Fov, x1))
    d = d + Pab(einsum("klce,eida,ia->klcd", l2, Wvovv, x1))
    d = d - Pij(einsum("kmcd,lima,ia->klcd", l2, Wooov, x1))
    d = d + Pab(Pij(einsum("mlca,kimd,ia->klcd", l2, Wooov, x1)))
    d = d + einsum("micd,klma,ia->klcd", l2, Wooov, x1)
    d = d - Pab(Pij(einsum("kied,elca,ia->klcd", l2, Wvovv, x1)))
    d = d - einsum("klea,eicd,ia->klcd", l2, Wvovv, x1)
    d = d - 0.5 * Pab(einsum("klca,ijdb,ijab->klcd", l2, Vv, x2))
    d = d - 0.5 * Pij(einsum("kicd,ljab,ijab->klcd", l2, Vv, x2))
    d = d + 0.25 * einsum("ijcd,klab,ijab->klcd", l2, Vv, x2)
    d = d + 0.25 * einsum("klab,ijcd,ijab->klcd", l2, Vv, x2)
    d = d + Pij(Pab(einsum("kjcb,lida,ijab->klcd", l2, Vv, x2)))
    d = d - 0.5 * Pij(einsum("ikab,jlcd,ijab->klcd", l2, Vv, x2))
    d = d - 0.5 * Pab(einsum("ijac,klbd,ijab->klcd", l2, Vv, x2))
    return s, d


# ------------------------------------------------------ CCSD ground state
def ccsd_residual(H: Hamiltonian, t1, t2):
    """Omega_mu = <mu|e^-T H_N e^T|R>, the CCSD amplitude equations that the
    first step of the implementation section solves for t.  The paper does not
    print them; written here in the spin-orbital intermediate form of Stanton
    and Gauss (J. Chem. Phys. 94, 4334 (1991)), with the diagonal Fock terms
    kept in F so that the result is the residual itself (not a Jacobi update),
    and every f_ov term kept (non-canonical references)."""
    V, f = H.V, H.fb
    tt = tau(t1, t2)
    ts = t2 + 0.25 * Pij(Pab(einsum("ia,jb->ijab", t1, t1)))  # tau-tilde: half the singles products
    Voovv = V("oovv")
    Fae = (f("vv") - 0.5 * einsum("me,ma->ae", f("ov"), t1) + einsum("mf,mafe->ae", t1, V("ovvv"))
           - 0.5 * einsum("mnaf,mnef->ae", ts, Voovv))
    Fmi = (f("oo") + 0.5 * einsum("ie,me->mi", t1, f("ov")) + einsum("ne,mnie->mi", t1, V("ooov"))
           + 0.5 * einsum("inef,mnef->mi", ts, Voovv))
    Fme = f("ov") + einsum("nf,mnef->me", t1, Voovv)
    # the two 1/4 tau <mn||ef> pieces (hole ladder and particle ladder) are
    # combined into the hole-ladder intermediate, giving 1/2 tau there
    w = einsum("je,mnie->mnij", t1, V("ooov"))
    Wmnij = V("oooo") + (w - w.swapaxes(2, 3)) + 0.5 * einsum("ijef,mnef->mnij", tt, Voovv)
    w = einsum("mb,amef->abef", t1, V("vovv"))
    Wabef = V("vvvv") - (w - w.swapaxes(0, 1))
    Wmbej = (V("ovvo") + einsum("jf,mbef->mbej", t1, V("ovvv")) - einsum("nb,mnej->mbej", t1, V("oovo"))
             - einsum("jnfb,mnef->mbej", 0.5 * t2 + einsum("jf,nb->jnfb", t1, t1), Voovv))
    o1 = (f("vo").T + einsum("ie,ae->ia", t1, Fae) - einsum("ma,mi->ia", t1, Fmi)
          + einsum("imae,me->ia", t2, Fme) - einsum("nf,naif->ia", t1, V("ovov"))
          - 0.5 * einsum("imef,maef->ia", t2, V("ovvv")) - 0.5 * einsum("mnae,nmei->ia", t2, V("oovo")))
    Fbe = Fae - 0.5 * einsum("mb,me->be", t1, Fme)
    Fmj = Fmi + 0.5 * einsum("je,me->mj", t1, Fme)
    o2 = V("vvoo").transpose(2, 3, 0, 1).copy()
    o2 = o2 + Pab(einsum("ijae,be->ijab", t2, Fbe)) - Pij(einsum("imab,mj->ijab", t2, Fmj))
    o2 = o2 + 0.5 * einsum("mnab,mnij->ijab", tt, Wmnij) + 0.5 * einsum("ijef,abef->ijab", tt, Wabef)
    o2 = o2 + Pij(Pab(einsum("imae,mbej->ijab", t2, Wmbej) - einsum("ie,ma,mbej->ijab", t1, t1, V("ovvo"))))
    o2 = o2 + Pij(einsum("ie,abej->ijab", t1, V("vvvo"))) - Pab(einsum("ma,mbij->ijab", t1, V("ovoo")))
    return o1, o2


def ccsd_energy(H: Hamiltonian, t1, t2):
    """Correlation energy <R|e^-T H_N e^T|R> = f_ia t^a_i + 1/4 <ij||ab> tau^ab_ij."""
    return np.sum(H.fb("ov") * t1) + 0.25 * np.sum(H.V("oovv") * tau(t1, t2))


def solve_ccsd(H: Hamiltonian, t1, t2, tol=1e-10, maxiter=200, nsub=3):
    """CCSD amplitudes from the start (t1, t2) by CROP, the solver the
    implementation section names for the ground state (conjugate residual
    with optimal trial vectors; Ziolkowski et al., J. Chem. Phys. 128, 204105
    (2008); Ettenhuber and Jorgensen, J. Chem. Theory Comput. 11, 1518 (2015)).

    Each iteration takes a Jacobi step from the current optimal vector with
    the Fock diagonal (x~ = x - Omega/D), evaluates the true residual there,
    and forms the next optimal vector as the affine combination (coefficients
    summing to one) of the kept optimal vectors and x~ that minimizes the
    norm of the same combination of their residuals.  At most nsub vectors
    take part (nsub - 1 optimal ones and the new one).  Stops when the true
    residual's 2-norm over unique amplitudes is <= tol; returns (t1, t2,
    energy, iterations)."""
    o, v = H.o, H.v
    fo, fv = np.diag(H.fb("oo")), np.diag(H.fb("vv"))
    D = pack(fv[None, :] - fo[:, None],
             fv[None, None, :, None] + fv[None, None, None, :] - fo[:, None, None, None] - fo[None, :, None, None])
    x = pack(t1, t2)
    r = pack(*ccsd_residual(H, t1, t2))
    if np.linalg.norm(r) <= tol:
        return t1, t2, ccsd_energy(H, t1, t2), 0
    X, R = [x], [r]
    for it in range(1, maxiter + 1):
        xt = X[-1] - R[-1] / D
        rt = pack(*ccsd_residual(H, *unpack(xt, o, v)))
        if np.linalg.norm(rt) <= tol:
            u1, u2 = unpack(xt, o, v)
            return u1, u2, ccsd_energy(H, u1, u2), it
        Xs, Rs = X[-(nsub - 1):] + [xt], R[-(nsub - 1):] + [rt]
        m = len(Rs)
        B = np.zeros((m + 1, m + 1), dtype=np.complex128)
        for a in range(m):
            for b in range(m):
                B[a, b] = np.vdot(Rs[a], Rs[b])
        B[m, :m] = B[:m, m] = 1.0
        rhs = np.zeros(m + 1, dtype=np.complex128)
        rhs[m] = 1.0
        c = np.linalg.solve(B, rhs)[:m]
        X.append(sum(ci * xi for ci, xi in zip(c, Xs)))
        R.append(sum(ci * ri for ci, ri in zip(c, Rs)))
        X, R = X[-(nsub - 1):], R[-(nsub - 1):]
    raise RuntimeError("CROP did not converge")


# ------------------------------------------------------ Cholesky integrals
def integrals_from_cholesky(o, L):
    """The six canonical <pq||rs> blocks from Cholesky vectors (the paper forms
    every integral class from them; section "Computational details").  L[P]
    are n x n Hermitian with Mulliken integrals (pq|rs) = sum_P L[P,p,q] L[P,r,s];
    <pq|rs> = (pr|qs), so <pq||rs> = sum_P (L[P,p,r] L[P,q,s] - L[P,p,s] L[P,q,r])."""
    L = np.asarray(L, dtype=np.complex128)
    sl = {"o": slice(0, o), "v": slice(o, None)}
    out = {}
    for kinds in ("oooo", "ooov", "oovv", "ovov", "ovvv", "vvvv"):
        p, q, r, s_ = (sl[k] for k in kinds)
        out[kinds] = (einsum("Ppr,Pqs->pqrs", L[:, p, r], L[:, q, s_])
                      - einsum("Pps,Pqr->pqrs", L[:, p, s_], L[:, q, r]))
    return out


# ------------------------------------------------------ excitation vectors
def dot(x, y):
    """Bilinear sum over unique excitations: sum x1 y1 + 1/4 sum x2 y2."""
    return np.sum(x[0] * y[0]) + 0.25 * np.sum(x[1] * y[1])


def pack(x1, x2):
    """Unique amplitudes: singles (i,a) then doubles i>j, a>b, row-major."""
    o, v = x1.shape
    ii, jj = np.tril_indices(o, -1)
    aa, bb = np.tril_indices(v, -1)
    d = x2[ii[:, None], jj[:, None], aa[None, :], bb[None, :]]
    return np.concatenate([x1.ravel(), d.ravel()])


def unpack(vec, o, v):
    ii, jj = np.tril_indices(o, -1)
    aa, bb = np.tril_indices(v, -1)
    x1 = vec[: o * v].reshape(o, v).copy()
    d = vec[o * v:].reshape(len(ii), len(aa))
    x2 = np.zeros((o, o, v, v), dtype=np.complex128)
    I, A = ii[:, None], aa[None, :]
    J, B = jj[:, None], bb[None, :]
    x2[I, J, A, B] = d
    x2[J, I, A, B] = -d
    x2[I, J, B, A] = -d
    x2[J, I, B, A] = d
    return x1, x2


# ------------------------------------------------------------ linear solves
class CCLR:
    """A CC linear-response problem: Hamiltonian, amplitudes, intermediates."""

    def __init__(self, H: Hamiltonian, t1, t2):
        self.H, self.t1, self.t2 = H, np.asarray(t1), np.asarray(t2)
        self.o, self.v = H.o, H.v
        self.hb = hbar(H, self.t1, self.t2)
        self.lam = None

    @property
    def dim(self):
        o, v = self.o, self.v
        return o * v + (o * (o - 1) // 2) * (v * (v - 1) // 2)

    def right(self, x1, x2, z=0.0):
        s1, s2 = sigma_right(self.H, self.hb, self.t1, self.t2, x1, x2)
        return s1 - z * x1, s2 - z * x2

    def left(self, x1, x2, z=0.0):
        s1, s2 = sigma_left(self.H, self.hb, self.t1, self.t2, x1, x2)
        return s1 - z * x1, s2 - z * x2

    def diagonal(self):
        """Fock-like diagonal used only to precondition GMRES."""
        fo = np.diag(self.hb["Foo"])
        fv = np.diag(self.hb["Fvv"])
        d1 = fv[None, :] - fo[:, None]
        d2 = fv[None, None, :, None] + fv[None, None, None, :] - fo[:, None, None, None] - fo[None, :, None, None]
        return pack(d1, d2)

    def matrix(self, side="right"):
        """Dense matrix of the right (A) or left (x -> xA) map on unique amplitudes."""
        n = self.dim
        M = np.empty((n, n), dtype=np.complex128)
        e = np.zeros(n, dtype=np.complex128)
        fn = self.right if side == "right" else self.left
        for k in range(n):
            e[k] = 1.0
            M[:, k] = pack(*fn(*unpack(e, self.o, self.v)))
            e[k] = 0.0
        return M

    def solve(self, side, rhs, z, method="dense", tol=1e-12, maxiter=2000):
        """RIGHT: (A - z) x = -rhs ;  LEFT: x (A - z) = -rhs.  Vectors as (x1, x2)."""
        b = -pack(*rhs)
        o, v = self.o, self.v
        if method == "dense":
            if not hasattr(self, "_dense"):
                self._dense = {}
            if side not in self._dense:
                self._dense[side] = self.matrix(side)
            M = self._dense[side] - z * np.eye(self.dim)
            return unpack(np.linalg.solve(M, b), o, v)
        import scipy.sparse.linalg as spla
        fn = self.right if side == "right" else self.left
        op = spla.LinearOperator((self.dim, self.dim), dtype=np.complex128,
                                 matvec=lambda x: pack(*fn(*unpack(x, o, v), z)))
        pre = 1.0 / (self.diagonal() - z)
        M = spla.LinearOperator((self.dim, self.dim), dtype=np.complex128, matvec=lambda x: pre * x)
        x, info = spla.gmres(op, b, M=M, rtol=tol, atol=0.0, restart=200, maxiter=maxiter)
        if info != 0:
            raise RuntimeError(f"GMRES did not converge (info={info})")
        return unpack(x, o, v)

    def solve_lambda(self, method="dense"):
        """lambda A = -eta0  (theory section, eq. Lambda)."""
        self.lam = self.solve("left", eta0(self.H, self.hb), 0.0, method)
        return self.lam

    def xi(self, X):
        return xi(self.H, X, self.t1, self.t2)

    def eta(self, X):
        return eta(self.H, X, self.t1, self.t2, *self.lam)

    def tF(self, x):
        return tF(self.H, self.hb, self.t1, self.t2, *self.lam, *x)

    def response_asym(self, Xs, Ys, z, method="dense"):
        """Asymmetric CC-CC form (eq. asymmetric response function):
          <<X;Y>>_z = 1/2 [ a(z) + conj a(-z*) ],  a_XY(z) = eta^X t^Y(z) + tbar^Y(z) xi^X,
        with the multiplier response tbar^Y(z) (A + z) = -(eta^Y + F t^Y(z)).
        Only the Y operators need response solves (right and left)."""
        if self.lam is None:
            self.solve_lambda(method)
        z = complex(z)
        xX = [self.xi(X) for X in Xs]
        eX = [self.eta(X) for X in Xs]
        out = np.empty((len(Xs), len(Ys)), dtype=np.complex128)

        def a_of(w):
            res = np.empty((len(Xs), len(Ys)), dtype=np.complex128)
            for q, Y in enumerate(Ys):
                tY = self.solve("right", self.xi(Y), w, method)
                eY, fY = self.eta(Y), self.tF(tY)
                tb = self.solve("left", (eY[0] + fY[0], eY[1] + fY[1]), -w, method)
                for p in range(len(Xs)):
                    res[p, q] = dot(eX[p], tY) + dot(tb, xX[p])
            return res

        out[:] = 0.5 * (a_of(z) + np.conj(a_of(-z.conjugate())))
        return out

    def eom_eta(self, X):
        return eom_eta(self.H, X, self.t1, self.t2, *self.lam)

    def response_ci(self, Xs, z, method="dense"):
        """CC-CI (EOM-CC) response function (eq. CC-CI response function) with
        the same P(X,Y) and C^{+-w} readings as response():
          <<X;Y>>_z = 1/2 [ h(z) + conj h(-z*) ],
          h_XY(z) = Eeta^X t^Y(z) + Eeta^Y t^X(-z)
                    - (lambda t^X(-z)) (lambda xi^Y) - (lambda t^Y(z)) (lambda xi^X),
        Eeta the EOM eta vector, lambda . v over unique excitations."""
        if self.lam is None:
            self.solve_lambda(method)
        z = complex(z)
        freqs = {}
        for w in (z, -z, z.conjugate(), -z.conjugate()):
            freqs.setdefault(w, None)
        xis = [self.xi(X) for X in Xs]
        eetas = [self.eom_eta(X) for X in Xs]
        tX = {w: [self.solve("right", x, w, method) for x in xis] for w in freqs}
        lxi = [dot(self.lam, x) for x in xis]
        nx = len(Xs)

        def h(p, q, w):
            return (dot(eetas[p], tX[w][q]) + dot(eetas[q], tX[-w][p])
                    - dot(self.lam, tX[-w][p]) * lxi[q] - dot(self.lam, tX[w][q]) * lxi[p])

        out = np.empty((nx, nx), dtype=np.complex128)
        for p in range(nx):
            for q in range(nx):
                out[p, q] = 0.5 * (h(p, q, z) + np.conj(h(p, q, -z.conjugate())))
        return out

    def response_derivative(self, Xs, z, dXs=None, dH=None, method="dense"):
        """Exact directional derivative of response(Xs, z) along changes dXs of
        the perturbation matrices (list like Xs, or None) and dH of the
        Hamiltonian (a Hamiltonian holding the change of f and of the canonical
        integral blocks, or None), with the amplitudes t held fixed.

        At fixed t every Hamiltonian-dependent piece of the response function
        is linear in the Hamiltonian: the Hbar intermediates, the Jacobian
        A (Table 1), eta^0 and the Hessian F; xi^X and eta^X are linear in X,
        and eta^X and F are affine in lambda.  With the inverse rule
        d(M^-1) = -M^-1 dM M^-1 the changes follow exactly (no difference
        quotients):
          d lambda:  d lambda A = -(eta^0(dH) + lambda A(dH))   (eq. Lambda),
          d t^X(w):  (A - w) d t^X = -(xi(dX) + A(dH) t^X(w))   (eq. LR response equation_cpp),
          d eta^X  = eta(dX; lambda) + [eta(X; d lambda) - eta(X; 0)],
          d (F x)  = F(dH; lambda) x + [F(d lambda) - F(0)] x + F d x,
        and d<<X;Y>> = 1/2 [dg(z) + conj dg(-z*)] for the g of response().
        Returns the (nx, nx) array of d<<X_p; X_q>>_z."""
        if self.lam is None:
            self.solve_lambda(method)
        z = complex(z)
        o, v = self.o, self.v
        nx = len(Xs)
        add = lambda a, b: (a[0] + b[0], a[1] + b[1])  # noqa: E731
        sub = lambda a, b: (a[0] - b[0], a[1] - b[1])  # noqa: E731
        zero = (np.zeros((o, v), dtype=np.complex128), np.zeros((o, o, v, v), dtype=np.complex128))
        t1, t2 = self.t1, self.t2
        if dH is not None:
            dcc = CCLR(dH, t1, t2)  # Hbar of the change (linear in H at fixed t)
            dA = lambda x: sigma_right(dH, dcc.hb, t1, t2, *x)  # noqa: E731
            rhs = add(eta0(dH, dcc.hb), sigma_left(dH, dcc.hb, t1, t2, *self.lam))
            dlam = self.solve("left", rhs, 0.0, method)
        else:
            dA, dlam = None, zero
        dX = dXs if dXs is not None else [np.zeros_like(X) for X in Xs]
        freqs = {}
        for w in (z, -z, z.conjugate(), -z.conjugate()):
            freqs.setdefault(w, None)
        xis = [self.xi(X) for X in Xs]
        dxis = [self.xi(X) for X in dX]
        etas = [self.eta(X) for X in Xs]
        deta = [add(self.eta(dX[p]), sub(eta(self.H, Xs[p], t1, t2, *dlam), eta(self.H, Xs[p], t1, t2, *zero)))
                for p in range(nx)]
        tX = {w: [self.solve("right", x, w, method) for x in xis] for w in freqs}
        dtX = {}
        for w in freqs:
            dtX[w] = []
            for p in range(nx):
                r = dxis[p] if dA is None else add(dxis[p], dA(tX[w][p]))
                dtX[w].append(self.solve("right", r, w, method))
        tFx = {w: [self.tF(t) for t in tX[w]] for w in freqs}

        def dF(x, dx):
            out = self.tF(dx)
            out = add(out, sub(tF(self.H, self.hb, t1, t2, *dlam, *x), tF(self.H, self.hb, t1, t2, *zero, *x)))
            if dH is not None:
                out = add(out, tF(dH, dcc.hb, t1, t2, *self.lam, *x))
            return out

        dtFx = {w: [dF(tX[w][p], dtX[w][p]) for p in range(nx)] for w in freqs}

        def dg(p, q, w):
            return (dot(deta[p], tX[w][q]) + dot(etas[p], dtX[w][q]) + dot(deta[q], tX[-w][p])
                    + dot(etas[q], dtX[-w][p]) + dot(dtFx[-w][p], tX[w][q]) + dot(tFx[-w][p], dtX[w][q]))

        out = np.empty((nx, nx), dtype=np.complex128)
        for p in range(nx):
            for q in range(nx):
                out[p, q] = 0.5 * (dg(p, q, z) + np.conj(dg(p, q, -z.conjugate())))
        return out

    def response(self, Xs, z, method="dense"):
        """<<X_p; X_q>>_z for all pairs, z = w + i*gamma (complex).

        Symmetric CC-CC form (eq. CC-CC response function):
          <<X;Y>>_z = 1/2 [ g_XY(z) + conj g_XY(-z*) ],
          g_XY(z)   = eta^X t^Y(z) + eta^Y t^X(-z) + F t^X(-z) t^Y(z),
        where P(X,Y) produced the first two terms and the two halves of F,
        and C^{+-w} pairs z with -z* (the frequency of X is -z, reading of
        the damped frequency condition).  Every product is over unique
        excitations.
        """
        if self.lam is None:
            self.solve_lambda(method)
        z = complex(z)
        freqs = {}
        for w in (z, -z, z.conjugate(), -z.conjugate()):
            freqs.setdefault(w, None)
        xis = [self.xi(X) for X in Xs]
        etas = [self.eta(X) for X in Xs]
        tX = {w: [self.solve("right", x, w, method) for x in xis] for w in freqs}
        tFx = {w: [self.tF(t) for t in tX[w]] for w in freqs}
        nx = len(Xs)

        def g(p, q, w):
            return dot(etas[p], tX[w][q]) + dot(etas[q], tX[-w][p]) + dot(tFx[-w][p], tX[w][q])

        out = np.empty((nx, nx), dtype=np.complex128)
        for p in range(nx):
            for q in range(nx):
                out[p, q] = 0.5 * (g(p, q, z) + np.conj(g(p, q, -z.conjugate())))
        return out
