"""Pins of the CPU oracle against things other than itself.

* formula-free second quantization (Table 1 definitions, brute force in the
  determinant space) for A r, l A, xi, eta, eta0 and t^X F;
* the CCSD residual: A r equals the directional derivative of Omega(t),
  evaluated with a five-point stencil that is exact for the quartic
  polynomial Omega;
* the exact FCI sum-over-states response function for two electrons, where
  CCSD is exact (checks the Lambda solve, eta, F and the C^{+-w}/P
  symmetrizers);
* invariants: antisymmetry, the bilinear transpose identity <l, A r> = <l A, r>,
  permutation/conjugation symmetry of the response function.
All with random complex data and a non-diagonal Fock matrix, so that index
transpositions and conjugation mistakes cannot hide.
"""
import numpy as np
import pytest
import torch

import bruteforce as B
from gen import synth as s
from helpers import blocks_from_full, config_problem, rel, small_problem, vec
from oracle import cclr_ref as O

SIZES = [(2, 3), (3, 4), (4, 5)]


@pytest.fixture(scope="module", params=SIZES, ids=[f"o{o}v{v}" for o, v in SIZES])
def case(request):
    o, v = request.param
    pb, Vf, f, H, t1, t2 = small_problem(o, v)
    sp = B.Space(o, v)
    bf = B.CCBrute(sp, f, Vf)
    bf.set_t(t1, t2)
    hb = O.hbar(H, t1, t2)
    return dict(o=o, v=v, pb=pb, Vf=Vf, f=f, H=H, t1=t1, t2=t2, sp=sp, bf=bf, hb=hb)


def _cmp(sp, mine, ref, tol=1e-12):
    m = sp.pack(*mine)
    assert np.abs(m - ref).max() <= tol * max(1.0, np.abs(ref).max())


def test_right_sigma_vs_table1(case):
    r1, r2 = vec(case["pb"], 0)
    mine = O.sigma_right(case["H"], case["hb"], case["t1"], case["t2"], r1, r2)
    _cmp(case["sp"], mine, case["bf"].jacobian_right(r1, r2))


def test_right_sigma_is_derivative_of_residual(case):
    """A r = d/dh Omega(t + h r) at h = 0; Omega is a quartic polynomial in t,
    so the five-point central stencil is exact up to rounding."""
    pb, bf, sp = case["pb"], case["bf"], case["sp"]
    t1, t2 = case["t1"], case["t2"]
    r1, r2 = vec(pb, 0)
    h = 0.05
    vals = {}
    for k in (-2, -1, 1, 2):
        bf.set_t(t1 + k * h * r1, t2 + k * h * r2)
        vals[k] = bf.omega()
    bf.set_t(t1, t2)
    fd = (vals[-2] - 8 * vals[-1] + 8 * vals[1] - vals[2]) / (12 * h)
    mine = sp.pack(*O.sigma_right(case["H"], case["hb"], t1, t2, r1, r2))
    assert np.abs(mine - fd).max() <= 1e-11 * np.abs(fd).max()


def test_left_sigma_vs_table1(case):
    l1, l2 = vec(case["pb"], 1)
    A = case["bf"].jacobian_matrix()
    ref = case["sp"].pack(l1, l2) @ A
    mine = O.sigma_left(case["H"], case["hb"], case["t1"], case["t2"], l1, l2)
    _cmp(case["sp"], mine, ref)


def test_xi_vs_table1(case):
    X = s.dipole(case["pb"], 0).numpy()
    mine = O.xi(case["H"], X, case["t1"], case["t2"])
    _cmp(case["sp"], mine, case["bf"].xi(X))


def test_eta_vs_table1(case):
    X = s.dipole(case["pb"], 1).numpy()
    lam = tuple(0.3 * x for x in vec(case["pb"], 2))
    mine = O.eta(case["H"], X, case["t1"], case["t2"], *lam)
    _cmp(case["sp"], mine, case["bf"].eta(X, case["sp"].pack(*lam)))


def test_eta0_vs_lagrangian(case):
    mine = O.eta0(case["H"], case["hb"])
    _cmp(case["sp"], mine, case["bf"].eta0())


def test_hessian_product_vs_table1(case):
    lam = tuple(0.3 * x for x in vec(case["pb"], 2))
    x1, x2 = vec(case["pb"], 3)
    mine = O.tF(case["H"], case["hb"], case["t1"], case["t2"], *lam, x1, x2)
    _cmp(case["sp"], mine, case["bf"].xF(case["sp"].pack(*lam), x1, x2))


def test_hessian_is_symmetric(case):
    lam = tuple(0.3 * x for x in vec(case["pb"], 2))
    x, y = vec(case["pb"], 3), vec(case["pb"], 4)
    a = O.dot(O.tF(case["H"], case["hb"], case["t1"], case["t2"], *lam, *x), y)
    b = O.dot(O.tF(case["H"], case["hb"], case["t1"], case["t2"], *lam, *y), x)
    assert abs(a - b) <= 1e-12 * abs(a)


def test_antisymmetry_preserved(case):
    r1, r2 = vec(case["pb"], 0)
    _, s2 = O.sigma_right(case["H"], case["hb"], case["t1"], case["t2"], r1, r2)
    _, l2 = O.sigma_left(case["H"], case["hb"], case["t1"], case["t2"], r1, r2)
    for x in (s2, l2):
        sc = np.abs(x).max()
        assert np.abs(x + x.swapaxes(0, 1)).max() <= 1e-14 * sc
        assert np.abs(x + x.swapaxes(2, 3)).max() <= 1e-14 * sc


def test_transpose_identity(case):
    """<l, A r> = <l A, r> with the unique-excitation bilinear product."""
    r = vec(case["pb"], 0)
    l = vec(case["pb"], 1)
    Ar = O.sigma_right(case["H"], case["hb"], case["t1"], case["t2"], *r)
    lA = O.sigma_left(case["H"], case["hb"], case["t1"], case["t2"], *l)
    a, b = O.dot(l, Ar), O.dot(lA, r)
    assert abs(a - b) <= 1e-13 * abs(a)


def test_mutations_are_caught(case):
    """Perturbing any Hbar block by a relative 1e-6 must break a pin."""
    if case["o"] < 3:
        pytest.skip("smallest size leaves some blocks without a contributing term")
    r1, r2 = vec(case["pb"], 0)
    l1, l2 = vec(case["pb"], 1)
    refR = case["bf"].jacobian_right(r1, r2)
    refL = case["sp"].pack(l1, l2) @ case["bf"].jacobian_matrix()
    for key in case["hb"]:
        if key == "Wbar":
            continue
        hb = dict(case["hb"])
        hb[key] = hb[key] * (1 + 1e-6)
        eR = np.abs(case["sp"].pack(*O.sigma_right(case["H"], hb, case["t1"], case["t2"], r1, r2)) - refR).max()
        eL = np.abs(case["sp"].pack(*O.sigma_left(case["H"], hb, case["t1"], case["t2"], l1, l2)) - refL).max()
        assert max(eR, eL) > 1e-9, key


# ------------------------------------------------------------------ FCI limit
@pytest.fixture(scope="module")
def two_electron():
    o, v = 2, 6
    pb = s.Problem(o, v, 11)
    Vf = s.full_integrals(pb).numpy()
    f = s.fock(pb).numpy()
    H = O.Hamiltonian(o, v, f, blocks_from_full(Vf, o))
    sp = B.Space(o, v)
    bf = B.CCBrute(sp, f, Vf)
    t1 = s.t1_amplitudes(pb).numpy()
    t2 = s.t2_amplitudes(pb, torch.tensor(H.blocks["oovv"])).numpy()
    for _ in range(30):  # Newton on the brute-force residual with its exact Jacobian
        bf.set_t(t1, t2)
        om = bf.omega()
        if np.abs(om).max() < 1e-13:
            break
        d1, d2 = sp.unpack(np.linalg.solve(bf.jacobian_matrix(), -om))
        t1, t2 = t1 + d1, t2 + d2
    assert np.abs(bf.omega()).max() < 1e-12
    w = np.linalg.eigvalsh(bf.H)
    state = int(np.argmin(np.abs(w - bf.energy().real)))
    assert abs(w[state] - bf.energy()) < 1e-10      # CCSD is exact for two electrons
    Xs = [s.dipole(pb, k).numpy() for k in range(3)]
    return dict(pb=pb, H=H, t1=t1, t2=t2, sp=sp, bf=bf, state=state, Xs=Xs)


@pytest.mark.parametrize("z", [0.1 + 0.005j, 0.0, 0.37 + 0.02j, -0.2 + 0.01j])
def test_response_equals_fci_sum_over_states(two_electron, z):
    d = two_electron
    cc = O.CCLR(d["H"], d["t1"], d["t2"])
    a = cc.response(d["Xs"], z)
    ex = np.array([[B.fci_response(d["sp"], d["bf"].H, X, Y, z, d["state"]) for Y in d["Xs"]] for X in d["Xs"]])
    assert np.abs(a - ex).max() <= 1e-12 * np.abs(ex).max()


@pytest.mark.parametrize("z", [0.3 + 0.02j, 0.0, 0.45 + 0.01j])
def test_cc_ci_response_equals_fci_sum_over_states(two_electron, z):
    """Two electrons: EOM-CCSD is full CI, so the CC-CI response function
    reproduces the exact sum over states as well."""
    d = two_electron
    cc = O.CCLR(d["H"], d["t1"], d["t2"])
    a = cc.response_ci(d["Xs"], z)
    ex = np.array([[B.fci_response(d["sp"], d["bf"].H, X, Y, z, d["state"]) for Y in d["Xs"]] for X in d["Xs"]])
    assert np.abs(a - ex).max() <= 1e-11 * np.abs(ex).max()


def test_cc_ci_differs_from_cc_cc_away_from_fci():
    """At o=3 (CCSD no longer exact) the two models differ slightly, as the
    paper reports for its molecules; a mistake that dropped the model
    difference (e.g. Eeta = eta and no lambda-xi product) would not."""
    pb, inst, H, t1, t2 = config_problem(3, 6, 4)
    cc = O.CCLR(H, t1, t2)
    Xs = [s.dipole(pb, 0).numpy(), s.dipole(pb, 1).numpy()]
    a = cc.response(Xs, 0.2 + 0.01j)
    b = cc.response_ci(Xs, 0.2 + 0.01j)
    d = np.abs(a - b).max() / np.abs(a).max()
    assert 1e-6 < d < 0.2


def test_asymmetric_form_equals_symmetric_form(cfg1):
    """The asymmetric form (multiplier responses for Y only) is the symmetric
    form regrouped: the t^X(-z) terms equal tbar^Y(z) xi^X exactly."""
    pb, cc, Xs = cfg1
    for z in (0.1 + 0.005j, 0.0):
        a = cc.response(Xs, z)
        b = cc.response_asym(Xs, Xs, z)
        assert np.abs(a - b).max() <= 1e-11 * np.abs(a).max()


def test_asymmetric_form_equals_fci(two_electron):
    d = two_electron
    cc = O.CCLR(d["H"], d["t1"], d["t2"])
    z = 0.3 + 0.02j
    a = cc.response_asym(d["Xs"], d["Xs"][:1], z)
    ex = np.array([[B.fci_response(d["sp"], d["bf"].H, X, Y, z, d["state"]) for Y in d["Xs"][:1]] for X in d["Xs"]])
    assert np.abs(a - ex).max() <= 1e-11 * np.abs(ex).max()


def test_response_pole_is_eigenvalue_of_jacobian(two_electron):
    """Near an eigenvalue w_n of A, Im alpha ~ |residue|/gamma: the damped
    response peaks at the poles, and the poles are eig(A) (= FCI gaps)."""
    d = two_electron
    cc = O.CCLR(d["H"], d["t1"], d["t2"])
    wA = np.sort(np.linalg.eigvals(cc.matrix("right")).real)
    wF = np.linalg.eigvalsh(d["bf"].H)
    gaps = np.sort(np.delete(wF, d["state"]) - wF[d["state"]])
    assert np.abs(wA - gaps).max() < 1e-10


# -------------------------------------------------- config-size invariants
@pytest.fixture(scope="module")
def cfg1():
    pb, inst, H, t1, t2 = config_problem(4, 16, 0)
    cc = O.CCLR(H, t1, t2)
    Xs = [s.dipole(pb, k).numpy() for k in range(3)]
    return pb, cc, Xs


def test_response_symmetries(cfg1):
    pb, cc, Xs = cfg1
    z = 0.1 + 0.005j
    a = cc.response(Xs, z)
    b = cc.response(Xs, -z)
    c = cc.response(Xs, -np.conj(z))
    assert np.abs(a - b.T).max() <= 1e-12 * np.abs(a).max()          # P symmetry
    assert np.abs(a - np.conj(c)).max() <= 1e-12 * np.abs(a).max()   # C^{+-w} symmetry


def test_lambda_residual_and_gmres_agrees_with_lu(cfg1):
    pb, cc, Xs = cfg1
    lam = cc.solve_lambda("dense")
    r = cc.left(*lam)
    e0 = O.eta0(cc.H, cc.hb)
    assert rel(r, (-e0[0], -e0[1])) < 1e-12
    xi = cc.xi(Xs[0])
    z = 0.1 + 0.005j
    a = cc.solve("right", xi, z, "dense")
    b = cc.solve("right", xi, z, "gmres")
    assert rel(b, a) < 1e-10


# ------------------------------------------------------- CCSD ground state
def test_ccsd_residual_vs_bruteforce(case):
    """Omega(t) and the correlation energy against <mu|e^-T H e^T|R> and
    <R|e^-T H e^T|R> - <R|H|R> in the determinant space (random complex
    amplitudes, non-diagonal Fock matrix)."""
    bf, sp = case["bf"], case["sp"]
    bf.set_t(case["t1"], case["t2"])
    ref = bf.omega()
    mine = sp.pack(*O.ccsd_residual(case["H"], case["t1"], case["t2"]))
    assert np.abs(mine - ref).max() <= 1e-12 * np.abs(ref).max()
    e_ref = bf.energy() - bf.H[sp.ref, sp.ref]
    assert abs(O.ccsd_energy(case["H"], case["t1"], case["t2"]) - e_ref) <= 1e-12 * max(1.0, abs(e_ref))


def test_crop_reaches_fci_for_two_electrons():
    """CROP from the MP2-seeded start: the brute-force residual vanishes at
    its result and the energy is an eigenvalue of H (CCSD is exact for two
    electrons)."""
    o, v = 2, 6
    pb = s.Problem(o, v, 11)
    Vf = s.full_integrals(pb).numpy()
    f = s.fock(pb).numpy()
    H = O.Hamiltonian(o, v, f, blocks_from_full(Vf, o))
    t1 = s.t1_amplitudes(pb).numpy()
    t2 = s.t2_amplitudes(pb, torch.tensor(H.blocks["oovv"])).numpy()
    u1, u2, E, it = O.solve_ccsd(H, t1, t2, tol=1e-12)
    sp = B.Space(o, v)
    bf = B.CCBrute(sp, f, Vf)
    bf.set_t(u1, u2)
    assert np.abs(bf.omega()).max() < 1e-12
    w = np.linalg.eigvalsh(bf.H)
    assert np.abs(w - (bf.H[sp.ref, sp.ref] + E)).min() < 1e-12
    assert 2 < it < 100


def test_crop_converges_at_config1_size():
    """CROP at o=4, v=16 (config 1 recipe): residual below the tolerance by
    an independent norm evaluation, in a modest number of iterations."""
    pb, inst, H, t1, t2 = config_problem(4, 16, 0)
    u1, u2, E, it = O.solve_ccsd(H, t1, t2, tol=1e-10)
    r1, r2 = O.ccsd_residual(H, u1, u2)
    assert np.sqrt(np.sum(np.abs(r1) ** 2) + 0.25 * np.sum(np.abs(r2) ** 2)) <= 1e-10
    assert it < 60


def test_cholesky_integrals_vs_mulliken_hamiltonian():
    """Blocks formed from Cholesky vectors define the same many-electron
    Hamiltonian as the Mulliken integrals sum_P L_pq L_rs inserted directly
    into 1/2 sum (pq|rs) p+ r+ s q (no antisymmetrization formula used)."""
    o, v = 2, 4
    pb = s.Problem(o, v, 5)
    n = o + v
    L = s.cholesky_vectors(pb, 9).numpy()
    H = O.Hamiltonian(o, v, s.fock(pb).numpy(), O.integrals_from_cholesky(o, L))
    import itertools
    sl = {"o": slice(0, o), "v": slice(o, None)}
    V = np.zeros((n, n, n, n), dtype=np.complex128)
    for k in itertools.product("ov", repeat=4):
        V[sl[k[0]], sl[k[1]], sl[k[2]], sl[k[3]]] = H.V("".join(k))
    assert np.abs(V + V.transpose(1, 0, 2, 3)).max() < 1e-15
    assert np.abs(V + V.transpose(0, 1, 3, 2)).max() < 1e-15
    assert np.abs(V - V.transpose(2, 3, 0, 1).conj()).max() < 1e-15
    sp = B.Space(o, v)
    h = H.f - np.einsum("piqi->pq", V[:, :o, :, :o])
    eri = np.einsum("Ppq,Prs->pqrs", L, L)
    M1 = sp.hamiltonian(H.f, V)
    M2 = B.hamiltonian_mulliken(sp, h, eri)
    assert np.abs(M1 - M2).max() <= 1e-14 * np.abs(M1).max()


# ----------------------------------------- exact derivative of the response function
def _symmetric_change(o, v, rng):
    """Random change of (f, <pq||rs>) that keeps their symmetries (f
    Hermitian; <pq||rs> antisymmetric in each pair and equal to conj <rs||pq>),
    as a Hamiltonian."""
    n = o + v
    cr = lambda *sh: rng.normal(size=sh) + 1j * rng.normal(size=sh)  # noqa: E731
    D = cr(n, n, n, n)
    D = D - D.transpose(1, 0, 2, 3)
    D = D - D.transpose(0, 1, 3, 2)
    D = 0.5 * (D + D.conj().transpose(2, 3, 0, 1))
    F = cr(n, n)
    F = F + F.conj().T
    return O.Hamiltonian(o, v, F / np.linalg.norm(F), blocks_from_full(D / np.linalg.norm(D), o))


@pytest.mark.parametrize("z", [0.3 + 0.02j, 0.0, -0.2 + 0.05j])
def test_response_derivative_vs_difference_quotients(z):
    """response_derivative along a change of the perturbations and of the
    Hamiltonian (t fixed) against central differences of response() at steps
    h and h/2, Richardson-extrapolated (error O(h^4))."""
    pb, inst, H, t1, t2 = config_problem(3, 5, 4)
    cc = O.CCLR(H, t1, t2)
    Xs = [s.dipole(pb, 0).numpy(), s.magnetic_like(pb, 0).numpy()]
    rng = np.random.default_rng(11)
    dX = [rng.normal(size=X.shape) + 1j * rng.normal(size=X.shape) for X in Xs]
    dH = _symmetric_change(3, 5, rng)
    exact = cc.response_derivative(Xs, z, dX, dH)

    def at(h):
        Hh = O.Hamiltonian(3, 5, H.f + h * dH.f, {k: H.blocks[k] + h * dH.blocks[k] for k in H.blocks})
        return O.CCLR(Hh, t1, t2).response([X + h * d for X, d in zip(Xs, dX)], z)

    h = 2e-3
    d1 = (at(h) - at(-h)) / (2 * h)
    d2 = (at(h / 2) - at(-h / 2)) / h
    fd = (4 * d2 - d1) / 3
    err = np.abs(exact - fd).max() / np.abs(exact).max()
    print(f"z={z}: exact derivative vs Richardson differences {err:.2e}")
    assert err < 1e-8


def test_response_derivative_in_x_is_the_bilinear_expansion():
    """<<X;Y>> is real-bilinear in (X, Y), so its derivative along dX equals
    <<dX_p; X_q>> + <<X_p; dX_q>>, read off one response() call with the
    operators [X, dX] (exact, no step)."""
    pb, inst, H, t1, t2 = config_problem(3, 5, 4)
    cc = O.CCLR(H, t1, t2)
    Xs = [s.dipole(pb, k).numpy() for k in range(2)]
    rng = np.random.default_rng(5)
    dX = [rng.normal(size=X.shape) + 1j * rng.normal(size=X.shape) for X in Xs]
    for z in (0.25 + 0.01j, 0.0):
        exact = cc.response_derivative(Xs, z, dX, None)
        R = cc.response(Xs + dX, z)
        bil = R[2:, :2] + R[:2, 2:]
        assert np.abs(exact - bil).max() <= 1e-12 * np.abs(bil).max()


def test_response_derivative_mutation_is_caught():
    """Dropping the lambda change from the derivative (a plausible mistake)
    is visible against the difference quotients."""
    pb, inst, H, t1, t2 = config_problem(3, 5, 4)
    cc = O.CCLR(H, t1, t2)
    Xs = [s.dipole(pb, 0).numpy()]
    dH = _symmetric_change(3, 5, np.random.default_rng(1))
    z = 0.3 + 0.02j
    cc.solve_lambda("dense")
    exact = cc.response_derivative(Xs, z, None, dH)
    orig = O.CCLR.solve
    calls = []

    def no_dlam(self, side, rhs, w, method="dense", **kw):
        calls.append(side)
        if side == "left" and len(calls) == 1 and self is cc:
            return tuple(np.zeros_like(x) for x in rhs)
        return orig(self, side, rhs, w, method, **kw)

    O.CCLR.solve = no_dlam
    try:
        wrong = cc.response_derivative(Xs, z, None, dH)
    finally:
        O.CCLR.solve = orig
    assert calls[0] == "left"   # the first solve is the lambda change
    assert np.abs(wrong - exact).max() > 1e-6 * np.abs(exact).max()
