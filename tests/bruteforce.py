"""Formula-free second-quantization reference (test pin for the oracle).

Everything here is computed from the definitions in the paper's Table 1 and
the Lagrangian/Lambda equation of the theory section, by brute force in the
space of all Slater determinants of ``o`` electrons in ``n = o + v`` spin
orbitals.  No coupled-cluster working equation is used: operators are dense
matrices built by applying creation/annihilation operators to bit strings,
and exponentials of the (nilpotent) cluster operator are finite series.

    A_mu,nu   = <mu| e^-T [H, tau_nu] e^T |R>         (Table 1)
    xi^X_mu   = <mu| e^-T X e^T |R>                  (Table 1)
    eta^X_nu  = <Lambda| [X, tau_nu] |CC>            (Table 1)
    F_mu,nu   = <Lambda| [[H, tau_mu], tau_nu] |CC>  (Table 1)
    eta0_nu   = <R| e^-T [H, tau_nu] e^T |R>         (Lambda equation)
    Omega_mu  = <mu| e^-T H e^T |R>                  (CCSD residual)

with <Lambda| = <R| + sum_mu lambda_mu <mu| e^-T.  Excitations mu run over
unique singles (i,a) and doubles (i>j, a>b); tau_ijab = a+_a a+_b a_j a_i.

The Hamiltonian is H = sum h_pq p+q + 1/4 sum <pq||rs> p+q+sr with
h = f - sum_i <pi||qi>, so that its Fock matrix relative to |R> is f.
Only for tiny spaces (a few hundred determinants).
"""
from __future__ import annotations

import itertools
import math

import numpy as np


def _ann(det: int, p: int):
    if not (det >> p) & 1:
        return None
    sign = -1 if bin(det & ((1 << p) - 1)).count("1") & 1 else 1
    return sign, det & ~(1 << p)


def _cre(det: int, p: int):
    if (det >> p) & 1:
        return None
    sign = -1 if bin(det & ((1 << p) - 1)).count("1") & 1 else 1
    return sign, det | (1 << p)


def _apply(det: int, ops):
    """ops: sequence of (orbital, is_creator) applied right-to-left (last first)."""
    sign = 1
    for p, cre in reversed(ops):
        r = _cre(det, p) if cre else _ann(det, p)
        if r is None:
            return None
        s, det = r
        sign *= s
    return sign, det


class Space:
    def __init__(self, o: int, v: int):
        self.o, self.v, self.n = o, v, o + v
        self.dets = [sum(1 << k for k in c) for c in itertools.combinations(range(self.n), o)]
        self.index = {d: k for k, d in enumerate(self.dets)}
        self.D = len(self.dets)
        self.ref = self.index[(1 << o) - 1]
        # unique excitations
        self.singles = [(i, a) for i in range(o) for a in range(v)]
        self.doubles = [(i, j, a, b) for i in range(o) for j in range(i) for a in range(v) for b in range(a)]
        self.nmu = len(self.singles) + len(self.doubles)
        self._tau = []
        for (i, a) in self.singles:
            self._tau.append(self._op_entries([(o + a, True), (i, False)]))
        for (i, j, a, b) in self.doubles:
            self._tau.append(self._op_entries([(o + a, True), (o + b, True), (j, False), (i, False)]))
        # position and sign of tau_mu|R> (the bra <mu|)
        self.mu_pos = np.empty(self.nmu, dtype=np.int64)
        self.mu_sign = np.empty(self.nmu)
        for k, (rows, cols, sg) in enumerate(self._tau):
            hit = np.nonzero(cols == self.ref)[0]
            assert len(hit) == 1
            self.mu_pos[k] = rows[hit[0]]
            self.mu_sign[k] = sg[hit[0]]

    # ---------------------------------------------------------------- operators
    def _op_entries(self, ops):
        rows, cols, sg = [], [], []
        for c, d in enumerate(self.dets):
            r = _apply(d, ops)
            if r is not None:
                rows.append(self.index[r[1]])
                cols.append(c)
                sg.append(r[0])
        return np.array(rows, dtype=np.int64), np.array(cols, dtype=np.int64), np.array(sg, dtype=np.float64)

    def excitation_operator(self, x1, x2):
        """sum_mu x_mu tau_mu as a dense matrix; x1[i,a], x2[i,j,a,b] (antisymmetric)."""
        M = np.zeros((self.D, self.D), dtype=np.complex128)
        coefs = self.pack(x1, x2)
        for c, (rows, cols, sg) in zip(coefs, self._tau):
            if c != 0:
                np.add.at(M, (rows, cols), c * sg)
        return M

    def tau_matrix(self, k):
        M = np.zeros((self.D, self.D), dtype=np.complex128)
        rows, cols, sg = self._tau[k]
        M[rows, cols] = sg
        return M

    def one_body(self, h):
        """sum_pq h[p,q] p+ q."""
        n = self.n
        M = np.zeros((self.D, self.D), dtype=np.complex128)
        for c, d in enumerate(self.dets):
            for q in range(n):
                r1 = _ann(d, q)
                if r1 is None:
                    continue
                for p in range(n):
                    r2 = _cre(r1[1], p)
                    if r2 is None:
                        continue
                    M[self.index[r2[1]], c] += h[p, q] * r1[0] * r2[0]
        return M

    def hamiltonian(self, f, V):
        """H with Fock matrix f relative to |R>; V[p,q,r,s] = <pq||rs> (n^4)."""
        o, n = self.o, self.n
        h = f - np.einsum("piqi->pq", V[:, :o, :, :o])
        M = self.one_body(h)
        for c, d in enumerate(self.dets):
            occ = [k for k in range(n) if (d >> k) & 1]
            for r, s in itertools.combinations(occ, 2):       # r < s
                a1 = _ann(d, r)
                a2 = _ann(a1[1], s)
                s12 = a1[0] * a2[0]
                d2 = a2[1]
                emp = [k for k in range(n) if not (d2 >> k) & 1]
                for p, q in itertools.combinations(emp, 2):   # p < q
                    c1 = _cre(d2, q)
                    c2 = _cre(c1[1], p)
                    # p+ q+ s r with r<s, p<q: 4 equal images of 1/4 sum
                    M[self.index[c2[1]], c] += V[p, q, r, s] * s12 * c1[0] * c2[0]
        return M

    # ------------------------------------------------------------------ vectors
    def pack(self, x1, x2):
        out = np.empty(self.nmu, dtype=np.complex128)
        k = 0
        for (i, a) in self.singles:
            out[k] = x1[i, a]
            k += 1
        for (i, j, a, b) in self.doubles:
            out[k] = x2[i, j, a, b]
            k += 1
        return out

    def unpack(self, vec):
        o, v = self.o, self.v
        x1 = np.zeros((o, v), dtype=np.complex128)
        x2 = np.zeros((o, o, v, v), dtype=np.complex128)
        ns = len(self.singles)
        for k, (i, a) in enumerate(self.singles):
            x1[i, a] = vec[k]
        for k, (i, j, a, b) in enumerate(self.doubles):
            val = vec[ns + k]
            x2[i, j, a, b] = val
            x2[j, i, a, b] = -val
            x2[i, j, b, a] = -val
            x2[j, i, b, a] = val
        return x1, x2

    def ref_vec(self):
        e = np.zeros(self.D, dtype=np.complex128)
        e[self.ref] = 1.0
        return e

    def project(self, state):
        """<mu|state> for every unique mu."""
        return self.mu_sign * state[self.mu_pos]

    def bra(self, lam):
        """Row vector sum_mu lam_mu <mu| (lam packed)."""
        row = np.zeros(self.D, dtype=np.complex128)
        np.add.at(row, self.mu_pos, lam * self.mu_sign)
        return row


def expm_nilpotent(T):
    out = np.eye(T.shape[0], dtype=np.complex128)
    term = out.copy()
    for k in range(1, T.shape[0] + 1):
        term = term @ T / k
        if not np.any(term):
            break
        out = out + term
    return out


class CCBrute:
    """Brute-force CC quantities for given f, V (n^4) and amplitudes."""

    def __init__(self, sp: Space, f, V):
        self.sp = sp
        self.H = sp.hamiltonian(np.asarray(f), np.asarray(V))
        self.f = np.asarray(f)

    def set_t(self, t1, t2):
        sp = self.sp
        self.T = sp.excitation_operator(t1, t2)
        self.eT = expm_nilpotent(self.T)
        self.emT = expm_nilpotent(-self.T)
        self.Hbar = self.emT @ self.H @ self.eT
        self.R = sp.ref_vec()

    def energy(self):
        return self.Hbar[self.sp.ref, self.sp.ref]

    def omega(self):
        return self.sp.project(self.Hbar[:, self.sp.ref])

    def jacobian_right(self, r1, r2):
        Rop = self.sp.excitation_operator(r1, r2)
        C = self.emT @ (self.H @ Rop - Rop @ self.H) @ self.eT
        return self.sp.project(C[:, self.sp.ref])

    def jacobian_matrix(self):
        sp = self.sp
        A = np.empty((sp.nmu, sp.nmu), dtype=np.complex128)
        for k in range(sp.nmu):
            tk = sp.tau_matrix(k)
            C = self.emT @ (self.H @ tk - tk @ self.H) @ self.eT
            A[:, k] = sp.project(C[:, sp.ref])
        return A

    def lambda_bra(self, lam_packed):
        """<Lambda| e^-T ... as the row <R| + sum lam <mu| (left of e^-T)."""
        return self.sp.ref_vec() + self.sp.bra(lam_packed)

    def eta0(self):
        sp = self.sp
        out = np.empty(sp.nmu, dtype=np.complex128)
        for k in range(sp.nmu):
            tk = sp.tau_matrix(k)
            C = self.emT @ (self.H @ tk - tk @ self.H) @ self.eT
            out[k] = C[sp.ref, sp.ref]
        return out

    def xi(self, X):
        Xop = self.sp.one_body(np.asarray(X))
        return self.sp.project((self.emT @ Xop @ self.eT)[:, self.sp.ref])

    def eta(self, X, lam_packed):
        sp = self.sp
        Xop = sp.one_body(np.asarray(X))
        row = self.lambda_bra(lam_packed) @ self.emT
        col = self.eT[:, sp.ref]
        out = np.empty(sp.nmu, dtype=np.complex128)
        for k in range(sp.nmu):
            tk = sp.tau_matrix(k)
            out[k] = row @ ((Xop @ tk - tk @ Xop) @ col)
        return out

    def xF(self, lam_packed, x1, x2):
        """(x F)_nu = <Lambda| [[H, X], tau_nu] |CC>,  X = sum_mu x_mu tau_mu."""
        sp = self.sp
        Xop = sp.excitation_operator(x1, x2)
        HX = self.H @ Xop - Xop @ self.H
        row = self.lambda_bra(lam_packed) @ self.emT
        col = self.eT[:, sp.ref]
        out = np.empty(sp.nmu, dtype=np.complex128)
        for k in range(sp.nmu):
            tk = sp.tau_matrix(k)
            out[k] = row @ ((HX @ tk - tk @ HX) @ col)
        return out


def fci_response(sp: Space, H, X, Y, z, state):
    """Exact <<X;Y>>_z = -sum_n [X_0n Y_n0/(w_n - z) + Y_0n X_n0/(w_n + z)].

    ``state`` selects the eigenvector of H used as |0> (index into eigh order).
    """
    w, U = np.linalg.eigh(H)
    Xop, Yop = sp.one_body(X), sp.one_body(Y)
    u0 = U[:, state]
    Xn = U.conj().T @ (Xop @ u0)      # <n|X|0>
    Yn = U.conj().T @ (Yop @ u0)
    X0 = (u0.conj() @ Xop) @ U        # <0|X|n>
    Y0 = (u0.conj() @ Yop) @ U
    tot = 0.0 + 0.0j
    for k in range(len(w)):
        if k == state:
            continue
        wn = w[k] - w[state]
        tot += X0[k] * Yn[k] / (wn - z) + Y0[k] * Xn[k] / (wn + z)
    return -tot


def hamiltonian_mulliken(sp: Space, h, eri):
    """H = sum h_pq p+ q + 1/2 sum (pq|rs) p+ r+ s q from Mulliken-ordered
    integrals eri[p,q,r,s] = (pq|rs) (no antisymmetrized integrals used)."""
    n = sp.n
    M = sp.one_body(np.asarray(h))
    for c, d in enumerate(sp.dets):
        for q in range(n):
            a1 = _ann(d, q)
            if a1 is None:
                continue
            for s in range(n):
                a2 = _ann(a1[1], s)
                if a2 is None:
                    continue
                for r in range(n):
                    c1 = _cre(a2[1], r)
                    if c1 is None:
                        continue
                    for p in range(n):
                        c2 = _cre(c1[1], p)
                        if c2 is None:
                            continue
                        sg = a1[0] * a2[0] * c1[0] * c2[0]
                        M[sp.index[c2[1]], c] += 0.5 * eri[p, q, r, s] * sg
    return M
