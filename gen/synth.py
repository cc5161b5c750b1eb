"""Seeded synthetic inputs for the CC linear-response hot path.

This module is shared test/bench infrastructure.  It produces the *inputs*
(orbital energies, antisymmetrized two-electron integrals, MP2-seeded
amplitudes, perturbation matrices, trial vectors) and contains none of the
method's arithmetic.  Both the CPU oracle and the GPU path consume what it
returns; they never exchange values with each other.

Random numbers
--------------
Every value is a pure function of (seed, stream, counter): the 64-bit output
function of SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014) applied to ``key + (counter + 1) * GOLDEN``.
Uniforms take the top 53 bits; Gaussians come from the Box-Muller transform
of two consecutive uniforms.  Because each entry is addressed by its own
counter, any block or slice of an integral tensor can be produced on its own,
on the CPU or on a GPU (the code below is plain torch integer/float ops).

Integral recipe
---------------
``<pq||rs>`` must satisfy ``<pq||rs> = -<qp||rs> = -<pq||sr>`` and
``<pq||rs> = conj(<rs||pq>)``.  One complex Gaussian is drawn per unique
canonical entry (p<q, r<s, pair(pq) <= pair(rs)), with standard deviation
``v_std`` per component; every other entry is obtained from it by the
symmetries.  For a generic entry this is the same distribution as averaging
the eight images of an unsymmetrized N(0, 0.1) tensor (std 0.1/sqrt(8)).
Entries with pair(pq) == pair(rs) are real (std v_std*sqrt(2)).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import torch

_GOLDEN = 0x9E3779B97F4A7C15
_M1 = 0xBF58476D1CE4E5B9
_M2 = 0x94D049BB133111EB
_MASK64 = (1 << 64) - 1

# stream ids
STREAM_EPS = 0
STREAM_V = 1
STREAM_T1 = 2
STREAM_VEC = 50          # + k : trial vectors
STREAM_PERT = 100        # + k : perturbation matrices
STREAM_CHOL = 3          # Cholesky vectors


def _s64(x: int) -> int:
    """Python int -> value of the same 64 bits as a signed int64."""
    x &= _MASK64
    return x - (1 << 64) if x >= (1 << 63) else x


def _mix_int(z: int) -> int:
    z &= _MASK64
    z = ((z ^ (z >> 30)) * _M1) & _MASK64
    z = ((z ^ (z >> 27)) * _M2) & _MASK64
    return z ^ (z >> 31)


def _srl(x: torch.Tensor, k: int) -> torch.Tensor:
    """Logical right shift of int64 bit patterns."""
    return (x >> k) & ((1 << (64 - k)) - 1)


def _mix(z: torch.Tensor) -> torch.Tensor:
    z = (z ^ _srl(z, 30)) * _s64(_M1)
    z = (z ^ _srl(z, 27)) * _s64(_M2)
    return z ^ _srl(z, 31)


def stream_key(seed: int, stream: int) -> int:
    return _mix_int(_mix_int(seed * _GOLDEN + 0x632BE59BD9B4E019) ^ (stream * 0xD1B54A32D192ED03))


def _raw(key: int, counter: torch.Tensor) -> torch.Tensor:
    # key + (counter+1)*GOLDEN with wrapping int64 arithmetic
    return _mix((counter + 1) * _s64(_GOLDEN) + _s64(key))


def uniform(key: int, counter: torch.Tensor) -> torch.Tensor:
    """U(0,1) (open interval) float64 for each int64 counter."""
    r = _raw(key, counter)
    return (_srl(r, 11).to(torch.float64) + 0.5) * (2.0 ** -53)


def cgauss(key: int, counter: torch.Tensor, std: float) -> torch.Tensor:
    """Complex Gaussian, each component N(0, std^2), one per counter."""
    u1 = uniform(key, 2 * counter)
    u2 = uniform(key, 2 * counter + 1)
    r = torch.sqrt(-2.0 * torch.log(u1)) * std
    th = (2.0 * math.pi) * u2
    return torch.complex(r * torch.cos(th), r * torch.sin(th))


# --------------------------------------------------------------------------
# problem description
# --------------------------------------------------------------------------

def default_v_std(o: int, v: int) -> float:
    """Per-component std of the unique integral entries: 0.1/sqrt(8), the
    same distribution as symmetrizing an N(0, 0.1) + i N(0, 0.1) tensor by
    averaging its eight symmetry images."""
    return 0.1 / math.sqrt(8.0)


@dataclass
class Problem:
    o: int
    v: int
    seed: int = 0
    v_std: float | None = None
    t1_std: float = 0.01
    eps_occ: tuple = (-2.0, -0.5)
    eps_vir: tuple = (0.3, 3.0)
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.o + self.v

    @property
    def vstd(self) -> float:
        return default_v_std(self.o, self.v) if self.v_std is None else float(self.v_std)


def orbital_energies(pb: Problem, device="cpu") -> torch.Tensor:
    key = stream_key(pb.seed, STREAM_EPS)
    c = torch.arange(pb.n, dtype=torch.int64, device=device)
    u = uniform(key, c)
    lo = torch.tensor([pb.eps_occ[0]] * pb.o + [pb.eps_vir[0]] * pb.v, dtype=torch.float64, device=device)
    hi = torch.tensor([pb.eps_occ[1]] * pb.o + [pb.eps_vir[1]] * pb.v, dtype=torch.float64, device=device)
    return lo + (hi - lo) * u


def fock(pb: Problem, device="cpu") -> torch.Tensor:
    """n x n Fock matrix, diag(eps), complex128."""
    return torch.diag(orbital_energies(pb, device)).to(torch.complex128)


def _pair(p: torch.Tensor, q: torch.Tensor) -> torch.Tensor:
    # index of the unordered pair {p<q}: q*(q-1)/2 + p
    return q * (q - 1) // 2 + p


def integrals_at(pb: Problem, p, q, r, s) -> torch.Tensor:
    """<pq||rs> for broadcastable int64 global-index tensors (occupied first)."""
    p, q, r, s = torch.broadcast_tensors(p, q, r, s)
    sign = torch.ones(p.shape, dtype=torch.float64, device=p.device)
    swap = p > q
    p, q = torch.where(swap, q, p), torch.where(swap, p, q)
    sign = torch.where(swap, -sign, sign)
    swap = r > s
    r, s = torch.where(swap, s, r), torch.where(swap, r, s)
    sign = torch.where(swap, -sign, sign)
    zero = (p == q) | (r == s)
    P = _pair(p, q)
    R = _pair(r, s)
    cj = P > R
    P, R = torch.where(cj, R, P), torch.where(cj, P, R)
    npair = pb.n * (pb.n - 1) // 2
    g = cgauss(stream_key(pb.seed, STREAM_V), P * npair + R, pb.vstd)
    diag = P == R
    g = torch.where(diag, torch.complex(g.real * math.sqrt(2.0), torch.zeros_like(g.real)), g)
    g = torch.where(cj, g.conj(), g)
    g = g * sign
    return torch.where(zero, torch.zeros_like(g), g)


def _range(kind: str, pb: Problem, device):
    if kind == "o":
        return torch.arange(pb.o, dtype=torch.int64, device=device)
    return torch.arange(pb.o, pb.n, dtype=torch.int64, device=device)


def integral_block(pb: Problem, blk: str, device="cpu", first=None) -> torch.Tensor:
    """Block of <pq||rs> with index kinds given by ``blk`` (e.g. 'oovv').

    ``first`` optionally restricts the first index to a python slice (local
    positions within its kind), so big blocks can be produced in pieces.
    """
    rg = [_range(k, pb, device) for k in blk]
    if first is not None:
        rg[0] = rg[0][first]
    p = rg[0].view(-1, 1, 1, 1)
    q = rg[1].view(1, -1, 1, 1)
    r = rg[2].view(1, 1, -1, 1)
    s = rg[3].view(1, 1, 1, -1)
    return integrals_at(pb, p, q, r, s)


CANONICAL_BLOCKS = ("oooo", "ooov", "oovv", "ovov", "ovvv", "vvvv")


def integral_blocks(pb: Problem, device="cpu", chunk: int = 16) -> dict:
    """The six canonical blocks, complex128, row-major [p][q][r][s]."""
    out = {}
    for blk in CANONICAL_BLOCKS:
        nfirst = pb.o if blk[0] == "o" else pb.v
        parts = []
        for s0 in range(0, nfirst, chunk):
            parts.append(integral_block(pb, blk, device, slice(s0, min(nfirst, s0 + chunk))))
        out[blk] = torch.cat(parts, 0).contiguous()
    return out


def full_integrals(pb: Problem, device="cpu") -> torch.Tensor:
    """All n^4 integrals (small n only)."""
    g = torch.arange(pb.n, dtype=torch.int64, device=device)
    return integrals_at(pb, g.view(-1, 1, 1, 1), g.view(1, -1, 1, 1), g.view(1, 1, -1, 1), g.view(1, 1, 1, -1))


def t1_amplitudes(pb: Problem, device="cpu") -> torch.Tensor:
    """t1[i,a] ~ complex N(0, t1_std^2) per component."""
    c = torch.arange(pb.o * pb.v, dtype=torch.int64, device=device)
    return cgauss(stream_key(pb.seed, STREAM_T1), c, pb.t1_std).view(pb.o, pb.v)


def t2_amplitudes(pb: Problem, oovv: torch.Tensor, device="cpu") -> torch.Tensor:
    """MP2-seeded doubles: t[i,j,a,b] = <ab||ij> / (e_i + e_j - e_a - e_b).

    <ab||ij> = conj(<ij||ab>), taken from the given oovv block.
    """
    e = orbital_energies(pb, device)
    eo, ev = e[: pb.o], e[pb.o:]
    d = eo.view(-1, 1, 1, 1) + eo.view(1, -1, 1, 1) - ev.view(1, 1, -1, 1) - ev.view(1, 1, 1, -1)
    return (oovv.conj() / d).contiguous()


def dipole(pb: Problem, k: int, device="cpu") -> torch.Tensor:
    """Hermitian n x n matrix X = (G + G^H)/2, Re/Im of G ~ N(0,1)."""
    n = pb.n
    c = torch.arange(n * n, dtype=torch.int64, device=device)
    g = cgauss(stream_key(pb.seed, STREAM_PERT + k), c, 1.0).view(n, n)
    return (0.5 * (g + g.conj().T)).contiguous()


def magnetic_like(pb: Problem, k: int, device="cpu") -> torch.Tensor:
    """Hermitian, purely imaginary n x n matrix i*(A - A^T)/2, A real N(0,1)."""
    n = pb.n
    c = torch.arange(n * n, dtype=torch.int64, device=device)
    a = cgauss(stream_key(pb.seed, STREAM_PERT + 50 + k), c, 1.0).real.view(n, n)
    m = 0.5 * (a - a.T)
    return torch.complex(torch.zeros_like(m), m).contiguous()


def excitation_vector(pb: Problem, k: int, device="cpu", std1: float = 1.0, std2: float = 1.0):
    """Random antisymmetric (r1[i,a], r2[i,j,a,b]) pair; r2 drawn on i>j, a>b."""
    o, v = pb.o, pb.v
    key = stream_key(pb.seed, STREAM_VEC + k)
    c1 = torch.arange(o * v, dtype=torch.int64, device=device)
    r1 = cgauss(key, c1, std1).view(o, v)
    i = torch.arange(o, device=device).view(-1, 1, 1, 1)
    j = torch.arange(o, device=device).view(1, -1, 1, 1)
    a = torch.arange(v, device=device).view(1, 1, -1, 1)
    b = torch.arange(v, device=device).view(1, 1, 1, -1)
    ii, jj = torch.maximum(i, j), torch.minimum(i, j)
    aa, bb = torch.maximum(a, b), torch.minimum(a, b)
    sgn = torch.where((i > j) == (a > b), 1.0, -1.0).to(torch.float64)
    zero = (i == j) | (a == b)
    ctr = o * v + ((ii * (ii - 1) // 2 + jj) * (v * (v - 1) // 2) + (aa * (aa - 1) // 2 + bb))
    r2 = cgauss(key, ctr, std2) * sgn
    r2 = torch.where(zero, torch.zeros_like(r2), r2)
    return r1.contiguous(), r2.contiguous()


def cholesky_vectors(pb: Problem, nchol: int, device="cpu", std: float | None = None) -> torch.Tensor:
    """nchol Hermitian n x n matrices L[P] = (G + G^H)/2 (complex Gaussian G),
    the form of MO-basis Cholesky vectors of the Coulomb integrals.  The
    default std puts sums of nchol products of entries at about the scale of
    the directly drawn integrals."""
    n = pb.n
    if std is None:
        std = math.sqrt(pb.vstd * math.sqrt(8.0) / math.sqrt(2.0 * nchol))
    c = torch.arange(nchol * n * n, dtype=torch.int64, device=device)
    g = cgauss(stream_key(pb.seed, STREAM_CHOL), c, std).view(nchol, n, n)
    return (0.5 * (g + g.conj().transpose(1, 2))).contiguous()


def instance(pb: Problem, device="cpu", with_blocks=True) -> dict:
    """Everything a CC linear-response run needs: f, V blocks, t1, t2."""
    out = {"f": fock(pb, device), "t1": t1_amplitudes(pb, device)}
    if with_blocks:
        out["V"] = integral_blocks(pb, device)
        out["t2"] = t2_amplitudes(pb, out["V"]["oovv"], device)
    return out
