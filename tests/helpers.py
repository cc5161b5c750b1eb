"""Shared test helpers: build oracle problems from the seeded generators."""
import numpy as np
import torch

from gen import synth as s
from oracle import cclr_ref as O


def blocks_from_full(Vf, o):
    sl = lambda k: slice(0, o) if k == "o" else slice(o, None)  # noqa: E731
    return {k: Vf[sl(k[0]), sl(k[1]), sl(k[2]), sl(k[3])] for k in s.CANONICAL_BLOCKS}


def small_problem(o, v, seed=3, fscale=0.05, t1_scale=10.0, t2_scale=0.1, v_std=0.1):
    """Random complex problem with a non-diagonal Hermitian Fock matrix and
    unconverged amplitudes: every term of every equation is exercised."""
    pb = s.Problem(o, v, seed, v_std=v_std)
    Vf = s.full_integrals(pb).numpy()
    f = s.fock(pb).numpy()
    if fscale:
        g = s.cgauss(s.stream_key(seed, 999), torch.arange(f.size, dtype=torch.int64), fscale).numpy().reshape(f.shape)
        f = f + g + g.conj().T
    H = O.Hamiltonian(o, v, f, blocks_from_full(Vf, o))
    t1 = s.t1_amplitudes(pb).numpy() * t1_scale
    t2 = s.excitation_vector(pb, 5)[1].numpy() * t2_scale
    return pb, Vf, f, H, t1, t2


def config_problem(o, v, seed):
    """Generator recipe of the benchmark configurations (diagonal Fock, MP2 t2)."""
    pb = s.Problem(o, v, seed)
    inst = s.instance(pb)
    H = O.Hamiltonian(o, v, inst["f"].numpy(), {k: x.numpy() for k, x in inst["V"].items()})
    return pb, inst, H, inst["t1"].numpy(), inst["t2"].numpy()


def vec(pb, k):
    r1, r2 = s.excitation_vector(pb, k)
    return r1.numpy(), r2.numpy()


def rel(a, b):
    """2-norm of the difference over all entries, relative to b (a diagnostic;
    the parity bars use block_errors)."""
    a = np.concatenate([np.ravel(x) for x in a]) if isinstance(a, tuple) else np.ravel(a)
    b = np.concatenate([np.ravel(x) for x in b]) if isinstance(b, tuple) else np.ravel(b)
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def block_errors(got, ref):
    """Element-wise errors per block of an excitation vector (singles, doubles)
    or of a single array: for each block, the largest |got - ref| relative to
    the block's largest |ref| entry, and the block's relative 2-norm error.
    Returns the worst of each over the blocks and a printable summary."""
    gs = got if isinstance(got, (tuple, list)) else (got,)
    rs = ref if isinstance(ref, (tuple, list)) else (ref,)
    names = ("singles", "doubles") if len(rs) == 2 else tuple(f"block{k}" for k in range(len(rs)))
    worst_max = worst_n2 = 0.0
    parts = []
    for name, a, b in zip(names, gs, rs):
        a, b = np.asarray(a), np.asarray(b)
        assert a.shape == b.shape, (name, a.shape, b.shape)
        d = np.abs(a - b)
        scale = np.abs(b).max() if b.size else 0.0
        em = d.max() / scale if scale > 0 else (0.0 if not d.size or d.max() == 0 else np.inf)
        nb = np.linalg.norm(b)
        e2 = np.linalg.norm(a - b) / nb if nb > 0 else (0.0 if em == 0 else np.inf)
        worst_max, worst_n2 = max(worst_max, em), max(worst_n2, e2)
        parts.append(f"{name} max {em:.2e} 2-norm {e2:.2e}")
    return worst_max, worst_n2, "; ".join(parts)


def assert_blocks(got, ref, tol, label=""):
    """Parity bar on excitation vectors: in each block (singles and doubles
    separately) every entry is within tol times that block's largest entry,
    and the block's 2-norm error is within tol relative."""
    em, e2, msg = block_errors(got, ref)
    print(f"{label}: {msg}", flush=True)
    assert em <= tol and e2 <= tol, f"{label}: {msg} (bar {tol:.0e})"


def alpha_errors(out, ref):
    """Response tensor errors: relative error of every entry whose magnitude
    is at least 1e-3 of the largest, the error of the other entries relative
    to the largest, and the Frobenius-norm relative error."""
    out, ref = np.asarray(out), np.asarray(ref)
    mx = np.abs(ref).max()
    big = np.abs(ref) >= 1e-3 * mx
    d = np.abs(out - ref)
    e_big = (d[big] / np.abs(ref[big])).max()
    e_small = d[~big].max() / mx if (~big).any() else 0.0
    e_f = np.linalg.norm(out - ref) / np.linalg.norm(ref)
    return e_big, e_small, e_f


def assert_alpha(out, ref, tol, label=""):
    e_big, e_small, e_f = alpha_errors(out, ref)
    print(f"{label}: entries rel {e_big:.2e}, small entries {e_small:.2e}, Frobenius {e_f:.2e}", flush=True)
    assert e_big <= tol and e_small <= tol and e_f <= tol, (label, e_big, e_small, e_f, tol)
