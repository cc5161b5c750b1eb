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
    a = np.concatenate([np.ravel(x) for x in a]) if isinstance(a, tuple) else np.ravel(a)
    b = np.concatenate([np.ravel(x) for x in b]) if isinstance(b, tuple) else np.ravel(b)
    return np.linalg.norm(a - b) / np.linalg.norm(b)
