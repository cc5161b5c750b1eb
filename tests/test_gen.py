"""Seeded input generators: symmetries, determinism, slice independence."""
import numpy as np
import torch

from gen import synth as s


def test_integral_symmetries():
    pb = s.Problem(3, 7, 5)
    V = s.full_integrals(pb)
    assert torch.equal(V, -V.transpose(0, 1))
    assert torch.equal(V, -V.transpose(2, 3))
    assert torch.equal(V, V.permute(2, 3, 0, 1).conj())


def test_blocks_match_full_tensor():
    pb = s.Problem(3, 7, 5)
    V = s.full_integrals(pb)
    o = pb.o
    sl = {"o": slice(0, o), "v": slice(o, None)}
    for k, b in s.integral_blocks(pb, chunk=2).items():
        assert torch.equal(b, V[sl[k[0]], sl[k[1]], sl[k[2]], sl[k[3]]])


def test_deterministic_and_seed_dependent():
    a = s.integral_blocks(s.Problem(2, 5, 1))["ovvv"]
    b = s.integral_blocks(s.Problem(2, 5, 1))["ovvv"]
    c = s.integral_blocks(s.Problem(2, 5, 2))["ovvv"]
    assert torch.equal(a, b)
    assert not torch.equal(a, c)


def test_statistics():
    pb = s.Problem(4, 16, 0)
    V = s.integral_blocks(pb)["vvvv"]
    x = V.real.flatten()
    x = x[x != 0]
    assert abs(x.std().item() - pb.vstd) < 0.1 * pb.vstd
    e = s.orbital_energies(pb).numpy()
    assert np.all((e[:4] > -2) & (e[:4] < -0.5)) and np.all((e[4:] > 0.3) & (e[4:] < 3))


def test_mp2_amplitudes_and_vectors_antisymmetric():
    pb = s.Problem(3, 6, 0)
    inst = s.instance(pb)
    t2 = inst["t2"]
    assert torch.allclose(t2, -t2.transpose(0, 1)) and torch.allclose(t2, -t2.transpose(2, 3))
    r1, r2 = s.excitation_vector(pb, 0)
    assert torch.equal(r2, -r2.transpose(0, 1)) and torch.equal(r2, -r2.transpose(2, 3))
    X = s.dipole(pb, 0)
    assert torch.equal(X, X.conj().T)
    m = s.magnetic_like(pb, 0)
    assert torch.equal(m, m.conj().T) and torch.all(m.real == 0)


def test_uniform_counter_is_splitmix64():
    """First outputs of SplitMix64 seeded with 0 (published reference values
    of the generator: state += golden; z = mix(state))."""
    ref = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    c = torch.arange(3, dtype=torch.int64)
    raw = s._raw(0, c)
    got = [int(x) & ((1 << 64) - 1) for x in raw.tolist()]
    assert got == ref
