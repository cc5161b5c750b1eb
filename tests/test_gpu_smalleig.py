"""The GPU eigensolver of the EOM-EE Davidson subspace (cclr_dbg_small_eig)
against numpy.linalg.eig: the eigenvalue set, the selection of the roots of
smallest real part, and unit-norm right eigenvectors with small residuals,
on random, Hermitian, triangular, tied and projected matrices up to the
largest subspace (120)."""
import ctypes

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


class C64(ctypes.Structure):
    _fields_ = [("re", ctypes.c_double), ("im", ctypes.c_double)]


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2307_14296_amd as cc
    L = cc.lib()
    P = ctypes.c_void_p
    L.cclr_dbg_small_eig.argtypes = [ctypes.c_int, P, ctypes.c_int, P, P, P]
    return L


def small_eig(L, H, nroots):
    n = H.shape[0]
    Hc = np.ascontiguousarray(H, dtype=np.complex128)
    w = np.zeros(n, np.complex128)
    th = np.zeros(nroots, np.complex128)
    V = np.zeros((nroots, n), np.complex128)
    rc = L.cclr_dbg_small_eig(n, Hc.ctypes.data, nroots, w.ctypes.data, th.ctypes.data, V.ctypes.data)
    return rc, w, th, V


def check(L, H, nroots, tol=1e-10):
    rc, w, th, V = small_eig(L, H, nroots)
    assert rc == 0
    n = H.shape[0]
    scale = max(1.0, np.abs(H).max() * n)
    ref = np.linalg.eigvals(H)
    # eigenvalue sets: each GPU eigenvalue matches a distinct reference one
    left = list(ref)
    for x in w:
        d = [abs(x - y) for y in left]
        k = int(np.argmin(d))
        assert d[k] <= tol * scale, (n, x, left[k])
        left.pop(k)
    # selection: the nroots smallest real parts (ties by position in w)
    order = sorted(range(n), key=lambda k: (w[k].real, k))
    np.testing.assert_array_equal(th, w[order[:nroots]])
    # unit-norm eigenvectors, small residuals
    for r in range(nroots):
        v = V[r]
        assert abs(np.linalg.norm(v) - 1.0) <= 1e-12
        assert np.linalg.norm(H @ v - th[r] * v) <= tol * scale, (n, r)
    return w, th, V


@pytest.mark.parametrize("n", [1, 2, 3, 8, 17, 63, 64, 65, 119, 120])
def test_random_complex(L, n):
    rng = np.random.default_rng(1000 + n)
    H = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    check(L, H, min(n, 6))


def test_hermitian_and_triangular(L):
    rng = np.random.default_rng(7)
    n = 40
    X = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    Hh = X + X.conj().T
    w, th, V = check(L, Hh, 5)
    assert np.abs(w.imag).max() <= 1e-10 * np.abs(Hh).max() * n
    np.testing.assert_allclose(np.sort(th.real), np.linalg.eigvalsh(Hh)[:5], atol=1e-10 * np.abs(Hh).max() * n)
    T = np.triu(X)  # already in Schur form
    check(L, T, 4)


def test_ties_and_repeated_eigenvalues(L):
    # diagonal with repeated entries: the tie between equal real parts goes to the lower position
    D = np.diag([3.0, 1.0, 2.0, 1.0, 5.0, 1.0 + 0.5j]).astype(np.complex128)
    rc, w, th, V = small_eig(L, D, 3)
    assert rc == 0
    assert sorted(w.real) == sorted(np.diag(D).real)
    assert np.allclose(th.real, [1.0, 1.0, 1.0])
    for r in range(3):
        assert np.linalg.norm(D @ V[r] - th[r] * V[r]) <= 1e-14


def test_projected_jacobian_like(L):
    """A Davidson-like projected matrix: B^H A B with A = D + a small
    non-Hermitian coupling and B orthonormal, at the largest subspace."""
    rng = np.random.default_rng(11)
    N, n = 600, 120
    A = np.diag(np.linspace(0.3, 3.0, N)) + 0.02 * (rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N)))
    B, _ = np.linalg.qr(rng.standard_normal((N, n)) + 1j * rng.standard_normal((N, n)))
    check(L, B.conj().T @ A @ B, 12)


def test_size_limits(L):
    H = np.eye(121, dtype=np.complex128)
    rc, *_ = small_eig(L, H, 1)
    import paper_2307_14296_amd as cc
    assert rc == cc.CCLR_EINVAL
    rc, *_ = small_eig(L, np.eye(4, dtype=np.complex128), 5)
    assert rc == cc.CCLR_EINVAL
