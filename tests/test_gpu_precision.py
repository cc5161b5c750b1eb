"""Mixed-precision path: the ladder and ring products on FP32 MFMA or on
split-BF16 MFMA (three bf16 products per real product, both operands split:
BF16X3; two, the operator rounded to bf16: BF16X2; FP32 accumulation)
inside the inner solves, FP64 true residuals (iterative refinement).

Bars: a reduced-precision GEMM is within its arithmetic's error of the
complex128 product (FP32: 1e-5, BF16X3: 5e-5 relative in the Frobenius
norm, since the split leaves about 2^-17 relative per operand and FP32
accumulation adds about sqrt(K) 2^-24; BF16X2: 3e-3, the bf16 rounding of
one operand, 2^-9 per element, averaged over the sum); a reduced-precision transform is within 1e-5 (FP32) / 1e-4 (BF16X3)
/ 3e-3 (BF16X2) relative of the FP64 oracle; the refined response function
is within 1e-6 relative of the FP64 oracle (the stated mixed-precision bar).
Each check also requires an error above 1e-12, which shows that the reduced
arithmetic really ran."""
import ctypes

import numpy as np
import pytest
import torch

from gen import synth as s
from helpers import alpha_errors, block_errors, config_problem, vec
from oracle import cclr_ref as O

pytestmark = pytest.mark.gpu


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x)).to(torch.complex128).cuda()


def make(H, t1, t2, prec, tol=1e-10):
    import paper_2307_14296_amd as cc
    op = cc.cclr_default_options()
    op.prec = prec
    op.tol = tol
    ctx = cc.cclr_create(H.o, H.v, op)
    keep = [dev(H.f)] + [dev(H.blocks[k]) for k in s.CANONICAL_BLOCKS] + [dev(t1), dev(t2)]
    cc.cclr_set_hamiltonian(ctx, *keep[:7])
    cc.cclr_set_amplitudes(ctx, *keep[7:])
    return cc, ctx


@pytest.fixture(scope="module")
def cfg1():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pb, inst, H, t1, t2 = config_problem(4, 16, 0)
    return pb, H, t1, t2, O.CCLR(H, t1, t2)


GEMM_CASES = [(1, 1, 1, 0, 0), (17, 33, 5, 1, 0), (130, 3, 129, 0, 1), (200, 260, 300, 1, 1), (300, 257, 1000, 0, 0),
              (600, 530, 70, 0, 0), (1030, 600, 200, 1, 1), (520, 700, 33, 1, 0),
              # at most 32 output columns, and 200 (the FP32 engine kernel's 32-column tiles), ragged row tiles
              (300, 20, 400, 0, 1), (257, 32, 64, 1, 0), (300, 200, 150, 0, 0), (130, 200, 70, 1, 1)]
PRECS = {"fp32": (1, 1e-5, 1e-5), "bf16x3": (2, 5e-5, 1e-4), "bf16x2": (3, 3e-3, 3e-3)}
# the engine's FP32 kernel of the remaining products (complex128 operands converted in the kernel)
GEMM_PRECS = {**PRECS, "fp32_engine": (16, 1e-5, None)}


@pytest.mark.parametrize("prec", list(GEMM_PRECS))
@pytest.mark.parametrize("M,N,K,ta,tb", GEMM_CASES)
def test_lowp_gemm(cfg1, prec, M, N, K, ta, tb):
    import paper_2307_14296_amd as cc
    L = cc.lib()
    P, LL = ctypes.c_void_p, ctypes.c_longlong
    L.cclr_dbg_zgemm_lowp.argtypes = [ctypes.c_int] * 4 + [P, LL, LL, ctypes.c_int, P, LL, LL, ctypes.c_int,
                                                          P, LL, LL, ctypes.c_double, ctypes.c_double, ctypes.c_int]
    code, gemm_bar, _ = GEMM_PRECS[prec]
    rng = np.random.default_rng(M + 7 * N + 13 * K)
    A = rng.normal(size=(M, K)) + 1j * rng.normal(size=(M, K))
    B = rng.normal(size=(K, N)) + 1j * rng.normal(size=(K, N))
    C0 = rng.normal(size=(M, N)) + 1j * rng.normal(size=(M, N))
    alpha = 0.7 - 0.3j
    for conjA, conjB, beta in [(0, 0, 0), (1, 0, 1), (0, 1, 1), (1, 1, 0)]:
        Ad = dev(A.T.copy() if ta else A)
        Bd = dev(B.T.copy() if tb else B)
        Cd = dev(C0)
        sAm, sAk = (1, M) if ta else (K, 1)
        sBk, sBn = (1, K) if tb else (N, 1)
        rc = L.cclr_dbg_zgemm_lowp(code, M, N, K, Ad.data_ptr(), sAm, sAk, conjA, Bd.data_ptr(), sBk, sBn, conjB,
                                   Cd.data_ptr(), N, 1, alpha.real, alpha.imag, beta)
        assert rc == 0
        a = A.conj() if conjA else A
        b = B.conj() if conjB else B
        prod = alpha * (a @ b)
        got = Cd.cpu().numpy() - (C0 if beta else 0)
        e = np.linalg.norm(got - prod) / np.linalg.norm(prod)
        print(f"{prec} GEMM {M}x{N}x{K} conj {conjA}{conjB} beta {beta}: rel err {e:.2e}", flush=True)
        assert (1e-12 < e or M * N * K == 1) and e < gemm_bar


@pytest.mark.parametrize("prec", list(PRECS))
def test_lowp_transform_accuracy(cfg1, prec):
    pb, H, t1, t2, ref = cfg1
    code, _, bar = PRECS[prec]
    cc, ctx = make(H, t1, t2, code)
    try:
        L = cc.lib()
        L.cclr_dbg_set_sigma_prec.argtypes = [ctypes.c_void_p, ctypes.c_int]
        assert L.cclr_dbg_set_sigma_prec(ctx, code) == 0
        xs = [vec(pb, k) for k in range(3)]
        r1, r2 = dev(np.stack([x[0] for x in xs])), dev(np.stack([x[1] for x in xs]))
        for fn, side in ((cc.cclr_jacobian_right, ref.right), (cc.cclr_jacobian_left, ref.left)):
            s1, s2 = torch.empty_like(r1), torch.empty_like(r2)
            fn(ctx, [0.1] * 3, [0.005] * 3, r1, r2, s1, s2)
            for k, x in enumerate(xs):
                em, e2, msg = block_errors((s1[k].cpu().numpy(), s2[k].cpu().numpy()), side(*x, 0.1 + 0.005j))
                print(f"{prec} {fn.__name__}: {msg}", flush=True)
                assert 1e-12 < e2 and em < bar and e2 < bar   # really low precision, and accurate to it
        L.cclr_dbg_set_sigma_prec(ctx, cc.CCLR_FP64)
    finally:
        cc.cclr_destroy(ctx)


@pytest.mark.parametrize("prec", list(PRECS))
def test_lowp_refined_response(cfg1, prec):
    pb, H, t1, t2, ref = cfg1
    cc, ctx = make(H, t1, t2, PRECS[prec][0], tol=1e-10)
    try:
        Xs = [s.dipole(pb, k).numpy() for k in range(3)]
        z = 0.1 + 0.005j
        a_ref = ref.response(Xs, z)
        rc, out, info = cc.cclr_response_function(ctx, [dev(X) for X in Xs], [z.real], [z.imag])
        e_big, e_small, e_f = alpha_errors(out[0], a_ref)
        print(f"{prec}-refined response: entries rel {e_big:.2e}, small {e_small:.2e}, Frobenius {e_f:.2e}, "
              f"info {info.as_dict()}", flush=True)
        assert rc == 0 and max(e_big, e_small, e_f) < 1e-6
    finally:
        cc.cclr_destroy(ctx)
