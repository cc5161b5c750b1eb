"""Building blocks of the GPU library against plain numpy on the same inputs:
the complex FP64-MFMA GEMM (layouts, ragged tiles, conjugation, alpha,
accumulate), the contraction engine on the index patterns the schedule uses,
and every Hbar intermediate against the oracle's."""
import ctypes

import numpy as np
import pytest
import torch

from helpers import small_problem
from oracle import cclr_ref as O

pytestmark = pytest.mark.gpu


def _cc():
    import paper_2307_14296_amd as cc
    L = cc.lib()
    LL = ctypes.c_longlong
    P = ctypes.c_void_p
    L.cclr_dbg_zgemm.argtypes = [ctypes.c_int] * 4 + [P, LL, LL, LL, ctypes.c_int, P, LL, LL, LL, ctypes.c_int,
                                                       P, LL, LL, LL, ctypes.c_double, ctypes.c_double, ctypes.c_int]
    L.cclr_dbg_contract.argtypes = [P, ctypes.c_double, ctypes.c_double, P, ctypes.c_char_p, ctypes.POINTER(LL),
                                    P, ctypes.c_char_p, ctypes.POINTER(LL), P, ctypes.c_char_p, ctypes.POINTER(LL)]
    L.cclr_dbg_get.argtypes = [P, ctypes.c_char_p, P, ctypes.POINTER(LL)]
    return cc, L


def crand(rng, *shape):
    return rng.normal(size=shape) + 1j * rng.normal(size=shape)


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x)).to(torch.complex128).cuda()


@pytest.fixture(scope="module")
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


GEMM_CASES = [
    (16, 16, 4, False, False), (64, 64, 16, False, False), (1, 1, 1, False, False), (17, 33, 5, True, False),
    (100, 70, 40, False, True), (130, 3, 129, True, True), (5, 200, 66, False, False),
]


@pytest.mark.parametrize("M,N,K,ta,tb", GEMM_CASES)
def test_zgemm(gpu, M, N, K, ta, tb):
    cc, L = _cc()
    rng = np.random.default_rng(M * 1000 + N * 10 + K)
    A = crand(rng, M, K)
    B = crand(rng, K, N)
    C0 = crand(rng, M, N)
    alpha = 0.7 - 0.3j
    for conjA, conjB, beta in [(0, 0, 0), (1, 0, 1), (0, 1, 1), (1, 1, 0)]:
        Ad = dev(A.T.copy() if ta else A)
        Bd = dev(B.T.copy() if tb else B)
        Cd = dev(C0)
        sAm, sAk = (1, M) if ta else (K, 1)
        sBk, sBn = (1, K) if tb else (N, 1)
        rc = L.cclr_dbg_zgemm(M, N, K, 1, Ad.data_ptr(), 0, sAm, sAk, conjA, Bd.data_ptr(), 0, sBk, sBn, conjB,
                              Cd.data_ptr(), 0, N, 1, alpha.real, alpha.imag, beta)
        assert rc == 0
        a = A.conj() if conjA else A
        b = B.conj() if conjB else B
        ref = alpha * (a @ b) + (C0 if beta else 0)
        got = Cd.cpu().numpy()
        assert np.abs(got - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max()), (conjA, conjB, beta)


VARIANT_CASES = [(1, 1, 1, 1), (130, 70, 33, 3), (300, 200, 50, 1), (257, 1, 64, 2), (64, 640, 17, 5),
                 (1100, 65, 40, 1), (260, 300, 70, 2), (129, 257, 160, 1), (5, 130, 15, 2)]


@pytest.mark.parametrize("M,N,K,batch", VARIANT_CASES)
def test_zgemm_every_variant(gpu, M, N, K, batch):
    """Every FP64 kernel variant and tile order (the autotuner runs only the
    fastest), batched, ragged tails, both operand orientations."""
    cc, L = _cc()
    LL, P = ctypes.c_longlong, ctypes.c_void_p
    L.cclr_dbg_zgemm_f64.argtypes = [ctypes.c_int] * 5 + [P, LL, LL, LL, ctypes.c_int, P, LL, LL, LL, ctypes.c_int,
                                                          P, LL, LL, LL, ctypes.c_double, ctypes.c_double,
                                                          ctypes.c_int]
    rng = np.random.default_rng(M * 31 + N * 7 + K + batch)
    A = crand(rng, batch, M, K)
    B = crand(rng, batch, K, N)
    C0 = crand(rng, batch, M, N)
    alpha = 0.3 + 1.1j
    # 100 + v: variant v on the transposed product (the autotuner's choice for 32-column tiles on short m sides)
    for variant in list(range(21)) + [101, 103, 116, 119, 120]:
        for ta, tb, beta, cj in [(False, False, 0, 1), (True, True, 1, 0), (False, True, 1, 1), (True, False, 0, 0),
                                 (False, True, 0, 0), (True, False, 1, 1)]:
            Ad = dev(A.transpose(0, 2, 1).copy() if ta else A)
            Bd = dev(B.transpose(0, 2, 1).copy() if tb else B)
            Cd = dev(C0)
            sAm, sAk = (1, M) if ta else (K, 1)
            sBk, sBn = (1, K) if tb else (N, 1)
            rc = L.cclr_dbg_zgemm_f64(variant, batch, M, N, K, Ad.data_ptr(), M * K, sAm, sAk, 0, Bd.data_ptr(),
                                      K * N, sBk, sBn, cj, Cd.data_ptr(), M * N, N, 1, alpha.real, alpha.imag, beta)
            assert rc == 0
            ref = alpha * (A @ (B.conj() if cj else B)) + (C0 if beta else 0)
            err = np.abs(Cd.cpu().numpy() - ref).max() / max(1.0, np.abs(ref).max())
            assert err <= 1e-12, (variant, ta, tb, beta, cj, err)


@pytest.mark.parametrize("M,N,K,kchunk", [(130, 70, 200, 48), (257, 129, 130, 64), (5, 300, 97, 32)])
def test_zgemm_split_k_every_variant(gpu, M, N, K, kchunk):
    """The split-K form (one partial product per K chunk, the last chunk
    ragged) of every MFMA variant, both operand orientations, against numpy
    chunk by chunk."""
    cc, L = _cc()
    LL, P = ctypes.c_longlong, ctypes.c_void_p
    L.cclr_dbg_zgemm_f64_splitk.argtypes = [ctypes.c_int] * 5 + [P, LL, LL, P, LL, LL, P]
    rng = np.random.default_rng(M + 3 * N + 7 * K + kchunk)
    A = crand(rng, M, K)
    B = crand(rng, K, N)
    S = (K + kchunk - 1) // kchunk
    ref = np.stack([A[:, s * kchunk:(s + 1) * kchunk] @ B[s * kchunk:(s + 1) * kchunk] for s in range(S)])
    for variant in range(1, 21):
        for ta, tb in [(False, False), (False, True), (True, False)]:
            Ad = dev(A.T.copy() if ta else A)
            Bd = dev(B.T.copy() if tb else B)
            Wd = torch.full((S, M, N), 3.0 + 0j, dtype=torch.complex128, device="cuda")
            sAm, sAk = (1, M) if ta else (K, 1)
            sBk, sBn = (1, K) if tb else (N, 1)
            rc = L.cclr_dbg_zgemm_f64_splitk(variant, M, N, K, kchunk, Ad.data_ptr(), sAm, sAk, Bd.data_ptr(), sBk,
                                             sBn, Wd.data_ptr())
            assert rc == 0
            err = np.abs(Wd.cpu().numpy() - ref).max() / max(1.0, np.abs(ref).max())
            assert err <= 1e-12, (variant, ta, tb, err)


@pytest.mark.parametrize("variant", [1, 2, 3, 4, 13, 15])
def test_zgemm_grouped_persistent_launch(gpu, variant):
    """The persistent grouped launch (several products of different shapes
    dealt as one tile sequence) in every tile shape that has a grouped form,
    both B orientations, against numpy per product."""
    cc, L = _cc()
    P = ctypes.c_void_p
    L.cclr_dbg_zgemm_group_f64.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                           ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                           ctypes.POINTER(P), ctypes.POINTER(P), ctypes.c_int, ctypes.POINTER(P)]
    # the last product alone has more 128x128 tiles than there are workgroups (256), so some
    # workgroups run several tiles, some with a K remainder
    shapes = [(257, 300, 140), (130, 70, 33), (64, 129, 17), (300, 260, 50), (1, 1, 1), (2100, 2100, 20)]
    rng = np.random.default_rng(17 + variant)
    for bt in (0, 1):
        As = [crand(rng, m, k) for m, n, k in shapes]
        Bs = [crand(rng, n, k) if bt else crand(rng, k, n) for m, n, k in shapes]
        Ad, Bd = [dev(a) for a in As], [dev(b) for b in Bs]
        Cd = [torch.full((m, n), 7.0 + 0j, dtype=torch.complex128, device="cuda") for m, n, k in shapes]
        ints = lambda xs: (ctypes.c_int * len(xs))(*xs)
        ptrs = lambda ts: (P * len(ts))(*[t.data_ptr() for t in ts])
        rc = L.cclr_dbg_zgemm_group_f64(variant, len(shapes), ints([m for m, n, k in shapes]),
                                        ints([n for m, n, k in shapes]), ints([k for m, n, k in shapes]),
                                        ptrs(Ad), ptrs(Bd), bt, ptrs(Cd))
        assert rc == 0
        for (m, n, k), a, b, c in zip(shapes, As, Bs, Cd):
            ref = a @ (b.T if bt else b)
            err = np.abs(c.cpu().numpy() - ref).max() / max(1.0, np.abs(ref).max())
            assert err <= 1e-12, (variant, bt, (m, n, k), err)
    # the single-buffer tiles have no grouped form
    assert L.cclr_dbg_zgemm_group_f64(9, 1, ints([1]), ints([1]), ints([1]), ptrs(Ad[:1]), ptrs(Bd[:1]), 0,
                                      ptrs(Cd[:1])) == cc.CCLR_EINVAL


# (M, N, K, batch): narrow outputs (either side, with and without the split
# along K), short reductions, split-K and plain MFMA products
DISPATCH_CASES = [(20, 300, 5000, 1), (300, 20, 700, 3), (3, 1000, 700, 2), (1, 240, 4000, 5), (40, 16, 100000, 1),
                  (4000, 12, 4000, 1), (33, 2000, 900, 1), (200, 200, 20, 7), (150, 140, 30000, 2),
                  (500, 300, 260, 2),
                  # at most 16 output columns (short-output kernel, direct and transposed, split and whole
                  # reductions, ragged row blocks and K chunks); 17 and more stay on MFMA
                  (16, 300, 2000, 3), (300, 16, 2000, 2), (260, 9, 5000, 4), (5000, 3, 40, 3), (70, 1, 129, 2),
                  (2, 500, 300, 2), (300, 6, 1000, 1),
                  (24, 700, 3000, 2), (130, 17, 129, 2),
                  # at most 8 output columns with the long operand contiguous in k (row-dot kernel, direct and
                  # transposed, split and whole reductions, ragged row blocks and K chunks)
                  (700, 2, 2000, 1), (1, 300, 3000, 2), (5, 257, 1500, 1), (1000, 8, 700, 2),
                  # at most 32 output columns or rows on the 32-column MFMA tiles (a short m side runs transposed)
                  (2000, 20, 200, 1), (20, 3000, 400, 2), (32, 1500, 64, 1),
                  # short reductions of every length class (K rounded up to a multiple of 4), ragged row blocks
                  (70, 300, 5, 2), (100, 600, 12, 1), (33, 257, 32, 3), (45, 130, 17, 2), (40, 270, 1, 2),
                  (60, 300, 20, 3), (35, 260, 23, 1), (50, 280, 27, 2), (70, 290, 8, 1), (36, 300, 14, 2)]


@pytest.mark.parametrize("M,N,K,batch", DISPATCH_CASES)
def test_run_gemm_dispatch(gpu, M, N, K, batch):
    """The context's GEMM dispatch (the path every contraction takes) on the
    shapes that select each kernel form, with conjugation, complex alpha and
    accumulation, and a transposed output layout."""
    cc, L = _cc()
    LL, P = ctypes.c_longlong, ctypes.c_void_p
    L.cclr_dbg_run_gemm.argtypes = [P] + [ctypes.c_int] * 4 + [P, LL, LL, LL, ctypes.c_int, P, LL, LL, LL,
                                                               ctypes.c_int, P, LL, LL, LL, ctypes.c_double,
                                                               ctypes.c_double, ctypes.c_int]
    ctx = cc.cclr_create(3, 6, cc.cclr_default_options())
    try:
        rng = np.random.default_rng(M + 7 * N + K + batch)
        for ta, tb, conjA, conjB, beta, tc in [(False, False, 0, 1, 0, False), (True, False, 1, 0, 1, True),
                                               (False, True, 1, 1, 1, False)]:
            A = crand(rng, batch, M, K)
            B = crand(rng, batch, K, N)
            C0 = crand(rng, batch, M, N)
            Ad = dev(A.transpose(0, 2, 1).copy() if ta else A)
            Bd = dev(B.transpose(0, 2, 1).copy() if tb else B)
            Cd = dev(C0.transpose(0, 2, 1).copy() if tc else C0)
            sAm, sAk = (1, M) if ta else (K, 1)
            sBk, sBn = (1, K) if tb else (N, 1)
            sCm, sCn = (1, M) if tc else (N, 1)
            alpha = 0.7 - 0.4j
            rc = L.cclr_dbg_run_gemm(ctx, M, N, K, batch, Ad.data_ptr(), M * K, sAm, sAk, conjA, Bd.data_ptr(), K * N,
                                     sBk, sBn, conjB, Cd.data_ptr(), M * N, sCm, sCn, alpha.real, alpha.imag, beta)
            assert rc == 0
            Ae = A.conj() if conjA else A
            Be = B.conj() if conjB else B
            ref = alpha * (Ae @ Be) + (C0 if beta else 0)
            got = Cd.cpu().numpy()
            if tc:
                got = got.transpose(0, 2, 1)
            err = np.abs(got - ref).max() / np.abs(ref).max()
            print(f"run_gemm {M}x{N}x{K} b{batch} ta={ta} tb={tb} conj=({conjA},{conjB}) beta={beta}: "
                  f"rel err {err:.1e}", flush=True)
            assert err <= 1e-12
    finally:
        cc.cclr_destroy(ctx)


# (M, N, K, batch, A stored transposed, B stored transposed, kernel form the dispatch must choose):
# -6 row-dot kernel, -4 short-output kernel, 19 the 128x32 MFMA tile (untimed choice for at most 32 columns)
FORM_CASES = [(700, 2, 2000, 1, False, False, -6), (700, 2, 2000, 1, True, False, -4),
              (1, 300, 3000, 2, False, True, -6), (1, 300, 3000, 2, False, False, -4),
              (1000, 8, 700, 2, False, False, -6), (2000, 20, 200, 1, False, False, 19),
              (20, 3000, 400, 2, False, False, 19), (32, 1500, 64, 1, True, True, 19)]


@pytest.mark.parametrize("M,N,K,batch,ta,tb,form", FORM_CASES)
def test_run_gemm_form_choice(gpu, M, N, K, batch, ta, tb, form):
    """The dispatch picks the row-dot kernel for at most 8 columns on a long
    operand contiguous in k (directly, or after transposing a product with
    a short m side), and the 32-column MFMA tiles for outputs at most 32
    wide (a short m side transposed first); the result is checked too."""
    cc, L = _cc()
    LL, P = ctypes.c_longlong, ctypes.c_void_p
    L.cclr_dbg_run_gemm.argtypes = [P] + [ctypes.c_int] * 4 + [P, LL, LL, LL, ctypes.c_int, P, LL, LL, LL,
                                                               ctypes.c_int, P, LL, LL, LL, ctypes.c_double,
                                                               ctypes.c_double, ctypes.c_int]
    L.cclr_dbg_gemm_trace.argtypes = [P, ctypes.c_int, ctypes.c_char_p, ctypes.c_longlong]
    ctx = cc.cclr_create(3, 6, cc.cclr_default_options())
    try:
        rng = np.random.default_rng(M + 5 * N + K)
        A = crand(rng, batch, M, K)
        B = crand(rng, batch, K, N)
        Ad = dev(A.transpose(0, 2, 1).copy() if ta else A)
        Bd = dev(B.transpose(0, 2, 1).copy() if tb else B)
        Cd = torch.zeros((batch, M, N), dtype=torch.complex128, device="cuda")
        sAm, sAk = (1, M) if ta else (K, 1)
        sBk, sBn = (1, K) if tb else (N, 1)
        assert L.cclr_dbg_gemm_trace(ctx, 1, None, 0) == 0
        rc = L.cclr_dbg_run_gemm(ctx, M, N, K, batch, Ad.data_ptr(), M * K, sAm, sAk, 0, Bd.data_ptr(), K * N, sBk,
                                 sBn, 0, Cd.data_ptr(), M * N, N, 1, 1.0, 0.0, 0)
        assert rc == 0
        buf = ctypes.create_string_buffer(1 << 16)
        assert L.cclr_dbg_gemm_trace(ctx, 0, buf, len(buf)) == 0
        lines = [ln for ln in buf.value.decode().splitlines() if ln]
        print(lines, flush=True)
        assert len(lines) == 1 and int(lines[0].split(" form ")[1].split()[0]) == form, lines
        ref = A @ B
        err = np.abs(Cd.cpu().numpy() - ref).max() / np.abs(ref).max()
        assert err <= 1e-12, err
    finally:
        cc.cclr_destroy(ctx)


@pytest.mark.parametrize("M,N,K,batch,inner", [(200, 400, 20, 20, "C"), (100, 120, 64, 100, "BC"),
                                                (300, 50, 80, 60, "A"), (70, 90, 40, 200, "ABC")])
def test_run_gemm_batch_innermost(gpu, M, N, K, batch, inner):
    """Products whose operands or output have the batch index as their unit
    stride (the dispatch copies them to a batch-outermost layout and adds the
    output back), with conjugation, complex alpha and accumulation."""
    cc, L = _cc()
    LL, P = ctypes.c_longlong, ctypes.c_void_p
    L.cclr_dbg_run_gemm.argtypes = [P] + [ctypes.c_int] * 4 + [P, LL, LL, LL, ctypes.c_int, P, LL, LL, LL,
                                                               ctypes.c_int, P, LL, LL, LL, ctypes.c_double,
                                                               ctypes.c_double, ctypes.c_int]
    ctx = cc.cclr_create(3, 6, cc.cclr_default_options())
    try:
        rng = np.random.default_rng(M + N + K + batch)
        A = crand(rng, batch, M, K)
        B = crand(rng, batch, K, N)
        C0 = crand(rng, batch, M, N)

        def store(X, innermost):
            # device copy and its (batch, row, column) strides
            b, r, q = X.shape
            if innermost:
                return dev(X.transpose(1, 2, 0).copy()), (1, q * b, b)
            return dev(X), (r * q, q, 1)

        Ad, (sAb, sAm, sAk) = store(A, "A" in inner)
        Bd, (sBb, sBk, sBn) = store(B, "B" in inner)
        Cd, (sCb, sCm, sCn) = store(C0, "C" in inner)
        alpha = -0.6 + 0.9j
        rc = L.cclr_dbg_run_gemm(ctx, M, N, K, batch, Ad.data_ptr(), sAb, sAm, sAk, 1, Bd.data_ptr(), sBb, sBk, sBn, 0,
                                 Cd.data_ptr(), sCb, sCm, sCn, alpha.real, alpha.imag, 1)
        assert rc == 0
        got = Cd.cpu().numpy()
        if "C" in inner:
            got = got.transpose(2, 0, 1)
        ref = alpha * (A.conj() @ B) + C0
        err = np.abs(got - ref).max() / np.abs(ref).max()
        print(f"batch-innermost {inner} {M}x{N}x{K} b{batch}: rel err {err:.1e}", flush=True)
        assert err <= 1e-12
    finally:
        cc.cclr_destroy(ctx)


@pytest.mark.parametrize("M,N,K,nb1,nb2,inner,shared_b", [(60, 100, 50, 4, 50, "AC", False),
                                                            (100, 80, 30, 3, 70, "C", True),
                                                            (90, 70, 40, 2, 120, "B", False)])
def test_run_gemm_two_level_batch_innermost(gpu, M, N, K, nb1, nb2, inner, shared_b):
    """Two-level batches (b = b1 nb2 + b2) whose second index is the unit
    stride of an operand or of the output, one case with B shared over b2
    (stride 0), through the dispatch's batch-outermost copies."""
    cc, L = _cc()
    LL, P = ctypes.c_longlong, ctypes.c_void_p
    L.cclr_dbg_run_gemm_b2.argtypes = [P] + [ctypes.c_int] * 5 + [P, LL, LL, LL, LL, P, LL, LL, LL, LL, P, LL, LL,
                                                                  LL, LL, ctypes.c_double, ctypes.c_double,
                                                                  ctypes.c_int]
    ctx = cc.cclr_create(3, 6, cc.cclr_default_options())
    try:
        rng = np.random.default_rng(M + N + K + nb1 + nb2)
        A = crand(rng, nb1, nb2, M, K)
        B = crand(rng, nb1, 1 if shared_b else nb2, K, N)
        C0 = crand(rng, nb1, nb2, M, N)

        def store(X, innermost):
            # device copy and its (b1, b2, row, column) strides
            b1, b2, r, q = X.shape
            if innermost:
                return dev(X.transpose(0, 2, 3, 1).copy()), (r * q * b2, 1, q * b2, b2)
            return dev(X), (b2 * r * q, 0 if b2 == 1 else r * q, q, 1)

        Ad, (sAb, sAb2, sAm, sAk) = store(A, "A" in inner)
        Bd, (sBb, sBb2, sBk, sBn) = store(B, "B" in inner)
        Cd, (sCb, sCb2, sCm, sCn) = store(C0, "C" in inner)
        alpha = 0.4 - 1.3j
        rc = L.cclr_dbg_run_gemm_b2(ctx, M, N, K, nb1, nb2, Ad.data_ptr(), sAb, sAb2, sAm, sAk, Bd.data_ptr(), sBb,
                                    sBb2, sBk, sBn, Cd.data_ptr(), sCb, sCb2, sCm, sCn, alpha.real, alpha.imag, 1)
        assert rc == 0
        got = Cd.cpu().numpy()
        if "C" in inner:
            got = got.transpose(0, 3, 1, 2)
        ref = alpha * (A @ B) + C0
        err = np.abs(got - ref).max() / np.abs(ref).max()
        print(f"two-level batch {inner} {M}x{N}x{K} b{nb1}x{nb2}: rel err {err:.1e}", flush=True)
        assert err <= 1e-12
    finally:
        cc.cclr_destroy(ctx)


@pytest.mark.parametrize("M,N,K,batch", [(600, 530, 300, 1), (512, 700, 256, 1), (600, 530, 300, 2), (300, 530, 300, 1)])
def test_run_gemm_dispatch_fp32(gpu, M, N, K, batch):
    """The context's GEMM dispatch inside a reduced-precision transform (FP32
    arithmetic): large single products on pre-split FP32 planes, batched or
    narrower ones on the in-kernel conversion, with conjugation, complex
    alpha, accumulation and a transposed output, within FP32 accuracy
    (relative Frobenius error below 1e-5, and above 1e-12: FP32 really ran)."""
    cc, L = _cc()
    LL, P = ctypes.c_longlong, ctypes.c_void_p
    L.cclr_dbg_run_gemm.argtypes = [P] + [ctypes.c_int] * 4 + [P, LL, LL, LL, ctypes.c_int, P, LL, LL, LL,
                                                               ctypes.c_int, P, LL, LL, LL, ctypes.c_double,
                                                               ctypes.c_double, ctypes.c_int]
    L.cclr_dbg_set_sigma_prec.argtypes = [P, ctypes.c_int]
    ctx = cc.cclr_create(3, 6, cc.cclr_default_options())
    try:
        assert L.cclr_dbg_set_sigma_prec(ctx, cc.CCLR_FP32) == 0
        rng = np.random.default_rng(M + 7 * N + K + batch)
        for ta, conjA, conjB, beta, tc in [(False, 0, 1, 0, False), (True, 1, 0, 1, True), (False, 1, 1, 1, False)]:
            A = crand(rng, batch, M, K)
            B = crand(rng, batch, K, N)
            C0 = crand(rng, batch, M, N)
            Ad = dev(A.transpose(0, 2, 1).copy() if ta else A)
            Bd = dev(B)
            Cd = dev(C0.transpose(0, 2, 1).copy() if tc else C0)
            sAm, sAk = (1, M) if ta else (K, 1)
            sCm, sCn = (1, M) if tc else (N, 1)
            alpha = 0.7 - 0.4j
            rc = L.cclr_dbg_run_gemm(ctx, M, N, K, batch, Ad.data_ptr(), M * K, sAm, sAk, conjA, Bd.data_ptr(), K * N,
                                     N, 1, conjB, Cd.data_ptr(), M * N, sCm, sCn, alpha.real, alpha.imag, beta)
            assert rc == 0
            Ae = A.conj() if conjA else A
            Be = B.conj() if conjB else B
            prod = alpha * (Ae @ Be)
            got = Cd.cpu().numpy()
            if tc:
                got = got.transpose(0, 2, 1)
            got = got - (C0 if beta else 0)
            err = np.linalg.norm(got - prod) / np.linalg.norm(prod)
            print(f"run_gemm FP32 {M}x{N}x{K} b{batch} ta={ta} conj=({conjA},{conjB}) beta={beta}: rel err {err:.1e}",
                  flush=True)
            assert 1e-12 < err < 1e-5
    finally:
        cc.cclr_destroy(ctx)


def test_zgemm_batched_and_transposed_output(gpu):
    cc, L = _cc()
    rng = np.random.default_rng(5)
    nb, M, N, K = 3, 37, 21, 19
    A = crand(rng, nb, M, K)
    B = crand(rng, nb, K, N)
    Cd = dev(np.zeros((nb, N, M)))
    Ad, Bd = dev(A), dev(B)
    rc = L.cclr_dbg_zgemm(M, N, K, nb, Ad.data_ptr(), M * K, K, 1, 0, Bd.data_ptr(), K * N, N, 1, 0,
                          Cd.data_ptr(), M * N, 1, M, 1.0, 0.0, 0)
    assert rc == 0
    ref = np.einsum("bmk,bkn->bnm", A, B)
    assert np.abs(Cd.cpu().numpy() - ref).max() <= 1e-12 * np.abs(ref).max()


CONTRACT_CASES = [
    ("ae", "kie", "kia", dict(a=5, e=5, k=2, i=3)),
    ("mbej", "kimae", "kijab", dict(m=3, b=5, e=5, j=3, k=2, i=3, a=5)),
    ("maei", "kme", "kia", dict(m=3, a=5, e=5, i=3, k=2)),
    ("amef", "kimef", "kia", dict(a=5, m=3, e=5, f=5, k=2, i=3)),
    ("mnie", "kmnea", "kia", dict(m=3, n=3, i=3, e=5, a=5, k=2)),
    ("ijaf", "kbf", "kijab", dict(i=3, j=3, a=5, f=5, k=2, b=5)),
    ("inef", "mnef", "im", dict(i=3, n=3, e=5, f=5, m=3)),
    ("ia", "jb", "ijab", dict(i=3, a=5, j=3, b=5)),
    ("efag", "mg", "efam", dict(e=5, f=5, a=5, g=5, m=3)),
    ("kmnaf", "mnef", "kea", dict(k=2, m=3, n=3, a=5, f=5, e=5)),
    # tiny output, long reduction: exercises the split-K path
    ("inef", "mnef", "im", dict(i=3, n=40, e=30, f=31, m=5)),
    ("kimfe", "nmfe", "kni", dict(k=2, i=4, m=9, f=60, e=61, n=7)),
    # output groups broken by the other operand's labels: one or two free batch indices
    ("mj", "kimab", "kijab", dict(m=3, j=3, k=2, i=3, a=5, b=5)),
    ("me", "kimea", "kia", dict(m=3, e=5, k=2, i=3, a=5)),
    ("mnie", "kmnea", "kia", dict(m=3, n=3, i=3, e=5, a=5, k=3)),
    ("mbij", "kma", "kijab", dict(m=3, b=5, i=3, j=3, k=2, a=5)),
    ("abej", "kie", "kijab", dict(a=5, b=5, e=7, j=3, k=2, i=3)),
    ("inab", "knj", "kijab", dict(i=3, n=4, a=5, b=5, k=2, j=3)),
]


@pytest.mark.parametrize("la,lb,lc,sz", CONTRACT_CASES, ids=[f"{a},{b}->{c}" for a, b, c, _ in CONTRACT_CASES])
def test_contract(gpu, la, lb, lc, sz):
    cc, L = _cc()
    rng = np.random.default_rng(len(la) * 7 + len(lb))
    A = crand(rng, *[sz[ch] for ch in la])
    B = crand(rng, *[sz[ch] for ch in lb])
    C = crand(rng, *[sz[ch] for ch in lc])
    ctx = cc.cclr_create(2, 2)
    try:
        LL = ctypes.c_longlong
        dims = lambda x: (LL * x.ndim)(*x.shape)  # noqa: E731
        Ad, Bd, Cd = dev(A), dev(B), dev(C)
        alpha = -0.5 + 0.25j
        rc = L.cclr_dbg_contract(ctx, alpha.real, alpha.imag, Ad.data_ptr(), la.encode(), dims(A), Bd.data_ptr(),
                                 lb.encode(), dims(B), Cd.data_ptr(), lc.encode(), dims(C))
        assert rc == 0, cc.cclr_last_error(ctx)
        ref = C + alpha * np.einsum(f"{la},{lb}->{lc}", A, B)
        assert np.abs(Cd.cpu().numpy() - ref).max() <= 1e-12 * np.abs(ref).max()
    finally:
        cc.cclr_destroy(ctx)


@pytest.mark.parametrize("o,v", [(2, 3), (3, 5)])
def test_intermediates(gpu, o, v):
    from gen import synth as s
    cc, L = _cc()
    pb, Vf, f, H, t1, t2 = small_problem(o, v)
    hb = O.hbar(H, t1, t2)
    ctx = cc.cclr_create(o, v)
    try:
        keep = [dev(H.f)] + [dev(H.blocks[k]) for k in s.CANONICAL_BLOCKS]
        cc.cclr_set_hamiltonian(ctx, *keep)
        tt = [dev(t1), dev(t2)]
        cc.cclr_set_amplitudes(ctx, *tt)
        bad = []
        for name, ref in hb.items():
            n = ctypes.c_longlong()
            assert L.cclr_dbg_get(ctx, name.encode(), None, ctypes.byref(n)) == 0
            out = torch.empty(n.value, dtype=torch.complex128, device="cuda")
            assert L.cclr_dbg_get(ctx, name.encode(), out.data_ptr(), None) == 0
            got = out.cpu().numpy().reshape(ref.shape)
            err = np.abs(got - ref).max() / max(1e-300, np.abs(ref).max())
            print(f"intermediate {name}: rel err {err:.2e}", flush=True)
            if not err < 1e-12:
                bad.append((name, err))
        assert not bad, bad
    finally:
        cc.cclr_destroy(ctx)


TCOPY_CASES = [
    ((100, 70), (1, 0)),            # 2-D transpose (LDS tiles, ragged edges)
    ((8, 40, 50), (2, 0, 1)),       # 3-D cyclic permutation
    ((6, 1, 33, 17, 5), (3, 1, 0, 4, 2)),  # unit extent, mixed sizes
    ((4, 5, 6, 7), (0, 1, 2, 3)),   # identity: all indices merge into one
    ((12, 9, 20), (0, 2, 1)),       # inner transpose with a batch index
    ((3, 7, 11), (2, 1, 0)),        # all extents below 16: element-wise path
    ((2, 3, 40, 2, 24, 3), (4, 1, 0, 5, 2, 3)),  # six indices, transpose of 40 and 24
]


@pytest.mark.parametrize("shape,perm", TCOPY_CASES)
def test_strided_copy_forms(gpu, shape, perm):
    """dst[i] = (acc ? dst : 0) + alpha op(src[P i]) for permutations through
    every form of the strided copy, with conjugation, accumulation and the
    alpha = 0 zero fill, against numpy."""
    cc, L = _cc()
    LL, P = ctypes.c_longlong, ctypes.c_void_p
    L.cclr_dbg_tcopy.argtypes = [ctypes.c_int, P, P, P, P, P, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                 ctypes.c_int]
    rng = np.random.default_rng(sum(shape) + 7 * len(shape))
    src = crand(rng, *shape)
    out_shape = tuple(shape[p] for p in perm)
    d0 = crand(rng, *out_shape)
    nd = len(shape)
    dims = (LL * nd)(*out_shape)
    sd = (LL * nd)(*[int(np.prod(out_shape[d + 1:])) for d in range(nd)])
    sstr = [int(np.prod(shape[d + 1:])) for d in range(nd)]
    ss = (LL * nd)(*[sstr[perm[d]] for d in range(nd)])
    want = np.transpose(src, perm)
    for alpha, conj, acc in [(1.0 + 0j, 0, 0), (0.5 - 2j, 1, 1), (0j, 0, 0)]:
        Sd, Dd = dev(src), dev(d0)
        rc = L.cclr_dbg_tcopy(nd, dims, sd, ss, Dd.data_ptr(), Sd.data_ptr(), alpha.real, alpha.imag, conj, acc)
        assert rc == 0
        ref = (d0 if acc else 0) + alpha * (want.conj() if conj else want)
        np.testing.assert_allclose(Dd.cpu().numpy(), ref, rtol=1e-14, atol=1e-14)
