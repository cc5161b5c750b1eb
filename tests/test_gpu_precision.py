"""Mixed-precision path: the ladder and ring products on FP32 MFMA inside the
inner solves, FP64 true residuals (iterative refinement).  Bars: a
low-precision transform is within 1e-5 relative of the FP64 oracle; the
refined response function is within 1e-6 relative of the FP64 oracle (the
stated mixed-precision bar) — here it reaches the FP64 tolerance."""
import ctypes

import numpy as np
import pytest
import torch

from gen import synth as s
from helpers import config_problem, rel, vec
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


def test_fp32_transform_accuracy(cfg1):
    pb, H, t1, t2, ref = cfg1
    import paper_2307_14296_amd as cc0
    cc, ctx = make(H, t1, t2, cc0.CCLR_FP32)
    try:
        L = cc.lib()
        L.cclr_dbg_set_sigma_prec.argtypes = [ctypes.c_void_p, ctypes.c_int]
        assert L.cclr_dbg_set_sigma_prec(ctx, cc.CCLR_FP32) == 0
        xs = [vec(pb, k) for k in range(3)]
        r1, r2 = dev(np.stack([x[0] for x in xs])), dev(np.stack([x[1] for x in xs]))
        for fn, side in ((cc.cclr_jacobian_right, ref.right), (cc.cclr_jacobian_left, ref.left)):
            s1, s2 = torch.empty_like(r1), torch.empty_like(r2)
            fn(ctx, [0.1] * 3, [0.005] * 3, r1, r2, s1, s2)
            for k, x in enumerate(xs):
                e = rel((s1[k].cpu().numpy(), s2[k].cpu().numpy()), side(*x, 0.1 + 0.005j))
                print(f"fp32 {fn.__name__}: rel err {e:.2e}", flush=True)
                assert 1e-12 < e < 1e-5   # really low precision, and accurate to it
        L.cclr_dbg_set_sigma_prec(ctx, cc.CCLR_FP64)
    finally:
        cc.cclr_destroy(ctx)


def test_fp32_refined_response(cfg1):
    pb, H, t1, t2, ref = cfg1
    import paper_2307_14296_amd as cc0
    cc, ctx = make(H, t1, t2, cc0.CCLR_FP32, tol=1e-10)
    try:
        Xs = [s.dipole(pb, k).numpy() for k in range(3)]
        z = 0.1 + 0.005j
        a_ref = ref.response(Xs, z)
        rc, out, info = cc.cclr_response_function(ctx, [dev(X) for X in Xs], [z.real], [z.imag])
        e = np.linalg.norm(out[0] - a_ref) / np.linalg.norm(a_ref)
        print(f"fp32-refined response: rel err {e:.2e}, info {info.as_dict()}", flush=True)
        assert rc == 0 and e < 1e-6
    finally:
        cc.cclr_destroy(ctx)
