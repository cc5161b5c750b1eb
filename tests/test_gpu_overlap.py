"""Right transforms with the ring and ladder products on a second stream
(concurrent with the other products) against the same transforms on one
stream, and against the oracle on the small case.  The kernels and their
order on each stream are the same, so the results must agree to rounding;
(4, 130) with 2 vectors splits the ring product along K, whose workspace the
arena must keep until the streams are joined."""
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


@pytest.fixture(scope="module")
def cc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2307_14296_amd as m
    m.lib().cclr_dbg_set_overlap.argtypes = [ctypes.c_void_p, ctypes.c_int]
    return m


def gpu_ctx(cc, o, v, seed):
    d = torch.device("cuda")
    pb = s.Problem(o, v, seed)
    with torch.no_grad():
        f = s.fock(pb, d)
        V = s.integral_blocks(pb, d, chunk=8)
        t1 = s.t1_amplitudes(pb, d)
        t2 = s.t2_amplitudes(pb, V["oovv"], d)
    ctx = cc.cclr_create(o, v, cc.cclr_default_options())
    cc.cclr_set_hamiltonian(ctx, f, *[V[k] for k in s.CANONICAL_BLOCKS])
    cc.cclr_set_amplitudes(ctx, t1, t2)
    return ctx, pb


@pytest.mark.parametrize("o,v,nv", [(6, 30, 3), (4, 130, 2), (20, 120, 5)])
def test_overlap_equals_one_stream(cc, o, v, nv):
    ctx, pb = gpu_ctx(cc, o, v, 31)
    L = cc.lib()
    try:
        x = [s.excitation_vector(pb, k, torch.device("cuda")) for k in range(nv)]
        r1 = torch.stack([a for a, _ in x]).contiguous()
        r2 = torch.stack([b for _, b in x]).contiguous()
        om, ga = [0.0774 + 0.01 * k for k in range(nv)], [0.005] * nv
        out = {}
        for mode in (0, 1, 0, 1):
            assert L.cclr_dbg_set_overlap(ctx, mode) == 0
            s1, s2 = torch.empty_like(r1), torch.empty_like(r2)
            cc.cclr_jacobian_right(ctx, om, ga, r1, r2, s1, s2)
            out.setdefault(mode, []).append((s1.cpu().numpy(), s2.cpu().numpy()))
        ref = out[0][0]
        for mode in (0, 1):
            for got in out[mode]:
                e = max(rel(got[0], ref[0]), rel(got[1], ref[1]))
                print(f"o={o} v={v} {nv} vectors, overlap={mode}: rel diff to one stream {e:.1e}", flush=True)
                assert e <= 1e-14
    finally:
        cc.cclr_destroy(ctx)


def test_overlap_matches_oracle(cc):
    o, v = 4, 16
    pb, inst, H, t1, t2 = config_problem(o, v, 3)
    ctx = cc.cclr_create(o, v, cc.cclr_default_options())
    try:
        keep = [dev(H.f)] + [dev(H.blocks[k]) for k in s.CANONICAL_BLOCKS] + [dev(t1), dev(t2)]
        cc.cclr_set_hamiltonian(ctx, *keep[:7])
        cc.cclr_set_amplitudes(ctx, *keep[7:])
        assert cc.lib().cclr_dbg_set_overlap(ctx, 1) == 0
        ref = O.CCLR(H, t1, t2)
        z = 0.0774 + 0.005j
        xs = [vec(pb, k) for k in range(2)]
        r1 = dev(np.stack([a for a, _ in xs]))
        r2 = dev(np.stack([b for _, b in xs]))
        s1, s2 = torch.empty_like(r1), torch.empty_like(r2)
        cc.cclr_jacobian_right(ctx, [z.real] * 2, [z.imag] * 2, r1, r2, s1, s2)
        for k in range(2):
            e = rel((s1[k].cpu().numpy(), s2[k].cpu().numpy()), ref.right(*xs[k], z))
            print(f"overlapped transform vector {k} vs oracle: rel err {e:.2e}", flush=True)
            assert e < 1e-10
    finally:
        cc.cclr_destroy(ctx)
