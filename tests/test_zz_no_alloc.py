"""The right transform that allocates nothing (cclr_jacobian_right_noalloc).

It runs the same transform as cclr_jacobian_right with every temporary in the
library's fixed per-device work space.  Its output is compared with that of
cclr_jacobian_right element by element (and both with the oracle) on two
calls in a row, the second with a smaller input, then on a second context of
another size that reuses the same work space; sizes beyond the work space are
rejected without writing anything.
"""
import ctypes

import numpy as np
import pytest
import torch

from helpers import assert_blocks, config_problem, small_problem, vec

pytestmark = pytest.mark.gpu
TOL = 1e-10
WS_BYTES = 256 << 20


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x)).to(torch.complex128).cuda()


def host(t):
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def cc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2307_14296_amd as m
    m.lib().cclr_dbg_fixed_ws_peak.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_longlong)]
    return m


def context(cc, H, t1, t2):
    from gen import synth as s
    ctx = cc.cclr_create(H.o, H.v)
    cc.cclr_set_hamiltonian(ctx, dev(H.f), *[dev(H.blocks[k]) for k in s.CANONICAL_BLOCKS])
    cc.cclr_set_amplitudes(ctx, dev(t1), dev(t2))
    return ctx


def peak(cc, ctx):
    n = ctypes.c_longlong()
    assert cc.lib().cclr_dbg_fixed_ws_peak(ctx, ctypes.byref(n)) == 0
    return n.value


def both(cc, ctx, pb, o, v, ks, zs):
    r1 = np.stack([vec(pb, k)[0] for k in ks])
    r2 = np.stack([vec(pb, k)[1] for k in ks])
    n = len(ks)
    outs = []
    for fn in (cc.cclr_jacobian_right, cc.cclr_jacobian_right_noalloc):
        s1 = torch.full((n, o, v), complex(7.0, -7.0), dtype=torch.complex128, device="cuda")
        s2 = torch.full((n, o, o, v, v), complex(7.0, -7.0), dtype=torch.complex128, device="cuda")
        fn(ctx, [z.real for z in zs], [z.imag for z in zs], dev(r1), dev(r2), s1, s2)
        torch.cuda.synchronize()
        outs.append((host(s1), host(s2)))
    return r1, r2, outs


def test_noalloc_matches_jacobian_right(cc):
    o, v = 5, 24
    pb, _, _, H, t1, t2 = small_problem(o, v, seed=11)
    from oracle import cclr_ref as O
    ref = O.CCLR(H, t1, t2)
    ctx = context(cc, H, t1, t2)
    try:
        # first call: three vectors; second call: one vector (smaller input)
        for ks, zs in (([0, 1, 2], [0.1 + 0.005j, -0.3 + 0.0j, 0.0 + 0.02j]), ([3], [0.25 + 0.001j])):
            print(f"noalloc o={o} v={v} nvec={len(ks)}", flush=True)
            r1, r2, (plain, noalloc) = both(cc, ctx, pb, o, v, ks, zs)
            used = peak(cc, ctx)
            print(f"  work space peak {used} bytes ({used / len(ks) / (16 * o * o * v * v):.2f} full doubles "
                  f"tensors per vector)", flush=True)
            assert 0 < used <= WS_BYTES
            for k in range(len(ks)):
                assert_blocks((noalloc[0][k], noalloc[1][k]), (plain[0][k], plain[1][k]), TOL,
                              f"noalloc vs jacobian_right, vector {k}")
                e = ref.right(r1[k], r2[k], zs[k])
                assert_blocks((noalloc[0][k], noalloc[1][k]), e, TOL, f"noalloc vs oracle, vector {k}")
    finally:
        cc.cclr_destroy(ctx)


def test_noalloc_second_context_and_limits(cc):
    # a second context of another size reuses the same work space
    o, v = 4, 16
    pb, _, H, t1, t2 = config_problem(o, v, 0)
    ctx = context(cc, H, t1, t2)
    try:
        print(f"noalloc o={o} v={v} nvec=2", flush=True)
        _, _, (plain, noalloc) = both(cc, ctx, pb, o, v, [0, 1], [0.1 + 0.005j, 0.0 + 0.0j])
        for k in range(2):
            assert_blocks((noalloc[0][k], noalloc[1][k]), (plain[0][k], plain[1][k]), TOL, f"second context {k}")
        # no vectors: nothing is read or written
        assert cc.lib().cclr_jacobian_right_noalloc(ctx, 0, None, None, None, None, None, None) == 0
    finally:
        cc.cclr_destroy(ctx)


def test_noalloc_rejects_what_does_not_fit(cc):
    o, v = 10, 80
    pb, _, H, t1, t2 = config_problem(o, v, 1)
    ctx = context(cc, H, t1, t2)
    try:
        r1, r2 = (dev(x[None]) for x in vec(pb, 0))
        s1 = torch.empty((1, o, v), dtype=torch.complex128, device="cuda")
        s2 = torch.empty((1, o, o, v, v), dtype=torch.complex128, device="cuda")
        print(f"noalloc o={o} v={v} nvec=1", flush=True)
        cc.cclr_jacobian_right_noalloc(ctx, [0.08], [0.004], r1, r2, s1, s2)
        p1 = peak(cc, ctx)
        R1, R2 = r1.expand(2, -1, -1).contiguous(), r2.expand(2, -1, -1, -1, -1).contiguous()
        S1 = torch.empty((2, o, v), dtype=torch.complex128, device="cuda")
        S2 = torch.empty((2, o, o, v, v), dtype=torch.complex128, device="cuda")
        cc.cclr_jacobian_right_noalloc(ctx, [0.08, 0.08], [0.004, 0.004], R1, R2, S1, S2)
        p2 = peak(cc, ctx)
        print(f"  work space peak: one vector {p1} bytes, two vectors {p2} bytes", flush=True)
        assert p2 > p1
        # more vectors than the work space holds (beyond the growth per vector
        # seen above, with room to spare): rejected, nothing written
        n = (WS_BYTES - p1) // (p2 - p1) + 3
        R1, R2 = r1.expand(n, -1, -1).contiguous(), r2.expand(n, -1, -1, -1, -1).contiguous()
        S1 = torch.full((n, o, v), complex(3.0, 1.0), dtype=torch.complex128, device="cuda")
        S2 = torch.full((n, o, o, v, v), complex(3.0, 1.0), dtype=torch.complex128, device="cuda")
        print(f"noalloc o={o} v={v} nvec={n} (expect CCLR_ENOMEM)", flush=True)
        with pytest.raises(cc.CclrError) as e:
            cc.cclr_jacobian_right_noalloc(ctx, [0.08] * n, [0.004] * n, R1, R2, S1, S2)
        assert e.value.code == cc.CCLR_ENOMEM
        assert "work space" in str(e.value)
        torch.cuda.synchronize()
        assert bool((S1 == complex(3.0, 1.0)).all()) and bool((S2 == complex(3.0, 1.0)).all())
        # the context and the work space still work afterwards
        plain1 = torch.empty_like(s1)
        plain2 = torch.empty_like(s2)
        cc.cclr_jacobian_right(ctx, [0.08], [0.004], r1, r2, plain1, plain2)
        cc.cclr_jacobian_right_noalloc(ctx, [0.08], [0.004], r1, r2, s1, s2)
        torch.cuda.synchronize()
        assert_blocks((host(s1), host(s2)), (host(plain1), host(plain2)), TOL, "after a rejected call")
    finally:
        cc.cclr_destroy(ctx)
