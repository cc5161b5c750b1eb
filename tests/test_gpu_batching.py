"""Several problems of different sizes in one call (cclr_jacobian_right_multi):
the ring and ladder products of all contexts run as one persistent launch.
Each result must match the oracle to the FP64 bar (1e-10 relative) and the
single-context transform of the same context to rounding."""
import numpy as np
import pytest
import torch

from gen import synth as s
from helpers import block_errors, config_problem, vec
from oracle import cclr_ref as O

pytestmark = pytest.mark.gpu


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x)).to(torch.complex128).cuda()


def make_ctx(cc, o, v, seed):
    pb, inst, H, t1, t2 = config_problem(o, v, seed)
    ctx = cc.cclr_create(o, v)
    keep = [dev(H.f)] + [dev(H.blocks[k]) for k in s.CANONICAL_BLOCKS] + [dev(t1), dev(t2)]
    cc.cclr_set_hamiltonian(ctx, *keep[:7])
    cc.cclr_set_amplitudes(ctx, *keep[7:])
    return ctx, pb, O.CCLR(H, t1, t2)


@pytest.fixture(scope="module")
def cc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2307_14296_amd as m
    return m


@pytest.mark.parametrize("shapes", [[(2, 5, 2), (3, 7, 1), (4, 9, 3)], [(4, 16, 2), (3, 11, 0), (5, 13, 1)]])
def test_multi_matches_oracle_and_single(cc, shapes):
    ctxs, refs, pbs = [], [], []
    try:
        for k, (o, v, nv) in enumerate(shapes):
            c, pb, ref = make_ctx(cc, o, v, 10 + k)
            ctxs.append(c), refs.append(ref), pbs.append(pb)
        r1s, r2s, s1s, s2s, oms, gas, xs = [], [], [], [], [], [], []
        for (o, v, nv), pb in zip(shapes, pbs):
            x = [vec(pb, j) for j in range(nv)]
            xs.append(x)
            r1s.append(dev(np.stack([a for a, _ in x]) if nv else np.zeros((0, o, v))))
            r2s.append(dev(np.stack([b for _, b in x]) if nv else np.zeros((0, o, o, v, v))))
            s1s.append(torch.empty_like(r1s[-1]))
            s2s.append(torch.empty_like(r2s[-1]))
            oms.append([0.1 * (j + 1) for j in range(nv)])
            gas.append([0.005] * nv)
        cc.cclr_jacobian_right_multi(ctxs, oms, gas, r1s, r2s, s1s, s2s)
        for i, (o, v, nv) in enumerate(shapes):
            if nv == 0:
                continue
            a1, a2 = torch.empty_like(r1s[i]), torch.empty_like(r2s[i])
            cc.cclr_jacobian_right(ctxs[i], oms[i], gas[i], r1s[i], r2s[i], a1, a2)
            for j in range(nv):
                z = oms[i][j] + 1j * gas[i][j]
                got = (s1s[i][j].cpu().numpy(), s2s[i][j].cpu().numpy())
                em, e2, msg = block_errors(got, refs[i].right(*xs[i][j], z))
                dm, d2, _ = block_errors(got, (a1[j].cpu().numpy(), a2[j].cpu().numpy()))
                print(f"instance o={o} v={v} vector {j}: vs oracle {msg}; vs single-context {dm:.2e}", flush=True)
                assert em < 1e-10 and e2 < 1e-10 and dm < 1e-13
    finally:
        for c in ctxs:
            cc.cclr_destroy(c)


def test_multi_rejects_bad_arguments(cc):
    c, pb, ref = make_ctx(cc, 2, 4, 1)
    try:
        r1 = dev(np.zeros((1, 2, 4)))
        r2 = dev(np.zeros((1, 2, 2, 4, 4)))
        with pytest.raises(cc.CclrError):
            cc.cclr_jacobian_right_multi([c, c], [[0.1], [0.1]], [[0.0], [0.0]], [r1, r1], [r2, r2], [r1, r1], [r2, r2])
        with pytest.raises(cc.CclrError):
            cc.cclr_jacobian_right_multi([c], [[0.1]], [[-1.0]], [r1], [r2], [r1], [r2])
    finally:
        cc.cclr_destroy(c)
