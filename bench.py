"""Benchmark of the CCSD linear-response hot path on one MI355X.

Workload (default): o = 20 occupied, v = 200 virtual spin orbitals, complex
FP64, synthetic MP2-seeded inputs from the seeded generators; three Hermitian
dipole perturbations at z = 0.0774 + 0.005i.  One step is one pass of the
whole hot path: the Hbar intermediate build, the Lambda solve, the damped
response solves for every perturbation at z, -z, z*, -z* (batched Davidson,
one right Jacobian transform per right-hand side per iteration), the
Hessian products and the response-function assembly.

The JSON line reports whole-job Jacobian transforms per second, the
roofline position of the dominant kernel (the packed particle-particle
ladder GEMM on FP64 MFMA, timed with HIP events on the library's stream),
and the CPU oracle timed on the host as a baseline.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6   # MI355X dense FP64 MFMA
PEAK_HBM_GBS = 8000.0


def sigma_flops(o: int, v: int) -> dict:
    """Algorithmic flops of one right Jacobian transform on packed pairs
    (8 real flops per complex multiply-add), by term group."""
    O2, V2 = o * (o - 1) // 2, v * (v - 1) // 2
    ov = o * v
    f = {
        "ladder": 8.0 * O2 * V2 * V2,                 # 1/2 W^ab_ef r^ef_ij
        "ring": 8.0 * ov * ov * ov,                   # P(ab)P(ij) W^mb_ej r^ae_im
        "hole": 8.0 * V2 * O2 * O2,                   # 1/2 W^mn_ij r^ab_mn
        "o2v3": 8.0 * (v * o * (o * V2) + V2 * o * v * o + 3 * (O2 * v * v * v) + v * v * o * v),
        "o3v2": 8.0 * (3 * o * o * o * v * v + 2 * O2 * o * v * v),
    }
    f["total"] = sum(f.values())
    return f


def make_inputs(o, v, seed, device, v_std=None):
    import torch
    from gen import synth as s
    pb = s.Problem(o, v, seed, v_std=v_std)
    with torch.no_grad():
        f = s.fock(pb, device)
        V = s.integral_blocks(pb, device, chunk=8)
        t1 = s.t1_amplitudes(pb, device)
        t2 = s.t2_amplitudes(pb, V["oovv"], device)
        X = [s.dipole(pb, k, device) for k in range(3)]
    return pb, f, V, t1, t2, X


def host_threads():
    """Cores this process may run on, and the BLAS library and its thread count."""
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        ncpu = os.cpu_count() or 1
    blas, nthr = "unknown", ncpu
    try:
        from threadpoolctl import threadpool_info
        info = [x for x in threadpool_info() if x.get("user_api") == "blas"]
        if info:
            blas = f"{info[0].get('internal_api')} {info[0].get('version')}"
            nthr = int(info[0].get("num_threads", ncpu))
    except Exception:  # pragma: no cover
        pass
    return ncpu, blas, nthr


def oracle_problem(o, v, seed, dev):
    """The benchmark generators' instance (generated on the GPU, copied to the
    host) as an oracle Hamiltonian and amplitudes."""
    import torch
    from gen import synth as s
    from oracle import cclr_ref as O
    pb, f, V, t1, t2, X = make_inputs(o, v, seed, dev)
    host = lambda x: x.cpu().numpy()  # noqa: E731
    H = O.Hamiltonian(o, v, host(f), {k: host(V[k]) for k in s.CANONICAL_BLOCKS})
    r = [host(x) for x in s.excitation_vector(pb, 0, dev)]
    Xs = [host(x) for x in X]
    out = (H, host(t1), host(t2), r, Xs)
    del f, V, t1, t2, X
    torch.cuda.empty_cache()
    return out


def time_oracle_sigma(H, t1, t2, r, reps, threads=None):
    """Median wall time of the oracle's right transform (after one warm-up
    call), and the Hbar build time, optionally with the BLAS limited."""
    import contextlib
    import statistics
    from oracle import cclr_ref as O
    lim = contextlib.nullcontext()
    if threads is not None:
        from threadpoolctl import threadpool_limits
        lim = threadpool_limits(limits=threads)
    with lim:
        t0 = time.perf_counter()
        ref = O.CCLR(H, t1, t2)
        t_hbar = time.perf_counter() - t0
        ref.right(*r, 0.0774 + 0.005j)
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            ref.right(*r, 0.0774 + 0.005j)
            ts.append(time.perf_counter() - t0)
    return statistics.median(ts), t_hbar


def cpu_baseline(dev, o, v, seed, reps=2):
    """The oracle's right Jacobian transform of the benchmark instance timed on
    the host, every core: a bounded sample of the workload (a warm-up and
    `reps` timed transforms after the oracle's Hbar build)."""
    ncpu, blas, nthr = host_threads()
    H, t1, t2, r, _ = oracle_problem(o, v, seed, dev)
    dt, t_hbar = time_oracle_sigma(H, t1, t2, r, reps)
    return {
        "value": 1.0 / dt,
        "unit": "Jacobian transforms/s",
        "cores": nthr,
        "kind": "oracle",
        "sample": (f"oracle right Jacobian transform (numpy, FP64 complex, {blas}) of one vector at o={o}, v={v}: "
                   f"median of {reps} after a warm-up, {dt:.2f} s each, "
                   f"{sigma_flops(o, v)['total'] / dt / 1e9:.1f} GFLOP/s algorithmic (the oracle's Hbar build, "
                   f"{t_hbar:.1f} s, not counted); {nthr} BLAS threads on {ncpu} cores"),
    }


def cpu_table(dev):
    """Oracle timings on the host: one right transform at (4,16), (10,80),
    (16,120) and (20,200) with every core and (below (20,200)) one thread,
    and the whole response tensor of the first two configurations."""
    import numpy as np
    from gen import synth as s
    from oracle import cclr_ref as O
    ncpu, blas, nthr = host_threads()
    rows = []
    for (o, v, seed) in ((4, 16, 0), (10, 80, 1), (16, 120, 2), (20, 200, 3)):
        tg = time.perf_counter()
        H, t1, t2, r, Xs = oracle_problem(o, v, seed, dev)
        row = {"o": o, "v": v, "input_s": round(time.perf_counter() - tg, 1),
               "sigma_gflop": sigma_flops(o, v)["total"] / 1e9}
        reps = 10 if o <= 10 else 3
        dt, th = time_oracle_sigma(H, t1, t2, r, reps)
        row.update({"all_cores_s": dt, "hbar_all_cores_s": round(th, 2), "reps": reps})
        log(f"cpu oracle o={o} v={v}: {dt:.3f} s per transform ({nthr} threads), Hbar {th:.1f} s")
        if o < 20:
            dt1, th1 = time_oracle_sigma(H, t1, t2, r, reps, threads=1)
            row.update({"one_thread_s": dt1, "hbar_one_thread_s": round(th1, 2)})
            log(f"cpu oracle o={o} v={v}: {dt1:.3f} s per transform (1 thread)")
        if o <= 10:
            z = 0.1 + 0.005j if o == 4 else 0.08 + 0.004j
            t0 = time.perf_counter()
            ref = O.CCLR(H, t1, t2)
            alpha = -ref.response(Xs, z, method="dense" if o == 4 else "gmres")
            row["alpha_all_cores_s"] = round(time.perf_counter() - t0, 2)
            row["alpha_z"] = [z.real, z.imag]
            log(f"cpu oracle o={o} v={v}: alpha in {row['alpha_all_cores_s']} s")
        rows.append(row)
        del H, t1, t2, r, Xs
    return {"cores": ncpu, "blas": blas, "blas_threads": nthr, "rows": rows}


def sigma_table(cc, dev, o, v, seed, reps=10):
    """Right transforms at o, v for 1, 3 and 12 vectors in every arithmetic:
    median of reps timed calls after a warm-up call (the paper's sigma
    benchmark runs each transform 10 times)."""
    import statistics
    import torch
    from gen import synth as s
    L = cc.lib()
    pb, f, V, t1, t2, X = make_inputs(o, v, seed, dev)
    ctx = cc.cclr_create(o, v, cc.cclr_default_options())
    rows = []
    try:
        cc.cclr_set_hamiltonian(ctx, f, *[V[k] for k in s.CANONICAL_BLOCKS])
        del V
        torch.cuda.empty_cache()
        cc.cclr_set_amplitudes(ctx, t1, t2)
        nmax = 12
        r1 = torch.zeros((nmax, o, v), dtype=torch.complex128, device=dev)
        r2 = torch.zeros((nmax, o, o, v, v), dtype=torch.complex128, device=dev)
        for k in range(nmax):
            r1[k], r2[k] = s.excitation_vector(pb, k, dev)
        fl = sigma_flops(o, v)["total"]
        for prec, code in (("fp64", cc.CCLR_FP64), ("fp32", cc.CCLR_FP32), ("bf16x3", cc.CCLR_BF16X3),
                           ("bf16x2", cc.CCLR_BF16X2)):
            L.cclr_dbg_set_sigma_prec(ctx, code)
            for n in (1, 3, 12):
                a, b = r1[:n].contiguous(), r2[:n].contiguous()
                s1, s2 = torch.empty_like(a), torch.empty_like(b)
                om, ga = [0.0774] * n, [0.005] * n
                cc.cclr_jacobian_right(ctx, om, ga, a, b, s1, s2)
                ts = []
                for _ in range(reps):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    cc.cclr_jacobian_right(ctx, om, ga, a, b, s1, s2)
                    torch.cuda.synchronize()
                    ts.append(time.perf_counter() - t0)
                t = statistics.median(ts)
                rows.append({"prec": prec, "nvec": n, "ms": round(1e3 * t, 3),
                             "transforms_per_s": round(n / t, 2),
                             "tflops_algorithmic": round(n * fl / t / 1e12, 2)})
                log(f"sigma table {prec} nvec={n}: {1e3 * t:.2f} ms")
                del a, b, s1, s2
        L.cclr_dbg_set_sigma_prec(ctx, cc.CCLR_FP64)
    finally:
        cc.cclr_destroy(ctx)
        del f, t1, t2, X
        torch.cuda.empty_cache()
    return {"workload": f"right Jacobian transforms o={o} v={v} complex128, median of {reps} after a warm-up "
                        "(wall time of the call, including the pack and unpack of the vectors)", "rows": rows}


def spectrum_bench(cc, dev, o=16, v=120, seed=2, nfreq=16):
    """Damped spectrum: 3 dipoles x nfreq frequencies on [0, 0.5] Eh, gamma
    0.005, solved in one call (every right-hand side in lockstep) against one
    call per frequency."""
    import numpy as np
    import torch
    from gen import synth as s
    pb, f, V, t1, t2, X = make_inputs(o, v, seed, dev)
    opt = cc.cclr_default_options()
    opt.max_subspace = 24
    opt.tol = 1e-8
    ctx = cc.cclr_create(o, v, opt)
    try:
        cc.cclr_set_hamiltonian(ctx, f, *[V[k] for k in s.CANONICAL_BLOCKS])
        del V
        torch.cuda.empty_cache()
        cc.cclr_set_amplitudes(ctx, t1, t2)
        om = [float(x) for x in np.linspace(0.0, 0.5, nfreq)]
        ga = [0.005] * nfreq
        L = cc.lib()
        L.cclr_dbg_tuning.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_char_p, ctypes.c_longlong]

        def tuned_classes():
            buf = ctypes.create_string_buffer(1 << 16)
            L.cclr_dbg_tuning(ctx, -1, buf, len(buf))
            return len([ln for ln in buf.value.decode().splitlines() if ln])

        # warm-up of both forms, the whole per-frequency sweep included (Lambda solve; first-use GEMM tuning
        # of every product shape class the two forms meet: the active right-hand sides of a call drop out as
        # they converge, so each form has row counts of its own)
        cc.cclr_response_function(ctx, X, om, ga)
        for w in range(nfreq):
            cc.cclr_response_function(ctx, X, [om[w]], [ga[w]])
        torch.cuda.synchronize()
        tuned0 = tuned_classes()
        t0 = time.perf_counter()
        rc, out, info = cc.cclr_response_function(ctx, X, om, ga)
        torch.cuda.synchronize()
        t_lock = time.perf_counter() - t0
        log(f"spectrum: lockstep call {t_lock:.2f} s, {info.nsigma} transforms")
        n_single, outs = 0, []
        t0 = time.perf_counter()
        for w in range(nfreq):
            rc1, one, info1 = cc.cclr_response_function(ctx, X, [om[w]], [ga[w]])
            n_single += info1.nsigma
            outs.append(one[0])
        torch.cuda.synchronize()
        t_single = time.perf_counter() - t0
        log(f"spectrum: one call per frequency {t_single:.2f} s, {n_single} transforms")
        # shape classes first met (and timed by the autotuner) inside the two timed forms
        tuned_while_timed = tuned_classes() - tuned0
        diff = max(float(np.linalg.norm(out[w] - outs[w]) / np.linalg.norm(outs[w])) for w in range(nfreq))
        return {"workload": f"damped spectrum o={o} v={v} complex128, 3 dipoles x {nfreq} frequencies on [0, 0.5] Eh, "
                            f"gamma 0.005, tol 1e-8",
                "lockstep": {"seconds": round(t_lock, 3), "transforms": info.nsigma,
                             "transforms_per_s": round(info.nsigma / t_lock, 2), "iterations": info.iters, "rc": rc},
                "one_call_per_frequency": {"seconds": round(t_single, 3), "transforms": n_single,
                                           "transforms_per_s": round(n_single / t_single, 2)},
                "speedup_lockstep": round(t_single / t_lock, 3), "max_rel_diff_alpha": diff,
                "shapes_tuned_while_timed": tuned_while_timed}
    finally:
        cc.cclr_destroy(ctx)
        del f, t1, t2, X
        torch.cuda.empty_cache()


def diff_bench(cc, dev, o=24, v=240, seed=5, omega=0.0774):
    """Differentiation at o=24, v=240: <<mu; m>>(omega) with an electric
    dipole mu and the magnetic-like m = i(A - A^T)/2, gamma = 0; forward, then
    the backward of Re and of Im <<mu; m>> with respect to the perturbation
    matrices, the Fock matrix and all six integral blocks."""
    import numpy as np
    import torch
    from gen import synth as s
    t0 = time.perf_counter()
    pb, f, V, t1, t2, X = make_inputs(o, v, seed, dev)
    mu, m = X[0], s.magnetic_like(pb, 0, dev)
    del X
    opt = cc.cclr_default_options()
    opt.max_subspace = 24
    opt.tol = 1e-8
    ctx = cc.cclr_create(o, v, opt)
    out = {"workload": f"<<mu; m>> backward o={o} v={v} complex128, omega {omega}, gamma 0 (Re and Im, "
                       f"gradients w.r.t. mu, m, f and the six integral blocks)"}
    try:
        cc.cclr_set_hamiltonian(ctx, f, *[V[k] for k in s.CANONICAL_BLOCKS])
        shapes = [tuple(V[k].shape) for k in s.CANONICAL_BLOCKS]
        del V
        torch.cuda.empty_cache()
        tb = time.perf_counter()
        cc.cclr_set_amplitudes(ctx, t1, t2)
        torch.cuda.synchronize()
        out["setup_s"] = round(time.perf_counter() - t0, 2)
        out["intermediates_s"] = round(time.perf_counter() - tb, 2)
        log(f"diff: o={o} v={v} set up in {out['setup_s']} s")
        tf = time.perf_counter()
        rc, val, info = cc.cclr_response_function(ctx, [mu, m], [omega], [0.0])
        torch.cuda.synchronize()
        out["forward_s"] = round(time.perf_counter() - tf, 2)
        out["forward_transforms"] = info.nsigma
        out["mu_m"] = [val[0][0][1].real, val[0][0][1].imag]
        log(f"diff: forward {out['forward_s']} s, <<mu;m>> = {val[0][0][1]}")
        n = o + v
        dX = [torch.empty((n, n), dtype=torch.complex128, device=dev) for _ in range(2)]
        df = torch.empty((n, n), dtype=torch.complex128, device=dev)
        dV = [torch.empty(sh, dtype=torch.complex128, device=dev) for sh in shapes]
        for part, w in (("re", 1.0), ("im", 1j)):
            G = np.zeros((1, 2, 2), dtype=np.complex128)
            G[0, 0, 1] = w
            tg = time.perf_counter()
            rcb, binfo = cc.cclr_response_backward(ctx, [mu, m], [omega], [0.0], G, dX=dX, df=df, dV=dV)
            torch.cuda.synchronize()
            dt = time.perf_counter() - tg
            out[f"backward_{part}_s"] = round(dt, 2)
            out[f"backward_{part}_transforms"] = binfo.nsigma
            out[f"grad_{part}_norms"] = {"d_mu": torch.linalg.norm(dX[0]).item(), "d_m": torch.linalg.norm(dX[1]).item(),
                                         "df": torch.linalg.norm(df).item(),
                                         "dV": float(sum(torch.linalg.norm(d).item() ** 2 for d in dV) ** 0.5)}
            log(f"diff: backward ({part}) {dt:.2f} s, rc {rcb}")
        free, total = torch.cuda.mem_get_info()
        out["device_memory_in_use_gb"] = round((total - free) / 1e9, 1)
        del dX, df, dV
    finally:
        cc.cclr_destroy(ctx)
        del f, t1, t2, mu, m
        torch.cuda.empty_cache()
    return out


def ground_bench(cc, dev, o, v, seed, tol=1e-8, nchol_per_orbital=3, v_std=0.002):
    """CCSD ground state at the benchmark size: CROP from the MP2-seeded start
    (iterations, residual evaluations, time per residual), and the formation
    of the six integral blocks from Cholesky vectors (nchol =
    nchol_per_orbital * n).  The integrals are drawn with a smaller scale
    (std v_std per component) than the response workload's: at that
    workload's scale dense random integrals make CCSD at v = 200 so strongly
    correlated that no Jacobi-preconditioned iteration converges (the
    particle-ladder block's spectral radius far exceeds the orbital-energy
    gap); the time per residual does not depend on the values."""
    import torch
    from gen import synth as s
    pb, f, V, t1, t2, X = make_inputs(o, v, seed, dev, v_std=v_std)
    del X
    ctx = cc.cclr_create(o, v, cc.cclr_default_options())
    out = {}
    try:
        cc.cclr_set_hamiltonian(ctx, f, *[V[k] for k in s.CANONICAL_BLOCKS])
        del V
        torch.cuda.empty_cache()
        # one residual evaluation first (packs <ab||ef> and tunes the ladder product)
        o1, o2 = torch.empty_like(t1), torch.empty_like(t2)
        cc.cclr_ccsd_residual(ctx, t1, t2, o1, o2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cc.cclr_ccsd_residual(ctx, t1, t2, o1, o2)
        torch.cuda.synchronize()
        t_res = time.perf_counter() - t0
        del o1, o2
        log(f"ground state: one CCSD residual in {1e3 * t_res:.1f} ms")
        t0 = time.perf_counter()
        rc, E, info = cc.cclr_solve_ccsd(ctx, t1, t2, tol=tol, maxiter=80, nsub=3)
        torch.cuda.synchronize()
        t_solve = time.perf_counter() - t0
        log(f"ground state: CROP rc {rc}, {info.iters} iterations, {t_solve:.2f} s")
        out.update({"workload": f"CCSD ground state o={o} v={v} complex128 (CROP, 3 vectors), MP2-seeded start, "
                                f"integral std {v_std}",
                    "residual_ms": round(1e3 * t_res, 2), "crop_rc": rc, "crop_iterations": info.iters,
                    "residual_evaluations": info.nsigma, "resnorm": info.resnorm, "tol": tol,
                    "solve_s_including_intermediates": round(t_solve, 3),
                    "correlation_energy": [E.real, E.imag]})
    finally:
        cc.cclr_destroy(ctx)
    del f, t1, t2
    torch.cuda.empty_cache()
    n = o + v
    nchol = nchol_per_orbital * n
    with torch.no_grad():
        Lc = s.cholesky_vectors(pb, nchol, dev)
        fd = s.fock(pb, dev)
    ctx = cc.cclr_create(o, v, cc.cclr_default_options())
    try:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cc.cclr_set_hamiltonian_cholesky(ctx, fd, Lc)  # first call: includes timing the product variants
        torch.cuda.synchronize()
        dt_first = time.perf_counter() - t0
        t0 = time.perf_counter()
        cc.cclr_set_hamiltonian_cholesky(ctx, fd, Lc)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        flop = 0
        for k in s.CANONICAL_BLOCKS:
            sz = 1
            for c in k:
                sz *= o if c == "o" else v
            flop += 2 * 8 * sz * nchol
        out["cholesky_integrals"] = {"nchol": nchol, "seconds": round(dt, 3), "first_call_seconds": round(dt_first, 3),
                                     "tflops": round(flop / dt / 1e12, 2),
                                     "input_gb": round(Lc.numel() * 16 / 1e9, 3),
                                     "blocks_gb": round(sum((o if k[0] == "o" else v) * (o if k[1] == "o" else v) *
                                                            (o if k[2] == "o" else v) * (o if k[3] == "o" else v)
                                                            for k in s.CANONICAL_BLOCKS) * 16 / 1e9, 2)}
        log(f"Cholesky integral blocks (nchol {nchol}) formed in {dt:.2f} s")
    finally:
        cc.cclr_destroy(ctx)
    del Lc, fd
    torch.cuda.empty_cache()
    return out


# The paper's sigma-vector benchmark (SI, "CPU vs GPU benchmarks", table of
# sigma-vector timings): wall seconds of one sigma evaluation on one
# Xeon Gold 6240 core and on one V100-PCIe, per (O, V).  Context only.
PAPER_SIGMA_S = {(10, 102): (6, 1), (10, 130): (13, 2), (10, 160): (26, 5), (10, 200): (58, 10),
                 (20, 102): (20, 2), (20, 130): (43, 4), (20, 160): (85, 8), (20, 200): (183, 16),
                 (30, 102): (48, 5), (30, 130): (103, 8), (30, 160): (203, 14), (30, 200): (429, 25),
                 (40, 102): (96, 8), (40, 130): (203, 13), (40, 160): (395, 21), (40, 200): (821, 37)}


def copy_bench(cc, dev, reps=5):
    """The library's strided copy (the engine's index permutations) on
    o=20, v=200 shaped tensors: median time of `reps` calls after one, and the
    algorithmic bandwidth (every element read and written once, 32 B)."""
    import numpy as np
    import torch
    L = cc.lib()
    LL, P = ctypes.c_longlong, ctypes.c_void_p
    L.cclr_dbg_tcopy.argtypes = [ctypes.c_int, P, P, P, P, P, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                 ctypes.c_int]
    rows = []
    for shape, perm in [((200, 20, 200, 200), (1, 0, 2, 3)), ((200, 20, 200, 200), (0, 1, 3, 2)),
                        ((20, 200, 20, 200), (0, 2, 1, 3)), ((4000, 4000), (1, 0)),
                        ((200, 200, 20, 200), (2, 3, 0, 1))]:
        g = torch.Generator(device=dev).manual_seed(5)
        src = torch.randn(shape, dtype=torch.complex128, device=dev, generator=g)
        out_shape = tuple(shape[p] for p in perm)
        dst = torch.empty(out_shape, dtype=torch.complex128, device=dev)
        nd = len(shape)
        dims = (LL * nd)(*out_shape)
        sd = (LL * nd)(*[int(np.prod(out_shape[d + 1:])) for d in range(nd)])
        sstr = [int(np.prod(shape[d + 1:])) for d in range(nd)]
        ss = (LL * nd)(*[sstr[perm[d]] for d in range(nd)])
        ts = []
        for r in range(reps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rc = L.cclr_dbg_tcopy(nd, dims, sd, ss, dst.data_ptr(), src.data_ptr(), 1.0, 0.0, 0, 0)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
            assert rc == 0, rc
        assert torch.equal(dst, src.permute(*perm))
        t = sorted(ts[1:])[reps // 2]
        tbs = 32 * src.numel() / t / 1e12
        rows.append({"shape": list(shape), "perm": list(perm), "ms": round(t * 1e3, 3), "TB_per_s": round(tbs, 2),
                     "frac_of_8TBs": round(tbs / 8.0, 3)})
        log(f"copy {shape} perm {perm}: {t * 1e3:.3f} ms, {tbs:.2f} TB/s")
        del src, dst
        torch.cuda.empty_cache()
    return rows


def products_bench(cc, dev, o, v, seed, z, max_subspace, tol, top=40):
    """Per-product record of the contraction engine's GEMMs over one whole FP64
    response step (after a warm-up step, so no product is tuned while
    recorded), aggregated by shape and layout: launches, total ms, TFLOP/s
    algorithmic.  Recording synchronizes after every product, so the step
    runs slower than untraced; the packed ladder and ring GEMMs of the
    transforms go through their own launcher and are not in the record.
    Plain-copy reference bandwidths of the same GPU come first."""
    import collections
    import torch
    from gen import synth as s
    L = cc.lib()
    P = ctypes.c_void_p
    L.cclr_dbg_gemm_trace.argtypes = [P, ctypes.c_int, ctypes.c_char_p, ctypes.c_longlong]
    ref = {}
    for gib in (0.25, 2.0):
        n = int(gib * (1 << 30) / 16)
        a = torch.randn(n, dtype=torch.complex128, device=dev)
        b = torch.empty_like(a)
        for name, fn, nbytes in (("copy", lambda: b.copy_(a), 32 * n), ("sum", lambda: torch.view_as_real(a).sum(),
                                                                           16 * n)):
            ts = []
            for _ in range(6):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                fn()
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            t = sorted(ts[1:])[2]
            ref[f"{name}_{gib}GiB_TB_per_s"] = round(nbytes / t / 1e12, 2)
        del a, b
        torch.cuda.empty_cache()
    log(f"plain-copy references: {ref}")
    pb, f, V, t1, t2, X = make_inputs(o, v, seed, dev)
    opt = cc.cclr_default_options()
    opt.max_subspace = max_subspace
    opt.tol = tol
    ctx = cc.cclr_create(o, v, opt)
    try:
        cc.cclr_set_hamiltonian(ctx, f, *[V[k] for k in s.CANONICAL_BLOCKS])
        del V
        torch.cuda.empty_cache()

        def step():
            cc.cclr_set_amplitudes(ctx, t1, t2)
            rc, out, info = cc.cclr_response_function(ctx, X, [z.real], [z.imag])
            torch.cuda.synchronize()
            return info.nsigma

        step()
        L.cclr_dbg_gemm_trace(ctx, 1, None, 0)
        t0 = time.perf_counter()
        ntr = step()
        traced_s = time.perf_counter() - t0
        buf = ctypes.create_string_buffer(1 << 24)
        L.cclr_dbg_gemm_trace(ctx, 0, buf, len(buf))
    finally:
        cc.cclr_destroy(ctx)
    agg = collections.defaultdict(lambda: [0, 0.0, 0.0])
    lines = [ln for ln in buf.value.decode().splitlines() if ln]
    for ln in lines:
        key, rest = ln.split(" form ")
        form, ms = rest.split()[0], float(rest.split()[1])
        M, N, K = (int(x) for x in key.split()[0].split("x"))
        nb = int(key.split()[1][1:])
        a = agg[key + " form " + form]
        a[0] += 1
        a[1] += ms
        a[2] += 8.0 * M * N * K * nb
    rows = [{"product": k, "launches": a[0], "ms": round(a[1], 3), "tflops": round(a[2] / (a[1] * 1e-3) / 1e12, 2)}
            for k, a in sorted(agg.items(), key=lambda kv: -kv[1][1])]
    return {"workload": f"engine GEMMs of one FP64 response step o={o} v={v}, z={z}", "plain_copy": ref,
            "traced_step_s": round(traced_s, 3), "transforms": ntr, "products": len(lines),
            "total_ms": round(sum(a[1] for a in agg.values()), 1), "top": rows[:top]}


def sweep_bench(cc, dev, seed=3, reps=3):
    """One right transform of one vector (FP64) at each of the paper's sigma
    benchmark shapes: median of reps timed calls after a warm-up call."""
    import statistics
    import torch
    from gen import synth as s
    rows = []
    for (o, v), (cpu_s, gpu_s) in PAPER_SIGMA_S.items():
        pb, f, V, t1, t2, X = make_inputs(o, v, seed, dev)
        ctx = cc.cclr_create(o, v, cc.cclr_default_options())
        try:
            cc.cclr_set_hamiltonian(ctx, f, *[V[k] for k in s.CANONICAL_BLOCKS])
            del V
            torch.cuda.empty_cache()
            cc.cclr_set_amplitudes(ctx, t1, t2)
            a, b = s.excitation_vector(pb, 0, dev)
            r1, r2 = a[None].contiguous(), b[None].contiguous()
            s1, s2 = torch.empty_like(r1), torch.empty_like(r2)
            cc.cclr_jacobian_right(ctx, [0.0774], [0.005], r1, r2, s1, s2)
            ts = []
            for _ in range(reps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                cc.cclr_jacobian_right(ctx, [0.0774], [0.005], r1, r2, s1, s2)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            t = statistics.median(ts)
            fl = sigma_flops(o, v)["total"]
            rows.append({"O": o, "V": v, "ms": round(1e3 * t, 3), "tflops": round(fl / t / 1e12, 2),
                         "paper_v100_s": gpu_s, "paper_cpu_1core_s": cpu_s, "ratio_vs_paper_gpu": round(gpu_s / t, 1)})
            log(f"sweep O={o} V={v}: {1e3 * t:.2f} ms ({fl / t / 1e12:.1f} TFLOP/s)")
        finally:
            cc.cclr_destroy(ctx)
            del f, t1, t2, X
            torch.cuda.empty_cache()
    return rows


def batching_bench(cc, dev, nvec=3, reps=3):
    """Four problems of uneven size, (o, v) = (8, 60), (12, 90), (16, 120),
    (20, 150), nvec right transforms each: one cclr_jacobian_right_multi call
    (grouped persistent ring and ladder launches) against one
    cclr_jacobian_right call per problem."""
    import torch
    from gen import synth as s
    shapes = [(8, 60), (12, 90), (16, 120), (20, 150)]
    ctxs, args = [], []
    try:
        for k, (o, v) in enumerate(shapes):
            pb, f, V, t1, t2, X = make_inputs(o, v, 20 + k, dev)
            c = cc.cclr_create(o, v)
            ctxs.append(c)
            cc.cclr_set_hamiltonian(c, f, *[V[b] for b in s.CANONICAL_BLOCKS])
            cc.cclr_set_amplitudes(c, t1, t2)
            del V
            r1 = torch.zeros((nvec, o, v), dtype=torch.complex128, device=dev)
            r2 = torch.zeros((nvec, o, o, v, v), dtype=torch.complex128, device=dev)
            for j in range(nvec):
                r1[j], r2[j] = s.excitation_vector(pb, j, dev)
            args.append((r1, r2, torch.empty_like(r1), torch.empty_like(r2), [0.0774] * nvec, [0.005] * nvec))
        torch.cuda.empty_cache()

        def seq():
            for c, (r1, r2, s1, s2, om, ga) in zip(ctxs, args):
                cc.cclr_jacobian_right(c, om, ga, r1, r2, s1, s2)

        def grouped():
            cc.cclr_jacobian_right_multi(ctxs, [a[4] for a in args], [a[5] for a in args], [a[0] for a in args],
                                         [a[1] for a in args], [a[2] for a in args], [a[3] for a in args])
        res = {}
        for name, fn in (("one_call_per_problem", seq), ("grouped_persistent", grouped)):
            fn()  # warm-up (autotuning)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                fn()
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / reps
            res[name] = {"ms": round(1e3 * dt, 2), "transforms_per_s": round(len(shapes) * nvec / dt, 2)}
            log(f"batching: {name} {1e3 * dt:.1f} ms per round of {len(shapes) * nvec} transforms")
        # agreement of the two paths
        outs = [(a[2].clone(), a[3].clone()) for a in args]
        seq()
        torch.cuda.synchronize()
        diff = max(float(((a[2] - o1).abs().max() / o1.abs().max()).item()) for a, (o1, o2) in zip(args, outs))
        work = sum(sigma_flops(o, v)["total"] for o, v in shapes) * nvec
        res.update({"problems": [list(x) for x in shapes], "vectors_per_problem": nvec,
                    "speedup_grouped": round(res["one_call_per_problem"]["ms"] / res["grouped_persistent"]["ms"], 3),
                    "tflops_grouped": round(work / (res["grouped_persistent"]["ms"] * 1e-3) / 1e12, 2),
                    "max_rel_diff_singles": diff})
        return res
    finally:
        for c in ctxs:
            cc.cclr_destroy(c)
        torch.cuda.empty_cache()


LADDER_TRAFFIC = os.path.join(ROOT, "profiles", "ladder_gemm_o20v200_traffic.md")
GEMM_SOURCE = os.path.join(ROOT, "paper_2307_14296_amd", "csrc", "gemm_f64.hip")


def gemm_kernel_digest():
    """sha256 of the source of the direct-load FP64 GEMM: its tile order
    function and its tile function and kernels, as marked in the GEMM source
    (the rest of that file does not change what it moves); None if the
    markers are not found."""
    import hashlib
    try:
        text = open(GEMM_SOURCE).read()
        i = text.index("__device__ __forceinline__ void tile_of(")
        order = text[i:text.index("\n}\n", i) + 3]
        j = text.index("four-product tile whose operand tiles go from HBM to LDS")
        tile = text[j:text.index("// grouped persistent form of the direct-load tile", j)]
    except (OSError, ValueError):
        return None
    return hashlib.sha256((order + tile).encode()).hexdigest()


def ladder_traffic(variant):
    """HBM bytes per launch of the batched FP64 ladder GEMM (12 vectors at
    o=20, v=200) in the kernel variant the autotuner chose, from the
    committed rocprofv3 --pmc summary (one figure per variant); None for a
    variant other than the direct-load tiles (15, 16) or when their source
    differs from the one the counters were taken on."""
    try:
        text = open(LADDER_TRAFFIC).read()
    except OSError:
        return None
    vals = dict(re.findall(r"^- (\w+): (\S+)$", text, flags=re.M))
    key = f"variant_{variant}_hbm_bytes_per_launch"
    digest = gemm_kernel_digest()
    if variant not in (15, 16) or digest is None or vals.get("dma_kernel_source_sha256") != digest or key not in vals:
        return None
    return float(vals[key])


def gemm_kernel_name(variant):
    """HIP kernel behind an FP64 GEMM variant number of the autotuner."""
    if variant is None:
        return "FP64 GEMM"
    variant %= 100  # 100 + v: variant v on the transposed product
    if variant == 19:
        return "k_zgemm_p1"
    if variant == 20:
        return "k_zgemm_p"
    if variant >= 15:
        return "k_zgemm_dma"
    if variant >= 13:
        return "k_zgemm_w1"
    return "k_zgemm_p1" if variant >= 9 else "k_zgemm_p"


def alpha_err(a, ref):
    """Errors of a response tensor against a reference: Frobenius-norm
    relative, the largest relative error of the entries at least 1e-3 of the
    largest, and the largest error of the other entries relative to the
    largest entry."""
    import numpy as np
    a, ref = np.asarray(a), np.asarray(ref)
    mx = float(np.abs(ref).max())
    big = np.abs(ref) >= 1e-3 * mx
    d = np.abs(a - ref)
    return {"frobenius": float(np.linalg.norm(a - ref) / np.linalg.norm(ref)),
            "entries": float((d[big] / np.abs(ref[big])).max()),
            "small_entries": float(d[~big].max() / mx) if (~big).any() else 0.0}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--o", type=int, default=20)
    ap.add_argument("--v", type=int, default=200)
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--omega", type=float, default=0.0774)
    ap.add_argument("--gamma", type=float, default=0.005)
    ap.add_argument("--mode", choices=["response", "sigma", "sweep", "cpu", "copy", "products"], default="response",
                    help="response: the whole job (default); sigma: transforms of --nvec vectors; sweep: one "
                         "transform at each of the paper's sigma-benchmark shapes; cpu: the oracle's timings on "
                         "the host (transforms at four sizes, every core and one thread, and two response tensors); "
                         "copy: the library's strided copy on index permutations of o=20, v=200 tensors; "
                         "products: per-product record of the engine's GEMMs over one FP64 response step")
    ap.add_argument("--nvec", type=int, default=12, help="vectors per transform call in --mode sigma")
    ap.add_argument("--max-subspace", type=int, default=24)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-probe-gib", type=float, default=0.0,
                    help="run a plain device copy of this many GiB first (reference for HBM byte counters)")
    ap.add_argument("--no-mixed", dest="mixed", action="store_false",
                    help="skip the mixed-precision runs (reduced-precision products + FP64 refinement)")
    ap.add_argument("--no-batching", dest="batching", action="store_false",
                    help="skip the uneven multi-problem transform comparison")
    ap.add_argument("--no-spectrum", dest="spectrum", action="store_false",
                    help="skip the damped-spectrum lockstep vs per-frequency comparison (o=16, v=120)")
    ap.add_argument("--no-diff", dest="diff", action="store_false",
                    help="skip the backward of <<mu; m>> at o=24, v=240 (about 240 GB of device memory)")
    ap.add_argument("--no-ground", dest="ground", action="store_false",
                    help="skip the CCSD ground-state (CROP) and Cholesky-integral timings")
    ap.add_argument("--mixed-precs", default="fp32,bf16x3,bf16x2",
                    help="comma list of reduced precisions to run after the FP64 run")
    ap.add_argument("--mixed-steps", type=int, default=5, help="timed steps of each reduced-precision run")
    ap.add_argument("--prec", choices=["fp64", "fp32", "bf16x3", "bf16x2"], default="fp64",
                    help="arithmetic of the main (reported) run; anything but fp64 is for profiling only")
    ap.add_argument("--tight-tol", type=float, default=1e-11,
                    help="tolerance of the untimed FP64 reference solve that the alpha errors are measured against")
    ap.add_argument("--no-sigma-table", dest="sigma_table", action="store_false",
                    help="skip the table of transform timings per precision and vector count")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {args.gpus} is not supported "
              "(independent response solves would shard across GPUs, see the design notes)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2307_14296_amd as cc
    from gen import synth as s

    L = cc.lib()
    L.cclr_dbg_profile.argtypes = [ctypes.c_void_p, ctypes.c_int]
    L.cclr_dbg_profile_read.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_longlong),
                                        ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    L.cclr_dbg_set_sigma_prec.argtypes = [ctypes.c_void_p, ctypes.c_int]
    L.cclr_dbg_tuning.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_char_p, ctypes.c_longlong]
    o, v = args.o, args.v
    dev = torch.device("cuda:0")
    z = complex(args.omega, args.gamma)

    PRECS = {"fp64": cc.CCLR_FP64, "fp32": cc.CCLR_FP32, "bf16x3": cc.CCLR_BF16X3, "bf16x2": cc.CCLR_BF16X2}

    def run(prec, steps, warmup, tight_tol=None):
        """Time `steps` steps with the given arithmetic; returns a dict.  With
        tight_tol, one more untimed response solve to that tolerance follows
        (FP64 reference of the alpha errors, conditioning estimate)."""
        t_gen = time.perf_counter()
        pb, f, V, t1, t2, X = make_inputs(o, v, args.seed, dev)
        torch.cuda.synchronize()
        t_gen = time.perf_counter() - t_gen
        log(f"[{prec}] inputs generated on the GPU in {t_gen:.1f} s")
        opt = cc.cclr_default_options()
        opt.max_subspace = args.max_subspace
        opt.tol = args.tol
        opt.prec = PRECS[prec]
        ctx = cc.cclr_create(o, v, opt)
        cc.cclr_set_hamiltonian(ctx, f, *[V[k] for k in s.CANONICAL_BLOCKS])
        if tight_tol is None:
            del V
            torch.cuda.empty_cache()
        log(f"[{prec}] Hamiltonian copied into the context")
        res = {"input_generation_s": round(t_gen, 2)}
        if args.mode == "sigma":
            tb = time.perf_counter()
            cc.cclr_set_amplitudes(ctx, t1, t2)
            log(f"[{prec}] intermediates built in {time.perf_counter() - tb:.2f} s")
            n = args.nvec
            r1 = torch.zeros((n, o, v), dtype=torch.complex128, device=dev)
            r2 = torch.zeros((n, o, o, v, v), dtype=torch.complex128, device=dev)
            for k in range(n):
                a, b = s.excitation_vector(pb, k, dev)
                r1[k], r2[k] = a, b
            s1, s2 = torch.empty_like(r1), torch.empty_like(r2)
            om, ga = [z.real] * n, [z.imag] * n
            if prec != "fp64":
                L.cclr_dbg_set_sigma_prec(ctx, opt.prec)

            def step():
                cc.cclr_jacobian_right(ctx, om, ga, r1, r2, s1, s2)
                return n
        else:
            def step():
                cc.cclr_set_amplitudes(ctx, t1, t2)
                rc, out, info = cc.cclr_response_function(ctx, X, [z.real], [z.imag])
                res["alpha"] = -out[0]
                res["solver"] = info.as_dict()
                res["rc"] = rc
                return info.nsigma

        for k in range(warmup):
            tw = time.perf_counter()
            step()
            torch.cuda.synchronize()
            log(f"[{prec}] warm-up step {k} done in {time.perf_counter() - tw:.2f} s")
        L.cclr_dbg_profile(ctx, 1)
        torch.cuda.synchronize()
        def tuning_record():
            buf = ctypes.create_string_buffer(1 << 16)
            L.cclr_dbg_tuning(ctx, -1, buf, len(buf))
            return [ln for ln in buf.value.decode().splitlines() if ln]

        tuned_before = len(tuning_record())
        t0 = time.perf_counter()
        ntr = 0
        step_s = []
        for k in range(steps):
            ts = time.perf_counter()
            ntr += step()
            torch.cuda.synchronize()
            step_s.append(round(time.perf_counter() - ts, 4))
            log(f"[{prec}] timed step {k} done ({time.perf_counter() - t0:.2f} s so far)")
        dt = time.perf_counter() - t0
        nl, ms, fl = ctypes.c_longlong(), ctypes.c_double(), ctypes.c_double()
        L.cclr_dbg_profile_read(ctx, 1, opt.prec, ctypes.byref(nl), ctypes.byref(ms), ctypes.byref(fl))
        L.cclr_dbg_profile(ctx, 0)
        res["gemm_tuning"] = tuning_record()
        # every timed step's duration, and the GEMM shape classes first tuned inside the timed steps (0 when
        # the warm-up covered them all)
        res["step_s"] = step_s
        res["shapes_tuned_while_timed"] = len(res["gemm_tuning"]) - tuned_before
        cc.cclr_destroy(ctx)
        if tight_tol and args.mode == "response":
            # untimed FP64 reference solved to the tight tolerance
            opt.tol = tight_tol
            opt.prec = cc.CCLR_FP64
            ctx = cc.cclr_create(o, v, opt)
            try:
                cc.cclr_set_hamiltonian(ctx, f, *[V[k] for k in s.CANONICAL_BLOCKS])
                cc.cclr_set_amplitudes(ctx, t1, t2)
                tt = time.perf_counter()
                rc, out, info = cc.cclr_response_function(ctx, X, [z.real], [z.imag])
                torch.cuda.synchronize()
                res["tight"] = {"tol": tight_tol, "alpha": -out[0], "rc": rc, "solver": info.as_dict(),
                                "seconds": round(time.perf_counter() - tt, 2)}
                log(f"[{prec}] reference solve to {tight_tol:g}: {info.as_dict()}")
            finally:
                cc.cclr_destroy(ctx)
            del V
        del f, t1, t2, X
        torch.cuda.empty_cache()
        res.update({"transforms": ntr, "dt": dt, "nl": nl.value, "ms": ms.value, "fl": fl.value})
        return res

    if args.mode == "cpu":
        print(json.dumps({"cpu_oracle_table": cpu_table(dev)}), flush=True)
        return
    if args.mode == "copy":
        print(json.dumps({"strided_copy": copy_bench(cc, dev)}), flush=True)
        return
    if args.mode == "products":
        print(json.dumps({"engine_products": products_bench(cc, dev, o, v, args.seed, z, args.max_subspace,
                                                             args.tol)}), flush=True)
        return
    if args.mode == "sweep":
        rows = sweep_bench(cc, dev)
        tot_ms = sum(r["ms"] for r in rows)
        print(json.dumps({"metric": "Jacobian transforms/s (one vector, the paper's sigma-benchmark shapes)",
                          "value": len(rows) / (tot_ms * 1e-3), "unit": "Jacobian transforms/s", "n_gpus": 1,
                          "steps": len(rows), "warmup": 1, "ms_per_step": tot_ms / len(rows),
                          "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c128 (f64)",
                          "data": "synthetic (seeded generators)",
                          "config": {"workload": "sigma-benchmark sweep O in {10,20,30,40} x V in {102,130,160,200}",
                                     "rows": rows}}), flush=True)
        return
    if args.copy_probe_gib > 0:
        nel = int(args.copy_probe_gib * (1 << 30) / 16)
        a = torch.ones(nel, dtype=torch.complex128, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"copy probe: {nel * 16 / (1 << 30):.3f} GiB read + written")
        del a, b
        torch.cuda.empty_cache()
    main_res = run(args.prec, args.steps, args.warmup,
                   tight_tol=args.tight_tol if args.mode == "response" and args.prec == "fp64" else None)
    mixed = {}
    if args.mixed:
        for p in [x for x in args.mixed_precs.split(",") if x]:
            mixed[p] = run(p, args.mixed_steps, 1)
    ntr, dt = main_res["transforms"], main_res["dt"]
    nl = ctypes.c_longlong(main_res["nl"])
    ms = ctypes.c_double(main_res["ms"])
    fl = ctypes.c_double(main_res["fl"])
    t_gen = main_res["input_generation_s"]
    extra = {k: main_res[k] for k in ("solver", "rc", "step_s", "shapes_tuned_while_timed") if k in main_res}
    extra["gemm_tuning"] = main_res.get("gemm_tuning", [])[:16]
    achieved = fl.value / (ms.value * 1e-3) / 1e12 if ms.value > 0 else 0.0
    sf = sigma_flops(o, v)
    ladder_shape = f"{(o * (o - 1) // 2) * args.nvec}x{v * (v - 1) // 2}x{v * (v - 1) // 2}"
    variant = [ln for ln in main_res.get("gemm_tuning", []) if ln.startswith(ladder_shape)]
    chosen = int(variant[0].rsplit("->", 1)[1]) if variant else None
    roofline = {
        "bound": "mfma",
        "kernel": f"{gemm_kernel_name(chosen)} (packed particle-particle ladder, FP64 MFMA), largest launches" +
                  (f"; autotuner: {variant[0]}" if variant else ""),
        "achieved": round(achieved, 3),
        "peak": PEAK_FP64_TFLOPS,
        "unit": "TFLOP/s",
        "frac": round(achieved / PEAK_FP64_TFLOPS, 4),
        "traffic": ladder_traffic(chosen),
        "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, scaled by a plain-copy reference)",
        "launches": nl.value,
        "avg_launch_ms": round(ms.value / max(1, nl.value), 4),
        "flop_per_launch": fl.value / max(1, nl.value),
    }
    line = {
        "metric": "Jacobian transforms/s (whole response-function job, o=20 v=200)",
        "value": ntr / dt,
        "unit": "Jacobian transforms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128 (f64)",
        "data": "synthetic (seeded generators: MP2-seeded amplitudes, random antisymmetrized integrals)",
        "config": {"workload": f"CCSD-LR {args.mode} o={o} v={v} complex128, 3 dipoles, z={z}",
                   "o": o, "v": v, "mode": args.mode, "transforms": ntr,
                   "tflops_algorithmic_sigma": round(ntr * sf["total"] / dt / 1e12, 3),
                   "input_generation_s": round(t_gen, 2)},
        "roofline": roofline,
    }
    line["config"].update(extra)
    ref_alpha = None
    if "alpha" in main_res:
        a = main_res["alpha"]
        line["config"]["alpha_fp64"] = [[[x.real, x.imag] for x in row] for row in a]
        if "tight" in main_res:
            tight = main_res["tight"]
            ref_alpha = tight["alpha"]
            line["config"]["alpha_reference"] = {
                "tol": tight["tol"], "rc": tight["rc"], "solve_seconds": tight["seconds"],
                "resnorm": tight["solver"]["resnorm"], "iters": tight["solver"]["iters"],
                "alpha": [[[x.real, x.imag] for x in row] for row in ref_alpha],
                "timed_fp64_alpha_vs_reference": alpha_err(a, ref_alpha)}
            line["config"]["conditioning"] = {
                "kappa_estimate": tight["solver"]["kappa"], "ritz_min": tight["solver"]["ritz_min"],
                "what": "Ritz values theta of (A - z) on the final Davidson subspaces of the reference solve "
                        "(the eigenvalues of the projected matrix): kappa = max|theta|/min|theta| (largest over "
                        "right-hand sides), ritz_min = min|theta|"}
    names = {"fp32": "FP32 MFMA ladder/ring products, FP64 refinement",
             "bf16x3": "split-BF16 MFMA ladder/ring products (both operands split hi+lo, 3 bf16 products per "
                       "real product, FP32 accumulation), FP64 refinement",
             "bf16x2": "split-BF16 MFMA ladder/ring products (trial vectors split hi+lo, operator rounded to "
                       "bf16, 2 bf16 products per real product, FP32 accumulation), FP64 refinement"}
    if mixed:
        line["mixed_precision"] = {}
    fp64_step = main_res["dt"] / args.steps
    for p, mres in mixed.items():
        step_s = mres["dt"] / args.mixed_steps
        mx = {"prec": names[p], "value": mres["transforms"] / mres["dt"], "steps": args.mixed_steps,
              "ms_per_step": 1e3 * step_s, "transforms": mres["transforms"],
              "job_speedup_vs_fp64": fp64_step / step_s, "step_s": mres.get("step_s"),
              "shapes_tuned_while_timed": mres.get("shapes_tuned_while_timed")}
        if "alpha" in mres:
            mx["alpha_err_vs_fp64_timed"] = alpha_err(mres["alpha"], main_res["alpha"])
            if ref_alpha is not None:
                mx["alpha_err_vs_fp64_reference"] = alpha_err(mres["alpha"], ref_alpha)
            mx["solver"] = mres.get("solver")
        if mres["ms"] > 0:
            # launches of the reduced-precision ladder product only (the FP64 residual transforms excluded);
            # a split-BF16 launch includes splitting the trial vectors
            mx["ladder_tflops_algorithmic"] = round(mres["fl"] / (mres["ms"] * 1e-3) / 1e12, 3)
            mx["ladder_avg_launch_ms"] = round(mres["ms"] / max(1, mres["nl"]), 4)
        line["mixed_precision"][p] = mx
    def section(name, fn):
        """Extra measurements: a failure is recorded in the line, not fatal to it."""
        try:
            line[name] = fn()
        except Exception as e:  # noqa: BLE001
            log(f"{name}: failed: {e}")
            line[name] = {"error": str(e)}
        torch.cuda.empty_cache()

    if args.batching and args.mode == "response":
        section("batching", lambda: batching_bench(cc, dev))
    if args.spectrum and args.mode == "response":
        section("spectrum", lambda: spectrum_bench(cc, dev))
    if args.ground and args.mode == "response":
        section("ground_state", lambda: ground_bench(cc, dev, o, v, args.seed))
    if args.diff and args.mode == "response":
        section("differentiation", lambda: diff_bench(cc, dev))
    if args.sigma_table and args.mode == "response":
        section("sigma_table", lambda: sigma_table(cc, dev, o, v, args.seed))
    if not args.no_cpu:
        log("timing the CPU oracle")
        line["cpu_baseline"] = cpu_baseline(dev, o, v, args.seed)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
