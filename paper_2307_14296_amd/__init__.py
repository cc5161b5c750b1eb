"""Python binding of libcclr, the MI355X CCSD linear-response library.

Argument marshalling only: every function forwards to the C entry point of
the same name in ``libcclr.so`` (declared in ``include/cclr.h``).  Tensor
arguments are torch tensors that live on the GPU (complex128, contiguous);
their device pointers are passed through.  Every step of the computation
runs in the library's HIP kernels; nothing here computes.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcclr.so")

CCLR_OK = 0
CCLR_ENOTCONV = 1
CCLR_EINVAL = -1
CCLR_ENOMEM = -2
CCLR_EHIP = -3
CCLR_ESTATE = -4
CCLR_FP64, CCLR_FP32, CCLR_BF16X3, CCLR_BF16X2 = 0, 1, 2, 3
CCLR_RIGHT, CCLR_LEFT = 0, 1

EXPORTED = (
    "cclr_default_options", "cclr_create", "cclr_destroy", "cclr_set_hamiltonian", "cclr_set_hamiltonian_cholesky",
    "cclr_set_amplitudes", "cclr_ccsd_residual", "cclr_solve_ccsd",
    "cclr_jacobian_right", "cclr_jacobian_right_noalloc", "cclr_jacobian_left", "cclr_jacobian_right_multi", "cclr_solve_damped", "cclr_eom_ee", "cclr_solve_lambda", "cclr_get_lambda",
    "cclr_response_function", "cclr_response_function_ci", "cclr_response_function_asym", "cclr_response_backward",
    "cclr_last_error",
)


class cclr_options(ctypes.Structure):
    _fields_ = [("prec", ctypes.c_int), ("tol", ctypes.c_double), ("maxiter", ctypes.c_int),
                ("max_subspace", ctypes.c_int), ("device_mem_cap", ctypes.c_size_t), ("hip_stream", ctypes.c_void_p)]


class cclr_solve_info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("converged", ctypes.c_int), ("resnorm", ctypes.c_double),
                ("time_ms", ctypes.c_double), ("nsigma", ctypes.c_long), ("kappa", ctypes.c_double),
                ("ritz_min", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class CclrError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libcclr error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load libcclr.so from the package directory; fail loudly if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
    L = ctypes.CDLL(LIB_PATH)
    P, I, D = ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_double)
    L.cclr_default_options.argtypes = [ctypes.POINTER(cclr_options)]
    L.cclr_create.argtypes = [I, I, ctypes.POINTER(cclr_options), ctypes.POINTER(P)]
    L.cclr_destroy.argtypes = [P]
    L.cclr_set_hamiltonian.argtypes = [P] + [P] * 7
    L.cclr_set_amplitudes.argtypes = [P, P, P]
    L.cclr_set_hamiltonian_cholesky.argtypes = [P, P, I, P]
    L.cclr_ccsd_residual.argtypes = [P, P, P, P, P, P]
    L.cclr_solve_ccsd.argtypes = [P, ctypes.c_double, I, I, P, P, P, ctypes.POINTER(cclr_solve_info)]
    L.cclr_jacobian_right.argtypes = [P, I, D, D, P, P, P, P]
    L.cclr_jacobian_right_noalloc.argtypes = [P, I, D, D, P, P, P, P]
    L.cclr_jacobian_left.argtypes = [P, I, D, D, P, P, P, P]
    PP = ctypes.POINTER(P)
    L.cclr_jacobian_right_multi.argtypes = [I, PP, ctypes.POINTER(I), PP, PP, PP, PP, PP, PP]
    L.cclr_solve_damped.argtypes = [P, I, I, D, D, P, P, P, P, ctypes.POINTER(cclr_solve_info)]
    L.cclr_solve_lambda.argtypes = [P, ctypes.POINTER(cclr_solve_info)]
    L.cclr_eom_ee.argtypes = [P, I, I, ctypes.c_double, P, P, P, ctypes.POINTER(cclr_solve_info)]
    L.cclr_get_lambda.argtypes = [P, P, P]
    L.cclr_response_function.argtypes = [P, I, ctypes.POINTER(P), I, D, D, P, ctypes.POINTER(cclr_solve_info)]
    L.cclr_response_function_ci.argtypes = [P, I, ctypes.POINTER(P), I, D, D, P, ctypes.POINTER(cclr_solve_info)]
    L.cclr_response_function_asym.argtypes = [P, I, ctypes.POINTER(P), I, ctypes.POINTER(P), I, D, D, P,
                                              ctypes.POINTER(cclr_solve_info)]
    L.cclr_response_backward.argtypes = [P, I, ctypes.POINTER(P), I, D, D, P, ctypes.POINTER(P), P,
                                         ctypes.POINTER(P), ctypes.POINTER(cclr_solve_info)]
    L.cclr_last_error.argtypes = [P]
    L.cclr_last_error.restype = ctypes.c_char_p
    for name in EXPORTED:
        if name not in ("cclr_last_error",):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _ptr(t, name):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name}: expected a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name}: tensor must be on the GPU")
    if t.dtype != torch.complex128:
        raise TypeError(f"{name}: expected complex128, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _dbl(xs):
    xs = [float(x) for x in xs]
    return (ctypes.c_double * max(1, len(xs)))(*xs)


def _check(ctx, rc, allow_notconv=False):
    if rc == CCLR_OK or (allow_notconv and rc == CCLR_ENOTCONV):
        return rc
    msg = lib().cclr_last_error(ctx)
    raise CclrError(rc, msg.decode() if msg else "")


def cclr_default_options():
    o = cclr_options()
    lib().cclr_default_options(ctypes.byref(o))
    return o


def cclr_create(o, v, options=None, stream=None):
    """Returns an opaque context handle.  ``stream``: a torch.cuda.Stream
    (default: torch's current stream)."""
    import torch
    opt = options if options is not None else cclr_default_options()
    if stream is None:
        stream = torch.cuda.current_stream()
    opt.hip_stream = ctypes.c_void_p(stream.cuda_stream)
    h = ctypes.c_void_p()
    rc = lib().cclr_create(int(o), int(v), ctypes.byref(opt), ctypes.byref(h))
    _check(None, rc)
    return h


def cclr_destroy(ctx):
    if ctx is not None:
        _loaded_h.pop(_ctx_key(ctx), None)
    return lib().cclr_destroy(ctx)


def cclr_last_error(ctx=None):
    m = lib().cclr_last_error(ctx)
    return m.decode() if m else ""


# The tensors last handed to cclr_set_hamiltonian, per context (weak
# references and version counters), so that response_function can check that
# the Hamiltonian it differentiates with respect to is the one loaded.
_loaded_h = {}


def _ctx_key(ctx):
    return ctx.value if isinstance(ctx, ctypes.c_void_p) else int(ctx)


def cclr_set_hamiltonian(ctx, f, oooo, ooov, oovv, ovov, ovvv, vvvv):
    import weakref
    ts = (f, oooo, ooov, oovv, ovov, ovvv, vvvv)
    args = [_ptr(x, n) for x, n in zip(ts, ("f", "oooo", "ooov", "oovv", "ovov", "ovvv", "vvvv"))]
    _loaded_h.pop(_ctx_key(ctx), None)
    rc = _check(ctx, lib().cclr_set_hamiltonian(ctx, *args))
    _loaded_h[_ctx_key(ctx)] = [(weakref.ref(t), t._version) for t in ts]
    return rc


def cclr_set_amplitudes(ctx, t1, t2):
    return _check(ctx, lib().cclr_set_amplitudes(ctx, _ptr(t1, "t1"), _ptr(t2, "t2")))


def cclr_set_hamiltonian_cholesky(ctx, f, L):
    """Integral blocks from Cholesky vectors L[nchol][n][n] (device tensor)."""
    _loaded_h.pop(_ctx_key(ctx), None)
    return _check(ctx, lib().cclr_set_hamiltonian_cholesky(ctx, _ptr(f, "f"), int(L.shape[0]), _ptr(L, "L")))


def cclr_ccsd_residual(ctx, t1, t2, o1, o2):
    """Omega(t) into o1, o2 (device tensors); returns the correlation energy."""
    import numpy as np
    e = np.zeros(1, dtype=np.complex128)
    _check(ctx, lib().cclr_ccsd_residual(ctx, _ptr(t1, "t1"), _ptr(t2, "t2"), _ptr(o1, "o1"), _ptr(o2, "o2"),
                                         ctypes.c_void_p(e.ctypes.data)))
    return complex(e[0])


def cclr_solve_ccsd(ctx, t1, t2, tol=1e-10, maxiter=100, nsub=3):
    """CROP solve in place on the device tensors t1, t2; returns (rc, energy, info)."""
    import numpy as np
    e = np.zeros(1, dtype=np.complex128)
    info = cclr_solve_info()
    rc = lib().cclr_solve_ccsd(ctx, float(tol), int(maxiter), int(nsub), _ptr(t1, "t1"), _ptr(t2, "t2"),
                               ctypes.c_void_p(e.ctypes.data), ctypes.byref(info))
    _check(ctx, rc, allow_notconv=True)
    return rc, complex(e[0]), info


def cclr_jacobian_right(ctx, omega, gamma, r1, r2, s1, s2):
    n = len(omega)
    return _check(ctx, lib().cclr_jacobian_right(ctx, n, _dbl(omega), _dbl(gamma), _ptr(r1, "r1"), _ptr(r2, "r2"),
                                                 _ptr(s1, "s1"), _ptr(s2, "s2")))


def cclr_jacobian_right_noalloc(ctx, omega, gamma, r1, r2, s1, s2):
    n = len(omega)
    return _check(ctx, lib().cclr_jacobian_right_noalloc(ctx, n, _dbl(omega), _dbl(gamma), _ptr(r1, "r1"),
                                                         _ptr(r2, "r2"), _ptr(s1, "s1"), _ptr(s2, "s2")))


def cclr_jacobian_left(ctx, omega, gamma, l1, l2, s1, s2):
    n = len(omega)
    return _check(ctx, lib().cclr_jacobian_left(ctx, n, _dbl(omega), _dbl(gamma), _ptr(l1, "l1"), _ptr(l2, "l2"),
                                                _ptr(s1, "s1"), _ptr(s2, "s2")))


def cclr_jacobian_right_multi(ctxs, omegas, gammas, r1s, r2s, s1s, s2s):
    """Right transforms of several contexts in one call (lists, one entry per
    context: frequency lists and GPU tensors as for cclr_jacobian_right)."""
    n = len(ctxs)
    arr = lambda xs: (ctypes.c_void_p * n)(*xs)  # noqa: E731
    om = [_dbl(w) for w in omegas]
    ga = [_dbl(g) for g in gammas]
    rc = lib().cclr_jacobian_right_multi(
        n, arr([c.value if isinstance(c, ctypes.c_void_p) else c for c in ctxs]),
        (ctypes.c_int * n)(*[len(w) for w in omegas]),
        arr([ctypes.cast(x, ctypes.c_void_p).value for x in om]), arr([ctypes.cast(x, ctypes.c_void_p).value for x in ga]),
        arr([_ptr(x, "r1").value for x in r1s]), arr([_ptr(x, "r2").value for x in r2s]),
        arr([_ptr(x, "s1").value for x in s1s]), arr([_ptr(x, "s2").value for x in s2s]))
    return _check(ctxs[0], rc)


def cclr_solve_damped(ctx, side, omega, gamma, b1, b2, x1, x2):
    info = cclr_solve_info()
    rc = lib().cclr_solve_damped(ctx, int(side), len(omega), _dbl(omega), _dbl(gamma), _ptr(b1, "b1"),
                                 _ptr(b2, "b2"), _ptr(x1, "x1"), _ptr(x2, "x2"), ctypes.byref(info))
    _check(ctx, rc, allow_notconv=True)
    return rc, info


def cclr_eom_ee(ctx, side, nroots, tol, x1=None, x2=None):
    """Returns (rc, omega as a host numpy complex128 array, info); x1/x2: optional GPU outputs."""
    import numpy as np
    om = np.zeros(max(int(nroots), 1), dtype=np.complex128)
    info = cclr_solve_info()
    rc = lib().cclr_eom_ee(ctx, int(side), int(nroots), float(tol), ctypes.c_void_p(om.ctypes.data),
                           _ptr(x1, "x1") if x1 is not None else None, _ptr(x2, "x2") if x2 is not None else None,
                           ctypes.byref(info))
    _check(ctx, rc, allow_notconv=True)
    return rc, om[:nroots], info


def cclr_solve_lambda(ctx):
    info = cclr_solve_info()
    rc = lib().cclr_solve_lambda(ctx, ctypes.byref(info))
    _check(ctx, rc, allow_notconv=True)
    return rc, info


def cclr_get_lambda(ctx, l1, l2):
    return _check(ctx, lib().cclr_get_lambda(ctx, _ptr(l1, "l1"), _ptr(l2, "l2")))


def cclr_response_function(ctx, X, omega, gamma, model="cc"):
    """Returns (rc, out[nfreq][nx][nx] as a host numpy complex128 array, info).
    model: "cc" (CC-CC, cclr_response_function) or "ci" (CC-CI, cclr_response_function_ci)."""
    import numpy as np
    nx, nf = len(X), len(omega)
    ptrs = (ctypes.c_void_p * nx)(*[_ptr(x, "X").value for x in X])
    out = np.zeros((max(nf, 1), nx, nx), dtype=np.complex128)
    info = cclr_solve_info()
    fn = {"cc": lib().cclr_response_function, "ci": lib().cclr_response_function_ci}[model]
    rc = fn(ctx, nx, ptrs, nf, _dbl(omega), _dbl(gamma),
                                      ctypes.c_void_p(out.ctypes.data), ctypes.byref(info))
    _check(ctx, rc, allow_notconv=True)
    return rc, out[:nf], info


def cclr_response_function_asym(ctx, X, Y, omega, gamma):
    """<<X_p; Y_q>> from responses of the Y operators only; returns (rc, out[nfreq][nx][ny], info)."""
    import numpy as np
    nx, ny, nf = len(X), len(Y), len(omega)
    px = (ctypes.c_void_p * nx)(*[_ptr(x, "X").value for x in X])
    py = (ctypes.c_void_p * ny)(*[_ptr(y, "Y").value for y in Y])
    out = np.zeros((max(nf, 1), nx, ny), dtype=np.complex128)
    info = cclr_solve_info()
    rc = lib().cclr_response_function_asym(ctx, nx, px, ny, py, nf, _dbl(omega), _dbl(gamma),
                                           ctypes.c_void_p(out.ctypes.data), ctypes.byref(info))
    _check(ctx, rc, allow_notconv=True)
    return rc, out[:nf], info


def cclr_response_backward(ctx, X, omega, gamma, G, dX=None, df=None, dV=None):
    """G: host array (nfreq, nx, nx) complex.  Outputs (GPU complex128, overwritten; None to skip):
    dX: list of nx (n, n) tensors; df: (n, n); dV: list of the six integral blocks in the order
    oooo, ooov, oovv, ovov, ovvv, vvvv."""
    import numpy as np
    nx = len(X)
    G = np.ascontiguousarray(np.asarray(G, dtype=np.complex128))
    ptrs = (ctypes.c_void_p * nx)(*[_ptr(x, "X").value for x in X])
    dptrs = (ctypes.c_void_p * nx)(*[_ptr(d, "dX").value for d in dX]) if dX is not None else None
    vptrs = (ctypes.c_void_p * 6)(*[_ptr(d, "dV").value for d in dV]) if dV is not None else None
    fptr = _ptr(df, "df") if df is not None else None
    info = cclr_solve_info()
    rc = lib().cclr_response_backward(ctx, nx, ptrs, len(omega), _dbl(omega), _dbl(gamma),
                                      ctypes.c_void_p(G.ctypes.data), dptrs, fptr, vptrs, ctypes.byref(info))
    _check(ctx, rc, allow_notconv=True)
    return rc, info


def response_function(ctx, X, omega, gamma, hamiltonian=None):
    """Differentiable <<X_p;X_q>>(omega + i gamma): returns a (nfreq, nx, nx)
    complex128 tensor on the GPU.  Gradients flow to the perturbation
    matrices X and, when ``hamiltonian`` is given, to the Fock matrix and the
    six integral blocks (f, oooo, ooov, oovv, ovov, ovvv, vvvv): the very
    tensors last passed to cclr_set_hamiltonian for this context, unchanged
    since (checked).  The amplitudes are held fixed.  Both directions come
    from cclr_response_backward; the gradient of f and of the integrals is the
    one projected onto changes that keep their symmetries.  A forward or
    backward call whose solves stop at maxiter warns (RuntimeWarning)."""
    hs = ()
    if hamiltonian is not None:
        hs = tuple(hamiltonian)
        if len(hs) != 7:
            raise ValueError("hamiltonian: expected (f, oooo, ooov, oovv, ovov, ovvv, vvvv)")
        rec = _loaded_h.get(_ctx_key(ctx))
        if rec is None or any(r() is not t or t._version != ver for (r, ver), t in zip(rec, hs)):
            raise ValueError("hamiltonian: these tensors are not the ones loaded in the context (or changed since); "
                             "call cclr_set_hamiltonian and cclr_set_amplitudes with them first")
    return _ResponseFunction.apply(ctx, list(omega), list(gamma), len(X), len(hs), *X, *hs)


def _autograd():
    import warnings

    import torch

    class ResponseFunction(torch.autograd.Function):
        @staticmethod
        def forward(fctx, handle, omega, gamma, nx, nh, *args):
            Xc = [x.detach().contiguous() for x in args[:nx]]
            rc, out, info = cclr_response_function(handle, Xc, omega, gamma)
            if rc == CCLR_ENOTCONV:
                warnings.warn(f"response_function: solves not converged ({info.as_dict()})", RuntimeWarning)
            fctx.handle, fctx.omega, fctx.gamma, fctx.nx, fctx.nh = handle, omega, gamma, nx, nh
            fctx.save_for_backward(*Xc, *[h.detach() for h in args[nx:]])
            return torch.as_tensor(out, device=args[0].device)

        @staticmethod
        def backward(fctx, gout):
            saved = fctx.saved_tensors
            nx, nh = fctx.nx, fctx.nh
            Xc, hs = list(saved[:nx]), saved[nx:]
            want_x = any(fctx.needs_input_grad[5:5 + nx])
            want_h = nh > 0 and any(fctx.needs_input_grad[5 + nx:])
            dX = [torch.empty_like(x) for x in Xc] if want_x else None
            df = torch.empty_like(hs[0]) if want_h else None
            dV = [torch.empty_like(h) for h in hs[1:]] if want_h else None
            if want_x or want_h:
                rc, info = cclr_response_backward(fctx.handle, Xc, fctx.omega, fctx.gamma,
                                                  gout.detach().cpu().numpy(), dX=dX, df=df, dV=dV)
                if rc == CCLR_ENOTCONV:
                    warnings.warn(f"response_function backward: solves not converged ({info.as_dict()})",
                                  RuntimeWarning)
            gx = dX if want_x else [None] * nx
            gh = ([df] + dV) if want_h else [None] * nh
            return (None, None, None, None, None, *gx, *gh)

    return ResponseFunction


class _Lazy:
    _fn = None

    @classmethod
    def apply(cls, *a):
        if cls._fn is None:
            cls._fn = _autograd()
        return cls._fn.apply(*a)


_ResponseFunction = _Lazy
