"""MI355X walk-based Laplacians: Python binding of libwalklap.so.

Every computation runs in the HIP library; this module only marshals pointers
and sizes.  torch supplies device memory and the stream (the library enqueues
on ``torch.cuda.current_stream()`` of the context's device).  There is no CPU
fallback: if the library is missing or no GPU is present, calls raise.
"""

import ctypes as C

from . import _lib
from ._lib import (  # noqa: F401
    WL_EST_BKS,
    WL_EST_HUTCHINSON,
    WL_EST_SURROGATE,
    WL_EST_XNYS,
    WL_F_EXP,
    WL_F_LINEAR,
    WL_F_RESOLVENT,
    WL_FP32,
    WL_FP64,
    WL_M_AMG_CG,
    WL_M_ARNOLDI,
    WL_M_AUTO,
    WL_M_LANCZOS,
    WL_M_RECURRENCE,
    WL_PROBE_GAUSS,
    WL_PROBE_RADEMACHER,
    RkInfo,
    WLError,
    check,
    load,
)

FUNCS = {"res": WL_F_RESOLVENT, "resolvent": WL_F_RESOLVENT, "exp": WL_F_EXP, "exponential": WL_F_EXP,
         "linear": WL_F_LINEAR}
METHODS = {"auto": WL_M_AUTO, "recurrence": WL_M_RECURRENCE, "lanczos": WL_M_LANCZOS, "arnoldi": WL_M_ARNOLDI,
           "amg": WL_M_AMG_CG}
ESTIMATORS = {"hutchinson": WL_EST_HUTCHINSON, "bks": WL_EST_BKS, "xnys": WL_EST_XNYS,
              "surrogate": WL_EST_SURROGATE}
LAWS = {"gauss": WL_PROBE_GAUSS, "gaussian": WL_PROBE_GAUSS, "rademacher": WL_PROBE_RADEMACHER}


def _torch():
    import torch
    return torch


def _prec_of(dtype):
    torch = _torch()
    if dtype == torch.float32:
        return WL_FP32
    if dtype == torch.float64:
        return WL_FP64
    raise TypeError(f"unsupported dtype {dtype}")


def _dtype_of(prec):
    torch = _torch()
    return torch.float32 if prec == WL_FP32 else torch.float64


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def _dptr(a):
    """Host pointer to a contiguous float64 numpy array."""
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _need(t, name, dtype, shape):
    """Check that a tensor handed to the library is a contiguous device tensor of the
    given dtype and shape (None in shape: any extent); the library cannot check the
    sizes of the buffers behind its pointers."""
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} has dtype {t.dtype}, expected {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    ok = t.dim() == len(shape) and all(s is None or t.shape[i] == s for i, s in enumerate(shape))
    if not ok:
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t


class Context:
    """A device and the stream the library enqueues on."""

    def __init__(self, device=0, stream=None):
        torch = _torch()
        lib = load()
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device).cuda_stream
        self.handle = C.c_void_p()
        check(lib.wl_ctx_create(device, C.c_void_p(stream), C.byref(self.handle)))

    def synchronize(self):
        check(load().wl_ctx_synchronize(self.handle))

    def set_profiling(self, on):
        check(load().wl_ctx_set_profiling(self.handle, 1 if on else 0))

    def kernel_stats(self, kernel_class):
        """(launches, total_ms, algorithmic_bytes) of a timed kernel class."""
        n, ms, by = C.c_int64(), C.c_double(), C.c_double()
        check(load().wl_ctx_kernel_stats(self.handle, int(kernel_class), C.byref(n), C.byref(ms), C.byref(by)))
        return n.value, ms.value, by.value

    def set_checks(self, finite=True):
        """Scan the outputs of fdeg / apply_phi / apply_L / expv for NaN or Inf
        (WL_ENUMERIC); synchronises after each such call."""
        check(load().wl_ctx_set_checks(self.handle, WL_CHECK_FINITE if finite else 0))

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            load().wl_ctx_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def torch_device(self):
        return _torch().device("cuda", self.device)


WL_CHECK_FINITE = 1


def inject_alloc_failure(k):
    """Test hook: the k-th device allocation of the library from now on fails as an
    out-of-memory would (k < 0: off)."""
    check(load().wl_test_fail_alloc(int(k)))


class Graph:
    """Symmetric unweighted CSR graph resident on the device (int32 rowptr / colidx)."""

    def __init__(self, ctx, rowptr, colidx, n=None, copy=False, validate=False):
        torch = _torch()
        dev = ctx.torch_device
        self.ctx = ctx
        self.rowptr = torch.as_tensor(rowptr).to(device=dev, dtype=torch.int32).contiguous()
        self.colidx = torch.as_tensor(colidx).to(device=dev, dtype=torch.int32).contiguous()
        self.n = int(self.rowptr.numel() - 1) if n is None else int(n)
        self.nnz = int(self.colidx.numel())
        flags = (_lib.WL_GRAPH_COPY if copy else 0) | (_lib.WL_GRAPH_VALIDATE if validate else 0)
        self.handle = C.c_void_p()
        check(load().wl_graph_create(ctx.handle, self.n, self.nnz, _ptr(self.rowptr), _ptr(self.colidx), flags,
                                     C.byref(self.handle)))
        if copy:
            self.rowptr = self.colidx = None

    def info(self):
        n, nnz, md = C.c_int64(), C.c_int64(), C.c_int32()
        check(load().wl_graph_info(self.handle, C.byref(n), C.byref(nnz), C.byref(md)))
        return n.value, nnz.value, md.value

    def spmm(self, X, Y=None):
        torch = _torch()
        X = X.contiguous()
        _prec_of(X.dtype)
        X2 = _need(X.view(-1, 1) if X.dim() == 1 else X, "X", X.dtype, (self.n, None))
        b = X2.shape[1]
        if Y is None:
            Y = torch.empty_like(X)
        _need(Y.view(self.n, -1) if Y.is_contiguous() and Y.numel() == X.numel() else Y, "Y", X.dtype, (self.n, b))
        check(load().wl_spmm(self.handle, _prec_of(X.dtype), _ptr(X), _ptr(Y), b))
        return Y

    def autotune(self, dtype, b):
        check(load().wl_autotune(self.handle, _prec_of(dtype), b))

    def shape(self, dtype, b):
        """(lanes per row, long-row threshold) used for (dtype, b)."""
        g, t = C.c_int32(), C.c_int32()
        check(load().wl_graph_shape(self.handle, _prec_of(dtype), b, C.byref(g), C.byref(t)))
        return g.value, t.value

    def set_shape(self, dtype, b, lanes_per_row, long_row_threshold):
        check(load().wl_graph_set_shape(self.handle, _prec_of(dtype), b, int(lanes_per_row),
                                        int(long_row_threshold)))

    def lambda_max(self, tol=1e-12):
        out = C.c_double()
        check(load().wl_lambda_max(self.handle, tol, C.byref(out)))
        return out.value

    def spectral_radius(self, mu, tol=1e-10):
        out = C.c_double()
        check(load().wl_spectral_radius(self.handle, float(mu), tol, C.byref(out)))
        return out.value

    def features(self, scale, out=None):
        """n x 8 float32 local features scaled by the operator parameter."""
        torch = _torch()
        if out is None:
            out = torch.empty((self.n, 8), dtype=torch.float32, device=self.ctx.torch_device)
        _need(out, "out", torch.float32, (self.n, 8))
        check(load().wl_features(self.handle, float(scale), _ptr(out)))
        return out

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            load().wl_graph_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Operator:
    """phi(A, c) and its walk Laplacian for one (mu, f, parameter) choice."""

    def __init__(self, graph, mu, func, param, dtype=None, krylov_dim=0, tol=0.0, method="auto", reorth=1,
                 rho_hint=0.0):
        torch = _torch()
        dtype = dtype or torch.float32
        self.graph = graph
        self.dtype = dtype
        d = _lib.OpDesc(mu=float(mu), func=FUNCS[func] if isinstance(func, str) else int(func), param=float(param),
                        prec=_prec_of(dtype), krylov_dim=int(krylov_dim), tol=float(tol),
                        method=METHODS[method] if isinstance(method, str) else int(method), reorth=int(reorth),
                        rho_hint=float(rho_hint))
        self.desc = d
        self.handle = C.c_void_p()
        check(load().wl_op_create(graph.handle, C.byref(d), C.byref(self.handle)))

    def _empty(self, *shape):
        return _torch().empty(shape, dtype=self.dtype, device=self.graph.ctx.torch_device)

    def info(self):
        """(truncation degree or Lanczos steps, method code)."""
        k, m = C.c_int32(), C.c_int32()
        check(load().wl_op_info(self.handle, C.byref(k), C.byref(m)))
        return k.value, m.value

    def fdeg(self, out=None):
        out = self._empty(self.graph.n) if out is None else out
        _need(out, "out", self.dtype, (self.graph.n,))
        check(load().wl_fdeg(self.handle, _ptr(out)))
        return out

    def _block(self, X):
        X = X.to(self.dtype).contiguous()
        if X.dim() == 1:
            X = X.view(-1, 1)
        return _need(X, "X", self.dtype, (self.graph.n, None))

    def _out(self, out, X):
        out = _torch().empty_like(X) if out is None else out
        return _need(out.view(X.shape) if out.is_contiguous() and out.numel() == X.numel() else out, "out",
                     self.dtype, tuple(X.shape))

    def apply_phi(self, X, out=None):
        X = self._block(X)
        out = self._out(out, X)
        check(load().wl_apply_phi(self.handle, _ptr(X), _ptr(out), X.shape[1]))
        return out

    def apply_L(self, X, out=None):
        X = self._block(X)
        out = self._out(out, X)
        check(load().wl_apply_L(self.handle, _ptr(X), _ptr(out), X.shape[1]))
        return out

    def expv(self, U0, ts, outer_dim=30, outs=None):
        U0 = self._block(U0)
        ts = [float(t) for t in ts]
        torch = _torch()
        outs = [torch.empty_like(U0) for _ in ts] if outs is None else outs
        if len(outs) != len(ts):
            raise ValueError("one output block per time is needed")
        outs = [self._out(o, U0) for o in outs]
        tarr = (C.c_double * len(ts))(*ts)
        parr = (C.c_void_p * len(ts))(*[o.data_ptr() for o in outs])
        err = (C.c_double * len(ts))()
        check(load().wl_expv(self.handle, _ptr(U0), U0.shape[1], tarr, len(ts), parr, int(outer_dim), err))
        return outs, list(err)

    def amg_info(self):
        """Hierarchy and last-solve figures of a multigrid-preconditioned CG operator."""
        st = _lib.AmgStats()
        check(load().wl_amg_info(self.handle, C.byref(st)))
        L = st.levels
        return {"levels": L, "rows": list(st.rows[:L]), "nnz": list(st.nnz[:L]),
                "operator_complexity": st.operator_complexity, "setup_ms": st.setup_ms,
                "iterations": st.iterations, "rel_residual": st.rel_residual, "products": st.products}

    # ---- caller workspace (no device allocation inside the call)
    CALLS = {"apply_phi": _lib.WL_CALL_APPLY_PHI, "apply_L": _lib.WL_CALL_APPLY_L, "expv": _lib.WL_CALL_EXPV}

    def workspace_size(self, call, b, outer_dim=0):
        """Bytes of device workspace one call ("apply_phi", "apply_L", "expv") needs."""
        v = C.c_size_t()
        check(load().wl_workspace_size(self.handle, self.CALLS[call], int(b), int(outer_dim), C.byref(v)))
        return v.value

    def _work(self, work):
        torch = _torch()
        if not (isinstance(work, torch.Tensor) and work.is_cuda and work.is_contiguous()):
            raise ValueError("work must be a contiguous device tensor")
        return _ptr(work), work.numel() * work.element_size()

    def apply_phi_ws(self, X, work, out=None):
        X = self._block(X)
        out = self._out(out, X)
        wp, wb = self._work(work)
        check(load().wl_apply_phi_ws(self.handle, _ptr(X), _ptr(out), X.shape[1], wp, wb))
        return out

    def apply_L_ws(self, X, work, out=None):
        X = self._block(X)
        out = self._out(out, X)
        wp, wb = self._work(work)
        check(load().wl_apply_L_ws(self.handle, _ptr(X), _ptr(out), X.shape[1], wp, wb))
        return out

    def apply_L_noalloc(self, X, out):
        """L X on the library's fixed region; out must be given (nothing is allocated)."""
        X = self._block(X)
        out = self._out(out, X)
        check(load().wl_apply_L_noalloc(self.handle, _ptr(X), _ptr(out), X.shape[1]))
        return out

    def expv_ws(self, U0, ts, work, outer_dim=30, outs=None):
        U0 = self._block(U0)
        ts = [float(t) for t in ts]
        torch = _torch()
        outs = [torch.empty_like(U0) for _ in ts] if outs is None else outs
        if len(outs) != len(ts):
            raise ValueError("one output block per time is needed")
        outs = [self._out(o, U0) for o in outs]
        tarr = (C.c_double * len(ts))(*ts)
        parr = (C.c_void_p * len(ts))(*[o.data_ptr() for o in outs])
        err = (C.c_double * len(ts))()
        wp, wb = self._work(work)
        check(load().wl_expv_ws(self.handle, _ptr(U0), U0.shape[1], tarr, len(ts), parr, int(outer_dim), err, wp, wb))
        return outs, list(err)

    def markov_step(self, X, steps=1, out=None):
        """Distributions held as the columns of X (n x b) after `steps` steps of the
        chain P = diag(w)^{-1} phi (p_{k+1} = p_k P)."""
        X = self._block(X)
        out = self._out(out, X)
        check(load().wl_markov_step(self.handle, _ptr(X), X.shape[1], int(steps), _ptr(out)))
        return out

    def markov_stationary(self, out=None):
        """pi = w / sum(w), the chain's stationary distribution."""
        out = self._empty(self.graph.n) if out is None else out
        _need(out, "out", self.dtype, (self.graph.n,))
        check(load().wl_markov_stationary(self.handle, _ptr(out)))
        return out

    def markov_gap(self, outer_dim=60, seed=7):
        """(lambda_2, lambda_min, gap) of the chain, by Lanczos on its symmetrised form."""
        l2, lm, gp = C.c_double(), C.c_double(), C.c_double()
        check(load().wl_markov_gap(self.handle, int(outer_dim), int(seed), C.byref(l2), C.byref(lm), C.byref(gp)))
        return l2.value, lm.value, gp.value

    def return_prob(self, Omega, ts, t_max, rho=0.0, pole_time=1.0, aaa_tol=1e-13, solve_tol=1e-6,
                    max_iters=500, rcond=1e-10):
        """Alg. 1: (p_hat, e_hat, poles, info) for the times ts, from the probe block
        Omega (n x M): AAA poles of exp(-x) on [0, t_max rho] / pole_time, the block
        rational Krylov basis, and the leave-one-out Nystrom estimate for every t."""
        import numpy as np
        Omega = self._block(Omega)
        ts = np.ascontiguousarray(ts, dtype=np.float64)
        nt = ts.size
        p = np.empty(nt)
        e = np.empty(nt)
        cap = 256
        pol = np.zeros(2 * cap)
        info = RkInfo()
        check(load().wl_return_prob(self.handle, _ptr(Omega), Omega.shape[1], _dptr(ts), nt, float(t_max), float(rho),
                                    float(pole_time), float(aaa_tol), float(solve_tol), int(max_iters), float(rcond),
                                    _dptr(p), _dptr(e), _dptr(pol), cap, C.byref(info)))
        k = min(info.npoles, cap)
        poles = pol[0:2 * k:2] + 1j * pol[1:2 * k:2]
        return p, e, poles, {f: getattr(info, f) for f, _ in RkInfo._fields_}

    def diag_est(self, M, seed, target="phi", t=0.0, law="gauss", estimator="hutchinson", cv=None, outer_dim=30):
        out = self._empty(self.graph.n)
        if cv is not None:
            _need(cv, "cv", self.dtype, (self.graph.n,))
        tr, te = C.c_double(), C.c_double()
        check(load().wl_diag_est(self.handle, 0 if target == "phi" else 1, float(t), int(M), int(seed), LAWS[law],
                                 ESTIMATORS[estimator], _ptr(cv), int(outer_dim), _ptr(out), C.byref(tr),
                                 C.byref(te)))
        return out, tr.value, te.value

    def surrogate_diag(self):
        """(base, scale): exact degree-3 part of diag phi and the scale of the rest (n each)."""
        base, scale = self._empty(self.graph.n), self._empty(self.graph.n)
        check(load().wl_surrogate_diag(self.handle, _ptr(base), _ptr(scale)))
        return base, scale

    def surrogate_target(self, nodes, width=32):
        """(diag phi - base) / scale at the given nodes (training targets)."""
        torch = _torch()
        nodes = torch.as_tensor(nodes).to(device=self.graph.ctx.torch_device, dtype=torch.int32).contiguous()
        out = self._empty(nodes.numel())
        check(load().wl_surrogate_target(self.handle, _ptr(nodes), nodes.numel(), int(width), _ptr(out)))
        return out

    def diag_exact(self, nodes, width=32):
        """phi[i, i] for the given node indices (unit-vector blocks through the operator)."""
        torch = _torch()
        nodes = torch.as_tensor(nodes).to(device=self.graph.ctx.torch_device, dtype=torch.int32).contiguous()
        out = self._empty(nodes.numel())
        check(load().wl_diag_exact(self.handle, _ptr(nodes), nodes.numel(), int(width), _ptr(out)))
        return out

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            load().wl_op_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def block_gram(ctx, X, Y, nblk=1):
    """[X_0 .. X_{nblk-1}]^T Y (double) for X of shape (nblk*n, bx) viewed as nblk blocks."""
    import numpy as np
    X = X.contiguous()
    Y = Y.contiguous()
    n, by = Y.shape
    bx = X.shape[1]
    _need(Y, "Y", X.dtype, (n, by))
    _need(X, "X", X.dtype, (nblk * n, bx))
    G = np.empty((nblk * bx, by), dtype=np.float64)
    check(load().wl_block_gram(ctx.handle, _prec_of(X.dtype), n, nblk, bx, _ptr(X), by, _ptr(Y),
                               G.ctypes.data_as(C.POINTER(C.c_double))))
    return G


def block_update(ctx, X, Cm, Yin=None, alpha=0.0, beta=1.0, out=None, nblk=1, want_gram=False):
    """alpha Yin + beta sum_k X_k C_k (and optionally its Gram)."""
    import numpy as np
    torch = _torch()
    X = X.contiguous()
    b = X.shape[1]
    n = X.shape[0] // nblk
    Cm = np.ascontiguousarray(Cm, dtype=np.float64)
    out = torch.empty((n, b), dtype=X.dtype, device=X.device) if out is None else out
    _need(X, "X", X.dtype, (nblk * n, b))
    if Cm.size != nblk * b * b:
        raise ValueError(f"C must hold {nblk} blocks of {b} x {b}")
    if Yin is not None:
        _need(Yin, "Yin", X.dtype, (n, b))
    _need(out, "out", X.dtype, (n, b))
    G = np.empty((b, b), dtype=np.float64) if want_gram else None
    check(load().wl_block_update(ctx.handle, _prec_of(X.dtype), n, nblk, b, _ptr(X),
                                 Cm.ctypes.data_as(C.POINTER(C.c_double)), _ptr(Yin), float(alpha), float(beta),
                                 _ptr(out), G.ctypes.data_as(C.POINTER(C.c_double)) if want_gram else None))
    return (out, G) if want_gram else out


def _poles_out(status, pol, npoles, cap):
    check(status)
    k = min(npoles.value, cap)
    return pol[0:2 * k:2] + 1j * pol[1:2 * k:2]


def aaa(Z, F, tol=1e-13, mmax=100):
    """AAA on real samples F = f(Z) (host computation): (poles, max error on Z)."""
    import numpy as np
    Z = np.ascontiguousarray(Z, dtype=np.float64)
    F = np.ascontiguousarray(F, dtype=np.float64)
    cap = max(1, min(mmax, Z.size))
    pol = np.zeros(2 * cap)
    npoles, err = C.c_int32(), C.c_double()
    st = load().wl_aaa(Z.size, _dptr(Z), _dptr(F), float(tol), int(mmax), _dptr(pol), cap, C.byref(npoles),
                       C.byref(err))
    return _poles_out(st, pol, npoles, cap), err.value


def exp_poles(xmax, tol=1e-13, mmax=100):
    """The AAA poles of exp(-x) on [0, xmax] that the rational Krylov estimate uses."""
    import numpy as np
    cap = mmax
    pol = np.zeros(2 * cap)
    npoles, err = C.c_int32(), C.c_double()
    st = load().wl_exp_poles(float(xmax), float(tol), int(mmax), _dptr(pol), cap, C.byref(npoles), C.byref(err))
    return _poles_out(st, pol, npoles, cap), err.value


def amg_describe(n, rowptr, colidx, mu, alpha, max_levels=20):
    """Host-only view of the multigrid hierarchy for a CSR graph (numpy int32 arrays):
    (rows per level, entries per level, finest-level aggregates)."""
    import numpy as np
    rp = np.ascontiguousarray(rowptr, dtype=np.int32)
    ci = np.ascontiguousarray(colidx, dtype=np.int32)
    lv = C.c_int32()
    rows = (C.c_int64 * max_levels)()
    nnz = (C.c_int64 * max_levels)()
    agg = np.empty(int(n), dtype=np.int32)
    check(load().wl_amg_describe(int(n), rp.ctypes.data, ci.ctypes.data, float(mu), float(alpha), int(max_levels),
                                 C.byref(lv), rows, nnz, agg.ctypes.data))
    return list(rows[:lv.value]), list(nnz[:lv.value]), agg


def probes(ctx, n, M, seed, law="gauss", dtype=None, stream=0):
    torch = _torch()
    dtype = dtype or torch.float32
    out = torch.empty((n, M), dtype=dtype, device=ctx.torch_device)
    check(load().wl_probes(ctx.handle, _prec_of(dtype), LAWS[law], int(seed), int(stream), n, M, _ptr(out)))
    return out


def estimate(ctx, Omega, Y, estimator="hutchinson", cv=None, rcond=1e-10, want_diag=True):
    torch = _torch()
    Omega = Omega.contiguous()
    Y = Y.contiguous()
    n, M = Omega.shape
    _need(Y, "Y", Omega.dtype, (n, M))
    if cv is not None:
        _need(cv, "cv", Omega.dtype, (n,))
    diag = torch.empty(n, dtype=Omega.dtype, device=Omega.device) if want_diag else None
    tr, te = C.c_double(), C.c_double()
    check(load().wl_estimate(ctx.handle, _prec_of(Omega.dtype), ESTIMATORS[estimator], n, M, _ptr(Omega), _ptr(Y),
                             _ptr(cv), float(rcond), _ptr(diag), C.byref(tr), C.byref(te)))
    return diag, tr.value, te.value


class MLP:
    """The control-variate network (8 -> 64 -> 64 -> 1, tanh), trained on the device."""

    def __init__(self, ctx, params=None, handle=None):
        import numpy as np
        self.ctx = ctx
        lib = load()
        self.nparams = lib.wl_mlp_num_params()
        self.handle = C.c_void_p()
        if handle is not None:
            self.handle = handle
            return
        arr = None if params is None else np.ascontiguousarray(params, dtype=np.float32)
        check(lib.wl_mlp_create(ctx.handle, arr.ctypes.data_as(C.c_void_p) if arr is not None else None,
                                C.byref(self.handle)))

    @classmethod
    def load_file(cls, ctx, path):
        h = C.c_void_p()
        check(load().wl_mlp_load(ctx.handle, str(path).encode(), C.byref(h)))
        return cls(ctx, handle=h)

    def save(self, path):
        check(load().wl_mlp_save(self.handle, str(path).encode()))

    def params(self):
        import numpy as np
        out = np.empty(self.nparams, dtype=np.float32)
        check(load().wl_mlp_get_params(self.handle, out.ctypes.data_as(C.c_void_p)))
        return out

    def forward(self, feat, out=None):
        torch = _torch()
        feat = _need(feat.contiguous(), "feat", torch.float32, (None, 8))
        out = torch.empty(feat.shape[0], dtype=torch.float32, device=feat.device) if out is None else out
        _need(out, "out", torch.float32, (feat.shape[0],))
        check(load().wl_mlp_forward(self.handle, _ptr(feat), feat.shape[0], _ptr(out)))
        return out

    def predict(self, feat, base=None, scale=None, out=None):
        """base + scale * net(feat) (FP32)."""
        torch = _torch()
        feat = _need(feat.contiguous(), "feat", torch.float32, (None, 8))
        n = feat.shape[0]
        for t, name in ((base, "base"), (scale, "scale")):
            if t is not None:
                _need(t, name, torch.float32, (n,))
        out = torch.empty(n, dtype=torch.float32, device=feat.device) if out is None else out
        _need(out, "out", torch.float32, (n,))
        check(load().wl_mlp_predict(self.handle, _ptr(feat), n, _ptr(base), _ptr(scale), _ptr(out)))
        return out

    def loss_grad(self, feat, target):
        import numpy as np
        torch = _torch()
        g = np.empty(self.nparams, dtype=np.float64)
        loss = C.c_double()
        feat = _need(feat.contiguous(), "feat", torch.float32, (None, 8))
        target = _need(target.contiguous(), "target", torch.float32, (feat.shape[0],))
        check(load().wl_mlp_loss_grad(self.handle, _ptr(feat), _ptr(target),
                                      feat.shape[0], C.byref(loss), g.ctypes.data_as(C.c_void_p)))
        return loss.value, g

    def train_step(self, feat, target, lr):
        torch = _torch()
        _need(feat, "feat", torch.float32, (None, 8))
        _need(target, "target", torch.float32, (feat.shape[0],))
        loss = C.c_double()
        check(load().wl_mlp_train_step(self.handle, _ptr(feat), _ptr(target), feat.shape[0], float(lr),
                                       C.byref(loss)))
        return loss.value

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            load().wl_mlp_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Multi:
    """Several operators of one graph (all truncated series or all Lanczos) evaluated
    side by side on one wide block."""

    def __init__(self, ops):
        self.ops = list(ops)
        self.graph = self.ops[0].graph
        self.dtype = self.ops[0].dtype
        handles = (C.c_void_p * len(self.ops))(*[o.handle.value for o in self.ops])
        self.handle = C.c_void_p()
        check(load().wl_multi_create(handles, len(self.ops), C.byref(self.handle)))

    def _run(self, X, out, laplacian):
        torch = _torch()
        X = X.to(self.dtype).contiguous()
        if X.dim() == 1:
            X = X.view(-1, 1)
        _need(X, "X", self.dtype, (self.graph.n, None))
        shape = (self.graph.n, X.shape[1] * len(self.ops))
        out = torch.empty(shape, dtype=self.dtype, device=X.device) if out is None else out
        _need(out, "out", self.dtype, shape)
        check(load().wl_multi_apply(self.handle, _ptr(X), X.shape[1], _ptr(out), 1 if laplacian else 0))
        return out

    def apply_phi(self, X, out=None):
        """n x (nops b): group g = phi_g X."""
        return self._run(X, out, False)

    def apply_L(self, X, out=None):
        """n x (nops b): group g = L_g X."""
        return self._run(X, out, True)

    def fdeg(self, out=None):
        """n x nops: column g = phi_g 1."""
        torch = _torch()
        shape = (self.graph.n, len(self.ops))
        out = torch.empty(shape, dtype=self.dtype, device=self.graph.ctx.torch_device) if out is None else out
        _need(out, "out", self.dtype, shape)
        check(load().wl_multi_fdeg(self.handle, _ptr(out)))
        return out

    def apply_fdeg(self, X, laplacian=True, out=None, out_w=None, nx=None):
        """(Y, W) in one evaluation: Y n x (nx b) with group g = L_g X (or phi_g X) for
        the first nx operators (all by default), W n x nops with column g = phi_g 1."""
        torch = _torch()
        X = X.to(self.dtype).contiguous()
        if X.dim() == 1:
            X = X.view(-1, 1)
        _need(X, "X", self.dtype, (self.graph.n, None))
        nx = len(self.ops) if nx is None else int(nx)
        shape = (self.graph.n, X.shape[1] * nx)
        out = torch.empty(shape, dtype=self.dtype, device=X.device) if out is None else out
        _need(out, "out", self.dtype, shape)
        wshape = (self.graph.n, len(self.ops))
        out_w = torch.empty(wshape, dtype=self.dtype, device=X.device) if out_w is None else out_w
        _need(out_w, "out_w", self.dtype, wshape)
        check(load().wl_multi_apply_fdeg(self.handle, _ptr(X), X.shape[1], nx, _ptr(out), _ptr(out_w),
                                         1 if laplacian else 0))
        return out, out_w

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            load().wl_multi_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many graphs evaluated together (one launch per Krylov step for the whole batch)."""

    def __init__(self, ctx, graphs, descs, tol=1e-10):
        """descs: list of dicts with mu, func ('exp' / 'res'), param [, krylov_dim, rho_hint]."""
        self.ctx = ctx
        self.graphs = list(graphs)
        arr = (_lib.OpDesc * len(graphs))()
        for i, d in enumerate(descs):
            arr[i] = _lib.OpDesc(mu=float(d["mu"]), func=FUNCS[d["func"]], param=float(d["param"]), prec=WL_FP32,
                                 krylov_dim=int(d.get("krylov_dim", 0)), tol=0.0, method=WL_M_RECURRENCE, reorth=1,
                                 rho_hint=float(d.get("rho_hint", 0.0)))
        handles = (C.c_void_p * len(graphs))(*[g.handle.value for g in graphs])
        self.handle = C.c_void_p()
        check(load().wl_batch_create(ctx.handle, len(graphs), handles, arr, float(tol), C.byref(self.handle)))
        import numpy as np
        total, kmax = C.c_int64(), C.c_int32()
        offs = np.zeros(len(graphs), dtype=np.int64)
        degs = np.zeros(len(graphs), dtype=np.int32)
        check(load().wl_batch_info(self.handle, C.byref(total), C.byref(kmax), offs.ctypes.data_as(C.c_void_p),
                                   degs.ctypes.data_as(C.c_void_p)))
        self.total_rows, self.max_series_degree, self.offsets = total.value, kmax.value, offs
        self.series_degrees = degs
        self.sizes = [g.n for g in graphs]

    def pack(self, blocks):
        """Place per-graph (n_g x b) tensors at their row offsets in one zero-padded block."""
        torch = _torch()
        b = blocks[0].shape[1]
        out = torch.zeros((self.total_rows, b), dtype=torch.float32, device=self.ctx.torch_device)
        for o, blk in zip(self.offsets, blocks):
            out[int(o):int(o) + blk.shape[0]] = blk.to(torch.float32)
        return out

    def unpack(self, packed):
        return [packed[int(o):int(o) + n] for o, n in zip(self.offsets, self.sizes)]

    def autotune(self, b):
        check(load().wl_batch_autotune(self.handle, int(b)))

    @property
    def xcd_grouped(self):
        v = C.c_int32()
        check(load().wl_batch_tile_order(self.handle, C.byref(v)))
        return bool(v.value)

    @xcd_grouped.setter
    def xcd_grouped(self, on):
        check(load().wl_batch_set_tile_order(self.handle, 1 if on else 0))

    def _blocks(self, X, out):
        torch = _torch()
        _need(X, "X", torch.float32, (self.total_rows, None))
        out = torch.empty_like(X) if out is None else out
        return _need(out, "out", torch.float32, tuple(X.shape))

    def apply_L(self, X, out=None):
        out = self._blocks(X, out)
        check(load().wl_batch_apply_L(self.handle, _ptr(X), _ptr(out), X.shape[1]))
        return out

    def expv(self, U0, ts, outer_dim=30, out=None, want_trace=True):
        import numpy as np
        torch = _torch()
        out = self._blocks(U0, out)
        t = np.ascontiguousarray(ts, dtype=np.float64)
        if t.shape != (len(self.graphs),):
            raise ValueError("one time per graph is needed")
        ph = np.zeros(len(self.graphs))
        pe = np.zeros(len(self.graphs))
        pd_ = C.POINTER(C.c_double)
        check(load().wl_batch_expv(self.handle, _ptr(U0), U0.shape[1], t.ctypes.data_as(pd_), int(outer_dim),
                                   _ptr(out), ph.ctypes.data_as(pd_) if want_trace else None,
                                   pe.ctypes.data_as(pd_) if want_trace else None))
        return out, ph, pe

    def graph(self, U0, Y, outer_dim=30):
        """Capture the batched diffusion for these fixed buffers (see BatchGraph)."""
        return BatchGraph(self, U0, Y, outer_dim)

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            load().wl_batch_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchGraph:
    """A captured batched diffusion bound to fixed U0 / Y buffers; launch() replays it."""

    def __init__(self, batch, U0, Y, outer_dim=30):
        torch = _torch()
        _need(U0, "U0", torch.float32, (batch.total_rows, None))
        _need(Y, "Y", torch.float32, tuple(U0.shape))
        self.batch, self.U0, self.Y = batch, U0, Y  # keep the buffers (and the batch) alive
        self.handle = C.c_void_p()
        check(load().wl_batch_graph_create(batch.handle, _ptr(U0), U0.shape[1], int(outer_dim), _ptr(Y),
                                           C.byref(self.handle)))

    def launch(self, ts, want_trace=False):
        import numpy as np
        t = np.ascontiguousarray(ts, dtype=np.float64)
        if t.shape != (len(self.batch.graphs),):
            raise ValueError("one time per graph is needed")
        ng = len(self.batch.graphs)
        ph, pe = np.zeros(ng), np.zeros(ng)
        pd_ = C.POINTER(C.c_double)
        check(load().wl_batch_graph_launch(self.handle, t.ctypes.data_as(pd_),
                                           ph.ctypes.data_as(pd_) if want_trace else None,
                                           pe.ctypes.data_as(pd_) if want_trace else None))
        return (ph, pe) if want_trace else None

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            load().wl_batch_graph_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
