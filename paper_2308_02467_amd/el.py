"""ctypes binding of the C ABI in include/el.h (libel.so, built for gfx950).

Argument marshalling only: torch tensors provide device memory and the
stream; every step of the hot path runs in the library's HIP kernels.  The
binding raises if the library is missing -- there is no CPU fallback.
Function names match the C entry points.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libel.so")

EL_OK = 0
EL_WARN_NOT_CONVERGED = 1
EL_ERR_ARG = -1
EL_ERR_HIP = -2
EL_ERR_SINGULAR = -3
EL_ERR_NONFINITE = -4
EL_ERR_NOMEM = -5
EL_SCATTER_ISO = 0
EL_SCATTER_HG = 1
EL_FP64 = 0
EL_FP32_IR = 1
EL_F64 = 0
EL_BF16 = 1
EL_F32 = 2
EL_F16 = 3
EL_ANG_ORDINATES = 0
EL_ANG_P0 = 1

_ERRNAMES = {EL_ERR_ARG: "EL_ERR_ARG", EL_ERR_HIP: "EL_ERR_HIP", EL_ERR_SINGULAR: "EL_ERR_SINGULAR",
             EL_ERR_NONFINITE: "EL_ERR_NONFINITE", EL_ERR_NOMEM: "EL_ERR_NOMEM"}


class ElError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


class el_disc(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int), ("n_a", ctypes.c_int), ("scatter", ctypes.c_int), ("g_hg", ctypes.c_double),
                ("angular", ctypes.c_int)]


class el_mesh(ctypes.Structure):
    _fields_ = [("n_x", ctypes.c_int), ("n_y", ctypes.c_int), ("x0", ctypes.c_double),
                ("y0", ctypes.c_double), ("h", ctypes.c_double)]


class el_net_desc(ctypes.Structure):
    _fields_ = [("n_in", ctypes.c_int), ("width", ctypes.c_int), ("depth", ctypes.c_int), ("act", ctypes.c_int),
                ("n_out", ctypes.c_int64), ("seed", ctypes.c_uint64)]


EL_ACT_GELU = 0
EL_ACT_ELU = 1
EL_ACT_LINEAR = 2
EL_FORM_IN2SOL, EL_FORM_IN2MEAN = 0, 1


class el_gmres_opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("restart", ctypes.c_int), ("max_iter", ctypes.c_int),
                ("graph", ctypes.c_int), ("x0", ctypes.c_int), ("basis", ctypes.c_int)]


class el_gmres_report(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("restarts", ctypes.c_int), ("relres", ctypes.c_double),
                ("converged", ctypes.c_int), ("reorth_passes", ctypes.c_int)]


_lib = None

_SIGS = {
    "el_create": [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.c_void_p],
    "el_destroy": [ctypes.c_void_p],
    "el_set_stream": [ctypes.c_void_p, ctypes.c_void_p],
    "el_last_error": [ctypes.c_void_p],
    "el_workspace_bytes": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)],
    "el_disc_sizes": [el_disc, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                      ctypes.POINTER(ctypes.c_int64)],
    "el_lgl": [ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)],
    "el_index_tables": [el_disc, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)],
    "el_angular_tables": [el_disc, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)],
    "el_trace_size": [el_disc, el_mesh, ctypes.POINTER(ctypes.c_int64)],
    "el_element_dofs": [ctypes.c_void_p, el_disc, el_mesh, ctypes.c_void_p, ctypes.c_void_p],
    "el_local_solve": [ctypes.c_void_p, el_disc, ctypes.c_int, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p],
    "el_trace_rhs": [ctypes.c_void_p, el_disc, el_mesh, ctypes.POINTER(ctypes.c_double), ctypes.c_void_p],
    "el_trace_rhs_nodal": [ctypes.c_void_p, el_disc, el_mesh, ctypes.c_void_p, ctypes.c_void_p],
    "el_trace_add_source": [ctypes.c_void_p, el_disc, el_mesh, ctypes.c_void_p, ctypes.c_void_p],
    "el_trace_matvec": [ctypes.c_void_p, el_disc, el_mesh, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                        ctypes.c_void_p],
    "el_gemm_tile": [ctypes.c_int],
    "el_matvec_shape": [ctypes.c_int],
    "el_tuning_report": [ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)],
    "el_tuning_save": [ctypes.c_char_p],
    "el_tuning_load": [ctypes.c_char_p, ctypes.POINTER(ctypes.c_int64)],
    "el_tuning_reset": [],
    "el_trace_solve": [ctypes.c_void_p, el_disc, ctypes.c_int, ctypes.POINTER(el_mesh),
                       ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.POINTER(ctypes.c_void_p),
                       ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(el_gmres_opts),
                       ctypes.POINTER(el_gmres_report)],
    "el_recover": [ctypes.c_void_p, el_disc, el_mesh, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p],
    "el_recover_mean": [ctypes.c_void_p, el_disc, el_mesh, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                        ctypes.c_void_p, ctypes.c_void_p],
    "el_mean_l2": [ctypes.c_void_p, el_disc, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                   ctypes.POINTER(ctypes.c_double)],
    "el_conserve": [ctypes.c_void_p, el_disc, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                    ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int],
    "el_net_create": [ctypes.c_void_p, ctypes.POINTER(el_net_desc), ctypes.POINTER(ctypes.c_void_p)],
    "el_net_destroy": [ctypes.c_void_p],
    "el_net_save": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)],
    "el_net_load": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_void_p)],
    "el_net_fit_normalization": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                 ctypes.c_void_p],
    "el_net_params": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p],
    "el_net_num_params": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)],
    "el_make_pairs": [ctypes.c_void_p, el_disc, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                      ctypes.c_int, ctypes.c_void_p],
    "el_train_step": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                      ctypes.c_float, ctypes.c_void_p],
    "el_net_forward": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p],
    "el_train_step_f32": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                          ctypes.c_float, ctypes.c_void_p],
    "el_net_forward_f32": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                           ctypes.c_int],
    "el_infer": [ctypes.c_void_p, ctypes.c_void_p, el_disc, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                 ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
                 ctypes.c_int, ctypes.POINTER(ctypes.c_int64)],
    "el_stream_read": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p],
    "el_infer_noalloc": [ctypes.c_void_p, ctypes.c_void_p, el_disc, ctypes.c_int64, ctypes.c_void_p,
                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                         ctypes.c_void_p],
}


def lib():
    """Load libel.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} not found: build it with paper_2308_02467_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_char_p if name == "el_last_error" else ctypes.c_int
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS)


def disc(p, n_a, g_hg=0.0, angular=None):
    """angular: EL_ANG_ORDINATES (default) or EL_ANG_P0."""
    return el_disc(int(p), int(n_a), EL_SCATTER_HG if g_hg else EL_SCATTER_ISO, float(g_hg),
                   EL_ANG_ORDINATES if angular is None else int(angular))


def mesh(n_x, n_y, h, x0=0.0, y0=0.0):
    return el_mesh(int(n_x), int(n_y), float(x0), float(y0), float(h))


def disc_sizes(d):
    nn, n, m = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    st = lib().el_disc_sizes(d, ctypes.byref(nn), ctypes.byref(n), ctypes.byref(m))
    if st != EL_OK:
        raise ElError(st, "unsupported discretization")
    return nn.value, n.value, m.value


def lgl(p):
    import numpy as np
    xi = (ctypes.c_double * (p + 1))()
    w = (ctypes.c_double * (p + 1))()
    st = lib().el_lgl(int(p), xi, w)
    if st != EL_OK:
        raise ElError(st, "el_lgl")
    return np.array(xi[:]), np.array(w[:])


def angular_tables(d):
    """(s [n_a, 2], Q [n_a, n_a]) of the discretization, from the host tables."""
    import numpy as np
    na = int(d.n_a)
    sb = (ctypes.c_double * (2 * na))()
    qb = (ctypes.c_double * (na * na))()
    st = lib().el_angular_tables(d, sb, qb)
    if st != EL_OK:
        raise ElError(st, "el_angular_tables")
    return np.array(sb).reshape(na, 2), np.array(qb).reshape(na, na)


def index_tables(d):
    import numpy as np
    _, _, m = disc_sizes(d)
    a = (ctypes.c_int32 * m)()
    b = (ctypes.c_int32 * m)()
    st = lib().el_index_tables(d, a, b)
    if st != EL_OK:
        raise ElError(st, "el_index_tables")
    return np.array(a[:], dtype=np.int64), np.array(b[:], dtype=np.int64)


def trace_size(d, ms):
    n = ctypes.c_int64()
    st = lib().el_trace_size(d, ms, ctypes.byref(n))
    if st != EL_OK:
        raise ElError(st, "el_trace_size")
    return n.value


def _ptr(t, dtype=None, numel=None, name="tensor"):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


def _op_dtype(t):
    if t.dtype == torch.float64:
        return EL_F64
    if t.dtype == torch.float32:
        return EL_F32
    if t.dtype == torch.float16:
        return EL_F16
    if t.dtype in (torch.bfloat16, torch.int16, torch.uint16):
        return EL_BF16
    raise ValueError(f"operator dtype {t.dtype} not supported (float64, float32, float16 or bfloat16)")


class Context:
    """One library context bound to a device and a HIP stream."""

    def __init__(self, device=0, stream=None):
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = ctypes.c_void_p()
        st = lib().el_create(ctypes.byref(h), int(device), ctypes.c_void_p(stream.cuda_stream))
        if st != EL_OK:
            raise ElError(st, "el_create failed")
        self.h = h

    def close(self):
        if self.h:
            lib().el_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, allow_warn=False):
        if st == EL_OK or (allow_warn and st == EL_WARN_NOT_CONVERGED):
            return st
        raise ElError(st, lib().el_last_error(self.h).decode())

    def last_error(self):
        return lib().el_last_error(self.h).decode()

    def workspace_bytes(self):
        b = ctypes.c_size_t()
        self._check(lib().el_workspace_bytes(self.h, ctypes.byref(b)))
        return b.value

    # -- local solve -----------------------------------------------------------
    def el_local_solve(self, d, h, kappa, sigma, precision=EL_FP64, in2out=None, in2sol=None, in2mean=None,
                       rel_resid=None, src=None, src2out=None, src2sol=None, src2mean=None):
        """src: nodal volume source [E][n_a][nn]; its responses f_hat_u
        (src2out [E][m]), f_u (src2sol [E][n]) and their ordinate average
        (src2mean [E][nn])."""
        nn, n, m = disc_sizes(d)
        E = h.numel()
        args = [_ptr(h, torch.float64, E, "h"), _ptr(kappa, torch.float64, E * nn, "kappa"),
                _ptr(sigma, torch.float64, E * nn, "sigma"),
                _ptr(in2out, torch.float64, E * m * m, "in2out"), _ptr(in2sol, torch.float64, E * n * m, "in2sol"),
                _ptr(in2mean, torch.float64, E * nn * m, "in2mean"),
                _ptr(rel_resid, torch.float64, E, "rel_resid"),
                _ptr(src, torch.float64, E * n, "src"), _ptr(src2out, torch.float64, E * m, "src2out"),
                _ptr(src2sol, torch.float64, E * n, "src2sol"), _ptr(src2mean, torch.float64, E * nn, "src2mean")]
        return self._check(lib().el_local_solve(self.h, d, int(precision), E, *args))

    def el_element_dofs(self, d, ms, in_dofs=None, out_dofs=None):
        _, _, m = disc_sizes(d)
        E = ms.n_x * ms.n_y
        return self._check(lib().el_element_dofs(self.h, d, ms, _ptr(in_dofs, torch.int32, E * m, "in_dofs"),
                                                 _ptr(out_dofs, torch.int32, E * m, "out_dofs")))

    # -- skeleton ----------------------------------------------------------------
    def el_trace_rhs(self, d, ms, g_side, b):
        import numpy as np
        g = np.ascontiguousarray(np.asarray(g_side, dtype=np.float64).reshape(4, d.n_a))
        nt = trace_size(d, ms)
        return self._check(lib().el_trace_rhs(self.h, d, ms, g.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                              _ptr(b, torch.float64, nt, "b")))

    def el_trace_rhs_nodal(self, d, ms, g_bnd, b):
        """b from boundary radiance g_bnd [2 (n_x + n_y), n_a, p + 1] (faces of
        the sides W, E, S, N in that order, FP64 on the device)."""
        nt = trace_size(d, ms)
        n_bnd = 2 * (ms.n_x + ms.n_y) * d.n_a * (d.p + 1)
        return self._check(lib().el_trace_rhs_nodal(self.h, d, ms, _ptr(g_bnd, torch.float64, n_bnd, "g_bnd"),
                                                    _ptr(b, torch.float64, nt, "b")))

    def el_stream_read(self, buf, sink):
        """Streaming-read reference: read every byte of the device tensor buf
        once; sink: one-element int32 device tensor receiving the XOR of the
        32-bit words read."""
        if not buf.is_contiguous():
            raise ValueError("buf must be contiguous")
        return self._check(lib().el_stream_read(self.h, _ptr(buf, name="buf"), buf.numel() * buf.element_size(),
                                                _ptr(sink, torch.int32, 1, "sink")))

    def el_trace_matvec(self, d, ms, in2out, x, y):
        nt = trace_size(d, ms)
        return self._check(lib().el_trace_matvec(self.h, d, ms, _ptr(in2out, name="in2out"), _op_dtype(in2out),
                                                 _ptr(x, torch.float64, nt, "x"), _ptr(y, torch.float64, nt, "y")))

    def el_trace_solve(self, d, meshes, in2outs, bs, traces, tol=1e-12, restart=50, max_iter=2000, graph=True,
                       x0=False, basis=torch.float64):
        """x0: start from the values in traces instead of zero; basis: storage
        of the Krylov basis (torch.float64 or torch.float32)."""
        if basis not in (torch.float64, torch.float32):
            raise ValueError("basis must be torch.float64 or torch.float32")
        k = len(meshes)
        M = (el_mesh * k)(*meshes)
        ops = (ctypes.c_void_p * k)(*[_ptr(t, name="in2out") for t in in2outs])
        dt = {_op_dtype(t) for t in in2outs}
        if len(dt) != 1:
            raise ValueError("all operators must share one dtype")
        B = (ctypes.c_void_p * k)(*[_ptr(b, torch.float64, trace_size(d, ms), "b") for b, ms in zip(bs, meshes)])
        X = (ctypes.c_void_p * k)(*[_ptr(x, torch.float64, trace_size(d, ms), "trace") for x, ms in zip(traces, meshes)])
        opts = el_gmres_opts(float(tol), int(restart), int(max_iter), int(bool(graph)), int(bool(x0)),
                             EL_F32 if basis == torch.float32 else EL_F64)
        rep = (el_gmres_report * k)()
        st = lib().el_trace_solve(self.h, d, k, M, ops, dt.pop(), B, X, ctypes.byref(opts), rep)
        self._check(st, allow_warn=True)
        return st, [dict(iters=r.iters, restarts=r.restarts, relres=r.relres, converged=bool(r.converged),
                         reorth_passes=r.reorth_passes) for r in rep]

    # -- recovery ------------------------------------------------------------------
    def el_recover(self, d, ms, in2sol, trace, u=None, mean=None, src2sol=None):
        nn, n, _ = disc_sizes(d)
        E = ms.n_x * ms.n_y
        return self._check(lib().el_recover(self.h, d, ms, _ptr(in2sol, name="in2sol"), _op_dtype(in2sol),
                                            _ptr(trace, torch.float64, trace_size(d, ms), "trace"),
                                            _ptr(u, torch.float64, E * n, "u"),
                                            _ptr(mean, torch.float64, E * nn, "mean"),
                                            _ptr(src2sol, torch.float64, E * n, "src2sol")))

    def el_recover_mean(self, d, ms, in2mean, trace, mean, src2mean=None):
        nn, _, _ = disc_sizes(d)
        E = ms.n_x * ms.n_y
        return self._check(lib().el_recover_mean(self.h, d, ms, _ptr(in2mean, name="in2mean"), _op_dtype(in2mean),
                                                 _ptr(trace, torch.float64, trace_size(d, ms), "trace"),
                                                 _ptr(mean, torch.float64, E * nn, "mean"),
                                                 _ptr(src2mean, torch.float64, E * nn, "src2mean")))

    def el_trace_add_source(self, d, ms, src2out, b):
        _, _, m = disc_sizes(d)
        E = ms.n_x * ms.n_y
        return self._check(lib().el_trace_add_source(self.h, d, ms, _ptr(src2out, torch.float64, E * m, "src2out"),
                                                     _ptr(b, torch.float64, trace_size(d, ms), "b")))

    def el_conserve(self, d, h, kappa, in2out, in2sol=None, mask=None, in2mean=None, out=None):
        """Energy-balance correction of in2out given in2sol or in2mean, in place
        or (out given) into out, which may be float16 or bfloat16 when the
        operators are float32 (rounded once, after the correction)."""
        nn, n, m = disc_sizes(d)
        E = h.numel()
        if (in2sol is None) == (in2mean is None):
            raise ValueError("give exactly one of in2sol, in2mean")
        vol, form, rows = (in2sol, EL_FORM_IN2SOL, n) if in2sol is not None else (in2mean, EL_FORM_IN2MEAN, nn)
        dt = _op_dtype(in2out)
        if _op_dtype(vol) != dt:
            raise ValueError("in2out and the volume operator must share one dtype")
        odt = _op_dtype(out) if out is not None else dt
        return self._check(lib().el_conserve(self.h, d, E, _ptr(h, torch.float64, E, "h"),
                                             _ptr(kappa, torch.float64, E * nn, "kappa"),
                                             _ptr(in2out, numel=E * m * m, name="in2out"),
                                             _ptr(vol, numel=E * rows * m, name="in2vol"), form, dt,
                                             _ptr(mask, torch.uint8, E, "mask"),
                                             _ptr(out, numel=E * m * m, name="out"), odt))

    def el_mean_l2(self, d, h, a, ref):
        nn, _, _ = disc_sizes(d)
        E = h.numel()
        out = (ctypes.c_double * 2)()
        self._check(lib().el_mean_l2(self.h, d, E, _ptr(h, torch.float64, E, "h"),
                                     _ptr(a, torch.float64, E * nn, "a"), _ptr(ref, torch.float64, E * nn, "ref"),
                                     out))
        return out[0], out[1]


def _bf16_ptr(t, numel=None, name="tensor"):
    if t is None:
        return None
    if t.dtype not in (torch.bfloat16, torch.int16, torch.uint16):
        raise ValueError(f"{name} must hold bfloat16 bits (bfloat16 or int16 tensor), got {t.dtype}")
    return _ptr(t, None, numel, name)


class Net:
    """Element network state on one context (el_net_*)."""

    def __init__(self, ctx, handle):
        self.ctx = ctx
        self.h = handle
        n = ctypes.c_int64()
        lib().el_net_num_params(self.h, ctypes.byref(n))
        self.n_params = n.value

    @classmethod
    def create(cls, ctx, n_in, width, depth, n_out, act=EL_ACT_GELU, seed=0):
        d = el_net_desc(int(n_in), int(width), int(depth), int(act), int(n_out), int(seed))
        h = ctypes.c_void_p()
        ctx._check(lib().el_net_create(ctx.h, ctypes.byref(d), ctypes.byref(h)))
        return cls(ctx, h)

    @classmethod
    def load(cls, ctx, blob):
        buf = ctypes.create_string_buffer(bytes(blob), len(blob))
        h = ctypes.c_void_p()
        ctx._check(lib().el_net_load(ctx.h, buf, len(blob), ctypes.byref(h)))
        return cls(ctx, h)

    def save(self):
        n = ctypes.c_size_t()
        self.ctx._check(lib().el_net_save(self.ctx.h, self.h, None, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        self.ctx._check(lib().el_net_save(self.ctx.h, self.h, buf, ctypes.byref(n)))
        return buf.raw[:n.value]

    def close(self):
        if self.h:
            lib().el_net_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self, which=0):
        out = torch.empty(self.n_params, dtype=torch.float32, device=f"cuda:{self.ctx.device}")
        self.ctx._check(lib().el_net_params(self.ctx.h, self.h, int(which), _ptr(out)))
        return out

    def fit_normalization(self, x, y):
        N = x.shape[0]
        self.ctx._check(lib().el_net_fit_normalization(self.ctx.h, self.h, N, _ptr(x, torch.float32, name="x"),
                                                        _bf16_ptr(y, name="y")))

    def train_step(self, x, y, lr, loss=None):
        B = x.shape[0]
        self.ctx._check(lib().el_train_step(self.ctx.h, self.h, B, _ptr(x, torch.float32, name="x"),
                                            _bf16_ptr(y, name="y"), ctypes.c_float(lr),
                                            _ptr(loss, torch.float32, 1, "loss")))

    def forward(self, x, y_norm):
        self.ctx._check(lib().el_net_forward(self.ctx.h, self.h, x.shape[0], _ptr(x, torch.float32, name="x"),
                                             _ptr(y_norm, torch.float32, name="y_norm")))

    def train_step_f32(self, x, y, lr, loss=None):
        """el_train_step_f32: FP32 operands throughout, float32 targets y."""
        B = x.shape[0]
        self.ctx._check(lib().el_train_step_f32(self.ctx.h, self.h, B, _ptr(x, torch.float32, name="x"),
                                                _ptr(y, torch.float32, name="y"), ctypes.c_float(lr),
                                                _ptr(loss, torch.float32, 1, "loss")))

    def forward_f32(self, x, y, denormalize=False):
        """el_net_forward_f32: normalized outputs, or the operators with denormalize."""
        self.ctx._check(lib().el_net_forward_f32(self.ctx.h, self.h, x.shape[0], _ptr(x, torch.float32, name="x"),
                                                 _ptr(y, torch.float32, name="y"), int(bool(denormalize))))

    def infer(self, d, h, kappa, sigma, in2out=None, in2sol=None, in_range=None, fallback=True,
              precision=EL_FP64, in2mean=None):
        """in2out and in2sol (network in the in2sol form) or in2mean (in2mean
        form): bfloat16, float16 or float32 device tensors of one dtype."""
        E, dt, vol = self._infer_args(d, h, in2out, in2sol, in2mean)
        nn, _, _ = disc_sizes(d)
        nfb = ctypes.c_int64()
        self.ctx._check(lib().el_infer(self.ctx.h, self.h, d, E, _ptr(h, torch.float64, E, "h"),
                                       _ptr(kappa, torch.float64, E * nn, "kappa"),
                                       _ptr(sigma, torch.float64, E * nn, "sigma"),
                                       _ptr(in2out, name="in2out"), _ptr(vol, name="in2vol"), int(dt),
                                       _ptr(in_range, torch.uint8, E, "in_range"), int(bool(fallback)),
                                       int(precision), ctypes.byref(nfb)))
        return nfb.value

    def infer_noalloc(self, d, h, kappa, sigma, in2out=None, in2sol=None, in_range=None, in2mean=None):
        """el_infer_noalloc: no fallback, no allocation, no synchronization."""
        E, dt, vol = self._infer_args(d, h, in2out, in2sol, in2mean)
        nn, _, _ = disc_sizes(d)
        self.ctx._check(lib().el_infer_noalloc(self.ctx.h, self.h, d, E, _ptr(h, torch.float64, E, "h"),
                                               _ptr(kappa, torch.float64, E * nn, "kappa"),
                                               _ptr(sigma, torch.float64, E * nn, "sigma"),
                                               _ptr(in2out, name="in2out"), _ptr(vol, name="in2vol"), int(dt),
                                               _ptr(in_range, torch.uint8, E, "in_range")))

    def _infer_args(self, d, h, in2out, in2sol, in2mean):
        nn, n, m = disc_sizes(d)
        E = h.numel()
        if in2sol is not None and in2mean is not None:
            raise ValueError("give in2sol or in2mean, not both")
        vol = in2sol if in2sol is not None else in2mean
        rows = n if in2mean is None else nn
        ref = in2out if in2out is not None else vol
        dt = _op_dtype(ref) if ref is not None else EL_BF16
        if dt not in (EL_BF16, EL_F32, EL_F16):
            raise ValueError("learned operators are stored as bfloat16, float16 or float32")
        for t, cnt, name in ((in2out, E * m * m, "in2out"), (vol, E * rows * m, "in2sol/in2mean")):
            if t is not None and (_op_dtype(t) != dt or t.numel() != cnt):
                raise ValueError(f"{name}: expected {cnt} elements of the common dtype")
        return E, dt, vol


def el_make_pairs(ctx, d, h, kappa, sigma, y, form=None):
    """bfloat16 targets (in2out, in2sol) or, with form EL_FORM_IN2MEAN, (in2out, in2mean)."""
    nn, n, m = disc_sizes(d)
    E = h.numel()
    form = EL_FORM_IN2SOL if form is None else form
    rows = n if form == EL_FORM_IN2SOL else nn
    ctx._check(lib().el_make_pairs(ctx.h, d, E, _ptr(h, torch.float64, E, "h"),
                                   _ptr(kappa, torch.float64, E * nn, "kappa"),
                                   _ptr(sigma, torch.float64, E * nn, "sigma"), int(form),
                                   _bf16_ptr(y, E * (m * m + rows * m), "y")))


# ---- network state blob (format documented in include/el.h) -------------------
import struct as _struct

_HDR = "<8s6i3q6d"
HEADER_BYTES = 112


def net_layout(n_in, width, depth, n_out):
    """(k0, [(w_off, b_off, out, in) per layer], n_params) of the theta vector."""
    k0 = (n_in + 31) // 32 * 32
    layers = []
    off = 0
    for l in range(depth + 1):
        fin = k0 if l == 0 else width
        fout = n_out if l == depth else width
        w_off = off
        off += fin * fout
        b_off = off
        off += fout
        off = (off + 63) // 64 * 64
        layers.append((w_off, b_off, fout, fin))
    return k0, layers, off


def pack_net_blob(n_in, width, depth, act, n_out, theta, feat_mean, feat_std, y_mean, y_std, box,
                  step=0, adam_m=None, adam_v=None):
    import numpy as np
    k0, _, P = net_layout(n_in, width, depth, n_out)
    theta = np.asarray(theta, dtype=np.float32)
    assert theta.size == P
    adam_m = np.zeros(P, np.float32) if adam_m is None else np.asarray(adam_m, np.float32)
    adam_v = np.zeros(P, np.float32) if adam_v is None else np.asarray(adam_v, np.float32)
    hdr = _struct.pack(_HDR, b"ELNET01\0", n_in, width, depth, act, k0, 0, n_out, step, P, *[float(b) for b in box])
    hdr = hdr + b"\0" * (HEADER_BYTES - len(hdr))
    parts = [np.asarray(a, dtype=np.float32).tobytes() for a in (feat_mean, feat_std, y_mean, y_std)]
    return hdr + b"".join(parts) + theta.tobytes() + adam_m.tobytes() + adam_v.tobytes()


def unpack_net_blob(blob):
    import numpy as np
    magic, n_in, width, depth, act, k0, _, n_out, step, P, *box = _struct.unpack_from(_HDR, blob, 0)
    if magic != b"ELNET01\0":
        raise ValueError("bad network blob")
    o = HEADER_BYTES
    def take(cnt):
        nonlocal o
        a = np.frombuffer(blob, dtype=np.float32, count=cnt, offset=o)
        o += 4 * cnt
        return a
    out = dict(n_in=n_in, width=width, depth=depth, act=act, k0=k0, n_out=n_out, step=step, n_params=P, box=box)
    out["feat_mean"], out["feat_std"] = take(n_in), take(n_in)
    out["y_mean"], out["y_std"] = take(n_out), take(n_out)
    out["theta"], out["adam_m"], out["adam_v"] = take(P), take(P), take(P)
    return out


def tuning_report():
    """The GEMM autotuner's choices so far (el_tuning_report), as text."""
    n = ctypes.c_size_t()
    lib().el_tuning_report(None, 0, ctypes.byref(n))
    buf = ctypes.create_string_buffer(max(n.value, 1))
    lib().el_tuning_report(buf, n.value, None)
    return buf.value.decode()


def tuning_save(path):
    """Write the autotuner's choices to a text file (el_tuning_save)."""
    if lib().el_tuning_save(os.fsencode(path)) != EL_OK:
        raise ElError(EL_ERR_ARG, f"el_tuning_save: cannot write {path}")


def tuning_load(path):
    """Take the autotuner's choices from a file written by tuning_save
    (el_tuning_load); returns the number of choices taken."""
    n = ctypes.c_int64()
    if lib().el_tuning_load(os.fsencode(path), ctypes.byref(n)) != EL_OK:
        raise ElError(EL_ERR_ARG, f"el_tuning_load: cannot read {path} as an autotuner file")
    return n.value


def tuning_reset():
    """Forget every autotuner choice of this process (el_tuning_reset)."""
    lib().el_tuning_reset()


def matvec_shape(shape):
    """Pin the skeleton product's row shape (el_matvec_shape); -1 restores
    the autotuner."""
    st = lib().el_matvec_shape(int(shape))
    if st != 0:
        raise ValueError(f"el_matvec_shape: bad shape {shape}")


def gemm_tile(variant):
    """Pin the block tile of the network GEMMs (el_gemm_tile); -1 restores the
    autotuner."""
    st = lib().el_gemm_tile(int(variant))
    if st != 0:
        raise ValueError(f"el_gemm_tile: bad variant {variant}")
