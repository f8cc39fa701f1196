"""Thin ctypes binding of libwbfbt.so (include/wbfbt.h); argument marshalling only.

Every numerical step runs in the HIP library.  Vector arguments are torch CUDA
(ROCm) tensors; streams default to torch's current stream.  The functions keep
the C names; Mesh / Viscosity / Solver own the opaque handles.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwbfbt.so")

WB_OK, WB_EINVAL, WB_ENOMEM, WB_EHIP, WB_ENOCONV, WB_ENAN, WB_EUNSUPPORTED = range(7)
WB_FP64, WB_FP32, WB_BF16, WB_BF16X1 = 0, 1, 2, 3


class WbError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"wbfbt status {code}: {msg}")
        self.code = code


class wb_opts(ctypes.Structure):
    _fields_ = [("a_l", ctypes.c_double), ("a_r", ctypes.c_double),
                ("cheb_degree", ctypes.c_int), ("lanczos_steps", ctypes.c_int),
                ("restart", ctypes.c_int), ("max_iter", ctypes.c_int),
                ("rtol", ctypes.c_double), ("precond_prec", ctypes.c_int),
                ("use_learned", ctypes.c_int), ("p_schedule", ctypes.c_int),
                ("verbose", ctypes.c_int), ("use_graph", ctypes.c_int),
                ("schur_sign", ctypes.c_int),
                ("assemble_mb", ctypes.c_double),
                ("schur_approx", ctypes.c_int),
                ("weights", ctypes.c_int)]


class wb_report(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("rel_res", ctypes.c_double),
                ("t_setup_s", ctypes.c_double), ("t_solve_s", ctypes.c_double),
                ("fell_back", ctypes.c_int), ("learned_used", ctypes.c_int),
                ("device_bytes", ctypes.c_size_t), ("learned_reduction", ctypes.c_double),
                ("history_ptr", ctypes.POINTER(ctypes.c_double)), ("history_len", ctypes.c_int)]

    @property
    def history(self):
        """Relative residual estimate after each iteration of the last solve (a copy)."""
        n = int(self.history_len)
        return [self.history_ptr[i] for i in range(n)] if n > 0 and self.history_ptr else []


class wb_train_opts(ctypes.Structure):
    _fields_ = [("pairs_per_field", ctypes.c_int), ("vcycles", ctypes.c_int),
                ("epochs", ctypes.c_int), ("batch", ctypes.c_int), ("lr", ctypes.c_double),
                ("seed", ctypes.c_ulonglong), ("delta", ctypes.c_double),
                ("omega", ctypes.c_double), ("mu_min", ctypes.c_double),
                ("mu_max", ctypes.c_double), ("n_valid", ctypes.c_int)]


class wb_train_report(ctypes.Structure):
    _fields_ = [("loss_first", ctypes.c_double), ("loss_last", ctypes.c_double),
                ("valid_loss", ctypes.c_double), ("t_pairs_s", ctypes.c_double),
                ("t_train_s", ctypes.c_double), ("n_params", ctypes.c_longlong),
                ("n_pairs", ctypes.c_int)]


_lib = None
VP, I, D, LL = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_longlong
PVP = ctypes.POINTER(ctypes.c_void_p)

# name -> (restype, argtypes) for every entry point of include/wbfbt.h
SIGNATURES = {
    "wb_opts_default": (None, [ctypes.POINTER(wb_opts)]),
    "wb_last_error": (ctypes.c_char_p, []),
    "wb_mesh_create": (I, [I, I, PVP]),
    "wb_mesh_destroy": (None, [VP]),
    "wb_mesh_sizes": (I, [VP, ctypes.POINTER(LL), ctypes.POINTER(LL), ctypes.POINTER(I)]),
    "wb_visc_create_sinker": (I, [VP, VP, I, D, D, D, D, VP, PVP]),
    "wb_visc_create_values": (I, [VP, VP, VP, VP, PVP]),
    "wb_visc_values": (I, [VP, VP, VP, VP]),
    "wb_visc_destroy": (None, [VP]),
    "wb_rhs_sinker": (I, [VP, VP, I, D, D, D, VP, VP]),
    "wb_apply_A": (I, [VP, VP, VP, VP, VP]),
    "wb_apply_A_noalloc": (I, [VP, VP, VP, VP, VP]),
    "wb_apply_B": (I, [VP, VP, VP, VP]),
    "wb_apply_B_lowp": (I, [VP, I, VP, VP, VP]),
    "wb_apply_BT_lowp": (I, [VP, I, VP, VP, VP]),
    "wb_apply_BT": (I, [VP, VP, VP, VP]),
    "wb_apply_A_add": (I, [VP, VP, VP, VP, VP]),
    "wb_apply_stokes": (I, [VP, VP, VP, VP, VP, VP, VP]),
    "wb_apply_A_lowp": (I, [VP, VP, I, VP, VP, VP]),
    "wb_solver_create": (I, [VP, VP, ctypes.POINTER(wb_opts), VP, PVP]),
    "wb_solver_destroy": (None, [VP]),
    "wb_apply_wbfbt": (I, [VP, VP, VP, VP]),
    "wb_apply_vcycle_A": (I, [VP, VP, VP, VP]),
    "wb_apply_K": (I, [VP, I, VP, VP, VP]),
    "wb_apply_vcycle_K": (I, [VP, I, VP, VP, VP]),
    "wb_apply_precond": (I, [VP, VP, VP, VP, VP, VP]),
    "wb_solve": (I, [VP, VP, VP, VP, ctypes.POINTER(wb_report), VP]),
    "wb_subsolve": (I, [VP, I, VP, VP, ctypes.POINTER(wb_report), VP]),
    "wb_solver_query": (I, [VP, I, I, VP, VP]),
    "wb_solver_levels": (I, [VP, I, ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(I),
                             ctypes.POINTER(D)]),
    "wb_train_opts_default": (None, [ctypes.POINTER(wb_train_opts)]),
    "wb_learned_train": (I, [VP, I, VP, VP, ctypes.POINTER(wb_train_opts),
                             ctypes.POINTER(wb_train_report), VP]),
    "wb_learned_get": (I, [VP, VP, ctypes.POINTER(LL)]),
    "wb_learned_set": (I, [VP, VP, LL]),
    "wb_learned_info": (I, [VP, ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(LL)]),
    "wb_learned_probe": (I, [VP, VP, VP, ctypes.POINTER(D), VP]),
    "wb_net_param_count": (LL, []),
    "wb_net_eval": (I, [I, I, VP, VP, VP, VP, VP, VP, ctypes.POINTER(D), VP]),
    "wb_net_adam": (I, [LL, VP, VP, VP, VP, I, D, VP]),
    "wb_net_feature": (I, [I, VP, VP, VP]),
    "wb_mem_trim": (None, []),
    "wb_profile_enable": (None, [I]),
    "wb_set_two_pass_limit": (D, [D]),
    "wb_set_matrix_core_ops": (I, [I]),
    "wb_profile_summary": (LL, [ctypes.c_char_p, LL, I]),
}


def lib():
    """Load libwbfbt.so; raises if the HIP library has not been built (no fallback)."""
    global _lib
    if _lib is None:
        # torch's bundled HIP runtime must be the one in the process: load it first so that the
        # library's libamdhip64.so.7 dependency resolves to it (one runtime, one device context)
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_1607_03936_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(code):
    if code != WB_OK:
        raise WbError(code, lib().wb_last_error().decode())
    return code


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t, dtype=None, numel=None):
    import torch
    if t is None:
        return None
    if not (t.is_cuda and t.is_contiguous()):
        raise ValueError("expected a contiguous device tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {t.dtype}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"expected {numel} elements, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


def opts(**kw) -> wb_opts:
    o = wb_opts()
    lib().wb_opts_default(ctypes.byref(o))
    names = {f[0] for f in wb_opts._fields_}
    for k, v in kw.items():
        if k not in names:
            raise TypeError(f"unknown solver option {k!r}")
        setattr(o, k, v)
    return o


class Mesh:
    def __init__(self, N: int, k: int):
        h = ctypes.c_void_p()
        _check(lib().wb_mesh_create(N, k, ctypes.byref(h)))
        self.h, self.N, self.k = h, N, k
        nn, ne, npm = LL(), LL(), I()
        _check(lib().wb_mesh_sizes(h, ctypes.byref(nn), ctypes.byref(ne), ctypes.byref(npm)))
        self.n_nodes, self.n_elem, self.n_p = nn.value, ne.value, npm.value
        self.u_len = 3 * self.n_nodes
        self.p_len = self.n_elem * self.n_p
        self.q_len = self.n_elem * (k + 1) ** 3

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.wb_mesh_destroy(self.h)
            self.h = None


class Viscosity:
    def __init__(self, mesh: Mesh, handle):
        self.mesh, self.h = mesh, handle

    @classmethod
    def sinker(cls, mesh, centers, delta, omega, mu_min, mu_max, stream=None):
        c = np.ascontiguousarray(np.asarray(centers, dtype=np.float64).reshape(-1, 3))
        h = ctypes.c_void_p()
        _check(lib().wb_visc_create_sinker(mesh.h, c.ctypes.data_as(VP), c.shape[0], delta, omega,
                                           mu_min, mu_max, _stream(stream), ctypes.byref(h)))
        return cls(mesh, h)

    @classmethod
    def values(cls, mesh, mu_q, mu_nodes, stream=None):
        import torch
        h = ctypes.c_void_p()
        _check(lib().wb_visc_create_values(mesh.h, _ptr(mu_q, torch.float64, mesh.q_len),
                                           _ptr(mu_nodes, torch.float64, mesh.n_nodes),
                                           _stream(stream), ctypes.byref(h)))
        return cls(mesh, h)

    def get(self, stream=None):
        import torch
        mq = torch.empty(self.mesh.q_len, dtype=torch.float64, device="cuda")
        mn = torch.empty(self.mesh.n_nodes, dtype=torch.float64, device="cuda")
        _check(lib().wb_visc_values(self.h, _ptr(mq), _ptr(mn), _stream(stream)))
        return mq, mn

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.wb_visc_destroy(self.h)
            self.h = None


def wb_rhs_sinker(mesh, centers, delta, omega, beta, f, stream=None):
    import torch
    c = np.ascontiguousarray(np.asarray(centers, dtype=np.float64).reshape(-1, 3))
    _check(lib().wb_rhs_sinker(mesh.h, c.ctypes.data_as(VP), c.shape[0], delta, omega, beta,
                               _ptr(f, torch.float64, mesh.u_len), _stream(stream)))


def wb_apply_A(mesh, visc, u, y, stream=None):
    import torch
    _check(lib().wb_apply_A(mesh.h, visc.h, _ptr(u, torch.float64, mesh.u_len),
                            _ptr(y, torch.float64, mesh.u_len), _stream(stream)))


def wb_apply_A_add(mesh, visc, u, y, stream=None):
    import torch
    _check(lib().wb_apply_A_add(mesh.h, visc.h, _ptr(u, torch.float64, mesh.u_len),
                                _ptr(y, torch.float64, mesh.u_len), _stream(stream)))


def wb_profile_enable(on: bool):
    lib().wb_profile_enable(1 if on else 0)


def wb_set_two_pass_limit(mb: float) -> float:
    return lib().wb_set_two_pass_limit(float(mb))


def wb_set_matrix_core_ops(on: bool) -> bool:
    return bool(lib().wb_set_matrix_core_ops(1 if on else 0))


def wb_profile_summary(reset: bool = True):
    """{kernel class: (launches, total ms)} of the event-timed operator launches."""
    n = lib().wb_profile_summary(None, 0, 0)
    buf = ctypes.create_string_buffer(int(n) + 1)
    lib().wb_profile_summary(buf, n + 1, 1 if reset else 0)
    out = {}
    for line in buf.value.decode().splitlines():
        key, cnt, ms = line.split("\t")
        out[key] = (int(cnt), float(ms))
    return out


def wb_apply_A_lowp(mesh, visc, prec, u, y, stream=None):
    import torch
    _check(lib().wb_apply_A_lowp(mesh.h, visc.h, prec, _ptr(u, torch.float32, mesh.u_len),
                                 _ptr(y, torch.float32, mesh.u_len), _stream(stream)))


def wb_apply_A_noalloc(mesh, visc, u, y, stream=None):
    import torch
    _check(lib().wb_apply_A_noalloc(mesh.h, visc.h, _ptr(u, torch.float64, mesh.u_len),
                                    _ptr(y, torch.float64, mesh.u_len), _stream(stream)))


def wb_apply_B(mesh, u, p, stream=None):
    import torch
    _check(lib().wb_apply_B(mesh.h, _ptr(u, torch.float64, mesh.u_len),
                            _ptr(p, torch.float64, mesh.p_len), _stream(stream)))


def wb_apply_B_lowp(mesh, prec, u, p, stream=None):
    import torch
    _check(lib().wb_apply_B_lowp(mesh.h, prec, _ptr(u, torch.float32, mesh.u_len),
                                 _ptr(p, torch.float32, mesh.p_len), _stream(stream)))


def wb_apply_BT_lowp(mesh, prec, p, u, stream=None):
    import torch
    _check(lib().wb_apply_BT_lowp(mesh.h, prec, _ptr(p, torch.float32, mesh.p_len),
                                  _ptr(u, torch.float32, mesh.u_len), _stream(stream)))


def wb_apply_BT(mesh, p, u, stream=None):
    import torch
    _check(lib().wb_apply_BT(mesh.h, _ptr(p, torch.float64, mesh.p_len),
                             _ptr(u, torch.float64, mesh.u_len), _stream(stream)))


def wb_apply_stokes(mesh, visc, u, p, yu, yp, stream=None):
    import torch
    f64 = torch.float64
    _check(lib().wb_apply_stokes(mesh.h, visc.h, _ptr(u, f64, mesh.u_len), _ptr(p, f64, mesh.p_len),
                                 _ptr(yu, f64, mesh.u_len), _ptr(yp, f64, mesh.p_len),
                                 _stream(stream)))


class Solver:
    def __init__(self, mesh: Mesh, visc: Viscosity, stream=None, **kw):
        self.mesh, self.visc = mesh, visc
        self.opts = opts(**kw)
        h = ctypes.c_void_p()
        _check(lib().wb_solver_create(mesh.h, visc.h, ctypes.byref(self.opts), _stream(stream),
                                      ctypes.byref(h)))
        self.h = h

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.wb_solver_destroy(self.h)
            self.h = None

    def wbfbt(self, r, z, stream=None):
        import torch
        m = self.mesh
        _check(lib().wb_apply_wbfbt(self.h, _ptr(r, torch.float64, m.p_len),
                                    _ptr(z, torch.float64, m.p_len), _stream(stream)))

    def vcycle_A(self, r, z, stream=None):
        import torch
        m = self.mesh
        _check(lib().wb_apply_vcycle_A(self.h, _ptr(r, torch.float64, m.u_len),
                                       _ptr(z, torch.float64, m.u_len), _stream(stream)))

    def apply_K(self, side, p, y, stream=None):
        import torch
        m = self.mesh
        _check(lib().wb_apply_K(self.h, side, _ptr(p, torch.float64, m.p_len),
                                _ptr(y, torch.float64, m.p_len), _stream(stream)))

    def vcycle_K(self, side, r, z, stream=None):
        import torch
        m = self.mesh
        _check(lib().wb_apply_vcycle_K(self.h, side, _ptr(r, torch.float64, m.p_len),
                                       _ptr(z, torch.float64, m.p_len), _stream(stream)))

    def precond(self, ru, rp, zu, zp, stream=None):
        import torch
        m, f64 = self.mesh, torch.float64
        _check(lib().wb_apply_precond(self.h, _ptr(ru, f64, m.u_len), _ptr(rp, f64, m.p_len),
                                      _ptr(zu, f64, m.u_len), _ptr(zp, f64, m.p_len),
                                      _stream(stream)))

    def solve(self, f, u, p, stream=None, allow_noconv=False):
        import torch
        m, f64 = self.mesh, torch.float64
        rep = wb_report()
        code = lib().wb_solve(self.h, _ptr(f, f64, m.u_len), _ptr(u, f64, m.u_len),
                              _ptr(p, f64, m.p_len), ctypes.byref(rep), _stream(stream))
        if not (allow_noconv and code == WB_ENOCONV):
            _check(code)
        return rep

    def subsolve(self, which, b, x, stream=None, allow_noconv=False):
        """GMRES on A (which=0) or K_l / K_r (1 / 2) with one V-cycle as preconditioner."""
        import torch
        rep = wb_report()
        code = lib().wb_subsolve(self.h, which, _ptr(b, torch.float64), _ptr(x, torch.float64),
                                 ctypes.byref(rep), _stream(stream))
        if not (allow_noconv and code == WB_ENOCONV):
            _check(code)
        return rep

    def query(self, what, level=0, size=None, stream=None):
        import torch
        out = torch.empty(size, dtype=torch.float64, device="cuda")
        _check(lib().wb_solver_query(self.h, what, level, _ptr(out), _stream(stream)))
        return out

    def levels(self, which):
        nl = I()
        Ns = (I * 16)()
        ks = (I * 16)()
        lm = (D * 16)()
        _check(lib().wb_solver_levels(self.h, which, ctypes.byref(nl), Ns, ks, lm))
        return [(Ns[i], ks[i], lm[i]) for i in range(nl.value)]

    # ---- learned coarse correction
    def learned_info(self):
        lv, M, n = I(), I(), LL()
        _check(lib().wb_learned_info(self.h, ctypes.byref(lv), ctypes.byref(M), ctypes.byref(n)))
        return lv.value, M.value, n.value

    def learned_train(self, centers_per_field, stream=None, **kw):
        """centers_per_field: list of [n_i][3] arrays (one per seeded field)."""
        o = wb_train_opts()
        lib().wb_train_opts_default(ctypes.byref(o))
        for k, v in kw.items():
            setattr(o, k, v)
        ns = np.array([len(c) for c in centers_per_field], dtype=np.int32)
        flat = (np.ascontiguousarray(np.concatenate([np.asarray(c, np.float64).reshape(-1, 3)
                                                     for c in centers_per_field]))
                if ns.sum() > 0 else np.zeros((1, 3)))
        rep = wb_train_report()
        _check(lib().wb_learned_train(self.h, len(ns), ns.ctypes.data_as(VP),
                                      flat.ctypes.data_as(VP), ctypes.byref(o), ctypes.byref(rep),
                                      _stream(stream)))
        return rep

    def learned_get(self):
        n = LL()
        _check(lib().wb_learned_get(self.h, None, ctypes.byref(n)))
        out = np.empty(n.value, dtype=np.float32)
        _check(lib().wb_learned_get(self.h, out.ctypes.data_as(VP), ctypes.byref(n)))
        return out

    def learned_set(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        _check(lib().wb_learned_set(self.h, p.ctypes.data_as(VP), p.size))

    def learned_probe(self, r, delta, stream=None):
        import torch
        a = D()
        _check(lib().wb_learned_probe(self.h, _ptr(r, torch.float64), _ptr(delta, torch.float64),
                                      ctypes.byref(a), _stream(stream)))
        return a.value


def wb_net_eval(M, B, params, x, out, t=None, w=None, grad=None, stream=None):
    """Network forward (and loss + gradient when t, w, grad are given); returns the loss."""
    import torch
    f32 = torch.float32
    loss = D()
    _check(lib().wb_net_eval(M, B, _ptr(params, f32), _ptr(x, f32), _ptr(t, f32), _ptr(w, f32),
                             _ptr(out, f32), _ptr(grad, f32), ctypes.byref(loss), _stream(stream)))
    return loss.value


def wb_net_adam(params, grad, m, v, step, lr, stream=None):
    import torch
    f32 = torch.float32
    _check(lib().wb_net_adam(params.numel(), _ptr(params, f32), _ptr(grad, f32), _ptr(m, f32),
                             _ptr(v, f32), step, lr, _stream(stream)))


def wb_net_feature(N, coef, feat, stream=None):
    import torch
    _check(lib().wb_net_feature(N, _ptr(coef, torch.float64), _ptr(feat, torch.float32),
                                _stream(stream)))
