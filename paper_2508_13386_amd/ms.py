"""ctypes binding of libms (the C ABI declared in include/ms.h).

Argument marshalling only: every computation runs in the HIP library.  The
functions keep the C names.  Device memory comes from PyTorch's caching
allocator through the ms_device callbacks, and work runs on a dedicated
torch.cuda.Stream.  Loading fails loudly when the library is not built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libms.so")

MS_OK, MS_E_ARG, MS_E_MESH, MS_E_ORDER, MS_E_DEVICE, MS_E_NOMEM, MS_E_NOCONV, MS_E_LINESEARCH, MS_E_NONFINITE = \
    0, -1, -2, -3, -4, -5, -6, -7, -8
PREC_FP64, PREC_MIXED = 0, 1
PC_BLOCK_JACOBI, PC_TWO_LEVEL, PC_TWO_LEVEL_ADDITIVE, PC_TWO_LEVEL_VCYCLE = 0, 1, 2, 3
MODE_PLAIN, MODE_PAPER = 0, 1
COARSE_EXACT, COARSE_CUBATURE = 0, 1

_ALLOC = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
_FREE = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class ms_device(C.Structure):
    _fields_ = [("device", C.c_int), ("hip_stream", C.c_void_p), ("alloc", _ALLOC), ("free", _FREE),
                ("user", C.c_void_p)]


class ms_solver_params(C.Structure):
    _fields_ = [("mode", C.c_int32), ("precision", C.c_int32), ("preconditioner", C.c_int32),
                ("max_newton", C.c_int32), ("max_pcg", C.c_int32), ("newton_tol", C.c_double),
                ("abs_floor", C.c_double), ("pcg_eta_max", C.c_double), ("pcg_eta_min", C.c_double),
                ("max_backtracks", C.c_int32), ("exact_endgame", C.c_int32),
                ("warm_start", C.c_int32), ("paper_eps", C.c_double), ("subspace_rtol", C.c_double),
                ("refine_iters", C.c_int32), ("lag_window", C.c_int32), ("lag_threshold", C.c_double),
                ("lag_min_gap", C.c_int32), ("forcing", C.c_int32), ("endgame_ratio", C.c_double),
                ("coarse_every", C.c_int32), ("predictor", C.c_int32), ("time_kernels", C.c_int32),
                ("coarse_move", C.c_double), ("mixed_max_newton", C.c_int32),
                ("mixed_endgame_fp64", C.c_int32), ("integrator", C.c_int32), ("projection", C.c_int32),
                ("smoother", C.c_int32)]


class ms_step_stats(C.Structure):
    _fields_ = [("newton_iters", C.c_int32), ("pcg_iters", C.c_int32), ("max_pcg_iters", C.c_int32),
                ("backtracks", C.c_int32), ("hessian_refreshes", C.c_int32), ("warm_start_used", C.c_int32),
                ("precision_escalations", C.c_int32), ("pcg_iters_fp64", C.c_int32),
                ("pcg_solves_fp64", C.c_int32), ("energy", C.c_double), ("last_dnorm", C.c_double), ("disp_norm", C.c_double),
                ("min_alpha", C.c_double), ("time_ms", C.c_double), ("subspace_pcg_iters", C.c_int32),
                ("refine_iters", C.c_int32), ("pcg_ms", C.c_double)]

    def asdict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ms_basis_params(C.Structure):
    _fields_ = [("n_handles", C.c_int32), ("oversample", C.c_double), ("jump_penalty", C.c_double),
                ("prune_ratio", C.c_double), ("prune_every", C.c_int32), ("prune_n", C.c_int32),
                ("max_lloyd", C.c_int32), ("lattice_seeding", C.c_int32), ("seed", C.c_uint64),
                ("n_threads", C.c_int32), ("gpu_min_unknowns", C.c_int32), ("rigid_contrast", C.c_double)]


_FP = C.POINTER(C.c_float)


class ms_mlp_desc(C.Structure):
    _fields_ = [("in_dim", C.c_int32), ("width", C.c_int32), ("out_dim", C.c_int32),
                ("W0", _FP), ("b0", _FP), ("W1", _FP), ("b1", _FP), ("W2", _FP), ("b2", _FP),
                ("in_mean", _FP), ("in_std", _FP), ("out_scale", _FP)]


_lib = None


def lib():
    """Load libms.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2508_13386_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, d, dp, ip = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_void_p, C.c_void_p
        sig = {
            "ms_create": [C.POINTER(ms_device), C.POINTER(C.c_void_p)],
            "ms_upload_mesh": [vp, i64, dp, i64, ip],
            "ms_upload_material": [vp, dp, dp, dp],
            "ms_set_gravity": [vp, dp],
            "ms_set_dirichlet": [vp, i64, ip, dp],
            "ms_add_halfspace": [vp, dp, d, d, d],
            "ms_set_friction": [vp, d, d],
            "ms_set_self_contact": [vp, d, d, i32],
            "ms_set_state": [vp, dp, dp],
            "ms_get_state": [vp, dp, dp],
            "ms_build_basis": [vp, C.POINTER(ms_basis_params)],
            "ms_get_basis_stats": [vp, C.POINTER(i32), C.POINTER(d)],
            "ms_set_basis": [vp, i32, dp, ip, ip, dp],
            "ms_get_basis_size": [vp, C.POINTER(i32), C.POINTER(i64)],
            "ms_get_basis": [vp, dp, ip, ip, dp, ip],
            "ms_step": [vp, d, C.POINTER(ms_solver_params), C.POINTER(ms_step_stats)],
            "ms_get_coarse": [vp, dp],
            "ms_set_warmstart": [vp, C.POINTER(ms_mlp_desc)],
            "ms_get_pattern": [vp, C.POINTER(i64), ip, ip],
            "ms_eval": [vp, dp, d, i32, dp, dp, dp],
            "ms_apply_preconditioner": [vp, i32, i32, dp, dp],
            "ms_get_coarse_matrix": [vp, dp],
            "ms_mat_create": [C.POINTER(ms_device), i64, ip, ip, dp, i32, C.POINTER(C.c_void_p)],
            "ms_mat_spmv": [vp, vp, vp],
            "ms_batch_step": [C.POINTER(C.c_void_p), i32, d, C.POINTER(ms_solver_params), C.POINTER(ms_step_stats)],
            "ms_batch_create": [C.POINTER(C.c_void_p), i32, C.POINTER(C.c_void_p)],
            "ms_batch_advance": [vp, d, C.POINTER(ms_solver_params), C.POINTER(ms_step_stats)],
            "ms_time_kernel": [vp, i32, i32, i32, C.POINTER(d), C.POINTER(d)],
            "ms_energy_difference": [vp, dp, dp, d, d, dp],
            "ms_basis_compute": [i64, dp, i64, ip, dp, i64, ip, C.POINTER(ms_basis_params), C.POINTER(C.c_void_p)],
            "ms_basis_get": [vp, C.POINTER(i32), C.POINTER(i64), dp, ip, ip, dp, ip],
            "ms_aggregates_compute": [i64, dp, ip, ip, i64, ip, C.POINTER(i64)],
            "ms_cubature_compute": [i64, dp, i64, ip, ip, i32, ip, ip, dp, d, i32, i32, i32, C.c_uint64, i32,
                                    C.POINTER(C.c_void_p)],
            "ms_cubature_get": [vp, C.POINTER(i64), ip, dp, C.POINTER(d)],
            "ms_build_cubature": [vp, d, i32, i32, i32, C.c_uint64, C.POINTER(d)],
            "ms_set_cubature": [vp, i64, ip, dp],
            "ms_get_cubature": [vp, C.POINTER(i64), ip, dp],
            "ms_set_coarse_integration": [vp, i32],
            "ms_contact_toi": [C.POINTER(ms_device), i64, ip, dp, dp, d, d, i32, dp, ip],
            "ms_contact_pairs": [C.POINTER(ms_device), i64, dp, i64, ip, i64, ip, i64, ip, d, d,
                                 C.POINTER(C.c_void_p)],
            "ms_pairs_get": [vp, C.POINTER(i64), ip, C.POINTER(i64), ip],
            "ms_mlp_forward": [C.POINTER(ms_device), i32, i32, i32, vp, i64, vp, vp],
            "ms_mlp_forward_noalloc": [C.POINTER(ms_device), i32, i32, i32, vp, i64, vp, vp],
            "ms_mlp_train": [C.POINTER(ms_device), i32, i32, i32, vp, i64, vp, vp, i32, i32, vp, C.c_float, vp, vp],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.ms_mat_bytes.argtypes = [vp]
        L.ms_mat_bytes.restype = C.c_double
        L.ms_mat_destroy.argtypes = [vp]
        L.ms_mat_destroy.restype = None
        L.ms_batch_destroy.argtypes = [vp]
        L.ms_batch_destroy.restype = None
        L.ms_basis_free.argtypes = [vp]
        L.ms_basis_free.restype = None
        L.ms_cubature_free.argtypes = [vp]
        L.ms_cubature_free.restype = None
        L.ms_pairs_free.argtypes = [vp]
        L.ms_pairs_free.restype = None
        L.ms_destroy.argtypes = [vp]
        L.ms_destroy.restype = None
        L.ms_last_error.argtypes = [vp]
        L.ms_last_error.restype = C.c_char_p
        for f in ("ms_solver_defaults",):
            getattr(L, f).argtypes = [C.POINTER(ms_solver_params)]
            getattr(L, f).restype = None
        L.ms_basis_defaults.argtypes = [C.POINTER(ms_basis_params)]
        L.ms_basis_defaults.restype = None
        _lib = L
    return _lib


class MSError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ms status {code}: {msg}")
        self.code = code


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def solver_defaults(**kw) -> ms_solver_params:
    p = ms_solver_params()
    lib().ms_solver_defaults(C.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise AttributeError(k)
        setattr(p, k, v)
    return p


def basis_defaults(**kw) -> ms_basis_params:
    p = ms_basis_params()
    lib().ms_basis_defaults(C.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise AttributeError(k)
        setattr(p, k, v)
    return p


class TorchDevice:
    """ms_device backed by torch's caching allocator and a torch stream."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.torch = torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible to torch")
        self.index = device
        self.stream = stream if stream is not None else torch.cuda.Stream(device=device)
        self._live = {}

        def _alloc(nbytes, user):
            t = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=f"cuda:{device}")
            p = t.data_ptr()
            self._live[p] = t
            return p

        def _free(p, user):
            self._live.pop(p, None)

        self._alloc_cb = _ALLOC(_alloc)
        self._free_cb = _FREE(_free)
        self.desc = ms_device(device, C.c_void_p(self.stream.cuda_stream), self._alloc_cb, self._free_cb, None)


class Context:
    """One simulation context (ms_ctx) with Python-friendly argument marshalling."""

    def __init__(self, dev: TorchDevice):
        self.dev = dev
        self.L = lib()
        h = C.c_void_p()
        self._check(self.L.ms_create(C.byref(dev.desc), C.byref(h)), ctx=None)
        self.h = h
        self.n = 0
        self.T = 0

    def _check(self, code, ctx="self"):
        if code != MS_OK:
            msg = ""
            if ctx is not None and getattr(self, "h", None):
                msg = (self.L.ms_last_error(self.h) or b"").decode()
            raise MSError(code, msg)

    def close(self):
        if getattr(self, "h", None):
            self.L.ms_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- uploads --------------------------------------------------------------
    def ms_upload_mesh(self, rest, tets):
        rest, tets = _f64(rest), _i32(tets)
        self.n, self.T = len(rest), len(tets)
        self._check(self.L.ms_upload_mesh(self.h, self.n, _ptr(rest), self.T, _ptr(tets)))

    def ms_upload_material(self, E, nu, rho):
        E, nu, rho = _f64(E), _f64(nu), _f64(rho)
        self._check(self.L.ms_upload_material(self.h, _ptr(E), _ptr(nu), _ptr(rho)))

    def ms_set_gravity(self, g):
        g = _f64(g)
        self._check(self.L.ms_set_gravity(self.h, _ptr(g)))

    def ms_set_dirichlet(self, verts, targets):
        verts, targets = _i32(verts), _f64(targets).reshape(-1, 3)
        self._check(self.L.ms_set_dirichlet(self.h, len(verts), _ptr(verts), _ptr(targets)))

    def ms_add_halfspace(self, normal, offset, dhat, kappa):
        nrm = _f64(normal)
        self._check(self.L.ms_add_halfspace(self.h, _ptr(nrm), float(offset), float(dhat), float(kappa)))

    def ms_set_friction(self, mu, eps_v=1e-3):
        self._check(self.L.ms_set_friction(self.h, float(mu), float(eps_v)))

    def ms_set_self_contact(self, dhat, kappa, slots=32):
        self._check(self.L.ms_set_self_contact(self.h, float(dhat), float(kappa), int(slots)))

    def ms_set_state(self, x, v):
        x, v = _f64(x), _f64(v)
        self._check(self.L.ms_set_state(self.h, _ptr(x), _ptr(v)))

    def ms_get_state(self):
        x = np.empty((self.n, 3))
        v = np.empty((self.n, 3))
        self._check(self.L.ms_get_state(self.h, _ptr(x), _ptr(v)))
        return x, v

    # -- basis ----------------------------------------------------------------
    def ms_build_basis(self, params=None, **kw):
        p = params or basis_defaults(**kw)
        self._check(self.L.ms_build_basis(self.h, C.byref(p)))

    def ms_set_basis(self, origins, vptr, vhandle, vphi):
        o, vp, vh, w = _f64(origins), np.ascontiguousarray(vptr, dtype=np.int64), _i32(vhandle), _f64(vphi)
        self._check(self.L.ms_set_basis(self.h, len(o), _ptr(o), _ptr(vp), _ptr(vh), _ptr(w)))

    def ms_get_basis_stats(self):
        """(local solves of the last ms_build_basis that ran on the GPU, its seconds)."""
        g, t = C.c_int32(), C.c_double()
        self._check(self.L.ms_get_basis_stats(self.h, C.byref(g), C.byref(t)))
        return g.value, t.value

    def ms_get_basis(self):
        m = C.c_int32()
        nnz = C.c_int64()
        self._check(self.L.ms_get_basis_size(self.h, C.byref(m), C.byref(nnz)))
        o = np.empty((m.value, 3))
        vp = np.empty(self.n + 1, dtype=np.int64)
        vh = np.empty(nnz.value, dtype=np.int32)
        w = np.empty(nnz.value)
        part = np.empty(self.T, dtype=np.int32)
        self._check(self.L.ms_get_basis(self.h, _ptr(o), _ptr(vp), _ptr(vh), _ptr(w), _ptr(part)))
        return dict(origins=o, vptr=vp, vhandle=vh, vphi=w, part=part, m=m.value)

    # -- cubature of the coarse matrix (Sec. 3.8) --------------------------------
    def ms_build_cubature(self, tol=1e-9, n_init=16, n_add=16, max_rounds=64, seed=0):
        res = C.c_double()
        self._check(self.L.ms_build_cubature(self.h, float(tol), int(n_init), int(n_add), int(max_rounds),
                                             int(seed), C.byref(res)))
        return res.value

    def ms_set_cubature(self, tets, weights):
        t, w = _i32(tets), _f64(weights)
        self._check(self.L.ms_set_cubature(self.h, len(t), _ptr(t) if len(t) else None, _ptr(w) if len(w) else None))

    def ms_get_cubature(self):
        n = C.c_int64()
        self._check(self.L.ms_get_cubature(self.h, C.byref(n), None, None))
        t = np.empty(n.value, dtype=np.int32)
        w = np.empty(n.value)
        self._check(self.L.ms_get_cubature(self.h, C.byref(n), _ptr(t), _ptr(w)))
        return t, w

    def ms_set_coarse_integration(self, mode):
        self._check(self.L.ms_set_coarse_integration(self.h, int(mode)))

    # -- stepping ---------------------------------------------------------------
    def ms_step(self, dt, params=None, **kw):
        p = params or solver_defaults(**kw)
        st = ms_step_stats()
        self._check(self.L.ms_step(self.h, float(dt), C.byref(p), C.byref(st)))
        return st.asdict()

    def ms_get_coarse(self, r):
        q = np.empty(r)
        self._check(self.L.ms_get_coarse(self.h, _ptr(q)))
        return q

    def ms_set_warmstart(self, params=None, in_mean=None, in_std=None, out_scale=None):
        """Install the warm-start network (dict W0 b0 W1 b1 W2 b2, float32
        row-major [out][in]) with its input standardisation and output scale;
        params None removes it."""
        if params is None:
            self._check(self.L.ms_set_warmstart(self.h, None))
            return
        keep = {k: np.ascontiguousarray(params[k], dtype=np.float32) for k in MLP_KEYS}
        keep["m"] = np.ascontiguousarray(in_mean, dtype=np.float32)
        keep["s"] = np.ascontiguousarray(in_std, dtype=np.float32)
        keep["o"] = np.ascontiguousarray(out_scale, dtype=np.float32)
        fp = lambda a: a.ctypes.data_as(_FP)
        w, i = keep["W0"].shape
        o = keep["W2"].shape[0]
        desc = ms_mlp_desc(i, w, o, fp(keep["W0"]), fp(keep["b0"]), fp(keep["W1"]), fp(keep["b1"]),
                           fp(keep["W2"]), fp(keep["b2"]), fp(keep["m"]), fp(keep["s"]), fp(keep["o"]))
        self._check(self.L.ms_set_warmstart(self.h, C.byref(desc)))

    # -- kernel-level queries ---------------------------------------------------
    def ms_get_pattern(self):
        nnzb = C.c_int64()
        self._check(self.L.ms_get_pattern(self.h, C.byref(nnzb), None, None))
        rp = np.empty(self.n + 1, dtype=np.int32)
        col = np.empty(nnzb.value, dtype=np.int32)
        self._check(self.L.ms_get_pattern(self.h, C.byref(nnzb), _ptr(rp), _ptr(col)))
        return rp, col

    def ms_eval(self, x, dt, prec=PREC_FP64, hess=True):
        x = _f64(x)
        e4 = np.empty(4)
        g = np.empty((self.n, 3))
        H = None
        if hess:
            nnzb = C.c_int64()
            self._check(self.L.ms_get_pattern(self.h, C.byref(nnzb), None, None))
            H = np.empty((nnzb.value, 3, 3))
        self._check(self.L.ms_eval(self.h, _ptr(x), float(dt), int(prec), _ptr(e4), _ptr(g), _ptr(H)))
        return e4, g, H

    def ms_energy_difference(self, x, d, alpha, dt):
        """{dK, h^2 dPsi, h^2 dG, h^2 dB, magnitude} of E(x + alpha d) - E(x)."""
        x, d = _f64(x), _f64(d)
        out = np.empty(5)
        self._check(self.L.ms_energy_difference(self.h, _ptr(x), _ptr(d), float(alpha), float(dt), _ptr(out)))
        return out

    def ms_apply_preconditioner(self, kind, r, prec=PREC_FP64):
        r = _f64(r)
        z = np.empty((self.n, 3))
        self._check(self.L.ms_apply_preconditioner(self.h, int(kind), int(prec), _ptr(r), _ptr(z)))
        return z

    def ms_time_kernel(self, kernel=0, prec=PREC_FP64, reps=100):
        us = C.c_double()
        nb = C.c_double()
        self._check(self.L.ms_time_kernel(self.h, int(kernel), int(prec), int(reps), C.byref(us), C.byref(nb)))
        return us.value, nb.value

    def ms_get_coarse_matrix(self, r):
        A = np.empty((r, r))
        self._check(self.L.ms_get_coarse_matrix(self.h, _ptr(A)))
        return A


def ms_aggregates_compute(rest, row_ptr, col):
    """Host-only vertex aggregates of the aggregate smoother: int32 [nagg][8]
    (vertex ids, -1 padding)."""
    L = lib()
    rest, row_ptr, col = _f64(rest), _i32(row_ptr), _i32(col)
    n = C.c_int64()
    code = L.ms_aggregates_compute(len(rest), _ptr(rest), _ptr(row_ptr), _ptr(col), 0, None, C.byref(n))
    if code != MS_OK:
        raise MSError(code, "ms_aggregates_compute")
    out = np.empty((n.value, 8), dtype=np.int32)
    code = L.ms_aggregates_compute(len(rest), _ptr(rest), _ptr(row_ptr), _ptr(col), out.size, _ptr(out), C.byref(n))
    if code != MS_OK:
        raise MSError(code, "ms_aggregates_compute")
    return out


def ms_basis_compute(rest, tets, E, dbc=(), params=None, **kw):
    """Host-only basis construction; returns the dict of ms_basis_get."""
    L = lib()
    rest, tets, E = _f64(rest), _i32(tets), _f64(E)
    dbc = _i32(np.asarray(dbc, dtype=np.int32))
    p = params or basis_defaults(**kw)
    h = C.c_void_p()
    code = L.ms_basis_compute(len(rest), _ptr(rest), len(tets), _ptr(tets), _ptr(E), len(dbc),
                              _ptr(dbc) if len(dbc) else None, C.byref(p), C.byref(h))
    if code != MS_OK:
        raise MSError(code, "ms_basis_compute")
    try:
        m = C.c_int32()
        nnz = C.c_int64()
        L.ms_basis_get(h, C.byref(m), C.byref(nnz), None, None, None, None, None)
        o = np.empty((m.value, 3))
        vp = np.empty(len(rest) + 1, dtype=np.int64)
        vh = np.empty(nnz.value, dtype=np.int32)
        w = np.empty(nnz.value)
        part = np.empty(len(tets), dtype=np.int32)
        L.ms_basis_get(h, C.byref(m), C.byref(nnz), _ptr(o), _ptr(vp), _ptr(vh), _ptr(w), _ptr(part))
    finally:
        L.ms_basis_free(h)
    return dict(origins=o, vptr=vp, vhandle=vh, vphi=w, part=part, m=m.value)


def ms_cubature_compute(rest, tets, part, basis, tol=1e-9, n_init=16, n_add=16, max_rounds=64, seed=0,
                        n_threads=0):
    """Host-only cubature fit (Alg. 3); basis = dict(m, vptr, vhandle, vphi).
    Returns (tets ascending, weights, largest relative moment residual)."""
    L = lib()
    rest, tets, part = _f64(rest), _i32(tets), _i32(part)
    vp = np.ascontiguousarray(basis["vptr"], dtype=np.int64)
    vh, w = _i32(basis["vhandle"]), _f64(basis["vphi"])
    h = C.c_void_p()
    code = L.ms_cubature_compute(len(rest), _ptr(rest), len(tets), _ptr(tets), _ptr(part), int(basis["m"]),
                                 _ptr(vp), _ptr(vh), _ptr(w), float(tol), int(n_init), int(n_add),
                                 int(max_rounds), int(seed), int(n_threads), C.byref(h))
    if code != MS_OK:
        raise MSError(code, "ms_cubature_compute")
    try:
        n = C.c_int64()
        res = C.c_double()
        L.ms_cubature_get(h, C.byref(n), None, None, None)
        t = np.empty(n.value, dtype=np.int32)
        wt = np.empty(n.value)
        L.ms_cubature_get(h, C.byref(n), _ptr(t), _ptr(wt), C.byref(res))
    finally:
        L.ms_cubature_free(h)
    return t, wt, res.value


def ms_contact_toi(dev, kind, x12, p12, s=0.1, t_max=1.0, max_iter=100000):
    """Additive CCD of point-triangle (kind 0) / edge-edge (kind 1) pairs on
    the GPU; returns (hit [n] bool, toi [n])."""
    L = lib()
    kind = _i32(kind)
    x12, p12 = _f64(np.asarray(x12).reshape(-1, 12)), _f64(np.asarray(p12).reshape(-1, 12))
    n = len(kind)
    toi = np.empty(n)
    hit = np.empty(n, dtype=np.int32)
    code = L.ms_contact_toi(C.byref(dev.desc), n, _ptr(kind), _ptr(x12), _ptr(p12), float(s), float(t_max), int(max_iter),
                            _ptr(toi), _ptr(hit))
    if code != MS_OK:
        raise MSError(code, "ms_contact_toi")
    return hit.astype(bool), toi


def ms_contact_pairs(dev, x, sverts, tris, edges, dhat, cell=0.0):
    """Self-contact constraint set on the GPU: (pt [k,2] of (vertex, triangle
    index), ee [k,2] of (edge index, edge index), i < j), both ascending."""
    L = lib()
    x = _f64(np.asarray(x).reshape(-1, 3))
    sv, tr, ed = _i32(sverts), _i32(np.asarray(tris).reshape(-1, 3)), _i32(np.asarray(edges).reshape(-1, 2))
    h = C.c_void_p()
    code = L.ms_contact_pairs(C.byref(dev.desc), len(x), _ptr(x), len(sv), _ptr(sv) if len(sv) else None, len(tr),
                              _ptr(tr) if len(tr) else None, len(ed), _ptr(ed) if len(ed) else None, float(dhat),
                              float(cell), C.byref(h))
    if code != MS_OK:
        raise MSError(code, "ms_contact_pairs")
    try:
        npt, nee = C.c_int64(), C.c_int64()
        L.ms_pairs_get(h, C.byref(npt), None, C.byref(nee), None)
        pt = np.empty((npt.value, 2), dtype=np.int32)
        ee = np.empty((nee.value, 2), dtype=np.int32)
        L.ms_pairs_get(h, C.byref(npt), _ptr(pt), C.byref(nee), _ptr(ee))
    finally:
        L.ms_pairs_free(h)
    return pt, ee


MLP_KEYS = ("W0", "b0", "W1", "b1", "W2", "b2")


def mlp_pack(p):
    return np.concatenate([np.asarray(p[k], dtype=np.float32).ravel() for k in MLP_KEYS])


def mlp_unpack(flat, in_dim, width, out_dim):
    shapes = {"W0": (width, in_dim), "b0": (width,), "W1": (width, width), "b1": (width,),
              "W2": (out_dim, width), "b2": (out_dim,)}
    out, k = {}, 0
    for name in MLP_KEYS:
        size = int(np.prod(shapes[name]))
        out[name] = np.asarray(flat[k:k + size], dtype=np.float32).reshape(shapes[name]).copy()
        k += size
    return out


def _mlp_dims(p):
    w, i = np.asarray(p["W0"]).shape
    return i, w, np.asarray(p["W2"]).shape[0]


def ms_mlp_forward(dev, params, Z):
    """Network outputs for Z [n][in] (standardised inputs) on the GPU."""
    L = lib()
    i, w, o = _mlp_dims(params)
    flat = mlp_pack(params)
    Z = np.ascontiguousarray(Z, dtype=np.float32)
    Y = np.empty((len(Z), o), dtype=np.float32)
    code = L.ms_mlp_forward(C.byref(dev.desc), i, w, o, _ptr(flat), len(Z), _ptr(Z), _ptr(Y))
    if code != MS_OK:
        raise MSError(code, "ms_mlp_forward")
    return Y


MLP_NOALLOC_SCRATCH_FLOATS = 1 << 20


def ms_mlp_forward_noalloc(dev, dims, params_dev, Z_dev, Y_dev):
    """The forward pass on device tensors (torch, float32, contiguous) with
    no allocation by the library; dims = (in, width, out).  Asynchronous on
    dev's stream."""
    i, w, o = dims
    n = Z_dev.shape[0]
    code = lib().ms_mlp_forward_noalloc(C.byref(dev.desc), i, w, o, C.c_void_p(params_dev.data_ptr()), n,
                                        C.c_void_p(Z_dev.data_ptr()), C.c_void_p(Y_dev.data_ptr()))
    if code != MS_OK:
        raise MSError(code, "ms_mlp_forward_noalloc")


def ms_mlp_train(dev, params, X, T, order, lr, grads=False):
    """Adam on the GPU over the minibatches order [n_steps][batch]; returns
    (trained params, per-step losses, first-step gradients or None)."""
    L = lib()
    i, w, o = _mlp_dims(params)
    flat = mlp_pack(params)
    X = np.ascontiguousarray(X, dtype=np.float32)
    T = np.ascontiguousarray(T, dtype=np.float32)
    order = np.ascontiguousarray(order, dtype=np.int32)
    n_steps, batch = order.shape
    losses = np.empty(n_steps, dtype=np.float32)
    g = np.empty_like(flat) if grads else None
    code = L.ms_mlp_train(C.byref(dev.desc), i, w, o, _ptr(flat), len(X), _ptr(X), _ptr(T), n_steps, batch,
                          _ptr(order), C.c_float(lr), _ptr(losses), _ptr(g) if grads else None)
    if code != MS_OK:
        raise MSError(code, "ms_mlp_train")
    return mlp_unpack(flat, i, w, o), losses, (mlp_unpack(g, i, w, o) if grads else None)


def ms_batch_step(contexts, dt, params=None, **kw):
    L = lib()
    p = params or solver_defaults(**kw)
    arr = (C.c_void_p * len(contexts))(*[c.h for c in contexts])
    stats = (ms_step_stats * len(contexts))()
    code = L.ms_batch_step(arr, len(contexts), float(dt), C.byref(p), stats)
    if code != MS_OK:
        msg = (L.ms_last_error(contexts[0].h) or b"").decode()
        raise MSError(code, msg)
    return [s.asdict() for s in stats]


class Batch:
    """A batch of contexts (ms_batch_create); advance() steps them together.
    The contexts must outlive the batch."""

    def __init__(self, contexts):
        self.L = lib()
        self.contexts = list(contexts)
        arr = (C.c_void_p * len(self.contexts))(*[c.h for c in self.contexts])
        h = C.c_void_p()
        code = self.L.ms_batch_create(arr, len(self.contexts), C.byref(h))
        if code != MS_OK:
            raise MSError(code, (self.L.ms_last_error(self.contexts[0].h) or b"").decode())
        self.h = h

    def advance(self, dt, params=None, **kw):
        p = params or solver_defaults(**kw)
        stats = (ms_step_stats * len(self.contexts))()
        code = self.L.ms_batch_advance(self.h, float(dt), C.byref(p), stats)
        if code != MS_OK:
            raise MSError(code, (self.L.ms_last_error(self.contexts[0].h) or b"").decode())
        return [s.asdict() for s in stats]

    def close(self):
        if getattr(self, "h", None):
            self.L.ms_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Matrix:
    """Standalone sliced-BSR3 matrix (ms_mat) for SpMV measurements."""

    def __init__(self, dev: TorchDevice, row_ptr, col, vals, dtype=0):
        self.L = lib()
        rp, cl, vv = _i32(row_ptr), _i32(col), _f64(vals).reshape(-1, 9)
        h = C.c_void_p()
        code = self.L.ms_mat_create(C.byref(dev.desc), len(rp) - 1, _ptr(rp), _ptr(cl), _ptr(vv), int(dtype),
                                    C.byref(h))
        if code != MS_OK:
            raise MSError(code, "ms_mat_create")
        self.h = h
        self.n = len(rp) - 1
        self.dtype = dtype

    def spmv(self, x_ptr: int, y_ptr: int):
        code = self.L.ms_mat_spmv(self.h, C.c_void_p(x_ptr), C.c_void_p(y_ptr))
        if code != MS_OK:
            raise MSError(code, "ms_mat_spmv")

    @property
    def bytes(self):
        return self.L.ms_mat_bytes(self.h)

    def close(self):
        if getattr(self, "h", None):
            self.L.ms_mat_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def context_from_scene(dev: TorchDevice, s, step: int = 1):
    """Create a context and upload a scene dict from the `scenes` generators."""
    c = Context(dev)
    c.ms_upload_mesh(s["rest"], s["tets"])
    if s.get("selfcontact") is not None:
        c.ms_set_self_contact(s["selfcontact"]["dhat"], s["selfcontact"]["kappa"], s["selfcontact"].get("slots", 32))
    c.ms_upload_material(s["E"], s["nu"], s["rho"])
    c.ms_set_gravity(s["gravity"])
    if len(s["dirichlet"]):
        c.ms_set_dirichlet(s["dirichlet"], s["dbc_targets"](step))
    if s["halfspace"] is not None:
        hs = s["halfspace"]
        c.ms_add_halfspace(hs["normal"], hs["offset"], hs["dhat"], hs["kappa"])
        if float(hs.get("mu", 0.0)) > 0.0:
            c.ms_set_friction(hs["mu"], hs.get("eps_v", 1e-3))
    c.ms_set_state(s["x0"], s["v0"])
    return c
