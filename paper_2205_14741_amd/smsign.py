"""Thin ctypes binding of libsmsign.so (the C ABI declared in include/smsign.h).

Only argument marshalling lives here: every step of the method runs in the HIP
kernels behind the C ABI.  PyTorch supplies device memory and the stream.
Loading fails loudly when the library has not been built; there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsmsign.so")

SM_OK, SM_ERR_ARG, SM_ERR_HIP, SM_ERR_NONFINITE, SM_ERR_OOM, SM_ERR_STATE = 0, -1, -2, -3, -4, -5
SM_F64, SM_F32, SM_BF16, SM_F16, SM_BF16X3 = 0, 1, 2, 3, 4
PREC = {"f64": SM_F64, "f32": SM_F32, "bf16": SM_BF16, "f16": SM_F16, "bf16x3": SM_BF16X3}
SM_SCALE_GERSHGORIN, SM_SCALE_POWER, SM_SCALE_LEARNED = 0, 1, 2

EXPORTED = (
    "sm_default_opts", "sm_plan_create", "sm_plan_destroy", "sm_plan_sizes", "sm_plan_info",
    "sm_plan_ws_layout", "build_submatrices", "submatrix_sign", "assemble_P", "energy_trace",
    "sm_density_matrix", "sm_find_mu", "sm_gershgorin_bracket", "sm_selftest_mfma",
    "sm_profile_enable", "sm_profile_read", "sm_last_error", "sm_version",
    "sm_mlp_create", "sm_mlp_destroy", "sm_mlp_set_weights", "sm_mlp_get_weights", "sm_mlp_infer",
    "sm_mlp_loss_grad", "sm_mlp_train", "sm_plan_set_mlp", "sm_autotune", "sm_plan_tuning", "sm_ws_storage",
    "sm_comm_probe", "sm_gershgorin_bracket_noalloc", "sm_overlap_inv_sqrt", "build_submatrices_overlap",
    "assemble_P_overlap", "sm_density_matrix_overlap", "sm_gemm_variants", "sm_scaling_pairs",
    "sm_fermi_dirac", "assemble_P_fermi", "sm_density_matrix_fermi", "sm_find_mu_fermi",
    "sm_plan_set_positions", "sm_plan_chunk_variants",
)


class SmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"smsign error {code}: {msg}")
        self.code = code


class BsrPattern(C.Structure):
    _fields_ = [("n_atoms", C.c_int32), ("block_size", C.c_void_p), ("col_ptr", C.c_void_p),
                ("row_idx", C.c_void_p), ("panel_off", C.c_void_p)]


class SignOpts(C.Structure):
    _fields_ = [("phase1", C.c_int32), ("refine", C.c_int32), ("refine_steps", C.c_int32),
                ("max_iter", C.c_int32), ("tol", C.c_double), ("switch_tol", C.c_double),
                ("stall_below", C.c_double), ("stall_ratio", C.c_double), ("scaling", C.c_int32),
                ("power_steps", C.c_int32), ("scale_margin", C.c_double), ("probes", C.c_int32),
                ("variant", C.c_int32), ("graph_iters", C.c_int32), ("accel", C.c_int32),
                ("lbound", C.c_double), ("comm_probes", C.c_int32), ("retry", C.c_int32),
                ("force_scale", C.c_double)]

    def copy(self) -> "SignOpts":
        o = SignOpts()
        C.pointer(o)[0] = self
        return o


class SubStats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("iters_low", C.c_int32), ("status", C.c_int32),
                ("scale_src", C.c_int32), ("scale", C.c_double), ("res", C.c_double),
                ("res_probe", C.c_double), ("gersh", C.c_double), ("rho_est", C.c_double),
                ("lb0", C.c_double), ("lb_est", C.c_double), ("res_comm", C.c_double),
                ("feat", C.c_float * 16), ("retried", C.c_int32), ("top1", C.c_float)]


STATS_DTYPE = np.dtype([("iters", "<i4"), ("iters_low", "<i4"), ("status", "<i4"),
                        ("scale_src", "<i4"), ("scale", "<f8"), ("res", "<f8"),
                        ("res_probe", "<f8"), ("gersh", "<f8"), ("rho_est", "<f8"),
                        ("lb0", "<f8"), ("lb_est", "<f8"), ("res_comm", "<f8"), ("feat", "<f4", (16,)),
                        ("retried", "<i4"), ("top1", "<f4")])
STATS_FEAT_OFFSET = 80   # bytes from the start of a record to feat[0]
assert STATS_DTYPE.itemsize == C.sizeof(SubStats) == 152
assert STATS_DTYPE.fields["feat"][1] == STATS_FEAT_OFFSET
assert C.sizeof(SignOpts) == 104

_lib = None


def lib() -> C.CDLL:
    """Load libsmsign.so once; raise if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run `python -m paper_2205_14741_amd.build` "
                          "(hipcc, gfx950); there is no CPU fallback")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    sig = {
        "sm_default_opts": (i32, [i32, C.POINTER(SignOpts)]),
        "sm_plan_create": (i32, [C.POINTER(BsrPattern), i32, i64, C.POINTER(vp)]),
        "sm_plan_destroy": (None, [vp]),
        "sm_plan_sizes": (i32, [vp, i32, vp, vp, vp, vp]),
        "sm_plan_info": (i32, [vp, vp, vp, vp, vp, vp]),
        "sm_plan_ws_layout": (i32, [vp, i32, vp, vp]),
        "build_submatrices": (i32, [vp, i32, vp, dbl, C.POINTER(SignOpts), vp, vp, vp]),
        "submatrix_sign": (i32, [vp, i32, vp, C.POINTER(SignOpts), vp, vp]),
        "assemble_P": (i32, [vp, i32, vp, vp, vp]),
        "energy_trace": (i32, [vp, vp, vp, vp, vp, vp]),
        "sm_density_matrix": (i32, [vp, vp, dbl, C.POINTER(SignOpts), vp, vp, vp, vp, vp, vp]),
        "sm_overlap_inv_sqrt": (i32, [vp, i32, vp, dbl, i32, vp, vp, vp, vp, vp]),
        "build_submatrices_overlap": (i32, [vp, i32, vp, dbl, C.POINTER(SignOpts), vp, vp, vp, vp]),
        "assemble_P_overlap": (i32, [vp, i32, vp, vp, vp, vp]),
        "sm_density_matrix_overlap": (i32, [vp, vp, vp, dbl, C.POINTER(SignOpts), vp, vp, vp, vp, vp, vp, vp]),
        "sm_find_mu": (i32, [vp, vp, dbl, dbl, i32, dbl, C.POINTER(SignOpts), vp, vp, vp, vp, vp, vp, vp, vp, vp,
                             vp]),
        "sm_fermi_dirac": (i32, [vp, i32, vp, dbl, vp, vp, vp]),
        "sm_plan_set_positions": (i32, [vp, vp, i32]),
        "sm_plan_chunk_variants": (i32, [vp, i32, vp, vp]),
        "assemble_P_fermi": (i32, [vp, i32, vp, vp, vp]),
        "sm_density_matrix_fermi": (i32, [vp, vp, dbl, dbl, C.POINTER(SignOpts), vp, vp, vp, vp, vp, vp, vp]),
        "sm_find_mu_fermi": (i32, [vp, vp, dbl, dbl, dbl, i32, dbl, C.POINTER(SignOpts), vp, vp, vp, vp, vp, vp,
                                   vp, vp, vp, vp]),
        "sm_gershgorin_bracket": (i32, [vp, vp, vp, vp, vp]),
        "sm_gershgorin_bracket_noalloc": (i32, [vp, vp, vp, vp]),
        "sm_selftest_mfma": (i32, [i32, vp]),
        "sm_profile_enable": (i32, [vp, i32]),
        "sm_profile_read": (i32, [vp, vp, vp]),
        "sm_mlp_create": (i32, [C.c_uint64, C.POINTER(vp)]),
        "sm_mlp_destroy": (None, [vp]),
        "sm_mlp_set_weights": (i32, [vp, vp, vp]),
        "sm_mlp_get_weights": (i32, [vp, vp, vp]),
        "sm_mlp_infer": (i32, [vp, vp, i64, i64, vp, vp]),
        "sm_mlp_loss_grad": (i32, [vp, vp, i64, vp, i64, vp, vp, vp]),
        "sm_mlp_train": (i32, [vp, vp, i64, vp, i64, i32, i32, C.c_float, i32, C.c_uint64, vp, vp]),
        "sm_plan_set_mlp": (i32, [vp, vp]),
        "sm_autotune": (i32, [vp, i32, vp, dbl, C.POINTER(SignOpts), vp, vp, i32, i32, vp, vp, vp]),
        "sm_plan_tuning": (i32, [vp, vp, vp]),
        "sm_gemm_variants": (i32, []),
        "sm_scaling_pairs": (i32, [vp, i64, vp, vp, vp, vp]),
        "sm_ws_storage": (i32, [C.POINTER(SignOpts)]),
        "sm_comm_probe": (i32, [vp, i32, vp, dbl, C.POINTER(SignOpts), vp, vp, vp]),
        "sm_last_error": (C.c_char_p, []),
        "sm_version": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(rc: int):
    if rc != SM_OK:
        raise SmError(rc, lib().sm_last_error().decode())


def _ptr(t) -> int | None:
    """Device pointer of a torch tensor (or None)."""
    if t is None:
        return None
    return t.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


def default_opts(prec="f64", **kw) -> SignOpts:
    o = SignOpts()
    p = PREC[prec] if isinstance(prec, str) else int(prec)
    _check(lib().sm_default_opts(p, C.byref(o)))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def storage_prec(opts: SignOpts) -> int:
    """Workspace storage code of a schedule: SM_F64 / SM_F32 for the iterate's
    type, or the main precision (SM_BF16 / SM_F16 / SM_BF16X3) for float32
    iterates plus the 16-bit operand copies their products read."""
    return int(lib().sm_ws_storage(C.byref(opts)))


def _check_ws(plan, ws, opts: SignOpts):
    """A workspace tensor must hold the bytes the schedule's storage needs."""
    if hasattr(ws, "element_size"):
        need = plan.sizes(storage_prec(opts))[2]
        have = ws.numel() * ws.element_size()
        if have < need:
            raise SmError(1, f"workspace of {have} bytes, the schedule needs {need} "
                             f"(storage code {storage_prec(opts)})")


class Plan:
    """Symbolic plan over a block pattern (host arrays are copied by the library)."""

    def __init__(self, m, pad_to: int = 64, max_chunk_elems: int = 0):
        self.n_atoms = int(m.block_size.shape[0])
        self._bs = np.ascontiguousarray(m.block_size, dtype=np.int32)
        self._cp = np.ascontiguousarray(m.col_ptr, dtype=np.int64)
        self._ri = np.ascontiguousarray(m.row_idx, dtype=np.int32)
        self._po = np.ascontiguousarray(m.panel_off, dtype=np.int64)
        pat = BsrPattern(self.n_atoms, self._bs.ctypes.data, self._cp.ctypes.data,
                         self._ri.ctypes.data, self._po.ctypes.data)
        h = C.c_void_p()
        _check(lib().sm_plan_create(C.byref(pat), int(pad_to), int(max_chunk_elems), C.byref(h)))
        self.handle = h

    def close(self):
        if self.handle:
            lib().sm_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_positions(self, xyz, bucket_rows: int = 512):
        """Processing order: size buckets of bucket_rows padded rows (larger
        first), Morton order of the atom centres inside a bucket.  Before the
        plan's first device use."""
        x = np.ascontiguousarray(xyz, dtype=np.float64).reshape(self.n_atoms, 3)
        _check(lib().sm_plan_set_positions(self.handle, x.ctypes.data, int(bucket_rows)))

    def chunk_variants(self, chunk: int):
        """(size class, GEMM variant per precision) of a chunk."""
        cls = C.c_int32()
        v = np.zeros(5, np.int32)
        _check(lib().sm_plan_chunk_variants(self.handle, int(chunk), C.byref(cls), v.ctypes.data))
        return int(cls.value), v.tolist()

    def sizes(self, storage: int):
        v = [C.c_int64() for _ in range(4)]
        _check(lib().sm_plan_sizes(self.handle, int(storage), *[C.byref(x) for x in v]))
        return tuple(int(x.value) for x in v)  # n_sub, n_chunks, ws_bytes, nvals

    def info(self) -> dict:
        n = self.n_atoms
        out = {k: np.zeros(n, np.int32) for k in ("n", "npad", "loc", "chunk", "order")}
        _check(lib().sm_plan_info(self.handle, *[out[k].ctypes.data for k in
                                                 ("n", "npad", "loc", "chunk", "order")]))
        return out

    def ws_layout(self, storage: int):
        reg = np.zeros(9, np.int64)
        off = np.zeros(self.n_atoms, np.int64)
        _check(lib().sm_plan_ws_layout(self.handle, int(storage), reg.ctypes.data, off.ctypes.data))
        return reg, off

    @property
    def n_chunks(self) -> int:
        return self.sizes(SM_F64)[1]


# ---- the C entry points, same names ----

def build_submatrices(plan: Plan, chunk: int, H, mu: float, opts: SignOpts, ws, stats, stream=None):
    _check_ws(plan, ws, opts)
    _check(lib().build_submatrices(plan.handle, int(chunk), _ptr(H), float(mu), C.byref(opts),
                                   _ptr(ws), _ptr(stats), _stream(stream)))


def submatrix_sign(plan: Plan, chunk: int, ws, opts: SignOpts, stats, stream=None):
    _check_ws(plan, ws, opts)
    _check(lib().submatrix_sign(plan.handle, int(chunk), _ptr(ws), C.byref(opts), _ptr(stats),
                                _stream(stream)))


def sm_comm_probe(plan: Plan, chunk: int, H, mu: float, opts: SignOpts, ws, stats, stream=None):
    _check_ws(plan, ws, opts)
    _check(lib().sm_comm_probe(plan.handle, int(chunk), _ptr(H), float(mu), C.byref(opts), _ptr(ws),
                               _ptr(stats), _stream(stream)))


def assemble_P(plan: Plan, chunk: int, ws, P, stream=None):
    _check(lib().assemble_P(plan.handle, int(chunk), _ptr(ws), _ptr(P), _stream(stream)))


def energy_trace(plan: Plan, H, P, stream=None):
    E, Ne = C.c_double(), C.c_double()
    _check(lib().energy_trace(plan.handle, _ptr(H), _ptr(P), C.byref(E), C.byref(Ne), _stream(stream)))
    return E.value, Ne.value


def sm_density_matrix(plan: Plan, H, mu: float, opts: SignOpts, ws, P, stats, stream=None):
    _check_ws(plan, ws, opts)
    E, Ne = C.c_double(), C.c_double()
    _check(lib().sm_density_matrix(plan.handle, _ptr(H), float(mu), C.byref(opts), _ptr(ws), _ptr(P),
                                   _ptr(stats), C.byref(E), C.byref(Ne), _stream(stream)))
    return E.value, Ne.value


def sm_overlap_inv_sqrt(plan: Plan, chunk: int, S, ws_aux, ws, tol=1e-12, max_iter=100, stream=None):
    """Z_i = T_i(S)^(-1/2) of the chunk's submatrices into ws_aux buffer 0;
    returns (steps, largest final residual)."""
    it, r = C.c_int32(), C.c_double()
    _check(lib().sm_overlap_inv_sqrt(plan.handle, int(chunk), _ptr(S), float(tol), int(max_iter), _ptr(ws_aux),
                                     _ptr(ws), C.byref(it), C.byref(r), _stream(stream)))
    return it.value, r.value


def build_submatrices_overlap(plan: Plan, chunk: int, H, mu: float, opts: SignOpts, ws, ws_aux, stats,
                              stream=None):
    _check_ws(plan, ws, opts)
    _check(lib().build_submatrices_overlap(plan.handle, int(chunk), _ptr(H), float(mu), C.byref(opts), _ptr(ws),
                                           _ptr(ws_aux), _ptr(stats), _stream(stream)))


def assemble_P_overlap(plan: Plan, chunk: int, ws, ws_aux, P, stream=None):
    _check(lib().assemble_P_overlap(plan.handle, int(chunk), _ptr(ws), _ptr(ws_aux), _ptr(P), _stream(stream)))


def sm_density_matrix_overlap(plan: Plan, H, S, mu: float, opts: SignOpts, ws, ws_aux, P, stats, stream=None):
    """P for S != I at fixed mu; returns (E = tr(PH), Ne = tr(PS))."""
    _check_ws(plan, ws, opts)
    _check_ws(plan, ws_aux, opts)
    E, Ne = C.c_double(), C.c_double()
    _check(lib().sm_density_matrix_overlap(plan.handle, _ptr(H), _ptr(S), float(mu), C.byref(opts), _ptr(ws),
                                           _ptr(ws_aux), _ptr(P), _ptr(stats), C.byref(E), C.byref(Ne),
                                           _stream(stream)))
    return E.value, Ne.value


def sm_find_mu(plan: Plan, H, n_target: float, opts: SignOpts, ws, stats, P=None, accept=0.5,
               max_steps=60, stream=None, energy=False, mu_start=None):
    """(mu, bisection steps, [(mu_k, Ne_k)]), and with energy=True (needs P)
    also E = tr(P H) and Ne = tr P of the returned P.  mu_start: warm start
    (evaluated first; None = the cold rule)."""
    _check_ws(plan, ws, opts)
    if energy and P is None:
        raise SmError(SM_ERR_ARG, "sm_find_mu: energy=True needs P")
    mu = C.c_double()
    steps = C.c_int32()
    E, Ne = C.c_double(), C.c_double()
    mh = np.zeros(max_steps)
    nh = np.zeros(max_steps)
    _check(lib().sm_find_mu(plan.handle, _ptr(H), float(n_target), float(accept), int(max_steps),
                            float("nan") if mu_start is None else float(mu_start), C.byref(opts), _ptr(ws), _ptr(P), _ptr(stats), C.byref(mu),
                            C.byref(steps), mh.ctypes.data, nh.ctypes.data,
                            C.byref(E) if energy else None, C.byref(Ne) if energy else None,
                            _stream(stream)))
    k = steps.value
    hist = list(zip(mh[:k].tolist(), nh[:k].tolist()))
    if energy:
        return mu.value, k, hist, E.value, Ne.value
    return mu.value, k, hist


def sm_fermi_dirac(plan: Plan, chunk: int, ws, beta: float, stats, stream=None):
    """f(T_i) = (I + exp(beta T_i))^-1 for the chunk's submatrices (after
    build_submatrices with the float64 schedule); returns the doublings m."""
    m = C.c_int32()
    _check(lib().sm_fermi_dirac(plan.handle, int(chunk), _ptr(ws), float(beta), _ptr(stats), C.byref(m),
                                _stream(stream)))
    return m.value


def assemble_P_fermi(plan: Plan, chunk: int, ws, P, stream=None):
    _check(lib().assemble_P_fermi(plan.handle, int(chunk), _ptr(ws), _ptr(P), _stream(stream)))


def sm_density_matrix_fermi(plan: Plan, H, mu: float, beta: float, opts: SignOpts, ws, P, stats, stream=None):
    """Finite-temperature P at fixed mu; returns (E = tr(PH), Ne = tr P, dNe/dmu)."""
    _check_ws(plan, ws, opts)
    E, Ne, dNe = C.c_double(), C.c_double(), C.c_double()
    _check(lib().sm_density_matrix_fermi(plan.handle, _ptr(H), float(mu), float(beta), C.byref(opts), _ptr(ws),
                                         _ptr(P), _ptr(stats), C.byref(E), C.byref(Ne), C.byref(dNe),
                                         _stream(stream)))
    return E.value, Ne.value, dNe.value


def sm_find_mu_fermi(plan: Plan, H, n_target: float, beta: float, opts: SignOpts, ws, P, stats, tol=1e-8,
                     max_steps=60, mu_start=None, stream=None):
    """(mu, evaluations, [(mu_k, Ne_k)], E, Ne) at inverse temperature beta:
    safeguarded Newton on the electron count; P holds P at mu."""
    _check_ws(plan, ws, opts)
    mu, steps = C.c_double(), C.c_int32()
    E, Ne = C.c_double(), C.c_double()
    mh = np.zeros(max_steps)
    nh = np.zeros(max_steps)
    _check(lib().sm_find_mu_fermi(plan.handle, _ptr(H), float(n_target), float(beta), float(tol), int(max_steps),
                                  float("nan") if mu_start is None else float(mu_start), C.byref(opts), _ptr(ws),
                                  _ptr(P), _ptr(stats), C.byref(mu), C.byref(steps), mh.ctypes.data,
                                  nh.ctypes.data, C.byref(E), C.byref(Ne), _stream(stream)))
    k = steps.value
    return mu.value, k, list(zip(mh[:k].tolist(), nh[:k].tolist())), E.value, Ne.value


def sm_gershgorin_bracket(plan: Plan, H, stream=None):
    lo, hi = C.c_double(), C.c_double()
    _check(lib().sm_gershgorin_bracket(plan.handle, _ptr(H), C.byref(lo), C.byref(hi), _stream(stream)))
    return lo.value, hi.value


def sm_gershgorin_bracket_noalloc(plan: Plan, H, lohi, stream=None):
    """[lo, hi] into the device tensor lohi (2 float64), allocating nothing;
    asynchronous."""
    _check(lib().sm_gershgorin_bracket_noalloc(plan.handle, _ptr(H), _ptr(lohi), _stream(stream)))


def sm_selftest_mfma(prec) -> np.ndarray:
    """prec: a precision name / code (its 16x16 instruction, 256 values) or
    5 / 6 (the 32x32x16 f16 / bf16 instruction, 1024 values)."""
    p = PREC[prec] if isinstance(prec, str) else int(prec)
    out = np.zeros(1024 if p >= 5 else 256)
    _check(lib().sm_selftest_mfma(p, out.ctypes.data))
    return out


def sm_profile_enable(plan: Plan, on: bool = True):
    _check(lib().sm_profile_enable(plan.handle, 1 if on else 0))


def sm_profile_read(plan: Plan):
    """(launches[10], ms[10]) per class 2 * precision + kind."""
    n = np.zeros(10, np.int64)
    t = np.zeros(10)
    _check(lib().sm_profile_read(plan.handle, n.ctypes.data, t.ctypes.data))
    return n, t


N_MLP_PARAMS = 5378


class Mlp:
    """The spectral-scaling network (device buffers owned by the library)."""

    def __init__(self, seed: int = 0):
        h = C.c_void_p()
        _check(lib().sm_mlp_create(int(seed), C.byref(h)))
        self.handle = h

    def close(self):
        if self.handle:
            lib().sm_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_weights(self, params=None, norm=None):
        p = None if params is None else np.ascontiguousarray(params, dtype=np.float32)
        q = None if norm is None else np.ascontiguousarray(norm, dtype=np.float32)
        _check(lib().sm_mlp_set_weights(self.handle, None if p is None else p.ctypes.data,
                                        None if q is None else q.ctypes.data))

    def get_weights(self):
        p = np.zeros(N_MLP_PARAMS, np.float32)
        q = np.zeros(32, np.float32)
        _check(lib().sm_mlp_get_weights(self.handle, p.ctypes.data, q.ctypes.data))
        return p, q


def sm_mlp_infer(mlp: Mlp, X, n: int, ldx: int = 16, Y=None, stream=None):
    import torch
    Y = Y if Y is not None else torch.empty((n, 2), dtype=torch.float32, device=X.device)
    _check(lib().sm_mlp_infer(mlp.handle, _ptr(X), int(ldx), int(n), _ptr(Y), _stream(stream)))
    return Y


def sm_mlp_loss_grad(mlp: Mlp, X, T, n: int, ldx: int = 16, stream=None):
    loss = C.c_double()
    g = np.zeros(N_MLP_PARAMS, np.float32)
    _check(lib().sm_mlp_loss_grad(mlp.handle, _ptr(X), int(ldx), _ptr(T), int(n), C.byref(loss),
                                  g.ctypes.data, _stream(stream)))
    return loss.value, g


def sm_mlp_train(mlp: Mlp, X, T, n: int, epochs: int, batch: int, lr: float, ldx: int = 16,
                 fit_norm: bool = True, shuffle_seed: int = 1, stream=None):
    hist = np.zeros(max(epochs, 1))
    _check(lib().sm_mlp_train(mlp.handle, _ptr(X), int(ldx), _ptr(T), int(n), int(epochs), int(batch),
                              float(lr), 1 if fit_norm else 0, int(shuffle_seed), hist.ctypes.data,
                              _stream(stream)))
    return hist[:epochs]


def sm_scaling_pairs(stats, n: int, stream=None):
    """Training pairs (X [k, 16], T [k, 2], device float32) of the scaling
    network from the records `stats` (device) of an explicit pass."""
    import torch
    X = torch.empty((max(n, 1), 16), dtype=torch.float32, device=stats.device)
    T = torch.empty((max(n, 1), 2), dtype=torch.float32, device=stats.device)
    k = C.c_int64()
    _check(lib().sm_scaling_pairs(_ptr(stats), int(n), _ptr(X), _ptr(T), C.byref(k), _stream(stream)))
    return X[:k.value], T[:k.value]


def sm_plan_set_mlp(plan: Plan, mlp: Mlp | None):
    _check(lib().sm_plan_set_mlp(plan.handle, None if mlp is None else mlp.handle))




def sm_autotune(plan: Plan, chunk: int, H, mu: float, opts: SignOpts, ws, stats, repeats: int = 2,
                variants=None, stream=None):
    """(best variant, sign-phase ms per variant) -- the plan keeps the choice."""
    _check_ws(plan, ws, opts)
    best = C.c_int32()
    t = np.zeros(int(lib().sm_gemm_variants()))
    mask = 0 if variants is None else sum(1 << v for v in variants)
    _check(lib().sm_autotune(plan.handle, int(chunk), _ptr(H), float(mu), C.byref(opts), _ptr(ws),
                             _ptr(stats), int(repeats), int(mask), C.byref(best), t.ctypes.data,
                             _stream(stream)))
    return best.value, t


def sm_plan_tuning(plan: Plan, table=None):
    """Current tuned variant per precision; replace it with `table` if given."""
    get = np.zeros(5, np.int32)
    st = None if table is None else np.ascontiguousarray(table, dtype=np.int32)
    _check(lib().sm_plan_tuning(plan.handle, get.ctypes.data, None if st is None else st.ctypes.data))
    return get


def version() -> str:
    return lib().sm_version().decode()


# ---- convenience: buffers owned by torch ----

class Workspace:
    """Device buffers for one plan and one storage precision (torch-owned)."""

    def __init__(self, plan: Plan, storage: int, device="cuda"):
        import torch
        n_sub, n_chunks, ws_bytes, nvals = plan.sizes(storage)
        self.plan = plan
        self.storage = storage
        self.ws = torch.empty(ws_bytes, dtype=torch.uint8, device=device)
        self.stats = torch.zeros(n_sub * STATS_DTYPE.itemsize, dtype=torch.uint8, device=device)
        self.P = torch.zeros(nvals, dtype=torch.float64, device=device)

    def stats_host(self) -> np.ndarray:
        return self.stats.cpu().numpy().view(STATS_DTYPE)


def density_matrix(plan: Plan, H, mu: float, opts: SignOpts, work: Workspace | None = None,
                   stream=None):
    """P, E = tr(PH), Ne = tr P and the per-submatrix records at fixed mu."""
    work = work or Workspace(plan, storage_prec(opts), H.device)
    E, Ne = sm_density_matrix(plan, H, mu, opts, work.ws, work.P, work.stats, stream)
    return work.P, E, Ne, work.stats_host()
