"""ctypes declarations for libsyk and thin wrappers with the C ABI's names."""
import ctypes as ct
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "libsyk.so")

C64, C128 = 0, 1
EXACT_K, BERNOULLI = 0, 1
BLOCK_U, BLOCK_D, FULL = 0, 1, 2

STATUS = {0: "SYK_OK", 1: "SYK_EINVAL", 2: "SYK_EUNSUPPORTED", 3: "SYK_ENOMEM", 4: "SYK_EDEVICE",
          5: "SYK_ENOTCONV", 6: "SYK_ENUMERIC", 7: "SYK_ECANCELLED", 8: "SYK_EAGAIN"}
EAGAIN, ECANCELLED = 8, 7


class SykError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


if not os.path.exists(_LIBPATH):
    raise ImportError(f"libsyk.so not built ({_LIBPATH}); run `python paper_2311_00639_amd/build.py`")
_lib = ct.CDLL(_LIBPATH)


def library_path() -> str:
    return _LIBPATH


class HamInfo(ct.Structure):
    _fields_ = [("N", ct.c_int), ("L", ct.c_int), ("K", ct.c_int), ("k", ct.c_double), ("p", ct.c_double),
                ("sigma", ct.c_double), ("sum_J2", ct.c_double), ("seed", ct.c_uint64), ("block_dim", ct.c_uint64)]


class KrylovOpts(ct.Structure):
    _fields_ = [("m", ct.c_int), ("tol", ct.c_double), ("reorth", ct.c_int), ("max_substeps", ct.c_int)]


class KrylovStats(ct.Structure):
    _fields_ = [("substeps", ct.c_int), ("matvecs", ct.c_int), ("breakdown", ct.c_int), ("err_est", ct.c_double),
                ("reorths", ct.c_int)]


PROGRESS_FN = ct.CFUNCTYPE(None, ct.c_void_p, ct.c_int, ct.c_int)


class OtocOpts(ct.Structure):
    _fields_ = [("nvec", ct.c_int), ("state_seed", ct.c_uint64), ("dtype", ct.c_int), ("krylov", KrylovOpts),
                ("profile", ct.c_int), ("layout", ct.c_int), ("autotune", ct.c_int),
                ("progress", PROGRESS_FN), ("progress_ctx", ct.c_void_p), ("precision_check", ct.c_int)]


class PlanDesc(ct.Structure):
    _fields_ = [("tiled", ct.c_int), ("variant", ct.c_int), ("tile_bits", ct.c_int), ("rot", ct.c_int),
                ("n_groups", ct.c_int),
                ("classes_xcd", ct.c_int), ("classes_gpu", ct.c_int), ("res_bits", ct.c_int),
                ("tiles_per_wg", ct.c_int), ("n_partners", ct.c_int), ("n_tiles", ct.c_uint64)]


class OtocStats(ct.Structure):
    _fields_ = [("matvecs", ct.c_longlong), ("substeps", ct.c_longlong), ("seconds", ct.c_double),
                ("max_err_est", ct.c_double), ("apply_ms", ct.c_double), ("apply_launches", ct.c_longlong),
                ("mp_err", ct.c_double), ("mp_seconds", ct.c_double)]


class EngineOpts(ct.Structure):
    _fields_ = [("budget_bytes", ct.c_uint64), ("max_active", ct.c_int), ("max_bypass", ct.c_int)]


class Request(ct.Structure):
    _fields_ = [("N", ct.c_int), ("k", ct.c_double), ("seed", ct.c_uint64), ("i", ct.c_int), ("j", ct.c_int),
                ("beta", ct.c_double), ("t", ct.POINTER(ct.c_double)), ("nt", ct.c_int), ("nvec", ct.c_int),
                ("state_seed", ct.c_uint64), ("dtype", ct.c_int), ("m", ct.c_int), ("m_min", ct.c_int),
                ("tol", ct.c_double), ("precision_check", ct.c_int)]


class ResultInfo(ct.Structure):
    _fields_ = [("id", ct.c_uint64), ("status", ct.c_int), ("nt", ct.c_int), ("m_used", ct.c_int),
                ("footprint_bytes", ct.c_uint64), ("t_submit", ct.c_double), ("t_start", ct.c_double),
                ("t_end", ct.c_double), ("stats", OtocStats)]


class EngineStats(ct.Structure):
    _fields_ = [("submitted", ct.c_longlong), ("completed", ct.c_longlong), ("failed", ct.c_longlong),
                ("cancelled", ct.c_longlong), ("queued", ct.c_int), ("active", ct.c_int),
                ("budget_bytes", ct.c_uint64), ("bytes_in_use", ct.c_uint64), ("peak_bytes", ct.c_uint64),
                ("p50_latency_s", ct.c_double), ("p99_latency_s", ct.c_double), ("busy_seconds", ct.c_double)]


class BatchItem(ct.Structure):
    _fields_ = [("N", ct.c_int), ("k", ct.c_double), ("seed", ct.c_uint64), ("i", ct.c_int), ("j", ct.c_int),
                ("state_seed", ct.c_uint64), ("ensemble", ct.c_int)]


class BatchOpts(ct.Structure):
    _fields_ = [("nvec", ct.c_int), ("beta", ct.c_double), ("m", ct.c_int), ("tol", ct.c_double),
                ("variant", ct.c_int), ("max_substeps", ct.c_int)]


class BatchStats(ct.Structure):
    _fields_ = [("matvecs", ct.c_longlong), ("n_jobs", ct.c_int), ("slots", ct.c_int), ("variant", ct.c_int),
                ("kernel_ms", ct.c_double), ("tuned_ms", ct.c_double * 3), ("seconds", ct.c_double)]


class EnsembleDesc(ct.Structure):
    _fields_ = [("N", ct.c_int), ("k", ct.c_double), ("ensemble", ct.c_int), ("seed", ct.c_uint64),
                ("n_real", ct.c_int), ("i", ct.c_int), ("j", ct.c_int), ("beta", ct.c_double), ("path", ct.c_int)]


class EnsembleStats(ct.Structure):
    _fields_ = [("path", ct.c_int), ("matvecs", ct.c_longlong), ("seconds", ct.c_double)]


class FitOpts(ct.Structure):
    _fields_ = [("method", ct.c_int), ("terms", ct.c_int), ("dN", ct.c_int)]


class FitResult(ct.Structure):
    _fields_ = [("lambda_", ct.c_double), ("lambda_err", ct.c_double), ("coef", ct.c_double * 3),
                ("coef_err", ct.c_double * 3), ("chi2", ct.c_double), ("n_points", ct.c_int), ("dof", ct.c_int)]


FIT_SLOPE, FIT_GLOBAL = 0, 1

_vp, _u64, _i, _d = ct.c_void_p, ct.c_uint64, ct.c_int, ct.c_double
_dp = ct.POINTER(ct.c_double)
_SIGS = {
    "syk_create_hamiltonian": [_i, _i, _d, _u64, ct.POINTER(_vp)],
    "syk_create_hamiltonian_ensemble": [_i, _i, _d, _u64, _i, ct.POINTER(_vp)],
    "syk_destroy_hamiltonian": [_vp],
    "syk_ham_get_info": [_vp, ct.POINTER(HamInfo)],
    "syk_get_terms": [_vp, ct.c_size_t, _vp, _vp, _vp, _vp, _vp, _vp],
    "syk_apply_H": [_vp, _i, _i, _vp, _vp, _u64, _i, _u64, _vp],
    "syk_haar_state": [_i, _u64, _i, _i, _vp, _vp, _vp],
    "syk_haar_state_noalloc": [_i, _u64, _i, _i, _vp, _vp, _vp],
    "syk_apply_majorana": [_i, _i, _i, _i, _vp, _vp, _u64, _d, _d, _vp],
    "syk_krylov_expm": [_vp, _i, _i, _d, _d, _vp, _vp, _u64, ct.POINTER(KrylovOpts), ct.POINTER(KrylovStats), _vp],
    "syk_otoc": [_vp, _i, _i, _d, _dp, _i, ct.POINTER(OtocOpts), _dp, _dp, _dp, ct.POINTER(OtocStats), _vp],
    "syk_workspace_bytes": [_i, _i, _i, _i, ct.POINTER(_u64)],
    "syk_tridiag_expm": [_i, _dp, _dp, _d, _d, _dp, _dp],
    "syk_release_workspace": [],
    "syk_plan_describe": [_vp, _i, _i, _i, ct.POINTER(PlanDesc)],
    "syk_plan_blocks": [_vp, _i, _i, _i, ct.c_void_p, ct.c_size_t, ct.POINTER(ct.c_size_t)],
    "syk_autotune": [_vp, _i, ct.POINTER(_i), ct.POINTER(ct.c_float), _i, _vp],
    "syk_select_variant": [_vp, _i, _i],
    "syk_op_create": [_i, ct.c_size_t, _vp, _vp, _dp, _dp, ct.POINTER(_vp)],
    "syk_op_destroy": [_vp],
    "syk_op_product": [_vp, _vp, ct.POINTER(_vp)],
    "syk_op_sum": [_vp, _vp, _d, _d, _d, _d, ct.POINTER(_vp)],
    "syk_op_adjoint": [_vp, ct.POINTER(_vp)],
    "syk_op_get_terms": [_vp, ct.c_size_t, ct.POINTER(ct.c_size_t), _vp, _vp, _dp, _dp],
    "syk_op_is_hermitian": [_vp, ct.POINTER(_i)],
    "syk_op_to_hamiltonian": [_vp, ct.POINTER(_vp)],
    "syk_otoc_batch": [ct.POINTER(BatchItem), _i, _dp, _i, ct.POINTER(BatchOpts), _dp, _dp, _dp,
                       ct.POINTER(BatchStats), _vp],
    "syk_green": [_vp, _i, _d, _dp, _i, ct.POINTER(OtocOpts), _dp, _dp, _dp, ct.POINTER(OtocStats), _vp],
    "syk_otoc_ensemble": [ct.POINTER(EnsembleDesc), _dp, _i, ct.POINTER(OtocOpts), _dp, _dp, _dp,
                          ct.POINTER(EnsembleStats), _vp],
    "syk_crossing_time": [_dp, _dp, _dp, _i, _d, _dp, _dp],
    "syk_lyapunov_fit": [_dp, _dp, _dp, _i, ct.POINTER(FitOpts), ct.POINTER(FitResult), _dp, _dp, _dp, _i],
    "syk_engine_create": [ct.POINTER(EngineOpts), ct.POINTER(_vp)],
    "syk_engine_submit": [_vp, ct.POINTER(Request), ct.POINTER(_u64)],
    "syk_engine_poll": [_vp, _i, ct.POINTER(ResultInfo), _dp, _dp, _dp, _i],
    "syk_engine_cancel": [_vp, _u64],
    "syk_engine_get_stats": [_vp, ct.POINTER(EngineStats)],
    "syk_engine_destroy": [_vp],
}
for _name, _args in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = ct.c_int
_lib.syk_status_string.argtypes = [ct.c_int]
_lib.syk_status_string.restype = ct.c_char_p
_lib.syk_last_error.argtypes = []
_lib.syk_last_error.restype = ct.c_char_p
_lib.syk_kernel_revision.argtypes = []
_lib.syk_kernel_revision.restype = ct.c_char_p
_lib.syk_krylov_default_opts.argtypes = [ct.c_int, ct.POINTER(KrylovOpts)]
_lib.syk_krylov_default_opts.restype = None


def _check(status):
    if status != 0:
        raise SykError(status, _lib.syk_last_error().decode())


def _ptr(a):
    """Device pointer of a torch tensor, or an int address."""
    if a is None:
        return None
    if isinstance(a, int):
        return a
    return a.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        if not torch.cuda.is_available():
            return None          # the library reports the missing device itself
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _dtype_of(t):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("state vectors must be torch tensors")
    if t.dtype == torch.complex64:
        return C64
    if t.dtype == torch.complex128:
        return C128
    raise TypeError("state vectors must be complex64 or complex128")


def _vectors(need: int, **tensors) -> int:
    """Check the state-vector tensors of one call before any pointer reaches the library:
    torch tensors of one complex dtype, contiguous, each holding at least `need` elements,
    on a GPU.  Returns the dtype code.  The library sees only raw addresses and sizes, so a
    short, strided or host tensor would otherwise be read or written out of bounds."""
    import torch
    dt = None
    for name, t in tensors.items():
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch tensor")
        d = _dtype_of(t)
        if dt is not None and d != dt:
            raise TypeError(f"{name} must have the dtype of the other vectors of the call")
        dt = d
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        if t.numel() < need:
            raise ValueError(f"{name} holds {t.numel()} elements, the call needs {need}")
    for name, t in tensors.items():
        if not t.is_cuda:
            raise TypeError(f"{name} must be on the GPU")
    return dt


class Hamiltonian:
    """Owned handle to one disorder realisation (syk_create_hamiltonian_ensemble)."""

    def __init__(self, N: int, q: int, k: float, seed: int, ensemble: int = EXACT_K):
        h = _vp()
        _check(_lib.syk_create_hamiltonian_ensemble(N, q, float(k), seed, ensemble, ct.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        inf = HamInfo()
        _check(_lib.syk_ham_get_info(self._h, ct.byref(inf)))
        return {f: getattr(inf, f) for f, _ in HamInfo._fields_}

    def terms(self) -> dict:
        K = self.info()["K"]
        ijkl = np.zeros((K, 4), dtype=np.int32)
        J = np.zeros(K)
        x = np.zeros(K, dtype=np.uint64)
        z = np.zeros(K, dtype=np.uint64)
        pu = np.zeros(K, dtype=np.int8)
        pd = np.zeros(K, dtype=np.int8)
        _check(_lib.syk_get_terms(self._h, K, ijkl.ctypes.data, J.ctypes.data, x.ctypes.data, z.ctypes.data,
                                  pu.ctypes.data, pd.ctypes.data))
        return {"ijkl": ijkl, "J": J, "xmask": x, "zmask": z, "phase_U": pu, "phase_D": pd}

    def close(self):
        if self._h:
            _lib.syk_destroy_hamiltonian(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def create_hamiltonian(N: int, q: int, k: float, seed: int, ensemble: int = EXACT_K) -> Hamiltonian:
    """One realisation: ensemble EXACT_K (exactly round(kN) subsets) or BERNOULLI (the
    paper's B(p) ensemble, p = kN / C(N,4); p = 1 is dense SYK)."""
    return Hamiltonian(N, q, k, seed, ensemble)


def apply_H(ham: Hamiltonian, block: int, x, y, nvec: int = 1, ld: int = None, stream=None):
    """y = H_block x for torch tensors x, y of complex dtype on the GPU (block FULL: the whole
    2^(N/2) space, U block then D block).

    With nvec > 1 the tensors hold nvec vectors of leading dimension ld (elements)."""
    n = (2 if block == FULL else 1) << ham.info()["L"]
    ld = n if ld is None else ld
    if nvec < 1 or ld < n:
        raise ValueError("nvec must be >= 1 and ld >= the vector length")
    dt = _vectors((nvec - 1) * ld + n, x=x, y=y)
    _check(_lib.syk_apply_H(ham.handle, block, dt, _ptr(x), _ptr(y), n, nvec, ld, _stream(stream)))


def haar_state(N: int, state_seed: int, v: int, psi_U, psi_D, stream=None):
    """The normalised Haar state number v of the seed, split into its U and D blocks."""
    if N < 6 or N % 2:
        raise ValueError("N must be even and >= 6")
    dt = _vectors(1 << (N // 2 - 1), psi_U=psi_U, psi_D=psi_D)
    _check(_lib.syk_haar_state(N, state_seed, v, dt, _ptr(psi_U), _ptr(psi_D), _stream(stream)))


def haar_state_noalloc(N: int, state_seed: int, v: int, psi_U, psi_D, stream=None):
    """haar_state through the entry point that allocates no device memory (its partial sums
    sit in the library's fixed device scratch); asynchronous on the stream."""
    if N < 6 or N % 2:
        raise ValueError("N must be even and >= 6")
    dt = _vectors(1 << (N // 2 - 1), psi_U=psi_U, psi_D=psi_D)
    _check(_lib.syk_haar_state_noalloc(N, state_seed, v, dt, _ptr(psi_U), _ptr(psi_D), _stream(stream)))


def apply_majorana(N: int, n: int, src_block: int, x, y, scale: complex = 1.0, stream=None):
    if N < 6 or N % 2:
        raise ValueError("N must be even and >= 6")
    amps = 1 << (N // 2 - 1)
    sc = complex(scale)
    dt = _vectors(amps, x=x, y=y)
    _check(_lib.syk_apply_majorana(N, n, src_block, dt, _ptr(x), _ptr(y), amps, sc.real, sc.imag,
                                   _stream(stream)))


def default_krylov_opts(dtype: int) -> KrylovOpts:
    o = KrylovOpts()
    _lib.syk_krylov_default_opts(dtype, ct.byref(o))
    return o


def krylov_expm(ham: Hamiltonian, block: int, z: complex, v, out, m: int = None, tol: float = None,
                reorth: int = None, max_substeps: int = None, stream=None) -> dict:
    """out = e^{z H_block} v.  Returns the Krylov statistics as a dict."""
    n = (2 if block == FULL else 1) << ham.info()["L"]
    dt = _vectors(n, v=v, out=out)
    o = default_krylov_opts(dt)
    if m is not None:
        o.m = m
    if tol is not None:
        o.tol = tol
    if reorth is not None:
        o.reorth = reorth
    if max_substeps is not None:
        o.max_substeps = max_substeps
    st = KrylovStats()
    z = complex(z)
    _check(_lib.syk_krylov_expm(ham.handle, block, dt, z.real, z.imag, _ptr(v), _ptr(out), n, ct.byref(o),
                                ct.byref(st), _stream(stream)))
    return {f: getattr(st, f) for f, _ in KrylovStats._fields_}


def otoc(ham: Hamiltonian, i: int, j: int, beta: float, t, nvec: int = 1, state_seed: int = 0, dtype: int = C128,
         m: int = None, tol: float = None, reorth: int = None, profile: bool = False, layout: int = -1,
         autotune: bool = True, progress=None, precision_check: bool = False, stream=None):
    """Regularised OTOC (Eq. (2)) by the random-state estimator.  Returns
    (F_raw, F_norm, F_imag, stats) with numpy float64 arrays.  progress(done, total) is
    called after each t point of each chain.  precision_check (complex64): stats["mp_err"]
    is the result's error against a complex128 re-evaluation at t = 0 and the last t."""
    t = np.ascontiguousarray(np.asarray(t, dtype=np.float64))
    nt = t.size
    o = OtocOpts()
    o.nvec = nvec
    o.state_seed = state_seed
    o.dtype = dtype
    o.krylov = default_krylov_opts(dtype)
    o.profile = 1 if profile else 0
    o.layout = layout
    o.autotune = 1 if autotune else 0
    o.precision_check = 1 if precision_check else 0
    cb = None
    if progress is not None:
        cb = PROGRESS_FN(lambda ctx, done, total: progress(done, total))
        o.progress = cb
    if m is not None:
        o.krylov.m = m
    if tol is not None:
        o.krylov.tol = tol
    if reorth is not None:
        o.krylov.reorth = reorth
    raw = np.zeros(nt)
    nrm = np.zeros(nt)
    im = np.zeros(nt)
    st = OtocStats()
    dp = lambda a: a.ctypes.data_as(_dp)
    _check(_lib.syk_otoc(ham.handle, i, j, float(beta), dp(t), nt, ct.byref(o), dp(raw), dp(nrm), dp(im),
                         ct.byref(st), _stream(stream)))
    return raw, nrm, im, {f: getattr(st, f) for f, _ in OtocStats._fields_}


def green(ham: Hamiltonian, n: int, beta: float, t, nvec: int = 1, state_seed: int = 0, dtype: int = C128,
          m: int = None, tol: float = None, profile: bool = False, layout: int = -1, autotune: bool = True,
          precision_check: bool = False, stream=None):
    """Green function of chi_n by the random-state estimator (syk_green).  Returns
    (G_raw, G_norm, G_imag, stats); G_norm is the paper's G_R(t) = Re G(t) / G(0)."""
    t = np.ascontiguousarray(np.asarray(t, dtype=np.float64))
    nt = t.size
    o = OtocOpts()
    o.nvec = nvec
    o.state_seed = state_seed
    o.dtype = dtype
    o.krylov = default_krylov_opts(dtype)
    o.profile = 1 if profile else 0
    o.layout = layout
    o.autotune = 1 if autotune else 0
    o.precision_check = 1 if precision_check else 0
    if m is not None:
        o.krylov.m = m
    if tol is not None:
        o.krylov.tol = tol
    raw, nrm, im = np.zeros(nt), np.zeros(nt), np.zeros(nt)
    st = OtocStats()
    dp = lambda a: a.ctypes.data_as(_dp)
    _check(_lib.syk_green(ham.handle, n, float(beta), dp(t), nt, ct.byref(o), dp(raw), dp(nrm), dp(im),
                          ct.byref(st), _stream(stream)))
    return raw, nrm, im, {f: getattr(st, f) for f, _ in OtocStats._fields_}


def otoc_batch(items, beta: float, t, nvec: int = 1, m: int = 30, tol: float = 1e-7, variant: int = -1,
               max_substeps: int = 0, stream=None):
    """Batched OTOC (syk_otoc_batch).  items: sequence of (N, k, seed, i, j, state_seed) or
    (N, k, seed, i, j, state_seed, ensemble).  Returns (F_raw, F_norm, F_imag, stats) with
    arrays of shape (len(items), len(t))."""
    t = np.ascontiguousarray(np.asarray(t, dtype=np.float64))
    nt = t.size
    n = len(items)
    arr = (BatchItem * n)(*[BatchItem(int(it[0]), float(it[1]), int(it[2]), int(it[3]), int(it[4]), int(it[5]),
                                      int(it[6]) if len(it) > 6 else EXACT_K) for it in items])
    o = BatchOpts(nvec, float(beta), m, float(tol), variant, max_substeps)
    raw, nrm, im = np.zeros((n, nt)), np.zeros((n, nt)), np.zeros((n, nt))
    st = BatchStats()
    dp = lambda a: a.ctypes.data_as(_dp)
    _check(_lib.syk_otoc_batch(arr, n, dp(t), nt, ct.byref(o), dp(raw), dp(nrm), dp(im), ct.byref(st),
                               _stream(stream)))
    out = {f: getattr(st, f) for f, _ in BatchStats._fields_ if f != "tuned_ms"}
    out["tuned_ms"] = list(st.tuned_ms)
    return raw, nrm, im, out


def otoc_ensemble(N: int, k: float, seed: int, n_real: int, i: int, j: int, beta: float, t, ensemble: int = EXACT_K,
                  nvec: int = 1, state_seed: int = 0, dtype: int = C64, m: int = None, tol: float = None,
                  path: int = -1, rows: bool = False, stream=None):
    """Disorder-averaged normalised OTOC (syk_otoc_ensemble).  Returns (F_mean, F_sem, stats),
    plus the per-realisation curves (n_real x nt) when rows is true."""
    t = np.ascontiguousarray(np.asarray(t, dtype=np.float64))
    nt = t.size
    d = EnsembleDesc(int(N), float(k), int(ensemble), int(seed), int(n_real), int(i), int(j), float(beta), int(path))
    o = OtocOpts()
    o.nvec = nvec
    o.state_seed = state_seed
    o.dtype = dtype
    o.krylov = default_krylov_opts(dtype)
    o.layout = -1
    o.autotune = 0
    if m is not None:
        o.krylov.m = m
    if tol is not None:
        o.krylov.tol = tol
    mean, sem = np.zeros(nt), np.zeros(nt)
    R = np.zeros((n_real, nt)) if rows else None
    st = EnsembleStats()
    dp = lambda a: None if a is None else a.ctypes.data_as(_dp)
    _check(_lib.syk_otoc_ensemble(ct.byref(d), dp(t), nt, ct.byref(o), dp(mean), dp(sem), dp(R), ct.byref(st),
                                  _stream(stream)))
    out = {f: getattr(st, f) for f, _ in EnsembleStats._fields_}
    return (mean, sem, out, R) if rows else (mean, sem, out)


def crossing_time(t, F, F0: float, F_err=None):
    """syk_crossing_time: (t*, sigma_t*); t* is nan when the curve never falls to F0."""
    t = np.ascontiguousarray(np.asarray(t, dtype=np.float64))
    F = np.ascontiguousarray(np.asarray(F, dtype=np.float64))
    if F.size != t.size:
        raise ValueError("t and F differ in length")
    e = None if F_err is None else np.ascontiguousarray(np.asarray(F_err, dtype=np.float64))
    if e is not None and e.size != t.size:
        raise ValueError("t and F_err differ in length")
    ts, err = ct.c_double(), ct.c_double()
    dp = lambda a: None if a is None else a.ctypes.data_as(_dp)
    _check(_lib.syk_crossing_time(dp(t), dp(F), dp(e), t.size, float(F0), ct.byref(ts), ct.byref(err)))
    return ts.value, err.value


def lyapunov_fit(N, tstar, tstar_err=None, method: int = FIT_SLOPE, terms: int = 1, dN: int = 8) -> dict:
    """syk_lyapunov_fit: lambda and the correction coefficients of Eq. (5) (method FIT_SLOPE:
    alpha1, alpha2) or Eq. (6) (FIT_GLOBAL: gamma0, gamma1, gamma2), their errors, chi2, dof
    and the fitted points (x, y, err)."""
    N = np.ascontiguousarray(np.asarray(N, dtype=np.float64))
    ts = np.ascontiguousarray(np.asarray(tstar, dtype=np.float64))
    if ts.size != N.size:
        raise ValueError("N and tstar differ in length")
    e = None if tstar_err is None else np.ascontiguousarray(np.asarray(tstar_err, dtype=np.float64))
    if e is not None and e.size != N.size:
        raise ValueError("N and tstar_err differ in length")
    cap = max(N.size * N.size, 1)
    px, py, pe = np.zeros(cap), np.zeros(cap), np.zeros(cap)
    o = FitOpts(int(method), int(terms), int(dN))
    r = FitResult()
    dp = lambda a: None if a is None else a.ctypes.data_as(_dp)
    _check(_lib.syk_lyapunov_fit(dp(N), dp(ts), dp(e), N.size, ct.byref(o), ct.byref(r), dp(px), dp(py), dp(pe), cap))
    out = {"lambda": r.lambda_, "lambda_err": r.lambda_err, "chi2": r.chi2, "n_points": r.n_points, "dof": r.dof}
    names = ("alpha1", "alpha2", None) if method == FIT_SLOPE else ("gamma0", "gamma1", "gamma2")
    for c, nm in enumerate(names):
        if nm:
            out[nm], out[nm + "_err"] = r.coef[c], r.coef_err[c]
    n = r.n_points
    out["points"] = (px[:n].copy(), py[:n].copy(), pe[:n].copy())
    return out


def workspace_bytes(N: int, m: int, dtype: int, nvec: int = 1) -> int:
    b = ct.c_uint64()
    _check(_lib.syk_workspace_bytes(N, m, dtype, nvec, ct.byref(b)))
    return b.value


def tridiag_expm(alpha, beta, z: complex) -> np.ndarray:
    """e^{z T} e_1 for the symmetric tridiagonal T (host computation in the library)."""
    a = np.ascontiguousarray(alpha, dtype=np.float64)
    b = np.ascontiguousarray(beta, dtype=np.float64)
    n = a.size
    cr = np.zeros(n)
    ci = np.zeros(n)
    z = complex(z)
    dp = lambda v: v.ctypes.data_as(_dp)
    _check(_lib.syk_tridiag_expm(n, dp(a), dp(b) if b.size else None, z.real, z.imag, dp(cr), dp(ci)))
    return cr + 1j * ci


def plan_describe(ham: Hamiltonian, block: int, dtype: int, layout: int = -1) -> dict:
    """Launch plan of the tiled apply_H kernel (host-only)."""
    d = PlanDesc()
    _check(_lib.syk_plan_describe(ham.handle, block, dtype, layout, ct.byref(d)))
    return {f: getattr(d, f) for f, _ in PlanDesc._fields_}


def plan_blocks(ham: Hamiltonian, block: int, dtype: int, layout: int = -1):
    """Control blocks of the tiled apply_H plan (host-only): uint32 array (blocks, 64)."""
    n = ct.c_size_t()
    _check(_lib.syk_plan_blocks(ham.handle, block, dtype, layout, None, 0, ct.byref(n)))
    out = np.zeros(n.value, dtype=np.uint32)
    _check(_lib.syk_plan_blocks(ham.handle, block, dtype, layout, out.ctypes.data, n.value, ct.byref(n)))
    return out.reshape(-1, 64)


def autotune(ham: Hamiltonian, dtype: int, stream=None):
    """Time the tiled apply_H variants on this Hamiltonian.  Returns (chosen variant,
    per-variant ms per apply, -1 where skipped)."""
    v = ct.c_int(-1)
    ms = (ct.c_float * 64)()
    _check(_lib.syk_autotune(ham.handle, dtype, ct.byref(v), ms, 64, _stream(stream)))
    return v.value, [round(float(t), 4) for t in ms if t != -1.0]


def select_variant(ham: Hamiltonian, dtype: int, variant: int):
    """Pin the tiled apply_H variant for this handle (tests, reproducible timings)."""
    _check(_lib.syk_select_variant(ham.handle, dtype, variant))


def kernel_revision() -> str:
    return _lib.syk_kernel_revision().decode()


def release_workspace():
    _check(_lib.syk_release_workspace())


class Engine:
    """Request engine (syk_engine_*): continuous batching of OTOC requests on the current
    device.  submit() returns an id; poll() returns finished results as dicts."""

    def __init__(self, budget_bytes: int = 0, max_active: int = 4, max_bypass: int = 8):
        o = EngineOpts(budget_bytes, max_active, max_bypass)
        h = ct.c_void_p()
        _check(_lib.syk_engine_create(ct.byref(o), ct.byref(h)))
        self._h = h
        self._nt = {}

    def submit(self, N: int, k: float, seed: int, beta: float, t, i: int = None, j: int = None, nvec: int = 1,
               state_seed: int = 0, dtype: int = C64, m: int = 30, m_min: int = 0, tol: float = 0.0,
               precision_check: bool = False) -> int:
        t = np.ascontiguousarray(np.asarray(t, dtype=np.float64))
        r = Request(N, float(k), seed, N - 1 if i is None else i, N - 2 if j is None else j, float(beta),
                    t.ctypes.data_as(_dp), t.size, nvec, state_seed, dtype, m, m_min, float(tol),
                    1 if precision_check else 0)
        rid = ct.c_uint64()
        _check(_lib.syk_engine_submit(self._h, ct.byref(r), ct.byref(rid)))
        self._nt[rid.value] = t.size
        return rid.value

    def poll(self, wait_ms: int = -1):
        """One finished request as a dict (F_raw, F_norm, F_imag, id, status, m_used,
        footprint_bytes, t_submit, t_start, t_end, stats), or None if none finished."""
        cap = max(self._nt.values(), default=1)
        raw, nrm, im = np.zeros(cap), np.zeros(cap), np.zeros(cap)
        info = ResultInfo()
        dp = lambda a: a.ctypes.data_as(_dp)
        st = _lib.syk_engine_poll(self._h, wait_ms, ct.byref(info), dp(raw), dp(nrm), dp(im), cap)
        if st == EAGAIN:
            return None
        _check(st)
        self._nt.pop(info.id, None)
        out = {f: getattr(info, f) for f, _ in ResultInfo._fields_ if f != "stats"}
        out["stats"] = {f: getattr(info.stats, f) for f, _ in OtocStats._fields_}
        out["F_raw"], out["F_norm"], out["F_imag"] = raw[:info.nt], nrm[:info.nt], im[:info.nt]
        return out

    def cancel(self, rid: int):
        _check(_lib.syk_engine_cancel(self._h, rid))

    def stats(self) -> dict:
        s = EngineStats()
        _check(_lib.syk_engine_get_stats(self._h, ct.byref(s)))
        return {f: getattr(s, f) for f, _ in EngineStats._fields_}

    def close(self):
        if self._h:
            _check(_lib.syk_engine_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Operator:
    """General spin operator on L qubits: a sum of Pauli strings c X^x Z^z (Z applied
    first) held by the library (syk_op_*); products, sums and adjoints are exact."""

    def __init__(self, L: int, x=(), z=(), c=(), _handle=None):
        if _handle is not None:
            self._h = _handle
            self.L = L
            return
        x = np.ascontiguousarray(np.asarray(x, dtype=np.uint64))
        z = np.ascontiguousarray(np.asarray(z, dtype=np.uint64))
        c = np.asarray(c, dtype=np.complex128)
        cr = np.ascontiguousarray(c.real)
        ci = np.ascontiguousarray(c.imag)
        h = _vp()
        _check(_lib.syk_op_create(L, x.size, x.ctypes.data, z.ctypes.data, cr.ctypes.data_as(_dp),
                                  ci.ctypes.data_as(_dp), ct.byref(h)))
        self._h = h
        self.L = L

    def _new(self, fn, *args):
        h = _vp()
        _check(fn(*args, ct.byref(h)))
        return Operator(self.L, _handle=h)

    def __matmul__(self, other):
        return self._new(_lib.syk_op_product, self._h, other._h)

    def __add__(self, other):
        return self.combine(other, 1.0, 1.0)

    def __sub__(self, other):
        return self.combine(other, 1.0, -1.0)

    def combine(self, other, alpha: complex, beta: complex):
        alpha, beta = complex(alpha), complex(beta)
        return self._new(_lib.syk_op_sum, self._h, other._h, alpha.real, alpha.imag, beta.real, beta.imag)

    def adjoint(self):
        return self._new(_lib.syk_op_adjoint, self._h)

    def terms(self):
        """(x, z, c) arrays sorted by (x, z)."""
        n = ct.c_size_t()
        _check(_lib.syk_op_get_terms(self._h, 0, ct.byref(n), None, None, None, None))
        k = n.value
        x = np.zeros(k, dtype=np.uint64)
        z = np.zeros(k, dtype=np.uint64)
        cr, ci = np.zeros(k), np.zeros(k)
        _check(_lib.syk_op_get_terms(self._h, k, ct.byref(n), x.ctypes.data, z.ctypes.data,
                                     cr.ctypes.data_as(_dp), ci.ctypes.data_as(_dp)))
        return x, z, cr + 1j * ci

    def is_hermitian(self) -> bool:
        v = ct.c_int()
        _check(_lib.syk_op_is_hermitian(self._h, ct.byref(v)))
        return bool(v.value)

    def to_hamiltonian(self) -> "Hamiltonian":
        """A handle for apply_H (either block) and, if Hermitian, krylov_expm."""
        h = _vp()
        _check(_lib.syk_op_to_hamiltonian(self._h, ct.byref(h)))
        ham = Hamiltonian.__new__(Hamiltonian)
        ham._h = h
        return ham

    def close(self):
        if getattr(self, "_h", None):
            _check(_lib.syk_op_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
