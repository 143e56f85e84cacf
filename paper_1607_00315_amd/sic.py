"""Python binding of the sic C-ABI (``include/sic.h``, ``include/sic_steps.h``).

Argument marshalling only: every step runs in ``libsic.so``. The library must
have been built (``python -m paper_1607_00315_amd.build``); loading fails
loudly otherwise. Arrays on the host are numpy arrays; device arrays may be
passed as torch tensors (their data pointer is handed to the library, which
detects host or device memory itself).
"""

from __future__ import annotations

import ctypes as ct
import os
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsic.so")

SIC_OK, SIC_EINVAL, SIC_ENONFINITE, SIC_ENOTPD, SIC_ENOMEM = 0, -1, -2, -3, -4
SIC_ENOCONV, SIC_EHIP, SIC_ECANCELED, SIC_ETOOBIG, SIC_EINTERNAL = -5, -6, -7, -8, -9
SIC_FP64, SIC_MIXED = 0, 1
SIC_X_F64, SIC_X_F32, SIC_X_BF16 = 0, 1, 2
FLAG_NO_MULTILEVEL, FLAG_FINAL_KKT, FLAG_VERBOSE, FLAG_NO_CERTIFY, FLAG_CLUSTER = 1, 2, 4, 8, 16
FLAG_CONTINUATION, FLAG_NO_WARM_CG, FLAG_NO_S_CACHE = 32, 64, 128


class SicError(RuntimeError):
    def __init__(self, code, where, message=""):
        super().__init__(f"{where}: {strerror(code)} ({code}) {message}".strip())
        self.code = code


class CSR(ct.Structure):
    _fields_ = [("n", ct.c_int64), ("nnz", ct.c_int64), ("rowptr", ct.POINTER(ct.c_int64)),
                ("col", ct.POINTER(ct.c_int32)), ("val", ct.POINTER(ct.c_double))]


class TraceEntry(ct.Structure):
    _fields_ = [("seconds", ct.c_double), ("objective", ct.c_double), ("kkt_max", ct.c_double),
                ("kkt_rel_l1", ct.c_double), ("nnz", ct.c_int64), ("cycle", ct.c_int32),
                ("levels", ct.c_int32)]


class Options(ct.Structure):
    _fields_ = [("device", ct.c_int), ("hbm_budget", ct.c_size_t), ("precision", ct.c_int),
                ("block", ct.c_int), ("cg_tol_I", ct.c_double), ("cg_tol_N", ct.c_double),
                ("cg_max_iter", ct.c_int), ("cd_tol", ct.c_double), ("cd_max_sweeps", ct.c_int),
                ("cd_hessian_max", ct.c_int), ("pcd_min_coords", ct.c_int),
                ("ls_max_trials", ct.c_int), ("max_cycles", ct.c_int), ("stream", ct.c_void_p),
                ("flags", ct.c_uint64), ("trace", ct.POINTER(TraceEntry)), ("trace_cap", ct.c_int)]


class Info(ct.Structure):
    _fields_ = [("objective", ct.c_double), ("kkt_max", ct.c_double), ("kkt_rel_l1", ct.c_double),
                ("nnz", ct.c_int64), ("max_nnz", ct.c_int64), ("cycles", ct.c_int),
                ("sweeps", ct.c_int), ("blocks", ct.c_int64), ("cg_iterations", ct.c_int64),
                ("cd_sweeps", ct.c_int64), ("seconds", ct.c_double), ("status", ct.c_int),
                ("trace_len", ct.c_int)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class ProblemSpec(ct.Structure):
    _fields_ = [("X", ct.c_void_p), ("n", ct.c_int64), ("m", ct.c_int64), ("x_dtype", ct.c_int),
                ("lambda_", ct.c_double), ("tol", ct.c_double), ("A0", ct.POINTER(CSR)),
                ("lambda_path", ct.POINTER(ct.c_double)), ("n_lambda", ct.c_int)]


class ServerOptions(ct.Structure):
    _fields_ = [("slots", ct.c_int), ("hbm_budget", ct.c_size_t), ("solver", Options),
                ("device", ct.c_int)]


class RequestTimes(ct.Structure):
    _fields_ = [("submitted", ct.c_double), ("admitted", ct.c_double), ("finished", ct.c_double),
                ("footprint", ct.c_size_t), ("slot", ct.c_int)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class BlockResult(ct.Structure):
    _fields_ = [("E", ct.c_int64), ("n_neighbors", ct.c_int64), ("n_level_nbrs", ct.c_int64),
                ("n_coords", ct.c_int64), ("cg_iterations_I", ct.c_int),
                ("cg_iterations_N", ct.c_int), ("cd_sweeps", ct.c_int),
                ("cd_last_max_mu", ct.c_double), ("alpha", ct.c_double), ("dF", ct.c_double),
                ("trials", ct.c_int), ("nnz_after", ct.c_int64)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib = None

_P = ct.c_void_p
_PP = ct.POINTER(ct.c_void_p)
_i64p = ct.POINTER(ct.c_int64)
_i32p = ct.POINTER(ct.c_int32)
_dp = ct.POINTER(ct.c_double)

# name -> (restype, argtypes); the exported entry points of include/*.h
SIGNATURES = {
    "sic_options_default": (None, [ct.POINTER(Options)]),
    "sic_create": (ct.c_int, [_PP, ct.POINTER(Options)]),
    "sic_destroy": (None, [_P]),
    "sic_solve": (ct.c_int, [_P, ct.c_void_p, ct.c_int64, ct.c_int64, ct.c_double, ct.c_double,
                             ct.POINTER(CSR), ct.POINTER(Info)]),
    "sic_solve_batch": (ct.c_int, [_P, ct.c_int, ct.POINTER(ProblemSpec), ct.POINTER(CSR),
                                   ct.POINTER(Info)]),
    "sic_csr_free": (None, [ct.POINTER(CSR)]),
    "sic_strerror": (ct.c_char_p, [ct.c_int]),
    "sic_last_error": (ct.c_char_p, []),
    "sic_prob_create": (ct.c_int, [_P, ct.c_void_p, ct.c_int64, ct.c_int64, ct.c_double, _PP]),
    "sic_prob_destroy": (None, [_P]),
    "sic_prob_set_A": (ct.c_int, [_P, ct.POINTER(CSR), ct.c_double]),
    "sic_prob_get_A": (ct.c_int, [_P, ct.POINTER(CSR)]),
    "sic_prob_objective": (ct.c_double, [_P]),
    "sic_step_cov_block": (ct.c_int, [_P, ct.c_int64, ct.c_int, _dp]),
    "sic_step_cov_pairs": (ct.c_int, [_P, _i32p, _i32p, ct.c_int64, _dp]),
    "sic_step_cov_block_low": (ct.c_int, [_P, ct.c_int64, ct.c_int, ct.c_int, _dp]),
    "sic_step_inverse_columns": (ct.c_int, [_P, _i32p, ct.c_int, ct.c_double, ct.c_int, _dp,
                                            ct.POINTER(ct.c_int), _dp]),
    "sic_step_inverse_columns_noalloc": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_void_p,
                                                    ct.c_int64, ct.c_int64, ct.c_void_p,
                                                    ct.c_int, ct.c_double, ct.c_int,
                                                    ct.c_void_p, ct.c_void_p,
                                                    ct.POINTER(ct.c_int), _dp]),
    "sic_step_inverse_columns_noalloc_limit": (ct.c_size_t, [ct.c_int64, ct.c_int64, ct.c_int]),
    "sic_step_set_level": (ct.c_int, [_P, _i64p, ct.c_int64]),
    "sic_cluster_order": (ct.c_int, [ct.c_int64, _i64p, ct.c_int64, ct.c_int, _i32p]),
    "sic_step_block": (ct.c_int, [_P, ct.c_int64, ct.c_int, ct.c_int, ct.c_double, ct.c_double,
                                  ct.POINTER(BlockResult)]),
    "sic_step_last_block": (ct.c_int, [_P, _i64p, _i32p, _dp, _i32p, _i32p, _i32p, _dp, _dp]),
    "sic_step_sweep": (ct.c_int, [_P, ct.c_int, ct.c_double, ct.c_double, _dp, _dp]),
    "sic_step_kkt": (ct.c_int, [_P, ct.c_double, _dp, _dp]),
    "sic_step_cd": (ct.c_int, [_P, ct.c_int, ct.c_int, _dp, _i64p, _i32p, _dp, _dp, ct.c_double,
                               ct.c_int, ct.c_double, _dp, _dp]),
    "sic_step_linesearch": (ct.c_int, [_P, ct.c_int, ct.c_int, _dp, _i64p, _i32p, _dp, _dp, _dp,
                                       ct.c_double, _dp, _dp, ct.POINTER(ct.c_int), _dp,
                                       ct.c_int]),
    "sic_server_options_default": (None, [ct.POINTER(ServerOptions)]),
    "sic_server_create": (ct.c_int, [_PP, ct.POINTER(ServerOptions)]),
    "sic_server_footprint": (ct.c_size_t, [_P, ct.POINTER(ProblemSpec)]),
    "sic_server_submit": (ct.c_int, [_P, ct.POINTER(ProblemSpec), ct.POINTER(ct.c_uint64)]),
    "sic_server_wait": (ct.c_int, [_P, ct.c_uint64, ct.c_double, ct.POINTER(CSR),
                                   ct.POINTER(Info), ct.POINTER(RequestTimes)]),
    "sic_server_cancel": (ct.c_int, [_P, ct.c_uint64]),
    "sic_request_results": (ct.c_int, [ct.POINTER(ProblemSpec)]),
    "sic_server_status": (None, [_P, ct.POINTER(ct.c_int), ct.POINTER(ct.c_int),
                                 ct.POINTER(ct.c_int), ct.POINTER(ct.c_size_t)]),
    "sic_server_destroy": (None, [_P]),
    "sic_profile_enable": (None, [ct.c_int]),
    "sic_profile_reset": (None, []),
    "sic_profile_select": (None, [ct.c_uint32]),
    "sic_profile_read": (ct.c_int, [ct.c_int, _i64p, _dp, _dp, _dp]),
    "sic_profile_kernel_name": (ct.c_char_p, [ct.c_int]),
    "sic_hierarchy": (ct.c_int, [ct.c_int64, _i64p, ct.c_int64, _i64p, _dp, ct.c_int64, _i64p,
                                 _i64p, _i64p, ct.POINTER(ct.c_int)]),
}


def lib():
    """Load libsic.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        # PyTorch ships its own HIP runtime (same soname as the system one).
        # Loading it first makes libsic.so bind to that runtime, so device
        # pointers and streams from torch are valid here and a single HIP
        # runtime lives in the process.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1607_00315_amd.build` (no CPU fallback exists)")
        L = ct.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def strerror(code: int) -> str:
    return lib().sic_strerror(code).decode()


def last_error() -> str:
    return lib().sic_last_error().decode()


def _check(code, where, ok=(SIC_OK,)):
    if code not in ok:
        raise SicError(code, where, last_error())
    return code


def _ptr(a, t):
    return a.ctypes.data_as(ct.POINTER(t))


def _data_ptr(X):
    """Raw pointer of a numpy array or torch tensor (float64, C-contiguous)."""
    if hasattr(X, "data_ptr"):
        if not X.is_contiguous():
            raise ValueError("X must be contiguous")
        return ct.c_void_p(X.data_ptr())
    if not (isinstance(X, np.ndarray) and X.flags["C_CONTIGUOUS"]):
        raise ValueError("X must be a C-contiguous numpy array or a torch tensor")
    return ct.c_void_p(X.ctypes.data)


def _csr_to_numpy(c: CSR):
    n, nnz = c.n, c.nnz
    rowptr = np.ctypeslib.as_array(c.rowptr, shape=(n + 1,)).copy()
    col = np.ctypeslib.as_array(c.col, shape=(max(nnz, 1),))[:nnz].copy()
    val = np.ctypeslib.as_array(c.val, shape=(max(nnz, 1),))[:nnz].copy()
    lib().sic_csr_free(ct.byref(c))
    return rowptr, col, val


def csr_from_arrays(rowptr, col, val):
    """Build a CSR view over numpy arrays (kept alive by the returned tuple)."""
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    val = np.ascontiguousarray(val, dtype=np.float64)
    c = CSR(rowptr.size - 1, val.size, _ptr(rowptr, ct.c_int64), _ptr(col, ct.c_int32),
            _ptr(val, ct.c_double))
    return c, (rowptr, col, val)


def options(**kw) -> Options:
    o = Options()
    lib().sic_options_default(ct.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def _fill_spec(s: ProblemSpec, p: dict, keep: list) -> int:
    """Fill a sic_problem from a dict; returns its result count. Arrays that
    must outlive the call are appended to ``keep``."""
    X = p["X"]
    s.X = _data_ptr(X).value
    s.n, s.m = X.shape[1], X.shape[0]
    s.x_dtype = p.get("x_dtype", SIC_X_F64)
    s.tol = p["tol"]
    if p.get("A0") is not None:
        c, arrs = csr_from_arrays(*p["A0"])
        keep.extend([c, arrs])
        s.A0 = ct.pointer(c)
    path = p.get("lambda_path")
    if path is not None:
        arr = np.ascontiguousarray(path, dtype=np.float64)
        keep.append(arr)
        s.lambda_path = _ptr(arr, ct.c_double)
        s.n_lambda = arr.size
        return arr.size
    s.lambda_ = p["lam"]
    s.n_lambda = 0
    return 1


class Context:
    """One library context on one GPU: its two HIP streams, device workspace and
    the last solve's problem storage (kept for the next solve; close() frees it)."""

    def __init__(self, trace_cap: int = 0, **opts):
        o = options(**opts)
        self._trace = None
        if trace_cap:
            self._trace = (TraceEntry * trace_cap)()
            o.trace = ct.cast(self._trace, ct.POINTER(TraceEntry))
            o.trace_cap = trace_cap
        self._opts = o
        self._probs = weakref.WeakSet()
        h = ct.c_void_p()
        _check(lib().sic_create(ct.byref(h), ct.byref(o)), "sic_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            for p in list(self._probs):
                p.close()
            lib().sic_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, X, lam: float, tol: float):
        """Solve one problem; returns ((rowptr, col, val), info dict, trace list)."""
        n = X.shape[1]
        m = X.shape[0]
        out = CSR()
        info = Info()
        code = lib().sic_solve(self.h, _data_ptr(X), n, m, float(lam), float(tol),
                               ct.byref(out), ct.byref(info))
        _check(code, "sic_solve", ok=(SIC_OK, SIC_ENOCONV))
        A = _csr_to_numpy(out)
        return A, info.as_dict(), self.trace(info.trace_len)

    def solve_batch(self, problems):
        """problems: list of dicts with X, lam or lambda_path, tol, optional x_dtype, A0."""
        count = len(problems)
        specs = (ProblemSpec * count)()
        keep = []
        slots = 0
        for k, p in enumerate(problems):
            slots += _fill_spec(specs[k], p, keep)
        outs = (CSR * slots)()
        infos = (Info * slots)()
        code = lib().sic_solve_batch(self.h, count, specs, outs, infos)
        results = [(_csr_to_numpy(outs[i]) if outs[i].rowptr else None, infos[i].as_dict())
                   for i in range(slots)]
        return code, results

    def trace(self, length):
        if self._trace is None:
            return []
        return [dict(seconds=e.seconds, objective=e.objective, kkt_max=e.kkt_max,
                     kkt_rel_l1=e.kkt_rel_l1, nnz=e.nnz, cycle=e.cycle, levels=e.levels)
                for e in self._trace[:length]]


class Server:
    """The serving loop of include/sic_serve.h: submit problems, wait for them.

    ``slots`` problems run concurrently (one HIP stream and host worker each);
    ``hbm_budget`` bounds their device memory together (0: 80% of free).
    Solver options are passed as keyword arguments, as for :class:`Context`.
    """

    def __init__(self, slots: int = 4, hbm_budget: int = 0, device: int = 0, **opts):
        o = ServerOptions()
        lib().sic_server_options_default(ct.byref(o))
        o.slots, o.hbm_budget, o.device = slots, hbm_budget, device
        so = options(**opts)
        o.solver = so
        h = ct.c_void_p()
        _check(lib().sic_server_create(ct.byref(h), ct.byref(o)), "sic_server_create")
        self.h = h
        self._live = {}   # ticket -> (spec, arrays the request reads, result count)

    def footprint(self, problem: dict) -> int:
        s = ProblemSpec()
        keep = []
        _fill_spec(s, problem, keep)
        return lib().sic_server_footprint(self.h, ct.byref(s))

    def submit(self, problem: dict) -> int:
        """Queue a problem (dict as for Context.solve_batch); returns its ticket.
        X is read when the request is admitted: it is kept alive here until
        :meth:`wait` returns the request."""
        s = ProblemSpec()
        keep = [problem["X"]]
        nres = _fill_spec(s, problem, keep)
        t = ct.c_uint64()
        _check(lib().sic_server_submit(self.h, ct.byref(s), ct.byref(t)), "sic_server_submit")
        self._live[t.value] = (s, keep, nres)
        return t.value

    def wait(self, ticket: int, timeout: float = -1.0):
        """Returns (status, [(rowptr, col, val), ...], [info dict, ...], times dict),
        or None on timeout."""
        _, _, nres = self._live[ticket]
        outs = (CSR * nres)()
        infos = (Info * nres)()
        times = RequestTimes()
        code = lib().sic_server_wait(self.h, ticket, float(timeout), outs, infos, ct.byref(times))
        if code == 1:
            return None
        if code == SIC_EINVAL and ticket not in self._live:
            raise SicError(code, "sic_server_wait")
        del self._live[ticket]
        results = []
        for i in range(nres):
            results.append(_csr_to_numpy(outs[i]) if outs[i].rowptr else None)
        return code, results, [infos[i].as_dict() for i in range(nres)], times.as_dict()

    def cancel(self, ticket: int) -> bool:
        return lib().sic_server_cancel(self.h, ticket) == SIC_OK

    def status(self):
        q, r, d = ct.c_int(), ct.c_int(), ct.c_int()
        held = ct.c_size_t()
        lib().sic_server_status(self.h, ct.byref(q), ct.byref(r), ct.byref(d), ct.byref(held))
        return dict(queued=q.value, running=r.value, done=d.value, held_bytes=held.value)

    def close(self):
        if getattr(self, "h", None):
            lib().sic_server_destroy(self.h)
            self.h = None
            self._live.clear()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Prob:
    """Device-resident problem for the step-level entry points."""

    def __init__(self, ctx: Context, X, lam: float):
        self.ctx = ctx
        self.n, self.m = X.shape[1], X.shape[0]
        h = ct.c_void_p()
        _check(lib().sic_prob_create(ctx.h, _data_ptr(X), self.n, self.m, float(lam), ct.byref(h)),
               "sic_prob_create")
        self.h = h
        ctx._probs.add(self)

    def close(self):
        if getattr(self, "h", None):
            lib().sic_prob_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_A(self, rowptr, col, val, objective=float("nan")):
        c, keep = csr_from_arrays(rowptr, col, val)
        _check(lib().sic_prob_set_A(self.h, ct.byref(c), float(objective)), "sic_prob_set_A")

    def get_A(self):
        out = CSR()
        _check(lib().sic_prob_get_A(self.h, ct.byref(out)), "sic_prob_get_A")
        return _csr_to_numpy(out)

    def objective(self):
        return lib().sic_prob_objective(self.h)

    def cov_block(self, j0, b):
        out = np.empty((self.n, b))
        _check(lib().sic_step_cov_block(self.h, j0, b, _ptr(out, ct.c_double)), "cov_block")
        return out

    def cov_block_low(self, j0, b, x_dtype):
        out = np.empty((self.n, b))
        _check(lib().sic_step_cov_block_low(self.h, j0, b, int(x_dtype), _ptr(out, ct.c_double)),
               "cov_block_low")
        return out

    def cov_pairs(self, rows, cols):
        rows = np.ascontiguousarray(rows, dtype=np.int32)
        cols = np.ascontiguousarray(cols, dtype=np.int32)
        out = np.empty(rows.size)
        _check(lib().sic_step_cov_pairs(self.h, _ptr(rows, ct.c_int32), _ptr(cols, ct.c_int32),
                                        rows.size, _ptr(out, ct.c_double)), "cov_pairs")
        return out

    def inverse_columns(self, cols, tol=1e-12, max_iter=5000):
        cols = np.ascontiguousarray(cols, dtype=np.int32)
        out = np.empty((self.n, cols.size))
        it = ct.c_int()
        res = ct.c_double()
        _check(lib().sic_step_inverse_columns(self.h, _ptr(cols, ct.c_int32), cols.size, tol,
                                              max_iter, _ptr(out, ct.c_double), ct.byref(it),
                                              ct.byref(res)), "inverse_columns")
        return out, it.value, res.value

    def set_level(self, keys):
        keys = np.ascontiguousarray(keys, dtype=np.int64)
        _check(lib().sic_step_set_level(self.h, _ptr(keys, ct.c_int64), keys.size), "set_level")

    def block(self, j0, b, level=0, tol_I=0.0, tol_N=0.0):
        r = BlockResult()
        _check(lib().sic_step_block(self.h, j0, b, level, tol_I, tol_N, ct.byref(r)), "block")
        return r.as_dict()

    def last_block(self, res, b):
        E, nN, nc = res["E"], res["n_neighbors"], res["n_coords"]
        jp = b + nN
        colptr = np.empty(b + 1, dtype=np.int64)
        rows = np.empty(max(E, 1), dtype=np.int32)
        g = np.empty(max(E, 1))
        nbrs = np.empty(max(nN, 1), dtype=np.int32)
        cr = np.empty(max(nc, 1), dtype=np.int32)
        cc = np.empty(max(nc, 1), dtype=np.int32)
        d = np.empty(max(nc, 1))
        wjj = np.empty((jp, jp))
        _check(lib().sic_step_last_block(self.h, _ptr(colptr, ct.c_int64), _ptr(rows, ct.c_int32),
                                         _ptr(g, ct.c_double), _ptr(nbrs, ct.c_int32),
                                         _ptr(cr, ct.c_int32), _ptr(cc, ct.c_int32),
                                         _ptr(d, ct.c_double), _ptr(wjj, ct.c_double)),
               "last_block")
        return dict(colptr=colptr, rows=rows[:E], g=g[:E], nbrs=nbrs[:nN], coord_rows=cr[:nc],
                    coord_cols=cc[:nc], delta=d[:nc], wjj=wjj)

    def sweep(self, level=0, tol_I=0.0, tol_N=0.0):
        km, kl = ct.c_double(), ct.c_double()
        _check(lib().sic_step_sweep(self.h, level, tol_I, tol_N, ct.byref(km), ct.byref(kl)),
               "sweep")
        return km.value, kl.value

    def kkt(self, tol_cg=1e-11):
        km, kl = ct.c_double(), ct.c_double()
        _check(lib().sic_step_kkt(self.h, tol_cg, ct.byref(km), ct.byref(kl)), "kkt")
        return km.value, kl.value


def inverse_columns_noalloc(rowptr, col, val, cols, W, tol=1e-12, max_iter=5000, stream=None):
    """W = A^{-1} E_cols with no allocation inside the library.

    rowptr (int64), col (int32), val (float64): A as a full symmetric CSR;
    cols (int32, k); W (float64, n x k, written): all torch tensors on the
    current device. stream: a torch.cuda.Stream (default: the current one).
    Returns (iterations, max relative residual)."""
    import torch
    n = rowptr.numel() - 1
    k = cols.numel()
    for t, dt in ((rowptr, torch.int64), (col, torch.int32), (val, torch.float64),
                  (cols, torch.int32), (W, torch.float64)):
        if not t.is_cuda or t.dtype != dt or not t.is_contiguous():
            raise ValueError("inverse_columns_noalloc takes contiguous device tensors "
                             "(int64 rowptr, int32 col and cols, float64 val and W)")
    if W.shape != (n, k):
        raise ValueError(f"W must be {n} x {k}")
    if stream is None:
        stream = torch.cuda.current_stream()
    it = ct.c_int()
    res = ct.c_double()
    _check(lib().sic_step_inverse_columns_noalloc(
        rowptr.data_ptr(), col.data_ptr(), val.data_ptr(), n, col.numel(), cols.data_ptr(), k,
        tol, max_iter, W.data_ptr(), stream.cuda_stream, ct.byref(it), ct.byref(res)),
        "inverse_columns_noalloc")
    return it.value, res.value


def inverse_columns_noalloc_limit(n, nnz, k):
    """Scratch bytes the no-allocation solve needs for n x k with nnz entries
    (0: does not fit)."""
    return lib().sic_step_inverse_columns_noalloc_limit(n, nnz, k)


def step_cd(ctx: Context, wjj, b, cptr, cp, S, A, lam, max_sweeps=20, tol=1e-4):
    wjj = np.ascontiguousarray(wjj, dtype=np.float64)
    cptr = np.ascontiguousarray(cptr, dtype=np.int64)
    cp = np.ascontiguousarray(cp, dtype=np.int32)
    S = np.ascontiguousarray(S, dtype=np.float64)
    A = np.ascontiguousarray(A, dtype=np.float64)
    nc = int(cptr[-1])
    out = np.empty(max(nc, 1))
    st = np.empty(7)
    _check(lib().sic_step_cd(ctx.h, wjj.shape[0], b, _ptr(wjj, ct.c_double),
                             _ptr(cptr, ct.c_int64), _ptr(cp, ct.c_int32), _ptr(S, ct.c_double),
                             _ptr(A, ct.c_double), float(lam), int(max_sweeps), float(tol),
                             _ptr(out, ct.c_double), _ptr(st, ct.c_double)), "step_cd")
    return out[:nc], st


def step_linesearch(ctx: Context, wjj, b, cptr, cp, S, A, delta, lam, n_alpha=0):
    wjj = np.ascontiguousarray(wjj, dtype=np.float64)
    cptr = np.ascontiguousarray(cptr, dtype=np.int64)
    cp = np.ascontiguousarray(cp, dtype=np.int32)
    S = np.ascontiguousarray(S, dtype=np.float64)
    A = np.ascontiguousarray(A, dtype=np.float64)
    delta = np.ascontiguousarray(delta, dtype=np.float64)
    alpha, dF = ct.c_double(), ct.c_double()
    trials = ct.c_int()
    ld = np.empty(max(n_alpha, 1))
    _check(lib().sic_step_linesearch(ctx.h, wjj.shape[0], b, _ptr(wjj, ct.c_double),
                                     _ptr(cptr, ct.c_int64), _ptr(cp, ct.c_int32),
                                     _ptr(S, ct.c_double), _ptr(A, ct.c_double),
                                     _ptr(delta, ct.c_double), float(lam), ct.byref(alpha),
                                     ct.byref(dF), ct.byref(trials), _ptr(ld, ct.c_double),
                                     int(n_alpha)), "step_linesearch")
    return alpha.value, dF.value, trials.value, ld[:n_alpha]


def cluster_order(n, keys, b):
    """The clustered block order of the graph of pair keys (host computation)."""
    keys = np.ascontiguousarray(keys, dtype=np.int64)
    out = np.empty(n, dtype=np.int32)
    _check(lib().sic_cluster_order(n, _ptr(keys, ct.c_int64), keys.size, b,
                                   _ptr(out, ct.c_int32)), "cluster_order")
    return out


def hierarchy(n, supp_keys, free_keys, free_absg):
    s = np.ascontiguousarray(supp_keys, dtype=np.int64)
    f = np.ascontiguousarray(free_keys, dtype=np.int64)
    g = np.ascontiguousarray(free_absg, dtype=np.float64)
    rank = np.empty(max(s.size + f.size, 1), dtype=np.int64)
    rlen = ct.c_int64()
    sizes = np.empty(64, dtype=np.int64)
    nl = ct.c_int()
    _check(lib().sic_hierarchy(n, _ptr(s, ct.c_int64), s.size, _ptr(f, ct.c_int64),
                               _ptr(g, ct.c_double), f.size, _ptr(rank, ct.c_int64),
                               ct.byref(rlen), _ptr(sizes, ct.c_int64), ct.byref(nl)), "hierarchy")
    return rank[:rlen.value], list(sizes[:nl.value])


KERNEL_CLASSES = 14


def profile_enable(on=True):
    lib().sic_profile_enable(1 if on else 0)


def profile_reset():
    lib().sic_profile_reset()


def profile_select(names=None):
    """Time only the named kernel classes (None: every class)."""
    if names is None:
        mask = (1 << KERNEL_CLASSES) - 1
    else:
        index = {lib().sic_profile_kernel_name(k).decode(): k for k in range(KERNEL_CLASSES)}
        mask = 0
        for nm in names:
            if nm not in index:
                raise ValueError(f"unknown kernel class {nm!r}")
            mask |= 1 << index[nm]
    lib().sic_profile_select(mask)


def profile_read():
    """{kernel name: dict(launches, ms, bytes, flops)} since the last reset."""
    out = {}
    for k in range(KERNEL_CLASSES):
        n = ct.c_int64()
        ms, by, fl = ct.c_double(), ct.c_double(), ct.c_double()
        _check(lib().sic_profile_read(k, ct.byref(n), ct.byref(ms), ct.byref(by), ct.byref(fl)),
               "profile_read")
        out[lib().sic_profile_kernel_name(k).decode()] = dict(
            launches=n.value, ms=ms.value, bytes=by.value, flops=fl.value)
    return out
