"""ctypes binding of libtsylv.so (the C ABI declared in include/tsylv.h).

Argument marshalling only: every step of every solve runs in the library's
HIP kernels.  torch supplies device memory (the arena and the tensors) and
the stream.  Loading fails loudly when the library has not been built.

Tensors passed in are float64 CUDA(HIP) tensors of shape (rows, cols, p)
whose memory is frontal-slice major and column-major inside a slice, i.e.
``T.permute(2, 1, 0).is_contiguous()``; :func:`to_device` makes one from a
Fortran-ordered numpy array and :func:`to_host` brings it back.
"""

import ctypes
import os
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtsylv.so")

FP64, FP32, BF16 = 0, 1, 2
GMRES, FOM, TBA, TBS, GMRES_BATCHED, AUTO = 0, 1, 2, 3, 4, 5
APPLY = -1

STATUS = {0: "OK", 1: "NOT_CONVERGED", 2: "PENDING", -1: "EINVAL", -2: "ENOMEM",
          -3: "EBREAKDOWN", -4: "ESINGULAR", -5: "EHIP", -6: "ECANCELLED", -7: "ESCRATCH"}


class Opts(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int), ("max_cycles", ctypes.c_int), ("tol", ctypes.c_double),
                ("x0_given", ctypes.c_int), ("prec", ctypes.c_int), ("refine", ctypes.c_int),
                ("inner_m", ctypes.c_int), ("inner_tol", ctypes.c_double),
                ("max_outer", ctypes.c_int), ("res_hist", ctypes.POINTER(ctypes.c_double)),
                ("res_hist_cap", ctypes.c_int)]


class Info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("steps", ctypes.c_int), ("cycles", ctypes.c_int),
                ("outer", ctypes.c_int), ("relres_true", ctypes.c_double),
                ("relres_est", ctypes.c_double), ("seconds", ctypes.c_double),
                ("res_hist_len", ctypes.c_int), ("fom_fallback", ctypes.c_int)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class KStat(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("total_ms", ctypes.c_double)]


K_APPLY, K_ORTHO, K_XFORM, K_APPLY_LOW = 0, 1, 2, 3


class Request(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int), ("n", ctypes.c_int64), ("s", ctypes.c_int64),
                ("p", ctypes.c_int64), ("A", ctypes.c_void_p), ("B", ctypes.c_void_p),
                ("C", ctypes.c_void_p), ("X", ctypes.c_void_p), ("opts", Opts),
                ("gen_seed", ctypes.c_uint64)]


class Problem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("s", ctypes.c_int64), ("p", ctypes.c_int64),
                ("A", ctypes.c_void_p), ("B", ctypes.c_void_p), ("C", ctypes.c_void_p),
                ("X", ctypes.c_void_p)]


_lib = None
_lock = threading.Lock()

_SIGS = {
    "tsylv_default_opts": (None, [ctypes.c_int, ctypes.POINTER(Opts)]),
    "tsylv_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int,
                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t]),
    "tsylv_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "tsylv_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int, ctypes.c_int64, ctypes.c_int64,
                                                ctypes.c_int64, ctypes.POINTER(Opts)]),
    "tsylv_apply": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                   ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]),
    "tsylv_fom": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                 ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                 ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(Opts),
                                 ctypes.POINTER(Info)]),
    "tsylv_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Request),
                                    ctypes.POINTER(ctypes.c_uint64)]),
    "tsylv_generate": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int64,
                                      ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_void_p]),
    "tsylv_batch_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int, ctypes.c_void_p,
                                                      ctypes.POINTER(Opts)]),
    "tsylv_gmres_batch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                         ctypes.POINTER(Opts), ctypes.c_void_p]),
    "tsylv_tbs_batch_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int, ctypes.c_void_p]),
    "tsylv_tbs_batch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                       ctypes.POINTER(Opts), ctypes.c_void_p]),
    "tsylv_apply_default_variant": (ctypes.c_int, [ctypes.c_int, ctypes.c_int64, ctypes.c_int64]),
    "tsylv_apply_variants": (ctypes.c_int, [ctypes.c_int]),
    "tsylv_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                      ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                      ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_float),
                                      ctypes.c_int]),
    "tsylv_tune_set": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int64,
                                      ctypes.c_int64, ctypes.c_int64, ctypes.c_int]),
    "tsylv_tune_get": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int64,
                                      ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(ctypes.c_int)]),
    "tsylv_tune_save": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_char_p]),
    "tsylv_tune_load": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_char_p]),
    "tsylv_poll": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(Info)]),
    "tsylv_noalloc_scratch_bytes": (ctypes.c_size_t, []),
    "tsylv_apply_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                           ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]),
    "tsylv_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "tsylv_profile": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "tsylv_profile_families": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint]),
    "tsylv_profile_read": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]),
}
_SIGS["tsylv_gmres"] = _SIGS["tsylv_fom"]
_SIGS["tsylv_tba"] = _SIGS["tsylv_fom"]
_SIGS["tsylv_tbs"] = _SIGS["tsylv_fom"]

EXPORTED = sorted(_SIGS)


def load(path=None):
    """Load libtsylv.so (once).  Raises OSError if it is missing.  torch is
    imported first: it brings its own copy of the HIP runtime, and the
    library must bind to that one (loaded first, the library would bind to
    the system's copy, and torch's streams and memory would not be valid in
    it)."""
    global _lib
    import torch  # noqa: F401  (the HIP runtime the library binds to)
    with _lock:
        if _lib is None:
            p = path or LIB_PATH
            if not os.path.exists(p):
                raise OSError("libtsylv.so not built (%s): run python -m "
                              "paper_2405_09233_amd.build" % p)
            lib = ctypes.CDLL(p)
            for name, (res, args) in _SIGS.items():
                fn = getattr(lib, name)
                fn.restype = res
                fn.argtypes = args
            _lib = lib
    return _lib


class TsylvError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = load().tsylv_strerror(status).decode()
        super().__init__("%s: %s (%d)" % (where, msg, status))


def default_opts(method=GMRES, **kw):
    o = Opts()
    load().tsylv_default_opts(method, ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def workspace_bytes(method, n, s, p, opts=None):
    return load().tsylv_workspace_bytes(method, n, s, p, ctypes.byref(opts) if opts else None)


# ------------------------------------------------------------ torch helpers

def to_device(arr, device="cuda"):
    """Fortran-ordered float64 (rows, cols, p) numpy array -> device tensor
    with the library layout."""
    import torch
    a = np.asarray(arr, dtype=np.float64)
    t = torch.from_numpy(np.ascontiguousarray(np.transpose(a, (2, 1, 0))))
    return t.to(device).permute(2, 1, 0)


def empty_device(shape, device="cuda"):
    import torch
    r, c, p = shape
    return torch.empty((p, c, r), dtype=torch.float64, device=device).permute(2, 1, 0)


def to_host(t):
    return np.asfortranarray(np.transpose(t.permute(2, 1, 0).cpu().numpy(), (2, 1, 0)))


def apply_variants(prec):
    """Number of tile variants of the apply kernel in precision `prec`."""
    n = load().tsylv_apply_variants(prec)
    if n < 0:
        raise TsylvError(n, "tsylv_apply_variants")
    return n


def apply_default_variant(prec, n, s):
    """The apply tile variant of a shape without a tuning-table entry."""
    v = load().tsylv_apply_default_variant(prec, n, s)
    if v < 0:
        raise TsylvError(v, "tsylv_apply_default_variant")
    return v


def apply_noalloc(A, B, X, Y=None, prec=FP64, stream=None):
    """tsylv_apply_noalloc: Y = A*X - X*B on the tensors' device with the
    library's static scratch (no device allocation inside the call),
    enqueued on `stream` (default: torch's current stream) without waiting.
    Y (allocated here when None) is ready once that stream reaches the call."""
    import torch
    n, _, p = A.shape
    s = B.shape[0]
    if Y is None:
        Y = empty_device((n, s, p), A.device)
    st = stream if stream is not None else torch.cuda.current_stream(A.device)
    with torch.cuda.device(A.device):
        rc = load().tsylv_apply_noalloc(ctypes.c_void_p(st.cuda_stream), n, s, p, _ptr(A),
                                        _ptr(B), _ptr(X), _ptr(Y), prec)
    if rc != 0:
        raise TsylvError(rc, "tsylv_apply_noalloc")
    return Y


def noalloc_scratch_bytes():
    return load().tsylv_noalloc_scratch_bytes()


def _ptr(t):
    if t is None:
        return None
    if not t.permute(2, 1, 0).is_contiguous() or str(t.dtype) != "torch.float64":
        raise ValueError("tensor must be float64 with slice-major column-major layout")
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """A library context bound to one device, one stream and one arena."""

    def __init__(self, arena_bytes, device=0, stream=None, own_arena=False):
        import torch
        self.device = device
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        self.arena = None
        aptr = None
        if not own_arena:
            self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8,
                                     device="cuda:%d" % device)
            aptr = ctypes.c_void_p(self.arena.data_ptr())
        h = ctypes.c_void_p()
        st = load().tsylv_create(ctypes.byref(h), device, ctypes.c_void_p(self.stream.cuda_stream),
                                 aptr, ctypes.c_size_t(int(arena_bytes)))
        if st != 0:
            raise TsylvError(st, "tsylv_create")
        self.handle = h

    def close(self):
        """Destroy the library context (finishes admitted requests, cancels
        queued ones) and release the arena."""
        if getattr(self, "handle", None):
            load().tsylv_destroy(self.handle)
            self.handle = None
        self.arena = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- calls -------------------------------------------------------------
    def apply(self, A, B, X, Y=None, prec=FP64):
        n, _, p = A.shape
        s = B.shape[0]
        if Y is None:
            Y = empty_device((n, s, p), A.device)
        st = load().tsylv_apply(self.handle, n, s, p, _ptr(A), _ptr(B), _ptr(X), _ptr(Y), prec)
        if st != 0:
            raise TsylvError(st, "tsylv_apply")
        return Y

    def _solve(self, fname, A, B, C, X=None, opts=None, raise_on_error=True, **kw):
        n, _, p = A.shape
        s = B.shape[0]
        method = {"tsylv_gmres": GMRES, "tsylv_fom": FOM, "tsylv_tba": TBA,
                  "tsylv_tbs": TBS}[fname]
        o = opts if opts is not None else default_opts(method, **kw)
        if X is None:
            X = empty_device((n, s, p), A.device)
        info = Info()
        st = getattr(load(), fname)(self.handle, n, s, p, _ptr(A), _ptr(B), _ptr(C), _ptr(X),
                                    ctypes.byref(o), ctypes.byref(info))
        if st < 0 and raise_on_error:
            raise TsylvError(st, fname)
        return X, info

    def gmres(self, A, B, C, X=None, opts=None, **kw):
        return self._solve("tsylv_gmres", A, B, C, X, opts, **kw)

    def fom(self, A, B, C, X=None, opts=None, **kw):
        return self._solve("tsylv_fom", A, B, C, X, opts, **kw)

    def tba(self, A, B, C, X=None, opts=None, **kw):
        return self._solve("tsylv_tba", A, B, C, X, opts, **kw)

    def tbs(self, A, B, C, X=None, opts=None, **kw):
        return self._solve("tsylv_tbs", A, B, C, X, opts, **kw)

    @staticmethod
    def _problems(items):
        probs = (Problem * len(items))()
        for k, (A, B, C, X) in enumerate(items):
            n, _, p = A.shape
            probs[k].n, probs[k].s, probs[k].p = n, B.shape[0], p
            probs[k].A, probs[k].B, probs[k].C, probs[k].X = (_ptr(t).value for t in (A, B, C, X))
        return probs

    def gmres_batch(self, items, opts=None, raise_on_error=True, **kw):
        """Batched lockstep tGMRES over `items`, a list of (A, B, C, X)
        device tensors (X receives the solution).  Returns the list of
        per-instance Info records."""
        probs = self._problems(items)
        o = opts if opts is not None else default_opts(GMRES, **kw)
        infos = (Info * len(items))()
        st = load().tsylv_gmres_batch(self.handle, len(items), probs, ctypes.byref(o), infos)
        if st < 0 and raise_on_error:
            raise TsylvError(st, "tsylv_gmres_batch")
        return list(infos)

    def tbs_batch(self, items, tol=1e-8, raise_on_error=True):
        """Batched t-Bartels-Stewart over `items`, a list of (A, B, C, X)
        device tensors (instances with n or s above 64 are solved by
        tGMRES(30) to `tol` instead); X receives each solution.  Returns the
        list of per-instance Info records."""
        probs = self._problems(items)
        o = default_opts(TBS, tol=tol)
        infos = (Info * len(items))()
        st = load().tsylv_tbs_batch(self.handle, len(items), probs, ctypes.byref(o), infos)
        if st < 0 and raise_on_error:
            raise TsylvError(st, "tsylv_tbs_batch")
        return list(infos)

    @staticmethod
    def tbs_batch_workspace_bytes(items):
        return load().tsylv_tbs_batch_workspace_bytes(len(items), Context._problems(items))

    @staticmethod
    def batch_workspace_bytes(items, opts=None, **kw):
        o = opts if opts is not None else default_opts(GMRES, **kw)
        return load().tsylv_batch_workspace_bytes(len(items), Context._problems(items),
                                                  ctypes.byref(o))

    def generate(self, seed, n, s, p, device=None):
        """The synthetic instance of `seed` (tsylv_generate) as device
        tensors A, B, C."""
        dev = device if device is not None else "cuda:%d" % self.device
        A, B, C = (empty_device(sh, dev) for sh in ((n, n, p), (s, s, p), (n, s, p)))
        st = load().tsylv_generate(self.handle, seed, n, s, p, _ptr(A), _ptr(B), _ptr(C))
        if st != 0:
            raise TsylvError(st, "tsylv_generate")
        return A, B, C

    def submit(self, A, B, C, X, method=GMRES, opts=None, seed=None, **kw):
        """Queue a solve.  With A, B and C None the request solves the
        synthetic instance of `seed`, drawn on the device (its shape is X's)."""
        req = Request()
        req.method = method
        if A is None and B is None and C is None:
            if seed is None:
                raise ValueError("a generated request needs a seed")
            n, s, p = X.shape
            req.gen_seed = seed
        else:
            n, _, p = A.shape
            s = B.shape[0]
            req.A, req.B, req.C = (_ptr(t).value for t in (A, B, C))
        req.n, req.s, req.p = n, s, p
        req.X = _ptr(X).value
        req.opts = opts if opts is not None else default_opts(method, **kw)
        ticket = ctypes.c_uint64()
        st = load().tsylv_submit(self.handle, ctypes.byref(req), ctypes.byref(ticket))
        if st != 0:
            raise TsylvError(st, "tsylv_submit")
        return ticket.value

    def autotune(self, n, s, p, prec=FP64, reps=5):
        """Time every tile variant of the apply at (n, s, p); the fastest is
        used from now on.  Returns (best variant, [ms per variant])."""
        nv = apply_variants(prec)
        ms = (ctypes.c_float * nv)()
        best = ctypes.c_int(-1)
        st = load().tsylv_autotune(self.handle, n, s, p, prec, reps, ctypes.byref(best), ms, nv)
        if st != 0:
            raise TsylvError(st, "tsylv_autotune")
        return best.value, [float(x) for x in ms]

    def tune_set(self, n, s, p, prec, variant):
        st = load().tsylv_tune_set(self.handle, prec, n, s, p, variant)
        if st != 0:
            raise TsylvError(st, "tsylv_tune_set")

    def tune_get(self, n, s, p, prec):
        v = ctypes.c_int(-1)
        st = load().tsylv_tune_get(self.handle, prec, n, s, p, ctypes.byref(v))
        if st != 0:
            raise TsylvError(st, "tsylv_tune_get")
        return v.value

    def tune_save(self, path):
        st = load().tsylv_tune_save(self.handle, os.fsencode(path))
        if st != 0:
            raise TsylvError(st, "tsylv_tune_save")

    def tune_load(self, path):
        st = load().tsylv_tune_load(self.handle, os.fsencode(path))
        if st != 0:
            raise TsylvError(st, "tsylv_tune_load")

    def profile(self, enable=True, families=None):
        """Start (every family, or the kernel ids in `families`) or stop timing."""
        if families is None or not enable:
            st = load().tsylv_profile(self.handle, 1 if enable else 0)
        else:
            mask = 0
            for k in families:
                mask |= 1 << k
            st = load().tsylv_profile_families(self.handle, mask)
        if st != 0:
            raise TsylvError(st, "tsylv_profile")

    def profile_read(self, kernel_id):
        k = KStat()
        st = load().tsylv_profile_read(self.handle, kernel_id, ctypes.byref(k))
        if st != 0:
            raise TsylvError(st, "tsylv_profile_read")
        return k.launches, k.total_ms

    def poll(self, ticket):
        info = Info()
        st = load().tsylv_poll(self.handle, ctypes.c_uint64(ticket), ctypes.byref(info))
        return st, info
