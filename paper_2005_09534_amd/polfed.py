"""ctypes binding of libpolfed (include/polfed.h).  Argument marshalling only.

Device arrays are torch tensors on a HIP device (their data_ptr() is handed
to the library); the library runs on torch's current stream.  Host arrays are
numpy.  There is no fallback: if ``libpolfed.so`` is missing or fails to load,
importing this module raises.
"""

import ctypes
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpolfed.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "polfed.h")

OK, NOT_CONVERGED = 0, 1
FORM_CLENSHAW, FORM_FORWARD = 0, 1
EINVAL, ENOMEM, EDEVICE, EBOUNDS, EBREAKDOWN = -1, -2, -3, -4, -5

c_int, c_double, c_ll, c_ull, c_void_p = (ctypes.c_int, ctypes.c_double, ctypes.c_longlong,
                                          ctypes.c_ulonglong, ctypes.c_void_p)
P_double = ctypes.POINTER(c_double)


class Model(ctypes.Structure):
    _fields_ = [("L", c_int), ("J1", c_double), ("J2", c_double), ("Delta", c_double),
                ("h", P_double)]


DOS_GAUSS, DOS_KPM = 0, 1
DAMP_NONE, DAMP_JACKSON = 0, 1


class Opts(ctypes.Structure):
    _fields_ = [("target_kind", c_int), ("target", c_double), ("block_size", c_int),
                ("K", c_ll), ("p", c_double), ("precision", c_int),
                ("window_factor", c_double), ("max_cols", c_int), ("tol", c_double),
                ("eta", c_double), ("bounds_steps", c_int), ("seed", c_ull),
                ("max_order", c_ll), ("dos", c_int), ("dos_moments", c_int),
                ("dos_vectors", c_int), ("damping", c_int)]


class Info(ctypes.Structure):
    _fields_ = [("E0", c_double), ("E1", c_double), ("E0w", c_double), ("E1w", c_double),
                ("sigma_energy", c_double), ("sigma_tilde", c_double), ("normH", c_double),
                ("K", c_ll), ("nev_window", c_int), ("block_size", c_int), ("m", c_int),
                ("n_conv", c_int), ("refine_passes", c_int), ("max_resid", c_double),
                ("t_bounds", c_double), ("t_filter", c_double), ("t_orth", c_double),
                ("t_eig", c_double), ("t_rr", c_double), ("t_refine", c_double),
                ("t_total", c_double), ("hv_apps", c_double), ("filter_bytes", c_double),
                ("filter_gpu_s", c_double), ("filter_launches", c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class PolfedError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libpolfed status {code}: {msg}")
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2005_09534_amd.build` "
                          "(or __graft_entry__.build())")
    # The library must share torch's HIP runtime (torch brings its own copy;
    # a second copy loaded first can fail to see the device): importing torch
    # first makes the dynamic loader resolve the library's HIP dependency to
    # the copy torch loaded.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    sig = {
        "polfed_create": (c_int, [c_int, ctypes.POINTER(c_void_p)]),
        "polfed_destroy": (c_int, [c_void_p]),
        "polfed_last_error": (ctypes.c_char_p, [c_void_p]),
        "polfed_set_stream": (c_int, [c_void_p, c_void_p]),
        "polfed_synchronize": (c_int, [c_void_p]),
        "polfed_dim": (c_ll, [c_int]),
        "polfed_default_opts": (None, [ctypes.POINTER(Opts)]),
        "polfed_cheb_coeffs": (c_int, [c_double, c_ll, P_double, P_double]),
        "polfed_filter_order": (c_int, [ctypes.POINTER(Model), c_double, c_double, c_double, c_int,
                                        c_double, ctypes.POINTER(c_ll), P_double]),
        "polfed_window_order": (c_int, [ctypes.POINTER(Model), c_double, c_double, c_double, c_int,
                                        c_double, c_ll, ctypes.POINTER(c_int), ctypes.POINTER(c_ll)]),
        "polfed_basis": (c_int, [c_void_p, c_int, c_void_p]),
        "polfed_rank": (c_int, [c_void_p, c_int, c_ll, c_void_p, c_void_p]),
        "polfed_diag": (c_int, [c_void_p, ctypes.POINTER(Model), c_void_p]),
        "polfed_apply_h": (c_int, [c_void_p, ctypes.POINTER(Model), c_int, c_int, c_void_p,
                                   c_void_p]),
        "polfed_apply_filter": (c_int, [c_void_p, ctypes.POINTER(Model), c_double, c_double,
                                        c_double, c_ll, c_int, c_int, c_void_p, c_void_p]),
        "polfed_gram": (c_int, [c_void_p, c_ll, c_int, c_int, c_void_p, c_ll, c_void_p, c_ll,
                                c_void_p, c_ll]),
        "polfed_gram_static": (c_int, [c_void_p, c_ll, c_int, c_int, c_void_p, c_ll, c_void_p,
                                       c_ll, c_void_p, c_ll]),
        "polfed_update": (c_int, [c_void_p, c_ll, c_int, c_int, c_double, c_void_p, c_ll,
                                  c_void_p, c_ll, c_double, c_void_p, c_ll]),
        "polfed_sym_eig": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p]),
        "polfed_bounds": (c_int, [c_void_p, ctypes.POINTER(Model), c_int, c_ull, P_double,
                                  P_double, P_double, P_double]),
        "polfed_set_step_shape": (c_int, [c_void_p, c_int, c_int, c_int, c_int, c_int, c_int,
                                          c_int, c_int, c_int, c_int]),
        "polfed_get_step_shape": (c_int, [c_void_p, c_int, c_int, c_int] + [ctypes.POINTER(c_int)] * 7),
        "polfed_set_batch_shape": (c_int, [c_void_p, c_int, c_int, c_int, c_int, c_int, c_int,
                                           c_int, c_int, c_int]),
        "polfed_get_batch_shape": (c_int, [c_void_p, c_int, c_int, c_int] + [ctypes.POINTER(c_int)] * 6),
        "polfed_set_graphs": (c_int, [c_void_p, c_int]),
        "polfed_set_filter_form": (c_int, [c_void_p, c_int]),
        "polfed_set_block_size": (c_int, [c_void_p, c_int, c_int, c_int, c_int]),
        "polfed_filter_stats": (c_int, [c_void_p, P_double, P_double, P_double, c_int]),
        "polfed_entanglement": (c_int, [c_void_p, c_int, c_int, c_void_p, c_ll, c_int,
                                        ctypes.POINTER(c_int), P_double]),
        "polfed_gap_ratio": (c_int, [P_double, c_int, P_double]),
        "polfed_kpm_count": (c_int, [P_double, c_int, c_ll, c_double, c_double, P_double]),
        "polfed_kpm_order": (c_int, [P_double, c_int, c_ll, c_double, c_int, c_double, c_int,
                                     c_ll, ctypes.POINTER(c_int), ctypes.POINTER(c_ll)]),
        "polfed_filter_coeffs": (c_int, [c_double, c_ll, c_int, P_double, P_double]),
        "polfed_filter_order_damped": (c_int, [ctypes.POINTER(Model), c_double, c_double, c_double,
                                               c_int, c_double, c_int, c_ll,
                                               ctypes.POINTER(c_int), ctypes.POINTER(c_ll)]),
        "polfed_set_filter_damping": (c_int, [c_void_p, c_int]),
        "polfed_dos_moments": (c_int, [c_void_p, ctypes.POINTER(Model), c_double, c_double,
                                       c_int, c_int, c_void_p, c_ull, P_double]),
        "polfed_s_rmt": (c_double, [c_int]),
        "polfed_stream_copy": (c_int, [c_void_p, c_void_p, c_void_p, c_ll, c_int, P_double]),
        "polfed_solve": (c_int, [c_void_p, ctypes.POINTER(Model), ctypes.POINTER(Opts), c_int,
                                 P_double, P_double, P_double, ctypes.POINTER(Info)]),
        "polfed_solve_batch": (c_int, [c_void_p, c_int, ctypes.POINTER(Model),
                                       ctypes.POINTER(Opts), c_int, P_double, P_double, P_double,
                                       ctypes.POINTER(Info), ctypes.POINTER(c_int)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


LIB = _load()


def header_functions(path=HEADER):
    """Names of the functions include/polfed.h declares."""
    txt = open(path).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(polfed_[a-z_0-9]+)\s*\(", txt)))


def dim(L):
    return int(LIB.polfed_dim(L))


def default_opts(**kw):
    o = Opts()
    LIB.polfed_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def make_model(L, J1, J2, Delta, h):
    h = np.ascontiguousarray(h, dtype=np.float64)
    if h.shape != (L,):
        raise ValueError("h must have length L")
    m = Model(L, J1, J2, Delta, h.ctypes.data_as(P_double))
    m._h = h  # keep the array alive with the struct
    return m


def cheb_coeffs(sigma, K):
    c = np.empty(K + 1)
    D = c_double()
    rc = LIB.polfed_cheb_coeffs(sigma, K, c.ctypes.data_as(P_double), ctypes.byref(D))
    if rc != OK:
        raise PolfedError(rc, "polfed_cheb_coeffs")
    return c, D.value


def filter_order(model, E0w, E1w, sigma, nwin, p=0.17):
    K = c_ll()
    rho = c_double()
    rc = LIB.polfed_filter_order(ctypes.byref(model), E0w, E1w, sigma, nwin, p, ctypes.byref(K),
                                 ctypes.byref(rho))
    if rc != OK:
        raise PolfedError(rc, "polfed_filter_order")
    return K.value, rho.value


def window_order(model, E0w, E1w, sigma, nwin, max_order, p=0.17):
    """(window count, K) of the FP32 order cap (polfed_window_order)."""
    nw = c_int()
    K = c_ll()
    rc = LIB.polfed_window_order(ctypes.byref(model), E0w, E1w, sigma, nwin, p, max_order,
                                 ctypes.byref(nw), ctypes.byref(K))
    if rc != OK:
        raise PolfedError(rc, "polfed_window_order")
    return nw.value, K.value


def kpm_count(mu, N, x_lo, x_hi):
    """States of an N-state sector in [x_lo, x_hi] of H~ from the Chebyshev
    moments mu (polfed_kpm_count)."""
    mu = np.ascontiguousarray(mu, dtype=np.float64)
    out = c_double()
    rc = LIB.polfed_kpm_count(mu.ctypes.data_as(P_double), len(mu), N, x_lo, x_hi,
                              ctypes.byref(out))
    if rc != OK:
        raise PolfedError(rc, "polfed_kpm_count")
    return out.value


def kpm_order(mu, N, sigma, nwin, p=0.17, max_order=0, damping=0):
    """(window count, K) of the order rule with the KPM density (polfed_kpm_order)."""
    mu = np.ascontiguousarray(mu, dtype=np.float64)
    nw = c_int()
    K = c_ll()
    rc = LIB.polfed_kpm_order(mu.ctypes.data_as(P_double), len(mu), N, sigma, nwin, p, damping,
                              max_order, ctypes.byref(nw), ctypes.byref(K))
    if rc != OK:
        raise PolfedError(rc, "polfed_kpm_order")
    return nw.value, K.value


def filter_coeffs(sigma, K, damping=0):
    """(c[0..K], D) of the filter with the given damping (polfed_filter_coeffs)."""
    c = np.empty(K + 1)
    D = c_double()
    rc = LIB.polfed_filter_coeffs(sigma, K, damping, c.ctypes.data_as(P_double), ctypes.byref(D))
    if rc != OK:
        raise PolfedError(rc, "polfed_filter_coeffs")
    return c, D.value


def filter_order_damped(model, E0w, E1w, sigma, nwin, damping, p=0.17, max_order=0):
    """(window count, K) of the order rule for a damped filter."""
    nw = c_int()
    K = c_ll()
    rc = LIB.polfed_filter_order_damped(ctypes.byref(model), E0w, E1w, sigma, nwin, p, damping,
                                        max_order, ctypes.byref(nw), ctypes.byref(K))
    if rc != OK:
        raise PolfedError(rc, "polfed_filter_order_damped")
    return nw.value, K.value


def gap_ratio(E):
    """Mean gap ratio of the levels E (polfed_gap_ratio)."""
    E = np.ascontiguousarray(E, dtype=np.float64)
    r = c_double()
    rc = LIB.polfed_gap_ratio(E.ctypes.data_as(P_double), len(E), ctypes.byref(r))
    if rc != OK:
        raise PolfedError(rc, "polfed_gap_ratio")
    return r.value


def s_rmt(L):
    return float(LIB.polfed_s_rmt(L))


def _ptr(t):
    return c_void_p(t.data_ptr())


class Context:
    """A libpolfed context on one HIP device, bound to torch's current stream."""

    def __init__(self, device=0):
        import torch
        self._torch = torch
        h = c_void_p()
        rc = LIB.polfed_create(device, ctypes.byref(h))
        if rc != OK:
            msg = LIB.polfed_last_error(None).decode(errors="replace")
            raise PolfedError(rc, f"polfed_create({device}) failed: {msg}")
        self.h = h
        self.device = device
        self.bind_stream()

    def bind_stream(self, stream=None):
        torch = self._torch
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._check(LIB.polfed_set_stream(self.h, c_void_p(s.cuda_stream)), "set_stream")

    def close(self):
        if getattr(self, "h", None):
            LIB.polfed_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, what, allow_warning=False):
        if rc < 0 or (rc > 0 and not allow_warning):
            msg = LIB.polfed_last_error(self.h)
            raise PolfedError(rc, f"{what}: {msg.decode() if msg else ''}")
        return rc

    def synchronize(self):
        self._check(LIB.polfed_synchronize(self.h), "synchronize")

    # ---- stage calls (torch device tensors) ----
    def basis(self, L):
        torch = self._torch
        out = torch.empty(dim(L), dtype=torch.int32, device=f"cuda:{self.device}")
        self._check(LIB.polfed_basis(self.h, L, _ptr(out)), "basis")
        self.synchronize()
        return out

    def rank(self, L, states):
        torch = self._torch
        out = torch.empty(states.numel(), dtype=torch.int32, device=states.device)
        self._check(LIB.polfed_rank(self.h, L, states.numel(), _ptr(states), _ptr(out)), "rank")
        self.synchronize()
        return out

    def diag(self, model):
        torch = self._torch
        out = torch.empty(dim(model.L), dtype=torch.float64, device=f"cuda:{self.device}")
        self._check(LIB.polfed_diag(self.h, ctypes.byref(model), _ptr(out)), "diag")
        return out

    def apply_h(self, model, X):
        torch = self._torch
        prec = 0 if X.dtype == torch.float64 else 1
        X = X.contiguous()
        Y = torch.empty_like(X)
        self._check(LIB.polfed_apply_h(self.h, ctypes.byref(model), prec, X.shape[1], _ptr(X),
                                       _ptr(Y)), "apply_h")
        return Y

    def apply_filter(self, model, E0, E1, sigma, K, X, out=None):
        torch = self._torch
        prec = 0 if X.dtype == torch.float64 else 1
        X = X.contiguous()
        Y = torch.empty_like(X) if out is None else out
        self._check(LIB.polfed_apply_filter(self.h, ctypes.byref(model), E0, E1, sigma, K, prec,
                                            X.shape[1], _ptr(X), _ptr(Y)), "apply_filter")
        return Y

    def gram(self, X, Y):
        torch = self._torch
        n, p = X.shape
        q = Y.shape[1]
        C = torch.empty((p, q), dtype=torch.float64, device=X.device)
        self._check(LIB.polfed_gram(self.h, n, p, q, _ptr(X), X.stride(0), _ptr(Y), Y.stride(0),
                                    _ptr(C), q), "gram")
        self.synchronize()
        return C

    def gram_static(self, X, Y, out):
        """polfed_gram_static into the preallocated tensor out (p x q)."""
        n, p = X.shape
        q = Y.shape[1]
        self._check(LIB.polfed_gram_static(self.h, n, p, q, _ptr(X), X.stride(0), _ptr(Y),
                                           Y.stride(0), _ptr(out), out.stride(0)), "gram_static")
        return out

    def update(self, X, C, Y, alpha=1.0, beta=0.0):
        n, p = X.shape
        q = C.shape[1]
        self._check(LIB.polfed_update(self.h, n, p, q, alpha, _ptr(X), X.stride(0), _ptr(C),
                                      C.stride(0), beta, _ptr(Y), Y.stride(0)), "update")
        self.synchronize()
        return Y

    def sym_eig(self, A):
        torch = self._torch
        A = A.clone().contiguous()
        n = A.shape[0]
        w = torch.empty(n, dtype=torch.float64, device=A.device)
        V = torch.empty((n, n), dtype=torch.float64, device=A.device)
        self._check(LIB.polfed_sym_eig(self.h, n, _ptr(A), _ptr(w), _ptr(V)), "sym_eig")
        return w, V

    def bounds(self, model, steps=200, seed=7):
        out = [c_double() for _ in range(4)]
        self._check(LIB.polfed_bounds(self.h, ctypes.byref(model), steps, seed,
                                      *[ctypes.byref(o) for o in out]), "bounds")
        return tuple(o.value for o in out)

    # ---- tuning / measurement ----
    def set_step_shape(self, L, nvec, precision, threads, lpl, wg_per_cu, lds_tables=1,
                       early_loads=0, rank_incremental=0, xcd_slices=1):
        self._check(LIB.polfed_set_step_shape(self.h, L, nvec, precision, threads, lpl, wg_per_cu,
                                              int(lds_tables), int(early_loads),
                                              int(rank_incremental), int(xcd_slices)),
                    "set_step_shape")

    def set_batch_shape(self, L, nvec, precision, threads, lpl, wg_per_cu, lds_tables=1,
                        early_loads=0, xcd_slices=1):
        self._check(LIB.polfed_set_batch_shape(self.h, L, nvec, precision, threads, lpl,
                                               wg_per_cu, lds_tables, early_loads, xcd_slices),
                    "set_batch_shape")

    def get_batch_shape(self, L, nvec, precision):
        """(threads, lpl, wg_per_cu, lds_tables, early_loads, xcd_slices) of the
        batched kernel."""
        out = [c_int() for _ in range(6)]
        self._check(LIB.polfed_get_batch_shape(self.h, L, nvec, precision,
                                               *[ctypes.byref(o) for o in out]), "get_batch_shape")
        return tuple(o.value for o in out)

    def get_step_shape(self, L, nvec, precision):
        """(threads, lpl, wg_per_cu, lds_tables, early_loads, rank_incremental, xcd_slices)."""
        out = [c_int() for _ in range(7)]
        self._check(LIB.polfed_get_step_shape(self.h, L, nvec, precision,
                                              *[ctypes.byref(o) for o in out]), "get_step_shape")
        return tuple(o.value for o in out)

    def set_block_size(self, L, precision, nev, block_size):
        self._check(LIB.polfed_set_block_size(self.h, L, precision, nev, block_size),
                    "set_block_size")

    def set_graphs(self, on):
        self._check(LIB.polfed_set_graphs(self.h, int(bool(on))), "set_graphs")

    def set_filter_form(self, form):
        """FORM_CLENSHAW (default) or FORM_FORWARD."""
        self._check(LIB.polfed_set_filter_form(self.h, int(form)), "set_filter_form")

    def filter_stats(self, reset=True):
        g, l, b = c_double(), c_double(), c_double()
        self._check(LIB.polfed_filter_stats(self.h, ctypes.byref(g), ctypes.byref(l),
                                            ctypes.byref(b), int(reset)), "filter_stats")
        return dict(gpu_s=g.value, launches=l.value, bytes=b.value)

    def entanglement(self, L, V, cuts=None):
        """S_E of the columns of the device tensor V (n x nvec, FP64) for the
        cuts (bit offsets; default 0 .. L/2-1): numpy array nvec x ncut."""
        cuts = list(range(L // 2)) if cuts is None else list(cuts)
        c = (c_int * len(cuts))(*cuts)
        V = V.contiguous()
        S = np.empty((V.shape[1], len(cuts)))
        self._check(LIB.polfed_entanglement(self.h, L, V.shape[1], _ptr(V), V.stride(0),
                                            len(cuts), c, S.ctypes.data_as(P_double)),
                    "entanglement")
        return S

    def dos_moments(self, model, E0w, E1w, nmom, R=None, nvec=4, seed=1):
        """Chebyshev moments of H~ (polfed_dos_moments): from the columns of
        the device tensor R (n x nvec, FP64), or from nvec Philox +-1
        vectors keyed by seed when R is None.  numpy array of nmom."""
        mu = np.empty(nmom)
        if R is not None:
            R = R.contiguous()
            nvec = R.shape[1]
        self._check(LIB.polfed_dos_moments(self.h, ctypes.byref(model), E0w, E1w, nmom, nvec,
                                           None if R is None else _ptr(R), seed,
                                           mu.ctypes.data_as(P_double)), "dos_moments")
        return mu

    def set_filter_damping(self, damping):
        """DAMP_NONE or DAMP_JACKSON for apply_filter."""
        self._check(LIB.polfed_set_filter_damping(self.h, damping), "set_filter_damping")

    def stream_copy(self, src, dst, reps=10):
        """Copy rate (GB/s, read + write) of the library's plain copy kernel
        from tensor src to tensor dst (same byte size)."""
        gbs = c_double()
        nbytes = src.numel() * src.element_size()
        if dst.numel() * dst.element_size() != nbytes:
            raise ValueError("src and dst must have the same byte size")
        self._check(LIB.polfed_stream_copy(self.h, _ptr(src), _ptr(dst), nbytes, reps,
                                           ctypes.byref(gbs)), "stream_copy")
        return gbs.value

    # ---- the solve (host outputs) ----
    def solve(self, model, nev, opts=None, vectors=True, **kw):
        o = opts if opts is not None else default_opts(**kw)
        n = dim(model.L)
        ev = np.empty(nev)
        rs = np.empty(nev)
        V = np.empty((nev, n)) if vectors else None
        info = Info()
        rc = LIB.polfed_solve(self.h, ctypes.byref(model), ctypes.byref(o), nev,
                              ev.ctypes.data_as(P_double),
                              V.ctypes.data_as(P_double) if vectors else None,
                              rs.ctypes.data_as(P_double), ctypes.byref(info))
        self._check(rc, "solve", allow_warning=True)
        return dict(E=ev, V=(V.T if vectors else None), resid=rs, info=info.as_dict(), status=rc)

    def solve_batch(self, models, nev, opts=None, vectors=False, **kw):
        o = opts if opts is not None else default_opts(**kw)
        R = len(models)
        arr = (Model * R)(*models)
        ev = np.full((R, nev), np.nan)  # a member that fails leaves its rows untouched
        rs = np.full((R, nev), np.nan)
        tot = sum(dim(m.L) for m in models)
        V = np.empty(tot * nev) if vectors else None
        infos = (Info * R)()
        st = (c_int * R)()
        rc = LIB.polfed_solve_batch(self.h, R, arr, ctypes.byref(o), nev,
                                    ev.ctypes.data_as(P_double),
                                    V.ctypes.data_as(P_double) if vectors else None,
                                    rs.ctypes.data_as(P_double), infos, st)
        self._check(rc, "solve_batch", allow_warning=True)
        vecs = None
        if vectors:
            vecs, off = [], 0
            for m in models:
                n = dim(m.L)
                vecs.append(V[off:off + n * nev].reshape(nev, n).T)
                off += n * nev
        return dict(E=ev, resid=rs, V=vecs, info=[i.as_dict() for i in infos],
                    status=list(st), rc=rc)
