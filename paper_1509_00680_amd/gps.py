"""Thin ctypes binding of libgps (include/gps.h).

Argument marshalling only: every step of a solve runs in the HIP kernels of
libgps.so.  Functions keep the C names; `Plan` wraps a plan handle and
accepts torch tensors (float64, on the GPU) whose device pointers it passes
through.  Importing works without a GPU; loading the library fails loudly if
it has not been built (there is no fallback path).
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgps.so")

GPS_BC_FREE, GPS_BC_SURFACE, GPS_BC_PERIODIC, GPS_BC_WIRE = 0, 1, 2, 3
BC_CODES = {"free": GPS_BC_FREE, "surface": GPS_BC_SURFACE, "periodic": GPS_BC_PERIODIC,
            "wire": GPS_BC_WIRE}
GPS_PREC_FP64, GPS_PREC_MIXED = 0, 1
PRECISIONS = {"fp64": GPS_PREC_FP64, "mixed": GPS_PREC_MIXED}

STATUS = {0: "GPS_OK", 1: "GPS_E_INVALID", 2: "GPS_E_NOMEM", 3: "GPS_E_NOT_CONVERGED",
          4: "GPS_E_BREAKDOWN", 5: "GPS_E_NONFINITE", 6: "GPS_E_DEVICE", 7: "GPS_E_UNSUPPORTED",
          8: "GPS_PENDING"}
GPS_OK, GPS_E_INVALID, GPS_E_NOMEM, GPS_E_NOT_CONVERGED = 0, 1, 2, 3
GPS_E_BREAKDOWN, GPS_E_NONFINITE, GPS_E_DEVICE, GPS_E_UNSUPPORTED = 4, 5, 6, 7
GPS_PENDING = 8
NOALLOC_MAX_POINTS = 4194304          # GPS_NOALLOC_MAX_POINTS

# every symbol include/gps.h declares
EXPORTED = ("gps_plan_create", "gps_plan_set_options", "gps_plan_get_options",
            "gps_plan_device_bytes", "gps_plan_destroy", "gps_solve_generalized",
            "gps_solve_pb", "gps_solve_vacuum", "gps_solve_generalized_q", "gps_solve_sc",
            "gps_rigid_cavity",
            "gps_polarization_charge", "gps_polarization_charge_noalloc",
            "gps_last_info", "gps_last_history",
            "gps_plan_set_timing", "gps_plan_timing", "gps_status_string",
            "gps_plan_footprint", "gps_plan_release_buffers", "gps_server_create", "gps_server_submit", "gps_server_poll",
            "gps_server_wait", "gps_server_get_stats", "gps_server_destroy")
KERNEL_KINDS = {"xfwd": 1, "yfwd": 2, "zconv": 3, "yinv": 4, "xinv": 5}


class gps_options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("fd_order", ctypes.c_int),
                ("maxit", ctypes.c_int), ("check_every", ctypes.c_int),
                ("stream", ctypes.c_void_p), ("refine_every", ctypes.c_int),
                ("warm_start", ctypes.c_int)]


class gps_ions(ctypes.Structure):
    _fields_ = [("nspecies", ctypes.c_int), ("Z", ctypes.POINTER(ctypes.c_double)),
                ("c_bulk", ctypes.POINTER(ctypes.c_double)),
                ("c_max", ctypes.POINTER(ctypes.c_double)), ("kT", ctypes.c_double),
                ("gamma", ctypes.c_void_p), ("eps_bulk", ctypes.c_double),
                ("linear", ctypes.c_int), ("eta", ctypes.c_double),
                ("outer_maxit", ctypes.c_int)]


class gps_info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("iterations", ctypes.c_int),
                ("outer_iterations", ctypes.c_int), ("history_len", ctypes.c_int),
                ("rnorm0", ctypes.c_double), ("rel_residual", ctypes.c_double),
                ("energy", ctypes.c_double), ("outer_residual", ctypes.c_double),
                ("device_error", ctypes.c_int)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class gps_server_options(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_size_t), ("max_active", ctypes.c_int),
                ("precision", ctypes.c_int), ("fd_order", ctypes.c_int), ("maxit", ctypes.c_int),
                ("batch_slots", ctypes.c_int)]


class gps_request(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("h", ctypes.c_double), ("bc", ctypes.c_int), ("rho", ctypes.c_void_p),
                ("eps", ctypes.c_void_p), ("phi", ctypes.c_void_p),
                ("ions", ctypes.POINTER(gps_ions)), ("tol", ctypes.c_double),
                ("eps_key", ctypes.c_ulonglong)]


class gps_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("iterations", ctypes.c_int),
                ("outer_iterations", ctypes.c_int), ("rel_residual", ctypes.c_double),
                ("energy", ctypes.c_double), ("submit_ms", ctypes.c_double),
                ("start_ms", ctypes.c_double), ("done_ms", ctypes.c_double),
                ("worker", ctypes.c_int), ("plan_reused", ctypes.c_int),
                ("device_error", ctypes.c_int), ("warm_started", ctypes.c_int)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class gps_server_stats(ctypes.Structure):
    _fields_ = [("bytes_in_use", ctypes.c_size_t), ("bytes_peak", ctypes.c_size_t),
                ("plans_resident", ctypes.c_int), ("plans_created", ctypes.c_int),
                ("plans_evicted", ctypes.c_int), ("buffers_released", ctypes.c_int),
                ("max_in_flight", ctypes.c_int),
                ("submitted", ctypes.c_longlong), ("completed", ctypes.c_longlong),
                ("batched", ctypes.c_longlong), ("max_batch", ctypes.c_int)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib = None


def load(path=LIB_PATH):
    """Load libgps.so and declare the C signatures (raises if missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libgps.so is not built (%s); run __graft_entry__.build()" % path)
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    D = ctypes.c_double
    I = ctypes.c_int
    lib.gps_plan_create.argtypes = [I, I, I, D, I, ctypes.POINTER(P)]
    lib.gps_plan_create.restype = I
    lib.gps_plan_set_options.argtypes = [P, ctypes.POINTER(gps_options)]
    lib.gps_plan_set_options.restype = I
    lib.gps_plan_get_options.argtypes = [P, ctypes.POINTER(gps_options)]
    lib.gps_plan_get_options.restype = I
    lib.gps_plan_device_bytes.argtypes = [P]
    lib.gps_plan_device_bytes.restype = ctypes.c_size_t
    lib.gps_plan_destroy.argtypes = [P]
    lib.gps_plan_destroy.restype = None
    lib.gps_solve_generalized.argtypes = [P, P, P, P, D]
    lib.gps_solve_generalized.restype = I
    lib.gps_solve_pb.argtypes = [P, P, P, ctypes.POINTER(gps_ions), P, D]
    lib.gps_solve_pb.restype = I
    lib.gps_solve_vacuum.argtypes = [P, P, P]
    lib.gps_solve_vacuum.restype = I
    lib.gps_solve_generalized_q.argtypes = [P, P, P, P, P, D]
    lib.gps_solve_generalized_q.restype = I
    lib.gps_solve_sc.argtypes = [P, P, P, P, D, I, D]
    lib.gps_solve_sc.restype = I
    lib.gps_rigid_cavity.argtypes = [P, I, P, D, D, P, P]
    lib.gps_rigid_cavity.restype = I
    lib.gps_polarization_charge.argtypes = [P, P, P, P, P]
    lib.gps_polarization_charge.restype = I
    lib.gps_polarization_charge_noalloc.argtypes = [P, P, P, P, P]
    lib.gps_polarization_charge_noalloc.restype = I
    lib.gps_last_info.argtypes = [P, ctypes.POINTER(gps_info)]
    lib.gps_last_info.restype = I
    lib.gps_last_history.argtypes = [P, ctypes.POINTER(D), I]
    lib.gps_last_history.restype = I
    lib.gps_plan_set_timing.argtypes = [P, I]
    lib.gps_plan_set_timing.restype = I
    lib.gps_plan_timing.argtypes = [P, ctypes.POINTER(D), ctypes.POINTER(ctypes.c_longlong),
                                    ctypes.POINTER(D)]
    lib.gps_plan_timing.restype = I
    lib.gps_status_string.argtypes = [I]
    lib.gps_status_string.restype = ctypes.c_char_p
    SZ = ctypes.POINTER(ctypes.c_size_t)
    lib.gps_plan_footprint.argtypes = [I, I, I, I, I, I, I, I, SZ, SZ, SZ]
    lib.gps_plan_release_buffers.argtypes = [P]
    lib.gps_plan_release_buffers.restype = I
    lib.gps_plan_footprint.restype = I
    lib.gps_server_create.argtypes = [ctypes.POINTER(gps_server_options), ctypes.POINTER(P)]
    lib.gps_server_create.restype = I
    lib.gps_server_submit.argtypes = [P, ctypes.POINTER(gps_request),
                                      ctypes.POINTER(ctypes.c_longlong)]
    lib.gps_server_submit.restype = I
    lib.gps_server_poll.argtypes = [P, ctypes.c_longlong, ctypes.POINTER(gps_result)]
    lib.gps_server_poll.restype = I
    lib.gps_server_wait.argtypes = [P, ctypes.c_longlong, ctypes.POINTER(gps_result)]
    lib.gps_server_wait.restype = I
    lib.gps_server_get_stats.argtypes = [P, ctypes.POINTER(gps_server_stats)]
    lib.gps_server_get_stats.restype = I
    lib.gps_server_destroy.argtypes = [P]
    lib.gps_server_destroy.restype = None
    _lib = lib
    return lib


class GPSError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__("%s: %s (%d)" % (where, STATUS.get(status, "?"), status))


def _ptr(t):
    """Device pointer of a torch tensor (float64, contiguous, on the GPU)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("libgps takes device tensors")
    if not t.is_contiguous():
        raise ValueError("libgps takes contiguous tensors")
    return ctypes.c_void_p(t.data_ptr())


def _check_field(t, shape):
    import torch
    if t.dtype != torch.float64 or tuple(t.shape) != tuple(shape):
        raise ValueError("expected float64 tensor of shape %s, got %s %s"
                         % (shape, t.dtype, tuple(t.shape)))


def gps_plan_create(nx, ny, nz, h, bc):
    lib = load()
    out = ctypes.c_void_p()
    st = lib.gps_plan_create(int(nx), int(ny), int(nz), float(h), int(bc), ctypes.byref(out))
    return st, out


def ions_struct(ions, gamma=None):
    """gps_ions from a dict {Z, c_bulk, c_max, kT, eps_bulk, linear, eta, outer_maxit}."""
    n = len(ions["Z"])
    arr = ctypes.c_double * n
    z = arr(*ions["Z"])
    c = arr(*ions["c_bulk"])
    cm = arr(*ions["c_max"]) if ions.get("c_max") is not None else None
    s = gps_ions(n, z, c, cm, float(ions["kT"]), _ptr(gamma),
                 float(ions.get("eps_bulk", 78.36)), int(bool(ions.get("linear", False))),
                 float(ions.get("eta", 0.3)), int(ions.get("outer_maxit", 100)))
    s._keep = (z, c, cm)     # keep the host arrays alive with the struct
    return s


class Plan:
    """A libgps plan for one grid, spacing and boundary condition."""

    def __init__(self, shape, h, bc, precision="fp64", fd_order=16, maxit=1000,
                 check_every=8, stream=None, refine_every=0, warm_start=False):
        nz, ny, nx = shape
        self.shape = (nz, ny, nx)
        self.h = float(h)
        self.bc = bc
        st, handle = gps_plan_create(nx, ny, nz, h, BC_CODES[bc])
        if st != GPS_OK:
            raise GPSError(st, "gps_plan_create(%d,%d,%d,%g,%s)" % (nx, ny, nz, h, bc))
        self.handle = handle
        self.set_options(precision, fd_order, maxit, check_every, stream, refine_every,
                         warm_start)

    def set_options(self, precision="fp64", fd_order=16, maxit=1000, check_every=8,
                    stream=None, refine_every=0, warm_start=False):
        if stream is None:
            import torch
            stream = torch.cuda.current_stream().cuda_stream
        o = gps_options(PRECISIONS[precision], int(fd_order), int(maxit), int(check_every),
                        ctypes.c_void_p(stream), int(refine_every), int(bool(warm_start)))
        st = load().gps_plan_set_options(self.handle, ctypes.byref(o))
        if st != GPS_OK:
            raise GPSError(st, "gps_plan_set_options")

    def device_bytes(self):
        return int(load().gps_plan_device_bytes(self.handle))

    def release_buffers(self):
        st = load().gps_plan_release_buffers(self.handle)
        if st != GPS_OK:
            raise GPSError(st, "gps_plan_release_buffers")

    def solve_generalized(self, rho, eps, phi, tol):
        for t in (rho, eps, phi):
            _check_field(t, self.shape)
        return load().gps_solve_generalized(self.handle, _ptr(rho), _ptr(eps), _ptr(phi),
                                            float(tol))

    def solve_pb(self, rho, eps, ions, phi, tol, gamma=None):
        for t in (rho, eps, phi):
            _check_field(t, self.shape)
        s = ions_struct(ions, gamma)
        return load().gps_solve_pb(self.handle, _ptr(rho), _ptr(eps), ctypes.byref(s),
                                   _ptr(phi), float(tol))

    def solve_generalized_q(self, rho, eps, q, phi, tol):
        """gps_solve_generalized_q: PCG with a caller-supplied q (Eq. corr)."""
        for t in (rho, eps, q, phi):
            _check_field(t, self.shape)
        return load().gps_solve_generalized_q(self.handle, _ptr(rho), _ptr(eps), _ptr(q),
                                              _ptr(phi), float(tol))

    def solve_sc(self, rho, eps, phi, tol, method="sc", eta=0.6):
        """gps_solve_sc: Algorithm SC (method "sc", mixing eta), PSD with Algorithm
        PCG's step ("psd") or PSD with the step minimizing ||r/eps|| ("psd_weighted")."""
        for t in (rho, eps, phi):
            _check_field(t, self.shape)
        code = {"sc": 0, "psd": 1, "psd_weighted": 2}[method]
        return load().gps_solve_sc(self.handle, _ptr(rho), _ptr(eps), _ptr(phi), float(tol),
                                   code, float(eta))

    def rigid_cavity(self, atoms, delta, eps0, eps, q=None):
        """gps_rigid_cavity: atoms is a device float64 tensor of shape (natoms, 4)."""
        import torch
        if atoms.dtype != torch.float64 or atoms.dim() != 2 or atoms.shape[1] != 4:
            raise ValueError("atoms must be a float64 tensor of shape (natoms, 4)")
        _check_field(eps, self.shape)
        if q is not None:
            _check_field(q, self.shape)
        return load().gps_rigid_cavity(self.handle, int(atoms.shape[0]), _ptr(atoms),
                                       float(delta), float(eps0), _ptr(eps), _ptr(q))

    def polarization_charge(self, rho, eps, phi, rho_pol):
        """gps_polarization_charge (Eqs. rhoiter, remap, rhopol)."""
        for t in (rho, eps, phi, rho_pol):
            _check_field(t, self.shape)
        return load().gps_polarization_charge(self.handle, _ptr(rho), _ptr(eps), _ptr(phi),
                                              _ptr(rho_pol))

    def polarization_charge_noalloc(self, rho, eps, phi, rho_pol):
        """gps_polarization_charge_noalloc: as polarization_charge, with the ln eps
        scratch in the library's static device array (no allocation)."""
        for t in (rho, eps, phi, rho_pol):
            _check_field(t, self.shape)
        return load().gps_polarization_charge_noalloc(self.handle, _ptr(rho), _ptr(eps),
                                                      _ptr(phi), _ptr(rho_pol))

    def solve_vacuum(self, f, u):
        for t in (f, u):
            _check_field(t, self.shape)
        return load().gps_solve_vacuum(self.handle, _ptr(f), _ptr(u))

    def info(self):
        out = gps_info()
        load().gps_last_info(self.handle, ctypes.byref(out))
        return out.as_dict()

    def history(self):
        n = self.info()["history_len"]
        buf = (ctypes.c_double * (4 * max(n, 1)))()
        load().gps_last_history(self.handle, buf, n)
        return [tuple(buf[4 * k: 4 * k + 4]) for k in range(n)]

    def set_timing(self, kind):
        """Time every launch of one pass ("zconv", ...; None switches off)."""
        code = 0 if kind is None else KERNEL_KINDS[kind]
        st = load().gps_plan_set_timing(self.handle, code)
        if st != GPS_OK:
            raise GPSError(st, "gps_plan_set_timing")

    def timing(self):
        ms, n, b = ctypes.c_double(), ctypes.c_longlong(), ctypes.c_double()
        load().gps_plan_timing(self.handle, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(b))
        return {"total_ms": ms.value, "launches": n.value, "bytes_per_launch": b.value}

    def close(self):
        if getattr(self, "handle", None):
            load().gps_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def plan_footprint(shape, bc, precision="mixed", maxit=1000, nonlinear_pb=False, refine=False):
    """(tables, buffers, transient) device bytes of a plan (gps_plan_footprint)."""
    nz, ny, nx = shape
    tb, b, t = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
    st = load().gps_plan_footprint(int(nx), int(ny), int(nz), BC_CODES[bc], PRECISIONS[precision],
                                   int(maxit), int(bool(nonlinear_pb)), int(bool(refine)),
                                   ctypes.byref(tb), ctypes.byref(b), ctypes.byref(t))
    if st != GPS_OK:
        raise GPSError(st, "gps_plan_footprint")
    return tb.value, b.value, t.value


class Server:
    """A libgps server (gps_server_*): queued solves on resident plans.

    submit() keeps references to the request's tensors until its result has
    been taken by poll() or wait()."""

    def __init__(self, budget_bytes=0, max_active=4, precision="mixed", fd_order=16,
                 maxit=1000, batch_slots=4):
        o = gps_server_options(int(budget_bytes), int(max_active), PRECISIONS[precision],
                               int(fd_order), int(maxit), int(batch_slots))
        h = ctypes.c_void_p()
        st = load().gps_server_create(ctypes.byref(o), ctypes.byref(h))
        if st != GPS_OK:
            raise GPSError(st, "gps_server_create")
        self.handle = h
        self._live = {}

    def submit(self, rho, eps, phi, h, bc, tol, ions=None, gamma=None, sync=True, eps_key=0):
        """Queue one solve; returns (status, ticket).  With sync, the current
        torch stream is synchronized first so that the inputs are complete.
        eps_key: 0, or the caller's identity of eps (the warm-start cache)."""
        shape = tuple(rho.shape)
        for t in (rho, eps, phi):
            _check_field(t, shape)
        if sync:
            import torch
            torch.cuda.current_stream().synchronize()
        nz, ny, nx = shape
        s = ions_struct(ions, gamma) if ions is not None else None
        req = gps_request(nx, ny, nz, float(h), BC_CODES[bc], _ptr(rho), _ptr(eps), _ptr(phi),
                          ctypes.pointer(s) if s is not None else None, float(tol),
                          int(eps_key))
        ticket = ctypes.c_longlong()
        st = load().gps_server_submit(self.handle, ctypes.byref(req), ctypes.byref(ticket))
        if st == GPS_OK:
            self._live[ticket.value] = (rho, eps, phi, gamma)
        return st, ticket.value

    def _take(self, fn, ticket):
        out = gps_result()
        st = fn(self.handle, ctypes.c_longlong(ticket), ctypes.byref(out))
        if st == GPS_OK:
            self._live.pop(ticket, None)
            return out.as_dict()
        if st == GPS_PENDING:
            return None
        raise GPSError(st, "gps_server result of ticket %d" % ticket)

    def poll(self, ticket):
        """Result dict once finished, else None."""
        return self._take(load().gps_server_poll, ticket)

    def wait(self, ticket):
        return self._take(load().gps_server_wait, ticket)

    def stats(self):
        out = gps_server_stats()
        load().gps_server_get_stats(self.handle, ctypes.byref(out))
        return out.as_dict()

    def close(self):
        if getattr(self, "handle", None):
            load().gps_server_destroy(self.handle)
            self.handle = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
