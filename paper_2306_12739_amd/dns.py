"""ctypes binding of libdns_ensemble.so (the C ABI declared in include/dns.h).

Argument marshalling only: every step of the solver runs in the HIP library.
Host arrays are numpy; device arrays may be torch CUDA tensors (their
``data_ptr()`` is passed with ``on_device=1``).  There is no CPU fallback:
opening the library fails loudly when it is missing or was built for another
machine.
"""

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdns_ensemble.so")

DNS_OK = 0
DNS_E_INVALID = -1
DNS_E_NOMEM = -2
DNS_E_HIP = -3
DNS_E_NONFINITE = -4
DNS_E_UNSUPPORTED = -5
DNS_E_STATE = -6

COUETTE = 0
POISEUILLE = 1

OPT_PRECISION = 1
OPT_STREAM = 2
OPT_GRAPH = 3
OPT_STATS = 4
OPT_PLANE_ROWS = 5
OPT_MODE_TILE = 6
OPT_CHAINS = 7
OPT_ADVECTION = 8
OPT_SHARED_MEAN = 9
OPT_QUASILINEAR = 10
OPT_FROZEN_MEAN = 11
OPT_V_DISCRETIZATION = 12
OPT_GROUP_STREAMS = 13

VDISC_CLAMPED = 0
VDISC_KMM = 1

ADV_ADVECTIVE = 0
ADV_ROTATIONAL = 1

PREC_FP64 = 0
PREC_MIXED_FP32 = 1
PREC_MIXED_3XBF16 = 2
PREC_MIXED_FP32MM = 3

EXPORTED = ["dns_create", "dns_set_option", "dns_set_state", "dns_get_state", "dns_step",
            "dns_stats", "dns_stats_reset", "dns_sync", "dns_destroy", "dns_last_error",
            "dns_debug_stage0", "dns_kernel_times", "dns_host_operators",
            "dns_create_grouped", "dns_group_handle", "dns_tune",
            "dns_get_channels", "dns_set_channels", "dns_set_channels_noalloc", "dns_set_forcing",
            "dns_perturbation_energy", "dns_orthonormalize", "dns_check_state",
            "sno_create", "sno_set_option", "sno_num_params", "sno_set_params", "sno_get_params",
            "sno_forward", "sno_loss_grad", "sno_train_step", "sno_sync", "sno_last_error",
            "sno_destroy"]

SNO_MATH_BF16 = 0
SNO_MATH_FP32 = 1
SNO_OPT_MATH = 1
SNO_OPT_STREAM = 2

MAX_GROUPS = 16


class Geometry(ctypes.Structure):
    _fields_ = [("flow", ctypes.c_int), ("Lx", ctypes.c_double), ("Lz", ctypes.c_double),
                ("Uw", ctypes.c_double), ("flux", ctypes.c_double)]


class StateView(ctypes.Structure):
    _fields_ = [("v_hat", ctypes.c_void_p), ("eta_hat", ctypes.c_void_p),
                ("U00", ctypes.c_void_p), ("W00", ctypes.c_void_p), ("on_device", ctypes.c_int)]


class Group(ctypes.Structure):
    _fields_ = [("g", Geometry), ("Re", ctypes.c_double), ("Nx", ctypes.c_int),
                ("Ny", ctypes.c_int), ("Nz", ctypes.c_int), ("members", ctypes.c_int),
                ("dt", ctypes.c_double)]


class SnoConfig(ctypes.Structure):
    _fields_ = [("channels", ctypes.c_int), ("width", ctypes.c_int), ("layers", ctypes.c_int),
                ("Mx", ctypes.c_int), ("Mz", ctypes.c_int), ("modes_x", ctypes.c_int),
                ("modes_z", ctypes.c_int), ("max_batch", ctypes.c_int)]


class SnoAdamW(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float), ("weight_decay", ctypes.c_float)]


class Tuning(ctypes.Structure):
    _fields_ = [("plane_rows", ctypes.c_int), ("mode_members", ctypes.c_int),
                ("plane_ms", ctypes.c_double), ("mode_ms", ctypes.c_double),
                ("from_cache", ctypes.c_int)]


def _tuning_dict(t):
    return {"plane_rows": t.plane_rows, "mode_members": t.mode_members, "plane_ms": t.plane_ms,
            "mode_ms": t.mode_ms, "from_cache": bool(t.from_cache)}


_DP = ctypes.POINTER(ctypes.c_double)
_IP = ctypes.POINTER(ctypes.c_int)


class StatsOut(ctypes.Structure):
    _fields_ = [("energy", _DP), ("dissipation", _DP), ("power", _DP), ("flux", _DP),
                ("gamma", _DP), ("div_max", _DP), ("tau_lower", _DP), ("tau_upper", _DP),
                ("failed", _IP), ("U", _DP), ("W", _DP), ("urms", _DP), ("vrms", _DP),
                ("wrms", _DP), ("uv", _DP), ("tau_w", ctypes.c_double),
                ("re_tau", ctypes.c_double), ("samples", ctypes.c_longlong),
                ("steps", ctypes.c_longlong), ("member_profiles", _DP), ("member_tau", _DP)]


_lib = None


def library(path=LIB_PATH):
    """Open the HIP library (once).  Raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2306_12739_amd.build`")
    # torch ships its own HIP runtime under the same soname as the system one;
    # loading torch first makes the library bind to that one, so a process
    # holds a single runtime (with the library loaded first, torch later finds
    # no device)
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    vp = ctypes.c_void_p
    lib.dns_create.argtypes = [ctypes.POINTER(Geometry), ctypes.c_double, ctypes.c_int, ctypes.c_int,
                               ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.POINTER(vp)]
    lib.dns_set_option.argtypes = [vp, ctypes.c_int, ctypes.c_longlong]
    lib.dns_set_state.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(StateView)]
    lib.dns_get_state.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(StateView)]
    lib.dns_check_state.argtypes = [ctypes.POINTER(Geometry), ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_int, ctypes.POINTER(StateView)]
    lib.dns_step.argtypes = [vp, ctypes.c_int]
    lib.dns_stats.argtypes = [vp, ctypes.POINTER(StatsOut)]
    lib.dns_stats_reset.argtypes = [vp]
    lib.dns_sync.argtypes = [vp]
    lib.dns_destroy.argtypes = [vp]
    lib.dns_destroy.restype = None
    lib.dns_last_error.argtypes = [vp]
    lib.dns_last_error.restype = ctypes.c_char_p
    lib.dns_debug_stage0.argtypes = [vp, _DP, _DP, _DP]
    lib.dns_kernel_times.argtypes = [vp, ctypes.c_int, _DP, _DP]
    lib.dns_create_grouped.argtypes = [ctypes.POINTER(Group), ctypes.c_int, ctypes.POINTER(vp)]
    lib.dns_group_handle.argtypes = [vp, ctypes.c_int, ctypes.POINTER(vp)]
    lib.dns_tune.argtypes = [vp, ctypes.c_char_p, ctypes.POINTER(Tuning)]
    lib.dns_get_channels.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp]
    lib.dns_set_channels.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp]
    lib.dns_set_channels_noalloc.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp]
    lib.dns_set_forcing.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp, vp, ctypes.c_int]
    lib.dns_perturbation_energy.argtypes = [vp, _DP]
    lib.dns_orthonormalize.argtypes = [vp]
    lib.sno_create.argtypes = [ctypes.POINTER(SnoConfig), ctypes.c_ulonglong, ctypes.POINTER(vp)]
    lib.sno_set_option.argtypes = [vp, ctypes.c_int, ctypes.c_longlong]
    lib.sno_num_params.argtypes = [vp]
    lib.sno_num_params.restype = ctypes.c_longlong
    lib.sno_set_params.argtypes = [vp, vp, ctypes.c_longlong]
    lib.sno_get_params.argtypes = [vp, vp, ctypes.c_longlong]
    lib.sno_forward.argtypes = [vp, vp, vp, ctypes.c_int]
    lib.sno_loss_grad.argtypes = [vp, vp, vp, ctypes.c_int, ctypes.POINTER(ctypes.c_float), vp]
    lib.sno_train_step.argtypes = [vp, vp, vp, ctypes.c_int, ctypes.POINTER(SnoAdamW),
                                   ctypes.POINTER(ctypes.c_float)]
    lib.sno_sync.argtypes = [vp]
    lib.sno_last_error.argtypes = [vp]
    lib.sno_last_error.restype = ctypes.c_char_p
    lib.sno_destroy.argtypes = [vp]
    lib.sno_destroy.restype = None
    lib.dns_host_operators.argtypes = [ctypes.POINTER(Geometry), ctypes.c_double, ctypes.c_int,
                                       ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                       ctypes.c_int, _DP, _DP, _DP, _DP, _DP, _DP, _DP]
    for name in EXPORTED:
        if name not in ("dns_destroy", "dns_last_error", "sno_destroy", "sno_last_error",
                        "sno_num_params"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def check_state(flow, Nx, Ny, Nz, v, eta, U, W, Uw=1.0):
    """dns_check_state on host arrays (no GPU needed); raises DnsError with
    the library's message when a member breaks a rule of dns_set_state."""
    lib = library()
    v = np.ascontiguousarray(v, dtype=np.complex128)
    eta = np.ascontiguousarray(eta, dtype=np.complex128)
    U = np.ascontiguousarray(U, dtype=np.float64)
    W = np.ascontiguousarray(W, dtype=np.float64)
    sv = StateView(v.ctypes.data, eta.ctypes.data, U.ctypes.data, W.ctypes.data, 0)
    g = Geometry(flow, 1.0, 1.0, Uw, 0.0)
    rc = lib.dns_check_state(ctypes.byref(g), Nx, Ny, Nz, v.shape[0], ctypes.byref(sv))
    if rc != DNS_OK:
        raise DnsError(rc, lib.dns_last_error(None).decode())


def host_operators(flow, Re, Lx, Lz, Nx, Ny, Nz, dt, h_index, Uw=1.0, v_discretization=0):
    """Operators as built by the library's host builder (no GPU needed)."""
    lib = library()
    N = Ny - 2
    G = (Nx // 2) * (Nz // 2)
    out = {"ops": np.zeros((G, 4, N, N)), "mean_ops": np.zeros((2, N, N)), "lift": np.zeros(N),
           "green": np.zeros(N), "D1": np.zeros((Ny, Ny)), "D1c": np.zeros((Ny, N)),
           "ccw": np.zeros(Ny)}
    g = Geometry(flow, Lx, Lz, Uw, 0.0)
    rc = lib.dns_host_operators(ctypes.byref(g), Re, Nx, Ny, Nz, dt, h_index, v_discretization,
                                *[_ptr(out[k]) for k in ("ops", "mean_ops", "lift", "green",
                                                         "D1", "D1c", "ccw")])
    if rc != DNS_OK:
        raise DnsError(rc, lib.dns_last_error(None).decode())
    return out


class DnsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"dns error {code}: {msg}")
        self.code = code


def _ptr(a):
    return a.ctypes.data_as(_DP) if a is not None else None


class Ensemble:
    """One ensemble of flows sharing grid, box, Re and dt (include/dns.h)."""

    def __init__(self, flow, Re, Lx, Lz, Nx, Ny, Nz, ensemble, dt, Uw=1.0, flux=0.0,
                 _borrowed=None):
        self.lib = library()
        self.flow, self.Re, self.Lx, self.Lz = flow, Re, Lx, Lz
        self.Nx, self.Ny, self.Nz, self.E, self.dt = Nx, Ny, Nz, ensemble, dt
        self.owned = _borrowed is None
        if not self.owned:  # a group's handle, owned by its GroupedEnsemble
            self.h = _borrowed
            return
        self.h = ctypes.c_void_p()
        g = Geometry(flow, Lx, Lz, Uw, flux)
        rc = self.lib.dns_create(ctypes.byref(g), Re, Nx, Ny, Nz, ensemble, dt, ctypes.byref(self.h))
        if rc != DNS_OK:
            raise DnsError(rc, self.lib.dns_last_error(None).decode())

    # ---- helpers ---------------------------------------------------------------
    def _check(self, rc):
        if rc != DNS_OK:
            raise DnsError(rc, self.lib.dns_last_error(self.h).decode())
        return rc

    def close(self):
        if self.h and self.owned:
            self.lib.dns_destroy(self.h)
        self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def shape_spec(self):
        return (self.Nx // 2, self.Nz - 1, self.Ny - 2)

    # ---- C ABI calls -------------------------------------------------------------
    def set_option(self, key, value):
        return self._check(self.lib.dns_set_option(self.h, key, int(value)))

    def set_precision(self, prec):
        return self.set_option(OPT_PRECISION, prec)

    def set_advection(self, form):
        return self.set_option(OPT_ADVECTION, form)

    def set_stream(self, stream):
        """stream: a torch.cuda.Stream (or its integer handle)."""
        handle = getattr(stream, "cuda_stream", stream)
        return self.set_option(OPT_STREAM, int(handle))

    def set_state(self, v, eta, U, W, member0=0):
        """Host numpy arrays in the state layout of include/dns.h."""
        v = np.ascontiguousarray(v, dtype=np.complex128)
        eta = np.ascontiguousarray(eta, dtype=np.complex128)
        U = np.ascontiguousarray(U, dtype=np.float64)
        W = np.ascontiguousarray(W, dtype=np.float64)
        count = v.shape[0]
        if v.shape[1:] != self.shape_spec or eta.shape != v.shape or U.shape != (count, self.Ny) \
                or W.shape != U.shape:
            raise ValueError("state arrays do not match the grid")
        sv = StateView(v.ctypes.data, eta.ctypes.data, U.ctypes.data, W.ctypes.data, 0)
        return self._check(self.lib.dns_set_state(self.h, member0, count, ctypes.byref(sv)))

    def set_forcing(self, f_lapv=None, f_eta=None, member0=0):
        """Additive (Lap v, eta) forcing, host arrays in the state layout of
        v/eta (None: zero); both None turns the forcing off."""
        if f_lapv is None and f_eta is None:
            return self._check(self.lib.dns_set_forcing(self.h, member0, 0, None, None, 0))
        arrs = [None if f is None else np.ascontiguousarray(f, dtype=np.complex128) for f in (f_lapv, f_eta)]
        count = next(a.shape[0] for a in arrs if a is not None)
        for a in arrs:
            if a is not None and a.shape != (count,) + self.shape_spec:
                raise ValueError("forcing arrays do not match the grid")
        ptrs = [None if a is None else a.ctypes.data for a in arrs]
        return self._check(self.lib.dns_set_forcing(self.h, member0, count, ptrs[0], ptrs[1], 0))

    def perturbation_energy(self):
        out = np.zeros(self.E)
        self._check(self.lib.dns_perturbation_energy(self.h, out.ctypes.data_as(_DP)))
        return out

    def orthonormalize(self):
        return self._check(self.lib.dns_orthonormalize(self.h))

    def set_state_device(self, v, eta, U, W, member0=0):
        """torch device tensors (complex128 / float64, contiguous)."""
        count = v.shape[0]
        sv = StateView(v.data_ptr(), eta.data_ptr(), U.data_ptr(), W.data_ptr(), 1)
        return self._check(self.lib.dns_set_state(self.h, member0, count, ctypes.byref(sv)))

    def get_state(self, member0=0, count=None):
        count = self.E - member0 if count is None else count
        v = np.zeros((count,) + self.shape_spec, dtype=np.complex128)
        eta = np.zeros_like(v)
        U = np.zeros((count, self.Ny))
        W = np.zeros_like(U)
        sv = StateView(v.ctypes.data, eta.ctypes.data, U.ctypes.data, W.ctypes.data, 0)
        self._check(self.lib.dns_get_state(self.h, member0, count, ctypes.byref(sv)))
        return v, eta, U, W

    def step(self, nsteps=1):
        return self._check(self.lib.dns_step(self.h, int(nsteps)))

    def sync(self):
        return self._check(self.lib.dns_sync(self.h))

    def stats_reset(self):
        return self._check(self.lib.dns_stats_reset(self.h))

    # member_profiles rows: U00, W00, U00^2, W00^2 and the plane means of u^2,
    # v^2, w^2, u v (mean flow included), each a time average per member
    MEMBER_PROFILES = ("U", "W", "U2", "W2", "uu", "vv", "ww", "uv")

    def stats(self, allow_nonfinite=False):
        """Diagnostics and statistics (dns_stats).  'member_profiles' is
        (E, 8, Ny) in the order of MEMBER_PROFILES, 'member_tau' (E, 2)."""
        E, My = self.E, self.Ny
        out = {k: np.zeros(E) for k in ("energy", "dissipation", "power", "flux", "gamma",
                                         "div_max", "tau_lower", "tau_upper")}
        out["failed"] = np.zeros(E, dtype=np.int32)
        for k in ("U", "W", "urms", "vrms", "wrms", "uv"):
            out[k] = np.zeros(My)
        out["member_profiles"] = np.zeros((E, 8, My))
        out["member_tau"] = np.zeros((E, 2))
        so = StatsOut()
        for k, arr in out.items():
            setattr(so, k, arr.ctypes.data_as(_IP if k == "failed" else _DP))
        rc = self.lib.dns_stats(self.h, ctypes.byref(so))
        if rc != DNS_OK and not (allow_nonfinite and rc == DNS_E_NONFINITE):
            self._check(rc)
        out["tau_w"], out["re_tau"] = so.tau_w, so.re_tau
        out["samples"], out["steps"] = so.samples, so.steps
        out["rc"] = rc
        return out

    def get_channels(self, out, member0=0):
        """Channel form of members [member0, member0 + len(out)) into a float32
        CUDA tensor ``out`` of shape (count, 3 Ny, Mz Mx) (include/sno.h)."""
        self._check_channels(out)
        return self._check(self.lib.dns_get_channels(self.h, member0, out.shape[0], out.data_ptr()))

    def set_channels(self, x, member0=0):
        """Rebuild members' states from channel-form data (float32 CUDA tensor)."""
        self._check_channels(x)
        return self._check(self.lib.dns_set_channels(self.h, member0, x.shape[0], x.data_ptr()))

    def set_channels_noalloc(self, x, member0=0):
        """As set_channels, without allocating: intermediates in the library's
        fixed per-GPU scratch; queued on the handle's stream, not synchronised."""
        self._check_channels(x)
        return self._check(self.lib.dns_set_channels_noalloc(self.h, member0, x.shape[0], x.data_ptr()))

    def _check_channels(self, t):
        P = (3 * self.Nx // 2) * (3 * self.Nz // 2)
        if tuple(t.shape[1:]) != (3 * self.Ny, P) or str(t.dtype) != "torch.float32" \
                or not t.is_cuda or not t.is_contiguous():
            raise ValueError("channel tensors are contiguous float32 CUDA (count, 3 Ny, Mz Mx)")

    def tune(self, cache_path=None):
        """Pick the fastest plane chunk rows and mode member tile (dns_tune)."""
        t = Tuning()
        path = None if cache_path is None else os.fsencode(cache_path)
        self._check(self.lib.dns_tune(self.h, path, ctypes.byref(t)))
        return _tuning_dict(t)

    def kernel_times(self, nreps=10):
        """(plane_ms, mode_ms): average device time per launch, HIP events."""
        p = ctypes.c_double()
        m = ctypes.c_double()
        self._check(self.lib.dns_kernel_times(self.h, int(nreps), ctypes.byref(p), ctypes.byref(m)))
        return p.value, m.value

    def debug_stage0(self):
        E, My, L, NZ = self.E, self.Ny, self.Nx // 2, self.Nz - 1
        vel = np.zeros((5, E, My, L, NZ), dtype=np.complex128)
        nl = np.zeros((3, E, My, L, NZ), dtype=np.complex128)
        means = np.zeros((2, E, My))
        self._check(self.lib.dns_debug_stage0(
            self.h, vel.view(np.float64).ctypes.data_as(_DP),
            nl.view(np.float64).ctypes.data_as(_DP), _ptr(means)))
        return vel, nl, means


class GroupedEnsemble:
    """Several ensembles (different Re, grid, box, dt) advanced by one step call
    (dns_create_grouped).  ``groups``: list of dicts with keys flow, Re, Lx, Lz,
    Nx, Ny, Nz, members, dt and optionally Uw, flux.  Members are numbered
    group-major; ``self.groups[g]`` is group g's Ensemble (owned by this object)."""

    def __init__(self, groups):
        self.lib = library()
        self.specs = [dict(g) for g in groups]
        arr = (Group * len(groups))()
        for i, g in enumerate(groups):
            arr[i] = Group(Geometry(g["flow"], g["Lx"], g["Lz"], g.get("Uw", 1.0), g.get("flux", 0.0)),
                           g["Re"], g["Nx"], g["Ny"], g["Nz"], g["members"], g["dt"])
        self.h = ctypes.c_void_p()
        rc = self.lib.dns_create_grouped(arr, len(groups), ctypes.byref(self.h))
        if rc != DNS_OK:
            raise DnsError(rc, self.lib.dns_last_error(None).decode())
        self.base = list(np.cumsum([0] + [g["members"] for g in groups[:-1]]))
        self.E = int(sum(g["members"] for g in groups))
        self.groups = []
        for i, g in enumerate(groups):
            sub = ctypes.c_void_p()
            self._check(self.lib.dns_group_handle(self.h, i, ctypes.byref(sub)))
            self.groups.append(Ensemble(g["flow"], g["Re"], g["Lx"], g["Lz"], g["Nx"], g["Ny"],
                                        g["Nz"], g["members"], g["dt"], _borrowed=sub))

    def _check(self, rc):
        if rc != DNS_OK:
            raise DnsError(rc, self.lib.dns_last_error(self.h).decode())
        return rc

    def close(self):
        for g in getattr(self, "groups", []):
            g.h = ctypes.c_void_p()
        if self.h:
            self.lib.dns_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_option(self, key, value):
        return self._check(self.lib.dns_set_option(self.h, key, int(value)))

    def set_precision(self, prec):
        return self.set_option(OPT_PRECISION, prec)

    def set_advection(self, form):
        return self.set_option(OPT_ADVECTION, form)

    def set_stream(self, stream):
        handle = getattr(stream, "cuda_stream", stream)
        return self.set_option(OPT_STREAM, int(handle))

    def set_state(self, v, eta, U, W, member0):
        """State of members [member0, member0 + len(v)), inside one group, through
        the grouped handle (global member numbers)."""
        g = int(np.searchsorted(self.base, member0, side="right") - 1)
        ens = self.groups[g]
        v = np.ascontiguousarray(v, dtype=np.complex128)
        eta = np.ascontiguousarray(eta, dtype=np.complex128)
        U = np.ascontiguousarray(U, dtype=np.float64)
        W = np.ascontiguousarray(W, dtype=np.float64)
        if v.shape[1:] != ens.shape_spec or U.shape != (v.shape[0], ens.Ny):
            raise ValueError("state arrays do not match the group's grid")
        sv = StateView(v.ctypes.data, eta.ctypes.data, U.ctypes.data, W.ctypes.data, 0)
        return self._check(self.lib.dns_set_state(self.h, member0, v.shape[0], ctypes.byref(sv)))

    def get_state(self, member0, count):
        g = int(np.searchsorted(self.base, member0, side="right") - 1)
        ens = self.groups[g]
        v = np.zeros((count,) + ens.shape_spec, dtype=np.complex128)
        eta = np.zeros_like(v)
        U = np.zeros((count, ens.Ny))
        W = np.zeros_like(U)
        sv = StateView(v.ctypes.data, eta.ctypes.data, U.ctypes.data, W.ctypes.data, 0)
        self._check(self.lib.dns_get_state(self.h, member0, count, ctypes.byref(sv)))
        return v, eta, U, W

    def step(self, nsteps=1):
        return self._check(self.lib.dns_step(self.h, int(nsteps)))

    def sync(self):
        return self._check(self.lib.dns_sync(self.h))

    def stats_reset(self):
        return self._check(self.lib.dns_stats_reset(self.h))

    def tune(self, cache_path=None):
        """Tune every group; one dict per group."""
        arr = (Tuning * len(self.groups))()
        path = None if cache_path is None else os.fsencode(cache_path)
        self._check(self.lib.dns_tune(self.h, path, arr))
        return [_tuning_dict(t) for t in arr]

    def stats(self, allow_nonfinite=False):
        """Per-member diagnostics over all groups (group-major)."""
        E = self.E
        out = {k: np.zeros(E) for k in ("energy", "dissipation", "power", "flux", "gamma",
                                         "div_max", "tau_lower", "tau_upper")}
        out["failed"] = np.zeros(E, dtype=np.int32)
        out["member_tau"] = np.zeros((E, 2))
        so = StatsOut()
        for k, arr in out.items():
            setattr(so, k, arr.ctypes.data_as(_IP if k == "failed" else _DP))
        rc = self.lib.dns_stats(self.h, ctypes.byref(so))
        if rc != DNS_OK and not (allow_nonfinite and rc == DNS_E_NONFINITE):
            self._check(rc)
        out["samples"], out["steps"], out["rc"] = so.samples, so.steps, rc
        return out


class SNO:
    """Spectral neural operator of the learned spin-up (include/sno.h).  Tensors
    are contiguous float32 CUDA tensors of shape (batch, channels, Mx Mz)."""

    def __init__(self, channels, width=32, layers=4, Mx=48, Mz=48, modes_x=12, modes_z=12,
                 max_batch=32, seed=0):
        self.lib = library()
        self.cfg = SnoConfig(channels, width, layers, Mx, Mz, modes_x, modes_z, max_batch)
        self.h = ctypes.c_void_p()
        rc = self.lib.sno_create(ctypes.byref(self.cfg), int(seed), ctypes.byref(self.h))
        if rc != DNS_OK:
            raise DnsError(rc, self.lib.sno_last_error(None).decode())
        self.num_params = int(self.lib.sno_num_params(self.h))

    def _check(self, rc):
        if rc != DNS_OK:
            raise DnsError(rc, self.lib.sno_last_error(self.h).decode())
        return rc

    def close(self):
        if self.h:
            self.lib.sno_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_math(self, math):
        return self._check(self.lib.sno_set_option(self.h, SNO_OPT_MATH, int(math)))

    def set_stream(self, stream):
        handle = getattr(stream, "cuda_stream", stream)
        return self._check(self.lib.sno_set_option(self.h, SNO_OPT_STREAM, int(handle)))

    def get_params(self):
        out = np.zeros(self.num_params, dtype=np.float32)
        self._check(self.lib.sno_get_params(self.h, out.ctypes.data, self.num_params))
        return out

    def set_params(self, theta):
        theta = np.ascontiguousarray(theta, dtype=np.float32)
        if theta.size != self.num_params:
            raise ValueError("parameter count mismatch")
        return self._check(self.lib.sno_set_params(self.h, theta.ctypes.data, self.num_params))

    def _t(self, t):
        if str(t.dtype) != "torch.float32" or not t.is_cuda or not t.is_contiguous() \
                or tuple(t.shape[1:]) != (self.cfg.channels, self.cfg.Mx * self.cfg.Mz):
            raise ValueError("SNO tensors are contiguous float32 CUDA (batch, channels, Mx Mz)")
        return t.data_ptr()

    def forward(self, x, y):
        return self._check(self.lib.sno_forward(self.h, self._t(x), self._t(y), x.shape[0]))

    def loss_grad(self, x, target, want_grad=True):
        loss = ctypes.c_float()
        grad = np.zeros(self.num_params, dtype=np.float32) if want_grad else None
        self._check(self.lib.sno_loss_grad(self.h, self._t(x), self._t(target), x.shape[0],
                                           ctypes.byref(loss),
                                           grad.ctypes.data if want_grad else None))
        return loss.value, grad

    def train_step(self, x, target, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=1e-4,
                   want_loss=True):
        opt = SnoAdamW(lr, beta1, beta2, eps, weight_decay)
        loss = ctypes.c_float()
        self._check(self.lib.sno_train_step(self.h, self._t(x), self._t(target), x.shape[0],
                                            ctypes.byref(opt),
                                            ctypes.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def sync(self):
        return self._check(self.lib.sno_sync(self.h))
