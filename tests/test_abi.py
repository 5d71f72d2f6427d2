"""C ABI checks that need no GPU: the library loads, exports every function
declared in include/*.h, and rejects bad arguments before touching the device."""

import ctypes
import os
import re

import numpy as np

import pytest

from paper_2306_12739_amd import dns

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("dns.h", "sno.h")]


def declared_functions():
    names = set()
    for path in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(path).read(), flags=re.S)
        names |= set(re.findall(r"\b((?:dns|sno)_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_expected_api():
    names = declared_functions()
    for required in ("dns_create", "dns_step", "dns_stats", "dns_destroy", "dns_set_state",
                     "dns_get_state", "dns_last_error"):
        assert required in names
    assert set(names) == set(dns.EXPORTED)


def test_library_exports_every_declared_symbol():
    lib = dns.library()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_invalid_arguments_fail_before_the_device():
    lib = dns.library()
    h = ctypes.c_void_p()
    geo = dns.Geometry(0, 1.0, 1.0, 1.0, 0.0)
    assert lib.dns_create(None, 400.0, 16, 33, 16, 2, 0.02, ctypes.byref(h)) == dns.DNS_E_INVALID
    assert lib.dns_create(ctypes.byref(geo), -1.0, 16, 33, 16, 2, 0.02, ctypes.byref(h)) == dns.DNS_E_INVALID
    assert lib.dns_create(ctypes.byref(geo), 400.0, 15, 33, 16, 2, 0.02, ctypes.byref(h)) == dns.DNS_E_INVALID
    assert lib.dns_create(ctypes.byref(geo), 400.0, 16, 3, 16, 2, 0.02, ctypes.byref(h)) == dns.DNS_E_INVALID
    assert lib.dns_create(ctypes.byref(geo), 400.0, 16, 33, 16, 0, 0.02, ctypes.byref(h)) == dns.DNS_E_INVALID
    assert lib.dns_create(ctypes.byref(geo), 400.0, 20, 33, 20, 2, 0.02, ctypes.byref(h)) == dns.DNS_E_UNSUPPORTED
    # non-square grids: only the lane-parallel kernel's pairs are built
    assert lib.dns_create(ctypes.byref(geo), 400.0, 96, 33, 32, 2, 0.02, ctypes.byref(h)) == dns.DNS_E_UNSUPPORTED
    assert lib.dns_create(ctypes.byref(geo), 400.0, 48, 33, 16, 2, 0.02, ctypes.byref(h)) == dns.DNS_E_UNSUPPORTED
    assert h.value is None
    assert b"supported" in lib.dns_last_error(None)
    bad = dns.Geometry(7, 1.0, 1.0, 1.0, 0.0)
    assert lib.dns_create(ctypes.byref(bad), 400.0, 16, 33, 16, 2, 0.02, ctypes.byref(h)) == dns.DNS_E_INVALID


def test_null_handle_calls_are_rejected():
    lib = dns.library()
    assert lib.dns_step(None, 1) == dns.DNS_E_STATE
    assert lib.dns_sync(None) == dns.DNS_E_STATE
    assert lib.dns_stats(None, None) == dns.DNS_E_STATE
    assert lib.dns_set_option(None, dns.OPT_PRECISION, 0) == dns.DNS_E_STATE
    assert lib.dns_set_channels(None, 0, 1, None) == dns.DNS_E_STATE
    assert lib.dns_set_channels_noalloc(None, 0, 1, None) == dns.DNS_E_STATE
    lib.dns_destroy(None)   # NULL-safe


def test_grouped_arguments_rejected_without_gpu():
    lib = dns.library()
    h = ctypes.c_void_p()
    assert lib.dns_create_grouped(None, 1, ctypes.byref(h)) == dns.DNS_E_INVALID
    geo = dns.Geometry(0, 1.75 * np.pi, 1.2 * np.pi, 1.0, 0.0)
    arr = (dns.Group * (dns.MAX_GROUPS + 1))()
    for i in range(dns.MAX_GROUPS + 1):
        arr[i] = dns.Group(geo, 400.0, 16, 33, 16, 2, 0.02)
    assert lib.dns_create_grouped(arr, 0, ctypes.byref(h)) == dns.DNS_E_INVALID
    assert lib.dns_create_grouped(arr, dns.MAX_GROUPS + 1, ctypes.byref(h)) == dns.DNS_E_INVALID
    # a bad group is named in the message, before any device allocation
    bad = (dns.Group * 2)()
    bad[0] = dns.Group(geo, 400.0, 16, 33, 16, 2, 0.02)
    bad[1] = dns.Group(geo, 400.0, 16, 3, 16, 2, 0.02)
    bad_first = (dns.Group * 1)(bad[1])
    assert lib.dns_create_grouped(bad_first, 1, ctypes.byref(h)) == dns.DNS_E_INVALID
    assert b"group 0" in lib.dns_last_error(None)
    assert not h.value
    sub = ctypes.c_void_p()
    assert lib.dns_group_handle(None, 0, ctypes.byref(sub)) == dns.DNS_E_STATE


def test_sno_arguments_rejected_without_gpu():
    lib = dns.library()
    h = ctypes.c_void_p()
    assert lib.sno_create(None, 1, ctypes.byref(h)) == dns.DNS_E_INVALID
    bad = dns.SnoConfig(147, 32, 4, 48, 48, 25, 12, 8)     # modes_x > Mx / 2
    assert lib.sno_create(ctypes.byref(bad), 1, ctypes.byref(h)) == dns.DNS_E_INVALID
    bad = dns.SnoConfig(147, 32, 4, 48, 48, 12, 11, 8)     # odd modes_z
    assert lib.sno_create(ctypes.byref(bad), 1, ctypes.byref(h)) == dns.DNS_E_INVALID
    assert b"invalid" in lib.sno_last_error(None)
    assert lib.sno_sync(None) == dns.DNS_E_STATE
    assert lib.sno_num_params(None) == 0
    lib.sno_destroy(None)
    assert lib.dns_get_channels(None, 0, 1, None) == dns.DNS_E_STATE
    assert lib.dns_set_channels(None, 0, 1, None) == dns.DNS_E_STATE


def test_ny_beyond_mode_lds_is_unsupported_without_gpu():
    lib = dns.library()
    h = ctypes.c_void_p()
    geo = dns.Geometry(0, 1.75 * np.pi, 1.2 * np.pi, 1.0, 0.0)
    assert lib.dns_create(ctypes.byref(geo), 400.0, 16, 255, 16, 2, 0.02, ctypes.byref(h)) == dns.DNS_E_UNSUPPORTED
    assert b"Ny" in lib.dns_last_error(None)


def test_binding_constants_match_the_header():
    text = open(HEADERS[0]).read()
    defs = dict(re.findall(r"#define DNS_((?:OPT|PREC|ADV|VDISC)_[A-Z0-9_]+)\s+(-?\d+)", text))
    assert {"OPT_ADVECTION", "ADV_ADVECTIVE", "ADV_ROTATIONAL"} <= set(defs)
    for name, value in defs.items():
        assert getattr(dns, name) == int(value), name


# ---- dns_check_state: the host rules of dns_set_state (no GPU) -------------------
def _states_used_by_the_gpu_paths():
    from paper_2306_12739_amd import inputs, optimal
    for name, w in inputs.WORKLOADS.items():
        if "Nx" in w:
            yield name, w["flow"], w["Nx"], w["Ny"], w["Nz"], inputs.workload_state(name, ensemble=2)
    for name, w in inputs.GROUPED_WORKLOADS.items():
        for g in w["groups"] if isinstance(w, dict) else w:
            yield name, g["flow"], g["Nx"], g["Ny"], g["Nz"], inputs.group_state(g, members=2)
    ow = optimal.WORKLOAD
    base = optimal.base_flow(ow)
    yield "optimal", ow["flow"], ow["Nx"], ow["Ny"], ow["Nz"], optimal.initial_members(ow, 1, (1, 2), base)


def test_check_state_accepts_the_states_the_drivers_load():
    for name, flow, Nx, Ny, Nz, st in _states_used_by_the_gpu_paths():
        dns.check_state(flow, Nx, Ny, Nz, *st)


def _bad(st, what):
    v, eta, U, W = (a.copy() for a in st)
    if what == "v_herm":
        v[1, 0, 2, 3] += 1e-3                       # (0, 2) no longer conj of (0, -2)
    elif what == "eta_herm":
        eta[0, 0, -1, 0] += 1e-3j
    elif what == "v00":
        v[0, 0, 0, 4] = 1e-3
    elif what == "eta00_imag":
        eta[1, 0, 0, 2] = 1e-3j
    elif what == "U_wall_nan":
        U[1, 0] = np.nan
    elif what == "W_wall":
        W[0, -1] = 1e-6
    elif what == "column_nan":
        v[0, 0, 1, 1] = np.nan
    return v, eta, U, W


@pytest.mark.parametrize("what,rule", [
    ("v_herm", "v_hat: the n_x = 0 column is not Hermitian"),
    ("eta_herm", "eta_hat: the n_x = 0 column is not Hermitian"),
    ("v00", "v_hat: the (0,0) mode is not zero"),
    ("eta00_imag", "eta_hat: the (0,0) mode is not zero"),
    ("U_wall_nan", "wall values"),
    ("W_wall", "wall values"),
    ("column_nan", "v_hat"),
])
def test_check_state_rejects_each_broken_rule(what, rule):
    from paper_2306_12739_amd import inputs
    w = inputs.WORKLOADS["couette-re400-16x33x16-e2"]
    st = inputs.workload_state("couette-re400-16x33x16-e2")
    dns.check_state(w["flow"], w["Nx"], w["Ny"], w["Nz"], *st)
    with pytest.raises(dns.DnsError) as ei:
        dns.check_state(w["flow"], w["Nx"], w["Ny"], w["Nz"], *_bad(st, what))
    assert ei.value.code == dns.DNS_E_INVALID
    assert rule in str(ei.value), str(ei.value)


def test_check_state_leaves_other_modes_free():
    """A NaN outside the n_x = 0 column is accepted (the step flags the member)."""
    from paper_2306_12739_amd import inputs
    w = inputs.WORKLOADS["couette-re400-16x33x16-e2"]
    v, eta, U, W = inputs.workload_state("couette-re400-16x33x16-e2")
    v[1, 1, 2, 5] = np.nan
    dns.check_state(w["flow"], w["Nx"], w["Ny"], w["Nz"], v, eta, U, W)
    with pytest.raises(dns.DnsError):     # a channel's walls are at rest
        dns.check_state(1, w["Nx"], w["Ny"], w["Nz"], v, eta, U, W)
