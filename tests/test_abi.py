"""The C-ABI library builds for gfx950, loads, exports every function that
include/gempic.h declares, and rejects invalid configurations before touching
a device (so these run on the CPU)."""
import ctypes
import math
import os
import re

import pytest

import workloads
from paper_2509_16793_amd import gempic as gp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for f in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if f.endswith(".h"):
            src = open(os.path.join(ROOT, "include", f)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(gempic_[a-z_]+)\s*\(", src))
    return sorted(names)


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert "gempic_create" in names and "gempic_step" in names and "gempic_dn_train" in names
    L = gp.lib()
    for n in names:
        assert hasattr(L, n), n
    # and the binding marshals each of them
    assert set(names) <= set(gp._SIGS)


def test_struct_layout_matches_header():
    # offsets follow C alignment rules; the stream pointer is the last member
    c = gp.gempic_config
    assert c.stream.offset % 8 == 0
    assert ctypes.sizeof(c) == c.stream.offset + 8
    assert ctypes.sizeof(gp.gempic_diag) == 72


def _create(cfg, **kw):
    c = gp.make_config(cfg)
    for k, v in kw.items():
        setattr(c, k, v)
    h = ctypes.c_void_p()
    rc = gp.lib().gempic_create(ctypes.byref(c), ctypes.byref(h))
    return rc, h


def test_rejects_too_large_slow_step():
    cfg = workloads.lwfa2d_fp64()
    cfg["dtau"] = 0.04          # > h / 2 = 0.025 (config units)
    rc, h = _create(cfg)
    assert rc == -4 and not h.value
    assert b"2 dtau" in gp.lib().gempic_last_error(None)


def test_rejects_stability_bound():
    cfg = workloads.lwfa2d_fp64()
    cfg["n_e"] = 1e6            # Delta * h > 4 / omega_p^2
    rc, _ = _create(cfg)
    assert rc == -4


@pytest.mark.parametrize("field,value,code", [
    ("abi_version", 99, -7), ("dims", 4, -1), ("precision", 7, -1), ("filter_passes", 3, -1)])
def test_rejects_bad_fields(field, value, code):
    rc, _ = _create(workloads.lwfa2d_fp64(), **{field: value})
    assert rc == code


def test_rejects_non_power_of_two_and_bad_tile():
    cfg = workloads.lwfa2d_fp64()
    cfg["n"] = [60, 1, 256]
    assert _create(cfg)[0] == -1
    cfg = workloads.lwfa2d_fp64()
    cfg["tile"] = [6, 1, 8]
    assert _create(cfg)[0] == -1


def test_rejects_transverse_grid_beyond_lds_transforms():
    # rows longer than 512 nodes are beyond the sizes the transverse
    # transforms are tested at; both precisions and both axes are rejected
    cfg = workloads.lwfa2d_fp64()
    cfg["n"] = [1024, 1, 256]
    rc, _ = _create(cfg)
    assert rc == -1
    assert b"transverse grid too large" in gp.lib().gempic_last_error(None)
    cfg["precision"] = "fp32"
    assert _create(cfg)[0] == -1
    cfg3 = workloads.small3d(precision="fp32", n=(16, 1024, 16))
    assert _create(cfg3)[0] == -1


def test_rejects_capacity_beyond_int32_indices():
    # the PWFA grid at 8 ppc needs about 2.7e9 particle slots: rejected before
    # any device allocation (particle indices are int32)
    cfg = workloads.pwfa3d_fp32()
    cfg["ppc"] = [2, 2, 2]
    cfg["beam"] = None
    rc, h = _create(cfg)
    assert rc == -1 and not h.value
    assert b"2^31" in gp.lib().gempic_last_error(None)


def test_strerror():
    for code in range(0, -9, -1):
        assert gp.lib().gempic_strerror(code)


def test_denoiser_parameter_count_and_rejections():
    L = gp.lib()
    assert L.gempic_dn_nparams() == 30307
    h = ctypes.c_void_p()
    assert L.gempic_dn_create(None, 30307, None, ctypes.byref(h)) == -1 and not h.value
    assert L.gempic_dn_create(None, 5, None, ctypes.byref(h)) == -1
    assert L.gempic_dn_apply(None, None, None, 1.0, None, 1, 1e-3, None, None, None, None) == -1
    assert L.gempic_set_denoiser(None, None, 1e-3) == -1


def _march(**kw):
    cfg = workloads.small3d(precision="fp64", n=(16, 16, 32))
    cfg.update(scheme=1, delta=0.5)
    cfg.update(kw)
    return cfg


@pytest.mark.parametrize("change,why", [
    (dict(scheme=3), b"scheme"), (dict(delta=0.0), b"delta > 0"), (dict(precision="fp32abs"), b"FP64 or FP32_CELL"),
    (dict(beam=dict(n=1.0, sr=0.3, sz=0.3, gamma=100.0, np=10)), b"driver beam"),
    (dict(n_e=1e3, delta=50.0), b"4/omega_p^2"), (dict(ch_ratio=0.5, ch_radius=0.0), b"channel"),
    (dict(zeta_nodes=[0.0] + [0.05] * 32), b"increase"), (dict(zeta_nodes=[0.1 * k + 0.1 for k in range(33)]), b"start at 0")])
def test_zeta_march_rejections(change, why):
    cfg = _march(**change)
    rc, h = _create(cfg)
    assert rc in (-1, -4) and not h.value
    assert why in gp.lib().gempic_last_error(None)


def test_zeta_march_rejects_deposit_rho():
    c = gp.make_config(_march(), deposit_rho=True)
    h = ctypes.c_void_p()
    assert gp.lib().gempic_create(ctypes.byref(c), ctypes.byref(h)) == -1
    assert b"deposit_rho" in gp.lib().gempic_last_error(None)
