"""Thin ctypes binding of the gfx950 Galilean PIC library (include/gempic.h,
include/gempic_denoise.h).

Argument marshalling only: every step of the path runs in the HIP library.
The functions keep the C names (gempic_create, gempic_step, gempic_fields,
gempic_particles, gempic_set_state, gempic_get_spectral, gempic_destroy,
gempic_dn_*); ``Sim`` and ``Denoiser`` wrap handles for tests and the
benchmark.  PyTorch is optional and
only supplies device buffers and the current stream.
"""
import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libgempic.so")

ABI_VERSION = 3
BEAM_BIT = 1 << 30
FP64, FP32_CELL, FP32_ABS = 0, 1, 2
EX, EY, EZ, BX, BY, BZ, JX, JY, JZ, RHO = (1 << i for i in range(10))
FIELD_NAMES = ("Ex", "Ey", "Ez", "Bx", "By", "Bz", "Jx", "Jy", "Jz", "rho")

STATUS = {0: "GEMPIC_OK", -1: "GEMPIC_EINVAL", -2: "GEMPIC_ENOMEM", -3: "GEMPIC_EDEVICE",
          -4: "GEMPIC_ECFL", -5: "GEMPIC_ENUMERIC", -6: "GEMPIC_ESTATE", -7: "GEMPIC_EABI",
          -8: "GEMPIC_ECAPACITY"}


class GempicError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class gempic_config(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_int32), ("dims", ctypes.c_int32), ("n", ctypes.c_int32 * 3),
        ("d", ctypes.c_double * 3), ("length_unit", ctypes.c_double), ("dtau", ctypes.c_double),
        ("precision", ctypes.c_int32), ("tile", ctypes.c_int32 * 3), ("n_e", ctypes.c_double),
        ("ppc", ctypes.c_int32 * 3), ("load", ctypes.c_int32), ("a0", ctypes.c_double),
        ("waist", ctypes.c_double), ("fwhm", ctypes.c_double), ("zeta_c", ctypes.c_double),
        ("pol", ctypes.c_int32), ("seed", ctypes.c_uint64), ("filter_passes", ctypes.c_int32),
        ("track_ids", ctypes.c_int32), ("deposit_rho", ctypes.c_int32),
        ("beam_n", ctypes.c_double), ("beam_sr", ctypes.c_double), ("beam_sz", ctypes.c_double),
        ("beam_zc", ctypes.c_double), ("beam_gamma", ctypes.c_double), ("beam_dgamma", ctypes.c_double),
        ("beam_np", ctypes.c_int64), ("scheme", ctypes.c_int32), ("delta", ctypes.c_double),
        ("zeta_nodes", ctypes.c_void_p), ("ch_ratio", ctypes.c_double), ("ch_radius", ctypes.c_double),
        ("stream", ctypes.c_void_p),
    ]


class gempic_diag(ctypes.Structure):
    _fields_ = [
        ("tau", ctypes.c_double), ("step", ctypes.c_int64), ("n_particles", ctypes.c_int64),
        ("charge_particles", ctypes.c_double), ("charge_grid", ctypes.c_double),
        ("field_energy", ctypes.c_double), ("continuity_rel", ctypes.c_double),
        ("fallbacks", ctypes.c_int64), ("denoise_rel", ctypes.c_double),
    ]


class gempic_bunch(ctypes.Structure):
    _fields_ = [
        ("charge", ctypes.c_double), ("n_macro", ctypes.c_int64), ("gamma_mean", ctypes.c_double),
        ("gamma_rms", ctypes.c_double), ("mean", ctypes.c_double * 3), ("sigma", ctypes.c_double * 3),
        ("emittance", ctypes.c_double * 2),
    ]


_lib = None

# exported symbols and their signatures (argument marshalling only)
_SIGS = {
    "gempic_create": (ctypes.c_int, [ctypes.POINTER(gempic_config), ctypes.POINTER(ctypes.c_void_p)]),
    "gempic_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(gempic_diag)]),
    "gempic_fields": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_int32, ctypes.c_void_p,
                                     ctypes.c_size_t]),
    "gempic_fields_bytes": (ctypes.c_size_t, [ctypes.c_void_p, ctypes.c_uint32]),
    "gempic_particles": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                        ctypes.POINTER(ctypes.c_size_t)]),
    "gempic_set_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                        ctypes.c_size_t]),
    "gempic_get_spectral": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t]),
    "gempic_set_fields": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t]),
    "gempic_timing": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "gempic_get_timing": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_int64)]),
    "gempic_set_slow_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double]),
    "gempic_set_deterministic": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "gempic_axis_field": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                         ctypes.c_size_t]),
    "gempic_bunch_diag": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double, ctypes.POINTER(gempic_bunch)]),
    "gempic_march_particles": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                              ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)]),
    "gempic_destroy": (None, [ctypes.c_void_p]),
    "gempic_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "gempic_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
    "gempic_set_denoiser": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double]),
    "gempic_dn_nparams": (ctypes.c_size_t, []),
    "gempic_dn_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                        ctypes.POINTER(ctypes.c_void_p)]),
    "gempic_dn_destroy": (None, [ctypes.c_void_p]),
    "gempic_dn_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
    "gempic_dn_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t]),
    "gempic_dn_grad": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t]),
    "gempic_dn_apply": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32), ctypes.c_void_p,
                                       ctypes.c_double, ctypes.POINTER(ctypes.c_double), ctypes.c_int32,
                                       ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)]),
    "gempic_dn_apply_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32), ctypes.c_void_p,
                                               ctypes.c_double, ctypes.POINTER(ctypes.c_double), ctypes.c_int32,
                                               ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p,
                                               ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)]),
    "gempic_dn_train": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                       ctypes.POINTER(ctypes.c_double), ctypes.c_int32,
                                       ctypes.POINTER(ctypes.c_int32), ctypes.c_double,
                                       ctypes.POINTER(ctypes.c_double)]),
}


def lib():
    """Load the in-tree HIP library; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library missing: {LIB_PATH} (run __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc, handle=None):
    if rc != 0:
        msg = lib().gempic_last_error(handle)
        raise GempicError(rc, msg.decode() if msg else "")


def make_config(cfg, stream=None, track_ids=False, deposit_rho=False):
    """Workload dict (see workloads.py) -> gempic_config."""
    c = gempic_config()
    c.abi_version = ABI_VERSION
    c.dims = int(cfg["dims"])
    c.n[:] = [int(v) for v in cfg["n"]]
    c.d[:] = [float(v) for v in cfg["d"]]
    c.length_unit = float(cfg.get("length_unit", 1.0))
    c.dtau = float(cfg.get("dtau", 0.0))
    prec = cfg.get("precision", "fp32")
    modes = {"fp64": FP64, "fp32": FP32_CELL, "fp32abs": FP32_ABS}
    if prec not in modes:
        raise ValueError(f"precision {prec!r} not supported by the library")
    c.precision = modes[prec]
    c.tile[:] = [int(v) for v in cfg.get("tile", (8, 8, 8))]
    c.n_e = float(cfg.get("n_e", 0.0))
    c.ppc[:] = [int(v) for v in cfg.get("ppc", (1, 1, 1))]
    c.load = int(cfg.get("load", 0))
    c.a0 = float(cfg.get("a0", 0.0))
    c.waist = float(cfg.get("waist", 0.0))
    c.fwhm = float(cfg.get("fwhm", 0.0))
    zc = cfg.get("zeta_c", None)
    c.zeta_c = math.nan if zc is None else float(zc)
    c.pol = int(cfg.get("pol", 0))
    c.seed = int(cfg.get("seed", 0))
    c.filter_passes = int(cfg.get("filter_passes", 1))
    c.track_ids = int(bool(track_ids))
    c.deposit_rho = int(bool(deposit_rho))
    b = cfg.get("beam") or {}
    c.beam_n = float(b.get("n", 0.0))
    c.beam_sr = float(b.get("sr", 0.0))
    c.beam_sz = float(b.get("sz", 0.0))
    zb = b.get("zc", None)
    c.beam_zc = math.nan if zb is None else float(zb)
    c.beam_gamma = float(b.get("gamma", 1.0))
    c.beam_dgamma = float(b.get("dgamma", 0.0))
    c.beam_np = int(b.get("np", 0))
    c.scheme = int(cfg.get("scheme", 0))
    c.delta = float(cfg.get("delta", 0.0))
    zn = cfg.get("zeta_nodes")
    if zn is not None:
        arr = np.ascontiguousarray(zn, np.float64)
        c._zeta_nodes = arr            # kept alive with the struct until creation copies it
        c.zeta_nodes = arr.ctypes.data_as(ctypes.c_void_p)
    c.ch_ratio = float(cfg.get("ch_ratio", 0.0))
    c.ch_radius = float(cfg.get("ch_radius", 0.0))
    c.stream = stream
    return c


def gempic_create(cfg):
    h = ctypes.c_void_p()
    _check(lib().gempic_create(ctypes.byref(cfg), ctypes.byref(h)))
    return h


def gempic_step(h, n, want_diag=False):
    d = gempic_diag() if want_diag else None
    _check(lib().gempic_step(h, int(n), ctypes.byref(d) if d is not None else None), h)
    return d


def gempic_fields(h, mask, on_device, dst_ptr, nbytes):
    _check(lib().gempic_fields(h, mask, int(on_device), dst_ptr, nbytes), h)


def gempic_particles(h, on_device, cell, off, u, ids, capacity):
    cnt = ctypes.c_size_t()
    _check(lib().gempic_particles(h, int(on_device), cell, off, u, ids, capacity, ctypes.byref(cnt)), h)
    return cnt.value


def gempic_set_state(h, step, cell, off, u, ids, count, spectral, spectral_bytes):
    _check(lib().gempic_set_state(h, int(step), cell, off, u, ids, count, spectral, spectral_bytes), h)


def gempic_get_spectral(h, dst, nbytes):
    _check(lib().gempic_get_spectral(h, dst, nbytes), h)


def gempic_set_fields(h, src, nbytes):
    _check(lib().gempic_set_fields(h, src, nbytes), h)


def gempic_timing(h, enable):
    _check(lib().gempic_timing(h, int(enable)), h)


def gempic_get_timing(h):
    ms = (ctypes.c_double * 5)()
    n = ctypes.c_int64()
    _check(lib().gempic_get_timing(h, ms, ctypes.byref(n)), h)
    return list(ms), n.value


def gempic_destroy(h):
    lib().gempic_destroy(h)


def gempic_set_denoiser(h, dn, threshold):
    _check(lib().gempic_set_denoiser(h, dn, float(threshold)), h)


def _dn_check(rc, d):
    if rc != 0:
        msg = lib().gempic_dn_last_error(d)
        raise GempicError(rc, msg.decode() if msg else "")


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class Sim:
    """One handle.  Host-side getters return numpy arrays."""

    def __init__(self, cfg, stream=None, track_ids=False, deposit_rho=False):
        self.cfg = dict(cfg)
        self.c = make_config(cfg, stream, track_ids, deposit_rho)
        self.h = gempic_create(self.c)
        self.dtype = np.float64 if self.c.precision == FP64 else np.float32
        self.dims = self.c.dims
        self.Nx, self.Nz = self.c.n[0], self.c.n[2]
        self.Ny = self.c.n[1] if self.dims == 3 else 1
        self.P = self.c.filter_passes
        self.NPJ = self.Nz + self.P + 7

    def close(self):
        if self.h:
            gempic_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n=1, diag=False):
        d = gempic_step(self.h, n, diag)
        if d is None:
            return None
        return {f: getattr(d, f) for f, _ in gempic_diag._fields_}

    def fields(self, names=("Ex", "Ey", "Ez", "Bx", "By", "Bz")):
        out = {}
        for nm in names:
            bit = 1 << FIELD_NAMES.index(nm)
            planes = self.Nz if bit < JX else self.NPJ
            a = np.empty((planes, self.Ny, self.Nx), self.dtype)
            gempic_fields(self.h, bit, 0, _ptr(a), a.nbytes)
            out[nm] = a
        return out

    def particles(self, ids=False):
        cap = self._count()
        cell = np.empty(cap, np.int32)
        off = np.empty((3, cap), self.dtype)
        u = np.empty((3, cap), self.dtype)
        idv = np.empty(cap, np.int64) if ids else None
        n = gempic_particles(self.h, 0, _ptr(cell), _ptr(off), _ptr(u), _ptr(idv), cap)
        r = dict(cell=cell[:n], off=off[:, :n], u=u[:, :n])
        if ids:
            r["id"] = idv[:n]
        return r

    def _count(self):
        cnt = ctypes.c_size_t()
        rc = lib().gempic_particles(self.h, 0, None, None, None, None, 0, ctypes.byref(cnt))
        if rc not in (0, -1):
            _check(rc, self.h)
        return cnt.value

    def spectral(self):
        nxh = self.Nx // 2
        a = np.empty((6, self.Nz, self.Ny, nxh), np.complex128 if self.dtype == np.float64 else np.complex64)
        gempic_get_spectral(self.h, _ptr(a), a.nbytes)
        return a

    def timing(self, enable=True):
        gempic_timing(self.h, enable)

    def get_timing(self):
        """Accumulated ms per phase (clear, push+deposit, sort+window, fields,
        step) and the number of timed steps."""
        ms, n = gempic_get_timing(self.h)
        return dict(zip(("clear", "push_deposit", "sort_window", "fields", "step"), ms)), n

    def fields_device(self, names, out):
        """Copy fields into a contiguous device tensor ``out`` (torch), in
        the order of ``names``, each [planes][Ny][Nx]."""
        mask = 0
        for nm in names:
            mask |= 1 << FIELD_NAMES.index(nm)
        if [nm for nm in FIELD_NAMES if mask & (1 << FIELD_NAMES.index(nm))] != list(names):
            raise ValueError("names must follow the library order " + str(FIELD_NAMES))
        gempic_fields(self.h, mask, 1, ctypes.c_void_p(out.data_ptr()), out.numel() * out.element_size())
        return out

    def march_particles(self):
        """Zeta march: weights and remaining slow budgets, in the order of
        particles()."""
        cap = self._count()
        w = np.empty(cap, self.dtype)
        b = np.empty(cap, self.dtype)
        cnt = ctypes.c_size_t()
        _check(lib().gempic_march_particles(self.h, 0, _ptr(w), _ptr(b), cap, ctypes.byref(cnt)), self.h)
        return dict(w=w[:cnt.value], b=b[:cnt.value])

    def bunch(self, gamma_min):
        """Witness-bunch diagnostics of the particles with gamma >= gamma_min."""
        b = gempic_bunch()
        _check(lib().gempic_bunch_diag(self.h, float(gamma_min), ctypes.byref(b)), self.h)
        return dict(charge=b.charge, n_macro=b.n_macro, gamma_mean=b.gamma_mean, gamma_rms=b.gamma_rms,
                    mean_x=b.mean[0], mean_y=b.mean[1], mean_z=b.mean[2], sigma_x=b.sigma[0],
                    sigma_y=b.sigma[1], sigma_z=b.sigma[2], eps_x=b.emittance[0], eps_y=b.emittance[1])

    def set_slow_step(self, delta):
        """Zeta march: slow step of the following steps (config units)."""
        _check(lib().gempic_set_slow_step(self.h, float(delta)), self.h)

    def axis_field(self, name="Ez"):
        """FP64 copy of one E or B component along the axis node column
        (Nx/2, Ny/2), one value per zeta plane."""
        import numpy as np
        out = np.empty(self.Nz, np.float64)
        _check(lib().gempic_axis_field(self.h, FIELD_NAMES.index(name), out.ctypes.data_as(
            ctypes.POINTER(ctypes.c_double)), out.size), self.h)
        return out

    def set_deterministic(self, on=True):
        """Deterministic deposit (tau scheme, FP32, no driver beam): the current
        summed in 64-bit fixed point across tiles, the same bit for bit from
        run to run."""
        _check(lib().gempic_set_deterministic(self.h, 1 if on else 0), self.h)

    def set_denoiser(self, dn, threshold=1e-3):
        """Attach a Denoiser (None detaches); the Denoiser must outlive it."""
        gempic_set_denoiser(self.h, None if dn is None else dn.h, threshold)
        self._dn = dn

    def set_fields(self, F6):
        a = np.ascontiguousarray(F6, self.dtype)
        gempic_set_fields(self.h, _ptr(a), a.nbytes)

    def set_state(self, step, cell, off, u, spectral, ids=None):
        cell = np.ascontiguousarray(cell, np.int32)
        off = np.ascontiguousarray(off, self.dtype)
        u = np.ascontiguousarray(u, self.dtype)
        ct = np.complex128 if self.dtype == np.float64 else np.complex64
        sp = None if spectral is None else np.ascontiguousarray(spectral, ct)
        idv = None if ids is None else np.ascontiguousarray(ids, np.int64)
        gempic_set_state(self.h, step, _ptr(cell), _ptr(off), _ptr(u), _ptr(idv), len(cell),
                         _ptr(sp), 0 if sp is None else sp.nbytes)


class Denoiser:
    """Handle of the learned current denoiser (include/gempic_denoise.h).
    Currents are contiguous float32 device tensors [.., 3, Z, Y, X]."""

    def __init__(self, theta, stream=None):
        theta = np.ascontiguousarray(theta, np.float32)
        n = lib().gempic_dn_nparams()
        if theta.size != n:
            raise ValueError(f"expected {n} parameters, got {theta.size}")
        self.h = ctypes.c_void_p()
        _dn_check(lib().gempic_dn_create(_ptr(theta), n, stream, ctypes.byref(self.h)), None)
        self.n = n

    def close(self):
        if self.h:
            lib().gempic_dn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self):
        a = np.empty(self.n, np.float32)
        _dn_check(lib().gempic_dn_params(self.h, _ptr(a), self.n), self.h)
        return a

    def grad(self):
        a = np.empty(self.n, np.float32)
        _dn_check(lib().gempic_dn_grad(self.h, _ptr(a), self.n), self.h)
        return a

    @staticmethod
    def _dptr(t):
        if not (t.is_contiguous() and str(t.dtype) == "torch.float32" and t.is_cuda):
            raise ValueError("expected a contiguous float32 device tensor")
        return ctypes.c_void_p(t.data_ptr())

    def apply(self, jraw, n_e, h, passes=1, threshold=1e-3, jout=None, aout=None):
        """jraw [3, Z, Y, X] -> (J, used, rel); A into ``aout`` if given."""
        import torch
        box = (ctypes.c_int32 * 3)(*jraw.shape[1:])
        if jout is None:
            jout = torch.empty_like(jraw)
        used = ctypes.c_int32()
        rel = ctypes.c_double()
        hs = (ctypes.c_double * 3)(*h)
        _dn_check(lib().gempic_dn_apply(self.h, box, self._dptr(jraw), float(n_e), hs, int(passes),
                                        float(threshold), self._dptr(jout),
                                        None if aout is None else self._dptr(aout),
                                        ctypes.byref(used), ctypes.byref(rel)), self.h)
        return jout, bool(used.value), rel.value

    def apply_noalloc(self, jraw, n_e, h, passes=1, threshold=1e-3, jout=None, aout=None):
        """As apply, through the allocation-free entry point (boxes of at most
        2^18 voxels); jout must be given by callers that cannot allocate."""
        import torch
        box = (ctypes.c_int32 * 3)(*jraw.shape[1:])
        if jout is None:
            jout = torch.empty_like(jraw)
        used = ctypes.c_int32()
        rel = ctypes.c_double()
        hs = (ctypes.c_double * 3)(*h)
        _dn_check(lib().gempic_dn_apply_noalloc(self.h, box, self._dptr(jraw), float(n_e), hs, int(passes),
                                                float(threshold), self._dptr(jout),
                                                None if aout is None else self._dptr(aout),
                                                ctypes.byref(used), ctypes.byref(rel)), self.h)
        return jout, bool(used.value), rel.value

    def train(self, jraw, jtarget, n_e, h, region, lr, passes=1):
        """One step over a batch [B, 3, Z, Y, X]; returns the batch loss."""
        if jraw.shape != jtarget.shape or jraw.dim() != 5:
            raise ValueError("jraw and jtarget must both be [B, 3, Z, Y, X]")
        box = (ctypes.c_int32 * 3)(*jraw.shape[2:])
        reg = (ctypes.c_int32 * 2)(*region)
        hs = (ctypes.c_double * 3)(*h)
        loss = ctypes.c_double()
        _dn_check(lib().gempic_dn_train(self.h, box, int(jraw.shape[0]), self._dptr(jraw),
                                        self._dptr(jtarget), float(n_e), hs, int(passes), reg,
                                        float(lr), ctypes.byref(loss)), self.h)
        return loss.value
