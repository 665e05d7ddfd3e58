"""Thin Python binding of the C ABI in ``include/lqcd.h``.

Argument marshalling only: every step of the operator and the solve runs in
the gfx950 kernels of ``liblqcd.so``.  PyTorch provides device memory
(``torch.empty(..., device="cuda")``) and streams.  There is no fallback: if
the shared library is missing or cannot be loaded, importing a function
that needs it raises ``RuntimeError``.

Canonical layouts (complex128, C order): gauge ``U[t, z, y, x, mu, a, b]``,
spinor ``psi[rhs, t, z, y, x, alpha, a]`` (a single field may omit ``rhs``).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch  # noqa: F401  (loads the HIP runtime the library binds to)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblqcd.so")

# status codes
OK, PENDING, EINVAL, ENOMEM, EDEVICE, ENOCONV, ENUMERIC, ENOTFOUND, EBUSY, EUNSUPPORTED = (
    0, 1, -1, -2, -3, -4, -5, -6, -7, -8)
# boundary conditions
BC_PERIODIC, BC_SF, BC_OPEN = 0, 1, 2
# precisions and masks
F64, F32, BF16 = 0, 1, 2
PM_F64, PM_F32, PM_BF16 = 1, 2, 4
PM_PRECISIONS = PM_F64 | PM_F32 | PM_BF16
# gauge fields only: links stored as their first two rows (SU(3) links only)
PM_TWO_ROW = 8
TUNE_NT_STORE = 1  # lqcd_tuning.flags: non-temporal output stores in the hop kernels
TUNE_CACHED_GAUGE = 2  # lqcd_tuning.flags: cached (not non-temporal) link and clover loads
TUNE_OCC_SHIFT = 2  # lqcd_tuning.flags bits 2-3: cap of resident workgroups per CU (4, 3, 2)
TUNE_DIR_SPLIT = 16  # lqcd_tuning.flags: two waves per site block split the hop directions
# operators
(OP_DW, OP_DW_DAG, OP_G5DW, OP_DWDAGDW, OP_SCHUR, OP_SCHUR_DAG, OP_SCHUR_NORMAL, OP_HOP_EO,
 OP_HOP_OE) = range(9)
LAYOUT_CANON, LAYOUT_INTERNAL = 0, 1
SOLVER_CG_FULL, SOLVER_CG_EO = 0, 1


class LqcdError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"lqcd status {status}: {msg}")
        self.status = status


class GeomDesc(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32 * 4), ("bc", ctypes.c_int32),
                ("theta_re", ctypes.c_double * 4), ("theta_im", ctypes.c_double * 4)]


class Dirac(ctypes.Structure):
    _fields_ = [("kappa", ctypes.c_double), ("csw", ctypes.c_double), ("cF", ctypes.c_double),
                ("mu", ctypes.c_double)]


class SolveParams(ctypes.Structure):
    _fields_ = [("d", Dirac), ("solver", ctypes.c_int32), ("inner_prec", ctypes.c_int32),
                ("reliable_every", ctypes.c_int32), ("maxiter", ctypes.c_int32),
                ("tol", ctypes.c_double), ("nrhs", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("x0", ctypes.c_void_p)]


class Tuning(ctypes.Structure):
    _fields_ = [("nr_tile", ctypes.c_int32), ("block_order", ctypes.c_int32),
                ("rhs_lanes", ctypes.c_int32), ("flags", ctypes.c_int32)]

    def as_dict(self):
        return {"nr_tile": self.nr_tile, "block_order": self.block_order, "rhs_lanes": self.rhs_lanes,
                "nt_store": bool(self.flags & TUNE_NT_STORE), "cached_gauge": bool(self.flags & TUNE_CACHED_GAUGE),
                "occ_cap": (self.flags >> TUNE_OCC_SHIFT) & 3, "dir_split": bool(self.flags & TUNE_DIR_SPLIT)}


class SolveInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32),
                ("reliable_updates", ctypes.c_int32), ("restarts", ctypes.c_int32),
                ("fp64_from", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("true_residual", ctypes.c_double), ("seconds", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


_lib = None

# exported symbols and their signatures (restype, argtypes)
_P, _I, _Z, _D = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t, ctypes.c_double
SIGNATURES = {
    "lqcd_strerror": (ctypes.c_char_p, [_I]),
    "lqcd_last_error": (ctypes.c_char_p, []),
    "lqcd_geom": (_I, [ctypes.POINTER(GeomDesc), ctypes.POINTER(_P)]),
    "lqcd_geom_free": (None, [_P]),
    "lqcd_geom_volume": (ctypes.c_int64, [_P]),
    "lqcd_gauge_bytes": (_Z, [_P, _I]),
    "lqcd_gauge_create": (_I, [_P, _P, _I, _P, _Z, _P, ctypes.POINTER(_P)]),
    "lqcd_gauge_free": (None, [_P]),
    "lqcd_ws_bytes": (_Z, [_P, _I, _I]),
    "lqcd_ws_create": (_I, [_P, _I, _I, _P, _Z, ctypes.POINTER(_P)]),
    "lqcd_ws_free": (None, [_P]),
    "lqcd_clover": (_I, [_P, ctypes.POINTER(Dirac), _P, _P]),
    "lqcd_dw_apply": (_I, [_P, ctypes.POINTER(Dirac), _I, _I, _I, _I, _P, _P, _P, _P]),
    "lqcd_vec_bytes": (_Z, [_P, _I, _I, _I]),
    "lqcd_solve": (_I, [_P, ctypes.POINTER(SolveParams), _P, _P, _P, _P, ctypes.POINTER(SolveInfo)]),
    "lqcd_meson": (_I, [_P, _P, _I, ctypes.POINTER(ctypes.c_int32), _P, _P, _P, _P]),
    "lqcd_meson_noalloc": (_I, [_P, _P, _I, ctypes.POINTER(ctypes.c_int32), _P, _P, _P]),
    "lqcd_noalloc_scratch_bytes": (_Z, []),
    "lqcd_sf_source": (_I, [_P, _P, _P]),
    "lqcd_sf_correlators": (_I, [_P, ctypes.POINTER(SolveParams), _P, _P, _P, _P, _P, _P, ctypes.POINTER(SolveInfo)]),
    "lqcd_ws_set_tuning": (_I, [_P, _I, ctypes.POINTER(Tuning)]),
    "lqcd_ws_get_tuning": (_I, [_P, _I, ctypes.POINTER(Tuning)]),
    "lqcd_autotune": (_I, [_P, ctypes.POINTER(Dirac), _I, _I, _P, _P, ctypes.POINTER(Tuning),
                           ctypes.POINTER(ctypes.c_double)]),
    "lqcd_tune_cache_find": (_I, [_P, _I, _I, _I, _I, ctypes.POINTER(Tuning)]),
    "lqcd_tune_cache_put": (_I, [_P, _I, _I, _I, ctypes.POINTER(Tuning)]),
    "lqcd_tune_cache_size": (_I, []),
    "lqcd_tune_cache_clear": (None, []),
    "lqcd_tune_cache_save": (_I, [ctypes.c_char_p]),
    "lqcd_tune_cache_load": (_I, [ctypes.c_char_p]),
    "lqcd_server_create": (_I, [_P, _Z, _I, _I, _D, ctypes.POINTER(_P)]),
    "lqcd_server_warmup": (_I, [_P, _I, _I, _I]),
    "lqcd_server_add_gauge": (_I, [_P, ctypes.POINTER(GeomDesc), _P, _I, ctypes.POINTER(_I)]),
    "lqcd_request_bytes": (_Z, [_P, _I, ctypes.POINTER(SolveParams)]),
    "lqcd_submit": (_I, [_P, _I, ctypes.POINTER(SolveParams), _P, _P, ctypes.POINTER(ctypes.c_uint64)]),
    "lqcd_poll": (_I, [_P, ctypes.c_uint64, _P, _P]),
    "lqcd_server_peak_bytes": (_Z, [_P]),
    "lqcd_server_stop": (_I, [_P, _I]),
    "lqcd_server_destroy": (_I, [_P, _I]),
}
ECANCELED = -9


def lib():
    """Load liblqcd.so (raises if it is not built or cannot be loaded)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run paper_2503_16994_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(status: int):
    if status != OK:
        raise LqcdError(status, lib().lqcd_last_error().decode())


def _stream_ptr(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_bytes(nbytes: int) -> torch.Tensor:
    t = torch.empty(max(int(nbytes), 1) + 256, dtype=torch.uint8, device="cuda")
    return t


def _aligned_ptr(t: torch.Tensor) -> int:
    p = t.data_ptr()
    return (p + 255) & ~255


def _spinor_arg(name: str, t: torch.Tensor, lat, nrhs=None) -> torch.Tensor:
    """Checks a canonical spinor argument before its pointer crosses the ABI:
    complex128, on the GPU, a whole number of fields (nrhs of them if given);
    returns it as a contiguous (nrhs, T, Z, Y, X, 4, 3) tensor."""
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != torch.complex128:
        raise TypeError(f"{name} must be complex128, got {t.dtype}")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (device) tensor")
    per = 1
    for v in lat.spinor_shape():
        per *= v
    if t.numel() == 0 or t.numel() % per:
        raise ValueError(f"{name} holds {t.numel()} elements, not a multiple of one field ({per})")
    if nrhs is not None and t.numel() != nrhs * per:
        raise ValueError(f"{name} holds {t.numel() // per} fields, expected {nrhs}")
    return t.reshape((-1,) + lat.spinor_shape()).contiguous()


def _out_arg(name: str, t: torch.Tensor, like: torch.Tensor, others=()) -> torch.Tensor:
    """Checks a caller-supplied output: complex128 device tensor of exactly
    like's shape, contiguous (written in place), overlapping none of `others`."""
    if not isinstance(t, torch.Tensor) or t.dtype != torch.complex128 or not t.is_cuda:
        raise TypeError(f"{name} must be a complex128 CUDA tensor")
    if t.numel() != like.numel():
        raise ValueError(f"{name} holds {t.numel()} elements, expected {like.numel()}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous (it is written in place)")
    nb = t.numel() * t.element_size()
    for o in others:
        ob = o.numel() * o.element_size()
        if t.data_ptr() < o.data_ptr() + ob and o.data_ptr() < t.data_ptr() + nb:
            raise ValueError(f"{name} overlaps an input")
    return t.reshape(like.shape)


def m0_from_kappa(kappa: float) -> float:
    return 1.0 / (2.0 * kappa) - 4.0


class Lattice:
    """Geometry handle (lqcd_geom): extents (x, y, z, t), boundary type, theta."""

    def __init__(self, L, bc=BC_PERIODIC, theta=(1, 1, 1, 1)):
        d = GeomDesc()
        for i in range(4):
            d.L[i] = int(L[i])
            th = complex(theta[i])
            d.theta_re[i] = th.real
            d.theta_im[i] = th.imag
        d.bc = int(bc)
        h = ctypes.c_void_p()
        _check(lib().lqcd_geom(ctypes.byref(d), ctypes.byref(h)))
        self.handle = h
        self.L = tuple(int(v) for v in L)
        self.bc = int(bc)
        self.theta = tuple(complex(t) for t in theta)
        self.volume = int(lib().lqcd_geom_volume(h))

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.lqcd_geom_free(self.handle)
            self.handle = None

    def spinor_shape(self, nrhs=None):
        Lx, Ly, Lz, T = self.L
        s = (T, Lz, Ly, Lx, 4, 3)
        return s if nrhs is None else (nrhs,) + s


class GaugeField:
    """Device-resident gauge field (lqcd_gauge_create) in FP64 and `pmask` precisions;
    PM_TWO_ROW in `pmask` stores two rows per link (the field must be SU(3))."""

    def __init__(self, lat: Lattice, U, pmask=PM_F64, stream=None):
        self.lat = lat
        U = torch.as_tensor(U)
        if U.dtype != torch.complex128:
            raise TypeError("U must be complex128")
        U = U.to("cuda").contiguous()
        nbytes = lib().lqcd_gauge_bytes(lat.handle, pmask)
        self._mem = _dev_bytes(nbytes)
        h = ctypes.c_void_p()
        _check(lib().lqcd_gauge_create(lat.handle, ctypes.c_void_p(U.data_ptr()), pmask,
                                       ctypes.c_void_p(_aligned_ptr(self._mem)), nbytes,
                                       _stream_ptr(stream), ctypes.byref(h)))
        # keep the canonical copy alive until the import kernel has run
        torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()
        self.handle = h
        self.pmask = pmask

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.lqcd_gauge_free(self.handle)
            self.handle = None


class Workspace:
    """Solver/operator workspace (lqcd_ws_create) for up to `nrhs` fields."""

    def __init__(self, lat: Lattice, pmask=PM_F64, nrhs=1):
        self.lat = lat
        nbytes = lib().lqcd_ws_bytes(lat.handle, pmask, nrhs)
        self._mem = _dev_bytes(nbytes)
        h = ctypes.c_void_p()
        _check(lib().lqcd_ws_create(lat.handle, pmask, nrhs, ctypes.c_void_p(_aligned_ptr(self._mem)),
                                    nbytes, ctypes.byref(h)))
        self.handle = h
        self.nrhs = nrhs
        self.pmask = pmask
        self.nbytes = nbytes

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.lqcd_ws_free(self.handle)
            self.handle = None


def dirac(kappa, csw, cF=1.0, mu=0.0) -> Dirac:
    return Dirac(float(kappa), float(csw), float(cF), float(mu))


def clover(gauge: GaugeField, d: Dirac, ws: Workspace, stream=None):
    _check(lib().lqcd_clover(gauge.handle, ctypes.byref(d), ws.handle, _stream_ptr(stream)))


def dw_apply(gauge: GaugeField, d: Dirac, psi: torch.Tensor, op=OP_DW, prec=F64, ws=None,
             out=None, stream=None) -> torch.Tensor:
    """Apply an operator to canonical complex128 device field(s)."""
    lat = gauge.lat
    single = psi.dim() == 6
    x = _spinor_arg("psi", psi, lat)
    nrhs = x.shape[0]
    if ws is None:
        ws = Workspace(lat, gauge.pmask & PM_PRECISIONS, nrhs)
    if nrhs > ws.nrhs:
        raise ValueError(f"{nrhs} fields exceed the workspace's {ws.nrhs}")
    out = torch.empty_like(x) if out is None else _out_arg("out", out, x, (x,))
    _check(lib().lqcd_dw_apply(gauge.handle, ctypes.byref(d), op, prec, LAYOUT_CANON, nrhs,
                               ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                               ws.handle, _stream_ptr(stream)))
    return out[0] if single else out


def dw_apply_internal(gauge: GaugeField, d: Dirac, vin: torch.Tensor, vout: torch.Tensor, op, prec,
                      nrhs, ws: Workspace, stream=None):
    """Apply an operator to internal-layout vectors (benchmarking)."""
    need = vec_bytes(gauge.lat, prec, nrhs, 2)
    for name, v in (("vin", vin), ("vout", vout)):
        if not isinstance(v, torch.Tensor) or not v.is_cuda or not v.is_contiguous():
            raise TypeError(f"{name} must be a contiguous CUDA tensor")
        if v.numel() * v.element_size() < need:
            raise ValueError(f"{name} holds {v.numel() * v.element_size()} bytes, {need} needed")
    if vin.data_ptr() == vout.data_ptr():
        raise ValueError("vin and vout must differ")
    if nrhs > ws.nrhs:
        raise ValueError(f"{nrhs} fields exceed the workspace's {ws.nrhs}")
    _check(lib().lqcd_dw_apply(gauge.handle, ctypes.byref(d), op, prec, LAYOUT_INTERNAL, nrhs,
                               ctypes.c_void_p(vin.data_ptr()), ctypes.c_void_p(vout.data_ptr()),
                               ws.handle, _stream_ptr(stream)))


def set_tuning(ws: Workspace, prec, nr_tile=1, block_order=1, rhs_lanes=1, nt_store=False, cached_gauge=False,
               occ_cap=0, dir_split=False):
    t = Tuning(int(nr_tile), int(block_order), int(rhs_lanes),
               (TUNE_NT_STORE if nt_store else 0) | (TUNE_CACHED_GAUGE if cached_gauge else 0)
               | ((int(occ_cap) & 3) << TUNE_OCC_SHIFT) | (TUNE_DIR_SPLIT if dir_split else 0))
    _check(lib().lqcd_ws_set_tuning(ws.handle, prec, ctypes.byref(t)))


def get_tuning(ws: Workspace, prec) -> dict:
    t = Tuning()
    _check(lib().lqcd_ws_get_tuning(ws.handle, prec, ctypes.byref(t)))
    return t.as_dict()


def autotune(gauge: GaugeField, d: Dirac, prec, nrhs, ws: Workspace, stream=None):
    """Time the hop-kernel configurations and keep the fastest in `ws`.
    Returns (tuning dict, microseconds per Schur-operator application)."""
    t = Tuning()
    us = ctypes.c_double(0.0)
    _check(lib().lqcd_autotune(gauge.handle, ctypes.byref(d), prec, nrhs, ws.handle,
                               _stream_ptr(stream), ctypes.byref(t), ctypes.byref(us)))
    return t.as_dict(), us.value


def tune_cache_find(gauge: GaugeField, prec, nrhs, twisted=False, dir_split=False):
    """The cached tuning dict for this key, or None."""
    t = Tuning()
    st = lib().lqcd_tune_cache_find(gauge.handle, int(prec), int(nrhs), int(bool(twisted)), int(bool(dir_split)),
                                    ctypes.byref(t))
    if st == ENOTFOUND:
        return None
    _check(st)
    return t.as_dict()


def tune_cache_size() -> int:
    return int(lib().lqcd_tune_cache_size())


def tune_cache_clear():
    lib().lqcd_tune_cache_clear()


def tune_cache_save(path: str):
    _check(lib().lqcd_tune_cache_save(os.fsencode(path)))


def tune_cache_load(path: str):
    _check(lib().lqcd_tune_cache_load(os.fsencode(path)))


def vec_bytes(lat: Lattice, prec, nrhs, nparity=2) -> int:
    return int(lib().lqcd_vec_bytes(lat.handle, prec, nrhs, nparity))


@dataclass
class SolveResult:
    psi: torch.Tensor
    info: list
    status: int


def solve(gauge: GaugeField, eta: torch.Tensor, kappa, csw, cF=1.0, tol=1e-10, maxiter=20000,
          solver=SOLVER_CG_EO, inner_prec=F64, reliable_every=100, use_graph=False, ws=None,
          stream=None, psi=None, raise_on_noconv=True, mu=0.0, x0=None) -> SolveResult:
    """Solve D(mu) psi = eta (D(mu) = Dw + i mu g5) for canonical complex128 device source(s),
    from the initial guess x0 (same shape as eta; None: zero)."""
    lat = gauge.lat
    single = eta.dim() == 6
    e = _spinor_arg("eta", eta, lat)
    nrhs = e.shape[0]
    if ws is None:
        ws = Workspace(lat, gauge.pmask & PM_PRECISIONS, nrhs)
    if nrhs > ws.nrhs:
        raise ValueError(f"{nrhs} sources exceed the workspace's {ws.nrhs}")
    x0p = None
    if x0 is not None:
        x0 = _spinor_arg("x0", x0, lat, nrhs)
        x0p = ctypes.c_void_p(x0.data_ptr())
    psi = torch.empty_like(e) if psi is None else _out_arg("psi", psi, e, (e,))
    p = SolveParams(Dirac(float(kappa), float(csw), float(cF), float(mu)), solver, inner_prec,
                    int(reliable_every), int(maxiter), float(tol), nrhs, int(bool(use_graph)), x0p)
    infos = (SolveInfo * nrhs)()
    st = lib().lqcd_solve(gauge.handle, ctypes.byref(p), ctypes.c_void_p(e.data_ptr()),
                          ctypes.c_void_p(psi.data_ptr()), ws.handle, _stream_ptr(stream), infos)
    if st != OK and not (st == ENOCONV and not raise_on_noconv):
        _check(st)
    out = psi[0] if single else psi
    return SolveResult(out, [infos[i].as_dict() for i in range(nrhs)], st)


# gamma-matrix masks of lqcd_meson: Gamma_m = g_t^{m3} g_x^{m0} g_y^{m1} g_z^{m2}
GAMMA_1, GAMMA_X, GAMMA_Y, GAMMA_Z, GAMMA_T, GAMMA_5 = 0, 1, 2, 4, 8, 15


def meson(lat: Lattice, psi: torch.Tensor, pairs, ws: Workspace, want_G=True, stream=None):
    """lqcd_meson on a 12-column canonical propagator ``psi`` (device,
    complex128, shape (12, T, Z, Y, X, 4, 3)): returns (C, G) with C of shape
    (len(pairs), T) and G of shape (T, 4, 4, 4, 4) (None unless want_G)."""
    p = psi.contiguous()
    if p.dtype != torch.complex128 or not p.is_cuda or p.numel() != 12 * lat.volume * 12:
        raise ValueError("psi must be 12 canonical complex128 fields on the GPU")
    T = lat.L[3]
    n = len(pairs)
    flat = (ctypes.c_int32 * max(2 * n, 1))(*[int(m) for pr in pairs for m in pr])
    C = torch.empty((n, T), dtype=torch.complex128, device=p.device) if n else None
    G = torch.empty((T, 4, 4, 4, 4), dtype=torch.complex128, device=p.device) if want_G else None
    _check(lib().lqcd_meson(lat.handle, ctypes.c_void_p(p.data_ptr()), n, flat,
                            ctypes.c_void_p(C.data_ptr() if C is not None else 0),
                            ctypes.c_void_p(G.data_ptr() if G is not None else 0), ws.handle, _stream_ptr(stream)))
    return C, G


def meson_noalloc(lat: Lattice, psi: torch.Tensor, pairs, C=None, G=None, stream=None):
    """lqcd_meson_noalloc: the contraction of ``meson`` with the library's
    fixed per-GPU scratch array instead of a workspace.  The caller passes
    the outputs: C (complex128, (len(pairs), T)) and/or G (complex128,
    (T, 4, 4, 4, 4)), contiguous device tensors, written in place."""
    if psi.dtype != torch.complex128 or not psi.is_cuda or not psi.is_contiguous() \
            or psi.numel() != 12 * lat.volume * 12:
        raise ValueError("psi must be 12 contiguous canonical complex128 fields on the GPU")
    T = lat.L[3]
    n = len(pairs)
    for name, t, shape in (("C", C, (n, T)), ("G", G, (T, 4, 4, 4, 4))):
        if t is not None and (t.dtype != torch.complex128 or not t.is_cuda or not t.is_contiguous()
                              or tuple(t.shape) != shape):
            raise ValueError(f"{name} must be a contiguous complex128 CUDA tensor of shape {shape}")
    flat = (ctypes.c_int32 * max(2 * n, 1))(*[int(m) for pr in pairs for m in pr])
    _check(lib().lqcd_meson_noalloc(lat.handle, ctypes.c_void_p(psi.data_ptr()), n, flat,
                                    ctypes.c_void_p(C.data_ptr() if C is not None else 0),
                                    ctypes.c_void_p(G.data_ptr() if G is not None else 0), _stream_ptr(stream)))
    return C, G


def noalloc_scratch_bytes() -> int:
    return int(lib().lqcd_noalloc_scratch_bytes())


def sf_source(gauge: GaugeField, stream=None) -> torch.Tensor:
    """lqcd_sf_source: the 12-column SF boundary source, canonical (12, T, Z, Y, X, 4, 3)."""
    eta = torch.empty((12,) + gauge.lat.spinor_shape(), dtype=torch.complex128, device="cuda")
    _check(lib().lqcd_sf_source(gauge.handle, ctypes.c_void_p(eta.data_ptr()), _stream_ptr(stream)))
    return eta


def sf_correlators(gauge: GaugeField, kappa, csw, cF=1.0, tol=1e-10, maxiter=20000, inner_prec=F64,
                   reliable_every=100, use_graph=False, ws=None, stream=None):
    """lqcd_sf_correlators: returns (fP, fA, H, infos) with fP, fA complex128 (T,)."""
    lat = gauge.lat
    if ws is None:
        ws = Workspace(lat, gauge.pmask & PM_PRECISIONS, 12)
    shape = (12,) + lat.spinor_shape()
    eta = torch.empty(shape, dtype=torch.complex128, device="cuda")
    H = torch.empty_like(eta)
    fP = torch.empty(lat.L[3], dtype=torch.complex128, device="cuda")
    fA = torch.empty_like(fP)
    p = SolveParams(Dirac(float(kappa), float(csw), float(cF), 0.0), SOLVER_CG_EO, inner_prec,
                    int(reliable_every), int(maxiter), float(tol), 12, int(bool(use_graph)))
    infos = (SolveInfo * 12)()
    _check(lib().lqcd_sf_correlators(gauge.handle, ctypes.byref(p), ctypes.c_void_p(eta.data_ptr()),
                                     ctypes.c_void_p(H.data_ptr()), ctypes.c_void_p(fP.data_ptr()),
                                     ctypes.c_void_p(fA.data_ptr()), ws.handle, _stream_ptr(stream), infos))
    return fP, fA, H, [infos[i].as_dict() for i in range(12)]


class Server:
    """Continuous-batching solve server (lqcd_server_*).

    With ``sim_seconds`` set, the server runs in simulation mode (no device
    memory or work; each request holds its footprint for sim_seconds)."""

    def __init__(self, arena_bytes, max_streams=4, queue_cap=4096, sim_seconds=None):
        self._mem = None
        if sim_seconds is None:
            self._mem = _dev_bytes(arena_bytes)
            arena = ctypes.c_void_p(_aligned_ptr(self._mem))
            sim = 0.0
        else:
            arena = None
            sim = float(sim_seconds)
        h = ctypes.c_void_p()
        _check(lib().lqcd_server_create(arena, int(arena_bytes), int(max_streams), int(queue_cap), sim,
                                        ctypes.byref(h)))
        self.handle = h
        self._live = {}  # ticket -> (eta, psi, nrhs) kept alive until final
        self.nrhs_of = {}

    def add_gauge(self, L, bc, theta, U=None, pmask=PM_F64):
        d = GeomDesc()
        for i in range(4):
            d.L[i] = int(L[i])
            th = complex(theta[i])
            d.theta_re[i] = th.real
            d.theta_im[i] = th.imag
        d.bc = int(bc)
        ptr = None
        if U is not None:
            import numpy as np
            U = np.ascontiguousarray(U, dtype=np.complex128)
            ptr = ctypes.c_void_p(U.ctypes.data)
        gid = ctypes.c_int(-1)
        _check(lib().lqcd_server_add_gauge(self.handle, ctypes.byref(d), ptr, int(pmask), ctypes.byref(gid)))
        return gid.value

    def warmup(self, gauge_id, inner_prec, nrhs):
        """Autotune the kernels for (gauge field, inner precision, nrhs) on the idle GPU."""
        _check(lib().lqcd_server_warmup(self.handle, int(gauge_id), int(inner_prec), int(nrhs)))

    @staticmethod
    def params(kappa, csw, cF=1.0, tol=1e-10, maxiter=20000, inner_prec=F64, nrhs=1, reliable_every=100,
               use_graph=True):
        return SolveParams(Dirac(float(kappa), float(csw), float(cF), 0.0), SOLVER_CG_EO, int(inner_prec),
                           int(reliable_every), int(maxiter), float(tol), int(nrhs), int(bool(use_graph)))

    def request_bytes(self, gauge_id, p: SolveParams) -> int:
        return int(lib().lqcd_request_bytes(self.handle, int(gauge_id), ctypes.byref(p)))

    def submit(self, gauge_id, p: SolveParams, eta=None, psi=None, x0=None) -> int:
        """Enqueue a solve; eta/psi (and the initial guess x0) are host complex128
        arrays of p.nrhs fields (kept alive here until the final poll)."""
        import numpy as np
        ep = pp = None
        if eta is not None:
            eta = np.ascontiguousarray(eta, dtype=np.complex128)
            if psi is None:
                psi = np.empty_like(eta)
            if psi.dtype != np.complex128 or psi.shape != eta.shape or not psi.flags.c_contiguous:
                raise ValueError("psi must be a C-contiguous complex128 array shaped like eta")
            ep, pp = ctypes.c_void_p(eta.ctypes.data), ctypes.c_void_p(psi.ctypes.data)
        if x0 is not None:
            if eta is None:
                raise ValueError("x0 needs eta")
            x0 = np.ascontiguousarray(x0, dtype=np.complex128)
            if x0.shape != eta.shape:
                raise ValueError("x0 must be shaped like eta")
            p = SolveParams.from_buffer_copy(p)
            p.x0 = x0.ctypes.data
        t = ctypes.c_uint64(0)
        _check(lib().lqcd_submit(self.handle, int(gauge_id), ctypes.byref(p), ep, pp, ctypes.byref(t)))
        self._live[t.value] = (eta, psi, p.nrhs, x0)
        return t.value

    def poll(self, ticket):
        """None while pending; else (status, [info dicts], (t_submit, t_admit, t_done), psi)."""
        eta, psi, nrhs, _ = self._live[ticket]
        infos = (SolveInfo * nrhs)()
        times = (ctypes.c_double * 3)()
        st = lib().lqcd_poll(self.handle, ctypes.c_uint64(ticket), infos, times)
        if st == PENDING:
            return None
        if st == ENOTFOUND:
            _check(st)
        del self._live[ticket]
        return st, [infos[i].as_dict() for i in range(nrhs)], tuple(times), psi

    def poll_raw(self, ticket) -> int:
        return lib().lqcd_poll(self.handle, ctypes.c_uint64(ticket), None, None)

    def peak_bytes(self) -> int:
        return int(lib().lqcd_server_peak_bytes(self.handle))

    def stop(self, cancel_pending=False):
        _check(lib().lqcd_server_stop(self.handle, int(bool(cancel_pending))))

    def close(self, cancel_pending=False):
        if getattr(self, "handle", None):
            _check(lib().lqcd_server_destroy(self.handle, int(bool(cancel_pending))))
            self.handle = None

    def __del__(self):
        try:
            self.close(cancel_pending=True)
        except Exception:
            pass
