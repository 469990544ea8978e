"""Python binding of the fastrsd C ABI (include/fastrsd.h).

Argument marshalling only: every step of the estimator runs in the HIP
library ``libfastrsd.so`` built next to this file.  PyTorch provides device
memory and streams.  Importing this module raises if the library is not
built; there is no CPU fallback.

Low-level functions carry the C names (``frsd_plan_create``,
``frsd_mesh_assign``, ...).  ``Plan`` wraps them with torch-allocated
workspace and output buffers.
"""

from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfastrsd.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"fastrsd HIP library not built: {LIB_PATH} is missing "
                      "(run python -m paper_1506_02729_amd.build)")
_lib = ctypes.CDLL(LIB_PATH)

FRSD_OK, FRSD_EINVAL, FRSD_EDOM, FRSD_ENOMEM, FRSD_EHIP, FRSD_ESTATE = 0, -1, -2, -3, -4, -5
FRSD_F32, FRSD_F64 = 32, 64
_ERRNAMES = {-1: "FRSD_EINVAL", -2: "FRSD_EDOM", -3: "FRSD_ENOMEM", -4: "FRSD_EHIP", -5: "FRSD_ESTATE"}


class FrsdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


class frsd_params(ctypes.Structure):
    _fields_ = [
        ("n_grid", ctypes.c_int32), ("order", ctypes.c_int32), ("interlace", ctypes.c_int32),
        ("compensate", ctypes.c_int32), ("ell_max", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("box", ctypes.c_double), ("observer", ctypes.c_double * 3),
        ("pk_kmin", ctypes.c_double), ("pk_dk", ctypes.c_double), ("pk_nbins", ctypes.c_int32),
        ("bk_kmin", ctypes.c_double), ("bk_dk", ctypes.c_double), ("bk_nbins", ctypes.c_int32),
        ("bk_grid", ctypes.c_int32), ("max_objects", ctypes.c_int64),
        ("bk_ell_max", ctypes.c_int32), ("bk_shot_noise", ctypes.c_int32), ("bk_zero_area", ctypes.c_int32),
        ("random_cache", ctypes.c_int32), ("stream_moments", ctypes.c_int32), ("stream_slots", ctypes.c_int32),
    ]


class frsd_tuning(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int32) for name in ("tri_wg", "row_grid", "bin_blocks", "pair_batch", "sweep_x")]


FRSD_DEVICE, FRSD_HOST = 0, 1
FRSD_MAX_BATCH = 16


class frsd_catalog(ctypes.Structure):
    _fields_ = [("pos", ctypes.c_void_p), ("w", ctypes.c_void_p), ("nbar", ctypes.c_void_p),
                ("n", ctypes.c_int64), ("dtype", ctypes.c_int32), ("where", ctypes.c_int32)]


PK_ARRAYS = ("n_modes", "k_eff", "p0", "p2", "p4", "s00", "s20", "s40", "scalars", "p4b", "s22")
BK_ARRAYS = ("nt", "t0", "t2", "t4", "b0", "b2", "b4", "sn0", "sn2", "sn4", "t220", "b4za")


class frsd_pk_out(ctypes.Structure):
    _fields_ = [(name, ctypes.c_void_p) for name in PK_ARRAYS] + [("where", ctypes.c_int32)]


class frsd_bk_out(ctypes.Structure):
    _fields_ = [(name, ctypes.c_void_p) for name in BK_ARRAYS] + [("where", ctypes.c_int32)]


_P = ctypes.c_void_p
_proto = {
    "frsd_plan_create": (ctypes.c_int, [ctypes.POINTER(frsd_params), ctypes.POINTER(_P)]),
    "frsd_plan_destroy": (None, [_P]),
    "frsd_plan_workspace_bytes": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_size_t)]),
    "frsd_plan_set_tuning": (ctypes.c_int, [_P, ctypes.POINTER(frsd_tuning)]),
    "frsd_plan_get_tuning": (ctypes.c_int, [_P, ctypes.POINTER(frsd_tuning)]),
    "frsd_plan_init": (ctypes.c_int, [_P, _P, ctypes.c_size_t, _P]),
    "frsd_mesh_assign": (ctypes.c_int, [_P, _P, ctypes.POINTER(frsd_catalog), ctypes.POINTER(frsd_catalog),
                                        ctypes.c_double, _P]),
    "frsd_random_cache": (ctypes.c_int, [_P, _P, ctypes.POINTER(frsd_catalog), _P]),
    "frsd_mesh_assign_cached": (ctypes.c_int, [_P, _P, ctypes.POINTER(frsd_catalog), ctypes.c_double, _P]),
    "frsd_pk_multipoles": (ctypes.c_int, [_P, _P, ctypes.POINTER(frsd_pk_out), _P]),
    "frsd_pk_batch": (ctypes.c_int, [_P, _P, ctypes.c_int32, _P, _P, _P, _P, _P]),
    "frsd_bk_ntriangles": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int64)]),
    "frsd_bk_grid": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32)]),
    "frsd_bk_triangles": (ctypes.c_int, [_P, _P]),
    "frsd_bk_multipoles": (ctypes.c_int, [_P, _P, ctypes.POINTER(frsd_bk_out), _P]),
    "frsd_run_static": (ctypes.c_int, [_P, ctypes.POINTER(frsd_catalog), ctypes.POINTER(frsd_catalog),
                                       ctypes.c_double, ctypes.POINTER(frsd_pk_out), ctypes.POINTER(frsd_bk_out), _P]),
    "frsd_graph_create": (ctypes.c_int, [_P, _P, ctypes.POINTER(frsd_catalog), ctypes.POINTER(frsd_catalog),
                                         ctypes.c_double, ctypes.POINTER(frsd_pk_out), ctypes.POINTER(frsd_bk_out),
                                         _P, ctypes.POINTER(_P)]),
    "frsd_graph_launch": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_int64, ctypes.c_double, _P]),
    "frsd_graph_destroy": (None, [_P]),
    "frsd_graph_create_batch": (ctypes.c_int, [_P, _P, ctypes.c_int32, _P, _P, _P, _P, _P, ctypes.POINTER(_P)]),
    "frsd_graph_launch_batch": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "frsd_status": (ctypes.c_int, [_P, _P, ctypes.POINTER(ctypes.c_int64), _P]),
    "frsd_profile": (ctypes.c_int, [ctypes.c_int]),
    "frsd_profile_report": (ctypes.c_int, [ctypes.c_char_p, ctypes.c_size_t]),
    "frsd_last_error": (ctypes.c_char_p, []),
}
for _name, (_res, _args) in _proto.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args

EXPORTED = tuple(_proto)


def _check(rc):
    if rc != FRSD_OK:
        raise FrsdError(rc, _lib.frsd_last_error().decode())


# --- thin wrappers with the C names -------------------------------------------

def frsd_last_error() -> str:
    return _lib.frsd_last_error().decode()


def frsd_plan_create(params: frsd_params) -> int:
    h = _P()
    _check(_lib.frsd_plan_create(ctypes.byref(params), ctypes.byref(h)))
    return h.value


def frsd_plan_destroy(plan: int) -> None:
    _lib.frsd_plan_destroy(plan)


def frsd_plan_workspace_bytes(plan: int) -> int:
    v = ctypes.c_size_t()
    _check(_lib.frsd_plan_workspace_bytes(plan, ctypes.byref(v)))
    return v.value


def frsd_plan_set_tuning(plan: int, tuning: dict) -> None:
    t = frsd_tuning(**{k: int(v) for k, v in tuning.items()})
    _check(_lib.frsd_plan_set_tuning(plan, ctypes.byref(t)))


def frsd_plan_get_tuning(plan: int) -> dict:
    t = frsd_tuning()
    _check(_lib.frsd_plan_get_tuning(plan, ctypes.byref(t)))
    return {name: int(getattr(t, name)) for name, _ in frsd_tuning._fields_}


def frsd_plan_init(plan: int, ws_ptr: int, ws_bytes: int, stream: int) -> None:
    _check(_lib.frsd_plan_init(plan, ws_ptr, ws_bytes, stream))


def frsd_mesh_assign(plan, ws_ptr, gal: frsd_catalog, ran: frsd_catalog, alpha: float, stream) -> None:
    _check(_lib.frsd_mesh_assign(plan, ws_ptr, ctypes.byref(gal), ctypes.byref(ran), float(alpha), stream))


def frsd_random_cache(plan, ws_ptr, ran: frsd_catalog, stream) -> None:
    _check(_lib.frsd_random_cache(plan, ws_ptr, ctypes.byref(ran), stream))


def frsd_mesh_assign_cached(plan, ws_ptr, gal: frsd_catalog, alpha: float, stream) -> None:
    _check(_lib.frsd_mesh_assign_cached(plan, ws_ptr, ctypes.byref(gal), float(alpha), stream))


def frsd_pk_multipoles(plan, ws_ptr, out: frsd_pk_out, stream) -> None:
    _check(_lib.frsd_pk_multipoles(plan, ws_ptr, ctypes.byref(out), stream))


def frsd_pk_batch(plans, ws_ptrs, gals, rans, alphas, outs, stream) -> None:
    """plans, ws_ptrs: handles and workspace addresses; gals, outs: lists of
    frsd_catalog / frsd_pk_out; rans: list of frsd_catalog, or None for
    galaxies against each plan's random cache; alphas: list of floats."""
    n = len(plans)
    if not (len(ws_ptrs) == len(gals) == len(alphas) == len(outs) == n) or (rans is not None and len(rans) != n):
        raise ValueError("every per-request list of a batch must have one entry per plan")
    p_arr = (_P * n)(*plans)
    w_arr = (_P * n)(*ws_ptrs)
    g_arr = (frsd_catalog * n)(*gals)
    r_arr = (frsd_catalog * n)(*rans) if rans is not None else None
    a_arr = (ctypes.c_double * n)(*[float(a) for a in alphas])
    o_arr = (frsd_pk_out * n)(*outs)
    _check(_lib.frsd_pk_batch(p_arr, w_arr, n, g_arr, r_arr, a_arr, o_arr, stream))


def frsd_bk_ntriangles(plan) -> int:
    v = ctypes.c_int64()
    _check(_lib.frsd_bk_ntriangles(plan, ctypes.byref(v)))
    return v.value


def frsd_bk_grid(plan) -> int:
    v = ctypes.c_int32()
    _check(_lib.frsd_bk_grid(plan, ctypes.byref(v)))
    return v.value


def frsd_bk_triangles(plan) -> np.ndarray:
    n = frsd_bk_ntriangles(plan)
    arr = np.zeros((max(n, 1), 3), dtype=np.int32)
    _check(_lib.frsd_bk_triangles(plan, arr.ctypes.data))
    return arr[:n]


def frsd_bk_multipoles(plan, ws_ptr, out: frsd_bk_out, stream) -> None:
    _check(_lib.frsd_bk_multipoles(plan, ws_ptr, ctypes.byref(out), stream))


def frsd_run_static(plan, gal: frsd_catalog, ran: frsd_catalog, alpha: float, pk: frsd_pk_out,
                    bk: frsd_bk_out | None, stream) -> None:
    _check(_lib.frsd_run_static(plan, ctypes.byref(gal), ctypes.byref(ran), float(alpha), ctypes.byref(pk),
                                ctypes.byref(bk) if bk is not None else None, stream))


def frsd_graph_create(plan, ws_ptr, gal: frsd_catalog, ran: frsd_catalog, alpha: float, pk: frsd_pk_out,
                      bk: frsd_bk_out | None, stream) -> int:
    h = _P()
    _check(_lib.frsd_graph_create(plan, ws_ptr, ctypes.byref(gal), ctypes.byref(ran), float(alpha), ctypes.byref(pk),
                                  ctypes.byref(bk) if bk is not None else None, stream, ctypes.byref(h)))
    return h.value


def frsd_graph_launch(graph: int, n_gal: int, n_ran: int, alpha: float, stream) -> None:
    _check(_lib.frsd_graph_launch(graph, int(n_gal), int(n_ran), float(alpha), stream))


def frsd_graph_destroy(graph: int) -> None:
    _lib.frsd_graph_destroy(graph)


def frsd_graph_create_batch(plans, ws_ptrs, gals, rans, alphas, outs, stream) -> int:
    n = len(plans)
    h = _P()
    _check(_lib.frsd_graph_create_batch((_P * n)(*plans), (_P * n)(*ws_ptrs), n, (frsd_catalog * n)(*gals),
                                        (frsd_catalog * n)(*rans), (ctypes.c_double * n)(*[float(a) for a in alphas]),
                                        (frsd_pk_out * n)(*outs), stream, ctypes.byref(h)))
    return h.value


def frsd_graph_launch_batch(graph: int, n_gal, n_ran, alphas, stream) -> None:
    n = len(n_gal)
    _check(_lib.frsd_graph_launch_batch(graph, (ctypes.c_int64 * n)(*[int(v) for v in n_gal]),
                                        (ctypes.c_int64 * n)(*[int(v) for v in n_ran]),
                                        (ctypes.c_double * n)(*[float(a) for a in alphas]), stream))


def frsd_status(plan, ws_ptr, stream) -> int:
    v = ctypes.c_int64()
    rc = _lib.frsd_status(plan, ws_ptr, ctypes.byref(v), stream)
    if rc not in (FRSD_OK, FRSD_EDOM):
        _check(rc)
    return v.value


def frsd_profile(enable: bool) -> None:
    _check(_lib.frsd_profile(1 if enable else 0))


def frsd_profile_report() -> dict:
    """{kernel name: (launches, total_ms)} recorded since the last report."""
    buf = ctypes.create_string_buffer(1 << 16)
    _check(_lib.frsd_profile_report(buf, len(buf)))
    out = {}
    for line in buf.value.decode().splitlines():
        name, n, ms = line.split()
        out[name] = (int(n), float(ms))
    return out


# --- convenience plan object ---------------------------------------------------

@dataclass
class Config:
    n_grid: int
    box: float
    observer: tuple
    order: int = 3
    interlace: bool = True
    compensate: bool = True
    ell_max: int = 4
    precision: int = 32
    pk_kmin: float = 0.0
    pk_dk: float = 0.0
    pk_nbins: int = 0
    bk_kmin: float = 0.0
    bk_dk: float = 0.0
    bk_nbins: int = 0
    bk_grid: int = 0
    max_objects: int = 0
    bk_ell_max: int = -1
    bk_shot_noise: bool = False
    bk_zero_area: bool = False
    random_cache: bool = False
    stream_moments: bool = False
    stream_slots: int = 0

    def to_c(self) -> frsd_params:
        p = frsd_params()
        p.n_grid, p.order, p.interlace = self.n_grid, self.order, int(self.interlace)
        p.compensate, p.ell_max, p.precision = int(self.compensate), self.ell_max, self.precision
        p.box = self.box
        for d in range(3):
            p.observer[d] = float(self.observer[d])
        p.pk_kmin, p.pk_dk, p.pk_nbins = self.pk_kmin, self.pk_dk, self.pk_nbins
        p.bk_kmin, p.bk_dk, p.bk_nbins = self.bk_kmin, self.bk_dk, self.bk_nbins
        p.bk_grid, p.max_objects = self.bk_grid, int(self.max_objects)
        p.bk_ell_max, p.bk_shot_noise, p.bk_zero_area = self.bk_ell_max, int(self.bk_shot_noise), int(self.bk_zero_area)
        p.random_cache = int(self.random_cache)
        p.stream_moments = int(self.stream_moments)
        p.stream_slots = int(self.stream_slots)
        return p


def workspace_bytes(cfg: "Config") -> int:
    """Workspace bytes a plan of this configuration needs (no device memory touched)."""
    h = frsd_plan_create(cfg.to_c())
    try:
        return frsd_plan_workspace_bytes(h)
    finally:
        frsd_plan_destroy(h)


def pinned_catalog(cat: dict, dtype=torch.float64) -> dict:
    """Copy a host catalogue (NumPy arrays) into page-locked host tensors,
    which the library reads in place (no copy to the device)."""
    return {key: torch.as_tensor(np.ascontiguousarray(cat[key]), dtype=dtype).pin_memory()
            for key in ("pos", "w", "nbar")}


def device_catalog(cat: dict | None, device, dtype=torch.float64) -> dict:
    """Copy a host catalogue (NumPy arrays) to device tensors of `dtype`."""
    if cat is None or len(cat["w"]) == 0:
        z = torch.zeros(0, device=device, dtype=dtype)
        return {"pos": z.reshape(0, 3), "w": z, "nbar": z}
    out = {}
    for key in ("pos", "w", "nbar"):
        out[key] = torch.as_tensor(np.ascontiguousarray(cat[key]), dtype=dtype).to(device)
    return out


def _c_catalog(cat: dict) -> frsd_catalog:
    c = frsd_catalog()
    n = int(cat["w"].shape[0])
    c.n = n
    if n == 0:
        c.pos = c.w = c.nbar = None
        c.dtype = FRSD_F64
        return c
    host = not cat["pos"].is_cuda
    for key in ("pos", "w", "nbar"):
        t = cat[key]
        if not t.is_contiguous() or t.is_cuda == host or (host and not t.is_pinned()):
            raise ValueError(f"catalogue array {key} must be a contiguous device tensor, or all three pinned host tensors")
    c.where = FRSD_HOST if host else FRSD_DEVICE
    dt = cat["pos"].dtype
    if dt not in (torch.float32, torch.float64) or cat["w"].dtype != dt or cat["nbar"].dtype != dt:
        raise ValueError("catalogue arrays must share one dtype, float32 or float64")
    c.dtype = FRSD_F64 if dt == torch.float64 else FRSD_F32
    c.pos, c.w, c.nbar = cat["pos"].data_ptr(), cat["w"].data_ptr(), cat["nbar"].data_ptr()
    return c


class Plan:
    """A plan plus its device workspace and output buffers on one GPU."""

    def __init__(self, cfg: Config, device="cuda", stream: torch.cuda.Stream | None = None,
                 host_outputs: bool = False):
        """host_outputs: the output arrays are page-locked host tensors that the
        kernels write over the host link (no device-to-host copy afterwards)."""
        self.cfg = cfg
        self.device = torch.device(device)
        self.host_outputs = host_outputs
        self.handle = frsd_plan_create(cfg.to_c())
        self.ws_bytes = frsd_plan_workspace_bytes(self.handle)
        # 256-byte alignment: over-allocate and offset
        self._ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self._ws.data_ptr()
        self.ws_ptr = (base + 255) & ~255
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        nb = cfg.pk_nbins
        out_dev = torch.device("cpu") if host_outputs else self.device
        f64 = dict(dtype=torch.float64, device=out_dev, pin_memory=host_outputs)
        self.pk_buf = {"n_modes": torch.zeros(nb, dtype=torch.int64, device=out_dev, pin_memory=host_outputs)}
        for key in ("k_eff", "p0", "p2", "p4", "s00", "s20", "s40", "p4b", "s22"):
            self.pk_buf[key] = torch.zeros(nb, **f64)
        self.pk_buf["scalars"] = torch.zeros(4, **f64)
        self.ntri = frsd_bk_ntriangles(self.handle) if cfg.bk_nbins > 0 else 0
        self.bk_grid = frsd_bk_grid(self.handle)
        self.bk_buf = {}
        if self.ntri:
            for key in ("nt", "t0", "t2", "t4", "b0", "b2", "b4", "sn0", "sn2", "sn4"):
                self.bk_buf[key] = torch.zeros(self.ntri, **f64)
            if cfg.bk_zero_area:
                for key in ("t220", "b4za"):
                    self.bk_buf[key] = torch.zeros(self.ntri, **f64)
        frsd_plan_init(self.handle, self.ws_ptr, self.ws_bytes, self.stream.cuda_stream)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            frsd_plan_destroy(h)
            self.handle = None

    @property
    def triangles(self) -> np.ndarray:
        return frsd_bk_triangles(self.handle)

    def mesh_assign(self, gal: dict, ran: dict | None, alpha: float) -> None:
        empty = {"pos": torch.zeros(0, 3, device=self.device, dtype=torch.float64),
                 "w": torch.zeros(0, device=self.device, dtype=torch.float64),
                 "nbar": torch.zeros(0, device=self.device, dtype=torch.float64)}
        self._gal, self._ran = gal, (ran if ran is not None else empty)  # keep alive while queued
        frsd_mesh_assign(self.handle, self.ws_ptr, _c_catalog(self._gal), _c_catalog(self._ran), alpha,
                         self.stream.cuda_stream)

    def random_cache(self, ran: dict) -> None:
        """Grid, transform and keep the random catalogue (plans with random_cache)."""
        self._ran = ran
        frsd_random_cache(self.handle, self.ws_ptr, _c_catalog(ran), self.stream.cuda_stream)

    def mesh_assign_cached(self, gal: dict, alpha: float) -> None:
        self._gal = gal
        frsd_mesh_assign_cached(self.handle, self.ws_ptr, _c_catalog(gal), alpha, self.stream.cuda_stream)

    def run_cached(self, gal: dict, alpha: float, bispectrum: bool | None = None) -> dict:
        """mesh_assign_cached + pk (+ bk); synchronises and returns host NumPy arrays."""
        self.mesh_assign_cached(gal, alpha)
        out = {k: v for k, v in self.pk().items()}
        if (bispectrum is None and self.ntri) or bispectrum:
            out.update({"bk_" + k: v for k, v in self.bk().items()})
        rej = self.status()
        if rej:
            raise FrsdError(FRSD_EDOM, f"{rej} objects outside the box or at the observer")
        return {k: v.cpu().numpy().copy() for k, v in out.items()}

    def _pk_out(self) -> frsd_pk_out:
        o = frsd_pk_out()
        for name in PK_ARRAYS:
            setattr(o, name, self.pk_buf[name].data_ptr())
        o.where = FRSD_HOST if self.host_outputs else FRSD_DEVICE
        return o

    def pk(self) -> dict:
        frsd_pk_multipoles(self.handle, self.ws_ptr, self._pk_out(), self.stream.cuda_stream)
        return self.pk_buf

    def bk(self) -> dict:
        o = frsd_bk_out()
        for name in BK_ARRAYS:
            setattr(o, name, self.bk_buf[name].data_ptr() if name in self.bk_buf else None)
        o.where = FRSD_HOST if self.host_outputs else FRSD_DEVICE
        frsd_bk_multipoles(self.handle, self.ws_ptr, o, self.stream.cuda_stream)
        return self.bk_buf

    def capture(self, gal: dict, ran: dict, alpha: float, bispectrum: bool = True) -> "Graph":
        """Capture one request on this plan's stream into a HIP graph.  gal and ran
        are the (capacity-sized) device buffers the replays read."""
        po, bo = frsd_pk_out(), frsd_bk_out()
        for name in PK_ARRAYS:
            setattr(po, name, self.pk_buf[name].data_ptr())
        for name in BK_ARRAYS:
            setattr(bo, name, self.bk_buf[name].data_ptr() if name in self.bk_buf else None)
        po.where = bo.where = FRSD_HOST if self.host_outputs else FRSD_DEVICE
        use_bk = bispectrum and self.ntri > 0
        h = frsd_graph_create(self.handle, self.ws_ptr, _c_catalog(gal), _c_catalog(ran), alpha, po,
                              bo if use_bk else None, self.stream.cuda_stream)
        return Graph(self, h, (gal, ran))

    def status(self) -> int:
        return frsd_status(self.handle, self.ws_ptr, self.stream.cuda_stream)

    def run(self, gal: dict, ran: dict | None, alpha: float, bispectrum: bool | None = None) -> dict:
        """mesh_assign + pk (+ bk); synchronises and returns host NumPy arrays."""
        self.mesh_assign(gal, ran, alpha)
        pk = self.pk()
        out = {k: v for k, v in pk.items()}
        if (bispectrum is None and self.ntri) or bispectrum:
            bk = self.bk()
            out.update({"bk_" + k: v for k, v in bk.items()})
        rej = self.status()
        if rej:
            raise FrsdError(FRSD_EDOM, f"{rej} objects outside the box or at the observer")
        return {k: v.cpu().numpy().copy() for k, v in out.items()}


def pk_batch(plans: list, gals: list, rans: list | None, alphas: list) -> list:
    """One frsd_pk_batch call: request r (gals[r], rans[r], alphas[r]) on
    plans[r]; rans None: galaxies against each plan's random cache.  The plans
    share one configuration and one stream.  Returns each plan's pk_buf
    (device tensors, valid once the stream has run the batch)."""
    if not plans:
        return []
    stream = plans[0].stream
    if any(p.stream != stream for p in plans):
        raise ValueError("the plans of a batch must share one stream")
    for r, p in enumerate(plans):  # keep the catalogues alive while queued
        p._gal = gals[r]
        if rans is not None:
            p._ran = rans[r]
    frsd_pk_batch([p.handle for p in plans], [p.ws_ptr for p in plans], [_c_catalog(g) for g in gals],
                  None if rans is None else [_c_catalog(c) for c in rans], alphas,
                  [p._pk_out() for p in plans], stream.cuda_stream)
    return [p.pk_buf for p in plans]


def run_batch(plans: list, gals: list, rans: list | None, alphas: list) -> list:
    """pk_batch, then synchronises and returns host NumPy copies per request."""
    bufs = pk_batch(plans, gals, rans, alphas)
    for p in plans:
        rej = p.status()
        if rej:
            raise FrsdError(FRSD_EDOM, f"{rej} objects outside the box or at the observer")
    return [{k: v.cpu().numpy().copy() for k, v in b.items()} for b in bufs]


def capture_batch(plans: list, gals: list, rans: list, alphas: list) -> "BatchGraph":
    """Capture one frsd_pk_batch of these requests (catalogue buffers of
    capacity size, randoms required) on the plans' common stream."""
    stream = plans[0].stream
    if any(p.stream != stream for p in plans):
        raise ValueError("the plans of a batch must share one stream")
    h = frsd_graph_create_batch([p.handle for p in plans], [p.ws_ptr for p in plans], [_c_catalog(g) for g in gals],
                                [_c_catalog(c) for c in rans], alphas, [p._pk_out() for p in plans],
                                stream.cuda_stream)
    return BatchGraph(plans, h, (gals, rans))


class BatchGraph:
    """A batch captured by capture_batch; launch() replays it with request r
    taking the first n_gal[r] / n_ran[r] objects of its buffers."""

    def __init__(self, plans, handle: int, keep):
        self.plans, self.handle, self._keep = plans, handle, keep

    def launch(self, n_gal, n_ran, alphas) -> None:
        frsd_graph_launch_batch(self.handle, n_gal, n_ran, alphas, self.plans[0].stream.cuda_stream)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            frsd_graph_destroy(h)
            self.handle = None


class Graph:
    """A request captured on a Plan; launch() replays it with the first n_gal /
    n_ran objects of the captured buffers."""

    def __init__(self, plan: Plan, handle: int, keep):
        self.plan, self.handle, self._keep = plan, handle, keep

    def launch(self, n_gal: int, n_ran: int, alpha: float) -> None:
        frsd_graph_launch(self.handle, n_gal, n_ran, alpha, self.plan.stream.cuda_stream)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            frsd_graph_destroy(h)
            self.handle = None


def kf(box: float) -> float:
    return 2.0 * math.pi / box
