"""Python binding of liblbm.so, the C ABI of include/lbm.h.

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  Arrays are numpy arrays (host) or torch tensors on the GPU
(device); each call passes the matching on_device flag.  Layouts are those
of include/lbm.h: scalar fields (nz, ny, nx), vector fields (3, nz, ny, nx),
populations (2, 19, nz, ny, nx), all float64.

torch is imported before the library is loaded so that both bind to the
same HIP runtime.  There is no fallback: if liblbm.so is missing the import
fails.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch  # noqa: F401  (HIP runtime first)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm.so")

LBM_FP64, LBM_FP32, LBM_FP16S, LBM_BF16S = 0, 1, 2, 3
PRECISIONS = {"fp64": LBM_FP64, "fp32": LBM_FP32, "fp16s": LBM_FP16S, "bf16s": LBM_BF16S}
LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EDEVICE, LBM_ENONFINITE, LBM_EMASSDRIFT = 0, -1, -2, -3, -4, -5
ERROR_NAMES = {-1: "LBM_EINVAL", -2: "LBM_ENOMEM", -3: "LBM_EDEVICE", -4: "LBM_ENONFINITE", -5: "LBM_EMASSDRIFT"}

EXPORTED = ("lbm_init", "lbm_step", "lbm_moments", "lbm_reduce", "lbm_reduce_noalloc", "lbm_get_populations",
            "lbm_set_populations", "lbm_set_fields", "lbm_set_fields_strain", "lbm_residual", "lbm_distance",
            "lbm_info", "lbm_last_error", "lbm_free",
            "lbm_batch_create", "lbm_batch_step", "lbm_batch_last_error", "lbm_batch_free")


class lbm_params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("prec", ctypes.c_int32),
        ("tau", ctypes.c_double * 2),
        ("G", ctypes.c_double),
        ("g", ctypes.c_double * 3),
        ("rho_s", ctypes.c_double),
        ("eq_kind", ctypes.c_int32),
        ("force_kind", ctypes.c_int32),
        ("check_every", ctypes.c_int32),
        ("inputs_on_device", ctypes.c_int32),
        ("mass_tol", ctypes.c_double),
        ("rho_ref", ctypes.c_double * 2),
        ("solid", ctypes.c_void_p),
        ("rho_init", ctypes.c_void_p * 2),
        ("u_init", ctypes.c_void_p),
        ("stream", ctypes.c_void_p),
        ("tile_x", ctypes.c_int32), ("tile_y", ctypes.c_int32),
        ("zchunk", ctypes.c_int32),
        ("wall_kind", ctypes.c_int32),
        ("tau_crit", ctypes.c_double),
    ]


class lbm_info_t(ctypes.Structure):
    _fields_ = [
        ("n_sites", ctypes.c_int64), ("n_fluid", ctypes.c_int64), ("steps_done", ctypes.c_int64),
        ("bytes_per_lu", ctypes.c_int32),
        ("tile_x", ctypes.c_int32), ("tile_y", ctypes.c_int32), ("zchunk", ctypes.c_int32),
        ("blocks", ctypes.c_int32),
        ("mass0", ctypes.c_double * 2),
    ]


class LBMError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None


def load_library():
    """Loads liblbm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(there is no non-GPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)
    lib.lbm_init.argtypes = [ctypes.POINTER(lbm_params), ctypes.POINTER(vp)]
    lib.lbm_step.argtypes = [vp, ctypes.c_int64]
    lib.lbm_moments.argtypes = [vp, vp, vp, vp, ctypes.c_int]
    lib.lbm_reduce.argtypes = [vp, dp]
    lib.lbm_reduce_noalloc.argtypes = [vp, vp]
    lib.lbm_get_populations.argtypes = [vp, vp, ctypes.c_int]
    lib.lbm_set_populations.argtypes = [vp, vp, ctypes.c_int]
    lib.lbm_set_fields.argtypes = [vp, vp, vp, vp, ctypes.c_int]
    lib.lbm_set_fields_strain.argtypes = [vp, vp, vp, vp, ctypes.c_int]
    lib.lbm_residual.argtypes = [vp, dp]
    lib.lbm_distance.argtypes = [vp, vp, vp, ctypes.c_int, dp]
    lib.lbm_info.argtypes = [vp, ctypes.POINTER(lbm_info_t)]
    lib.lbm_last_error.argtypes = [vp]
    lib.lbm_last_error.restype = ctypes.c_char_p
    lib.lbm_free.argtypes = [vp]
    lib.lbm_free.restype = None
    lib.lbm_batch_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int32, ctypes.POINTER(vp)]
    lib.lbm_batch_step.argtypes = [vp, ctypes.c_int64]
    lib.lbm_batch_last_error.argtypes = [vp]
    lib.lbm_batch_last_error.restype = ctypes.c_char_p
    lib.lbm_batch_free.argtypes = [vp]
    lib.lbm_batch_free.restype = None
    for name in EXPORTED:
        if name not in ("lbm_last_error", "lbm_free", "lbm_batch_last_error", "lbm_batch_free"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a, dtype=np.float64):
    """(pointer, on_device) of a numpy array or a torch tensor on the GPU."""
    if a is None:
        return None, None
    if isinstance(a, torch.Tensor):
        want = torch.float64 if dtype == np.float64 else torch.uint8
        if a.dtype != want or not a.is_contiguous():
            raise TypeError(f"tensor must be contiguous {want}")
        return a.data_ptr(), 1 if a.is_cuda else 0
    if not isinstance(a, np.ndarray) or a.dtype != dtype or not a.flags["C_CONTIGUOUS"]:
        raise TypeError(f"array must be a C-contiguous numpy {np.dtype(dtype)} array")
    return a.ctypes.data, 0


@dataclass
class Params:
    """The problem statement of include/lbm.h (Section 2 of the paper):
    lattice, storage precision, per-component tau (Eq. 5), coupling G
    (Eq. 7, paper sign), body acceleration, wall parameter rho^s, readings
    (eq_kind, force_kind), check period, initial fields and launch shape."""
    nx: int
    ny: int
    nz: int
    prec: int = LBM_FP32
    tau: tuple = (1.0, 1.0)
    G: float = 0.0
    g: tuple = (0.0, 0.0, 0.0)
    rho_s: float = 0.0
    eq_kind: int = 0
    force_kind: int = 0
    wall_kind: int = 0
    check_every: int = 0
    mass_tol: float = 0.0
    rho_ref: tuple = (0.0, 0.0)
    solid: object = None
    rho_init: tuple = (None, None)
    u_init: object = None
    stream: object = None
    tile: tuple = (0, 0)
    zchunk: int = 0
    tau_crit: float = 0.0


class Context:
    """Owns one lbm_ctx*."""

    def __init__(self, handle, params: Params):
        self.handle = ctypes.c_void_p(handle)
        self.params = params
        self.shape = (params.nz, params.ny, params.nx)
        self.n_sites = params.nx * params.ny * params.nz

    def __del__(self):
        try:
            lbm_free(self)
        except Exception:
            pass


def _check(ctx, rc):
    if rc != LBM_OK:
        lib = load_library()
        msg = lib.lbm_last_error(ctx.handle if ctx is not None else None).decode()
        raise LBMError(rc, msg)


def lbm_init(p: Params) -> Context:
    lib = load_library()
    s = lbm_params()
    s.nx, s.ny, s.nz, s.prec = p.nx, p.ny, p.nz, p.prec
    s.tau[0], s.tau[1] = p.tau
    s.G = p.G
    for d in range(3):
        s.g[d] = p.g[d]
    s.rho_s = p.rho_s
    s.eq_kind, s.force_kind, s.check_every = p.eq_kind, p.force_kind, p.check_every
    s.wall_kind = p.wall_kind
    s.mass_tol = p.mass_tol
    s.rho_ref[0], s.rho_ref[1] = p.rho_ref
    flags = set()
    keep = []
    if p.solid is not None:
        m = p.solid
        if isinstance(m, np.ndarray):
            m = np.ascontiguousarray(m, dtype=np.uint8)
        ptr, dev = _ptr(m, np.uint8)
        keep.append(m)
        s.solid = ptr
        flags.add(dev)
    for k in range(2):
        r = p.rho_init[k]
        if r is None:
            raise ValueError("rho_init needs both component densities")
        ptr, dev = _ptr(r)
        s.rho_init[k] = ptr
        flags.add(dev)
    if p.u_init is not None:
        ptr, dev = _ptr(p.u_init)
        s.u_init = ptr
        flags.add(dev)
    if len(flags) > 1:
        raise ValueError("inputs must be all on the host or all on the device")
    s.inputs_on_device = flags.pop() if flags else 0
    if p.stream is not None:
        s.stream = p.stream.cuda_stream if hasattr(p.stream, "cuda_stream") else int(p.stream)
    s.tile_x, s.tile_y = p.tile
    s.zchunk = p.zchunk
    s.tau_crit = p.tau_crit
    h = ctypes.c_void_p()
    rc = lib.lbm_init(ctypes.byref(s), ctypes.byref(h))
    if rc != LBM_OK:
        raise LBMError(rc, lib.lbm_last_error(None).decode())
    del keep
    return Context(h.value, p)


def lbm_step(ctx: Context, n: int) -> None:
    _check(ctx, load_library().lbm_step(ctx.handle, int(n)))


def lbm_moments(ctx: Context, rho1=None, rho2=None, uF=None):
    """Fills the given arrays (all host or all device); with none given,
    returns new host arrays (rho1, rho2, uF)."""
    if rho1 is None and rho2 is None and uF is None:
        rho1 = np.zeros(ctx.shape)
        rho2 = np.zeros(ctx.shape)
        uF = np.zeros((3,) + ctx.shape)
    ptrs, devs = [], set()
    for a in (rho1, rho2, uF):
        p, d = _ptr(a)
        ptrs.append(p)
        if d is not None:
            devs.add(d)
    if len(devs) > 1:
        raise ValueError("outputs must be all on the host or all on the device")
    _check(ctx, load_library().lbm_moments(ctx.handle, ptrs[0], ptrs[1], ptrs[2], devs.pop()))
    return rho1, rho2, uF


def lbm_reduce(ctx: Context) -> np.ndarray:
    out = np.zeros(5)
    _check(ctx, load_library().lbm_reduce(ctx.handle, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return out


def lbm_reduce_noalloc(ctx: Context, out):
    """The sums of lbm_reduce into out, a float64 torch tensor of 5 on the
    GPU, enqueued on the context's stream (not synchronized)."""
    p, d = _ptr(out)
    if not d or out.numel() < 5:
        raise LBMError(LBM_EINVAL, "lbm_reduce_noalloc writes a device array of 5 doubles")
    _check(ctx, load_library().lbm_reduce_noalloc(ctx.handle, p))
    return out


def lbm_get_populations(ctx: Context, f=None):
    if f is None:
        f = np.zeros((2, 19) + ctx.shape)
    p, d = _ptr(f)
    _check(ctx, load_library().lbm_get_populations(ctx.handle, p, d))
    return f


def lbm_set_populations(ctx: Context, f) -> None:
    if isinstance(f, np.ndarray):
        f = np.ascontiguousarray(f, dtype=np.float64)
    p, d = _ptr(f)
    _check(ctx, load_library().lbm_set_populations(ctx.handle, p, d))


def _field_args(rho1, rho2, u):
    """Pointers and the common on_device flag of the field arrays; the
    returned list keeps any contiguous copies alive for the call."""
    ptrs, devs, keep = [], set(), []
    for a in (rho1, rho2, u):
        if isinstance(a, np.ndarray):
            a = np.ascontiguousarray(a, dtype=np.float64)
        keep.append(a)
        p, d = _ptr(a)
        ptrs.append(p)
        if d is not None:
            devs.add(d)
    if len(devs) > 1:
        raise ValueError("inputs must be all on the host or all on the device")
    return ptrs, devs.pop(), keep


def lbm_set_fields(ctx: Context, rho1, rho2, u=None) -> None:
    ptrs, dev, keep = _field_args(rho1, rho2, u)
    _check(ctx, load_library().lbm_set_fields(ctx.handle, ptrs[0], ptrs[1], ptrs[2], dev))
    del keep


def lbm_set_fields_strain(ctx: Context, rho1, rho2, u) -> None:
    """lbm_set_fields plus the non-equilibrium part of u's strain."""
    if u is None:
        raise LBMError(LBM_EINVAL, "lbm_set_fields_strain needs a velocity field")
    ptrs, dev, keep = _field_args(rho1, rho2, u)
    _check(ctx, load_library().lbm_set_fields_strain(ctx.handle, ptrs[0], ptrs[1], ptrs[2], dev))
    del keep


def lbm_residual(ctx: Context) -> tuple[float, float]:
    """(relative change of u_F, relative change of rho1) since the previous
    call, in FP64 on the device."""
    out = np.zeros(2)
    _check(ctx, load_library().lbm_residual(ctx.handle, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return float(out[0]), float(out[1])


def lbm_distance(ctx: Context, rho1, u) -> tuple[float, float]:
    """(||u_F - u|| / ||u||, ||rho1 - rho1_given|| / ||rho1_given||) of the
    current state against given fields (host arrays or device tensors), in
    FP64 on the device."""
    ptrs, dev, keep = _field_args(rho1, u, None)
    out = np.zeros(2)
    _check(ctx, load_library().lbm_distance(ctx.handle, ptrs[0], ptrs[1], dev,
                                            out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    del keep
    return float(out[0]), float(out[1])


def lbm_info(ctx: Context) -> dict:
    i = lbm_info_t()
    _check(ctx, load_library().lbm_info(ctx.handle, ctypes.byref(i)))
    return {"n_sites": i.n_sites, "n_fluid": i.n_fluid, "steps_done": i.steps_done,
            "bytes_per_lu": i.bytes_per_lu, "tile": (i.tile_x, i.tile_y), "zchunk": i.zchunk,
            "blocks": i.blocks, "mass0": (i.mass0[0], i.mass0[1])}


def lbm_last_error(ctx: Context | None = None) -> str:
    return load_library().lbm_last_error(ctx.handle if ctx is not None else None).decode()


def lbm_free(ctx: Context) -> None:
    if ctx.handle and ctx.handle.value:
        load_library().lbm_free(ctx.handle)
        ctx.handle = ctypes.c_void_p()


class Batch:
    """Owns one lbm_batch* (and keeps its contexts alive)."""

    def __init__(self, handle, ctxs):
        self.handle = ctypes.c_void_p(handle)
        self.ctxs = list(ctxs)

    def __del__(self):
        try:
            lbm_batch_free(self)
        except Exception:
            pass


def lbm_batch_create(ctxs) -> Batch:
    lib = load_library()
    arr = (ctypes.c_void_p * len(ctxs))(*[c.handle.value for c in ctxs])
    h = ctypes.c_void_p()
    rc = lib.lbm_batch_create(arr, len(ctxs), ctypes.byref(h))
    if rc != LBM_OK:
        raise LBMError(rc, lib.lbm_batch_last_error(None).decode())
    return Batch(h.value, ctxs)


def lbm_batch_step(b: Batch, n: int) -> None:
    lib = load_library()
    rc = lib.lbm_batch_step(b.handle, int(n))
    if rc != LBM_OK:
        raise LBMError(rc, lib.lbm_batch_last_error(b.handle).decode())


def lbm_batch_last_error(b: Batch | None = None) -> str:
    return load_library().lbm_batch_last_error(b.handle if b is not None else None).decode()


def lbm_batch_free(b: Batch) -> None:
    if b.handle and b.handle.value:
        load_library().lbm_batch_free(b.handle)
        b.handle = ctypes.c_void_p()
