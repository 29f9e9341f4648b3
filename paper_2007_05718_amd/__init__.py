"""lbrt: fused stream-and-collide step of the grey radiative-transfer
lattice-Boltzmann scheme (Weih et al. 2020) on AMD MI355X.

This module is a thin ctypes binding over the C ABI in ``include/lbrt.h``:
the functions below carry the same names as the C entry points and only
marshal arguments (torch tensors -> device pointers, the current torch
stream -> hipStream_t).  Every step of the computation runs in the HIP
kernels of ``_lib/liblbrt.so``; there is no Python or CPU fallback, and
importing this module fails loudly when the library has not been built
(``python paper_2007_05718_amd/build.py``).
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "liblbrt.so")

LBRT_OK, LBRT_E_INVAL, LBRT_E_CFL, LBRT_E_QUAD = 0, -1, -2, -3
LBRT_E_NOMEM, LBRT_E_HIP, LBRT_E_UNSUPPORTED = -4, -5, -6
LBRT_BC_OUTFLOW, LBRT_BC_PERIODIC, LBRT_BC_INFLOW = 0, 1, 2
LBRT_FP32, LBRT_FP64, LBRT_BF16, LBRT_FP16 = 0, 1, 2, 3
LBRT_BF16_SHIFTED, LBRT_FP16_SHIFTED = 4, 5
LBRT_COLL_IMPLICIT, LBRT_COLL_EXPLICIT, LBRT_COLL_LAMBDA = 0, 1, 2
LBRT_ROUND_STOCHASTIC, LBRT_ROUND_NEAREST = 0, 1
LBRT_MAX_DIRS, LBRT_MAX_INFLOW, LBRT_DIAG_LEN = 200, 32, 9

STORAGE_BYTES = {LBRT_FP32: 4, LBRT_FP64: 8, LBRT_BF16: 2, LBRT_FP16: 2}
STORAGE_NAMES = {LBRT_FP32: "fp32", LBRT_FP64: "fp64", LBRT_BF16: "bf16", LBRT_FP16: "fp16"}


class lbrt_desc(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("dx", ctypes.c_double), ("dt", ctypes.c_double),
        ("ndir", ctypes.c_int32),
        ("dirs", ctypes.POINTER(ctypes.c_double)),
        ("weights", ctypes.POINTER(ctypes.c_double)),
        ("scale", ctypes.POINTER(ctypes.c_double)),
        ("bc", ctypes.c_int32 * 6),
        ("storage", ctypes.c_int32),
        ("collision", ctypes.c_int32),
        ("lambda_iters", ctypes.c_int32),
        ("lambda_aniso", ctypes.c_double),
        ("moving_fluid", ctypes.c_int32),
        ("rounding", ctypes.c_int32),
    ]


class lbrt_inflow(ctypes.Structure):
    _fields_ = [("face", ctypes.c_int32), ("dir", ctypes.c_int32),
                ("values", ctypes.c_void_p)]


class lbrt_domain(ctypes.Structure):
    _fields_ = [("ctx", ctypes.c_void_p), ("I_a", ctypes.c_void_p), ("I_b", ctypes.c_void_p),
                ("kappa_a", ctypes.c_void_p), ("kappa_s", ctypes.c_void_p),
                ("eta", ctypes.c_void_p), ("vel", ctypes.c_void_p), ("nsteps", ctypes.c_int32),
                ("E", ctypes.c_void_p), ("F", ctypes.c_void_p)]


class lbrt_coupling_out(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in ("E", "F", "P", "J", "H", "S")]


class LbrtError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"lbrt error {code}: {msg}")
        self.code = code


def _load():
    # torch's bundled HIP runtime must be the one in the process: importing
    # torch first makes the library bind to it rather than to a second copy.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"lbrt HIP library missing at {LIB_PATH}; build it with "
                          "`python paper_2007_05718_amd/build.py`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)
    lib.lbrt_validate.argtypes = [ctypes.POINTER(lbrt_desc)]
    lib.lbrt_validate.restype = ctypes.c_int
    lib.lbrt_init.argtypes = [ctypes.POINTER(lbrt_desc), ctypes.POINTER(vp)]
    lib.lbrt_init.restype = ctypes.c_int
    lib.lbrt_destroy.argtypes = [vp]
    lib.lbrt_destroy.restype = None
    lib.lbrt_step.argtypes = [vp, vp, vp, vp, vp, vp, vp, ctypes.POINTER(lbrt_inflow), i32,
                              i32, vp, vp, vp, vp]
    lib.lbrt_step.restype = ctypes.c_int
    lib.lbrt_step_noalloc.argtypes = lib.lbrt_step.argtypes
    lib.lbrt_step_noalloc.restype = ctypes.c_int
    lib.lbrt_moments.argtypes = [vp, vp, vp, vp, vp]
    lib.lbrt_moments.restype = ctypes.c_int
    lib.lbrt_coupling.argtypes = [vp, vp, vp, vp, vp, vp, ctypes.POINTER(lbrt_coupling_out), vp]
    lib.lbrt_coupling.restype = ctypes.c_int
    lib.lbrt_state_bytes.argtypes = [i32, i32, ctypes.c_int64]
    lib.lbrt_state_bytes.restype = ctypes.c_int64
    lib.lbrt_state_e_offset.argtypes = [i32, i32, ctypes.c_int64]
    lib.lbrt_state_e_offset.restype = ctypes.c_int64
    lib.lbrt_convert.argtypes = [vp, vp, i32, vp, i32, vp]
    lib.lbrt_convert.restype = ctypes.c_int
    lib.lbrt_adjoint_step.argtypes = [vp, vp, vp, vp, i32, vp, vp, vp, vp, vp, vp, vp,
                                      ctypes.POINTER(lbrt_inflow), i32, vp]
    lib.lbrt_adjoint_step.restype = ctypes.c_int
    lib.lbrt_set_tiling.argtypes = [vp, i32, i32, i32, i32]
    lib.lbrt_set_tiling.restype = ctypes.c_int
    pi32 = ctypes.POINTER(i32)
    lib.lbrt_get_tiling.argtypes = [vp, pi32, pi32, pi32, pi32]
    lib.lbrt_get_tiling.restype = ctypes.c_int
    lib.lbrt_batch_create.argtypes = [ctypes.POINTER(lbrt_domain), i32, ctypes.POINTER(vp)]
    lib.lbrt_batch_create.restype = ctypes.c_int
    lib.lbrt_step_batched.argtypes = [vp, vp]
    lib.lbrt_step_batched.restype = ctypes.c_int
    lib.lbrt_batch_destroy.argtypes = [vp]
    lib.lbrt_batch_destroy.restype = None
    lib.lbrt_stream_copy.argtypes = [vp, vp, ctypes.c_int64, vp]
    lib.lbrt_stream_copy.restype = ctypes.c_int
    lib.lbrt_last_error.argtypes = []
    lib.lbrt_last_error.restype = ctypes.c_char_p
    return lib


_lib = _load()


def lbrt_last_error() -> str:
    return (_lib.lbrt_last_error() or b"").decode()


def _check(rc: int) -> None:
    if rc != LBRT_OK:
        raise LbrtError(rc, lbrt_last_error())


class Desc:
    """An ``lbrt_desc`` plus the host arrays it points to."""

    def __init__(self, nx: int, ny: int, nz: int, dt: float, dirs, weights,
                 bc: Sequence[int] = (LBRT_BC_OUTFLOW,) * 6, dx: float = 1.0,
                 storage: int = LBRT_FP32, collision: int = LBRT_COLL_IMPLICIT,
                 lambda_iters: int = 5, lam: float = 0.0, moving_fluid: bool = False,
                 scale=None, rounding: int = LBRT_ROUND_STOCHASTIC):
        self.dirs = np.ascontiguousarray(dirs, dtype=np.float64).reshape(-1, 3)
        self.weights = np.ascontiguousarray(weights, dtype=np.float64).reshape(-1)
        self.scale = None if scale is None else np.ascontiguousarray(scale, dtype=np.float64)
        d = lbrt_desc()
        d.nx, d.ny, d.nz = int(nx), int(ny), int(nz)
        d.dx, d.dt = float(dx), float(dt)
        d.ndir = int(self.weights.shape[0])
        dptr = ctypes.POINTER(ctypes.c_double)
        d.dirs = self.dirs.ctypes.data_as(dptr)
        d.weights = self.weights.ctypes.data_as(dptr)
        d.scale = self.scale.ctypes.data_as(dptr) if self.scale is not None else None
        for f in range(6):
            d.bc[f] = int(bc[f])
        d.storage = int(storage)
        d.collision = int(collision)
        d.lambda_iters = int(lambda_iters)
        d.lambda_aniso = float(lam)
        d.moving_fluid = 1 if moving_fluid else 0
        d.rounding = int(rounding)
        self.c = d

    @property
    def ncell(self) -> int:
        return self.c.nx * self.c.ny * self.c.nz

    @property
    def ndir(self) -> int:
        return self.c.ndir

    @classmethod
    def from_problem(cls, prob, storage: int = LBRT_FP32, **kw) -> "Desc":
        args = dict(nx=prob.nx, ny=prob.ny, nz=prob.nz, dt=prob.dt, dirs=prob.dirs,
                    weights=prob.weights, bc=prob.bc, dx=prob.dx, storage=storage,
                    collision=prob.collision, lambda_iters=prob.lambda_iters, lam=prob.lam,
                    moving_fluid=prob.vel is not None)
        args.update(kw)
        return cls(**args)


def lbrt_validate(desc: Desc) -> int:
    """Host-only validation; returns the lbrt status code."""
    return int(_lib.lbrt_validate(ctypes.byref(desc.c)))


class Context:
    """Owns an ``lbrt_ctx``; destroyed with ``lbrt_destroy`` when collected."""

    def __init__(self, handle: int, desc: Desc):
        self.handle = ctypes.c_void_p(handle)
        self.desc = desc

    def close(self):
        if self.handle:
            _lib.lbrt_destroy(self.handle)
            self.handle = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def lbrt_init(desc: Desc) -> Context:
    h = ctypes.c_void_p()
    _check(_lib.lbrt_init(ctypes.byref(desc.c), ctypes.byref(h)))
    return Context(h.value, desc)


def lbrt_destroy(ctx: Context) -> None:
    ctx.close()


# ---------------------------------------------------------------------------
# torch marshalling
# ---------------------------------------------------------------------------
def _torch():
    import torch
    return torch


def _ptr(t, what: str, numel: Optional[int] = None, dtype=None):
    if t is None:
        return None
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{what}: expected a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{what}: tensor must live on the GPU")
    if not t.is_contiguous():
        raise ValueError(f"{what}: tensor must be contiguous")
    if dtype is not None and t.dtype not in (dtype if isinstance(dtype, tuple) else (dtype,)):
        raise ValueError(f"{what}: dtype {t.dtype} not accepted")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{what}: {t.numel()} elements, expected {numel}")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is not None:
        return ctypes.c_void_p(int(stream))
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _pop_dtype(storage: int):
    torch = _torch()
    return {LBRT_FP32: torch.float32, LBRT_FP64: torch.float64,
            LBRT_BF16: (torch.bfloat16, torch.int16, torch.uint16),
            LBRT_FP16: (torch.float16, torch.int16, torch.uint16)}[storage]


def _is_shifted(storage: int) -> bool:
    return storage in (LBRT_BF16_SHIFTED, LBRT_FP16_SHIFTED)


def state_bytes(storage: int, ndir: int, ncell: int) -> int:
    """Bytes of one state buffer (lbrt_state_bytes)."""
    v = _lib.lbrt_state_bytes(int(storage), int(ndir), int(ncell))
    if v < 0:
        raise ValueError(f"storage {storage} is not a storage type")
    return int(v)


def state_e_offset(storage: int, ndir: int, ncell: int) -> int:
    """Byte offset of the E array of an equilibrium-shifted state (else 0)."""
    return int(_lib.lbrt_state_e_offset(int(storage), int(ndir), int(ncell)))


def alloc_state(ctx: "Context", storage: Optional[int] = None):
    """An uninitialised state buffer on the GPU for the context's problem (a
    uint8 tensor of lbrt_state_bytes for the equilibrium-shifted forms, else
    a tensor of the storage type)."""
    torch = _torch()
    d = ctx.desc
    st = d.c.storage if storage is None else storage
    if _is_shifted(st):
        return torch.empty(state_bytes(st, d.ndir, d.ncell), dtype=torch.uint8, device="cuda")
    dt = {LBRT_FP32: torch.float32, LBRT_FP64: torch.float64, LBRT_BF16: torch.bfloat16,
          LBRT_FP16: torch.float16}[st]
    return torch.empty(d.ndir * d.ncell, dtype=dt, device="cuda")


def _state(t, what: str, desc: "Desc", storage: Optional[int] = None):
    """Pointer of a state buffer, checked against the problem's size: a
    tensor of the storage type with ndir * ncell elements, or for the
    equilibrium-shifted forms a uint8 tensor of lbrt_state_bytes."""
    st = desc.c.storage if storage is None else storage
    if _is_shifted(st):
        return _ptr(t, what, state_bytes(st, desc.ndir, desc.ncell), _torch().uint8)
    return _ptr(t, what, desc.ndir * desc.ncell, _pop_dtype(st))


def _moment_dtype(storage: int):
    torch = _torch()
    return torch.float64 if storage == LBRT_FP64 else torch.float32


def _face_plane_size(desc: "Desc", face: int) -> int:
    """Elements of an inflow ghost plane on ``face`` (layouts of lbrt.h:
    x faces [z][y], y faces [z][x], z faces [y][x])."""
    nx, ny, nz = desc.c.nx, desc.c.ny, desc.c.nz
    return {0: nz * ny, 1: nz * nx, 2: ny * nx}[int(face) >> 1]


def _inflow_planes(desc: "Desc", inflow):
    if not inflow:
        return None, 0
    nin = len(inflow)
    planes = (lbrt_inflow * nin)()
    for j, (face, direction, vals) in enumerate(inflow):
        if not 0 <= int(face) <= 5:
            raise ValueError(f"inflow[{j}]: face {face} outside [0, 5]")
        planes[j].face = int(face)
        planes[j].dir = int(direction)
        planes[j].values = _ptr(vals, f"inflow[{j}]", _face_plane_size(desc, face),
                                dtype=_torch().float32).value
    return planes, nin


def lbrt_step(ctx: Context, I_a, I_b, kappa_a, kappa_s, eta, vel=None, inflow=None,
              nsteps: int = 1, E=None, F=None, diag=None, stream=None) -> None:
    """``nsteps`` steps, ping-pong between I_a and I_b (result in I_b when
    nsteps is odd).  ``inflow`` is a list of (face, dir, values_tensor)."""
    d = ctx.desc
    n, nc = d.ndir, d.ncell
    st = d.c.storage
    planes, nin = _inflow_planes(d, inflow)
    f32 = _torch().float32
    rc = _lib.lbrt_step(
        ctx.handle, _state(I_a, "I_a", d),
        _state(I_b, "I_b", d),
        _ptr(kappa_a, "kappa_a", nc, f32), _ptr(kappa_s, "kappa_s", nc, f32),
        _ptr(eta, "eta", nc, f32), _ptr(vel, "vel", 3 * nc, f32), planes, nin, int(nsteps),
        _ptr(E, "E", nc, _moment_dtype(st)), _ptr(F, "F", 3 * nc, _moment_dtype(st)),
        _ptr(diag, "diag", LBRT_DIAG_LEN, _torch().float64), _stream(stream))
    _check(rc)


def lbrt_step_noalloc(ctx: Context, I_a, I_b, kappa_a, kappa_s, eta, vel=None, inflow=None,
                      nsteps: int = 1, E=None, F=None, diag=None, stream=None) -> None:
    """``lbrt_step`` through the entry point that allocates nothing (its work
    memory is the library's fixed per-GPU scratch); same arguments."""
    d = ctx.desc
    n, nc = d.ndir, d.ncell
    st = d.c.storage
    planes, nin = _inflow_planes(d, inflow)
    f32 = _torch().float32
    rc = _lib.lbrt_step_noalloc(
        ctx.handle, _state(I_a, "I_a", d),
        _state(I_b, "I_b", d),
        _ptr(kappa_a, "kappa_a", nc, f32), _ptr(kappa_s, "kappa_s", nc, f32),
        _ptr(eta, "eta", nc, f32), _ptr(vel, "vel", 3 * nc, f32), planes, nin, int(nsteps),
        _ptr(E, "E", nc, _moment_dtype(st)), _ptr(F, "F", 3 * nc, _moment_dtype(st)),
        _ptr(diag, "diag", LBRT_DIAG_LEN, _torch().float64), _stream(stream))
    _check(rc)


def lbrt_adjoint_step(ctx: Context, I_n, lam_next, lam_out, detector_face: int, g_kappa_a,
                      g_kappa_s, g_eta, kappa_a, kappa_s, eta, vel=None, inflow=None,
                      stream=None) -> None:
    """Adjoint of one step (see include/lbrt.h): lam_out = d + S^T (dC/dI*)^T
    lam_next, and the step's field gradients are added into g_*."""
    d = ctx.desc
    n, nc = d.ndir, d.ncell
    st = d.c.storage
    planes, nin = _inflow_planes(d, inflow)
    f32 = _torch().float32
    gdt = _moment_dtype(st)
    _check(_lib.lbrt_adjoint_step(
        ctx.handle, _state(I_n, "I_n", d),
        _state(lam_next, "lam_next", d),
        _state(lam_out, "lam_out", d), int(detector_face),
        _ptr(g_kappa_a, "g_kappa_a", nc, gdt), _ptr(g_kappa_s, "g_kappa_s", nc, gdt),
        _ptr(g_eta, "g_eta", nc, gdt),
        _ptr(kappa_a, "kappa_a", nc, f32), _ptr(kappa_s, "kappa_s", nc, f32),
        _ptr(eta, "eta", nc, f32), _ptr(vel, "vel", 3 * nc, f32), planes, nin,
        _stream(stream)))


def lbrt_moments(ctx: Context, I, E=None, F=None, stream=None) -> None:
    d = ctx.desc
    st = d.c.storage
    _check(_lib.lbrt_moments(ctx.handle, _state(I, "I", d),
                             _ptr(E, "E", d.ncell, _moment_dtype(st)),
                             _ptr(F, "F", 3 * d.ncell, _moment_dtype(st)), _stream(stream)))


def lbrt_coupling(ctx: Context, I, vel=None, kappa_a=None, kappa_s=None, eta=None,
                  E=None, F=None, P=None, J=None, H=None, S=None, stream=None) -> None:
    """Moments, fluid-frame J, H and the radiative sources of a state (the
    C entry point of the same name); outputs not given are not computed."""
    d = ctx.desc
    st = d.c.storage
    torch = _torch()
    md = _moment_dtype(st)
    n = d.ncell
    out = lbrt_coupling_out(
        _ptr(E, "E", n, md), _ptr(F, "F", 3 * n, md), _ptr(P, "P", 6 * n, md),
        _ptr(J, "J", n, md), _ptr(H, "H", 4 * n, md), _ptr(S, "S", 4 * n, md))
    _check(_lib.lbrt_coupling(
        ctx.handle, _state(I, "I", d),
        _ptr(vel, "vel", 3 * n, torch.float32), _ptr(kappa_a, "kappa_a", n, torch.float32),
        _ptr(kappa_s, "kappa_s", n, torch.float32), _ptr(eta, "eta", n, torch.float32),
        ctypes.byref(out), _stream(stream)))


def lbrt_convert(ctx: Context, src, src_storage: int, dst, dst_storage: int,
                 stream=None) -> None:
    d = ctx.desc
    _check(_lib.lbrt_convert(ctx.handle, _state(src, "src", d, src_storage),
                             int(src_storage), _state(dst, "dst", d, dst_storage),
                             int(dst_storage), _stream(stream)))


def lbrt_set_tiling(ctx: Context, tx: int, ty: int, zlen: int, zlen_general: int) -> None:
    """Tile shape and z-range lengths of the context's kernels (speed only)."""
    _check(_lib.lbrt_set_tiling(ctx.handle, int(tx), int(ty), int(zlen), int(zlen_general)))


def lbrt_get_tiling(ctx: Context):
    """The context's current (tx, ty, zlen, zlen_general)."""
    v = [ctypes.c_int32() for _ in range(4)]
    _check(_lib.lbrt_get_tiling(ctx.handle, *[ctypes.byref(x) for x in v]))
    return tuple(int(x.value) for x in v)


class Batch:
    """Owns an ``lbrt_batch`` plan and keeps its domains' tensors alive."""

    def __init__(self, handle: int, keep):
        self.handle = ctypes.c_void_p(handle)
        self._keep = keep

    def close(self):
        if self.handle:
            _lib.lbrt_batch_destroy(self.handle)
            self.handle = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def lbrt_batch_create(domains) -> Batch:
    """``domains``: sequence of dicts with keys ctx, I_a, I_b, kappa_a, kappa_s,
    eta, nsteps and optionally vel, E, F (torch tensors on the GPU)."""
    arr = (lbrt_domain * len(domains))()
    f32 = _torch().float32
    for k, dm in enumerate(domains):
        ctx = dm["ctx"]
        d = ctx.desc
        n, nc, st = d.ndir, d.ncell, d.c.storage
        arr[k].ctx = ctx.handle.value
        arr[k].I_a = _state(dm["I_a"], f"domains[{k}].I_a", d).value
        arr[k].I_b = _state(dm["I_b"], f"domains[{k}].I_b", d).value
        arr[k].kappa_a = _ptr(dm["kappa_a"], "kappa_a", nc, f32).value
        arr[k].kappa_s = _ptr(dm["kappa_s"], "kappa_s", nc, f32).value
        arr[k].eta = _ptr(dm["eta"], "eta", nc, f32).value
        v = _ptr(dm.get("vel"), "vel", 3 * nc, f32)
        arr[k].vel = v.value if v is not None else None
        arr[k].nsteps = int(dm["nsteps"])
        e = _ptr(dm.get("E"), "E", nc, _moment_dtype(st))
        fF = _ptr(dm.get("F"), "F", 3 * nc, _moment_dtype(st))
        arr[k].E = e.value if e is not None else None
        arr[k].F = fF.value if fF is not None else None
    h = ctypes.c_void_p()
    _check(_lib.lbrt_batch_create(arr, len(domains), ctypes.byref(h)))
    return Batch(h.value, list(domains))


def lbrt_step_batched(batch: Batch, stream=None) -> None:
    _check(_lib.lbrt_step_batched(batch.handle, _stream(stream)))


def lbrt_batch_destroy(batch: Batch) -> None:
    batch.close()


def lbrt_stream_copy(src, dst, stream=None) -> None:
    """Streaming copy of a device tensor into another of the same size (the
    bandwidth ceiling of the measurements)."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("src and dst differ in size")
    _check(_lib.lbrt_stream_copy(_ptr(src, "src"), _ptr(dst, "dst"), int(nbytes),
                                 _stream(stream)))


def exported_symbols() -> list:
    """Names of the C entry points the binding wraps."""
    return ["lbrt_validate", "lbrt_init", "lbrt_destroy", "lbrt_step", "lbrt_step_noalloc",
            "lbrt_moments", "lbrt_coupling", "lbrt_state_bytes", "lbrt_state_e_offset",
            "lbrt_convert", "lbrt_adjoint_step", "lbrt_set_tiling", "lbrt_get_tiling",
            "lbrt_batch_create", "lbrt_step_batched", "lbrt_batch_destroy", "lbrt_stream_copy",
            "lbrt_last_error"]


def library():
    return _lib
