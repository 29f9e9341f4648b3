"""Host-side argument checks of the entry points that need a context, called
through the raw C ABI (the Python binding's own checks bypassed): each bad
call returns its error code and a message, and launches nothing."""
import ctypes

import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu

import gpu_helpers as gh  # noqa: E402

vp = ctypes.c_void_p


def _p(t):
    return vp(t.data_ptr()) if t is not None else None


def _setup(npoints=26, bc=(wl.BC_OUTFLOW,) * 6, moving=False):
    torch = gh.torch_mod()
    L = gh.lib()
    dirs, w = wl.lebedev(npoints)
    desc = L.Desc(nx=12, ny=10, nz=8, dt=0.5, dirs=dirs, weights=w, bc=bc, moving_fluid=moving)
    ctx = L.lbrt_init(desc)
    n = len(w) * desc.ncell
    bufs = dict(a=torch.zeros(n, device="cuda"), b=torch.zeros(n, device="cuda"),
                f=torch.ones(desc.ncell, device="cuda"),
                v=torch.zeros(3 * desc.ncell, device="cuda"))
    return L, ctx, desc, dirs, bufs


def _step(L, ctx, B, Ia, Ib, ka="f", vel=None, inflow=None, nin=0, nsteps=1):
    lib = L.library()
    return lib.lbrt_step(ctx.handle, _p(Ia), _p(Ib), _p(B[ka]) if ka else None, _p(B["f"]),
                         _p(B["f"]), _p(vel), inflow, nin, nsteps, None, None, None, None)


def _rejects(L, rc, *words):
    assert rc == L.LBRT_E_INVAL, rc
    msg = L.lbrt_last_error()
    for w in words:
        assert w in msg, msg


def test_step_rejects_bad_buffers_and_counts():
    L, ctx, desc, dirs, B = _setup()
    _rejects(L, _step(L, ctx, B, B["a"], B["a"]), "distinct")
    _rejects(L, _step(L, ctx, B, None, B["b"]), "required")
    _rejects(L, _step(L, ctx, B, B["a"], B["b"], nsteps=-1), "nsteps")
    _rejects(L, _step(L, ctx, B, B["a"], B["b"], ka=None), "kappa")
    assert _step(L, ctx, B, B["a"], B["b"]) == L.LBRT_OK
    gh.torch_mod().cuda.synchronize()
    ctx.close()


def test_moving_step_needs_velocity():
    L, ctx, desc, dirs, B = _setup(moving=True)
    _rejects(L, _step(L, ctx, B, B["a"], B["b"]), "vel")
    assert _step(L, ctx, B, B["a"], B["b"], vel=B["v"]) == L.LBRT_OK
    gh.torch_mod().cuda.synchronize()
    ctx.close()


def test_step_rejects_bad_inflow_planes():
    torch = gh.torch_mod()
    bc = (wl.BC_INFLOW,) + (wl.BC_OUTFLOW,) * 5
    L, ctx, desc, dirs, B = _setup(bc=bc)
    plane = torch.ones(desc.c.nz * desc.c.ny, device="cuda")
    enter = int(np.argmax(dirs[:, 0]))     # enters through -x
    leave = int(np.argmin(dirs[:, 0]))     # leaves through -x

    def planes(*items):
        arr = (L.lbrt_inflow * len(items))()
        for j, (face, d) in enumerate(items):
            arr[j].face, arr[j].dir, arr[j].values = face, d, plane.data_ptr()
        return arr, len(items)

    a, n = planes((1, enter))                 # +x is not an inflow face
    _rejects(L, _step(L, ctx, B, B["a"], B["b"], inflow=a, nin=n), "not an inflow face")
    a, n = planes((0, leave))
    _rejects(L, _step(L, ctx, B, B["a"], B["b"], inflow=a, nin=n), "does not enter")
    a, n = planes((0, enter), (0, enter))
    _rejects(L, _step(L, ctx, B, B["a"], B["b"], inflow=a, nin=n), "twice")
    a, n = planes((0, len(dirs)))
    _rejects(L, _step(L, ctx, B, B["a"], B["b"], inflow=a, nin=n), "dir")
    a, n = planes((0, enter))
    _rejects(L, _step(L, ctx, B, B["a"], B["b"], inflow=None, nin=1), "NULL")
    assert _step(L, ctx, B, B["a"], B["b"], inflow=a, nin=n) == L.LBRT_OK
    torch.cuda.synchronize()
    ctx.close()


def test_tiling_and_adjoint_arguments():
    torch = gh.torch_mod()
    L, ctx, desc, dirs, B = _setup()
    lib = L.library()
    _rejects(L, lib.lbrt_set_tiling(ctx.handle, 32, 4, 8, 8), "tile")
    _rejects(L, lib.lbrt_set_tiling(ctx.handle, 24, 2, 8, 8), "power of two")
    _rejects(L, lib.lbrt_set_tiling(ctx.handle, 64, 1, 0, 8), "lengths")
    assert lib.lbrt_set_tiling(ctx.handle, 32, 2, 4, 2) == L.LBRT_OK
    assert L.lbrt_get_tiling(ctx) == (32, 2, 4, 2)
    g = torch.zeros(desc.ncell, device="cuda")
    lam = torch.zeros_like(B["a"])
    rc = lib.lbrt_adjoint_step(ctx.handle, _p(B["a"]), _p(lam), _p(B["b"]), 6, _p(g), _p(g),
                               _p(g), _p(B["f"]), _p(B["f"]), _p(B["f"]), None, None, 0, None)
    _rejects(L, rc, "detector_face")
    ctx.close()


def test_batch_rejects_mismatched_domains():
    torch = gh.torch_mod()
    L, c1, d1, _, B1 = _setup(npoints=26)
    _, c2, d2, _, B2 = _setup(npoints=110)      # another direction bucket
    lib = L.library()

    def dom(ctx, B, Ia, Ib):
        d = L.lbrt_domain()
        d.ctx, d.I_a, d.I_b = ctx.handle, Ia.data_ptr(), Ib.data_ptr()
        d.kappa_a = d.kappa_s = d.eta = B["f"].data_ptr()
        d.nsteps = 3
        return d

    out = vp()
    arr = (L.lbrt_domain * 2)(dom(c1, B1, B1["a"], B1["b"]), dom(c2, B2, B2["a"], B2["b"]))
    _rejects(L, lib.lbrt_batch_create(arr, 2, ctypes.byref(out)), "bucket")
    arr = (L.lbrt_domain * 1)(dom(c1, B1, B1["a"], B1["a"]))
    _rejects(L, lib.lbrt_batch_create(arr, 1, ctypes.byref(out)))
    _rejects(L, lib.lbrt_batch_create(arr, 0, ctypes.byref(out)), "at least one")
    _rejects(L, lib.lbrt_step_batched(None, None), "NULL")
    arr = (L.lbrt_domain * 1)(dom(c1, B1, B1["a"], B1["b"]))
    assert lib.lbrt_batch_create(arr, 1, ctypes.byref(out)) == L.LBRT_OK
    assert lib.lbrt_step_batched(out, None) == L.LBRT_OK
    torch.cuda.synchronize()
    lib.lbrt_batch_destroy(out)
    c1.close()
    c2.close()
