"""C ABI checks that need no GPU: the library loads, exports every entry
point that include/lbrt.h declares, and lbrt_validate (host-only) accepts
good problem statements and rejects each class of bad one with its code."""
import os
import re

import numpy as np
import pytest

import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    import paper_2007_05718_amd as L
    return L


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "lbrt.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(lbrt_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = _lib()
    names = declared_functions()
    assert "lbrt_step" in names and "lbrt_init" in names
    lib = L.library()
    for n in names:
        assert hasattr(lib, n), n
    for n in L.exported_symbols():
        assert n in names


def _desc(**kw):
    L = _lib()
    dirs, w = wl.lebedev(50)
    args = dict(nx=16, ny=12, nz=10, dt=0.5, dirs=dirs, weights=w)
    args.update(kw)
    return L.Desc(**args)


def test_validate_accepts_good_descriptions():
    L = _lib()
    assert L.lbrt_validate(_desc()) == L.LBRT_OK
    assert L.lbrt_validate(_desc(dt=1.0)) == L.LBRT_OK
    assert L.lbrt_validate(_desc(storage=L.LBRT_BF16)) == L.LBRT_OK
    assert L.lbrt_validate(_desc(moving_fluid=True)) == L.LBRT_OK
    assert L.lbrt_validate(_desc(bc=(1, 1, 0, 2, 1, 1))) == L.LBRT_OK
    for n in (6, 14, 26, 38, 74, 86, 110, 146):
        dirs, w = wl.lebedev(n)
        assert L.lbrt_validate(_desc(dirs=dirs, weights=w)) == L.LBRT_OK


def test_validate_rejects_bad_descriptions():
    L = _lib()
    dirs, w = wl.lebedev(50)
    assert L.lbrt_validate(_desc(dt=1.01)) == L.LBRT_E_CFL
    assert L.lbrt_validate(_desc(dt=0.0)) == L.LBRT_E_CFL
    assert L.lbrt_validate(_desc(nx=1)) == L.LBRT_E_INVAL
    assert L.lbrt_validate(_desc(weights=w * 1.001)) == L.LBRT_E_QUAD
    bad = dirs.copy()
    bad[0] *= 1.01
    assert L.lbrt_validate(_desc(dirs=bad)) == L.LBRT_E_QUAD
    shifted = dirs.copy()
    shifted[:, 0] += 0.0
    ww = w.copy()
    ww[0] += 1e-6
    ww[1] -= 1e-6                      # sum still 1, first moment broken
    assert L.lbrt_validate(_desc(weights=ww)) == L.LBRT_E_QUAD
    assert L.lbrt_validate(_desc(bc=(1, 0, 0, 0, 0, 0))) == L.LBRT_E_INVAL
    assert L.lbrt_validate(_desc(bc=(3, 3, 0, 0, 0, 0))) == L.LBRT_E_INVAL
    assert L.lbrt_validate(_desc(storage=7)) == L.LBRT_E_INVAL
    assert L.lbrt_validate(_desc(collision=5)) == L.LBRT_E_INVAL
    assert L.lbrt_validate(_desc(collision=L.LBRT_COLL_LAMBDA, lambda_iters=0)) == L.LBRT_E_INVAL
    assert (L.lbrt_validate(_desc(moving_fluid=True, collision=L.LBRT_COLL_EXPLICIT))
            == L.LBRT_E_UNSUPPORTED)
    assert L.lbrt_validate(_desc(moving_fluid=True, lam=0.5)) == L.LBRT_E_UNSUPPORTED
    assert L.lbrt_validate(_desc(scale=-np.ones(50))) == L.LBRT_E_INVAL
    # a rule that is not exact to degree 2 (Gauss-type points perturbed)
    rng = np.random.default_rng(0)
    r = rng.standard_normal((40, 3))
    r /= np.linalg.norm(r, axis=1, keepdims=True)
    assert L.lbrt_validate(_desc(dirs=r, weights=np.full(40, 1 / 40))) == L.LBRT_E_QUAD
    # too many directions
    assert L.lbrt_validate(_desc(dirs=np.tile(dirs, (5, 1)), weights=np.tile(w, 5) / 5)) \
        == L.LBRT_E_INVAL
    assert "ndir" in L.lbrt_last_error()


def test_state_bytes():
    """lbrt_state_bytes / lbrt_state_e_offset: ndir ncell elements of the
    storage type; the equilibrium-shifted forms add an FP32 E array at the
    first multiple of 256 bytes after the 16-bit deviations."""
    L = _lib()
    assert L.state_bytes(L.LBRT_FP32, 110, 1000) == 4 * 110 * 1000
    assert L.state_bytes(L.LBRT_FP64, 3, 7) == 8 * 21
    assert L.state_bytes(L.LBRT_BF16, 50, 33) == 2 * 50 * 33
    for st in (L.LBRT_BF16_SHIFTED, L.LBRT_FP16_SHIFTED):
        off = L.state_e_offset(st, 50, 33)
        assert off == 3328 and off % 256 == 0 and off >= 2 * 50 * 33
        assert L.state_bytes(st, 50, 33) == off + 4 * 33
    assert L.state_e_offset(L.LBRT_FP32, 50, 33) == 0
    assert L.library().lbrt_state_bytes(9, 50, 33) == -1


def test_validate_survives_malformed_statements():
    """Seeded malformed problem statements (bad sizes, NaN or negative
    dt/dx, broken or empty rules, unknown boundary, storage, collision and
    rounding codes) are each answered with one of the documented status
    codes and a message, never a crash; a good statement still passes after
    them."""
    import random
    L = _lib()
    rng = random.Random(5)
    rules = [wl.lebedev(k) for k in (6, 26, 110, 194)]
    codes = {L.LBRT_OK, L.LBRT_E_INVAL, L.LBRT_E_CFL, L.LBRT_E_QUAD, L.LBRT_E_UNSUPPORTED}
    for it in range(3000):
        dirs, w = (a.copy() for a in rules[rng.randrange(len(rules))])
        m = rng.random()
        if m < 0.1 and len(w) > 1:
            dirs, w = dirs[:-1], w[:-1]
        elif m < 0.2:
            dirs[rng.randrange(len(w))] *= rng.choice([0.0, 2.0, float("nan"), -1.0])
        elif m < 0.3:
            w[rng.randrange(len(w))] = rng.choice([-1.0, 0.0, float("inf"), float("nan")])
        elif m < 0.35:
            dirs, w = np.zeros((0, 3)), np.zeros(0)
        dims = [rng.choice([-5, 0, 1, 2, 3, 17, 64, 2048, 1 << 16, 1 << 30]) for _ in range(3)]
        d = L.Desc(nx=dims[0], ny=dims[1], nz=dims[2],
                   dt=rng.choice([0.5, 1.0, 1.5, 0.0, -1.0, float("nan")]), dirs=dirs, weights=w,
                   bc=[rng.choice([0, 1, 2, -1, 3, 99]) for _ in range(6)],
                   dx=rng.choice([1.0, 0.0, -2.0, float("inf")]),
                   storage=rng.choice([0, 1, 2, 3, 4, 5, 6, -1, 77]),
                   collision=rng.choice([0, 1, 2, 3, -2]),
                   lambda_iters=rng.choice([-1, 0, 1, 5, 1000]),
                   lam=rng.choice([0.0, 0.5, 3.0, -3.0, float("nan")]),
                   moving_fluid=rng.random() < 0.3, rounding=rng.choice([0, 1, 2, -1]))
        rc = L.lbrt_validate(d)
        assert rc in codes, (it, rc)
        if rc != L.LBRT_OK:
            assert L.lbrt_last_error()
    assert L.lbrt_validate(_desc()) == L.LBRT_OK
