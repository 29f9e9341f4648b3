"""GPU parity at the full workload sizes, in the launch configuration that
bench.py times (default tiling, inflow ghosts, E, F and FP64 diagnostics on):

* crossing beams + opaque sphere, 256^3 x 110 directions, FP32, BF16, FP16
  and equilibrium-shifted BF16 storage, one step from a seeded random state,
  checked against the FP64
  oracle's one-step update at sampled cells (interior, faces, edges,
  corners, tile and z-range seams, both beam footprints, the sphere);
* the moving-fluid shear flow, 192^3 x 146, one step, same check;
* the adjoint at 192^3 x 146: the gradient of the energy leaving through +x
  against a central finite difference of the forward runs.

The sampled-cell oracle (`step_cells`) is pinned against the full oracle
step in the CPU tests.  Host memory: the 256^3 x 110 FP32 state is 7.4 GB.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import lbrt_oracle as orc

pytestmark = pytest.mark.gpu

import gpu_helpers as gh  # noqa: E402


def _sample_cells(prob, rng, extra=()):
    nz, ny, nx = prob.shape
    cells = [np.stack([rng.integers(0, nz, 150), rng.integers(0, ny, 150),
                       rng.integers(0, nx, 150)], axis=1)]
    for axis in range(3):              # 15 cells on each of the six faces
        for side in (0, (nz, ny, nx)[axis] - 1):
            c = np.stack([rng.integers(0, nz, 15), rng.integers(0, ny, 15),
                          rng.integers(0, nx, 15)], axis=1)
            c[:, axis] = side
            cells.append(c)
    for z in (0, nz - 1):              # corners
        for y in (0, ny - 1):
            for x in (0, nx - 1):
                cells.append(np.array([[z, y, x]]))
    seams_x = [v for v in (63, 64, 127, 128, 191, 192) if v < nx]
    seams_z = [v for v in (15, 16, 31, 32, 33, nz - 33, nz - 32) if 0 <= v < nz]
    cells.append(np.stack([rng.choice(seams_z, 40), rng.choice([0, 1, 2, ny - 3, ny - 2, ny - 1], 40),
                           rng.choice(seams_x, 40)], axis=1))
    for c in extra:
        cells.append(np.asarray(c, dtype=np.int64).reshape(-1, 3))
    return np.unique(np.concatenate(cells).astype(np.int64), axis=0)


def _random_state(prob, seed):
    """Seeded uniform state, I_i = w_i U(0, 1), as float32 [dir, z, y, x]."""
    rng = np.random.default_rng(seed)
    I0 = np.empty((prob.ndir,) + prob.shape, dtype=np.float32)
    for i in range(prob.ndir):
        I0[i] = rng.random(prob.shape, dtype=np.float32)
        I0[i] *= np.float32(prob.weights[i])
    return I0


class _Shifted:
    """Directions of an equilibrium-shifted state, s_i d_i + w_i E, as
    float64 values on demand."""

    def __init__(self, q16, E, weights, scale):
        self.q16, self.E, self.w, self.scale = q16, E.astype(np.float64), weights, scale
        self._i, self._v = None, None

    def __getitem__(self, i):
        if i != self._i:
            self._i = i
            self._v = (self.q16[i].float().double().numpy() * float(self.scale[i])
                       + float(self.w[i]) * self.E)
        return self._v


class _Scaled:
    """Directions of a reduced-storage state as float64 values on demand."""

    def __init__(self, q16, scale):
        self.q16, self.scale = q16, scale
        self._i, self._v = None, None

    def __getitem__(self, i):      # the oracle reads a direction once per tap
        if i != self._i:
            self._i, self._v = i, self.q16[i].float().double().numpy() * float(self.scale[i])
        return self._v


def _gpu_step(prob, state_dev, storage):
    torch = gh.torch_mod()
    L = gh.lib()
    ctx = L.lbrt_init(L.Desc.from_problem(prob, storage=storage))
    ka, ks, eta, vel, inflow = gh.upload_fields(prob)
    Ib = torch.empty_like(state_dev)
    mdt = torch.float64 if storage == L.LBRT_FP64 else torch.float32
    E = torch.empty(prob.ncell, dtype=mdt, device="cuda")
    F = torch.empty(3 * prob.ncell, dtype=mdt, device="cuda")
    diag = torch.zeros(L.LBRT_DIAG_LEN, dtype=torch.float64, device="cuda")
    L.lbrt_step(ctx, state_dev, Ib, ka, ks, eta, vel=vel, inflow=inflow or None, nsteps=1,
                E=E, F=F, diag=diag)
    torch.cuda.synchronize()
    return ctx, Ib, E, F


def _gather(ctx, prob, out, E, F, cells, storage):
    torch = gh.torch_mod()
    L = gh.lib()
    idx = torch.as_tensor(cells[:, 0] * prob.ny * prob.nx + cells[:, 1] * prob.nx + cells[:, 2],
                          device="cuda")
    if storage in (L.LBRT_BF16, L.LBRT_FP16, L.LBRT_BF16_SHIFTED, L.LBRT_FP16_SHIFTED):
        dec = torch.empty(prob.ndir * prob.ncell, dtype=torch.float32, device="cuda")
        L.lbrt_convert(ctx, out, storage, dec, L.LBRT_FP32)
        out = dec
    I = out.view(prob.ndir, prob.ncell)[:, idx].double().cpu().numpy()
    e = E[idx].double().cpu().numpy()
    f = F.view(3, prob.ncell)[:, idx].double().cpu().numpy()
    return I, e, f


def _check(prob, I_gpu, E_gpu, F_gpu, ref, tol_I, tol_EF):
    E_ref = ref.sum(axis=0)
    F_ref = prob.dirs.T @ ref
    scale = np.max(np.abs(ref), axis=0) + 1e-300
    err_I = np.max(np.abs(I_gpu - ref) / scale)
    err_E = np.max(np.abs(E_gpu - E_ref) / (np.abs(E_ref) + 1e-300))
    err_F = np.max(np.abs(F_gpu - F_ref)) / np.max(np.abs(F_ref))
    print(f"{prob.name}: {ref.shape[1]} cells, max rel err I {err_I:.2e} E {err_E:.2e} "
          f"F {err_F:.2e}", flush=True)
    assert err_I < tol_I
    assert err_E < tol_EF
    assert err_F < tol_EF


def _beam_cells(prob):
    s = prob.nx / 256.0
    zc, yc, xc = int(128 * s), int(96 * s), int(32 * s)
    a = [[zc + dz, yc + dy, x] for dz in (-3, 0, 4) for dy in (-2, 0, 3) for x in (0, 1)]
    b = [[int(98 * s) + dz, y, xc + dx] for dz in (-3, 0, 4) for dx in (-2, 0, 3) for y in (0, 1)]
    c = prob.meta["obstacle_centre"]
    r = prob.meta["obstacle_radius"]
    sph = [[int(c[2]), int(c[1]), int(c[0] - r + k)] for k in (-1, 0, 1, 2)]
    sph += [[int(c[2]), int(c[1]), int(c[0])]]
    return a + b + sph


@pytest.mark.parametrize("scatter", [False, True])
def test_beams_256_fp32_sampled_cells(scatter):
    torch = gh.torch_mod()
    L = gh.lib()
    prob = wl.beams(n=256, alloc_state=False)
    if scatter:   # the full collision: scattering and emission fields too
        rng = np.random.default_rng(77)
        prob.kappa_s = (10.0 ** rng.uniform(-2, 1, prob.shape)).astype(np.float32)
        prob.eta = (10.0 ** rng.uniform(-3, 0, prob.shape)).astype(np.float32)
    print(prob.name, prob.shape, prob.ndir, "scatter" if scatter else "", flush=True)
    I0 = _random_state(prob, 2026)
    state = torch.from_numpy(I0).reshape(-1).cuda()
    ctx, out, E, F = _gpu_step(prob, state, L.LBRT_FP32)
    del state
    cells = _sample_cells(prob, np.random.default_rng(5), extra=_beam_cells(prob))
    I_gpu, E_gpu, F_gpu = _gather(ctx, prob, out, E, F, cells, L.LBRT_FP32)
    del out, E, F
    ctx.close()
    torch.cuda.empty_cache()
    ref = orc.step_cells(I0, prob, cells)
    _check(prob, I_gpu, E_gpu, F_gpu, ref, 1e-5, 1e-5)


@pytest.mark.parametrize("fmt", ["bf16", "fp16"])
def test_beams_256_16bit_sampled_cells(fmt):
    torch = gh.torch_mod()
    L = gh.lib()
    st, tdt, p = {"bf16": (L.LBRT_BF16, torch.bfloat16, 8), "fp16": (L.LBRT_FP16, torch.float16, 11)}[fmt]
    prob = wl.beams(n=256, alloc_state=False)
    print(prob.name, prob.shape, prob.ndir, fmt, flush=True)
    scale = np.abs(prob.weights)
    g = torch.Generator().manual_seed(2027)
    q16 = torch.empty((prob.ndir,) + prob.shape, dtype=tdt)
    for i in range(prob.ndir):       # stored values U(0, 1): I_i = w_i q
        q16[i] = torch.rand(prob.shape, generator=g).to(tdt)
    state = q16.reshape(-1).cuda()
    ctx, out, E, F = _gpu_step(prob, state, st)
    del state
    cells = _sample_cells(prob, np.random.default_rng(6), extra=_beam_cells(prob))
    I_gpu, E_gpu, F_gpu = _gather(ctx, prob, out, E, F, cells, st)
    del out, E, F
    ctx.close()
    torch.cuda.empty_cache()
    ref = orc.step_cells(_Scaled(q16, scale), prob, cells)
    # one stochastic rounding of each stored value to the format (p
    # significant bits: 8 for BF16, 11 for FP16) picks one of the two
    # neighbouring representable values, so it is within one unit in the
    # last place, 2^(1 - p) of a value just above a power of two, plus a few
    # FP32 roundings; E and F (from the FP32 collision) to the
    # precision-form bound
    _check(prob, I_gpu, E_gpu, F_gpu, ref, 2.0 ** (1 - p) * (1 + 1e-4), 2e-3)


def test_beams_256_bf16_shifted_sampled_cells():
    """The equilibrium-shifted BF16 form (the pair kernel with its E
    staging, at the bench's launch configuration): a seeded state of cell
    energies E ~ U(0.5, 1.5) (FP32) and stored deviations d_i ~ U(-0.5, 0.5)
    (BF16), so I_i = w_i (d_i + E).  Bounds, element by element: the stored
    new deviation is one stochastic rounding of (I_i' - w_i E') / w_i to BF16,
    within one unit in its last place, so |I_i - ref_i| <= 2^-7 |ref_i -
    w_i E_ref| plus FP32 slack (1e-5 of the cell's largest population); E'
    and F' are formed in FP32 before any rounding: 1e-5, as for FP32 storage."""
    torch = gh.torch_mod()
    L = gh.lib()
    st = L.LBRT_BF16_SHIFTED
    prob = wl.beams(n=256, alloc_state=False)
    print(prob.name, prob.shape, prob.ndir, "bf16 shifted", flush=True)
    w = np.asarray(prob.weights, dtype=np.float64)
    scale = np.abs(w)
    g = torch.Generator().manual_seed(2028)
    Ecell = (0.5 + torch.rand(prob.shape, generator=g)).numpy().astype(np.float32)
    q16 = torch.empty((prob.ndir,) + prob.shape, dtype=torch.bfloat16)
    for i in range(prob.ndir):
        q16[i] = (torch.rand(prob.shape, generator=g) - 0.5).to(torch.bfloat16)
    nbytes = L.state_bytes(st, prob.ndir, prob.ncell)
    state = torch.zeros(nbytes, dtype=torch.uint8, device="cuda")
    state[:2 * prob.ndir * prob.ncell] = q16.reshape(-1).view(torch.uint8).cuda()
    off = L.state_e_offset(st, prob.ndir, prob.ncell)
    state[off:off + 4 * prob.ncell] = torch.from_numpy(Ecell.reshape(-1)).view(torch.uint8).cuda()
    ctx, out, E, F = _gpu_step(prob, state, st)
    del state
    cells = _sample_cells(prob, np.random.default_rng(8), extra=_beam_cells(prob))
    I_gpu, E_gpu, F_gpu = _gather(ctx, prob, out, E, F, cells, st)
    del out, E, F
    ctx.close()
    torch.cuda.empty_cache()
    ref = orc.step_cells(_Shifted(q16, Ecell, w, scale), prob, cells)
    E_ref = ref.sum(axis=0)
    F_ref = prob.dirs.T @ ref
    dev = np.abs(ref - w[:, None] * E_ref[None, :])
    bound = 2.0 ** -7 * dev + 1e-5 * np.max(np.abs(ref), axis=0)[None, :]
    excess = np.max(np.abs(I_gpu - ref) / bound)
    err_E = np.max(np.abs(E_gpu - E_ref) / np.abs(E_ref))
    err_F = np.max(np.abs(F_gpu - F_ref)) / np.max(np.abs(F_ref))
    print(f"{len(cells)} cells: max |I - ref| / bound {excess:.3f}, max rel err E {err_E:.2e}, "
          f"F {err_F:.2e}", flush=True)
    assert excess <= 1.0
    assert err_E < 1e-5 and err_F < 1e-5


def test_moving_192_fp32_sampled_cells():
    torch = gh.torch_mod()
    L = gh.lib()
    prob = wl.moving(n=192, alloc_state=False)
    print(prob.name, prob.shape, prob.ndir, flush=True)
    I0 = _random_state(prob, 2028)
    state = torch.from_numpy(I0).reshape(-1).cuda()
    ctx, out, E, F = _gpu_step(prob, state, L.LBRT_FP32)
    del state
    cells = _sample_cells(prob, np.random.default_rng(7),
                          extra=[[z, 96 + dy, x] for z in (5, 100) for dy in (-1, 0, 1)
                                 for x in (0, 64, 191)])
    I_gpu, E_gpu, F_gpu = _gather(ctx, prob, out, E, F, cells, L.LBRT_FP32)
    del out, E, F
    ctx.close()
    torch.cuda.empty_cache()
    ref = orc.step_cells(I0, prob, cells)
    _check(prob, I_gpu, E_gpu, F_gpu, ref, 1e-5, 1e-5)


def test_moving_192_adjoint_matches_finite_difference():
    """d L / d(kappa_a, kappa_s, eta) along a seeded positive direction, from
    the adjoint, against (L(+h) - L(-h)) / 2h of the forward runs (16 steps,
    checkpoints every 8)."""
    torch = gh.torch_mod()
    L = gh.lib()
    from paper_2007_05718_amd import autodiff
    prob = wl.moving(n=192, steps=16, alloc_state=False)
    print(prob.name, prob.shape, prob.ndir, "adjoint", flush=True)
    ctx = L.lbrt_init(L.Desc.from_problem(prob, storage=L.LBRT_FP32))
    ka, ks, eta, vel, _ = gh.upload_fields(prob)
    I0 = torch.zeros(prob.ndir * prob.ncell, device="cuda")
    Lv, ga, gs, ge = autodiff.detected_energy_gradient(ctx, I0, ka, ks, eta, prob.steps, face=1,
                                                       checkpoint_every=8, vel=vel)
    g = torch.Generator(device="cuda").manual_seed(11)
    da = ka * torch.empty_like(ka).uniform_(0.5, 1.5, generator=g)
    ds = ks * torch.empty_like(ks).uniform_(0.5, 1.5, generator=g)
    de = eta * torch.empty_like(eta).uniform_(0.5, 1.5, generator=g)
    ad = float((ga.double() * da.double()).sum() + (gs.double() * ds.double()).sum()
               + (ge.double() * de.double()).sum())
    h = 1e-3
    with torch.no_grad():
        Lp = float(autodiff.detected_energy(ctx, I0, ka + h * da, ks + h * ds, eta + h * de,
                                            prob.steps, face=1, checkpoint_every=8, vel=vel))
        Lm = float(autodiff.detected_energy(ctx, I0, ka - h * da, ks - h * ds, eta - h * de,
                                            prob.steps, face=1, checkpoint_every=8, vel=vel))
    fd = (Lp - Lm) / (2 * h)
    print(f"L {float(Lv):.6e} adjoint {ad:.6e} fd {fd:.6e} rel {abs(fd - ad) / abs(ad):.2e}",
          flush=True)
    assert abs(fd - ad) < 1e-2 * abs(ad)
    ctx.close()


def test_moving_192_fp64_adjoint_per_cell_finite_differences():
    """The moving-fluid workload at its full size (192^3 x 146, 64 steps,
    checkpoints every 8) in FP64 storage: d L / d kappa_a (eta = kappa_a, B = 1)
    from the adjoint at 20 random cells inside the detector's light cone
    (where the gradient is not 0), against central differences of two
    forward runs per cell, (L(k + h) - L(k - h)) / (k_+ - k_-), h = 1e-3 k
    (the perturbed values rounded to the float32 inputs).  Bound:
    2e-6 |g| for the O(h^2) truncation, plus the rounding of the difference
    of two FP64 values of L (about 5e5, each a fixed-order sum of ~10^7 FP64
    terms): 8e-15 |L| / (k_+ - k_-), a few units in the last place of L.
    The FP32 adjoint's gradient against the FP64 one: 1e-3 relative L2."""
    torch = gh.torch_mod()
    L = gh.lib()
    from paper_2007_05718_amd import autodiff
    prob = wl.moving(n=192, steps=64, alloc_state=False)
    print(prob.name, prob.shape, prob.ndir, "FP64 adjoint + per-cell FD", flush=True)
    ka, ks, _, vel, _ = gh.upload_fields(prob)
    grads = {}
    for st in (L.LBRT_FP64, L.LBRT_FP32):
        ctx = L.lbrt_init(L.Desc.from_problem(prob, storage=st))
        dt = torch.float64 if st == L.LBRT_FP64 else torch.float32
        I0 = torch.zeros(prob.ndir * prob.ncell, dtype=dt, device="cuda")
        Lv, ga, gs, ge = autodiff.detected_energy_gradient(ctx, I0, ka, ks, ka * 1.0, prob.steps,
                                                           face=1, checkpoint_every=8, vel=vel)
        grads[st] = (float(Lv), (ga + ge).double())
        del I0
        if st == L.LBRT_FP64:
            ctx64 = ctx
        else:
            ctx.close()
        torch.cuda.empty_cache()
    L64, g64 = grads[L.LBRT_FP64]
    e32 = float((grads[L.LBRT_FP32][1] - g64).norm() / g64.norm())
    print(f"L fp64 {L64:.12e} fp32 {grads[L.LBRT_FP32][0]:.12e}; fp32 grad rel L2 {e32:.2e}",
          flush=True)
    assert e32 < 1e-3
    gmax = float(g64.abs().max())
    live = torch.nonzero(g64.abs() > 1e-3 * gmax).flatten().cpu().numpy()
    rng = np.random.default_rng(2020)
    cells = rng.choice(live, 20, replace=False)
    I0 = torch.zeros(prob.ndir * prob.ncell, dtype=torch.float64, device="cuda")
    worst = 0.0
    with torch.no_grad():
        for c in cells:
            k0 = float(ka[c])
            kp, km = np.float32(k0 * (1 + 1e-3)), np.float32(k0 * (1 - 1e-3))
            Ls = []
            for kv in (kp, km):
                kk = ka.clone()
                kk[c] = float(kv)
                Ls.append(float(autodiff.detected_energy(ctx64, I0, kk, ks, kk * 1.0, prob.steps,
                                                         face=1, checkpoint_every=prob.steps,
                                                         vel=vel)))
            dk = float(kp) - float(km)
            fd = (Ls[0] - Ls[1]) / dk
            ad = float(g64[c])
            bound = 2e-6 * abs(ad) + 8e-15 * abs(L64) / dk
            worst = max(worst, abs(fd - ad) / bound)
            print(f"cell {c}: adjoint {ad:.10e} fd {fd:.10e} rel {abs(fd - ad) / abs(ad):.2e} "
                  f"err/bound {abs(fd - ad) / bound:.2f}", flush=True)
    ctx64.close()
    assert worst < 1.0


def test_largest_grid_exact_shift():
    """The largest grid the library takes (1023 x 1024 x 2048 cells, just
    under 2^31; 12.9e9 populations per state with the six axis directions),
    periodic faces, dt = dx and no medium: one step moves every population
    by exactly one cell along its axis (Sec. 4.1.1), bit for bit, and the
    FP64 energy sum is the input's.  The direction planes then lie up to
    48 GB apart, past every 32-bit element or byte offset."""
    torch = gh.torch_mod()
    L = gh.lib()
    nz, ny, nx = 1023, 1024, 2048
    dirs, w = wl.lebedev(6)
    desc = L.Desc(nx=nx, ny=ny, nz=nz, dt=1.0, dirs=dirs, weights=w,
                  bc=(L.LBRT_BC_PERIODIC,) * 6)
    n = desc.ncell
    assert n < 2 ** 31 and 6 * n > 2 ** 33
    print(f"largest grid {nz}x{ny}x{nx} x 6, {n} cells", flush=True)
    ctx = L.lbrt_init(desc)
    g = torch.Generator(device="cuda").manual_seed(71)
    Ia = torch.rand(6 * n, generator=g, device="cuda")
    Ib = torch.empty_like(Ia)
    zero = torch.zeros(n, device="cuda")
    diag = torch.zeros(L.LBRT_DIAG_LEN, dtype=torch.float64, device="cuda")
    L.lbrt_step(ctx, Ia, Ib, zero, zero, zero, nsteps=1, diag=diag)
    torch.cuda.synchronize()
    E0 = 0.0
    for i in range(6):
        a = int(np.argmax(np.abs(dirs[i])))
        src = Ia[i * n:(i + 1) * n].view(nz, ny, nx)
        ref = torch.roll(src, int(np.sign(dirs[i][a])), dims=2 - a)
        assert torch.equal(Ib[i * n:(i + 1) * n].view(nz, ny, nx), ref), i
        del ref
        E0 += float(torch.sum(src, dtype=torch.float64))
    d = diag.cpu().numpy()
    print(f"sum E {d[0]:.12e} vs input {E0:.12e}", flush=True)
    # per-cell E is an FP32 sum of six values, the total an FP64 sum
    assert abs(d[0] - E0) < 1e-6 * E0
    assert np.all(d[1:8] == 0.0)
    ctx.close()
    # hand the ~120 GB back to the device for the tests that follow
    del Ia, Ib, zero, src
    torch.cuda.empty_cache()
