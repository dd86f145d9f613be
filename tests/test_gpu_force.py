"""pd_force parity against the FP64 direct-summation oracle, element by
element over the whole field.

Bars (tests/parity.py): FP64 max |L - L_oracle| / max |L_oracle| <= 1e-12;
FP32 max |L32 - L_oracle| / (lambda_max max |u|) <= 1e-5 (lambda_max from
the plan's stability bound) and max |L32 - L_oracle| / max |L_oracle| <= 1e-4.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2105_06055_amd import workloads as wl

import parity

pytestmark = pytest.mark.gpu


def _plan(w, dtype, **kw):
    from paper_2105_06055_amd import binding
    return binding.Plan.from_workload(w, dtype=dtype, **kw)


def _dev(a, dtype):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _check(L, Lo, u, plan, rho, dtype, tag=""):
    return parity.check_force(L, Lo, u, plan, rho, dtype == torch.float64, tag)


def _same(La, Lb, Lo, dtype, what):
    """Two GPU paths on the same plan agree element-wise to rounding."""
    tol = 1e-13 if dtype == torch.float64 else 1e-5
    e = float(np.max(np.abs(La - Lb)) / np.max(np.abs(Lo)))
    assert e <= tol, (what, e)


DT = [torch.float64, torch.float32]


@pytest.mark.parametrize("dtype", DT)
def test_bb2d_plate_full_size(orc, dtype):
    """The 64x64 plate in a 128x128 box (the paper-style 2D plate, full size)."""
    w = wl.plate_2d(seed=1)
    plan = _plan(w, dtype)
    L = plan.force(_dev(w.u0, dtype)).cpu().numpy()
    g = orc.geom(w.body, w.dx, w.delta)
    Lo = orc.bb_force(g, orc.bb_alpha(2, w.E, w.delta), w.chiB.astype(float), w.u0)
    _check(L, Lo, w.u0, plan, w.rho, dtype)
    plan.close()


@pytest.mark.parametrize("dtype", DT)
@pytest.mark.parametrize("body,fft,m", [((37, 45), (64, 64), 3), ((50, 19), (64, 32), 4),
                                        ((100, 40), (128, 64), 4), ((9, 13), (16, 32), 2)])
def test_bb2d_masked_ragged(orc, dtype, body, fft, m):
    dx = 1e-3
    w = wl.Workload(name="t", dim=2, body=body, fft=fft, dx=dx, delta=m * dx, model="bb", E=72e9, nu=1 / 3)
    w.chiB = wl.random_mask(body, 3)
    w.chiO = np.stack([w.chiB] * 2)
    u = wl.random_field((2,) + body, 4, 1e-6)
    plan = _plan(w, dtype)
    L = plan.force(_dev(u, dtype)).cpu().numpy()
    g = orc.geom(body, dx, w.delta)
    Lo = orc.bb_force(g, orc.bb_alpha(2, w.E, w.delta), w.chiB.astype(float), u)
    _check(L, Lo, u, plan, w.rho, dtype)
    plan.close()


@pytest.mark.parametrize("dtype", DT)
@pytest.mark.parametrize("body,fft,m", [((20, 23, 17), (32, 32, 32), 2), ((12, 30, 21), (16, 64, 32), 3)])
def test_bb3d_masked(orc, dtype, body, fft, m):
    dx = 1e-3
    w = wl.Workload(name="t", dim=3, body=body, fft=fft, dx=dx, delta=m * dx, model="bb", E=70e9, nu=0.25)
    w.chiB = wl.random_mask(body, 7)
    w.chiO = np.stack([w.chiB] * 3)
    u = wl.random_field((3,) + body, 8, 1e-6)
    plan = _plan(w, dtype)
    L = plan.force(_dev(u, dtype)).cpu().numpy()
    g = orc.geom(body, dx, w.delta)
    Lo = orc.bb_force(g, orc.bb_alpha(3, w.E, w.delta), w.chiB.astype(float), u)
    _check(L, Lo, u, plan, w.rho, dtype)
    plan.close()


@pytest.mark.parametrize("dtype", DT)
@pytest.mark.parametrize("nu", [0.25, 0.4])
@pytest.mark.parametrize("nb,nfft", [(24, 32), (32, 64)])
def test_lps3d_cube_void(orc, dtype, nu, nb, nfft):
    """Cube with a spherical void (the static-config geometry, scaled)."""
    w = wl.cube_void_static(seed=2, nb=nb, nfft=nfft, E=200e9, nu=nu)
    u = wl.random_field((3,) + w.body, 5, 1e-6)
    plan = _plan(w, dtype)
    L = plan.force(_dev(u, dtype)).cpu().numpy()
    g = orc.geom(w.body, w.dx, w.delta)
    Lo, th = orc.lps_force(g, w.E, nu, w.chiB.astype(float), u)
    _check(L, Lo, u, plan, 2440.0, dtype)
    plan.close()


@pytest.mark.parametrize("dtype", DT)
def test_lps3d_ragged_voids(orc, dtype):
    body, dx = (20, 17, 23), 1e-3
    chi = wl.random_mask(body, 19)
    u = wl.random_field((3,) + body, 6, 1e-6)
    from paper_2105_06055_amd import binding
    plan = binding.Plan((32, 32, 32), body, dx, 3 * dx, model="lps", E=70e9, nu=0.3,
                        chiB=chi, dtype=dtype)
    L = plan.force(_dev(u, dtype)).cpu().numpy()
    g = orc.geom(body, dx, 3 * dx)
    Lo, _ = orc.lps_force(g, 70e9, 0.3, chi.astype(float), u)
    _check(L, Lo, u, plan, 2700.0, dtype)
    plan.close()


# Lines of 512 points along the last axis (numpy axis 0) with a horizon of 3
# spacings: the default path (3D: direct (y, z) correlation; 2D: direct line
# correlation), the y transform with the direct z line correlation, the
# specialised 512-point transform kernel and the runtime-length transform
# kernel, each against the
# oracle (ragged body up to the largest body the padding allows) and against
# each other on the same plan.
@pytest.mark.parametrize("dtype", DT)
@pytest.mark.parametrize("model,body", [("lps", (300, 11, 13)), ("lps", (509, 9, 12)), ("bb", (300, 11, 13)),
                                        ("bb", (509, 9, 12)), ("bb", (300, 41)), ("bb", (509, 17))])
def test_specialised_lastaxis_512(orc, dtype, model, body):
    from paper_2105_06055_amd import binding
    dx, D = 1e-3, len(body)
    chi = wl.random_mask(body, 23)
    u = wl.random_field((D,) + body, 24, 1e-6)
    fft = (512, 16, 16) if D == 3 else (512, 64)
    plan = binding.Plan(fft, body, dx, 3 * dx, model=model, E=70e9, nu=0.3 if D == 3 else 1 / 3,
                        chiB=chi, dtype=dtype)
    L = plan.force(_dev(u, dtype)).cpu().numpy()
    g = orc.geom(body, dx, 3 * dx)
    if model == "lps":
        Lo, _ = orc.lps_force(g, 70e9, 0.3, chi.astype(float), u)
    else:
        Lo = orc.bb_force(g, orc.bb_alpha(D, 70e9, 3 * dx), chi.astype(float), u)
    _check(L, Lo, u, plan, 2700.0, dtype)
    for mode in ("fft", "fft_generic", "yfft"):
        plan.set_lastaxis(mode)
        Lg = plan.force(_dev(u, dtype)).cpu().numpy()
        _check(Lg, Lo, u, plan, 2700.0, dtype)
        _same(L, Lg, Lo, dtype, mode)
    plan.close()


@pytest.mark.parametrize("dtype", DT)
def test_bb2d_integrity_weights_and_energy(orc, dtype):
    body, fft, dx, m = (40, 50), (64, 64), 1e-3, 3
    w = wl.Workload(name="t", dim=2, body=body, fft=fft, dx=dx, delta=m * dx, model="bb", E=72e9, nu=1 / 3,
                    G0=3.8)
    w.chiB = wl.random_mask(body, 11)
    w.chiO = np.stack([w.chiB] * 2)
    rng = np.random.default_rng(12)
    lam = (rng.random(body) > 0.1).astype(np.uint8)
    w.lam0 = lam
    u = wl.random_field((2,) + body, 13, 1e-6)
    plan = _plan(w, dtype, weight="integrity")
    L, W = plan.force(_dev(u, dtype), weight=_dev(lam, torch.uint8), energy=True)
    L, W = L.cpu().numpy(), W.cpu().numpy()
    g = orc.geom(body, dx, w.delta)
    alpha = orc.bb_alpha(2, w.E, w.delta)
    phi = (w.chiB * lam).astype(float)
    Lo = orc.bb_force(g, alpha, phi, u)
    Wo = orc.bb_energy(g, alpha, phi, u)
    _check(L, Lo, u, plan, w.rho, dtype)
    # W by the convolution form cancels terms of order (chi u)^2 against a
    # result of order (u' - u)^2 (reading A18): its error is measured on the
    # scale of those terms, lambda_max max|u|^2, and reported
    lam = parity.lam_max(plan, w.rho)
    eW = float(np.max(np.abs(W - Wo)) / (lam * np.max(np.abs(u)) ** 2))
    relW = parity.rel_max(W, Wo)
    print(f"energy density W: max err / (lambda_max max|u|^2) {eW:.2e}, rel_max {relW:.2e}")
    if dtype == torch.float64:
        assert relW <= 1e-11, relW
    else:
        assert eW <= 1e-5, eW
        assert relW <= 1e-2, relW
    plan.close()


@pytest.mark.parametrize("dtype", DT)
def test_bb2d_scale_weights(orc, dtype):
    body, fft, dx, m = (33, 47), (64, 64), 1e-3, 3
    w = wl.Workload(name="t", dim=2, body=body, fft=fft, dx=dx, delta=m * dx, model="bb", E=72e9, nu=1 / 3)
    w.chiB = wl.random_mask(body, 14)
    w.chiO = np.stack([w.chiB] * 2)
    s = np.sqrt(1 + 0.2 * wl.gaussian_random_field(body, 3.0, 15))
    u = wl.random_field((2,) + body, 16, 1e-6)
    plan = _plan(w, dtype, weight="scale")
    L = plan.force(_dev(u, dtype), weight=_dev(s, dtype)).cpu().numpy()
    g = orc.geom(body, dx, w.delta)
    Lo = orc.bb_force(g, orc.bb_alpha(2, w.E, w.delta), w.chiB * s, u)
    _check(L, Lo, u, plan, w.rho, dtype)
    plan.close()


@pytest.mark.parametrize("dtype", DT)
def test_damage_index_bit_exact(orc, dtype):
    w = wl.notched_plate_fracture(nx=100, ny=40, fft=(64, 128), steps=0)
    rng = np.random.default_rng(17)
    lam = w.lam0 * (rng.random(w.body) > 0.05).astype(np.uint8)
    plan = _plan(w, dtype, weight="integrity")
    d = plan.damage_index(_dev(lam, torch.uint8)).cpu().numpy()
    g = orc.geom(w.body, w.dx, w.delta)
    do, _ = orc.damage_index(g, w.chiB, lam)
    if dtype == torch.float32:
        do = do.astype(np.float32)
    assert np.array_equal(d, do)
    plan.close()


def test_plan_validation_errors():
    from paper_2105_06055_amd import binding
    # padding smaller than the horizon: a bond would wrap around the box
    with pytest.raises(binding.PDError) as e:
        binding.Plan((64, 64), (62, 40), 1e-3, 3e-3)
    assert e.value.status == binding.PD_EINVAL
    # non power-of-two grid
    with pytest.raises(binding.PDError) as e:
        binding.Plan((60, 64), (40, 40), 1e-3, 3e-3)
    assert e.value.status == binding.PD_EUNSUPPORTED
    # LPS in 2D is not provided
    with pytest.raises(binding.PDError) as e:
        binding.Plan((64, 64), (40, 40), 1e-3, 3e-3, model="lps")
    assert e.value.status == binding.PD_EUNSUPPORTED


# The direct (y, z) pass (3D default): bodies spanning two y tiles (b2 > 256)
# and several z chunks with a ragged last one, a narrow body (128-row
# tiles), horizons of 2 and 3 spacings, LPS and bond-based, against the
# oracle and against the y transform path on the same plan.  A horizon of
# 2.5 spacings has a (y, z) footprint beyond the disc of radius 2 and takes
# the y transform path.
@pytest.mark.parametrize("dtype", DT)
@pytest.mark.parametrize("model,body,fft,r", [("lps", (12, 300, 40), (16, 512, 64), 3.0),
                                              ("bb", (12, 300, 40), (16, 512, 64), 2.0),
                                              ("lps", (20, 100, 30), (32, 128, 64), 2.0),
                                              ("bb", (20, 100, 30), (32, 128, 64), 3.0),
                                              ("lps", (14, 37, 29), (32, 64, 64), 2.5)])
def test_yz_direct_tiles(orc, dtype, model, body, fft, r):
    from paper_2105_06055_amd import binding
    dx = 1e-3
    chi = wl.random_mask(body, 31)
    u = wl.random_field((3,) + body, 32, 1e-6)
    plan = binding.Plan(fft, body, dx, r * dx, model=model, E=70e9, nu=0.3, chiB=chi, dtype=dtype)
    L = plan.force(_dev(u, dtype)).cpu().numpy()
    g = orc.geom(body, dx, r * dx)
    if model == "lps":
        Lo, _ = orc.lps_force(g, 70e9, 0.3, chi.astype(float), u)
    else:
        Lo = orc.bb_force(g, orc.bb_alpha(3, 70e9, r * dx), chi.astype(float), u)
    _check(L, Lo, u, plan, 2700.0, dtype)
    plan.set_lastaxis("yfft")
    Ly = plan.force(_dev(u, dtype)).cpu().numpy()
    _check(Ly, Lo, u, plan, 2700.0, dtype)
    _same(L, Ly, Lo, dtype, "yfft")
    plan.close()


# The second influence function, omega = 1 (the paper's runs use 1/r): the
# bond-based micromodulus, the LPS weighted volume and every kernel sample
# change with it.
@pytest.mark.parametrize("dtype", DT)
@pytest.mark.parametrize("model,body,fft,m", [("bb", (37, 45), (64, 64), 3), ("bb", (20, 23, 17), (32, 32, 32), 2),
                                              ("lps", (20, 17, 23), (32, 32, 32), 3)])
def test_influence_one(orc, dtype, model, body, fft, m):
    from paper_2105_06055_amd import binding
    dx, D = 1e-3, len(body)
    chi = wl.random_mask(body, 61)
    u = wl.random_field((D,) + body, 62, 1e-6)
    nu = 0.3 if model == "lps" else (1 / 3 if D == 2 else 0.25)
    plan = binding.Plan(fft, body, dx, m * dx, model=model, E=70e9, nu=nu, rho=2700.0, chiB=chi, dtype=dtype,
                        influence=1)
    L = plan.force(_dev(u, dtype)).cpu().numpy()
    g = orc.geom(body, dx, m * dx, influence=1)
    if model == "lps":
        Lo, _ = orc.lps_force(g, 70e9, nu, chi.astype(float), u)
        assert plan.info["m0"] == pytest.approx(orc.m0(g), rel=1e-14)
    else:
        alpha = orc.bb_alpha(D, 70e9, m * dx, influence=1)
        assert plan.info["alpha"] == pytest.approx(alpha, rel=1e-14)
        Lo = orc.bb_force(g, alpha, chi.astype(float), u)
    _check(L, Lo, u, plan, 2700.0, dtype, f"omega=1 {model} {body}")
    plan.close()


# Horizons beyond the (y, z) pass's reach (m = 4, 6 spacings): every path
# the plan offers for them (the y transform with the direct z line
# correlation or, beyond 4 spacings, the transform form; transforms along all
# axes), LPS, against the oracle.
@pytest.mark.parametrize("dtype", DT)
@pytest.mark.parametrize("m", [4, 6])
def test_lps3d_long_horizons_all_paths(orc, dtype, m):
    from paper_2105_06055_amd import binding
    dx, body = 1e-3, (20, 21, 23)
    chi = wl.random_mask(body, 63)
    u = wl.random_field((3,) + body, 64, 1e-6)
    plan = binding.Plan((32, 32, 32), body, dx, m * dx, model="lps", E=70e9, nu=0.3, rho=2700.0, chiB=chi,
                        dtype=dtype)
    g = orc.geom(body, dx, m * dx)
    Lo, _ = orc.lps_force(g, 70e9, 0.3, chi.astype(float), u)
    for mode in ("auto", "yfft", "fft", "fft_generic"):
        plan.set_lastaxis(mode)
        L = plan.force(_dev(u, dtype)).cpu().numpy()
        _check(L, Lo, u, plan, 2700.0, dtype, f"LPS m={m} {mode}")
    plan.close()


@pytest.mark.parametrize("dtype", DT)
def test_energy_density_large_displacement(orc, dtype):
    """W with displacements of two grid spacings (a translated, stretched,
    noisy plate with integrity weights): the direct bond sums match the
    oracle to rounding in both precisions; the convolution form (Eq. 102),
    whose terms of order (chi u)^2 cancel down to (u' - u)^2, loses about
    (|u| / |u' - u|)^2 of its accuracy and is kept as a test mode only."""
    from paper_2105_06055_amd import binding
    body, fft, dx, m = (40, 50), (64, 64), 1e-3, 3
    w = wl.Workload(name="t", dim=2, body=body, fft=fft, dx=dx, delta=m * dx, model="bb", E=72e9, nu=1 / 3,
                    G0=3.8)
    w.chiB = wl.random_mask(body, 65)
    w.chiO = np.stack([w.chiB] * 2)
    lam = (np.random.default_rng(66).random(body) > 0.1).astype(np.uint8)
    w.lam0 = lam
    y, x = np.meshgrid((np.arange(body[0]) + 0.5) * dx, (np.arange(body[1]) + 0.5) * dx, indexing="ij")
    u = np.stack([2e-3 + 1e-3 * x, -1.5e-3 + 5e-4 * y]) + wl.random_field((2,) + body, 67, 1e-7)
    # the oracle sees the values the GPU holds
    u = u.astype(np.float32 if dtype == torch.float32 else np.float64).astype(np.float64)
    plan = _plan(w, dtype, weight="integrity")
    g = orc.geom(body, dx, w.delta)
    Wo = orc.bb_energy(g, orc.bb_alpha(2, w.E, w.delta), (w.chiB * lam).astype(float), u)
    res = {}
    for form in ("direct", "convolution"):
        plan.set_energy_form(form)
        _, W = plan.force(_dev(u, dtype), weight=_dev(lam, torch.uint8), energy=True)
        res[form] = parity.rel_max(W.cpu().numpy(), Wo)
    print(f"W with |u| ~ 2 dx, {dtype}: rel_max direct {res['direct']:.2e}, convolution {res['convolution']:.2e}")
    if dtype == torch.float64:
        assert res["direct"] <= 1e-12 and res["convolution"] <= 1e-5, res
    else:
        assert res["direct"] <= 1e-5, res
        assert res["convolution"] > 100 * res["direct"], res
    plan.close()


# Minimum-padding x grids (Sec. 4.2.2 needs only one horizon of padding):
# x lengths n1 = 2 R 2^p with R = 3, 5, 9, through every chain and path the
# plan runs, against the oracle (which does not depend on the grid).
MIXED = [(48, 3), (80, 5), (144, 9), (96, 3)]


@pytest.mark.parametrize("dtype", DT)
@pytest.mark.parametrize("n1,R", MIXED)
def test_mixed_radix_x_bb2d(orc, dtype, n1, R):
    from paper_2105_06055_amd import binding
    dx, m = 1e-3, 3
    body = (37, n1 - m - 1)
    chi = wl.random_mask(body, 71)
    u = wl.random_field((2,) + body, 72, 1e-6)
    plan = binding.Plan((64, n1), body, dx, m * dx, model="bb", E=72e9, nu=1 / 3, chiB=chi, dtype=dtype)
    L = plan.force(_dev(u, dtype)).cpu().numpy()
    g = orc.geom(body, dx, m * dx)
    Lo = orc.bb_force(g, orc.bb_alpha(2, 72e9, m * dx), chi.astype(float), u)
    _check(L, Lo, u, plan, 2440.0, dtype, f"mixed x n1={n1} bb2d")
    plan.close()


@pytest.mark.parametrize("dtype", DT)
@pytest.mark.parametrize("n1,R", MIXED)
def test_mixed_radix_x_lps3d_all_paths(orc, dtype, n1, R):
    from paper_2105_06055_amd import binding
    dx, m = 1e-3, 3
    body = (17, 21, n1 - m - 2)
    chi = wl.random_mask(body, 73)
    u = wl.random_field((3,) + body, 74, 1e-6)
    plan = binding.Plan((32, 32, n1), body, dx, m * dx, model="lps", E=70e9, nu=0.3, rho=2700.0, chiB=chi,
                        dtype=dtype)
    g = orc.geom(body, dx, m * dx)
    Lo, _ = orc.lps_force(g, 70e9, 0.3, chi.astype(float), u)
    for mode in ("auto", "yfft", "fft"):
        plan.set_lastaxis(mode)
        L = plan.force(_dev(u, dtype)).cpu().numpy()
        _check(L, Lo, u, plan, 2700.0, dtype, f"mixed x n1={n1} lps {mode}")
    plan.close()


@pytest.mark.parametrize("dtype", DT)
def test_mixed_radix_x_weighted_energy_2d(orc, dtype):
    """Integrity weights and W (the fracture chain) on an x grid of 80."""
    from paper_2105_06055_amd import binding
    body, fft, dx, m = (40, 75), (64, 80), 1e-3, 3
    w = wl.Workload(name="t", dim=2, body=body, fft=fft, dx=dx, delta=m * dx, model="bb", E=72e9, nu=1 / 3,
                    G0=3.8)
    w.chiB = wl.random_mask(body, 75)
    w.chiO = np.stack([w.chiB] * 2)
    lam = (np.random.default_rng(76).random(body) > 0.1).astype(np.uint8)
    w.lam0 = lam
    u = wl.random_field((2,) + body, 77, 1e-6)
    plan = _plan(w, dtype, weight="integrity")
    L, W = plan.force(_dev(u, dtype), weight=_dev(lam, torch.uint8), energy=True)
    g = orc.geom(body, dx, w.delta)
    alpha = orc.bb_alpha(2, w.E, w.delta)
    phi = (w.chiB * lam).astype(float)
    _check(L.cpu().numpy(), orc.bb_force(g, alpha, phi, u), u, plan, w.rho, dtype, "mixed x weighted")
    assert parity.rel_max(W.cpu().numpy(), orc.bb_energy(g, alpha, phi, u)) <= (1e-12 if dtype == torch.float64
                                                                                 else 1e-5)
    plan.close()
