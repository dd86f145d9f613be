"""Pins of the oracle's nonlinear rotation-invariant bond-based force
(Sec. 3.2, Eq. 19-20) against facts that do not come from it: hand values,
invariance under finite rigid rotations, the small-displacement limit (the
linearized model, Eq. 17-18), the gradient of the bond energy it derives
from, the balance of forces and torques, and the paper's convolution form
(Eq. 21-26, sign-consistent reading) evaluated with numpy FFTs on a periodic
grid.  CPU only."""
import os

import numpy as np
import pytest

from paper_2105_06055_amd import workloads as wl

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    out = {}
    for line in open(os.path.join(GOLD, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            k, v = line.split()[:2]
            out[k] = float(v)
    return out


def _coords(shape, dx):
    """Node coordinates, component-major like the fields ((y, x) or (z, y, x))."""
    grids = np.meshgrid(*[np.arange(n) * dx for n in shape], indexing="ij")
    return np.stack(grids[::-1])   # x first


def test_two_node_hand_values(orc):
    gold = _gold("two_node.txt")
    g = orc.geom((1, 2), [1.0, 1.0], 1.5)
    phi = np.ones((1, 2))
    u = np.zeros((2, 1, 2))
    u[0, 0, 1] = 0.5
    L = orc.nbb_force(g, 2.0, phi, u)
    assert L[0, 0, 0] == pytest.approx(gold["NBB_stretch_L0x"], rel=1e-15)
    assert L[0, 0, 1] == pytest.approx(gold["NBB_stretch_L1x"], rel=1e-15)
    assert abs(L[1]).max() == 0.0
    u[0, 0, 1] = -0.5
    L = orc.nbb_force(g, 2.0, phi, u)
    assert L[0, 0, 0] == pytest.approx(gold["NBB_compress_L0x"], rel=1e-15)
    assert L[0, 0, 1] == pytest.approx(gold["NBB_compress_L1x"], rel=1e-15)


def _rotation(dim, seed):
    rng = np.random.default_rng(seed)
    if dim == 2:
        t = 0.4
        return np.array([[np.cos(t), -np.sin(t)], [np.sin(t), np.cos(t)]])
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    return q if np.linalg.det(q) > 0 else -q


@pytest.mark.parametrize("shape,m", [((13, 17), 3), ((7, 9, 8), 2)])
def test_finite_rigid_rotation_gives_zero_force(orc, shape, m):
    """Every bond keeps its length under u = (R - I) x + c: s = 0 and f = 0
    on every bond, at the boundary too (the linearized model fails this)."""
    dim, dx = len(shape), 1e-3
    g = orc.geom(shape, dx, m * dx)
    chi = wl.random_mask(shape, 3).astype(float)
    X = _coords(shape, dx)
    R = _rotation(dim, 4)
    u = np.einsum("ij,j...->i...", R - np.eye(dim), X) + 0.37 * dx
    alpha = orc.bb_alpha(dim, 70e9, m * dx)
    L = orc.nbb_force(g, alpha, chi, u)
    # the linearized model does not vanish for the same field; its force is
    # the scale of the rounding left in the nonlinear one
    Lb = orc.bb_force(g, alpha, chi, u)
    assert np.abs(L).max() <= 1e-12 * np.abs(Lb).max()


@pytest.mark.parametrize("shape,m", [((12, 15), 3), ((6, 7, 8), 2)])
def test_small_displacement_limit_is_the_linear_model(orc, shape, m):
    """L_nl(eps u)/eps -> L_lin(u) with an O(eps) remainder (Eq. 19 vs 17)."""
    dim, dx = len(shape), 1e-3
    g = orc.geom(shape, dx, m * dx)
    chi = wl.random_mask(shape, 5).astype(float)
    u = wl.random_field((dim,) + shape, 6, dx)
    alpha = orc.bb_alpha(dim, 70e9, m * dx)
    Lb = orc.bb_force(g, alpha, chi, u)
    errs = []
    for eps in (1e-4, 5e-5):
        Ln = orc.nbb_force(g, alpha, chi, eps * u) / eps
        errs.append(np.linalg.norm(Ln - Lb) / np.linalg.norm(Lb))
    assert errs[0] < 1e-3
    assert errs[1] == pytest.approx(errs[0] / 2, rel=0.05)   # first order in eps


def _bond_energy(g_shape, dx, delta, alpha, phi, u, S):
    """Total energy 1/2 sum_x sum_o phi phi' w dV^2 with the bond energy
    w = alpha omega r^2 s^2 (2 + s)^2 / 8, whose eta-gradient is Eq. 19's f
    (numpy, non-periodic, written independently of the oracle)."""
    dim = len(g_shape)
    dV = dx ** dim
    pad = [(0, 0)] + [(5, 5)] * dim
    up = np.pad(u, pad)
    pp = np.pad(phi, pad[1:])
    core = tuple(slice(5, 5 + n) for n in g_shape)
    E = 0.0
    for o in S:
        o = o[:dim][::-1]   # (z, y, x) order of the arrays
        sh = tuple(slice(5 + oo, 5 + oo + n) for oo, n in zip(o, g_shape))
        xi = np.array(o[::-1], dtype=float) * dx          # x first
        eta = up[(slice(None),) + sh] - up[(slice(None),) + core]
        y = xi.reshape((dim,) + (1,) * dim) + eta
        r = np.linalg.norm(xi)
        s = (np.sqrt((y * y).sum(0)) - r) / r
        w = alpha / r * r * r * s * s * (2 + s) ** 2 / 8
        E += 0.5 * (pp[core] * pp[sh] * w).sum() * dV * dV
    return E


def test_force_is_minus_the_energy_gradient(orc):
    shape, dx, m = (9, 11), 1e-3, 3
    g = orc.geom(shape, dx, m * dx)
    S = orc.stencil(g)
    chi = wl.random_mask(shape, 7).astype(float)
    u = wl.random_field((2,) + shape, 8, 0.05 * dx)
    alpha = orc.bb_alpha(2, 70e9, m * dx)
    L = orc.nbb_force(g, alpha, chi, u)
    rng = np.random.default_rng(9)
    for _ in range(3):
        du = rng.normal(size=u.shape) * 0.01 * dx
        h = 1e-3
        Ep = _bond_energy(shape, dx, m * dx, alpha, chi, u + h * du, S)
        Em = _bond_energy(shape, dx, m * dx, alpha, chi, u - h * du, S)
        fd = (Ep - Em) / (2 * h)
        an = -(L * du).sum() * dx ** 2
        assert fd == pytest.approx(an, rel=1e-7)


@pytest.mark.parametrize("shape,m", [((10, 13), 3), ((6, 7, 5), 2)])
def test_force_and_torque_balance(orc, shape, m):
    """Pairwise bond forces are equal and opposite and lie along the deformed
    bond: zero net force and zero net torque about the origin of the
    deformed configuration."""
    dim, dx = len(shape), 1e-3
    g = orc.geom(shape, dx, m * dx)
    chi = wl.random_mask(shape, 10).astype(float)
    u = wl.random_field((dim,) + shape, 11, 0.2 * dx)
    alpha = orc.bb_alpha(dim, 70e9, m * dx)
    L = orc.nbb_force(g, alpha, chi, u)
    ref = np.abs(L).sum()
    assert np.abs(L.reshape(dim, -1).sum(1)).max() <= 1e-13 * ref
    y = _coords(shape, dx) + u
    if dim == 2:
        tq = [(y[0] * L[1] - y[1] * L[0]).sum()]
    else:
        tq = [(y[a] * L[b] - y[b] * L[a]).sum() for a, b in ((1, 2), (2, 0), (0, 1))]
    assert np.abs(tq).max() <= 1e-13 * ref * np.abs(y).max()


def test_convolution_form_matches(orc):
    """The convolution form (Eq. 21-26, derived with xi = x' - x; masks as
    bond weights) on a periodic grid, with the correlations evaluated by
    numpy FFTs, equals the oracle's bond-by-bond Eq. 19."""
    shape, dx, m = (16, 20), 1e-3, 3
    g = orc.geom(shape, dx, m * dx, periodic=True)
    S = orc.stencil(g)
    chi = wl.random_mask(shape, 12).astype(float)
    u = wl.random_field((2,) + shape, 13, 0.3 * dx)
    alpha = orc.bb_alpha(2, 70e9, m * dx)
    L = orc.nbb_force(g, alpha, chi, u)
    # kernels on the periodic grid: C_ij, a_i, c with c = alpha omega / r^2 dV
    ny, nx = shape
    Kc = np.zeros(shape)
    Ka = np.zeros((2,) + shape)
    KC = np.zeros((2, 2) + shape)
    for o in S:
        ox, oy = int(o[0]), int(o[1])
        xi = np.array([ox, oy], float) * dx
        r = np.linalg.norm(xi)
        cc = alpha / r / r ** 2 * dx * dx
        Kc[oy % ny, ox % nx] += cc
        Ka[:, oy % ny, ox % nx] += cc * xi
        KC[:, :, oy % ny, ox % nx] += cc * np.outer(xi, xi)

    def corr(K, f):   # sum_o K(o) f(x + o)
        return np.real(np.fft.ifft2(np.conj(np.fft.fft2(K)) * np.fft.fft2(f)))
    cu = chi * u
    u2 = (u * u).sum(0)
    P = np.array([[corr(KC[i, j], chi) for j in range(2)] for i in range(2)])
    q = np.array([corr(Ka[i], chi) for i in range(2)])
    p = corr(Kc, chi)
    A = np.array([[corr(Ka[i], cu[j]) for j in range(2)] for i in range(2)])
    B = np.array([[corr(Kc, chi * u[i] * u[j]) for j in range(2)] for i in range(2)])
    b = corr(Kc, chi * u2)
    cvec = np.array([corr(Kc, cu[j]) for j in range(2)])
    Lc = np.zeros_like(u)
    for i in range(2):
        t = sum(corr(KC[i, j], cu[j]) for j in range(2))
        t = t + 0.5 * corr(Ka[i], chi * u2) + sum(corr(Ka[j], chi * u[j] * u[i]) for j in range(2))
        t = t + 0.5 * corr(Kc, chi * u2 * u[i])
        for j in range(2):
            t = t - P[i, j] * u[j] - A[i, j] * u[j] - A[j, j] * u[i] - A[j, i] * u[j]
            t = t + q[j] * u[j] * u[i] - B[i, j] * u[j] + cvec[j] * u[j] * u[i]
        t = t + 0.5 * q[i] * u2 - 0.5 * b * u[i] + 0.5 * cvec[i] * u2 - 0.5 * p * u2 * u[i]
        Lc[i] = chi * t
    assert np.linalg.norm(Lc - L) <= 1e-11 * np.linalg.norm(L)
