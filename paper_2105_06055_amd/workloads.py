"""Seeded synthetic inputs shaped like the paper's workloads.

This module holds geometry and random draws only -- none of the method's
arithmetic (no micromoduli, no kernels, no forces).  Both the HIP path and the
FP64 oracle are fed from here, so neither needs the other's code.

Arrays follow the component-major body-box layout used everywhere in the
library: a vector field is ``(dim, [nz,] ny, nx)`` with x fastest; masks are
``uint8``.  Node centres sit at ``(i + 1/2) dx`` inside the body box.

The paper's own workloads (the 3D dog-bone of Sec. 5.1 and the 2D glass plate
of Sec. 5.2) exist only as figures, so these stand in for them with the same
kind of shapes: a box with an interior void and a clamped layer for statics,
a notched plate under edge tractions for fracture, a block with voids for
explicit dynamics.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Tuple

import numpy as np


@dataclass
class Workload:
    """One synthetic problem: grid, material constants and inputs."""
    name: str
    dim: int
    body: Tuple[int, ...]          # body box in (z, y, x) / (y, x) order
    fft: Tuple[int, ...]           # FFT grid, same order
    dx: float
    delta: float
    model: str                     # "bb" or "lps"
    E: float
    nu: float
    rho: float = 2440.0
    G0: float = 0.0                # critical energy release rate (damage) or 0
    dt: float = 1e-8
    steps: int = 1
    chiB: np.ndarray = None        # body mask
    chiO: np.ndarray = None        # per-component unknown mask (dim, ...)
    u0: np.ndarray = None
    v0: np.ndarray = None
    b: np.ndarray = None
    w: np.ndarray = None
    lam0: np.ndarray = None        # initial integrity (damage runs)
    s: np.ndarray = None           # sqrt(c/c0) (heterogeneous micromodulus)
    extra: dict = field(default_factory=dict)

    @property
    def nodes(self) -> int:
        return int(np.prod(self.body))


def _centres(n, dx):
    return (np.arange(n) + 0.5) * dx


def plate_2d(seed=1, nb=64, nfft=128, dx=1e-3, m=3, E=72e9, rho=2440.0, dt=1e-8, steps=100):
    """Square plate, linearized bond-based, i.i.d. N(0, (1e-6 m)^2) initial
    displacement, zero velocity, free edges (64x64 nodes in a 128x128 box)."""
    rng = np.random.default_rng(seed)
    body = (nb, nb)
    chiB = np.ones(body, np.uint8)
    u0 = rng.normal(0.0, 1e-6, size=(2,) + body)
    return Workload(name=f"bb2d_plate_{nb}", dim=2, body=body, fft=(nfft, nfft), dx=dx,
                    delta=m * dx, model="bb", E=E, nu=1.0 / 3.0, rho=rho, dt=dt, steps=steps,
                    chiB=chiB, chiO=np.stack([chiB, chiB]), u0=u0, v0=np.zeros_like(u0),
                    b=np.zeros_like(u0), w=np.zeros_like(u0))


def cube_void_static(seed=2, nb=128, nfft=256, dx=1e-3, m=3, E=200e9, nu=0.25, clamp_layers=None,
                     bmag=1e8):
    """Cube minus a centred spherical void of radius 0.2 L, clamped (u = 0 on
    all components) on a 3-horizon-thick layer at z = 0, loaded by a seeded
    uniform body force U(-1, 1) * 1e8 N/m^3 per component on the unknowns."""
    rng = np.random.default_rng(seed)
    body = (nb, nb, nb)
    L = nb * dx
    c = _centres(nb, dx)
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    r = np.sqrt((x - L / 2) ** 2 + (y - L / 2) ** 2 + (z - L / 2) ** 2)
    chiB = (r > 0.2 * L).astype(np.uint8)
    k = 3 * m if clamp_layers is None else clamp_layers
    omega = chiB.copy()
    omega[:k] = 0
    chiO = np.stack([omega, omega, omega])
    b = rng.uniform(-1.0, 1.0, size=(3,) + body) * bmag * chiO
    return Workload(name=f"lps3d_static_{nb}", dim=3, body=body, fft=(nfft,) * 3, dx=dx,
                    delta=m * dx, model="lps", E=E, nu=nu, chiB=chiB, chiO=chiO,
                    u0=np.zeros((3,) + body), b=b, w=np.zeros((3,) + body))


def notched_plate_fracture(nx=1000, ny=400, fft=(512, 1024), Lx=0.1, Ly=0.04, m=4, E=72e9,
                           rho=2440.0, G0=3.8, sigma=12e6, notch=0.05, dt=1e-8, steps=10000):
    """Glass-like plate with a pre-notch on the mid-line: integrity 0 on a
    one-horizon-thick layer of nodes for x < notch, tractions +-sigma applied
    as body forces sigma/delta on the one-horizon-thick top and bottom
    layers (tension).  Deterministic (no random draws)."""
    dx = Lx / nx
    assert abs(Ly / ny - dx) < 1e-15
    delta = m * dx
    body = (ny, nx)
    chiB = np.ones(body, np.uint8)
    xc = _centres(nx, dx)
    yc = _centres(ny, dx)
    Y, X = np.meshgrid(yc, xc, indexing="ij")
    lam0 = np.ones(body, np.uint8)
    lam0[(X < notch) & (np.abs(Y - Ly / 2) < delta / 2)] = 0
    b = np.zeros((2,) + body)
    top = Y > Ly - delta
    bot = Y < delta
    b[1][top] = sigma / delta
    b[1][bot] = -sigma / delta
    return Workload(name=f"bb2d_fracture_{nx}x{ny}", dim=2, body=body, fft=fft, dx=dx, delta=delta,
                    model="bb", E=E, nu=1.0 / 3.0, rho=rho, G0=G0, dt=dt, steps=steps, chiB=chiB,
                    chiO=np.stack([chiB, chiB]), u0=np.zeros((2,) + body),
                    v0=np.zeros((2,) + body), b=b, w=np.zeros((2,) + body), lam0=lam0,
                    extra={"sigma": sigma})


def gaussian_random_field(shape, corr_nodes, seed):
    """Unit-variance periodic Gaussian random field: white N(0,1) noise
    smoothed by a Gaussian of standard deviation ``corr_nodes`` nodes, then
    rescaled to unit standard deviation and clipped to [-4, 4]."""
    from scipy.ndimage import gaussian_filter
    rng = np.random.default_rng(seed)
    g = gaussian_filter(rng.normal(size=shape), sigma=corr_nodes, mode="wrap")
    g = (g - g.mean()) / g.std()
    return np.clip(g, -4.0, 4.0)


def hetero_plate_adjoint(nb=512, nfft=1024, dx=1e-3, m=3, E=72e9, rho=2440.0, dt=1e-8, steps=200,
                         seeds=(4, 40, 41, 42), ndirs=32):
    """Square plate with a spatially varying micromodulus c = c0 (1 + 0.2 g),
    g a seeded Gaussian random field with correlation length 20 dx; seeded
    initial velocities N(0, 1 m/s), zero initial displacement, a seeded target
    displacement field and seeded unit finite-difference directions."""
    body = (nb, nb)
    g = gaussian_random_field(body, 20.0 * (nb / 512.0) if nb < 512 else 20.0, seeds[0])
    c_rel = 1.0 + 0.2 * g
    rng_v = np.random.default_rng(seeds[1])
    v0 = rng_v.normal(0.0, 1.0, size=(2,) + body)
    rng_t = np.random.default_rng(seeds[2])
    u_target = rng_t.normal(0.0, steps * dt, size=(2,) + body)
    rng_d = np.random.default_rng(seeds[3])
    du = rng_d.normal(size=(ndirs, 2) + body)
    du /= np.sqrt((du ** 2).sum(axis=tuple(range(1, du.ndim)), keepdims=True))
    dc = rng_d.normal(size=(ndirs,) + body)
    dc /= np.sqrt((dc ** 2).sum(axis=tuple(range(1, dc.ndim)), keepdims=True))
    chiB = np.ones(body, np.uint8)
    return Workload(name=f"bb2d_adjoint_{nb}", dim=2, body=body, fft=(nfft, nfft), dx=dx,
                    delta=m * dx, model="bb", E=E, nu=1.0 / 3.0, rho=rho, dt=dt, steps=steps,
                    chiB=chiB, chiO=np.stack([chiB, chiB]), u0=np.zeros((2,) + body), v0=v0,
                    b=np.zeros((2,) + body), w=np.zeros((2,) + body), s=np.sqrt(c_rel),
                    extra={"c_rel": c_rel, "u_target": u_target, "dirs_u": du, "dirs_c": dc})


def block_voids_dynamics(seed=5, vseed=50, nb=256, nfft=512, dx=1e-3, m=3, E=70e9, nu=0.25,
                         rho=2700.0, dt=1e-8, steps=1000, nvoids=8):
    """Cube with a seeded set of axis-aligned ellipsoidal voids (centres in
    [0.25 L, 0.75 L]^3, semi-axes in [0.05 L, 0.12 L]); seeded impulsive
    velocity N(0, 1 m/s) on the nodes within one horizon of the x = 0 face."""
    rng = np.random.default_rng(seed)
    body = (nb, nb, nb)
    L = nb * dx
    c = _centres(nb, dx)
    chiB = np.ones(body, np.uint8)
    zz = c[:, None, None]
    yy = c[None, :, None]
    xx = c[None, None, :]
    for _ in range(nvoids):
        ctr = rng.uniform(0.25 * L, 0.75 * L, size=3)
        ax = rng.uniform(0.05 * L, 0.12 * L, size=3)
        inside = (((xx - ctr[0]) / ax[0]) ** 2 + ((yy - ctr[1]) / ax[1]) ** 2
                  + ((zz - ctr[2]) / ax[2]) ** 2) <= 1.0
        chiB[inside] = 0
    rng_v = np.random.default_rng(vseed)
    v0 = np.zeros((3,) + body)
    layer = int(round(m))
    v0[:, :, :, :layer] = rng_v.normal(0.0, 1.0, size=(3, nb, nb, layer))
    v0 *= chiB[None]
    return Workload(name=f"lps3d_voids_{nb}", dim=3, body=body, fft=(nfft,) * 3, dx=dx,
                    delta=m * dx, model="lps", E=E, nu=nu, rho=rho, dt=dt, steps=steps, chiB=chiB,
                    chiO=np.stack([chiB] * 3), u0=np.zeros((3,) + body), v0=v0,
                    b=np.zeros((3,) + body), w=np.zeros((3,) + body))


def random_field(shape, seed, scale=1.0, dist="normal"):
    rng = np.random.default_rng(seed)
    if dist == "normal":
        return rng.normal(0.0, scale, size=shape)
    return rng.uniform(-scale, scale, size=shape)


def random_mask(shape, seed, p_hole=0.15, blobs=3):
    """A body mask with a few seeded rectangular holes and ragged edges, for
    exercising the embedded constraints on small grids."""
    rng = np.random.default_rng(seed)
    chi = np.ones(shape, np.uint8)
    for _ in range(blobs):
        lo = [rng.integers(0, n) for n in shape]
        hi = [min(n, l + max(1, int(n * 0.3))) for l, n in zip(lo, shape)]
        chi[tuple(slice(l, h) for l, h in zip(lo, hi))] = 0
    chi[rng.random(shape) < p_hole * 0.1] = 0
    return chi


def _grid_len(n, m, mixed_ok=False):
    """Smallest supported FFT length >= n + m: a power of two (>= 16), or for
    the x axis also 2 R 2^p with R = 3, 5, 9 and 2^p >= 8."""
    need = max(16, n + m)
    best = 16
    while best < need:
        best *= 2
    if mixed_ok:
        for R in (3, 5, 9):
            p = 8
            while 2 * R * p < need:
                p *= 2
            best = min(best, 2 * R * p)
    return best


def cube_void_refined(m, delta=3e-3, edge_horizons=16, E=60e9, nu=0.4, b0=1e8):
    """The static cube of the refinement study (Sec. 5.1, Eq. 99): edge
    L = edge_horizons * delta, nodes at x = i dx (i = 0 .. N, N = L/dx), so
    that halving dx keeps every node (the coarse nodes are the even fine
    ones); a centred spherical void of radius 0.2 L, clamped (u = 0) on the
    layer z < 3 delta, a uniform body force -b0 along z on the unknowns.
    Same physical problem for every m = delta/dx; deterministic."""
    dx = delta / m
    N = edge_horizons * m
    n = N + 1
    L = N * dx
    c = np.arange(n) * dx
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    r2 = (x - L / 2) ** 2 + (y - L / 2) ** 2 + (z - L / 2) ** 2
    chiB = (r2 > (0.2 * L) ** 2).astype(np.uint8)
    omega = chiB.copy()
    omega[z < 3 * delta - 1e-12 * dx] = 0
    chiO = np.stack([omega, omega, omega])
    b = np.zeros((3, n, n, n))
    b[2] = -b0 * omega
    f = _grid_len(n, m)
    return Workload(name=f"lps3d_static_refined_m{m}", dim=3, body=(n, n, n),
                    fft=(f, f, _grid_len(n, m, mixed_ok=True)), dx=dx, delta=delta, model="lps", E=E, nu=nu,
                    chiB=chiB, chiO=chiO, u0=np.zeros((3, n, n, n)), b=b, w=np.zeros((3, n, n, n)),
                    extra={"m": m})


def notched_plate_refined(m, delta=1e-3, Lx=0.1, Ly=0.04, E=72e9, rho=2440.0, G0=3.8, sigma=4e6,
                          notch=0.05, dt=2.5e-8, steps=2000):
    """The notched glass plate of the fracture refinement study (Sec. 5.2,
    Fig. 15: sigma = 4 MPa, delta = 1 mm): a fixed horizon delta,
    dx = delta/m, nodes at x = i dx (i = 0 .. Lx/dx, so halving dx keeps
    every node), integrity 0 on a delta-thick notch layer on the mid-line for
    x < notch, tractions +-sigma as body forces sigma/delta on the
    delta-thick top and bottom layers, 50 us of loading.  Same physical
    problem for every m; deterministic."""
    dx = delta / m
    nx, ny = int(round(Lx / dx)) + 1, int(round(Ly / dx)) + 1
    xc, yc = np.arange(nx) * dx, np.arange(ny) * dx
    Y, X = np.meshgrid(yc, xc, indexing="ij")
    body = (ny, nx)
    chiB = np.ones(body, np.uint8)
    lam0 = np.ones(body, np.uint8)
    lam0[(X < notch) & (np.abs(Y - Ly / 2) < delta / 2)] = 0
    b = np.zeros((2,) + body)
    b[1][Y > Ly - delta] = sigma / delta
    b[1][Y < delta] = -sigma / delta
    fft = (_grid_len(ny, m), _grid_len(nx, m, mixed_ok=True))
    return Workload(name=f"bb2d_fracture_refined_m{m}", dim=2, body=body, fft=fft, dx=dx, delta=delta,
                    model="bb", E=E, nu=1.0 / 3.0, rho=rho, G0=G0, dt=dt, steps=steps, chiB=chiB,
                    chiO=np.stack([chiB, chiB]), u0=np.zeros((2,) + body), v0=np.zeros((2,) + body), b=b,
                    w=np.zeros((2,) + body), lam0=lam0, extra={"sigma": sigma, "m": m})
