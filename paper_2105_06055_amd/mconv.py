"""m-convergence harness: the GPU force density of a quadratic displacement
field at the centre of a fully interior block, against the continuum Navier
operator of the same elastic constants, as the grid is refined under a fixed
horizon (m = delta/dx grows).

For u_i = 1/2 H_ijk x_j x_k the continuum operator is constant,
  L_i = (lambda + mu) sum_j H_jji + mu sum_j H_ijj,
with the Lame constants of the model (bond-based: lambda = mu, 3E/8 in 2D
plane stress and 2E/5 in 3D; LPS: from E and nu).  The discrete operator
differs from it by the error of the one-point quadrature of the bond sums
(no partial-volume correction, Sec. 4.1.1), which this harness measures; it
decreases with m only on average (which lattice points fall inside the
horizon ball changes from one m to the next).
Inputs are the seeded quadratic field only; the block is sized so that the
centre's whole dependence (one horizon for bond-based, two for LPS) lies
inside the body.
"""
from __future__ import annotations

import numpy as np


def lame(model: str, dim: int, E: float, nu: float):
    if model == "bb":
        lam = 3 * E / 8 if dim == 2 else 2 * E / 5
        return lam, lam
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    return lam, E / (2 * (1 + nu))


def case(model: str, dim: int, m: int, delta: float = 3e-3, seed: int = 7):
    """Body, grid, spacing, field and continuum value for one m."""
    dx = delta / m
    reach = m if model == "bb" else 2 * m
    n = 2 * reach + 5
    nfft = 16
    while nfft < n + m:
        nfft *= 2
    shape = (n,) * dim
    rng = np.random.default_rng(seed)
    H = rng.normal(size=(dim, dim, dim)) / delta   # |u| ~ delta-scale curvature
    H = 0.5 * (H + H.transpose(0, 2, 1))
    X = np.stack(np.meshgrid(*[(np.arange(k) - k // 2) * dx for k in shape], indexing="ij")[::-1])
    u = 0.5 * np.einsum("jkl,k...,l...->j...", H, X, X) * 1e-6
    return dict(shape=shape, fft=(nfft,) * dim, dx=dx, u=u, H=H * 1e-6, centre=(n // 2,) * dim)


def navier(H, lam, mu):
    return (lam + mu) * np.einsum("jji->i", H) + mu * np.einsum("ijj->i", H)


def run(models=(("bb", 2), ("bb", 3), ("lps", 3)), ms=(2, 3, 4, 6, 8), E=70e9, nu=0.3, dtype=None):
    """GPU pd_force (FP64 by default) at the block centre for each m; returns
    {f"{model}{dim}d": [(m, rel. error vs Navier), ...]}."""
    import torch

    from . import binding
    dtype = dtype or torch.float64
    out = {}
    for model, dim in models:
        rows = []
        for m in ms:
            c = case(model, dim, m)
            plan = binding.Plan(c["fft"], c["shape"], c["dx"], m * c["dx"], model=model, E=E, nu=nu, dtype=dtype)
            L = plan.force(torch.tensor(c["u"], dtype=dtype, device="cuda")).cpu().numpy()
            plan.close()
            lam, mu = lame(model, dim, E, nu)
            ref = navier(c["H"], lam, mu)
            got = L[(slice(None),) + c["centre"]]
            rows.append((m, float(np.abs(got - ref).max() / np.abs(ref).max())))
        out[f"{model}{dim}d"] = rows
    return out
