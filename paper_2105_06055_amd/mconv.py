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


def static_refinement(ms=(2, 3, 4, 6, 8), rtol=1e-10, precond=True):
    """Convergence of elastostatic solutions under refinement at a fixed
    horizon (Sec. 5.1, Fig. 10): the voided, clamped LPS cube
    (workloads.cube_void_refined) solved on the GPU (FP64 CG, spectral
    preconditioner by default) for each m = delta/dx, and the relative error
    of Eq. 99 between solutions with dx_new = dx_old / 2, on the coarse
    nodes (the even nodes of the fine grid).  Returns the per-m solve
    records and the Eq. 99 rows."""
    import time

    import torch

    from . import binding, workloads
    sol, solves = {}, []
    for m in ms:
        w = workloads.cube_void_refined(m)
        plan = binding.Plan.from_workload(w, dtype=torch.float64)
        b = torch.tensor(w.b, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u, info = plan.static_solve(b, rtol=rtol, maxit=50000, precond=precond)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        sol[m] = u.cpu().numpy()
        plan.close()
        del u, b
        torch.cuda.empty_cache()
        solves.append({"m": m, "dx": w.dx, "nodes": w.nodes, "fft": list(w.fft), "iterations": info["iters_fp64"],
                       "rel_res": info["rel_res"], "seconds": dt,
                       "max_abs_u": float(np.abs(sol[m]).max())})
    rows = []
    for m in ms:
        if 2 * m in sol:
            old, new = sol[m], sol[2 * m][:, ::2, ::2, ::2]
            rows.append({"m_old": m, "m_new": 2 * m, "dx_old": solves[ms.index(m)]["dx"],
                         "rel_error": float(np.linalg.norm(new - old) / np.linalg.norm(new))})
    return {"solves": solves, "eq99": rows}


def fracture_refinement(ms=(2, 3, 4, 6, 8), dtype=None, chunk=100):
    """Fracture under refinement at a fixed horizon (Sec. 5.2, Fig. 15): the
    notched plate of workloads.notched_plate_refined with the pointwise
    energy failure rule, run for the same physical time at each m; every
    `chunk` steps the crack tip (largest x of a failed node beyond the notch
    in the central half of the plate height, away from the loaded layers)
    and the failed area there; at the end the failed area of the whole plate
    and the difference of the damage maps between m and 2m on the coarse
    nodes, |d_2m - d_m| / |d_2m| (the Eq. 99 measure applied to the damage
    index)."""
    import torch

    from . import binding, workloads
    dtype = dtype or torch.float32
    out, dmaps = [], {}
    for m in ms:
        w = workloads.notched_plate_refined(m)
        plan = binding.Plan.from_workload(w, dtype=dtype, weight="integrity")
        dev = lambda a, t=dtype: torch.tensor(np.ascontiguousarray(a), dtype=t, device="cuda")
        st = {"u": dev(w.u0), "v": dev(w.v0), "F": torch.zeros((2,) + w.body, dtype=dtype, device="cuda"),
              "lam": dev(w.lam0, torch.uint8), "W": torch.zeros(w.body, dtype=dtype, device="cuda"), "step": 0}
        b = dev(w.b)
        xs = np.arange(w.body[1]) * w.dx
        ys = np.arange(w.body[0]) * w.dx
        Ly = ys[-1]
        band = torch.tensor(np.abs(ys - Ly / 2) < Ly / 4, device="cuda")
        beyond = torch.tensor(xs >= 0.05, device="cuda")
        lam0_band = torch.tensor(w.lam0, device="cuda")[band]
        tips = []
        done = 0
        while done < w.steps:
            n = min(chunk, w.steps - done)
            plan.verlet(st, w.dt, n, b=b)
            done += n
            failed = (lam0_band == 1) & (st["lam"][band] == 0)
            failed_cols = (failed.any(dim=0) & beyond).nonzero()
            tip = float(xs[int(failed_cols.max().item())]) if failed_cols.numel() else 0.05
            tips.append([done * w.dt, tip, float(failed.sum().item() * w.dx * w.dx)])
        d = plan.damage_index(st["lam"]).double().cpu().numpy()
        lam = st["lam"].cpu().numpy()
        plan.close()
        dmaps[m] = d
        out.append({"m": m, "dx": w.dx, "nodes": w.nodes, "steps": w.steps, "dt": w.dt,
                    "failed_nodes": int((w.lam0.astype(int) - lam.astype(int)).sum()),
                    "failed_area_m2": float((w.lam0.astype(int) - lam.astype(int)).sum() * w.dx * w.dx),
                    "tip_x_and_band_area_vs_time": tips})
    # node-by-node damage maps differ wherever a crack or a branch sits one
    # node apart, so this measure stays of order one for cracks; the crack
    # tip history is the converging quantity
    diffs = []
    for m in ms:
        if 2 * m in dmaps:
            old, new = dmaps[m], dmaps[2 * m][::2, ::2]
            diffs.append({"m_old": m, "m_new": 2 * m,
                          "damage_rel_diff": float(np.linalg.norm(new - old) / np.linalg.norm(new))})
    fine = np.array([t[1] for t in out[-1]["tip_x_and_band_area_vs_time"]])
    for r in out:
        tip = np.array([t[1] for t in r["tip_x_and_band_area_vs_time"]])
        r["tip_max_abs_dev_from_finest_m"] = float(np.abs(tip - fine).max())
    return {"runs": out, "damage_map_diffs": diffs}
