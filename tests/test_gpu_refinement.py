"""Refinement studies at a fixed horizon (paper_2105_06055_amd/mconv.py):
their coarsest points against the oracle.

* Statics (Sec. 5.1, Eq. 99): the voided, clamped LPS cube of the
  refinement study at m = 2 (33^3 nodes on vertex-centred grids), solved on
  the GPU (FP64, spectral preconditioner) and by the oracle's plain CG.
* Fracture (Sec. 5.2, Fig. 15): the notched plate of the study at m = 3
  (delta = 1 mm, 4 MPa, 50 us, FP64): integrity map bit-exact against the
  oracle stepped one step at a time (tie margin checked every step), then
  the oracle's critical bond-strain rule on the same plate alongside:
  both cracks grow from the notch tip.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2105_06055_amd import workloads as wl

import parity

pytestmark = pytest.mark.gpu


def _dev(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def test_static_refinement_coarse_point(orc):
    from paper_2105_06055_amd import binding
    w = wl.cube_void_refined(2)
    plan = binding.Plan.from_workload(w, dtype=torch.float64)
    u, info = plan.static_solve(_dev(w.b), rtol=1e-10, maxit=20000, precond=True)
    plan.close()
    g = orc.geom(w.body, w.dx, w.delta)
    mdl = orc.model("lps", E=w.E, nu=w.nu)
    uo, it, rr = orc.static_cg(g, mdl, w.chiB, w.chiO, w.b, rtol=1e-12, maxit=50000)
    e = parity.rel_max(u.cpu().numpy(), uo)
    print(f"refined cube m=2: GPU PCG {info['iters_fp64']} iterations, oracle CG {it}; rel_max {e:.2e}")
    assert info["rel_res"] <= 1e-10 and rr <= 2e-12
    assert e <= 1e-7, e


def _new_cols(new, xs, band):
    """x of the columns holding new damage in the central band."""
    return xs[np.nonzero(new[band].any(axis=0))[0]]


def test_fracture_refinement_coarse_point_and_bond_rule(orc):
    """Energy rule: GPU integrity map bit-exact against the oracle after
    every 5 us; the crack starts at the notch tip and runs through the
    plate.  The oracle's bond rule on the same plate: its crack also starts
    at the notch tip and crosses the plate.  Tip histories printed."""
    from paper_2105_06055_amd import binding
    w = wl.notched_plate_refined(3)
    ny, nx = w.body
    xs = np.arange(nx) * w.dx
    ys = np.arange(ny) * w.dx
    band = np.abs(ys - ys[-1] / 2) < ys[-1] / 4
    chunk = 200
    plan = binding.Plan.from_workload(w, dtype=torch.float64, weight="integrity")
    st = {"u": _dev(w.u0), "v": _dev(w.v0), "F": torch.zeros((2,) + w.body, dtype=torch.float64, device="cuda"),
          "lam": _dev(w.lam0, torch.uint8), "W": torch.zeros(w.body, dtype=torch.float64, device="cuda"),
          "step": 0}
    b = _dev(w.b)
    g = orc.geom(w.body, w.dx, w.delta)
    alpha = orc.bb_alpha(2, w.E, w.delta)
    Wc = w.G0 / w.delta
    mdl = orc.model("bb", E=w.E, alpha=alpha, rho=w.rho, Wc=Wc)
    o = {"u": w.u0, "v": w.v0, "F": None, "W": None, "lam": w.lam0}
    margin = np.inf
    hist_en, first_en = [], None
    for k in range(w.steps):
        o = orc.verlet(g, mdl, w.chiB, w.chiO, o["u"], o["v"], w.dt, 1, b=w.b, lam=o["lam"], F=o["F"],
                       W=o["W"], init=(k == 0))
        alive = o["lam"] == 1
        margin = min(margin, float(np.abs(o["W"][alive] - Wc).min() / Wc))
        if (k + 1) % chunk == 0:
            plan.verlet(st, w.dt, chunk, b=b)
            assert np.array_equal(st["lam"].cpu().numpy(), o["lam"]), k + 1
            cols = _new_cols((o["lam"] == 0) & (w.lam0 == 1), xs, band)
            if len(cols) and first_en is None:
                first_en = (float(cols.min()), float(cols.max()))
            hist_en.append(float(cols.max()) if len(cols) else 0.05)
    plan.close()
    assert margin > 1e-9, margin

    # the critical bond-strain rule on the same plate: the notch as the bonds
    # crossing the mid-line left of the notch tip
    S = orc.stencil(g)
    mu = orc.bond_mu(g).reshape(ny, nx, -1)
    Y, X = np.meshgrid(ys, xs, indexing="ij")
    ymid = ys[-1] / 2
    for k, (ox, oy, _) in enumerate(S):
        if oy == 0:
            continue
        y2 = Y + oy * w.dx
        cross = (np.minimum(Y, y2) < ymid) & (np.maximum(Y, y2) >= ymid)
        xcross = X + (ymid - Y) / (oy * w.dx) * ox * w.dx
        mu[:, :, k] &= ~(cross & (xcross < 0.05)).astype(np.uint8)
    mu = np.ascontiguousarray(mu.reshape(ny * nx, -1))
    db0 = orc.bond_damage(g, w.chiB, mu)
    sc = orc.bond_sc(2, alpha, w.G0, w.delta)
    ob = {"u": w.u0, "v": w.v0, "F": None}
    hist_bd, first_bd = [], None
    for k in range(0, w.steps, chunk):
        ob, _ = orc.bond_verlet(g, alpha, w.rho, sc, w.chiB, w.chiO, mu, ob["u"], ob["v"], w.dt, chunk, b=w.b,
                                F=ob["F"], init=(k == 0))
        cols = _new_cols(orc.bond_damage(g, w.chiB, mu) > db0 + 1e-12, xs, band)
        if len(cols) and first_bd is None:
            first_bd = (float(cols.min()), float(cols.max()))
        hist_bd.append(float(cols.max()) if len(cols) else 0.05)
    t = [round((k + 1) * chunk * w.dt * 1e6, 1) for k in range(len(hist_en))]
    print(f"refined plate m=3: tie margin {margin:.2e}")
    print("  t (us)          " + " ".join(f"{v:6.1f}" for v in t))
    print("  energy-rule tip " + " ".join(f"{v:6.4f}" for v in hist_en))
    print("  bond-rule tip   " + " ".join(f"{v:6.4f}" for v in hist_bd))
    print(f"  first new damage in the band: energy rule x in {first_en}, bond rule x in {first_bd}")
    # both cracks start at the notch tip (within a horizon) and cross the plate
    for first in (first_en, first_bd):
        assert first is not None and 0.05 - w.delta - 1e-12 <= first[0] and first[1] <= 0.05 + 3 * w.delta
    assert hist_en[-1] > 0.09 and hist_bd[-1] > 0.09
