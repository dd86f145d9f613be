"""Forward-plus-adjoint on the heterogeneous-micromodulus plate at full size:
512 x 512 nodes on a 1024 x 1024 grid, delta = 3 dx, micromodulus
c = c0 (1 + 0.2 g) with g a Gaussian random field of correlation length
20 dx, 200 Verlet steps from seeded velocities, loss |u(T) - u_target|^2,
checkpoints every 20 steps.  Gradients with respect to the micromodulus
field and the initial displacement from the checkpointed adjoint (the
autograd wrapper over pd_verlet_adjoint) against central finite differences
on 32 random directions each (Richardson-extrapolated for the nonlinear
micromodulus dependence), in FP64 to 1e-6; the FP32 gradients against the
FP64 ones.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2105_06055_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _dev(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _grads(w, dtype):
    from paper_2105_06055_amd import binding
    from paper_2105_06055_amd.autograd import VerletRollout
    plan = binding.Plan.from_workload(w, dtype=dtype)
    u0 = _dev(w.u0, dtype).requires_grad_(True)
    v0 = _dev(w.v0, dtype)
    s = _dev(w.s, dtype).requires_grad_(True)
    target = _dev(w.extra["u_target"], dtype)
    uT, _ = VerletRollout.apply(plan, u0, v0, s, w.dt, w.steps, 20)
    ((uT - target) ** 2).sum().backward()
    gc = (s.grad / (2 * s)).detach()   # s = sqrt(c / c0)
    return plan, u0.grad.detach(), gc


def test_hetero_plate_512_adjoint_vs_fd():
    w = wl.hetero_plate_adjoint()          # 512^2 body, 1024^2 grid, 200 steps, 32 directions
    plan, gu, gc = _grads(w, torch.float64)
    target = _dev(w.extra["u_target"])
    v0 = _dev(w.v0)
    c_rel = _dev(w.extra["c_rel"])

    def loss(u0, c):
        with torch.no_grad():
            st = {"u": u0.clone().contiguous(), "v": v0.clone(), "F": torch.zeros_like(u0),
                  "s": torch.sqrt(c).contiguous(), "step": 0}
            plan.verlet(st, w.dt, w.steps)
            return float(((st["u"] - target) ** 2).sum())

    u0 = _dev(w.u0)
    ndir = w.extra["dirs_u"].shape[0]
    assert ndir == 32
    worst_u = worst_c = 0.0
    for d in range(ndir):
        # the loss is quadratic in u0: central differences are exact up to rounding
        du = _dev(w.extra["dirs_u"][d])
        eps = 1e-4
        fd = (loss(u0 + eps * du, c_rel) - loss(u0 - eps * du, c_rel)) / (2 * eps)
        an = float((gu * du).sum())
        worst_u = max(worst_u, abs(an - fd) / abs(fd))
        # nonlinear in c: central differences at eps and eps/2, Richardson
        # extrapolated (truncation error O(eps^4)).  The directional
        # derivatives are ~1e-6 of the loss, so the steps are large enough to
        # keep the rounding of the loss itself (FP64) below ~1e-8 relative.
        dc = _dev(w.extra["dirs_c"][d])
        eps = 2e-2
        fd1 = (loss(u0, c_rel + eps * dc) - loss(u0, c_rel - eps * dc)) / (2 * eps)
        fd2 = (loss(u0, c_rel + 0.5 * eps * dc) - loss(u0, c_rel - 0.5 * eps * dc)) / eps
        fd = (4 * fd2 - fd1) / 3
        an = float((gc * dc).sum())
        worst_c = max(worst_c, abs(an - fd) / abs(fd))
    print(f"adjoint vs central differences, 32 directions each: max rel err dL/du0 {worst_u:.2e}, "
          f"dL/dc {worst_c:.2e}")
    assert worst_u <= 1e-6
    assert worst_c <= 1e-6
    plan.close()
    # the FP32 path against the FP64 gradients
    plan32, gu32, gc32 = _grads(w, torch.float32)
    ru = float(torch.linalg.vector_norm(gu32.double() - gu) / torch.linalg.vector_norm(gu))
    rc = float(torch.linalg.vector_norm(gc32.double() - gc) / torch.linalg.vector_norm(gc))
    print(f"FP32 gradients against FP64: rel err dL/du0 {ru:.2e}, dL/dc {rc:.2e}")
    assert ru <= 1e-3 and rc <= 1e-3
    plan32.close()
