"""Element-wise parity bars shared by the GPU tests (not a test module).

Every comparison is node by node and component by component:

* ``rel_max = max |x - x_ref| / max |x_ref|``, the largest error over the
  whole field relative to the field's largest value;
* ``op_err = max |L - L_ref| / (lambda_max * max |u|)``, the largest force
  error relative to the operator scale (lambda_max from the plan's stability
  bound), the measure that stays meaningful in FP32 when the force is much
  smaller than lambda_max |u| (smooth fields, the reading of "relative" for
  FP32).

Bars: FP64 forces ``rel_max <= 1e-12``; FP32 forces ``op_err <= 1e-5`` and
``rel_max <= 1e-4``.
"""
import numpy as np

FP64_REL = 1e-12
FP32_OP = 1e-5
FP32_REL = 1e-4


def rel_max(x, ref):
    x, ref = np.asarray(x), np.asarray(ref)
    return float(np.max(np.abs(x - ref)) / np.max(np.abs(ref)))


def lam_max(plan, rho):
    """Largest eigenvalue bound of the operator (per unit volume), from the
    plan's velocity-Verlet stability bound dt_max = 2 / sqrt(lambda_max / rho)."""
    return rho * (2.0 / plan.info["dt_max"]) ** 2


def op_err(L, L_ref, u, lam):
    return float(np.max(np.abs(np.asarray(L) - np.asarray(L_ref))) / (lam * np.max(np.abs(u))))


def check_force(L, L_ref, u, plan, rho, fp64, tag=""):
    """Assert the force bars; returns (rel_max, op_err) and prints them."""
    r = rel_max(L, L_ref)
    e = op_err(L, L_ref, u, lam_max(plan, rho))
    print(f"parity {tag}: rel_max {r:.2e} op_err {e:.2e}", flush=True)
    if fp64:
        assert r <= FP64_REL, (r, e)
    else:
        assert e <= FP32_OP, (r, e)
        assert r <= FP32_REL, (r, e)
    return r, e
