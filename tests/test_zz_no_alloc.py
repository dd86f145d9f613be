"""pd_static_solve_noalloc (the solve with its vectors in the library's
static device array instead of per-call hipMalloc) against pd_static_solve:
two calls in a row on different plans, the second one smaller, in every
solve variant; the results are the same bit for bit (same kernels in the
same order), and a solve larger than the array is refused."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2105_06055_amd import workloads as wl

pytestmark = pytest.mark.gpu

VARIANTS = [(False, False), (True, False), (False, True), (True, True)]


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("mixed,precond", VARIANTS)
def test_noalloc_solve_equals_solve(mixed, precond):
    from paper_2105_06055_amd import binding
    for nb, nfft in ((24, 32), (12, 16)):   # second call: smaller input
        w = wl.cube_void_static(seed=2, nb=nb, nfft=nfft, clamp_layers=3)
        plan = binding.Plan.from_workload(w, dtype=torch.float64, mixed=mixed)
        b = _dev(w.b)
        print(f"noalloc solve: body {nb}^3, mixed={mixed}, precond={precond}", flush=True)
        u_ref, inf_ref = plan.static_solve(b, rtol=1e-10, maxit=20000, mixed=mixed, precond=precond)
        u_na, inf_na = plan.static_solve(b, rtol=1e-10, maxit=20000, mixed=mixed, precond=precond,
                                         noalloc=True)
        torch.cuda.synchronize()
        assert inf_na["status"] == binding.PD_OK
        assert inf_na["rel_res"] <= 1e-10
        for k in ("iters_fp64", "iters_fp32", "applies_fp64", "applies_fp32", "precond_applies"):
            assert inf_na[k] == inf_ref[k], k
        assert inf_na["rel_res"] == inf_ref["rel_res"]
        assert torch.equal(u_na, u_ref)
        plan.close()


def test_noalloc_refuses_oversized_solve():
    from paper_2105_06055_amd import binding
    nb = 144                     # 3 * 144^3 unknowns * 32 B > 256 MiB
    body = (nb, nb, nb)
    plan = binding.Plan((256, 256, 256), body, 1e-3, 3e-3, model="lps", E=200e9, nu=0.25,
                        dtype=torch.float64)
    b = torch.zeros((3,) + body, dtype=torch.float64, device="cuda")
    u, info = plan.static_solve(b, rtol=1e-10, maxit=10, noalloc=True, check=False)
    assert info["status"] == binding.PD_EINVAL
    plan.close()
