"""FFT machinery on the GPU: correlation with separable even/odd test kernels
through the same passes as pd_force, against shifted copies (numpy.roll on
the zero-padded periodic grid).  Exercises r2c/c2r, every line length,
the strided z pass, pruning to the body box, normalisation and the i^P
factors of odd kernels."""
import itertools

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def expected_conv(x, fft, shift, parity):
    dim = x.ndim
    pad = np.zeros(fft)
    pad[tuple(slice(0, n) for n in x.shape)] = x
    out = np.zeros(fft)
    # shift/parity in (x, y, z) order; arrays in (z, y, x) order
    choices = []
    for d in range(dim):
        s = shift[d]
        choices.append([(s, 1.0), (-s, -1.0 if (parity >> d) & 1 else 1.0)] if s else [(0, 1.0)])
    for combo in itertools.product(*choices):
        sgn = np.prod([c[1] for c in combo])
        offs = [c[0] for c in combo]  # x, y, z
        rolled = pad
        for d in range(dim):
            axis = dim - 1 - d
            rolled = np.roll(rolled, -offs[d], axis=axis)  # out(x) = pad(x + o)
        out += sgn * rolled
    return out[tuple(slice(0, n) for n in x.shape)]


CASES_2D = [((16, 32), (13, 21)), ((64, 128), (40, 100)), ((128, 64), (100, 40)),
            ((512, 1024), (400, 1000)), ((32, 2048), (9, 1700)), ((1024, 64), (1000, 33))]
CASES_3D = [((16, 16, 32), (9, 11, 20)), ((16, 32, 16), (12, 20, 12)), ((32, 64, 32), (20, 50, 17)), ((64, 32, 128), (50, 21, 100)),
            ((256, 16, 64), (200, 5, 40))]
# x lengths n1 = 2 R 2^p (R = 3, 5, 9): the mixed-radix x transforms
CASES_MIXED = [((16, 48), (13, 21)), ((64, 80), (40, 60)), ((32, 144), (20, 100)), ((16, 96), (9, 50)),
               ((16, 384), (9, 256)), ((16, 320), (9, 256)), ((16, 288), (9, 256)), ((64, 2 * 9 * 64), (40, 1000)),
               ((16, 16, 48), (9, 11, 20)), ((32, 64, 80), (20, 50, 60)), ((16, 32, 288), (9, 20, 256)),
               ((16, 16, 384), (10, 12, 256))]


def _plan(fft, body, dtype):
    from paper_2105_06055_amd import binding
    return binding.Plan(fft, body, 1e-3, 1.5e-3, model="bb", E=1e9, dtype=dtype)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("fft,body", CASES_2D + CASES_3D + CASES_MIXED)
def test_conv_shift_kernels(fft, body, dtype):
    dim = len(fft)
    td = torch.float64 if dtype == "f64" else torch.float32
    plan = _plan(fft, body, td)
    rng = np.random.default_rng(sum(fft) + sum(body))
    x = rng.normal(size=body)
    xt = torch.tensor(x, dtype=td, device="cuda")
    tol = 1e-13 if dtype == "f64" else 2e-6
    shifts = [(1, 0, 0), (2, 1, 0), (0, 3, 1), (1, 2, 3)]
    for sh in shifts:
        sh = sh[:dim]
        if dim == 2 and sh == (0, 3):
            pass
        nz = [d for d in range(dim) if sh[d]]
        for parity in range(1 << dim):
            if any(((parity >> d) & 1) and not sh[d] for d in range(dim)):
                continue
            out = plan.test_conv(xt, tuple(reversed(sh)), parity).cpu().numpy()
            ref = expected_conv(x, fft, sh, parity)
            err = np.abs(out - ref).max() / np.abs(ref).max()
            assert err <= tol, (fft, body, sh, parity, err)
    plan.close()
