"""ctypes binding of ``libpdfcbm.so`` (C ABI in ``include/pd_fcbm.h``).

Argument marshalling only: PyTorch tensors provide device memory and the
current HIP stream; every arithmetic step runs in the library's kernels.
There is no CPU fallback -- if the library is missing, calls raise.

Array conventions match the library: body-box fields, component-major,
shapes ``(dim, [nz,] ny, nx)`` for vectors and ``([nz,] ny, nx)`` for
scalars, x fastest; grid tuples are given in the same (z, y, x) / (y, x)
order as the arrays.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

from .build import LIB

PD_OK, PD_EINVAL, PD_ENOMEM, PD_EDEVICE, PD_ENOTCONV, PD_ENUMERIC, PD_EUNSUPPORTED = range(7)
_WEIGHTS = {"none": 0, "integrity": 1, "scale": 2}
_MODELS = {"bb": 0, "lps": 1, "nbb": 2}   # nbb: nonlinear bond-based (Eq. 19-26), pd_force only


class PDError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__(f"{where}: {status_str(status)} (status {status})")


class Grid(C.Structure):
    _fields_ = [("dim", C.c_int), ("fft_n", C.c_int64 * 3), ("body_n", C.c_int64 * 3),
                ("dx", C.c_double * 3)]


class Horizon(C.Structure):
    _fields_ = [("delta", C.c_double), ("influence", C.c_int)]


class Kernel(C.Structure):
    _fields_ = [("model", C.c_int), ("E", C.c_double), ("nu", C.c_double), ("rho", C.c_double),
                ("G0", C.c_double), ("weight", C.c_int)]


class Mask(C.Structure):
    _fields_ = [("chi_B", C.c_void_p), ("chi_Omega", C.c_void_p)]


class PlanInfo(C.Structure):
    _fields_ = [("dim", C.c_int), ("body_nodes", C.c_int64), ("fft_points", C.c_int64),
                ("stencil_size", C.c_int), ("alpha", C.c_double), ("m0", C.c_double),
                ("Wc", C.c_double), ("dt_max", C.c_double), ("workspace_bytes", C.c_int64),
                ("lds_per_block", C.c_int64)]


class State(C.Structure):
    _fields_ = [("u", C.c_void_p), ("v", C.c_void_p), ("F", C.c_void_p), ("W", C.c_void_p),
                ("lam", C.c_void_p), ("s", C.c_void_p), ("step", C.c_int64), ("flags", C.c_int32)]


STATE_EXACT_STEPS = 1


class SolveInfo(C.Structure):
    _fields_ = [("iters_fp64", C.c_int), ("iters_fp32", C.c_int), ("applies_fp64", C.c_int),
                ("applies_fp32", C.c_int), ("rel_res", C.c_double), ("precond_applies", C.c_int)]


SOLVE_MIXED, SOLVE_PRECOND = 1, 2


EXPORTS = ["pd_plan_create", "pd_plan_destroy", "pd_plan_query", "pd_force", "pd_force_adjoint",
           "pd_verlet_step", "pd_verlet_adjoint", "pd_static_solve", "pd_static_solve_noalloc", "pd_damage_index",
           "pd_status_str", "pd_test_conv", "pd_test_set_lastaxis", "pd_test_set_energy_form"]

_lib = None


def lib():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB):
        raise RuntimeError(f"libpdfcbm.so not found at {LIB}; run __graft_entry__.build() "
                           "(the FCBM path has no CPU fallback)")
    L = C.CDLL(LIB)
    vp = C.c_void_p
    L.pd_plan_create.argtypes = [C.POINTER(Grid), C.POINTER(Horizon), C.POINTER(Kernel),
                                 C.POINTER(Mask), C.c_int, C.c_int, vp, C.POINTER(vp)]
    L.pd_plan_destroy.argtypes = [vp]
    L.pd_plan_destroy.restype = None
    L.pd_plan_query.argtypes = [vp, C.POINTER(PlanInfo)]
    L.pd_force.argtypes = [vp, vp, vp, vp, vp, vp]
    L.pd_force_adjoint.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    L.pd_verlet_step.argtypes = [vp, C.POINTER(State), vp, vp, C.c_double, C.c_int,
                                 C.POINTER(C.c_double), vp]
    L.pd_verlet_adjoint.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, C.c_double, vp]
    L.pd_static_solve.argtypes = [vp, vp, vp, vp, C.c_double, C.c_int, C.c_int,
                                  C.POINTER(SolveInfo), vp]
    L.pd_static_solve_noalloc.argtypes = [vp, vp, vp, vp, C.c_double, C.c_int, C.c_int,
                                          C.POINTER(SolveInfo), vp]
    L.pd_damage_index.argtypes = [vp, vp, vp, vp]
    L.pd_status_str.argtypes = [C.c_int]
    L.pd_status_str.restype = C.c_char_p
    L.pd_test_conv.argtypes = [vp, vp, C.POINTER(C.c_int), C.c_int, vp, vp]
    L.pd_test_set_lastaxis.argtypes = [vp, C.c_int]
    L.pd_test_set_energy_form.argtypes = [vp, C.c_int]
    for name in EXPORTS:
        if name not in ("pd_plan_destroy", "pd_status_str"):
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


def status_str(s):
    try:
        return lib().pd_status_str(int(s)).decode()
    except Exception:  # library missing: still give a readable message
        return str(s)


def _check(s, where):
    if s != PD_OK:
        raise PDError(s, where)


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


class Plan:
    """An FCBM-EC operator on one GPU (see ``pd_plan_create``)."""

    def __init__(self, fft, body, dx, delta, model="bb", E=72e9, nu=0.25, rho=2440.0, G0=0.0,
                 weight="none", chiB=None, chiO=None, dtype=torch.float64, mixed=False,
                 influence=0):
        dim = len(body)
        assert len(fft) == dim and dim in (2, 3)
        self.dim = dim
        self.body = tuple(int(v) for v in body)
        self.fft = tuple(int(v) for v in fft)
        self.dtype = dtype
        self.weight = weight
        g = Grid()
        g.dim = dim
        bx = list(reversed(self.body)) + [1] * (3 - dim)
        fx = list(reversed(self.fft)) + [1] * (3 - dim)
        dxs = (list(dx) if np.ndim(dx) else [float(dx)] * dim)[::-1] + [1.0] * (3 - dim)
        for d in range(3):
            g.fft_n[d] = fx[d]
            g.body_n[d] = bx[d]
            g.dx[d] = dxs[d]
        h = Horizon(delta=float(delta), influence=int(influence))
        k = Kernel(model=_MODELS[model], E=float(E), nu=float(nu), rho=float(rho), G0=float(G0),
                   weight=_WEIGHTS[weight])
        self._chiB = None if chiB is None else np.ascontiguousarray(chiB, dtype=np.uint8)
        self._chiO = None if chiO is None else np.ascontiguousarray(chiO, dtype=np.uint8)
        if self._chiB is not None:
            assert self._chiB.shape == self.body
        if self._chiO is not None:
            assert self._chiO.shape == (dim,) + self.body
        m = Mask(chi_B=None if self._chiB is None else self._chiB.ctypes.data,
                 chi_Omega=None if self._chiO is None else self._chiO.ctypes.data)
        dt = 0 if dtype == torch.float32 else 1
        self._h = C.c_void_p()
        _check(lib().pd_plan_create(C.byref(g), C.byref(h), C.byref(k), C.byref(m), dt,
                                    1 if mixed else 0, _stream(), C.byref(self._h)), "pd_plan_create")
        inf = PlanInfo()
        _check(lib().pd_plan_query(self._h, C.byref(inf)), "pd_plan_query")
        self.info = {f: getattr(inf, f) for f, _ in PlanInfo._fields_}

    @classmethod
    def from_workload(cls, wl, dtype=torch.float64, weight=None, mixed=False, **kw):
        if weight is None:
            weight = "integrity" if wl.lam0 is not None else ("scale" if wl.s is not None else "none")
        return cls(wl.fft, wl.body, wl.dx, wl.delta, model=wl.model, E=wl.E, nu=wl.nu, rho=wl.rho,
                   G0=wl.G0, weight=weight, chiB=wl.chiB, chiO=wl.chiO, dtype=dtype, mixed=mixed, **kw)

    # -- helpers ------------------------------------------------------
    def _vec(self, t, name, dtype=None):
        dtype = dtype or self.dtype
        if t is None:
            return None
        if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()
                and tuple(t.shape) == (self.dim,) + self.body):
            raise ValueError(f"{name}: expected contiguous {dtype} CUDA tensor of shape "
                             f"{(self.dim,) + self.body}, got {t.dtype} {tuple(t.shape)}")
        return t

    def _sca(self, t, name, dtype=None):
        dtype = dtype or self.dtype
        if t is None:
            return None
        if not (t.is_cuda and t.dtype == dtype and t.is_contiguous() and tuple(t.shape) == self.body):
            raise ValueError(f"{name}: expected contiguous {dtype} CUDA tensor of shape {self.body}")
        return t

    def _weight(self, w):
        if self.weight == "none":
            if w is not None:
                raise ValueError("this plan takes no weight")
            return None
        if self.weight == "integrity":
            return self._sca(w, "lambda", torch.uint8)
        return self._sca(w, "s")

    def empty_vec(self):
        return torch.empty((self.dim,) + self.body, dtype=self.dtype, device="cuda")

    # -- entry points -------------------------------------------------
    def force(self, u, weight=None, energy=False, out=None):
        u = self._vec(u, "u")
        w = self._weight(weight)
        L = out if out is not None else self.empty_vec()
        W = torch.empty(self.body, dtype=self.dtype, device="cuda") if energy else None
        _check(lib().pd_force(self._h, _ptr(u), _ptr(w), _ptr(L), _ptr(W), _stream()), "pd_force")
        return (L, W) if energy else L

    def force_adjoint(self, u, g, weight=None, want_weight_bar=False):
        u = self._vec(u, "u")
        g = self._vec(g, "g_bar")
        w = self._weight(weight)
        ub = self.empty_vec()
        wb = torch.empty(self.body, dtype=self.dtype, device="cuda") if want_weight_bar else None
        _check(lib().pd_force_adjoint(self._h, _ptr(u), _ptr(w), _ptr(g), _ptr(ub), _ptr(wb), _stream()),
               "pd_force_adjoint")
        return (ub, wb) if want_weight_bar else ub

    def verlet(self, state, dt, nsteps, b=None, w=None, energy=False, exact_steps=False):
        """Advance ``state`` (dict with u, v, F and optionally W, lam, s, step).
        exact_steps: every step reads and writes (v, F), so the call equals
        nsteps one-step calls bit for bit (PD_STATE_EXACT_STEPS)."""
        for k in ("u", "v", "F"):
            self._vec(state[k], k)
        b = self._vec(b, "b")
        w = self._vec(w, "w")
        st = State(u=state["u"].data_ptr(), v=state["v"].data_ptr(), F=state["F"].data_ptr(),
                   W=None if state.get("W") is None else self._sca(state["W"], "W").data_ptr(),
                   lam=None if state.get("lam") is None else self._sca(state["lam"], "lam", torch.uint8).data_ptr(),
                   s=None if state.get("s") is None else self._sca(state["s"], "s").data_ptr(),
                   step=int(state.get("step", 0)), flags=STATE_EXACT_STEPS if exact_steps else 0)
        en = (C.c_double * (4 * nsteps))() if energy else None
        _check(lib().pd_verlet_step(self._h, C.byref(st), _ptr(b), _ptr(w), float(dt), int(nsteps),
                                    en, _stream()), "pd_verlet_step")
        state["step"] = st.step
        if energy:
            return np.array(en, dtype=np.float64).reshape(nsteps, 4)
        return None

    def verlet_adjoint(self, u_n, u_np1, u_bar, v_bar, dt, s=None, s_bar=None, b_bar=None):
        _check(lib().pd_verlet_adjoint(self._h, _ptr(self._vec(u_n, "u_n")), _ptr(self._vec(u_np1, "u_np1")),
                                       _ptr(self._sca(s, "s")), _ptr(self._vec(u_bar, "u_bar")),
                                       _ptr(self._vec(v_bar, "v_bar")), _ptr(self._sca(s_bar, "s_bar")),
                                       _ptr(self._vec(b_bar, "b_bar")), float(dt), _stream()), "pd_verlet_adjoint")

    def static_solve(self, b, w=None, u0=None, rtol=1e-10, maxit=100000, mixed=False, precond=False,
                     check=True, noalloc=False, out=None):
        """pd_static_solve (noalloc=True: pd_static_solve_noalloc; ``out``, if
        given, is the FP64 tensor that receives the solution, initial guess
        taken from u0 or zero)."""
        b = self._vec(b, "b", torch.float64)
        w = self._vec(w, "w", torch.float64)
        if out is not None:
            u = self._vec(out, "out", torch.float64)
            if u0 is None:
                u.zero_()
            else:
                u.copy_(self._vec(u0, "u0", torch.float64))
        else:
            u = torch.zeros_like(b) if u0 is None else self._vec(u0, "u0", torch.float64).clone()
        inf = SolveInfo()
        opts = (SOLVE_MIXED if mixed else 0) | (SOLVE_PRECOND if precond else 0)
        fn = lib().pd_static_solve_noalloc if noalloc else lib().pd_static_solve
        s = fn(self._h, _ptr(b), _ptr(w), _ptr(u), float(rtol), int(maxit), opts, C.byref(inf), _stream())
        if check:
            _check(s, "pd_static_solve_noalloc" if noalloc else "pd_static_solve")
        info = {f: getattr(inf, f) for f, _ in SolveInfo._fields_}
        info["status"] = s
        return u, info

    def damage_index(self, lam):
        lam = self._sca(lam, "lambda", torch.uint8)
        d = torch.empty(self.body, dtype=self.dtype, device="cuda")
        _check(lib().pd_damage_index(self._h, _ptr(lam), _ptr(d), _stream()), "pd_damage_index")
        return d

    def test_conv(self, x, shift, parity):
        x = self._sca(x, "x")
        out = torch.empty_like(x)
        sh = (C.c_int * 3)(*(list(reversed(list(shift))) + [0] * (3 - len(shift))))
        _check(lib().pd_test_conv(self._h, _ptr(x), sh, int(parity), _ptr(out), _stream()), "pd_test_conv")
        return out

    LASTAXIS = {"auto": 0, "fft": 1, "fft_generic": 2, "yfft": 3}

    def set_lastaxis(self, mode="auto"):
        """Kernel choice after the x transform (A/B tests): 'auto' (3D: the
        direct (y, z) correlation where it applies), 'yfft' (transform along
        y, direct line correlation along the last axis), 'fft' (transforms on
        every axis, spectral multiply, specialised where it applies) or
        'fft_generic'."""
        _check(lib().pd_test_set_lastaxis(self._h, self.LASTAXIS[mode]), "pd_test_set_lastaxis")

    ENERGY_FORMS = {"direct": 0, "convolution": 1}

    def set_energy_form(self, form="direct"):
        """How W is evaluated (A/B tests): 'direct' bond sums (default) or the
        paper's 'convolution' form in the force chain."""
        _check(lib().pd_test_set_energy_form(self._h, self.ENERGY_FORMS[form]), "pd_test_set_energy_form")

    def close(self):
        if getattr(self, "_h", None):
            lib().pd_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
