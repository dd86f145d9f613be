"""Python access to the FP64 direct-summation oracle (``pd_oracle.c``).

TEST INFRASTRUCTURE ONLY.  The product library never imports this module;
only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` use it.  It shares no code with the HIP path: it receives plain
NumPy arrays produced by the seeded input generators and returns NumPy
arrays.

Every function follows the one-point quadrature of the peridynamic integrals
(paper Sec. 4.1.1, Eq. 55) summed bond by bond; see the C file for the exact
formulas and the equation each follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pd_oracle.c")
_SO = os.path.join(_HERE, "_build", "libpdoracle.so")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (FP64, OpenMP over nodes)."""
    os.makedirs(os.path.dirname(_SO), exist_ok=True)
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


class Geom(C.Structure):
    _fields_ = [("dim", C.c_int), ("nb", C.c_int * 3), ("periodic", C.c_int),
                ("dx", C.c_double * 3), ("delta", C.c_double), ("influence", C.c_int)]


class Model(C.Structure):
    _fields_ = [("model", C.c_int), ("E", C.c_double), ("nu", C.c_double),
                ("alpha", C.c_double), ("rho", C.c_double), ("Wc", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        dp = C.POINTER(C.c_double)
        up = C.POINTER(C.c_uint8)
        gp = C.POINTER(Geom)
        mp = C.POINTER(Model)
        _lib.orc_threads.restype = C.c_int
        _lib.orc_stencil.argtypes = [gp, C.POINTER(C.c_int), C.c_int]
        _lib.orc_stencil.restype = C.c_int
        _lib.orc_bb_alpha.argtypes = [C.c_int, C.c_int, C.c_double, C.c_double]
        _lib.orc_bb_alpha.restype = C.c_double
        _lib.orc_m0.argtypes = [gp]
        _lib.orc_m0.restype = C.c_double
        _lib.orc_bb_force.argtypes = [gp, C.c_double, dp, dp, dp]
        _lib.orc_bb_energy.argtypes = [gp, C.c_double, dp, dp, dp]
        _lib.orc_nbb_force.argtypes = [gp, C.c_double, dp, dp, dp]
        _lib.orc_lps_force.argtypes = [gp, C.c_double, C.c_double, dp, dp, dp, dp]
        _lib.orc_damage_index.argtypes = [gp, up, up, dp, C.POINTER(C.c_int32)]
        _lib.orc_verlet.argtypes = [gp, mp, up, up, up, dp, dp, dp, dp, dp, dp, dp,
                                    C.c_double, C.c_int, C.c_int, dp]
        _lib.orc_bond_sc.argtypes = [C.c_int, C.c_int, C.c_double, C.c_double, C.c_double]
        _lib.orc_bond_sc.restype = C.c_double
        _lib.orc_bond_force.argtypes = [gp, C.c_double, up, up, dp, dp]
        _lib.orc_bond_break.argtypes = [gp, C.c_double, up, up, dp]
        _lib.orc_bond_break.restype = C.c_long
        _lib.orc_bond_damage.argtypes = [gp, up, up, dp]
        _lib.orc_bond_verlet.argtypes = [gp, C.c_double, C.c_double, C.c_double, up, up, up, dp, dp, dp,
                                         dp, dp, C.c_double, C.c_int, C.c_int]
        _lib.orc_bond_verlet.restype = C.c_long
        _lib.orc_static_cg.argtypes = [gp, mp, up, up, dp, dp, dp, C.c_double, C.c_int, dp]
        _lib.orc_static_cg.restype = C.c_int
        _lib.orc_bb_force_adjoint.argtypes = [gp, C.c_double, dp, dp, dp, dp, dp]
        _lib.orc_verlet_adjoint.argtypes = [gp, C.c_double, C.c_double, up, dp, dp, dp, dp,
                                            C.c_double, C.c_int, dp, dp, dp, dp]
    return _lib


def threads() -> int:
    """Host threads the oracle's parallel loops use."""
    return int(lib().orc_threads())


def _d(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def _u8(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_uint8))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _mask(a):
    return np.ascontiguousarray(a, dtype=np.uint8)


def geom(shape, dx, delta, periodic=False, influence=0) -> Geom:
    """Grid description.  ``shape`` is the box in (z, y, x) order for 3D or
    (y, x) for 2D, matching the component-major array layout."""
    dim = len(shape)
    g = Geom()
    g.dim = dim
    nb = list(reversed(shape)) + [1] * (3 - dim)
    for d in range(3):
        g.nb[d] = nb[d]
    dxs = list(dx) if np.ndim(dx) else [float(dx)] * dim
    dxs = dxs + [1.0] * (3 - dim)
    for d in range(3):
        g.dx[d] = dxs[d]
    g.delta = float(delta)
    g.periodic = int(bool(periodic))
    g.influence = int(influence)
    return g


def stencil(g: Geom) -> np.ndarray:
    """Bond offsets (ox, oy, oz) of the horizon, o != 0."""
    n = lib().orc_stencil(C.byref(g), None, 0)
    buf = (C.c_int * (3 * n))()
    lib().orc_stencil(C.byref(g), buf, n)
    return np.array(buf, dtype=np.int64).reshape(n, 3)


def bb_alpha(dim, E, delta, influence=0) -> float:
    return lib().orc_bb_alpha(dim, influence, E, delta)


def m0(g: Geom) -> float:
    return lib().orc_m0(C.byref(g))


def bb_force(g: Geom, alpha, phi, u):
    """Weighted linearized bond-based force density (Eq. 18/46/75/100)."""
    phi = _f64(phi)
    u = _f64(u)
    L = np.empty_like(u)
    lib().orc_bb_force(C.byref(g), alpha, _d(phi), _d(u), _d(L))
    return L


def nbb_force(g: Geom, alpha, phi, u):
    """Nonlinear rotation-invariant bond-based force density (Eq. 19-20),
    bond by bond, with bond weights phi."""
    phi = _f64(phi)
    u = _f64(u)
    L = np.empty_like(u)
    lib().orc_nbb_force(C.byref(g), alpha, _d(phi), _d(u), _d(L))
    return L


def bb_energy(g: Geom, alpha, phi, u):
    """Strain energy density, direct bond form of Eq. 42/47/102."""
    phi = _f64(phi)
    u = _f64(u)
    W = np.empty(phi.shape, dtype=np.float64)
    lib().orc_bb_energy(C.byref(g), alpha, _d(phi), _d(u), _d(W))
    return W


def lps_force(g: Geom, E, nu, chi, u):
    """Linearized LPS force density and dilatation with the EC mask
    (Eq. 33-36, 92-94).  Returns (L, theta)."""
    chi = _f64(chi)
    u = _f64(u)
    L = np.empty_like(u)
    th = np.empty(chi.shape, dtype=np.float64)
    lib().orc_lps_force(C.byref(g), E, nu, _d(chi), _d(u), _d(th), _d(L))
    return L, th


def damage_index(g: Geom, chiB, lam):
    """Damage index (Eq. 12/49) and the integer intact-partner count."""
    chiB = _mask(chiB)
    lam = _mask(lam)
    d = np.empty(chiB.shape, dtype=np.float64)
    cnt = np.empty(chiB.shape, dtype=np.int32)
    lib().orc_damage_index(C.byref(g), _u8(chiB), _u8(lam), _d(d),
                           cnt.ctypes.data_as(C.POINTER(C.c_int32)))
    return d, cnt


def model(kind, E=0.0, nu=0.25, alpha=0.0, rho=1.0, Wc=0.0) -> Model:
    m = Model()
    m.model = {"bb": 0, "lps": 1}[kind]
    m.E, m.nu, m.alpha, m.rho, m.Wc = E, nu, alpha, rho, Wc
    return m


def verlet(g: Geom, mdl: Model, chiB, chiO, u, v, dt, nsteps, b=None, w=None, lam=None,
           s=None, F=None, W=None, init=True, energy=False):
    """Embedded-constraint velocity Verlet (Eq. 67, 83-84) with optional
    pointwise energy damage (Eq. 40, 43, 63).  Returns a dict with the final
    state and, if asked, the per-step energies."""
    chiB = _mask(chiB)
    chiO = _mask(chiO)
    u = _f64(u).copy()
    v = _f64(v).copy()
    F = np.zeros_like(u) if F is None else _f64(F).copy()
    W = np.zeros(chiB.shape, dtype=np.float64) if W is None else _f64(W).copy()
    lam = None if lam is None else _mask(lam).copy()
    s = None if s is None else _f64(s)
    b = None if b is None else _f64(b)
    w = None if w is None else _f64(w)
    en = np.zeros((nsteps, 4), dtype=np.float64) if energy else None
    lib().orc_verlet(C.byref(g), C.byref(mdl), _u8(chiB), _u8(chiO), _u8(lam), _d(s), _d(u),
                     _d(v), _d(F), _d(W), _d(b), _d(w), dt, nsteps, int(bool(init)), _d(en))
    out = {"u": u, "v": v, "F": F, "W": W, "lam": lam}
    if energy:
        out["energy"] = en
    return out


def static_cg(g: Geom, mdl: Model, chiB, chiO, b, w=None, u0=None, rtol=1e-10, maxit=100000):
    """Embedded-constraint statics by plain FP64 CG (Eq. 89).  Returns
    (u, iterations, relative residual)."""
    chiB = _mask(chiB)
    chiO = _mask(chiO)
    b = _f64(b)
    u = np.zeros_like(b) if u0 is None else _f64(u0).copy()
    w = None if w is None else _f64(w)
    rr = C.c_double(0)
    it = lib().orc_static_cg(C.byref(g), C.byref(mdl), _u8(chiB), _u8(chiO), _d(b), _d(w), _d(u),
                             rtol, maxit, C.byref(rr))
    return u, it, rr.value


def bb_force_adjoint(g: Geom, alpha, phi, u, gbar):
    """Cotangents of <gbar, L_phi(u)> with respect to u and phi."""
    phi = _f64(phi)
    u = _f64(u)
    gbar = _f64(gbar)
    ub = np.empty_like(u)
    pb = np.empty(phi.shape, dtype=np.float64)
    lib().orc_bb_force_adjoint(C.byref(g), alpha, _d(phi), _d(u), _d(gbar), _d(ub), _d(pb))
    return ub, pb


def verlet_adjoint(g: Geom, alpha, rho, chiO, phi, b, u0, v0, dt, nsteps, ubarT, vbarT, want_bbar=False):
    """Reverse sweep of the fixed-weight EC Verlet rollout.  Returns
    (ubar0, vbar0, phibar), and bbar (the cotangent of the body force) as a
    fourth value when want_bbar is set."""
    chiO = _mask(chiO)
    phi = _f64(phi)
    b = _f64(b)
    u0 = _f64(u0)
    v0 = _f64(v0)
    ub = _f64(ubarT).copy()
    vb = _f64(vbarT).copy()
    pb = np.zeros(phi.shape, dtype=np.float64)
    bb = np.zeros_like(ub) if want_bbar else None
    lib().orc_verlet_adjoint(C.byref(g), alpha, rho, _u8(chiO), _d(phi), _d(b), _d(u0), _d(v0),
                             dt, nsteps, _d(ub), _d(vb), _d(pb), _d(bb))
    return (ub, vb, pb, bb) if want_bbar else (ub, vb, pb)


# --------------------------------------------------------------------------
# Comparator only: the critical bond-strain rule (Sec. 2, Eq. 10-12), which
# has no convolution structure.  ``mu`` is a uint8 array of shape
# (nodes, len(stencil(g))), one intact flag per bond, node-major.

def bond_sc(dim, alpha, G0, delta, influence=0) -> float:
    """Critical stretch calibrated to the fracture energy G0 (planar-crack
    energy balance of the linearized bond energy)."""
    return lib().orc_bond_sc(dim, influence, alpha, G0, delta)


def bond_mu(g: Geom):
    """All bonds intact."""
    n = 1
    for d in range(3):
        n *= g.nb[d]
    return np.ones((n, len(stencil(g))), dtype=np.uint8)


def bond_force(g: Geom, alpha, chiB, mu, u):
    """Linearized bond-based force with per-bond intact flags (Eq. 10, 18)."""
    u = _f64(u)
    chiB = _mask(chiB)
    mu = _mask(mu)
    L = np.empty_like(u)
    lib().orc_bond_force(C.byref(g), alpha, _u8(chiB), _u8(mu), _d(u), _d(L))
    return L


def bond_break(g: Geom, s_c, chiB, mu, u) -> int:
    """Clear, in place, the flags of bonds stretched beyond s_c."""
    assert mu.dtype == np.uint8 and mu.flags.c_contiguous
    chiB = _mask(chiB)
    u = _f64(u)
    return lib().orc_bond_break(C.byref(g), s_c, _u8(chiB), _u8(mu), _d(u))


def bond_damage(g: Geom, chiB, mu):
    """Damage index of Eq. 12 from per-bond flags."""
    chiB = _mask(chiB)
    mu = _mask(mu)
    d = np.empty(chiB.shape, dtype=np.float64)
    lib().orc_bond_damage(C.byref(g), _u8(chiB), _u8(mu), _d(d))
    return d


def bond_verlet(g: Geom, alpha, rho, s_c, chiB, chiO, mu, u, v, dt, nsteps, b=None, w=None, F=None,
                init=True):
    """EC velocity Verlet under the critical bond-strain rule.  ``mu`` is
    updated in place; returns (state dict, number of flags cleared)."""
    assert mu.dtype == np.uint8 and mu.flags.c_contiguous
    chiB = _mask(chiB)
    chiO = _mask(chiO)
    u = _f64(u).copy()
    v = _f64(v).copy()
    F = np.zeros_like(u) if F is None else _f64(F).copy()
    b = None if b is None else _f64(b)
    w = None if w is None else _f64(w)
    nbk = lib().orc_bond_verlet(C.byref(g), alpha, rho, s_c, _u8(chiB), _u8(chiO), _u8(mu), _d(u), _d(v),
                                _d(F), _d(b), _d(w), dt, nsteps, int(bool(init)))
    return {"u": u, "v": v, "F": F, "mu": mu}, nbk
