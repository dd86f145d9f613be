#!/usr/bin/env python3
"""Benchmark of the FCBM-EC peridynamic hot path on one MI355X.

Workload (default): 3D linearized state-based (LPS) block with 8 seeded
ellipsoidal voids, 256^3 body nodes on a 512^3 FFT grid, delta = 3 dx,
E = 70 GPa, nu = 0.25, FP32, seeded impulsive velocity on the x = 0 face.
A "step" is one embedded-constraint velocity-Verlet step: position update,
the two-stage LPS force (dilatation convolution, then force convolutions;
forward real FFTs, spectral multiply, inverse FFTs, assembly) and the
velocity update.  value = body nodes x steps / time (Gnode/s).

Also reported: the same step in FP64 and in FP32 with transforms along all
three axes (the last axis otherwise uses the equivalent direct line
correlation), pd_force alone, per-pass HIP-event timings over the timed
steps with algorithmic bytes (roofline of the dominant pass; its HBM traffic
from the committed rocprofv3 counter summary when the sources match), the
elastostatic CG time to a 1e-10 relative residual on the 128^3-node /
256^3-grid static cube (plain FP64 vs mixed FP32-operator / FP64 CG), and
the FP64 direct-summation oracle timed on host cores on a bounded slab of
the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "PD force evals/s (Gnode/s) at 256³ FP32 vs FP64; % HBM roofline; CG time-to-1e-10"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


class ProfileSession:
    """Per-launch HIP-event timing of a plan (pd_profile_enable / read)."""

    def __init__(self, plan):
        import ctypes as C

        from paper_2105_06055_amd import binding

        class PassTime(C.Structure):
            _fields_ = [("name", C.c_char * 32), ("launches", C.c_int64), ("total_ms", C.c_double),
                        ("bytes", C.c_double)]

        self.C, self.PassTime, self.plan = C, PassTime, plan
        self.L = binding.lib()
        self.L.pd_profile_enable.argtypes = [C.c_void_p, C.c_int]
        self.L.pd_profile_read.argtypes = [C.c_void_p, C.POINTER(PassTime), C.c_int, C.POINTER(C.c_int)]
        assert self.L.pd_profile_enable(plan._h, 1) == 0

    def read(self):
        C = self.C
        buf = (self.PassTime * 64)()
        n = C.c_int(0)
        assert self.L.pd_profile_read(self.plan._h, buf, 64, C.byref(n)) == 0
        self.L.pd_profile_enable(self.plan._h, 0)
        out = []
        for i in range(min(n.value, 64)):
            r = buf[i]
            out.append({"name": r.name.decode(), "launches": int(r.launches), "total_ms": r.total_ms,
                        "avg_ms": r.total_ms / max(1, r.launches),
                        "bytes_per_launch": r.bytes / max(1, r.launches),
                        "GBps": (r.bytes / 1e9) / (r.total_ms / 1e3) if r.total_ms > 0 else 0.0})
        return out


def pass_roofline(passes, steps):
    """Dominant pass (largest summed duration) of a profiled run: its
    algorithmic bytes per launch over its average event-measured duration,
    and the whole step's algorithmic bytes over the summed pass time."""
    dom = max(passes, key=lambda p: p["total_ms"])
    achieved = dom["bytes_per_launch"] / 1e9 / (dom["avg_ms"] / 1e3)
    step_bytes = sum(p["bytes_per_launch"] * p["launches"] for p in passes) / steps
    step_ms = sum(p["total_ms"] for p in passes) / steps
    return {"bound": "hbm", "kernel": dom["name"], "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "kernel_avg_ms": dom["avg_ms"], "kernel_bytes": dom["bytes_per_launch"],
            "step_alg_bytes": step_bytes, "step_kernel_ms": step_ms,
            "step_alg_GBps": step_bytes / 1e9 / (step_ms / 1e3)}


def run_m_crossover(nb, nfft, reps, warmup, ms=(2, 3, 4, 6)):
    """pd_force (FP32 LPS, the voided block) at horizons of m = delta/dx
    spacings, on each path the plan offers: the default (the direct (y, z)
    correlation for m <= 3, else the y transform), the y transform with the
    direct z line correlation (transform form beyond 4 spacings) and
    transforms along all three axes."""
    import torch

    from paper_2105_06055_amd import binding, workloads
    rows = []
    for m in ms:
        w = workloads.block_voids_dynamics(nb=nb, nfft=nfft, m=m)
        plan = binding.Plan.from_workload(w, dtype=torch.float32)
        u = torch.tensor(np.random.default_rng(7).normal(0.0, 1e-6, size=(3,) + w.body), dtype=torch.float32,
                         device="cuda")
        L = torch.empty_like(u)
        row = {"m": m, "bonds": plan.info["stencil_size"]}
        for mode in ("auto", "yfft", "fft"):
            plan.set_lastaxis(mode)
            for _ in range(max(1, warmup)):
                plan.force(u, out=L)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                plan.force(u, out=L)
            torch.cuda.synchronize()
            row[f"{mode}_force_ms"] = (time.perf_counter() - t0) / reps * 1e3
        plan.close()
        del u, L
        torch.cuda.empty_cache()
        rows.append(row)
        log(f"[bench] m-crossover {row}")
    return rows


def kernel_source_hash():
    """Hash of the HIP sources: HBM counter results taken for other sources
    are not reported."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2105_06055_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".hpp")):
            with open(os.path.join(d, f), "rb") as fh:
                h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()


def measured_traffic(pass_name, path="auto"):
    """HBM bytes per launch of a pass of the 256^3 FP32 step on a force path
    ("auto" or "fft") from the committed rocprofv3 counter summary
    (FETCH_SIZE, WRITE_SIZE, scaled by the 1 GiB copy calibration), or None
    if there is none for these sources."""
    name = {"auto": "hbm_traffic_lps256_fp32_step.json", "fft": "hbm_traffic_lps256_fp32_step_allaxes.json"}.get(path)
    if name is None:
        return None
    p = os.path.join(ROOT, "profiles", name)
    try:
        with open(p) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("source_sha256") != kernel_source_hash():
        return None
    k = t.get("passes", {}).get(pass_name)
    return None if k is None else float(k["hbm_bytes_per_launch"])


def run_dynamics(wl, dtype, steps, warmup, with_profile, lastaxis="auto"):
    """Warm up, then time exactly `steps` Verlet steps (one library call)
    between two device synchronisations, with no instrumentation; then, if
    with_profile, run `steps` more steps with a HIP event pair recorded
    around every launch (on the launch stream) for the per-pass timings.
    Plan creation is timed on its own."""
    import torch

    from paper_2105_06055_amd import binding
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = binding.Plan.from_workload(wl, dtype=dtype)
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t0
    if lastaxis != "auto":
        plan.set_lastaxis(lastaxis)
    dev = lambda a: torch.tensor(a, dtype=dtype, device="cuda").contiguous()
    st = {"u": dev(wl.u0), "v": dev(wl.v0), "F": torch.zeros((wl.dim,) + wl.body, dtype=dtype, device="cuda"),
          "step": 0}
    dt = wl.dt
    plan.verlet(st, dt, max(1, warmup))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.verlet(st, dt, steps)
    torch.cuda.synchronize()
    t_step = (time.perf_counter() - t0) / steps
    prof = None
    if with_profile:
        prof = ProfileSession(plan)
        plan.verlet(st, dt, steps)
        torch.cuda.synchronize()
        prof = prof.read()
    # pd_force alone
    L = torch.empty_like(st["u"])
    for _ in range(2):
        plan.force(st["u"], out=L)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.force(st["u"], out=L)
    torch.cuda.synchronize()
    t_force = (time.perf_counter() - t0) / steps
    finite = bool(torch.isfinite(st["u"]).all().item())
    info = plan.info
    plan.close()
    del st, L
    torch.cuda.empty_cache()
    return {"s_per_step": t_step, "s_per_force": t_force, "passes": prof, "finite": finite,
            "workspace_GB": info["workspace_bytes"] / 1e9, "lds_per_block": info["lds_per_block"],
            "plan_create_s": t_plan}


def run_fracture(steps, warmup, chunk=1000):
    """The notched glass plate (1000 x 400 nodes, delta = 4 dx, 512 x 1024
    grid, +-12 MPa edge tractions) with the pointwise energy damage, from
    rest: `steps` Verlet steps (the configuration's 10,000) in FP32 and, side
    by side, in FP64, issued in library calls of `chunk` steps (after `warmup`
    steps on a scratch state).  Reports the time per step, node-steps/s, the
    failed nodes and, after every chunk, how many nodes the FP32 and FP64
    integrity maps differ in."""
    import torch

    from paper_2105_06055_amd import binding, workloads
    w = workloads.notched_plate_fracture()
    out = {"workload": "notched plate 1000x400 nodes, delta = 4 dx, 512x1024 grid, +-12 MPa, energy damage, "
                       "from rest", "steps": steps, "chunk": chunk}
    runs = {}
    for dn, dtype in (("fp32", torch.float32), ("fp64", torch.float64)):
        plan = binding.Plan.from_workload(w, dtype=dtype, weight="integrity")
        dev = lambda a, t=dtype: torch.tensor(np.ascontiguousarray(a), dtype=t, device="cuda")

        def fresh():
            return {"u": dev(w.u0), "v": dev(w.v0), "F": torch.zeros((2,) + w.body, dtype=dtype, device="cuda"),
                    "lam": dev(w.lam0, torch.uint8), "W": torch.zeros(w.body, dtype=dtype, device="cuda"),
                    "step": 0}
        b = dev(w.b)
        plan.verlet(fresh(), w.dt, warmup, b=b)
        runs[dn] = {"plan": plan, "st": fresh(), "b": b, "t": 0.0}
    diff = []
    done = 0
    while done < steps:
        n = min(chunk, steps - done)
        lam = {}
        for dn, r in runs.items():
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r["plan"].verlet(r["st"], w.dt, n, b=r["b"])
            torch.cuda.synchronize()
            r["t"] += time.perf_counter() - t0
            lam[dn] = r["st"]["lam"]
        done += n
        diff.append([done, int((lam["fp32"] != lam["fp64"]).sum().item())])
    for dn, r in runs.items():
        st = r["st"]
        t = r["t"] / steps
        out[dn] = {"ms_per_step": t * 1e3, "Gnode_steps_s": w.nodes / t / 1e9,
                   "failed_nodes": int((w.lam0.astype(int) - st["lam"].cpu().numpy().astype(int)).sum()),
                   "finite": bool(torch.isfinite(st["u"]).all().item())}
    # pass durations of 200 FP32 steps from a scratch state (a separate,
    # instrumented run): their sum per step against the uninstrumented time
    # per step shows the gaps between launches
    r = runs["fp32"]
    prof = ProfileSession(r["plan"])
    st = {k: (v.clone() if hasattr(v, "clone") else v) for k, v in r["st"].items()}
    r["plan"].verlet(st, w.dt, 200, b=r["b"])
    torch.cuda.synchronize()
    passes = prof.read()
    out["fp32"]["passes"] = passes
    out["fp32"]["kernel_ms_per_step"] = sum(p["total_ms"] for p in passes) / 200
    del st
    d32 = runs["fp32"]["plan"].damage_index(runs["fp32"]["st"]["lam"]).double()
    d64 = runs["fp64"]["plan"].damage_index(runs["fp64"]["st"]["lam"])
    out["fp32_vs_fp64"] = {"integrity_nodes_differing_after_steps": diff,
                           "damage_nodes_differing": int((d32 != d64).sum().item()),
                           "damage_mean_fp32": float(d32.mean().item()), "damage_mean_fp64": float(d64.mean().item())}
    for r in runs.values():
        r["plan"].close()
    out["ms_per_step"] = out["fp32"]["ms_per_step"]
    return out


def run_adjoint_plate(dtype_name):
    """The heterogeneous-micromodulus plate (512 x 512 nodes, 1024 x 1024
    grid, 200 Verlet steps, checkpoints every 20): time one forward rollout
    plus the checkpointed adjoint for dL/du0 and dL/ds, after one untimed
    pass."""
    import torch

    from paper_2105_06055_amd import binding, workloads
    from paper_2105_06055_amd.autograd import VerletRollout
    dtype = {"fp32": torch.float32, "fp64": torch.float64}[dtype_name]
    w = workloads.hetero_plate_adjoint()
    plan = binding.Plan.from_workload(w, dtype=dtype)
    dev = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")
    target = dev(w.extra["u_target"])

    def once():
        u0 = dev(w.u0).requires_grad_(True)
        s = dev(w.s).requires_grad_(True)
        uT, _ = VerletRollout.apply(plan, u0, dev(w.v0), s, w.dt, w.steps, 20)
        ((uT - target) ** 2).sum().backward()
        return u0.grad, s.grad

    once()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gu, gs = once()
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    finite = bool(torch.isfinite(gu).all().item() and torch.isfinite(gs).all().item())
    plan.close()
    return {"seconds": t, "ms_per_step_fwd_plus_adj": t / w.steps * 1e3, "finite": finite}


def run_cg(nb, nfft, maxit):
    import torch

    from paper_2105_06055_amd import binding, workloads
    wl = workloads.cube_void_static(nb=nb, nfft=nfft)
    plan = binding.Plan.from_workload(wl, dtype=torch.float64, mixed=True)
    b = torch.tensor(wl.b, dtype=torch.float64, device="cuda").contiguous()
    res = {}
    u_plain = None
    for precond in (False, True):
        for mixed in (False, True):
            # one untimed solve with a loose tolerance warms caches and code paths
            plan.static_solve(b, rtol=1e-2, maxit=maxit, mixed=mixed, precond=precond, check=False)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            u, info = plan.static_solve(b, rtol=1e-10, maxit=maxit, mixed=mixed, precond=precond, check=False)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            key = ("mixed_fp32_fp64" if mixed else "fp64") + ("_precond" if precond else "")
            res[key] = {"seconds": dt, "rel_res": info["rel_res"], "status": info["status"],
                        "iters_fp64": info["iters_fp64"], "iters_fp32": info["iters_fp32"],
                        "applies_fp64": info["applies_fp64"], "applies_fp32": info["applies_fp32"],
                        "precond_applies": info["precond_applies"]}
            if u_plain is None:
                u_plain = u
            else:
                res[key]["solution_rel_diff_vs_fp64_cg"] = float(torch.linalg.vector_norm(u - u_plain) /
                                                                 torch.linalg.vector_norm(u_plain))
    plan.close()
    torch.cuda.empty_cache()
    res["workload"] = f"LPS cube {nb}^3 nodes with spherical void, {nfft}^3 FFT grid, clamped 3-delta layer"
    return res


def run_force_rate(wl, dtype, reps, warmup):
    """pd_force alone: mean time over `reps` calls after `warmup`."""
    import torch

    from paper_2105_06055_amd import binding
    plan = binding.Plan.from_workload(wl, dtype=dtype)
    u = torch.tensor(np.random.default_rng(7).normal(0.0, 1e-6, size=(wl.dim,) + wl.body), dtype=dtype,
                     device="cuda")
    L = torch.empty_like(u)
    for _ in range(max(1, warmup)):
        plan.force(u, out=L)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        plan.force(u, out=L)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / reps
    plan.close()
    del u, L
    torch.cuda.empty_cache()
    return t


def run_plate_force_rate(model, dtype, reps, warmup, nb=512, nfft=1024, dim=2):
    """pd_force alone on the 2D plate (nb^2 body with holes on an nfft^2 grid)
    or the 3D block (nb^3 on nfft^3), delta = 3 dx: mean time over `reps`
    calls.  The displacement is a seeded field of amplitude 0.1 dx, so the
    nonlinear model's higher-order terms are well inside its range."""
    import torch

    from paper_2105_06055_amd import binding
    from paper_2105_06055_amd import workloads
    dx = 1e-3
    body = (nb,) * dim
    chi = workloads.random_mask(body, 44)
    plan = binding.Plan((nfft,) * dim, body, dx, 3 * dx, model=model, E=72e9, rho=2440.0, chiB=chi, dtype=dtype)
    u = torch.tensor(workloads.random_field((dim,) + body, 45, 0.1 * dx), dtype=dtype, device="cuda")
    L = torch.empty_like(u)
    for _ in range(max(1, warmup)):
        plan.force(u, out=L)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        plan.force(u, out=L)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / reps
    prof = ProfileSession(plan)
    plan.force(u, out=L)
    torch.cuda.synchronize()
    passes = prof.read()
    plan.close()
    del u, L
    torch.cuda.empty_cache()
    return t, passes


def run_energy(wl, dtype, nsteps):
    """nsteps EC Verlet steps from the workload's initial state with FP64
    energy accounting every step; returns the energy histories."""
    import torch

    from paper_2105_06055_amd import binding
    plan = binding.Plan.from_workload(wl, dtype=dtype)
    dev = lambda a: torch.tensor(a, dtype=dtype, device="cuda").contiguous()
    st = {"u": dev(wl.u0), "v": dev(wl.v0), "F": torch.zeros((wl.dim,) + wl.body, dtype=dtype, device="cuda"),
          "step": 0}
    t0 = time.perf_counter()
    en = plan.verlet(st, wl.dt, nsteps, energy=True)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    plan.close()
    del st
    torch.cuda.empty_cache()
    return en, t


def energy_report(wl, nsteps):
    """C5: energy drift of FP32 and FP64 runs of nsteps steps (E = KE + PE +
    EXT, and the Verlet shadow energy), and the FP32 run against FP64."""
    import torch
    out = {"steps": nsteps}
    hist = {}
    for name, dt_ in (("fp32", torch.float32), ("fp64", torch.float64)):
        en, t = run_energy(wl, dt_, nsteps)
        E = en[:, 0] + en[:, 1] + en[:, 2]
        hist[name] = (E, en[:, 3])
        out[name] = {"E0_J": float(E[0]), "E_end_J": float(E[-1]),
                     "drift_rel": float((E[-1] - E[0]) / E[0]),
                     "max_abs_drift_rel": float(np.max(np.abs(E - E[0])) / abs(E[0])),
                     "shadow_drift_rel": float((en[-1, 3] - en[0, 3]) / en[0, 3]),
                     "seconds": t}
    E32, E64 = hist["fp32"][0], hist["fp64"][0]
    out["fp32_vs_fp64_max_rel"] = float(np.max(np.abs(E32 - E64)) / abs(E64[0]))
    return out


def cpu_baseline(wl, budget_s=10.0):
    """FP64 direct-summation oracle, one EC Verlet step (one LPS force) on a
    z-slab of the same workload, slab sized for ~budget_s seconds."""
    import numpy as np

    from oracle import oracle as orc
    orc.build()
    nb = wl.body

    def step(nz):
        sl = slice(0, nz)
        g = orc.geom((nz,) + nb[1:], wl.dx, wl.delta)
        mdl = orc.model("lps", E=wl.E, nu=wl.nu, rho=wl.rho)
        chi = wl.chiB[sl]
        t0 = time.perf_counter()
        orc.verlet(g, mdl, chi, np.stack([chi] * 3), wl.u0[:, sl], wl.v0[:, sl], wl.dt, 1,
                   F=np.zeros((3, nz) + nb[1:]), init=False)
        return time.perf_counter() - t0

    nz = 4
    t = step(nz)
    nz = int(min(nb[0], max(4, nz * budget_s / max(t, 1e-3))))
    t = step(nz)
    nodes = nz * nb[1] * nb[2]
    threads = orc.threads()
    return {"value": nodes / t / 1e9, "unit": "Gnode/s", "cores": threads, "kind": "oracle",
            "sample": f"one EC velocity-Verlet step (one LPS direct-sum force, FP64) on a {nz}x{nb[1]}x{nb[2]} "
                      f"z-slab of the 256^3 block-with-voids workload ({nodes} nodes, {t:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--size", type=int, default=256, help="body nodes per edge")
    ap.add_argument("--fft", type=int, default=512, help="FFT grid per edge")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cg", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-nbb", action="store_true", help="skip the 2D nonlinear bond-based force rate")
    ap.add_argument("--no-mconv", action="store_true", help="skip the m-convergence table")
    ap.add_argument("--no-fracture", action="store_true", help="skip the fracture-plate step timing")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the forward + adjoint plate timing")
    ap.add_argument("--fracture-steps", type=int, default=10000)
    ap.add_argument("--no-fft-variant", action="store_true",
                    help="skip the step timing with FFTs along all three axes")
    ap.add_argument("--no-energy", action="store_true", help="skip the 1000-step energy-drift runs")
    ap.add_argument("--no-c2", action="store_true", help="skip the 128^3/256^3 force rates")
    ap.add_argument("--energy-steps", type=int, default=1000)
    ap.add_argument("--no-mcross", action="store_true", help="skip the horizon (m) crossover of the force paths")
    ap.add_argument("--no-minpad", action="store_true", help="skip the minimum-padding (mixed-radix) x grids")
    ap.add_argument("--no-refine", action="store_true", help="skip the static and fracture refinement studies")
    ap.add_argument("--cg-size", type=int, default=128)
    ap.add_argument("--cg-fft", type=int, default=256)
    ap.add_argument("--lastaxis", choices=("auto", "yfft", "fft"), default="auto",
                    help="force path of the headline step (for profiling the transform paths on their own): "
                         "auto = the (y, z) correlation pass, yfft = y transform + direct z line correlation, "
                         "fft = transforms on all three axes")
    ap.add_argument("--copy-calib", action="store_true",
                    help="run one 1 GiB device copy first (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the library runs on one GPU; the multi-GPU (slab + halo) path is a design "
              "only, so --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2105_06055_amd import workloads
    torch.cuda.set_device(0)
    if args.copy_calib:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("[bench] calibration copy: 1 GiB read + 1 GiB written")
        del src, dst
        torch.cuda.empty_cache()
    log(f"[bench] workload: LPS {args.size}^3 nodes in {args.fft}^3 FFT grid")
    wl = workloads.block_voids_dynamics(nb=args.size, nfft=args.fft)
    nodes = wl.nodes
    r32 = run_dynamics(wl, torch.float32, args.steps, args.warmup, with_profile=True, lastaxis=args.lastaxis)
    log(f"[bench] fp32 step {r32['s_per_step'] * 1e3:.3f} ms, force {r32['s_per_force'] * 1e3:.3f} ms"
        + ("" if args.lastaxis == "auto" else f" (path {args.lastaxis})"))
    r64 = None
    if not args.no_fp64:
        r64 = run_dynamics(wl, torch.float64, args.steps, args.warmup, with_profile=True)
        log(f"[bench] fp64 step {r64['s_per_step'] * 1e3:.3f} ms, force {r64['s_per_force'] * 1e3:.3f} ms")
    r32f = r32y = None
    if not args.no_fft_variant:
        # the same step with the y transform and the direct line correlation
        # along z, and with transforms on all three axes
        r32y = run_dynamics(wl, torch.float32, args.steps, args.warmup, with_profile=True, lastaxis="yfft")
        log(f"[bench] fp32 step, y transform + direct z: {r32y['s_per_step'] * 1e3:.3f} ms")
        r32f = run_dynamics(wl, torch.float32, args.steps, args.warmup, with_profile=True, lastaxis="fft")
        log(f"[bench] fp32 step, FFT on all three axes: {r32f['s_per_step'] * 1e3:.3f} ms")
    passes = r32["passes"]
    roof = pass_roofline(passes, args.steps)
    dom = {"name": roof["kernel"], "avg_ms": roof["kernel_avg_ms"], "bytes_per_launch": roof["kernel_bytes"]}
    achieved = roof["achieved"]
    step_bytes, step_kernel_ms = roof["step_alg_bytes"], roof["step_kernel_ms"]
    minpad = None
    if not args.no_minpad:
        # minimum-padding x grids (one horizon is all Sec. 4.2.2 needs): the
        # same step with n1 = 384 = 2*3*2^6, 320 = 2*5*2^5, 288 = 2*9*2^4
        import dataclasses
        rows = [{"n1": args.fft, "ms_per_step": r32["s_per_step"] * 1e3,
                 "Gnode_s": nodes / r32["s_per_step"] / 1e9, "force_ms": r32["s_per_force"] * 1e3,
                 "step_alg_bytes": roof["step_alg_bytes"], "roofline": roof}]
        for n1 in (384, 320, 288):
            wm = dataclasses.replace(wl, fft=(args.fft, args.fft, n1))
            rm = run_dynamics(wm, torch.float32, args.steps, args.warmup, with_profile=True)
            rf = pass_roofline(rm["passes"], args.steps)
            rows.append({"n1": n1, "ms_per_step": rm["s_per_step"] * 1e3, "Gnode_s": nodes / rm["s_per_step"] / 1e9,
                         "force_ms": rm["s_per_force"] * 1e3, "step_alg_bytes": rf["step_alg_bytes"],
                         "finite": rm["finite"], "roofline": rf, "passes": rm["passes"]})
            log(f"[bench] min-padding n1={n1}: step {rm['s_per_step'] * 1e3:.3f} ms")
        minpad = {"workload": f"FP32 LPS EC Verlet step, {args.size}^3 voided block, x grid n1 (y, z grids "
                              f"{args.fft}; the (y, z) pass works on the body planes only)", "rows": rows}
    mcross = None
    if not args.no_mcross:
        mcross = {"workload": f"FP32 LPS pd_force, {args.size}^3 voided block on {args.fft}^3, delta = m dx",
                  "rows": run_m_crossover(args.size, args.fft, args.steps, args.warmup)}
    c2 = None
    if not args.no_c2:
        w2 = workloads.cube_void_static()
        t32 = run_force_rate(w2, torch.float32, args.steps, args.warmup)
        t64 = run_force_rate(w2, torch.float64, args.steps, args.warmup)
        c2 = {"workload": "LPS cube 128^3 nodes with spherical void, 256^3 FFT grid (pd_force alone)",
              "fp32_force_ms": t32 * 1e3, "fp32_Gnode_s": w2.nodes / t32 / 1e9,
              "fp32_fft_grid_Gpoint_s": 256 ** 3 / t32 / 1e9,
              "fp64_force_ms": t64 * 1e3, "fp64_Gnode_s": w2.nodes / t64 / 1e9,
              "fp64_fft_grid_Gpoint_s": 256 ** 3 / t64 / 1e9}
        log(f"[bench] c2 {json.dumps(c2)}")
    nbb = None
    if not args.no_nbb:
        nbb = {"workload": "2D plate 512^2 nodes with holes on a 1024^2 FFT grid and 3D block 128^3 nodes "
                           "with holes on a 256^3 grid, delta = 3 dx, displacement amplitude 0.1 dx "
                           "(pd_force alone)"}
        for model, tag in (("nbb", "nonlinear"), ("bb", "linear")):
            for dt, dn in ((torch.float32, "fp32"), (torch.float64, "fp64")):
                t, ps = run_plate_force_rate(model, dt, args.steps, args.warmup)
                nbb[f"{tag}_{dn}_force_ms"] = t * 1e3
                nbb[f"{tag}_{dn}_Gnode_s"] = 512 * 512 / t / 1e9
                if model == "nbb":
                    nbb[f"{tag}_{dn}_passes"] = ps
                # the 3D block: 128^3 nodes with holes on the 256^3 grid
                t, ps = run_plate_force_rate(model, dt, args.steps, args.warmup, nb=128, nfft=256, dim=3)
                nbb[f"{tag}_3d128_{dn}_force_ms"] = t * 1e3
                nbb[f"{tag}_3d128_{dn}_Gnode_s"] = 128 ** 3 / t / 1e9
                if model == "nbb":
                    nbb[f"{tag}_3d128_{dn}_passes"] = ps
        log(f"[bench] nbb {json.dumps({k: v for k, v in nbb.items() if not k.endswith('passes')})}")
    mconv_tab = None
    if not args.no_mconv:
        from paper_2105_06055_amd import mconv
        mconv_tab = {"workload": "quadratic field, force at the centre of an interior block, fixed horizon "
                                 "delta = 3e-3 m, m = delta/dx; FP64; relative error vs the continuum Navier operator",
                     "rows": mconv.run()}
        log(f"[bench] m-convergence {json.dumps(mconv_tab['rows'])}")
    refine = None
    if not args.no_refine:
        from paper_2105_06055_amd import mconv
        refine = {"static_eq99": dict(mconv.static_refinement(),
                                      workload="LPS cube, edge 16 delta, delta = 3 mm, centred spherical void r = "
                                               "0.2 L, clamped z < 3 delta, uniform body force 1e8 N/m^3, E = 60 "
                                               "GPa, nu = 0.4; FP64 PCG to 1e-10; Eq. 99 on the coarse nodes"),
                  "fracture": dict(mconv.fracture_refinement(),
                                   workload="notched glass plate 10 x 4 cm, delta = 1 mm, sigma = 4 MPa, 50 us "
                                            "(dt 25 ns), FP32, energy failure rule")}
        log(f"[bench] refinement eq99 {json.dumps(refine['static_eq99']['eq99'])}")
    energy = None
    if not args.no_energy:
        log(f"[bench] energy drift over {args.energy_steps} steps (FP32 and FP64)")
        energy = energy_report(wl, args.energy_steps)
        log(f"[bench] energy {json.dumps(energy)}")
    adj = None
    if not args.no_adjoint:
        adj = {"workload": "heterogeneous plate 512x512 nodes, 1024x1024 grid, 200 Verlet steps, checkpoints "
                           "every 20; forward rollout + checkpointed adjoint (dL/du0, dL/ds)"}
        for dn in ("fp32", "fp64"):
            adj[dn] = run_adjoint_plate(dn)
        log(f"[bench] adjoint {json.dumps(adj)}")
    frac = None
    if not args.no_fracture:
        frac = run_fracture(args.fracture_steps, 20)
        log(f"[bench] fracture {json.dumps(frac)}")
    cg = None
    if not args.no_cg:
        log("[bench] CG time-to-1e-10 (static cube)")
        cg = run_cg(args.cg_size, args.cg_fft, maxit=20000)
        log(f"[bench] cg {json.dumps(cg)}")
    cpu = None
    if not args.no_cpu:
        log("[bench] CPU oracle baseline")
        cpu = cpu_baseline(wl)
        log(f"[bench] cpu {cpu}")
    out = {
        "metric": METRIC,
        "value": nodes / r32["s_per_step"] / 1e9,
        "unit": "Gnode/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["s_per_step"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"3D LPS EC velocity-Verlet step, {args.size}^3 body nodes (8 seeded ellipsoidal "
                               f"voids) on a {args.fft}^3 FFT grid, delta=3dx, E=70GPa, nu=0.25",
                   "body_nodes": nodes, "fft_grid": args.fft ** 3, "parallelism": "single GPU",
                   "path": {"auto": "x transform + (y, z) correlation", "yfft": "x, y transforms + z line correlation",
                            "fft": "transforms on all three axes"}[args.lastaxis]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(dom["name"], args.lastaxis),
                     "kernel": dom["name"], "kernel_avg_ms": dom["avg_ms"],
                     "kernel_bytes": dom["bytes_per_launch"]},
        "cpu_baseline": cpu,
        "detail": {
            "fp32": {"step_Gnode_s": nodes / r32["s_per_step"] / 1e9,
                     "force_Gnode_s": nodes / r32["s_per_force"] / 1e9,
                     "force_ms": r32["s_per_force"] * 1e3, "finite": r32["finite"],
                     "step_alg_bytes": step_bytes, "step_kernel_ms": step_kernel_ms,
                     "step_alg_GBps": step_bytes / 1e9 / (step_kernel_ms / 1e3),
                     "workspace_GB": r32["workspace_GB"], "lds_per_block": r32["lds_per_block"],
                     "plan_create_s": r32["plan_create_s"],
                     "passes": passes},
            "fp64": None if r64 is None else {
                "step_Gnode_s": nodes / r64["s_per_step"] / 1e9, "ms_per_step": r64["s_per_step"] * 1e3,
                "force_Gnode_s": nodes / r64["s_per_force"] / 1e9, "force_ms": r64["s_per_force"] * 1e3,
                "finite": r64["finite"], "passes": r64["passes"]},
            "fp32_yfft_zdirect": None if r32y is None else {
                "step_Gnode_s": nodes / r32y["s_per_step"] / 1e9, "ms_per_step": r32y["s_per_step"] * 1e3,
                "force_Gnode_s": nodes / r32y["s_per_force"] / 1e9, "force_ms": r32y["s_per_force"] * 1e3,
                "finite": r32y["finite"], "passes": r32y["passes"]},
            "fp32_fft_all_axes": None if r32f is None else {
                "step_Gnode_s": nodes / r32f["s_per_step"] / 1e9, "ms_per_step": r32f["s_per_step"] * 1e3,
                "force_Gnode_s": nodes / r32f["s_per_force"] / 1e9, "force_ms": r32f["s_per_force"] * 1e3,
                "finite": r32f["finite"],
                "roofline": dict(pass_roofline(r32f["passes"], args.steps),
                                 traffic=measured_traffic(pass_roofline(r32f["passes"], args.steps)["kernel"], "fft")),
                "passes": r32f["passes"]},
            "m_crossover": mcross,
            "min_padding_x": minpad,
            "cg_time_to_1e-10": cg,
            "c2_force": c2,
            "nonlinear_bb_plate_force": nbb,
            "m_convergence": mconv_tab,
            "refinement": refine,
            "fracture_plate": frac,
            "adjoint_plate": adj,
            "energy_drift": energy,
        },
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
