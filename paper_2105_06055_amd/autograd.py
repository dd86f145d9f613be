"""torch.autograd wrappers over the C ABI (differentiation of the FCBM-EC path).

``PDForce``      L = pd_force(u; s) with backward = pd_force_adjoint
                 (cotangents for u and, for micromodulus-scale plans, for s).
``VerletRollout`` nsteps embedded-constraint velocity-Verlet steps from
                 (u0, v0) with checkpoints every ``checkpoint_every`` steps;
                 the backward pass recomputes each segment from its
                 checkpoint and sweeps it in reverse with pd_verlet_adjoint,
                 giving cotangents for u0, v0, the micromodulus scale s and
                 the body force b.  A checkpoint holds (u, v, F), so the
                 recomputation resumes with the force the forward pass
                 carried and repeats the forward states bit for bit.

Both forward and backward run entirely in the library's kernels; PyTorch only
provides the tensors and the autograd bookkeeping.  The adjoint assumes fixed
weights, a time-independent body force and w = 0 on constrained components
(the setting of pd_verlet_adjoint).
"""
from __future__ import annotations

import torch


class PDForce(torch.autograd.Function):
    @staticmethod
    def forward(ctx, plan, u, s=None):
        u = u.contiguous()
        L = plan.force(u, weight=s)
        ctx.plan = plan
        ctx.save_for_backward(u, s if s is not None else torch.empty(0, device=u.device))
        ctx.has_s = s is not None
        return L

    @staticmethod
    def backward(ctx, gL):
        u, s = ctx.saved_tensors
        s = s if ctx.has_s else None
        plan = ctx.plan
        gL = gL.contiguous()
        if ctx.has_s and ctx.needs_input_grad[2]:
            ub, sb = plan.force_adjoint(u, gL, weight=s, want_weight_bar=True)
        else:
            ub, sb = plan.force_adjoint(u, gL, weight=s), None
        return None, ub, sb


class VerletRollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, plan, u0, v0, s, dt, nsteps, checkpoint_every=20, b=None):
        dev, dt_ = u0.device, float(dt)
        st = {"u": u0.detach().clone().contiguous(), "v": v0.detach().clone().contiguous(),
              "F": torch.zeros_like(u0), "step": 0}
        if s is not None:
            st["s"] = s.detach().contiguous()
        b = None if b is None else b.detach().contiguous()
        ckpts = [(st["u"].clone(), st["v"].clone(), None)]
        k = max(1, int(checkpoint_every))
        # one library call per segment, its steps exactly those of the
        # backward pass's one-step recompute (no regrouping around the
        # half-step velocity), so the two trajectories agree bit for bit
        for k0 in range(0, nsteps, k):
            plan.verlet(st, dt_, min(k, nsteps - k0), b=b, exact_steps=True)
            if k0 + k < nsteps:
                ckpts.append((st["u"].clone(), st["v"].clone(), st["F"].clone()))
        ctx.plan, ctx.dt, ctx.nsteps, ctx.k, ctx.b = plan, dt_, nsteps, k, b
        ctx.ckpts = ckpts
        ctx.s = st.get("s")
        return st["u"].clone(), st["v"].clone()

    @staticmethod
    def backward(ctx, ubT, vbT):
        plan, dt, nsteps, k, b = ctx.plan, ctx.dt, ctx.nsteps, ctx.k, ctx.b
        ref = ctx.ckpts[0][0]
        ub = torch.zeros_like(ref) if ubT is None else ubT.detach().clone().contiguous()
        vb = torch.zeros_like(ref) if vbT is None else vbT.detach().clone().contiguous()
        s = ctx.s
        sb = torch.zeros_like(s) if s is not None else None
        bb = torch.zeros_like(b) if (b is not None and ctx.needs_input_grad[7]) else None
        nseg = len(ctx.ckpts)
        for seg in range(nseg - 1, -1, -1):
            k0 = seg * k
            length = min(k, nsteps - k0)
            u_c, v_c, F_c = ctx.ckpts[seg]
            # from the first checkpoint the call forms F itself (step 0), as
            # the forward pass did; later ones resume with the stored F
            st = {"u": u_c.clone(), "v": v_c.clone(),
                  "F": torch.zeros_like(u_c) if F_c is None else F_c.clone(),
                  "step": 0 if F_c is None else k0}
            if s is not None:
                st["s"] = s
            us = [st["u"].clone()]
            for _ in range(length):
                plan.verlet(st, dt, 1, b=b)
                us.append(st["u"].clone())
            for i in range(length - 1, -1, -1):
                plan.verlet_adjoint(us[i], us[i + 1], ub, vb, dt, s=s, s_bar=sb, b_bar=bb)
        return None, ub, vb, sb, None, None, None, bb
