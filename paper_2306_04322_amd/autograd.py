"""torch.autograd.Function over an FS rollout, backed by the hand-written
discrete adjoint of libpfspec (pf_adjoint_fs).

Forward: copies u0 into the solver's fields, stores a checkpoint of the
fields every K steps and advances with pf_step_fs.  Backward: walks the
segments last to first; for each, pf_adjoint_fs recomputes the segment's
states from its checkpoint (same kernels, so bit-identical) and runs the
adjoint steps, turning dJ/du^end into dJ/du^start and accumulating
dJ/d(M, kappa_c, L, kappa_eta) in double precision.
"""

import numpy as np
import torch


class FSRollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u0, params, solver, dt, nsteps, K):
        p = [float(v) for v in params.detach().to("cpu", torch.float64).tolist()]
        solver.set_params(*p)
        solver.fields.copy_(u0.detach().reshape(solver.shape).to(solver.dtype))
        ckpts, lens = [], []
        done = 0
        while done < nsteps:
            k = min(K, nsteps - done)
            ckpts.append(solver.fields.clone())
            lens.append(k)
            solver.step_fs(dt, k)
            done += k
        ctx.solver = solver
        ctx.dt = dt
        ctx.params = p
        ctx.ckpts = ckpts
        ctx.lens = lens
        ctx.K = K
        ctx.u_dtype = u0.dtype
        ctx.p_dtype = params.dtype
        ctx.p_device = params.device
        return solver.fields.clone().to(u0.dtype)

    @staticmethod
    def backward(ctx, grad_out):
        s = ctx.solver
        s.set_params(*ctx.params)
        lam = grad_out.detach().reshape(s.shape).to(s.dtype).contiguous().clone()
        seg = s.segment_store(max(ctx.lens)) if ctx.lens else None
        dpar = np.zeros(4)
        for ck, k in zip(reversed(ctx.ckpts), reversed(ctx.lens)):
            dpar = s.adjoint_fs(ctx.dt, k, ck, lam, seg, dpar)
        gp = torch.tensor(dpar, dtype=ctx.p_dtype, device=ctx.p_device)
        return lam.to(ctx.u_dtype), gp, None, None, None, None


def fs_rollout(u0, params, solver, dt, nsteps, K):
    """u_T = FS^nsteps(u0) with parameters params = (M, kappa_c, L, kappa_eta);
    differentiable in u0 and params through the discrete adjoint."""
    return FSRollout.apply(u0, params, solver, dt, nsteps, K)
