"""torch.autograd.Function over the library's K-step particle map.

PushDeposit.apply(EB, u0, ctx, dt, K, m) runs K particle steps with the
contravariant fields EB ([6, np3, np2, np1], the padded layout of the
library) and the initial four-velocities u0 ([3, capacity], the particle
order of the context) and returns (J_K, u_K): the conformal current of the
last step and the final four-velocities.  Its backward runs the library's
hand-written adjoint kernels with checkpoints every m steps and returns
dL/dEB (periodic ghost contributions added into their images) and dL/du0.
Positions are inputs of the map taken from the context; they are not
differentiated.  The K steps run exactly as ctx.push_deposit would run them,
sorts of the context's cadence included: u_K is in the particle order at
step K (ctx.checkpointed_order() gives each slot's step-0 slot), u0 and
dL/du0 in the order at step 0.

A context holds one checkpointed forward at a time: backward() of an
earlier apply() on the same context, after a later one, raises.
"""
import torch


class PushDeposit(torch.autograd.Function):
    @staticmethod
    def forward(fctx, EB, u0, ctx, dt, K, m):
        ctx.fields().copy_(EB)
        ctx.fields_fill_ghosts()
        arr = ctx.particle_arrays()
        for a in range(3):
            arr["u"][a].copy_(u0[a])
        gen = ctx.forward_checkpointed(dt, K, m)
        J = ctx.current().clone()
        arr = ctx.particle_arrays()
        uK = torch.stack([arr["u"][a] for a in range(3)]).clone()
        fctx.pic = ctx
        fctx.args = (dt, K, m)
        fctx.generation = gen
        return J, uK

    @staticmethod
    def backward(fctx, gJ, gu):
        ctx = fctx.pic
        dt, K, m = fctx.args
        if ctx.forward_generation != fctx.generation:
            raise RuntimeError("PushDeposit.backward: a later forward on the same context replaced "
                               "this one's checkpoints (one forward may be outstanding per context)")
        dEB, du0 = ctx.backward(dt, K, m, lamJ=gJ, lam_u=gu)
        return dEB, du0, None, None, None, None


def push_deposit(EB, u0, ctx, dt, K, m):
    return PushDeposit.apply(EB, u0, ctx, dt, K, m)
