"""The trajectory objective as a torch.autograd.Function.

forward: J[s] = C_goal + C_smooth + C_world + limit penalty of trajectory
X[s] (App. A.6) from the library's cost kernel.  backward: the hand-written
adjoint kernel (ds_cost_grad with the incoming dJ), which recomputes the
kinematics at X instead of storing per-joint transforms, and returns
dJ[s] * dJ_s/dX (row 0 is zero: waypoint 0 is pinned).  With fused=True
the forward runs the cost+gradient kernel once when X needs a gradient and
the backward scales that saved gradient by dJ (the same float32 product the
adjoint kernel forms) -- one launch instead of two when backward is sure to
follow.  Every evaluation runs on the GPU through the C ABI; nothing is
computed in Python."""
import torch


class DSCost(torch.autograd.Function):
    @staticmethod
    def forward(ctx, X, plan, scene_id, q_start, goal, fused):
        Xc = X.detach().contiguous()
        ctx.plan, ctx.scene_id, ctx.q_start, ctx.goal = plan, scene_id, q_start, goal
        ctx.fused = bool(fused) and ctx.needs_input_grad[0]
        if ctx.fused:
            J, G = plan.cost_grad(scene_id, q_start, goal, Xc)
            ctx.save_for_backward(G)
        else:
            J = plan.cost(scene_id, q_start, goal, Xc)
            ctx.save_for_backward(Xc)
        return J

    @staticmethod
    def backward(ctx, dJ):
        (saved,) = ctx.saved_tensors
        dJc = dJ.detach().to(torch.float32).contiguous()
        if ctx.fused:
            return saved * dJc.view(-1, 1, 1), None, None, None, None, None
        _, dX = ctx.plan.cost_grad(ctx.scene_id, ctx.q_start, ctx.goal, saved, dJ=dJc)
        return dX, None, None, None, None, None


def trajectory_cost(X, plan, scene_id, q_start, goal, fused=False):
    """J [S] for X [S, T, 7] (float32, cuda), differentiable in X: the
    backward launches the adjoint kernel (fused=True: the gradient comes
    from the forward's single cost+gradient launch)."""
    return DSCost.apply(X, plan, scene_id, q_start, goal, fused)
