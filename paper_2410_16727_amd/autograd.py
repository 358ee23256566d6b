"""The trajectory objective as a torch.autograd.Function.

forward: J[s] = C_goal + C_smooth + C_world + limit penalty of trajectory
X[s] (App. A.6) from the library's cost kernel.  backward: the hand-written
adjoint kernel, which recomputes the kinematics rather than storing
per-joint transforms; row 0 of the gradient is zero (waypoint 0 pinned).
Both run on the GPU through the C ABI; nothing is computed in Python."""
import torch


class DSCost(torch.autograd.Function):
    @staticmethod
    def forward(ctx, X, plan, scene_id, q_start, goal):
        Xc = X.detach().contiguous()
        J = plan.cost(scene_id, q_start, goal, Xc)
        ctx.save_for_backward(Xc)
        ctx.plan, ctx.scene_id, ctx.q_start, ctx.goal = plan, scene_id, q_start, goal
        return J

    @staticmethod
    def backward(ctx, dJ):
        (X,) = ctx.saved_tensors
        _, dX = ctx.plan.cost_grad(ctx.scene_id, ctx.q_start, ctx.goal, X,
                                   dJ.detach().contiguous().float())
        return dX, None, None, None, None


def trajectory_cost(X, plan, scene_id, q_start, goal):
    """J [S] for X [S, T, 7] (float32, cuda), differentiable in X."""
    return DSCost.apply(X, plan, scene_id, q_start, goal)
