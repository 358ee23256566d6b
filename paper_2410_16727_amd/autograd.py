"""The trajectory objective as a torch.autograd.Function.

forward: J[s] = C_goal + C_smooth + C_world + limit penalty of trajectory
X[s] (App. A.6) from the library's cost kernel -- when X needs a gradient,
the cost+gradient kernel instead, one launch for both (the hand-written
adjoint, which recomputes the kinematics rather than storing per-joint
transforms; row 0 of the gradient is zero, waypoint 0 being pinned).
backward: dJ[s] times the saved gradient, the same float32 product the
kernel forms when given dJ.  Every evaluation runs on the GPU through the
C ABI; nothing is computed in Python."""
import torch


class DSCost(torch.autograd.Function):
    @staticmethod
    def forward(ctx, X, plan, scene_id, q_start, goal):
        Xc = X.detach().contiguous()
        if ctx.needs_input_grad[0]:
            J, G = plan.cost_grad(scene_id, q_start, goal, Xc)
            ctx.save_for_backward(G)
        else:
            J = plan.cost(scene_id, q_start, goal, Xc)
        return J

    @staticmethod
    def backward(ctx, dJ):
        (G,) = ctx.saved_tensors
        return G * dJ.detach().to(G.dtype).view(-1, 1, 1), None, None, None, None


def trajectory_cost(X, plan, scene_id, q_start, goal):
    """J [S] for X [S, T, 7] (float32, cuda), differentiable in X."""
    return DSCost.apply(X, plan, scene_id, q_start, goal)
