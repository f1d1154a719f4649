"""torch.autograd binding of the adjoint gradient (fbt_grad).

``matern_loglik(theta, context)`` returns the exact log-likelihood (Eq. (1))
of the data held by ``context`` as a 0-d tensor that is differentiable in
theta = (sigma2, alpha, nu); its backward uses the score of Eq. (2) computed by
the library's adjoint path.  The forward pass computes the score only when
theta requires a gradient (otherwise it is a plain Algorithm 2 call).
"""
import numpy as np
import torch


class MaternLoglik(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, context):
        th = theta.detach().to("cpu", torch.float64).numpy()
        if ctx.needs_input_grad[0]:
            ll, score = context.grad(th)
        else:
            ll, score = context.loglik(th), np.zeros(3)
        ctx.save_for_backward(torch.as_tensor(score, dtype=theta.dtype, device=theta.device))
        return torch.tensor(ll, dtype=theta.dtype, device=theta.device)

    @staticmethod
    def backward(ctx, g):
        (score,) = ctx.saved_tensors
        return g * score, None


def matern_loglik(theta: torch.Tensor, context) -> torch.Tensor:
    return MaternLoglik.apply(theta, context)
