"""The discrete energy as a differentiable PyTorch function.

``energy(X, prob)`` returns E_h(X) (Sec. 3) as a float64 scalar tensor.  Its
backward is the library's gradient kernel (gpe_grad, Euclidean) and the
backward of that gradient -- the double backward of the energy -- is the
library's Hessian-vector product (gpe_set_point + gpe_hvp, Euclidean).

Gradient convention.  The library's gradient G satisfies
E(X + D) = E(X) + Re<G, D> + O(|D|^2) with <X, Y> = sum X conj(Y); that is
exactly the gradient PyTorch expects for a real function of a complex tensor
(for E = |z|^2 both give 2z).  The Hessian is a real-linear map that is
symmetric for Re<., .>, so the vector-Jacobian product of the gradient with a
vector V is nabla^2 E[V].

Only argument marshalling happens here; ``prob`` is a binding.Problem (its
work precision decides the precision of the HVP).
"""

import torch


class _Gradient(torch.autograd.Function):
    @staticmethod
    def forward(ctx, X, prob):
        G, _, _ = prob.grad(X.detach().contiguous(), riemannian=False)
        ctx.save_for_backward(X)
        ctx.prob = prob
        return G

    @staticmethod
    def backward(ctx, V):
        (X,) = ctx.saved_tensors
        prob = ctx.prob
        prob.set_point(X.detach().contiguous())
        HV = prob.hvp(V.detach().contiguous().to(prob.work_dtype), riemannian=False)
        return HV.to(X.dtype), None


class EnergyFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, X, prob):
        ctx.save_for_backward(X)
        ctx.prob = prob
        return torch.tensor(prob.energy(X.detach().contiguous()), dtype=torch.float64, device=X.device)

    @staticmethod
    def backward(ctx, gE):
        (X,) = ctx.saved_tensors
        G = _Gradient.apply(X, ctx.prob)
        return gE.to(G.real.dtype) * G, None


def energy(X, prob):
    """E_h(X) with backward = gradient kernel and double backward = HVP kernel."""
    return EnergyFn.apply(X, prob)
