"""Compliance as a differentiable torch function.

Forward: densities -> SIMP operator refresh -> MGCG solve -> c = sum_l f_l^T u_l.
Backward: the hand-written adjoint kernel.  Compliance is self-adjoint
(the adjoint state is -u), so dc/drho_i = -p rho_i^{p-1} (E0 - Emin)
sum_l u_{l,e}^T K^(e_i) u_{l,e} (Sec. 3.4), evaluated on the device from the
forward solution; the incoming gradient scales it.
"""

import torch


class Compliance(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rho, problem, rtol=1e-10, maxit=2000, warm_start=True):
        if not rho.is_cuda:
            raise TypeError("rho must live on the GPU")
        problem.use_torch_stream()
        r = rho.detach().to(torch.float64).contiguous()
        problem.set_densities(r)
        info = problem.solve(rtol=rtol, maxit=maxit, warm_start=warm_start)
        # the adjoint kernel runs with the forward solve (the problem's u may
        # change before backward), and only when a gradient is wanted
        if ctx.needs_input_grad[0]:
            dc = torch.empty(problem.nrho, dtype=torch.float64, device=rho.device)
            c, _ = problem.compliance_sensitivity(dc_out=dc)
            ctx.save_for_backward(dc)
        else:
            c, _ = problem.compliance_sensitivity(want_dc=False)
        ctx.shape = rho.shape
        ctx.dtype = rho.dtype
        ctx.info = info
        return torch.tensor(c[-1], dtype=torch.float64, device=rho.device)

    @staticmethod
    def backward(ctx, g):
        (dc,) = ctx.saved_tensors
        return (g * dc).view(ctx.shape).to(ctx.dtype), None, None, None, None


def compliance(rho, problem, rtol=1e-10, maxit=2000, warm_start=True):
    return Compliance.apply(rho, problem, rtol, maxit, warm_start)


class Project(torch.autograd.Function):
    """rho = W x (Sec. 3.2 eq. (5)) on the device; backward: W^T g, the chain
    rule of Sec. 3.4, by the library's transpose kernel."""

    @staticmethod
    def forward(ctx, x, proj):
        if not x.is_cuda:
            raise TypeError("x must live on the GPU")
        ctx.proj = proj
        ctx.shape = x.shape
        ctx.dtype = x.dtype
        xv = x.detach().to(torch.float64).contiguous().view(-1)
        return proj.apply(xv)

    @staticmethod
    def backward(ctx, g):
        gx = ctx.proj.apply_transpose(g.detach().to(torch.float64).contiguous().view(-1))
        return gx.view(ctx.shape).to(ctx.dtype), None


def project(x, proj):
    return Project.apply(x, proj)

