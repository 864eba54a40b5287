"""torch.autograd wrapper of the forward and adjoint library calls (marshalling only).

    sigma = XsecFn.apply(plan, upper, lower, T, P, logA, gamma_ref, n_exp)

`plan` must be a Voigt Plan created with a_is_log=True and per-line broadening; T and P
are 0-d float64 tensors.  The backward pass calls xs_cross_section_adjoint, which
recomputes the profiles; it uses the line set of the latest forward on this plan, so
call backward before the plan's next forward.  The library returns the per-line
gradients in double precision; they are cast to the dtypes of logA, gamma_ref and n_exp
(float32 parameters receive float32 gradients, which underflow to subnormals or zero for
losses on cross sections of ~1e-20 cm^2: pass float64 parameters, or scale the loss, to
keep their digits).
"""
import torch


class XsecFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, plan, upper, lower, T, P, logA, gamma_ref, n_exp):
        plan.set_lines(upper, lower, logA.detach().contiguous(), gamma_ref.detach().contiguous(),
                       n_exp.detach().contiguous())
        sigma = plan.cross_section([float(T)], [float(P)])[0]
        ctx.plan = plan
        ctx.T, ctx.P = float(T), float(P)
        ctx.n = logA.numel()
        ctx.ptypes = (logA.dtype, gamma_ref.dtype, n_exp.dtype)
        ctx.dtypes = (T.dtype if torch.is_tensor(T) else torch.float64,
                      P.dtype if torch.is_tensor(P) else torch.float64)
        return sigma

    @staticmethod
    def backward(ctx, grad_sigma):
        g = grad_sigma.detach().to(ctx.plan.dtype).contiguous()
        dT, dP, dlnA, dg, dn = ctx.plan.cross_section_adjoint(ctx.T, ctx.P, g, ctx.n)
        return (None, None, None, dT.reshape(()).to(ctx.dtypes[0]), dP.reshape(()).to(ctx.dtypes[1]),
                dlnA.to(ctx.ptypes[0]), dg.to(ctx.ptypes[1]), dn.to(ctx.ptypes[2]))
