"""The total potential as a differentiable torch function.

Pi(u) = sum_e vol_e Psi_e(u) - f_ext . u is the physics-informed loss of the
paper's pretraining stage (Sec. 'Pretraining'; loss equations of the
linear-elastic and Neo-Hookean experiments).  Its derivatives are the
explicit finite-element ones (App. A: shape-function differentiation rather
than automatic differentiation):

    dPi/du      = f_int(u) - f_ext          (internal-force kernel)
    d2Pi/du2 v  = K_T(u) v                  (Hessian-vector kernel)

so `energy(u).backward()` runs the force kernel and a double backward runs
the Hessian-vector kernel.  All three are hand-written HIP kernels behind
the C ABI; nothing here computes.
"""
import torch


class _HVP(torch.autograd.Function):
    """y = K_T(u) v.  Gradient w.r.t. v is K_T(u) g (K_T symmetric); the
    third derivative (w.r.t. u) is not provided."""

    @staticmethod
    def forward(ctx, u, v, mesh, prec, layout):
        ctx.save_for_backward(u)
        ctx.cfg = (mesh, prec, layout)
        return mesh.hvp(u.detach(), v.detach(), prec=prec, layout=layout)

    @staticmethod
    def backward(ctx, g):
        (u,) = ctx.saved_tensors
        mesh, prec, layout = ctx.cfg
        gv = _HVP.apply(u, g, mesh, prec, layout) if ctx.needs_input_grad[1] else None
        return None, gv, None, None, None


class _Force(torch.autograd.Function):
    """g = f_int(u) - f_ext; its vector-Jacobian product is K_T(u) w."""

    @staticmethod
    def forward(ctx, u, mesh, prec, layout):
        ctx.save_for_backward(u)
        ctx.cfg = (mesh, prec, layout)
        return mesh.force(u.detach(), prec=prec, layout=layout)

    @staticmethod
    def backward(ctx, w):
        (u,) = ctx.saved_tensors
        mesh, prec, layout = ctx.cfg
        return _HVP.apply(u, w, mesh, prec, layout), None, None, None


class _Energy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u, mesh, prec, layout):
        ctx.save_for_backward(u)
        ctx.cfg = (mesh, prec, layout)
        return mesh.energy(u.detach(), prec=prec, layout=layout)

    @staticmethod
    def backward(ctx, g):
        (u,) = ctx.saved_tensors
        mesh, prec, layout = ctx.cfg
        f = _Force.apply(u, mesh, prec, layout)
        return (g.to(f.dtype) * f), None, None, None


def energy(mesh, u, prec="fp32", layout="user"):
    """Differentiable Pi(u) (float64 scalar tensor) for a finalized Mesh."""
    return _Energy.apply(u, mesh, prec, layout)


def force(mesh, u, prec="fp32", layout="user"):
    """Differentiable f_int(u) - f_ext."""
    return _Force.apply(u, mesh, prec, layout)


# ------------------------------------------------------------------ batches
class _BatchHVP(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u, v, batch, prec):
        ctx.save_for_backward(u)
        ctx.cfg = (batch, prec)
        return batch.hvp(u.detach(), v.detach(), prec=prec)

    @staticmethod
    def backward(ctx, g):
        (u,) = ctx.saved_tensors
        batch, prec = ctx.cfg
        gv = _BatchHVP.apply(u, g, batch, prec) if ctx.needs_input_grad[1] else None
        return None, gv, None, None


class _BatchForce(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u, batch, prec):
        ctx.save_for_backward(u)
        ctx.cfg = (batch, prec)
        return batch.force(u.detach(), prec=prec)

    @staticmethod
    def backward(ctx, w):
        (u,) = ctx.saved_tensors
        batch, prec = ctx.cfg
        return _BatchHVP.apply(u, w, batch, prec), None, None


class _BatchEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u, batch, prec):
        ctx.save_for_backward(u)
        ctx.cfg = (batch, prec)
        return batch.energy(u.detach(), prec=prec)

    @staticmethod
    def backward(ctx, g):
        (u,) = ctx.saved_tensors
        batch, prec = ctx.cfg
        f = _BatchForce.apply(u, batch, prec)
        off = batch.offsets
        scale = torch.repeat_interleave(
            g.to(f.dtype), torch.as_tensor(off[1:] - off[:-1], device=f.device))
        return scale * f, None, None


def batch_energy(batch, u, prec="fp32"):
    """Per-mesh energies (float64, one per mesh) of a concatenated field in
    the batch's internal layout; differentiable twice."""
    return _BatchEnergy.apply(u, batch, prec)
