"""torch.autograd.Function around the adjoint-method backward of libqsv.

Forward: the parametrised circuit runs on |0...0> through a plan, then
E = <psi| J sum Z_i Z_{i+1} + h sum X_i |psi> (qsv_expval_zz_x, float64).
Backward: lam = H psi (qsv_apply_tfim) and qsv_adjoint_grad walks the gates
backwards (Jones and Gacon, arXiv:2009.02823).  Every step runs in the
library's kernels; this module only sequences the calls.
"""
import torch

from . import (PLAN_PER_GATE, QSV_C64, QSV_C128, qsv_adjoint_grad, qsv_apply_tfim, qsv_expval_zz_x,
               qsv_plan_create, qsv_plan_execute)

ROTATIONS = ("RX", "RY", "RZ")


def bind(template, theta):
    """Copy of the circuit with the rotation angles replaced by theta (in order)."""
    vals = [float(v) for v in theta.detach().cpu().tolist()]
    out, k = [], 0
    for g in template:
        g = dict(g)
        if g["name"] in ROTATIONS:
            g["params"] = [vals[k]] + list(g.get("params", [])[1:])
            k += 1
        out.append(g)
    if k != len(vals):
        raise ValueError("circuit has %d rotations, theta has %d entries" % (k, len(vals)))
    return out


class ExpvalFn(torch.autograd.Function):
    """E(theta) = <0| U(theta)^dag H U(theta) |0>, H = J sum ZZ + h sum X."""

    @staticmethod
    def forward(ctx, theta, template, n, dtype, J, h, periodic, mode):
        circ = bind(template, theta)
        tdt = torch.complex64 if dtype == QSV_C64 else torch.complex128
        psi = torch.zeros(1 << n, dtype=tdt, device="cuda")
        psi[0] = 1.0
        plan = qsv_plan_create(n, dtype, circ, mode=mode)
        qsv_plan_execute(plan, psi)
        e = qsv_expval_zz_x(psi, J, h, periodic)
        ctx.save_for_backward(psi)
        ctx.circ, ctx.J, ctx.h, ctx.periodic = circ, J, h, periodic
        return e[0].to(theta.dtype)

    @staticmethod
    def backward(ctx, grad_out):
        (psi,) = ctx.saved_tensors
        psi = psi.clone()
        lam = torch.empty_like(psi)
        qsv_apply_tfim(psi, lam, ctx.J, ctx.h, ctx.periodic)
        g = qsv_adjoint_grad(psi, lam, ctx.circ)
        return (grad_out * g.to(grad_out.dtype), None, None, None, None, None, None, None)


def expval(theta, template, n, dtype=QSV_C64, J=1.0, h=0.5, periodic=False, mode=PLAN_PER_GATE):
    return ExpvalFn.apply(theta, template, n, dtype, J, h, periodic, mode)
