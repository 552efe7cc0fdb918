"""Differentiable ISAM forward operator and calibration fitting.

``IsamForward`` wraps isam_forward as a torch.autograd.Function of the object eta and
the calibration theta = (a2, a3, z_focus) (Eq. 7, 13).  Its backward runs the library's
own kernels: isam_adjoint for the object and isam_calibration_grad for theta.  Nothing is
computed by torch here; it only sequences the calls and holds the tensors.

``fit_calibration`` fits theta to measured spectra by gradient descent on the data
fidelity of Eq. 12 (the first term).  The paper takes a_i from an external autofocus;
here they are fitted from the data through the operator itself.  The dispersion phase
error grows with |k - k0|, so the fit is continued over widening spectral windows
(coarse to fine), and it runs in the recipe's natural units: phase at the band edge for
a2 and a3, depth rows for z_focus.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import torch

from .isam import Plan


def _calibration(plan: Plan) -> tuple:
    return getattr(plan, "_calib", (plan.geometry.a2, plan.geometry.a3, plan.geometry.z_focus))


def _set_calibration(plan: Plan, theta: tuple) -> None:
    theta = tuple(float(v) for v in theta)
    if _calibration(plan) != theta:
        plan.set_calibration(*theta)
        plan._calib = theta


class IsamForward(torch.autograd.Function):
    """s = Re(K^_theta eta) (Eq. 5, 13, 16) with gradients for eta and theta.

    eta: device complex64 [nx][nk]; theta: float64 tensor (3,) = (a2, a3, z_focus) in
    SI units (held on the host: the three scalars configure the plan's tables).
    """

    @staticmethod
    def forward(ctx, eta: torch.Tensor, theta: torch.Tensor, plan: Plan) -> torch.Tensor:
        th = tuple(float(v) for v in theta.detach().cpu().tolist())
        _set_calibration(plan, th)
        eta_c = eta.detach().contiguous()
        ctx.plan = plan
        ctx.theta = th
        ctx.theta_device = theta.device
        ctx.save_for_backward(eta_c)
        return plan.forward(eta_c)

    @staticmethod
    def backward(ctx, grad_s: torch.Tensor):
        (eta,) = ctx.saved_tensors
        plan = ctx.plan
        _set_calibration(plan, ctx.theta)
        g = grad_s.detach().contiguous().to(torch.float32)
        g_eta = plan.adjoint(g) if ctx.needs_input_grad[0] else None
        g_theta = None
        if ctx.needs_input_grad[1]:
            g_theta = torch.tensor(plan.calibration_grad(eta, g), dtype=torch.float64,
                                   device=ctx.theta_device)
        return g_eta, g_theta, None


def isam_forward(plan: Plan, eta: torch.Tensor, theta: torch.Tensor) -> torch.Tensor:
    """Functional form of IsamForward."""
    return IsamForward.apply(eta, theta, plan)


def natural_units(geometry) -> tuple:
    """(half band [rad/m], depth row pitch [m]) of a geometry: a2 = phase2 / half^2,
    a3 = phase3 / half^3, z_focus = rows * dz (uniform-in-k band, Nz = Nk rows)."""
    band = 2.0 * math.pi * geometry.dlambda / geometry.lambda_c ** 2
    return band / 2.0, math.pi / band


@dataclass
class FitResult:
    theta: tuple            # fitted (a2, a3, z_focus), SI units
    natural: tuple          # (edge phase2 [rad], edge phase3 [rad], focus rows)
    loss: float             # final full-band data fidelity 1/2 ||A eta - y||^2
    history: list           # (window, loss, natural) at the end of each stage


DEFAULT_SCHEDULE = ((0.15, 60, 0.02), (0.3, 60, 0.01), (0.5, 60, 0.005), (0.75, 60, 0.003),
                    (1.0, 80, 0.002))


def fit_calibration(plan: Plan, eta: torch.Tensor, y: torch.Tensor, theta0, schedule=DEFAULT_SCHEDULE
                    ) -> FitResult:
    """Fit theta = (a2, a3, z_focus) to spectra y for a known object eta.

    Minimises 1/2 sum_n W_f(k_n) sum_p (A_theta eta - y)^2 with W_f the indicator of
    |k - k0| <= f * band/2, for each stage (f, steps, lr) of ``schedule``.  Each stage runs
    Adam in coordinates relative to the stage's starting point (steps of about lr of the
    current value).  Gradients come from IsamForward's backward.
    """
    half, dz = natural_units(plan.geometry)
    unit = torch.tensor([1.0 / half ** 2, 1.0 / half ** 3, dz], dtype=torch.float64)
    nat = torch.tensor(theta0, dtype=torch.float64) / unit
    nk = plan.nk
    u = (torch.arange(nk, dtype=torch.float64) - nk // 2).abs() / (nk / 2)
    history = []
    for f, steps, lr in schedule:
        window = (u <= f).to(torch.float32).to(y.device)[None, :]
        scale = nat.abs().clamp_min(1e-30)
        x = torch.ones(3, dtype=torch.float64, requires_grad=True)
        opt = torch.optim.Adam([x], lr=lr)
        loss_v = float("nan")
        for _ in range(steps):
            opt.zero_grad()
            theta = x * scale * unit
            r = isam_forward(plan, eta, theta) - y
            loss = 0.5 * (window * r * r).sum()
            loss.backward()
            opt.step()
            loss_v = float(loss.detach())
        nat = (x.detach() * scale).clone()
        history.append((f, loss_v, tuple(nat.tolist())))
    theta = tuple((nat * unit).tolist())
    with torch.no_grad():
        _set_calibration(plan, theta)
        r = plan.forward(eta.contiguous()) - y
        final = 0.5 * float((r.double() ** 2).sum())
    return FitResult(theta, tuple(nat.tolist()), final, history)
