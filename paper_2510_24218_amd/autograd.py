"""Differentiable sampling objectives on top of the engine.

The circuit's output distribution p_theta(x) = |<x|C(theta)|0^n>|^2 is
sampled exactly (Algorithm 1) and its log-probability is differentiable in
theta: the forward value comes from the whole-circuit amplitude contraction
(``pws_amplitudes``) and the backward pass from the adjoint contraction
through each sample's tree (``pws_grad``), both on the device.

An expectation E_{x ~ p_theta}[f(x)] of a cost that does not depend on theta
has the score-function gradient E[(f(x) - b) d log p_theta(x) / d theta] for
any constant baseline b; ``sampled_expectation`` returns the sample mean of f
with exactly that estimator attached as its gradient, so a training loop is
``loss = sampled_expectation(...); loss.backward(); opt.step()``.
"""
from __future__ import annotations

import math
from typing import Callable

import numpy as np
import torch

__all__ = ["LogProbability", "log_probability", "sampled_expectation"]

_LN2 = math.log(2.0)


def _theta_host(theta: torch.Tensor) -> np.ndarray:
    return theta.detach().to("cpu", torch.float64).contiguous().numpy()


class LogProbability(torch.autograd.Function):
    """log p_theta(x_i) for a batch of bitstrings, differentiable in theta.

    forward(theta (P,), plan, samples (K, words) int64) -> (K,) float64.
    The plan's angles are set to theta (``Plan.set_theta``) before the
    amplitudes are taken and again before the adjoint pass, so one plan can
    serve several parameter vectors in the same graph."""

    @staticmethod
    def forward(ctx, theta, plan, samples):
        th = _theta_host(theta)
        plan.set_theta(th)
        m, e = plan.amplitudes(samples)
        mag2 = m[:, 0] * m[:, 0] + m[:, 1] * m[:, 1]
        logp = torch.log(mag2) + (2.0 * _LN2) * e.to(torch.float64)
        ctx.plan = plan
        ctx.theta_host = th
        ctx.theta_meta = (theta.dtype, theta.device)
        ctx.save_for_backward(samples)
        return logp.to(samples.device)

    @staticmethod
    def backward(ctx, grad_out):
        (samples,) = ctx.saved_tensors
        plan = ctx.plan
        plan.set_theta(ctx.theta_host)
        d = plan.grad(samples)                      # (K, P) float64, samples' device
        g = (grad_out.to(d.device, torch.float64)[:, None] * d).sum(0)
        dtype, device = ctx.theta_meta
        return g.to(device=device, dtype=dtype), None, None


def log_probability(plan, theta: torch.Tensor, samples: torch.Tensor) -> torch.Tensor:
    """log p_theta(x) of each row of ``samples`` (int64, (K, words))."""
    return LogProbability.apply(theta, plan, samples)


def sampled_expectation(plan, theta: torch.Tensor, cost: Callable[[torch.Tensor], torch.Tensor],
                        n_chains: int, seed: int, baseline: bool = True,
                        device: str | torch.device = "cuda"):
    """Sample mean of cost(x) over n_chains exact samples at theta, carrying
    the score-function gradient estimate.

    cost maps the (K, words) int64 sample tensor to a (K,) tensor.  With
    ``baseline`` b is the batch mean of the cost, which lowers the
    estimator's variance; because b includes each sample's own cost, the
    expected estimate is (K-1)/K times the true gradient.  Without it b = 0
    and the estimate is unbiased.  Returns (value, samples): value's gradient
    with respect to theta is mean_i[(f(x_i) - b) d log p(x_i) / d theta]."""
    with torch.no_grad():
        plan.set_theta(_theta_host(theta))
        x = torch.zeros((n_chains, plan.words), dtype=torch.int64, device=device)
        plan.sample(n_chains, seed, out=x)
        f = cost(x).to(torch.float64)
        b = f.mean() if baseline else torch.zeros((), dtype=torch.float64, device=f.device)
    logp = LogProbability.apply(theta, plan, x)
    w = (f - b).to(logp.device)
    value = f.mean().to(logp.device) + (w * (logp - logp.detach())).mean()
    return value.to(theta.dtype), x
