"""Differentiable rendering: torch.autograd.Function over the batch renderer.

Each job's differentiable parameters form a row of 13 values,
    theta = (c0, c1, c2, c3, n, plane0 n_x, n_y, n_z, d, plane1 n_x, n_y, n_z, d)
(Julia constant, Mandelbulb power, raw cut planes; entries that a job does
not use get zero gradient).  The forward pass renders with the row's values;
the backward pass is the library's adjoint (implicit differentiation at the
hit points), which reads only the saved depth and status planes.
"""
import copy

import numpy as np
import torch

from . import alloc_workspace, render_backward, render_batch

N_PARAMS = 13


def job_params(job):
    """The 13-value parameter row of a job (float64 numpy)."""
    row = np.zeros(N_PARAMS)
    fr = job["fractal"]
    row[0:4] = fr.get("c", (0.0, 0.0, 0.0, 0.0))
    row[4] = fr.get("power", 2.0)
    for k, pl in enumerate(job.get("planes", [])):
        row[5 + 4 * k:8 + 4 * k] = pl["n"]
        row[8 + 4 * k] = pl["d"]
    return row


def job_with_params(job, row):
    """Copy of `job` with its fractal and plane parameters set from `row`."""
    out = copy.deepcopy(job)
    row = [float(x) for x in row]
    if out["fractal"]["kind"] == "julia":
        out["fractal"]["c"] = row[0:4]
    else:
        out["fractal"]["power"] = row[4]
    for k, pl in enumerate(out.get("planes", [])):
        pl["n"] = row[5 + 4 * k:8 + 4 * k]
        pl["d"] = row[8 + 4 * k]
    return out


class FractalRender(torch.autograd.Function):
    """forward(theta [n_jobs, 13], jobs, device) -> colour [3, H, W] of every
    job, then depth [H, W] of every job, then normal [3, H, W] of every job."""

    @staticmethod
    def forward(ctx, theta, jobs, device):
        rows = theta.detach().to("cpu", torch.float64).numpy()
        rjobs = [job_with_params(j, r) for j, r in zip(jobs, rows)]
        frames = render_batch(rjobs, device)
        ctx.jobs = rjobs
        ctx.device = device
        ctx.theta_meta = (theta.device, theta.dtype)
        ctx.save_for_backward(*[f["depth"] for f in frames], *[f["status"] for f in frames])
        ctx.set_materialize_grads(False)
        cols, deps, nrms = [], [], []
        for j, f in zip(rjobs, frames):
            H, W = int(j["camera"]["height"]), int(j["camera"]["width"])
            cols.append(f["colour"].view(3, H, W))
            deps.append(f["depth"].view(H, W))
            nrms.append(f["normal"].view(3, H, W))
        return tuple(cols + deps + nrms)

    @staticmethod
    def backward(ctx, *grads):
        n = len(ctx.jobs)
        saved = ctx.saved_tensors
        frames = [{"depth": saved[k], "status": saved[n + k], "normal": None, "colour": None} for k in range(n)]

        def flat(gs):
            if all(g is None for g in gs):
                return None
            return [g.reshape(-1).contiguous().float() if g is not None else None for g in gs]

        gc, gd, gn = flat(grads[:n]), flat(grads[n:2 * n]), flat(grads[2 * n:])
        grad_c, grad_n, grad_pl = render_backward(ctx.jobs, frames, gc, gd, gn, ctx.device,
                                                  workspace=alloc_workspace(n, ctx.device))
        g = torch.cat([grad_c, grad_n.view(n, 1), grad_pl.view(n, 8)], dim=1)
        dev, dt = ctx.theta_meta
        return g.to(dev, dt), None, None


def render_diff(jobs, theta, device="cuda"):
    """Differentiable batch render: list of {colour, depth, normal} tensors
    per job that carry gradients back to theta [n_jobs, 13]."""
    outs = FractalRender.apply(theta, jobs, device)
    n = len(jobs)
    return [{"colour": outs[k], "depth": outs[n + k], "normal": outs[2 * n + k]} for k in range(n)]
