"""Transmittance optimisation (Sec. 7.2): refine the primitives of a model so
that its transmittance images match reference images, by Adam on the L2 loss
of the accumulated free-flight CDF (eq. accum_cdf) over several views.

Every step runs in the HIP library: camera rays (``ugp_camera_rays``), the
CDF, loss and gradient (``ugp_accum_cdf``), the Adam update with its clamps
(``ugp_fit_adam``) and the hierarchy update after the primitives moved
(``ugp_build_bvh``, or ``ugp_refit_bvh`` between rebuilds).  This module
only sequences the calls.
"""
from __future__ import annotations

import time


def view_rays(ctx, cams: list, seed: int, sample: int):
    """One jittered ray per pixel of every view, concatenated view by view."""
    import torch
    return torch.cat([ctx.camera_rays(cam, seed=seed + 104729 * (k + 1), sample=sample)
                      for k, cam in enumerate(cams)])


def reference_images(ctx, scene: dict, cams: list, seed: int = 0, samples: int = 16):
    """The accumulated CDF of `scene` per pixel of every view (concatenated
    view by view), averaged over `samples` jittered rays per pixel: the
    reference the fit matches."""
    ctx.build_bvh(scene)
    acc = None
    for s in range(samples):
        C = ctx.accum_cdf(view_rays(ctx, cams, seed, s))
        acc = C if acc is None else acc + C
    return acc / samples


def _update_hierarchy(ctx, params: dict, it: int, rebuild_every: int):
    # the primitives moved: a new hierarchy every rebuild_every steps, a refit
    # of the last one in between
    if rebuild_every <= 1 or (it - 1) % rebuild_every == 0:
        ctx.build_bvh(params)
    else:
        ctx.refit_bvh(params)


def fit_transmittance(ctx, params: dict, cams: list, target, iters: int, lr=(1e-4, 1e-2, 2e-5, 1e-4),
                      min_scale: float = 1e-6, seed: int = 1, on_step=None, rebuild_every: int = 1) -> dict:
    """Optimise params (device float32 tensors mean, scale, rotation, density,
    updated in place; plus albedo, roughness, emission, material for the
    hierarchy build) for `iters` Adam steps with rates lr = (means, log
    scales, rotations, densities).  Loss: mean over the views' pixels of
    (C - target)^2, one jittered ray per pixel per step, all views in one
    batch.  The hierarchy is rebuilt every `rebuild_every` steps and refitted
    in between.  Returns the loss of every step and the wall time."""
    import torch
    n = params["mean"].shape[0]
    dev = params["mean"].device
    m = torch.zeros((n, 11), device=dev, dtype=torch.float32)
    v = torch.zeros_like(m)
    grad = torch.zeros_like(m)
    npix = sum(c["width"] * c["height"] for c in cams)
    losses = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for it in range(1, iters + 1):
        _update_hierarchy(ctx, params, it, rebuild_every)
        grad.zero_()
        loss = torch.zeros(1, device=dev, dtype=torch.float32)
        rays = view_rays(ctx, cams, seed, it)
        ctx.accum_cdf(rays, target=target, want_C=False, loss_scale=1.0 / npix, loss=loss, grad=grad)
        ctx.fit_adam(params, grad, m, v, it, lr=lr, min_scale=min_scale)
        losses.append(loss)
        if on_step is not None:
            on_step(it)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return {"loss": [float(x.item()) for x in losses], "seconds": wall}


def reference_rf_images(ctx, scene: dict, cams: list, seed: int = 0, samples: int = 16):
    """Radiance-field images (Sec. 8, eq. rf) of `scene`, per pixel of every
    view [sum of pixels, 3], averaged over `samples` jittered rays."""
    ctx.build_bvh(scene)
    acc = None
    for s in range(samples):
        L = ctx.rf_render(view_rays(ctx, cams, seed, s))
        acc = L if acc is None else acc + L
    return acc / samples


def fit_radiance_field(ctx, params: dict, cams: list, target, iters: int, lr=(1e-4, 1e-2, 2e-5, 1e-4, 1e-2),
                       min_scale: float = 1e-6, seed: int = 1, on_step=None, rebuild_every: int = 1) -> dict:
    """Image-based radiance-field reconstruction (Sec. 8): Adam on the mean
    over the views' pixels of |L - target|^2 with L of eq. rf, one jittered
    ray per pixel per step, every parameter of every primitive including its
    emission; lr = rates of the means, log scales, rotations, densities and
    emissions.  params as fit_transmittance (emission updated too)."""
    import torch
    n = params["mean"].shape[0]
    dev = params["mean"].device
    m = torch.zeros((n, 14), device=dev, dtype=torch.float32)
    v = torch.zeros_like(m)
    grad = torch.zeros_like(m)
    npix = sum(c["width"] * c["height"] for c in cams)
    losses = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for it in range(1, iters + 1):
        _update_hierarchy(ctx, params, it, rebuild_every)
        grad.zero_()
        loss = torch.zeros(1, device=dev, dtype=torch.float32)
        ctx.rf_render(view_rays(ctx, cams, seed, it), target=target, want_L=False, loss_scale=1.0 / npix,
                      loss=loss, grad=grad)
        ctx.fit_adam(params, grad, m, v, it, lr=lr, min_scale=min_scale, emission=True)
        losses.append(loss)
        if on_step is not None:
            on_step(it)
    torch.cuda.synchronize()
    return {"loss": [float(x.item()) for x in losses], "seconds": time.perf_counter() - t0}
