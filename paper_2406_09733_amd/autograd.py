"""torch.autograd functions over the library's differentiable images: the
accumulated free-flight CDF of each ray (Sec. 7.2, eq. accum_cdf), the
radiance-field image (Sec. 8, eq. rf), and the path-traced image as a
function of the primitives' albedo and roughness (the shading adjoints by
path replay).

The forward builds the hierarchy of the given parameters and renders with
ugp_accum_cdf / ugp_rf_render; the backward is the library's
vector-Jacobian product (ugp_accum_cdf_backward / ugp_rf_render_backward),
each primitive's term differentiated with t_sat held fixed as in Sec. 7.2.
Only argument marshalling happens here.  The hierarchy is the one piece of
state between the two passes: when another build has replaced it by the
time the backward runs, it is rebuilt from the saved parameters.
"""
import torch

_SHAPE = ("mean", "scale", "rotation", "density")


class _Image(torch.autograd.Function):
    @staticmethod
    def forward(fctx, ugp, rgb, rays, exclude, fixed, mean, scale, rotation, density, emission):
        scene = dict(fixed, mean=mean.detach(), scale=scale.detach(), rotation=rotation.detach(),
                     density=density.detach(), emission=emission.detach())
        ugp.build_bvh(scene)
        out = ugp.rf_render(rays, exclude=exclude) if rgb else ugp.accum_cdf(rays, exclude=exclude)
        fctx.ugp, fctx.rgb, fctx.fixed, fctx.build_id = ugp, rgb, fixed, ugp.build_id
        fctx.save_for_backward(rays, exclude, mean, scale, rotation, density, emission)
        return out

    @staticmethod
    def backward(fctx, g):
        ugp, rgb = fctx.ugp, fctx.rgb
        rays, exclude, mean, scale, rotation, density, emission = fctx.saved_tensors
        if ugp.build_id != fctx.build_id:
            ugp.build_bvh(dict(fctx.fixed, mean=mean.detach(), scale=scale.detach(), rotation=rotation.detach(),
                               density=density.detach(), emission=emission.detach()))
            fctx.build_id = ugp.build_id
        grad = torch.zeros((ugp.n, 14 if rgb else 11), device=ugp.device, dtype=torch.float32)
        if rgb:
            ugp.rf_render_backward(rays, g.contiguous(), grad, exclude)
        else:
            ugp.accum_cdf_backward(rays, g.contiguous(), grad, exclude)
        g_em = grad[:, 11:14] if rgb else None
        return (None, None, None, None, None, grad[:, 0:3], grad[:, 3:6], grad[:, 6:10], grad[:, 10], g_em)


def _apply(ugp, params: dict, rays, exclude, rgb: bool):
    dev = ugp.device
    f32 = lambda k: torch.as_tensor(params[k]).to(device=dev, dtype=torch.float32)
    fixed = {k: params[k] for k in ("albedo", "roughness", "material")}
    for k in ("sggx", "metallic"):
        if params.get(k) is not None:
            fixed[k] = params[k]
    rays = torch.as_tensor(rays).to(device=dev, dtype=torch.float32).contiguous()
    if exclude is not None:
        exclude = torch.as_tensor(exclude).to(device=dev, dtype=torch.int32).contiguous()
    return _Image.apply(ugp, rgb, rays, exclude, fixed, *[f32(k) for k in _SHAPE], f32("emission"))


def accum_cdf(ugp, params: dict, rays, exclude=None):
    """C per ray (float32 [n], eq. accum_cdf), differentiable with respect to
    params' mean [P, 3], scale [P, 3], rotation [P, 4] (w, x, y, z; the
    rotation of q / |q|) and density [P].  params is a scene dict (as
    Context.build_bvh takes it) whose float tensors may require grad; ugp is
    a Context, whose hierarchy this call rebuilds."""
    return _apply(ugp, params, rays, exclude, False)


def rf_render(ugp, params: dict, rays, exclude=None):
    """Radiance per ray (float32 [n, 3], eq. rf), differentiable with respect
    to mean, scale, rotation, density and emission [P, 3]."""
    return _apply(ugp, params, rays, exclude, True)


class _Render(torch.autograd.Function):
    @staticmethod
    def forward(fctx, ugp, cam, rparams, bparams, fixed, albedo, roughness, density):
        scene = dict(fixed, albedo=albedo.detach(), roughness=roughness.detach(), density=density.detach())
        ugp.build_bvh(scene)
        spp = int(rparams.get("spp", 1))
        s, _ = ugp.render(cam, dict(rparams, want_sumsq=False))
        fctx.ugp, fctx.cam, fctx.rparams, fctx.fixed, fctx.build_id = ugp, cam, bparams, fixed, ugp.build_id
        fctx.save_for_backward(albedo, roughness, density)
        return s / spp

    @staticmethod
    def backward(fctx, g):
        ugp = fctx.ugp
        albedo, roughness, density = fctx.saved_tensors
        if ugp.build_id != fctx.build_id:
            ugp.build_bvh(dict(fctx.fixed, albedo=albedo.detach(), roughness=roughness.detach(),
                               density=density.detach()))
            fctx.build_id = ugp.build_id
        # every wanted gradient from one forward pass and one replay
        ga = gr = gd = None
        if fctx.needs_input_grad[5]:
            ga = torch.zeros((ugp.n, 3), device=ugp.device, dtype=torch.float32)
        if fctx.needs_input_grad[6]:
            gr = torch.zeros(ugp.n, device=ugp.device, dtype=torch.float32)
        if fctx.needs_input_grad[7]:
            gd = torch.zeros(ugp.n, device=ugp.device, dtype=torch.float32)
        if ga is not None or gr is not None or gd is not None:
            ugp.render_grads(fctx.cam, fctx.rparams, g.contiguous(), ga, gr, gd)
        return None, None, None, None, None, ga, gr, gd


def render(ugp, params: dict, cam: dict, render_params: dict, backward_params: dict | None = None):
    """Mean path-traced image (float32 [H, W, 3], ugp_render's sum / spp),
    differentiable with respect to params["albedo"] [P, 3],
    params["roughness"] [P] and params["density"] [P] (the other scene fields
    are held fixed).  The backward is one ugp_render_grads call for the
    inputs that require a gradient: the albedo adjoint (the exact derivative
    of this estimate: same camera, render parameters and seed) and the
    roughness and density adjoints (unbiased estimates of the derivative of
    the expected image).  The radiance cache must be off.  backward_params
    overrides render parameters of the backward pass only: another seed there
    makes the gradient estimate independent of this image's noise (the
    gradient of a loss that multiplies the two, such as |image - target|^2,
    is otherwise biased by their correlation; the exact albedo derivative
    then is of another estimate)."""
    dev = ugp.device
    albedo = torch.as_tensor(params["albedo"]).to(device=dev, dtype=torch.float32)
    rough = torch.as_tensor(params["roughness"]).to(device=dev, dtype=torch.float32)
    dens = torch.as_tensor(params["density"]).to(device=dev, dtype=torch.float32)
    fixed = {k: params[k] for k in ("mean", "scale", "rotation", "emission", "material") if k in params}
    for k in ("sggx", "metallic"):
        if params.get(k) is not None:
            fixed[k] = params[k]
    bparams = dict(render_params, **(backward_params or {}))
    return _Render.apply(ugp, cam, dict(render_params), bparams, fixed, albedo, rough, dens)
