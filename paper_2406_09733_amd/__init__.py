"""paper_2406_09733_amd -- MI355X-native path tracing of scenes made of
linear-transmittance Gaussian primitives ("Unified Gaussian Primitives for
Scene Representation and Rendering", arXiv 2406.09733).

The compute lives in ``libugp.so`` (hand-written HIP for gfx950, C ABI in
``include/ugp.h``).  This module is a thin ctypes binding with the same names:
it checks shapes and dtypes, takes device pointers from torch tensors and the
current HIP stream, and raises on any non-OK status.  There is no CPU path: if
the library is missing the import of ``Context`` fails loudly.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libugp.so")
_lib = None

NOALLOC_MAX_RAYS = 4194304  # UGP_NOALLOC_MAX_RAYS

STATUS = {0: "ok", 1: "invalid argument", 2: "out of device memory", 3: "device error",
          4: "no scene has been built", 5: "unsupported", 6: "a per-ray buffer overflowed"}


class UGPError(RuntimeError):
    def __init__(self, call: str, code: int):
        super().__init__(f"{call}: {STATUS.get(code, code)} (status {code})")
        self.code = code


class _Scene(C.Structure):
    _fields_ = [("n", C.c_int64), ("mean", C.c_void_p), ("scale", C.c_void_p), ("rotation", C.c_void_p),
                ("density", C.c_void_p), ("albedo", C.c_void_p), ("roughness", C.c_void_p),
                ("emission", C.c_void_p), ("material", C.c_void_p), ("sggx", C.c_void_p),
                ("metallic", C.c_void_p)]


class _Camera(C.Structure):
    _fields_ = [("origin", C.c_float * 3), ("target", C.c_float * 3), ("up", C.c_float * 3),
                ("vfov_deg", C.c_float), ("width", C.c_int32), ("height", C.c_int32)]


def _camera(cam: dict) -> _Camera:
    c = _Camera()
    for i in range(3):
        c.origin[i] = cam["origin"][i]
        c.target[i] = cam["target"][i]
        c.up[i] = cam["up"][i]
    c.vfov_deg = cam["vfov_deg"]
    c.width, c.height = int(cam["width"]), int(cam["height"])
    return c


class _Params(C.Structure):
    _fields_ = [("spp", C.c_int32), ("max_depth", C.c_int32), ("seed", C.c_uint64),
                ("sample_offset", C.c_int64), ("env_radiance", C.c_float * 3), ("mis_mode", C.c_int32),
                ("nrc_mode", C.c_int32), ("nrc_terminate_after", C.c_int32),
                ("nrc_train_records", C.c_int32), ("nrc_lr", C.c_float), ("nrc_box", C.c_float * 6),
                ("nrc_train_steps", C.c_int32), ("nrc_radiance_scale", C.c_float),
                ("nrc_target_clamp", C.c_float), ("transport", C.c_int32)]


class _Stats(C.Structure):
    _fields_ = [("paths", C.c_int64), ("collision_rays", C.c_int64), ("light_rays", C.c_int64),
                ("env_rays", C.c_int64), ("node_visits", C.c_int64), ("prim_tests", C.c_int64),
                ("prim_reloads", C.c_int64), ("ms_collide", C.c_double), ("ms_collide_wide", C.c_double),
                ("ms_light", C.c_double), ("ms_env", C.c_double), ("ms_shade", C.c_double),
                ("ms_sort", C.c_double),
                ("launches_collide", C.c_int32),
                ("launches_light", C.c_int32), ("launches_env", C.c_int32),
                ("cat_nodes", C.c_int64 * 4), ("cat_prims", C.c_int64 * 4), ("cat_reloads", C.c_int64 * 4),
                ("nrc_queries", C.c_int64), ("nrc_records", C.c_int64), ("ms_nrc_infer", C.c_double),
                ("ms_nrc_train", C.c_double), ("nrc_loss", C.c_float), ("ms_tail", C.c_double)]


EXPORTS = ["ugp_create", "ugp_destroy", "ugp_set_stream", "ugp_build_bvh", "ugp_refit_bvh", "ugp_transmittance",
           "ugp_sample_collision", "ugp_sample_collision_noalloc", "ugp_saturation", "ugp_emitter_query", "ugp_render", "ugp_render_albedo_grad",
           "ugp_render_roughness_grad", "ugp_render_density_grad", "ugp_render_grads", "ugp_sync",
           "ugp_set_profiling", "ugp_set_path_pool", "ugp_set_tail_paths", "ugp_get_render_stats", "ugp_trace_counts", "ugp_status_string",
           "ugp_nrc_num_params", "ugp_nrc_set_weights", "ugp_nrc_get_weights", "ugp_nrc_encode",
           "ugp_nrc_forward", "ugp_nrc_train_step", "ugp_nrc_records", "ugp_exp_transmittance",
           "ugp_exp_sample_collision", "ugp_accum_cdf", "ugp_rf_render", "ugp_accum_cdf_backward",
           "ugp_rf_render_backward", "ugp_camera_rays", "ugp_fit_adam", "ugp_sggx_phase", "ugp_ray_integral",
           "ugp_philox"]


def lib():
    """Load libugp.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run `python -m paper_2406_09733_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, i64 = C.c_void_p, C.c_int64
        L.ugp_create.argtypes = [C.c_int, vp, C.POINTER(vp)]
        L.ugp_destroy.argtypes = [vp]
        L.ugp_set_stream.argtypes = [vp, vp]
        L.ugp_build_bvh.argtypes = [vp, C.POINTER(_Scene), C.c_float]
        L.ugp_refit_bvh.argtypes = [vp, C.POINTER(_Scene)]
        L.ugp_transmittance.argtypes = [vp, i64, vp, vp, vp, vp]
        L.ugp_sample_collision.argtypes = [vp, i64, vp, vp, vp, vp, vp]
        L.ugp_sample_collision_noalloc.argtypes = [vp, i64, vp, vp, vp, vp, vp]
        L.ugp_saturation.argtypes = [vp, i64, vp, vp, vp]
        L.ugp_ray_integral.argtypes = [vp, i64, vp, vp, vp]
        L.ugp_philox.argtypes = [vp, i64, vp, C.c_uint64, vp]
        L.ugp_emitter_query.argtypes = [vp, i64, vp, vp, vp, vp]
        L.ugp_render.argtypes = [vp, C.POINTER(_Camera), C.POINTER(_Params), vp, vp]
        L.ugp_render_albedo_grad.argtypes = [vp, C.POINTER(_Camera), C.POINTER(_Params), vp, vp, vp]
        L.ugp_render_roughness_grad.argtypes = [vp, C.POINTER(_Camera), C.POINTER(_Params), vp, vp, vp]
        L.ugp_render_density_grad.argtypes = [vp, C.POINTER(_Camera), C.POINTER(_Params), vp, vp, vp]
        L.ugp_render_grads.argtypes = [vp, C.POINTER(_Camera), C.POINTER(_Params), vp, vp, vp, vp, vp]
        L.ugp_sync.argtypes = [vp]
        L.ugp_set_profiling.argtypes = [vp, C.c_int]
        L.ugp_set_path_pool.argtypes = [vp, C.c_int64]
        L.ugp_set_tail_paths.argtypes = [vp, C.c_int64]
        L.ugp_trace_counts.argtypes = [vp, C.c_int, i64, vp, vp, vp, vp, vp]
        L.ugp_get_render_stats.argtypes = [vp, C.POINTER(_Stats)]
        L.ugp_nrc_num_params.argtypes = []
        L.ugp_nrc_set_weights.argtypes = [vp, vp]
        L.ugp_nrc_get_weights.argtypes = [vp, vp]
        L.ugp_nrc_encode.argtypes = [vp, i64, vp, vp, vp]
        L.ugp_nrc_forward.argtypes = [vp, i64, vp, C.c_int32, vp, vp]
        L.ugp_nrc_train_step.argtypes = [vp, i64, vp, C.c_int32, vp, vp, C.c_float, vp, vp]
        L.ugp_nrc_records.argtypes = [vp, i64, vp, vp, C.POINTER(C.c_int64)]
        L.ugp_accum_cdf.argtypes = [vp, vp, i64, vp, vp, vp, C.c_float, vp, vp, vp]
        L.ugp_camera_rays.argtypes = [vp, vp, C.c_uint64, i64, vp]
        L.ugp_sggx_phase.argtypes = [vp, i64, vp, vp, vp, vp, vp]
        L.ugp_rf_render.argtypes = [vp, vp, i64, vp, vp, vp, C.c_float, vp, vp, vp]
        L.ugp_accum_cdf_backward.argtypes = [vp, vp, i64, vp, vp, vp, vp]
        L.ugp_rf_render_backward.argtypes = [vp, vp, i64, vp, vp, vp, vp]
        L.ugp_exp_transmittance.argtypes = [vp, i64, vp, vp, vp]
        L.ugp_exp_sample_collision.argtypes = [vp, i64, vp, vp, C.c_uint64, vp, vp]
        L.ugp_fit_adam.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, vp, vp, C.c_int32, C.POINTER(C.c_float),
                                   C.c_float]
        L.ugp_status_string.argtypes = [C.c_int]
        L.ugp_status_string.restype = C.c_char_p
        for name in EXPORTS:
            if name != "ugp_status_string":
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(call: str, code: int):
    if code != 0:
        raise UGPError(call, code)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _render_params(params: dict):
    """ugp_render_params from a dict (defaults: 1 spp, depth 4, seed 0, no cache)."""
    p = _Params()
    p.spp = int(params.get("spp", 1))
    p.max_depth = int(params.get("max_depth", 4))
    p.seed = int(params.get("seed", 0))
    p.sample_offset = int(params.get("sample_offset", 0))
    env = params.get("env_radiance", (0.0, 0.0, 0.0))
    for i in range(3):
        p.env_radiance[i] = float(env[i])
    p.mis_mode = int(params.get("mis_mode", 0))
    p.nrc_mode = int(params.get("nrc_mode", 0))
    p.nrc_terminate_after = int(params.get("nrc_terminate_after", 2))
    p.nrc_train_records = int(params.get("nrc_train_records", 65536))
    p.nrc_lr = float(params.get("nrc_lr", 0.0))
    box = params.get("nrc_box", None)
    for i in range(6):
        p.nrc_box[i] = 0.0 if box is None else float(box[i])
    p.nrc_train_steps = int(params.get("nrc_train_steps", 1))
    p.nrc_radiance_scale = float(params.get("nrc_radiance_scale", 0.0))
    p.nrc_target_clamp = float(params.get("nrc_target_clamp", 0.0))
    p.transport = int(params.get("transport", 0))
    return p


class Context:
    """A libugp context bound to one GPU and a HIP stream (torch's current
    stream by default).  Owns the packed scene and the BVH."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        self._stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        _check("ugp_create", lib().ugp_create(device, C.c_void_p(self._stream.cuda_stream), C.byref(h)))
        self.h = h
        self.n = 0

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().ugp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _dev(self, a, dtype, shape=None):
        t = self.torch.as_tensor(a)
        t = t.to(device=self.device, dtype=dtype).contiguous()
        if shape is not None:
            assert tuple(t.shape) == tuple(shape), (t.shape, shape)
        return t

    # ---- scene -----------------------------------------------------------
    def build_bvh(self, scene: dict, cutoff_eps: float = 0.01):
        """ugp_build_bvh: pack the primitives and build the hierarchy."""
        return self._scene_call(scene, lambda s: ("ugp_build_bvh", lib().ugp_build_bvh(self.h, C.byref(s),
                                                                                        float(cutoff_eps))))

    def refit_bvh(self, scene: dict):
        """ugp_refit_bvh: new parameters for the built scene's primitives (same
        n), the hierarchy refitted in its topology."""
        return self._scene_call(scene, lambda s: ("ugp_refit_bvh", lib().ugp_refit_bvh(self.h, C.byref(s))))

    def _scene_call(self, scene: dict, call):
        torch = self.torch
        n = int(np.asarray(scene["mean"]).shape[0]) if not torch.is_tensor(scene["mean"]) else scene["mean"].shape[0]
        t = {
            "mean": self._dev(scene["mean"], torch.float32, (n, 3)),
            "scale": self._dev(scene["scale"], torch.float32, (n, 3)),
            "rotation": self._dev(scene["rotation"], torch.float32, (n, 4)),
            "density": self._dev(scene["density"], torch.float32, (n,)),
            "albedo": self._dev(scene["albedo"], torch.float32, (n, 3)),
            "roughness": self._dev(scene["roughness"], torch.float32, (n,)),
            "emission": self._dev(scene["emission"], torch.float32, (n, 3)),
            "material": self._dev(scene["material"], torch.int32, (n,)),
        }
        for key, w in (("sggx", 6), ("metallic", None)):
            if scene.get(key) is not None:
                t[key] = self._dev(scene[key], torch.float32, (n, w) if w else (n,))
        s = _Scene(n, *[t[k].data_ptr() for k in ("mean", "scale", "rotation", "density", "albedo",
                                                  "roughness", "emission", "material")],
                   *[t[k].data_ptr() if k in t else None for k in ("sggx", "metallic")])
        _check(*call(s))
        self.n = n
        self._scene_t, self._scene_s = t, s  # the parameters the hierarchy was built from
        self.build_id = getattr(self, "build_id", 0) + 1
        return self

    # ---- per-ray queries --------------------------------------------------
    def _rays(self, rays):
        r = self._dev(rays, self.torch.float32)
        assert r.ndim == 2 and r.shape[1] == 8
        return r

    def _excl(self, exclude, n):
        return None if exclude is None else self._dev(exclude, self.torch.int32, (n,))

    def transmittance(self, rays, exclude=None, want_F: bool = False):
        """ugp_transmittance -> (T, F or None)"""
        r = self._rays(rays)
        n = r.shape[0]
        e = self._excl(exclude, n)
        T = self.torch.empty(n, device=self.device, dtype=self.torch.float32)
        F = self.torch.empty_like(T) if want_F else None
        _check("ugp_transmittance", lib().ugp_transmittance(self.h, n, _ptr(r), _ptr(e), _ptr(T), _ptr(F)))
        return T, F

    def sample_collision(self, rays, u, exclude=None):
        """ugp_sample_collision -> (prim int32, t float32)"""
        r = self._rays(rays)
        n = r.shape[0]
        e = self._excl(exclude, n)
        uu = self._dev(u, self.torch.float32, (n,))
        prim = self.torch.empty(n, device=self.device, dtype=self.torch.int32)
        t = self.torch.empty(n, device=self.device, dtype=self.torch.float32)
        _check("ugp_sample_collision",
               lib().ugp_sample_collision(self.h, n, _ptr(r), _ptr(e), _ptr(uu), _ptr(prim), _ptr(t)))
        return prim, t

    def sample_collision_noalloc(self, rays, u, exclude=None, prim=None, t=None):
        """ugp_sample_collision_noalloc -> (prim int32, t float32): the
        allocation-free variant (the library allocates nothing; the outputs
        are the caller's, allocated here unless given)"""
        r = self._rays(rays)
        n = r.shape[0]
        e = self._excl(exclude, n)
        uu = self._dev(u, self.torch.float32, (n,))
        if prim is None:
            prim = self.torch.empty(n, device=self.device, dtype=self.torch.int32)
        if t is None:
            t = self.torch.empty(n, device=self.device, dtype=self.torch.float32)
        assert prim.dtype == self.torch.int32 and prim.numel() == n and prim.is_contiguous()
        assert t.dtype == self.torch.float32 and t.numel() == n and t.is_contiguous()
        _check("ugp_sample_collision_noalloc",
               lib().ugp_sample_collision_noalloc(self.h, n, _ptr(r), _ptr(e), _ptr(uu), _ptr(prim), _ptr(t)))
        return prim, t

    def ray_integral(self, rays, prim):
        """ugp_ray_integral -> I float32 [n]: the integral of primitive prim[i]'s
        kernel along ray i's clipped chord (test hook)"""
        r = self._rays(rays)
        n = r.shape[0]
        pr = self._dev(prim, self.torch.int32, (n,))
        out = self.torch.empty(n, device=self.device, dtype=self.torch.float32)
        _check("ugp_ray_integral", lib().ugp_ray_integral(self.h, n, _ptr(r), _ptr(pr), _ptr(out)))
        return out

    def philox(self, counters, key: int):
        """ugp_philox -> uint32 words [n, 4] (as int32 storage) of Philox4x32-10
        of counters [n, 4] under key (test hook)"""
        c = self.torch.as_tensor(np.ascontiguousarray(np.asarray(counters, np.uint32)).view(np.int32))
        c = c.to(self.device).contiguous()
        assert c.ndim == 2 and c.shape[1] == 4
        out = self.torch.empty_like(c)
        _check("ugp_philox", lib().ugp_philox(self.h, c.shape[0], _ptr(c), int(key), _ptr(out)))
        return out

    def saturation(self, rays, exclude=None):
        """ugp_saturation -> t_sat float32"""
        r = self._rays(rays)
        n = r.shape[0]
        e = self._excl(exclude, n)
        t = self.torch.empty(n, device=self.device, dtype=self.torch.float32)
        _check("ugp_saturation", lib().ugp_saturation(self.h, n, _ptr(r), _ptr(e), _ptr(t)))
        return t

    def emitter_query(self, rays, target, exclude=None):
        """ugp_emitter_query -> 1/2 I_target(a, min(b, t_sat)) float32"""
        r = self._rays(rays)
        n = r.shape[0]
        e = self._excl(exclude, n)
        tg = self._dev(target, self.torch.int32, (n,))
        out = self.torch.empty(n, device=self.device, dtype=self.torch.float32)
        _check("ugp_emitter_query", lib().ugp_emitter_query(self.h, n, _ptr(r), _ptr(e), _ptr(tg), _ptr(out)))
        return out

    def sggx_phase(self, sggx, dirs, u, base=None):
        """ugp_sggx_phase -> float32 [n, 12]: f_p estimate (rgb), approximate
        pdf, sampled direction (3), its weight (rgb), its approximate pdf, ok.
        base [n, 5] (albedo rgb, roughness, metallic) selects material 3; None
        the Lambertian base of unit albedo (material 2)."""
        torch = self.torch
        d = self._dev(dirs, torch.float32)
        n = d.shape[0]
        g = self._dev(sggx, torch.float32, (n, 6))
        uu = self._dev(u, torch.float32, (n, 12))
        b = None if base is None else self._dev(base, torch.float32, (n, 5))
        d = d.reshape(n, 6)
        out = torch.empty((n, 12), device=self.device, dtype=torch.float32)
        _check("ugp_sggx_phase", lib().ugp_sggx_phase(self.h, n, _ptr(g), _ptr(b), _ptr(d), _ptr(uu), _ptr(out)))
        return out

    def trace_counts(self, mode: int, rays, u=None, target=None, exclude=None):
        """ugp_trace_counts -> int32 [n, 4] (nodes, prims, reloads, rounds) per ray"""
        r = self._rays(rays)
        n = r.shape[0]
        e = self._excl(exclude, n)
        uu = None if u is None else self._dev(u, self.torch.float32, (n,))
        tg = None if target is None else self._dev(target, self.torch.int32, (n,))
        out = self.torch.zeros((n, 4), device=self.device, dtype=self.torch.int32)
        _check("ugp_trace_counts", lib().ugp_trace_counts(self.h, int(mode), n, _ptr(r), _ptr(e), _ptr(uu),
                                                          _ptr(tg), _ptr(out)))
        return out

    # ---- exponential variant ----------------------------------------------
    def exp_transmittance(self, rays, exclude=None):
        """ugp_exp_transmittance -> T = exp(-sum_k I_k) float32 [n]."""
        r = self._rays(rays)
        n = r.shape[0]
        e = self._excl(exclude, n)
        T = self.torch.empty(n, device=self.device, dtype=self.torch.float32)
        _check("ugp_exp_transmittance", lib().ugp_exp_transmittance(self.h, n, _ptr(r), _ptr(e), _ptr(T)))
        return T

    def exp_sample_collision(self, rays, seed: int, exclude=None):
        """ugp_exp_sample_collision -> (prim int32, t float32) by analog decomposition tracking."""
        r = self._rays(rays)
        n = r.shape[0]
        e = self._excl(exclude, n)
        prim = self.torch.empty(n, device=self.device, dtype=self.torch.int32)
        t = self.torch.empty(n, device=self.device, dtype=self.torch.float32)
        _check("ugp_exp_sample_collision",
               lib().ugp_exp_sample_collision(self.h, n, _ptr(r), _ptr(e), int(seed), _ptr(prim), _ptr(t)))
        return prim, t

    # ---- differentiation (transmittance optimisation) ---------------------
    def accum_cdf(self, rays, target=None, exclude=None, loss_scale: float = 1.0, want_C: bool = True,
                  loss=None, grad=None):
        """ugp_accum_cdf -> C (float32 [n]) or None.  With target, adds
        loss_scale * sum (C - target)^2 into `loss` (device float32 [1]) and its
        gradient into `grad` (float32 [n_prims, 11]: mean, scale, rotation,
        density), each when given; the scene is the one of the last build_bvh."""
        torch = self.torch
        r = self._rays(rays)
        n = r.shape[0]
        e = self._excl(exclude, n)
        tg = None if target is None else self._dev(target, torch.float32, (n,))
        C_out = torch.empty(n, device=self.device, dtype=torch.float32) if want_C else None
        if grad is not None:
            assert grad.dtype == torch.float32 and tuple(grad.shape) == (self.n, 11) and grad.is_contiguous()
        if loss is not None:
            assert loss.dtype == torch.float32 and loss.numel() >= 1
        sp = C.byref(self._scene_s) if grad is not None else None
        _check("ugp_accum_cdf", lib().ugp_accum_cdf(self.h, sp, n, _ptr(r), _ptr(e), _ptr(tg), float(loss_scale),
                                                    _ptr(C_out), _ptr(loss), _ptr(grad)))
        return C_out

    def rf_render(self, rays, target=None, exclude=None, loss_scale: float = 1.0, want_L: bool = True,
                  loss=None, grad=None):
        """ugp_rf_render -> L (float32 [n, 3]) or None.  With target ([n, 3]),
        adds loss_scale * sum |L - target|^2 into `loss` and its gradient into
        `grad` (float32 [n_prims, 14]: mean, scale, rotation, density,
        emission), each when given; the scene is the one of the last build_bvh."""
        torch = self.torch
        r = self._rays(rays)
        n = r.shape[0]
        e = self._excl(exclude, n)
        tg = None if target is None else self._dev(target, torch.float32, (n, 3))
        L_out = torch.empty((n, 3), device=self.device, dtype=torch.float32) if want_L else None
        if grad is not None:
            assert grad.dtype == torch.float32 and tuple(grad.shape) == (self.n, 14) and grad.is_contiguous()
        if loss is not None:
            assert loss.dtype == torch.float32 and loss.numel() >= 1
        sp = C.byref(self._scene_s) if grad is not None else None
        _check("ugp_rf_render", lib().ugp_rf_render(self.h, sp, n, _ptr(r), _ptr(e), _ptr(tg), float(loss_scale),
                                                    _ptr(L_out), _ptr(loss), _ptr(grad)))
        return L_out

    def accum_cdf_backward(self, rays, dC, grad, exclude=None):
        """ugp_accum_cdf_backward: grad (float32 [n_prims, 11]) += sum_i dC_i
        dC_i/d(mean, scale, rotation, density), t_sat held fixed; the scene is
        the one of the last build_bvh."""
        return self._vjp("ugp_accum_cdf_backward", rays, dC, grad, exclude, 1, 11)

    def rf_render_backward(self, rays, dL, grad, exclude=None):
        """ugp_rf_render_backward: grad (float32 [n_prims, 14]) += sum_i dL_i .
        dL_i/d(mean, scale, rotation, density, emission), dL [n, 3]."""
        return self._vjp("ugp_rf_render_backward", rays, dL, grad, exclude, 3, 14)

    def _vjp(self, name, rays, d, grad, exclude, nc, ng):
        torch = self.torch
        r = self._rays(rays)
        n = r.shape[0]
        e = self._excl(exclude, n)
        d = self._dev(d, torch.float32, (n,) if nc == 1 else (n, nc))
        assert grad.dtype == torch.float32 and tuple(grad.shape) == (self.n, ng) and grad.is_contiguous()
        _check(name, getattr(lib(), name)(self.h, C.byref(self._scene_s), n, _ptr(r), _ptr(e), _ptr(d),
                                          _ptr(grad)))
        return grad

    def camera_rays(self, cam: dict, seed: int = 0, sample: int = 0):
        """ugp_camera_rays -> float32 [height * width, 8] jittered pinhole rays."""
        c = _camera(cam)
        rays = self.torch.empty((cam["width"] * cam["height"], 8), device=self.device, dtype=self.torch.float32)
        _check("ugp_camera_rays", lib().ugp_camera_rays(self.h, C.byref(c), int(seed), int(sample), _ptr(rays)))
        return rays

    def fit_adam(self, params: dict, grad, m, v, step: int, lr=(1e-4, 1e-2, 2e-5, 1e-4, 1e-2),
                 min_scale: float = 1e-6, emission: bool = False):
        """ugp_fit_adam: one Adam step on params (device float32 tensors mean,
        scale, rotation, density, and with emission=True the emission; updated
        in place); lr = rates of the means, the log scales, the rotations, the
        densities (and the emissions); clamps and renormalised rotations."""
        n = params["mean"].shape[0]
        keys = ("mean", "scale", "rotation", "density") + (("emission",) if emission else ())
        for k in keys:
            assert params[k].is_contiguous() and params[k].dtype == self.torch.float32
        lr = list(lr) + [0.0] * (5 - len(lr))
        rates = (C.c_float * 5)(*[float(x) for x in lr[:5]])
        _check("ugp_fit_adam", lib().ugp_fit_adam(self.h, n, _ptr(params["mean"]), _ptr(params["scale"]),
                                                  _ptr(params["rotation"]), _ptr(params["density"]),
                                                  _ptr(params["emission"]) if emission else None, _ptr(grad),
                                                  _ptr(m), _ptr(v), int(step), rates, float(min_scale)))

    # ---- path tracing -----------------------------------------------------
    def render(self, cam: dict, params: dict, sum_rgb=None, sumsq_rgb=None):
        """ugp_render: adds this call's per-pixel sums of path radiance (and of
        its square) into sum_rgb / sumsq_rgb [H, W, 3] float32 (allocated if
        None) and returns them."""
        torch = self.torch
        W, H = int(cam["width"]), int(cam["height"])
        if sum_rgb is None:
            sum_rgb = torch.zeros((H, W, 3), device=self.device, dtype=torch.float32)
        if sumsq_rgb is None and params.get("want_sumsq", True):
            sumsq_rgb = torch.zeros((H, W, 3), device=self.device, dtype=torch.float32)
        c = _camera(cam)
        p = _render_params(params)
        _check("ugp_render", lib().ugp_render(self.h, C.byref(c), C.byref(p), _ptr(sum_rgb), _ptr(sumsq_rgb)))
        return sum_rgb, sumsq_rgb

    def render_albedo_grad(self, cam: dict, params: dict, d_image, grad, sum_rgb=None):
        """ugp_render_albedo_grad: grad (float32 [n_prims, 3]) += dLoss/dalbedo
        for d_image = dLoss/d(mean image) [H, W, 3]; the forward pass's
        per-pixel sums are added into sum_rgb when given.  Returns grad."""
        torch = self.torch
        W, H = int(cam["width"]), int(cam["height"])
        d = self._dev(d_image, torch.float32, (H, W, 3))
        assert grad.dtype == torch.float32 and tuple(grad.shape) == (self.n, 3) and grad.is_contiguous()
        if sum_rgb is not None:
            assert sum_rgb.dtype == torch.float32 and tuple(sum_rgb.shape) == (H, W, 3) and sum_rgb.is_contiguous()
        c = _camera(cam)
        p = _render_params(params)
        _check("ugp_render_albedo_grad", lib().ugp_render_albedo_grad(self.h, C.byref(c), C.byref(p), _ptr(d),
                                                                      _ptr(grad), _ptr(sum_rgb)))
        return grad

    def render_roughness_grad(self, cam: dict, params: dict, d_image, grad, sum_rgb=None):
        """ugp_render_roughness_grad: grad (float32 [n_prims]) += an unbiased
        estimate of dLoss/droughness for d_image = dLoss/d(mean image)
        [H, W, 3]; sum_rgb as in render_albedo_grad.  Returns grad."""
        torch = self.torch
        W, H = int(cam["width"]), int(cam["height"])
        d = self._dev(d_image, torch.float32, (H, W, 3))
        assert grad.dtype == torch.float32 and tuple(grad.shape) == (self.n,) and grad.is_contiguous()
        if sum_rgb is not None:
            assert sum_rgb.dtype == torch.float32 and tuple(sum_rgb.shape) == (H, W, 3) and sum_rgb.is_contiguous()
        c = _camera(cam)
        p = _render_params(params)
        _check("ugp_render_roughness_grad", lib().ugp_render_roughness_grad(self.h, C.byref(c), C.byref(p),
                                                                            _ptr(d), _ptr(grad), _ptr(sum_rgb)))
        return grad

    def render_grads(self, cam: dict, params: dict, d_image, grad_albedo=None, grad_roughness=None,
                     grad_density=None, sum_rgb=None):
        """ugp_render_grads: the albedo ([n_prims, 3]), roughness ([n_prims])
        and density ([n_prims]) gradients that are given (float32, added to)
        from one forward pass and one replay; sum_rgb as in
        render_albedo_grad.  Returns (grad_albedo, grad_roughness,
        grad_density)."""
        torch = self.torch
        W, H = int(cam["width"]), int(cam["height"])
        d = self._dev(d_image, torch.float32, (H, W, 3))
        for g, shape in ((grad_albedo, (self.n, 3)), (grad_roughness, (self.n,)), (grad_density, (self.n,))):
            if g is not None:
                assert g.dtype == torch.float32 and tuple(g.shape) == shape and g.is_contiguous()
        if sum_rgb is not None:
            assert sum_rgb.dtype == torch.float32 and tuple(sum_rgb.shape) == (H, W, 3) and sum_rgb.is_contiguous()
        c = _camera(cam)
        p = _render_params(params)
        _check("ugp_render_grads", lib().ugp_render_grads(self.h, C.byref(c), C.byref(p), _ptr(d), _ptr(grad_albedo),
                                                          _ptr(grad_roughness), _ptr(grad_density), _ptr(sum_rgb)))
        return grad_albedo, grad_roughness, grad_density

    def render_density_grad(self, cam: dict, params: dict, d_image, grad, sum_rgb=None):
        """ugp_render_density_grad: grad (float32 [n_prims]) += an unbiased
        estimate of dLoss/ddensity for d_image = dLoss/d(mean image)
        [H, W, 3]; sum_rgb as in render_albedo_grad.  Returns grad."""
        torch = self.torch
        W, H = int(cam["width"]), int(cam["height"])
        d = self._dev(d_image, torch.float32, (H, W, 3))
        assert grad.dtype == torch.float32 and tuple(grad.shape) == (self.n,) and grad.is_contiguous()
        if sum_rgb is not None:
            assert sum_rgb.dtype == torch.float32 and tuple(sum_rgb.shape) == (H, W, 3) and sum_rgb.is_contiguous()
        c = _camera(cam)
        p = _render_params(params)
        _check("ugp_render_density_grad", lib().ugp_render_density_grad(self.h, C.byref(c), C.byref(p), _ptr(d),
                                                                        _ptr(grad), _ptr(sum_rgb)))
        return grad

    def sync(self):
        _check("ugp_sync", lib().ugp_sync(self.h))

    def set_profiling(self, level: int):
        """ugp_set_profiling: 0 off, 1 time kernels with HIP events, 2 also count traversal work."""
        _check("ugp_set_profiling", lib().ugp_set_profiling(self.h, int(level)))

    def set_path_pool(self, slots: int):
        """ugp_set_path_pool: path slots of later renders (0: every path of a chunk in flight)."""
        _check("ugp_set_path_pool", lib().ugp_set_path_pool(self.h, int(slots)))

    def set_tail_paths(self, paths: int):
        """ugp_set_tail_paths: live paths at or below which a chunk's last bounces run in one kernel (0: never)."""
        _check("ugp_set_tail_paths", lib().ugp_set_tail_paths(self.h, int(paths)))

    def render_stats(self) -> dict:
        """ugp_get_render_stats of the last render (synchronises)."""
        st = _Stats()
        _check("ugp_get_render_stats", lib().ugp_get_render_stats(self.h, C.byref(st)))
        d = {}
        for name, _ in _Stats._fields_:
            v = getattr(st, name)
            d[name] = list(v) if name.startswith("cat_") else v
        d["rays"] = d["collision_rays"] + d["light_rays"] + d["env_rays"]
        return d

    # ---- neural radiance cache -------------------------------------------
    def _box(self, box):
        if box is None:
            return None
        b = (C.c_float * 6)(*[float(v) for v in box])
        return b

    def nrc_set_weights(self, w):
        """ugp_nrc_set_weights: float32 [P] master weights (resets Adam)."""
        t = self._dev(w, self.torch.float32, (nrc_num_params(),))
        _check("ugp_nrc_set_weights", lib().ugp_nrc_set_weights(self.h, _ptr(t)))

    def nrc_get_weights(self):
        out = self.torch.empty(nrc_num_params(), device=self.device, dtype=self.torch.float32)
        _check("ugp_nrc_get_weights", lib().ugp_nrc_get_weights(self.h, _ptr(out)))
        return out

    def nrc_encode(self, inputs, box=None):
        """ugp_nrc_encode: float32 [n,16] -> [n,96]"""
        x = self._dev(inputs, self.torch.float32)
        assert x.ndim == 2 and x.shape[1] == 16
        out = self.torch.empty((x.shape[0], 96), device=self.device, dtype=self.torch.float32)
        _check("ugp_nrc_encode", lib().ugp_nrc_encode(self.h, x.shape[0], _ptr(x), self._box(box), _ptr(out)))
        return out

    def nrc_forward(self, x, box=None):
        """ugp_nrc_forward: x float32 [n,16] (inputs) or [n,96] (features) -> [n,3]"""
        t = self._dev(x, self.torch.float32)
        assert t.ndim == 2 and t.shape[1] in (16, 96)
        kind = 0 if t.shape[1] == 16 else 1
        y = self.torch.empty((t.shape[0], 3), device=self.device, dtype=self.torch.float32)
        _check("ugp_nrc_forward", lib().ugp_nrc_forward(self.h, t.shape[0], _ptr(t), kind, self._box(box), _ptr(y)))
        return y

    def nrc_train_step(self, x, targets, lr: float = 1e-3, box=None, want_grad: bool = False):
        """ugp_nrc_train_step -> (loss tensor [1], gradient [P] or None)"""
        t = self._dev(x, self.torch.float32)
        assert t.ndim == 2 and t.shape[1] in (16, 96)
        kind = 0 if t.shape[1] == 16 else 1
        tg = self._dev(targets, self.torch.float32, (t.shape[0], 3))
        loss = self.torch.empty(1, device=self.device, dtype=self.torch.float32)
        g = self.torch.empty(nrc_num_params(), device=self.device, dtype=self.torch.float32) if want_grad else None
        _check("ugp_nrc_train_step", lib().ugp_nrc_train_step(self.h, t.shape[0], _ptr(t), kind, self._box(box),
                                                              _ptr(tg), float(lr), _ptr(loss), _ptr(g)))
        return loss, g

    def nrc_records(self, cap: int):
        """ugp_nrc_records -> (records [n,24], targets [n,3]) of the last training pass"""
        rec = self.torch.empty((cap, 24), device=self.device, dtype=self.torch.float32)
        tgt = self.torch.empty((cap, 3), device=self.device, dtype=self.torch.float32)
        n = C.c_int64(0)
        _check("ugp_nrc_records", lib().ugp_nrc_records(self.h, int(cap), _ptr(rec), _ptr(tgt), C.byref(n)))
        return rec[:n.value], tgt[:n.value]


def nrc_num_params() -> int:
    """ugp_nrc_num_params"""
    return int(lib().ugp_nrc_num_params())
