"""FP64 CPU oracle for the Gaussian-primitive path tracer -- TEST INFRASTRUCTURE.

This package is the plain, slow reference the GPU library is checked against.
Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import it.  It shares no code with the HIP library and never
calls it; the product path must not import it.

The arithmetic lives in ``ugp_oracle.c`` (double precision, libm, pthreads);
this module only compiles it with gcc and marshals numpy arrays through ctypes.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ugp_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle into ``oracle/liborc.so`` (gcc, -O2, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra",
               "-Wno-unused-parameter", "-D_GNU_SOURCE", _SRC, "-o", tmp, "-lm", "-lpthread"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Camera(C.Structure):
    _fields_ = [("origin", C.c_double * 3), ("target", C.c_double * 3), ("up", C.c_double * 3),
                ("vfov_deg", C.c_double), ("width", C.c_int32), ("height", C.c_int32)]


class _Params(C.Structure):
    _fields_ = [("spp", C.c_int32), ("max_depth", C.c_int32), ("seed", C.c_uint64),
                ("sample_offset", C.c_int64), ("env_radiance", C.c_double * 3),
                ("mis_mode", C.c_int32), ("nrc_mode", C.c_int32), ("nrc_terminate_after", C.c_int32),
                ("nrc_train_frac", C.c_double), ("nrc_weights", C.c_void_p), ("nrc_box", C.c_double * 6),
                ("transport", C.c_int32)]


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct)) if a is not None else None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        vp = C.c_void_p
        L.orc_scene_create.argtypes = [C.c_int64] + [vp] * 8 + [C.c_double, C.POINTER(vp)]
        L.orc_scene_destroy.argtypes = [vp]
        L.orc_scene_build_bvh.argtypes = [vp]
        L.orc_cutoff_radius.argtypes = [vp]
        L.orc_cutoff_radius.restype = C.c_double
        L.orc_prim_frame.argtypes = [vp, C.c_int64, vp, vp, vp, vp]
        L.orc_chord.argtypes = [vp, C.c_int64, vp, vp]
        L.orc_ray_integral.argtypes = [vp, C.c_int64, vp, C.c_double, C.c_double]
        L.orc_ray_integral.restype = C.c_double
        L.orc_transmittance.argtypes = [vp, C.c_int64, vp, vp, C.c_int, vp, vp]
        L.orc_saturation.argtypes = [vp, C.c_int64, vp, vp, C.c_int, vp]
        L.orc_F_at.argtypes = [vp, C.c_int64, vp, vp, vp, C.c_int, vp]
        L.orc_rf_radiance.argtypes = [vp, C.c_int64, vp, vp, vp, C.c_int, vp]
        L.orc_exp_transmittance.argtypes = [vp, C.c_int64, vp, vp, C.c_int, vp]
        L.orc_exp_sample.argtypes = [vp, C.c_int64, vp, vp, C.c_uint64, C.c_int, vp, vp, vp]
        L.orc_sample_collision.argtypes = [vp, C.c_int64, vp, vp, vp, C.c_int, vp, vp, vp, vp, vp]
        L.orc_emitter_query.argtypes = [vp, C.c_int64, vp, vp, vp, C.c_int, vp]
        L.orc_light_pdf.argtypes = [vp, C.c_int64, vp, vp]
        L.orc_light_pdf.restype = C.c_double
        L.orc_light_dir.argtypes = [vp, C.c_int64, vp, vp, vp]
        L.orc_light_dir.restype = C.c_int
        L.orc_phase_eval.argtypes = [C.c_int, vp, C.c_double, vp, vp, vp, vp, vp]
        L.orc_phase_sample.argtypes = [C.c_int, vp, C.c_double, vp, vp, C.c_double, C.c_double,
                                       vp, vp, vp]
        L.orc_sggx_phase_quad.argtypes = [vp, vp, vp, C.c_int, C.c_int]
        L.orc_sggx_phase_quad.restype = C.c_double
        L.orc_sggx_pdf_approx.argtypes = [vp, vp]
        L.orc_sggx_pdf_approx.restype = C.c_double
        L.orc_sggx_eval_n.argtypes = [vp, C.c_int64, vp, vp, C.c_int, vp]
        L.orc_sggx_sample_vndf_n.argtypes = [vp, vp, C.c_int64, vp, vp]
        L.orc_sggx_phase_est_n.argtypes = [vp, vp, vp, C.c_int64, vp, vp]
        L.orc_sggx_sample_dir_n.argtypes = [vp, vp, C.c_int64, vp, vp]
        L.orc_scene_set_sggx.argtypes = [vp, vp]
        L.orc_scene_set_metallic.argtypes = [vp, vp]
        L.orc_disney_spec_prob.argtypes = [vp, C.c_double]
        L.orc_disney_spec_prob.restype = C.c_double
        L.orc_disney_base.argtypes = [vp, C.c_double, C.c_double, vp, vp, vp, vp, vp]
        L.orc_sggx_disney_est.argtypes = [vp, vp, C.c_double, C.c_double, vp, vp, vp, vp]
        L.orc_sggx_disney_sample.argtypes = [vp, vp, C.c_double, C.c_double, vp, C.c_double, C.c_double, vp,
                                             vp, vp]
        L.orc_sggx_disney_sample.restype = C.c_int
        L.orc_sggx_roughened.argtypes = [vp, C.c_double, vp]
        L.orc_sggx_disney_pdf_approx.argtypes = [vp, vp, C.c_double, C.c_double, vp, vp]
        L.orc_sggx_disney_pdf_approx.restype = C.c_double
        L.orc_sggx_disney_quad.argtypes = [vp, vp, C.c_double, C.c_double, vp, vp, C.c_int, C.c_int, vp]
        L.orc_camera_rays.argtypes = [C.POINTER(_Camera), C.c_uint64, C.c_uint32, vp]
        L.orc_render.argtypes = [vp, C.POINTER(_Camera), C.POINTER(_Params), C.c_int64, vp,
                                 C.c_int, vp, vp]
        L.orc_render.restype = C.c_int64
        L.orc_path_radiance.argtypes = [vp, C.POINTER(_Camera), C.POINTER(_Params), C.c_uint32,
                                        C.c_uint32, vp]
        L.orc_path_records.argtypes = [vp, C.POINTER(_Camera), C.POINTER(_Params), C.c_uint32, C.c_uint32,
                                       vp, C.c_int, vp]
        L.orc_path_records.restype = C.c_int
        L.orc_philox4x32_10.argtypes = [vp, vp, vp]
        L.orc_philox4x32_10_batch.argtypes = [C.c_int64, vp, vp, vp]
        L.orc_nrc_num_params.restype = C.c_int
        L.orc_nrc_encode.argtypes = [C.c_int64, vp, vp, vp, vp]
        L.orc_nrc_forward.argtypes = [C.c_int64, vp, vp, vp]
        L.orc_nrc_loss_grad.argtypes = [C.c_int64, vp, vp, vp, vp]
        L.orc_nrc_loss_grad.restype = C.c_double
        L.orc_nrc_adam.argtypes = [C.c_int64, vp, vp, vp, vp, C.c_int, C.c_double, C.c_double, C.c_double,
                                   C.c_double]
        L.orc_philox4x64_10.argtypes = [vp, vp, vp]
        _lib = L
    return _lib


def _addr(a):
    return None if a is None else a.ctypes.data


def philox4x32_10(ctr, key) -> np.ndarray:
    """Philox4x32-10 of one counter [4] or of counters [n, 4] under key [2]"""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    if c.ndim == 2:
        out = np.zeros_like(c)
        lib().orc_philox4x32_10_batch(c.shape[0], _addr(c), _addr(k), _addr(out))
        return out
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_addr(c), _addr(k), _addr(out))
    return out


def philox4x64_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().orc_philox4x64_10(_addr(c), _addr(k), _addr(out))
    return out


def _rays(rays):
    r = np.ascontiguousarray(rays, dtype=np.float32)
    assert r.ndim == 2 and r.shape[1] == 8
    return r


def _excl(exclude, n):
    if exclude is None:
        return None
    e = np.ascontiguousarray(exclude, dtype=np.int32)
    assert e.shape == (n,)
    return e


class Scene:
    """A scene held by the oracle (widened to float64 inside)."""

    def __init__(self, scene: dict, eps: float = 0.01, bvh: bool = True):
        self._keep = {}
        n = int(np.asarray(scene["mean"]).shape[0])
        fields = [("mean", np.float32, 3), ("scale", np.float32, 3), ("rotation", np.float32, 4),
                  ("density", np.float32, 1), ("albedo", np.float32, 3),
                  ("roughness", np.float32, 1), ("emission", np.float32, 3),
                  ("material", np.int32, 1)]
        ptrs = []
        for name, dt, w in fields:
            a = np.ascontiguousarray(scene[name], dtype=dt).reshape(n, w) if n else np.zeros((0, w), dt)
            self._keep[name] = a
            ptrs.append(_addr(a) if n else None)
        h = C.c_void_p()
        rc = lib().orc_scene_create(n, *ptrs, float(eps), C.byref(h))
        if rc != 0:
            raise ValueError("oracle rejected the scene")
        self.h = h
        self.n = n
        mats = self._keep["material"].reshape(-1)
        if scene.get("sggx") is not None:
            g = np.ascontiguousarray(scene["sggx"], dtype=np.float32).reshape(n, 6)
            self._keep["sggx"] = g
            if n and lib().orc_scene_set_sggx(self.h, _addr(g)) != 0:
                raise ValueError("oracle rejected the SGGX matrices (not positive definite)")
        elif n and bool((mats >= 2).any()):
            raise ValueError("materials 2 and 3 (SGGX microflakes) need scene['sggx']")
        if scene.get("metallic") is not None:
            mt = np.ascontiguousarray(scene["metallic"], dtype=np.float32).reshape(n)
            self._keep["metallic"] = mt
            if n and lib().orc_scene_set_metallic(self.h, _addr(mt)) != 0:
                raise ValueError("oracle rejected the metallic values (outside [0, 1])")
        self.use_bvh = 0
        if bvh:
            lib().orc_scene_build_bvh(self.h)
            self.use_bvh = 1

    def __del__(self):
        try:
            lib().orc_scene_destroy(self.h)
        except Exception:
            pass

    @property
    def cutoff_radius(self) -> float:
        return lib().orc_cutoff_radius(self.h)

    def prim_frame(self, k: int):
        M = np.zeros(9); n = np.zeros(3); lo = np.zeros(3); hi = np.zeros(3)
        lib().orc_prim_frame(self.h, int(k), _addr(M), _addr(n), _addr(lo), _addr(hi))
        return M.reshape(3, 3), n, lo, hi

    def chord(self, k: int, ray):
        r = np.ascontiguousarray(ray, dtype=np.float32).reshape(8)
        out = np.zeros(2)
        hit = lib().orc_chord(self.h, int(k), _addr(r), _addr(out))
        return (float(out[0]), float(out[1])) if hit else None

    def ray_integral(self, k: int, ray, x: float, y: float) -> float:
        r = np.ascontiguousarray(ray, dtype=np.float64).reshape(8)
        return lib().orc_ray_integral(self.h, int(k), _addr(r), float(x), float(y))

    def transmittance(self, rays, exclude=None, use_bvh=None):
        r = _rays(rays)
        n = r.shape[0]
        e = _excl(exclude, n)
        F = np.zeros(n); T = np.zeros(n)
        ub = self.use_bvh if use_bvh is None else int(use_bvh)
        lib().orc_transmittance(self.h, n, _addr(r), _addr(e), ub, _addr(F), _addr(T))
        return F, T

    def saturation(self, rays, exclude=None, use_bvh=None):
        r = _rays(rays)
        n = r.shape[0]
        e = _excl(exclude, n)
        t = np.zeros(n)
        ub = self.use_bvh if use_bvh is None else int(use_bvh)
        lib().orc_saturation(self.h, n, _addr(r), _addr(e), ub, _addr(t))
        return t

    def F_at(self, rays, t, exclude=None, use_bvh=None):
        """F(t) = 1/2 sum_k I_k(a_k, min(b_k, t)) per ray."""
        r = _rays(rays)
        n = r.shape[0]
        e = _excl(exclude, n)
        tt = np.ascontiguousarray(t, dtype=np.float64)
        F = np.zeros(n)
        ub = self.use_bvh if use_bvh is None else int(use_bvh)
        lib().orc_F_at(self.h, n, _addr(r), _addr(e), _addr(tt), ub, _addr(F))
        return F

    def accum_cdf(self, rays, exclude=None, tsat=None, use_bvh=None):
        """Accumulated free-flight CDF (Sec. 7.2, eq. accum_cdf): the sum of the
        primitives' free-flight probabilities, each chord clipped at the ray's
        saturating distance -- F at t_sat (at t1 when the ray never saturates).
        `tsat` may be given (held fixed, as the derivative of Sec. 7.2 takes
        it).  Returns (C, tsat)."""
        if tsat is None:
            tsat = self.saturation(rays, exclude, use_bvh)
        return self.F_at(rays, tsat, exclude, use_bvh), tsat

    def rf_radiance(self, rays, exclude=None, tsat=None, use_bvh=None):
        """Radiance-field mode (Sec. 8, eq. rf): per ray the sum of the
        primitives' free-flight probabilities up to the saturating distance
        times their emission.  `tsat` may be given (held fixed).  [n, 3]."""
        r = _rays(rays)
        n = r.shape[0]
        e = _excl(exclude, n)
        ts = None if tsat is None else np.ascontiguousarray(tsat, dtype=np.float64)
        L = np.zeros((n, 3))
        ub = self.use_bvh if use_bvh is None else int(use_bvh)
        lib().orc_rf_radiance(self.h, n, _addr(r), _addr(e), _addr(ts), ub, _addr(L))
        return L

    def exp_transmittance(self, rays, exclude=None, use_bvh=None):
        """Exponential variant (App. D, eq. exp_ff): T = exp(-sum_k I_k)."""
        r = _rays(rays)
        n = r.shape[0]
        e = _excl(exclude, n)
        T = np.zeros(n)
        ub = self.use_bvh if use_bvh is None else int(use_bvh)
        lib().orc_exp_transmittance(self.h, n, _addr(r), _addr(e), ub, _addr(T))
        return T

    def exp_sample(self, rays, seed: int, exclude=None, use_bvh=None):
        """Analog decomposition tracking of the exponential variant (App. D):
        (prim or -1, t or NaN, margin) per ray."""
        r = _rays(rays)
        n = r.shape[0]
        e = _excl(exclude, n)
        prim = np.zeros(n, np.int32)
        t = np.zeros(n)
        margin = np.zeros(n)
        ub = self.use_bvh if use_bvh is None else int(use_bvh)
        lib().orc_exp_sample(self.h, n, _addr(r), _addr(e), int(seed), ub, _addr(prim), _addr(t), _addr(margin))
        return prim, t, margin

    def sample_collision(self, rays, u, exclude=None, use_bvh=None):
        r = _rays(rays)
        n = r.shape[0]
        e = _excl(exclude, n)
        uu = np.ascontiguousarray(u, dtype=np.float64)
        assert uu.shape == (n,)
        prim = np.zeros(n, dtype=np.int32)
        t = np.zeros(n); F = np.zeros(n); ts = np.zeros(n); mg = np.zeros(n)
        ub = self.use_bvh if use_bvh is None else int(use_bvh)
        lib().orc_sample_collision(self.h, n, _addr(r), _addr(e), _addr(uu), ub, _addr(prim),
                                   _addr(t), _addr(F), _addr(ts), _addr(mg))
        return {"prim": prim, "t": t, "F": F, "tsat": ts, "margin": mg}

    def emitter_query(self, rays, target, exclude=None, use_bvh=None):
        r = _rays(rays)
        n = r.shape[0]
        e = _excl(exclude, n)
        tg = np.ascontiguousarray(target, dtype=np.int32)
        L = np.zeros(n)
        ub = self.use_bvh if use_bvh is None else int(use_bvh)
        lib().orc_emitter_query(self.h, n, _addr(r), _addr(e), _addr(tg), ub, _addr(L))
        return L

    def light_pdf(self, k: int, x, w) -> float:
        """Solid-angle pdf of the path tracer's light sample toward emissive
        primitive k from x in direction w (times the choice 1/n_emit)."""
        xx = np.ascontiguousarray(x, dtype=np.float64)
        ww = np.ascontiguousarray(w, dtype=np.float64)
        return float(lib().orc_light_pdf(self.h, int(k), _addr(xx), _addr(ww)))

    def light_dir(self, j: int, x, u):
        """Light-sampled direction from x toward emitter slot j (the j-th
        emissive primitive in index order) from four uniforms, or None."""
        xx = np.ascontiguousarray(x, dtype=np.float64)
        uu = np.ascontiguousarray(u, dtype=np.float64)
        w = np.zeros(3)
        ok = lib().orc_light_dir(self.h, int(j), _addr(xx), _addr(uu), _addr(w))
        return w if ok else None

    def render(self, cam: dict, params: dict, pixels=None, nthreads: int | None = None):
        c = make_camera(cam)
        p = make_params(params)
        W, H = int(cam["width"]), int(cam["height"])
        if pixels is None:
            npix, pp = W * H, None
        else:
            pp = np.ascontiguousarray(pixels, dtype=np.int64)
            npix = pp.shape[0]
        s = np.zeros((npix, 3)); s2 = np.zeros((npix, 3))
        nt = nthreads or os.cpu_count() or 1
        rays = lib().orc_render(self.h, C.byref(c), C.byref(p), npix, _addr(pp), int(nt),
                                _addr(s), _addr(s2))
        return s, s2, int(rays)

    def path_radiance(self, cam: dict, params: dict, pixel: int, sample: int):
        c = make_camera(cam)
        p = make_params(params)
        L = np.zeros(3)
        lib().orc_path_radiance(self.h, C.byref(c), C.byref(p), int(pixel), int(sample), _addr(L))
        return L

    def path_records(self, cam: dict, params: dict, pixel: int, sample: int, max_rec: int = 64):
        """(radiance [3], records [n, 24]) of one path; records as in orc_path_records"""
        c = make_camera(cam)
        p = make_params(params)
        L = np.zeros(3)
        rec = np.zeros((max_rec, 24))
        n = lib().orc_path_records(self.h, C.byref(c), C.byref(p), int(pixel), int(sample), _addr(rec),
                                   int(max_rec), _addr(L))
        return L, rec[:min(n, max_rec)]


def camera_rays(cam: dict, seed: int, sample: int) -> np.ndarray:
    """float32 [height * width, 8]: the oracle's camera rays of one sample of
    every pixel, jittered as its path tracer jitters them."""
    n = int(cam["width"]) * int(cam["height"])
    out = np.zeros((n, 8), dtype=np.float32)
    c = make_camera(cam)
    lib().orc_camera_rays(C.byref(c), int(seed), int(sample), _addr(out))
    return out


def make_camera(cam: dict) -> _Camera:
    c = _Camera()
    for i in range(3):
        c.origin[i] = float(cam["origin"][i])
        c.target[i] = float(cam["target"][i])
        c.up[i] = float(cam["up"][i])
    c.vfov_deg = float(cam["vfov_deg"])
    c.width = int(cam["width"])
    c.height = int(cam["height"])
    return c


def make_params(p: dict) -> _Params:
    q = _Params()
    q.spp = int(p.get("spp", 1))
    q.max_depth = int(p.get("max_depth", 4))
    q.seed = int(p.get("seed", 0))
    q.sample_offset = int(p.get("sample_offset", 0))
    env = p.get("env_radiance", (0.0, 0.0, 0.0))
    for i in range(3):
        q.env_radiance[i] = float(env[i])
    q.mis_mode = int(p.get("mis_mode", 0))
    q.nrc_mode = int(p.get("nrc_mode", 0))
    q.nrc_terminate_after = int(p.get("nrc_terminate_after", 2))
    q.nrc_train_frac = float(p.get("nrc_train_frac", 0.0))
    q.transport = int(p.get("transport", 0))
    if q.nrc_mode in (1, 2):
        W = np.ascontiguousarray(p["nrc_weights"], dtype=np.float64)
        assert W.shape == (nrc_num_params(),)
        q._keep = W  # the array must outlive the call
        q.nrc_weights = W.ctypes.data
    box = p.get("nrc_box", None)
    if q.nrc_mode != 0:
        assert box is not None, "nrc_box (lo[3], hi[3]) is required with a cache mode"
        for i in range(6):
            q.nrc_box[i] = float(box[i])
    return q


def phase_eval(mat, albedo, rough, normal, wo, wi):
    a = np.ascontiguousarray(albedo, dtype=np.float64)
    n = np.ascontiguousarray(normal, dtype=np.float64)
    o = np.ascontiguousarray(wo, dtype=np.float64)
    i = np.ascontiguousarray(wi, dtype=np.float64)
    f = np.zeros(3)
    pdf = np.zeros(1)
    lib().orc_phase_eval(int(mat), _addr(a), float(rough), _addr(n), _addr(o), _addr(i), _addr(f),
                         _addr(pdf))
    return f, float(pdf[0])


def phase_sample(mat, albedo, rough, normal, wo, u1, u2):
    a = np.ascontiguousarray(albedo, dtype=np.float64)
    n = np.ascontiguousarray(normal, dtype=np.float64)
    o = np.ascontiguousarray(wo, dtype=np.float64)
    wi = np.zeros(3); w = np.zeros(3); pdf = np.zeros(1)
    lib().orc_phase_sample(int(mat), _addr(a), float(rough), _addr(n), _addr(o), float(u1),
                           float(u2), _addr(wi), _addr(w), _addr(pdf))
    return wi, w, float(pdf[0])


# ---------------------------------------------------------------------------
# SGGX microflake phase function with a Lambertian base (per unit albedo)
# ---------------------------------------------------------------------------
def _s6(s6):
    return np.ascontiguousarray(s6, dtype=np.float64).reshape(6)


def sggx_sigma(s6, w) -> np.ndarray:
    """projected area sigma(w) for directions w [n,3]"""
    v = np.ascontiguousarray(w, dtype=np.float64).reshape(-1, 3)
    out = np.zeros(v.shape[0]); s = _s6(s6)
    lib().orc_sggx_eval_n(_addr(s), v.shape[0], None, _addr(v), 0, _addr(out))
    return out


def sggx_D(s6, nrm) -> np.ndarray:
    """normal distribution D(n) for unit normals [n,3]"""
    v = np.ascontiguousarray(nrm, dtype=np.float64).reshape(-1, 3)
    out = np.zeros(v.shape[0]); s = _s6(s6)
    lib().orc_sggx_eval_n(_addr(s), v.shape[0], None, _addr(v), 1, _addr(out))
    return out


def sggx_vndf(s6, wo, nrm) -> np.ndarray:
    """visible normal distribution D_wo(n) for unit normals [n,3]"""
    v = np.ascontiguousarray(nrm, dtype=np.float64).reshape(-1, 3)
    o = np.ascontiguousarray(wo, dtype=np.float64).reshape(3)
    out = np.zeros(v.shape[0]); s = _s6(s6)
    lib().orc_sggx_eval_n(_addr(s), v.shape[0], _addr(o), _addr(v), 2, _addr(out))
    return out


def sggx_sample_vndf(s6, wo, u) -> np.ndarray:
    """visible normals from uniforms u [n,2] -> [n,3]"""
    uu = np.ascontiguousarray(u, dtype=np.float64).reshape(-1, 2)
    o = np.ascontiguousarray(wo, dtype=np.float64).reshape(3)
    out = np.zeros((uu.shape[0], 3)); s = _s6(s6)
    lib().orc_sggx_sample_vndf_n(_addr(s), _addr(o), uu.shape[0], _addr(uu), _addr(out))
    return out


def sggx_sample_dir(s6, wo, u) -> np.ndarray:
    """importance-sampled incident directions from uniforms u [n,4]: a visible
    normal from u[:, :2], then cosine sampling about it from u[:, 2:]"""
    uu = np.ascontiguousarray(u, dtype=np.float64).reshape(-1, 4)
    o = np.ascontiguousarray(wo, dtype=np.float64).reshape(3)
    out = np.zeros((uu.shape[0], 3)); s = _s6(s6)
    lib().orc_sggx_sample_dir_n(_addr(s), _addr(o), uu.shape[0], _addr(uu), _addr(out))
    return out


def sggx_phase_est(s6, wo, wi, u) -> np.ndarray:
    """stochastic estimates of f_p(wi, wo) / albedo from uniforms u [n,4]"""
    uu = np.ascontiguousarray(u, dtype=np.float64).reshape(-1, 4)
    o = np.ascontiguousarray(wo, dtype=np.float64).reshape(3)
    i = np.ascontiguousarray(wi, dtype=np.float64).reshape(3)
    out = np.zeros(uu.shape[0]); s = _s6(s6)
    lib().orc_sggx_phase_est_n(_addr(s), _addr(o), _addr(i), uu.shape[0], _addr(uu), _addr(out))
    return out


def sggx_phase_quad(s6, wo, wi, nz: int = 400, nphi: int = 800) -> float:
    """f_p(wi, wo) / albedo by midpoint quadrature over the sphere of normals"""
    o = np.ascontiguousarray(wo, dtype=np.float64).reshape(3)
    i = np.ascontiguousarray(wi, dtype=np.float64).reshape(3)
    s = _s6(s6)
    return lib().orc_sggx_phase_quad(_addr(s), _addr(o), _addr(i), int(nz), int(nphi))


def _v3(v):
    return np.ascontiguousarray(v, dtype=np.float64).reshape(3)


def disney_spec_prob(c, met) -> float:
    return lib().orc_disney_spec_prob(_addr(_v3(c)), float(met))


def disney_base(c, rough, met, n, wo, wi):
    """(specular, diffuse) cosine-weighted base BSDF at the flake normal n"""
    fs = np.zeros(3); fd = np.zeros(3)
    cc, nn, o, i = _v3(c), _v3(n), _v3(wo), _v3(wi)
    lib().orc_disney_base(_addr(cc), float(rough), float(met), _addr(nn), _addr(o), _addr(i), _addr(fs), _addr(fd))
    return fs, fd


def sggx_disney_est(s6, c, rough, met, wo, wi, u) -> np.ndarray:
    """material 3: improved stochastic estimates of f_p (rgb) from uniforms u [n,6]"""
    uu = np.ascontiguousarray(u, dtype=np.float64).reshape(-1, 6)
    out = np.zeros((uu.shape[0], 3)); s = _s6(s6)
    cc, o, i = _v3(c), _v3(wo), _v3(wi)
    for k in range(uu.shape[0]):
        lib().orc_sggx_disney_est(_addr(s), _addr(cc), float(rough), float(met), _addr(o), _addr(i),
                                  _addr(uu[k]), out[k].ctypes.data)
    return out


def sggx_disney_sample(s6, c, rough, met, wo, u):
    """material 3: importance samples from uniforms u [n,5] (visible normal u0,u1;
    lobe u2; direction u3,u4) -> (wi [n,3], weight [n,3], ok [n])"""
    uu = np.ascontiguousarray(u, dtype=np.float64).reshape(-1, 5)
    wi = np.zeros((uu.shape[0], 3)); w = np.zeros((uu.shape[0], 3)); ok = np.zeros(uu.shape[0], bool)
    s, cc, o = _s6(s6), _v3(c), _v3(wo)
    for k in range(uu.shape[0]):
        v = np.ascontiguousarray(uu[k, 2:5])
        ok[k] = bool(lib().orc_sggx_disney_sample(_addr(s), _addr(cc), float(rough), float(met), _addr(o),
                                                  float(uu[k, 0]), float(uu[k, 1]), _addr(v),
                                                  wi[k].ctypes.data, w[k].ctypes.data))
    return wi, w, ok


def sggx_roughened(s6, rough) -> np.ndarray:
    out = np.zeros(6); s = _s6(s6)
    lib().orc_sggx_roughened(_addr(s), float(rough), _addr(out))
    return out


def sggx_disney_pdf_approx(s6, c, rough, met, wo, wi) -> float:
    s, cc, o, i = _s6(s6), _v3(c), _v3(wo), _v3(wi)
    return lib().orc_sggx_disney_pdf_approx(_addr(s), _addr(cc), float(rough), float(met), _addr(o), _addr(i))


def sggx_disney_quad(s6, c, rough, met, wo, wi, nz: int = 400, nphi: int = 800) -> np.ndarray:
    """material 3: f_p (rgb) by midpoint quadrature over the sphere of normals"""
    f = np.zeros(3)
    s, cc, o, i = _s6(s6), _v3(c), _v3(wo), _v3(wi)
    lib().orc_sggx_disney_quad(_addr(s), _addr(cc), float(rough), float(met), _addr(o), _addr(i), int(nz),
                               int(nphi), _addr(f))
    return f


def sggx_pdf_approx(wo, wi) -> float:
    o = np.ascontiguousarray(wo, dtype=np.float64).reshape(3)
    i = np.ascontiguousarray(wi, dtype=np.float64).reshape(3)
    return lib().orc_sggx_pdf_approx(_addr(o), _addr(i))


# ---------------------------------------------------------------------------
# neural radiance cache reference (double precision)
# ---------------------------------------------------------------------------
NRC_LAYERS = [(64, 96), (64, 64), (64, 64), (64, 64), (3, 64)]  # (n_out, n_in)


def nrc_num_params() -> int:
    return lib().orc_nrc_num_params()


def nrc_encode(inputs, lo, hi) -> np.ndarray:
    """inputs float32 [n,16] = pos, wo, normal, roughness, albedo, pad -> [n,96]"""
    x = np.ascontiguousarray(inputs, dtype=np.float32)
    n = x.shape[0]
    f = np.zeros((n, 96))
    lo_ = np.ascontiguousarray(lo, dtype=np.float64)
    hi_ = np.ascontiguousarray(hi, dtype=np.float64)
    lib().orc_nrc_encode(n, _addr(x), _addr(lo_), _addr(hi_), _addr(f))
    return f


def nrc_forward(W, feat) -> np.ndarray:
    W = np.ascontiguousarray(W, dtype=np.float64)
    f = np.ascontiguousarray(feat, dtype=np.float64)
    y = np.zeros((f.shape[0], 3))
    lib().orc_nrc_forward(f.shape[0], _addr(W), _addr(f), _addr(y))
    return y


def nrc_loss_grad(W, feat, target):
    W = np.ascontiguousarray(W, dtype=np.float64)
    f = np.ascontiguousarray(feat, dtype=np.float64)
    t = np.ascontiguousarray(target, dtype=np.float64)
    g = np.zeros(W.shape[0])
    loss = lib().orc_nrc_loss_grad(f.shape[0], _addr(W), _addr(f), _addr(t), _addr(g))
    return loss, g


def nrc_adam(W, m, v, g, t, lr=1e-3, b1=0.9, b2=0.99, eps=1e-8):
    W = np.array(W, dtype=np.float64); m = np.array(m, dtype=np.float64); v = np.array(v, dtype=np.float64)
    gg = np.ascontiguousarray(g, dtype=np.float64)
    lib().orc_nrc_adam(W.shape[0], _addr(W), _addr(m), _addr(v), _addr(gg), int(t), lr, b1, b2, eps)
    return W, m, v
