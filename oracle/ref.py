"""ctypes wrapper of the FP64 oracle (test infrastructure only).

Inputs come from the seeded generators in the package's scenegen module as
float32/uint32 arrays; they are converted here, exactly, to float64.  Outputs
are float64 record arrays:
  G-buffer (W*H, 14): pos[3] nrm[3] albedo[3] emit[3] view_depth prim
  reservoir (W*H, 14): y[3] n_y[3] L[3] wsum W M tag prim
  probe textures: irr (P, (Ni+2)^2, 3), dep (P, (Nd+2)^2, 2)
"""
from __future__ import annotations

import ctypes as C
import math

import numpy as np

from . import build as _build

MISS = 0xFFFFFFFF
FILL_FRAME_BASE = 0xF0000000      # frame index used by the probe fill passes
GB_N = 14
R_N = 14

_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(_build.ensure_built())
        _setup(_lib)
    return _lib


class OScene(C.Structure):
    _fields_ = [("n_prims", C.c_int32), ("has_room", C.c_int32), ("prims", C.c_void_p),
                ("room_lo", C.c_double * 3), ("room_hi", C.c_double * 3),
                ("wall_albedo", C.c_double * 3), ("wall_emit", C.c_double * 3),
                ("sky", C.c_double * 3), ("eps", C.c_double), ("glossy", C.c_int32), ("pad", C.c_int32)]


class OCamera(C.Structure):
    _fields_ = [("eye", C.c_double * 3), ("fwd", C.c_double * 3), ("right", C.c_double * 3),
                ("up", C.c_double * 3), ("tan_half_fovy", C.c_double),
                ("width", C.c_int32), ("height", C.c_int32)]


class OProbes(C.Structure):
    _fields_ = [("dims", C.c_int32 * 3), ("irr_res", C.c_int32), ("dep_res", C.c_int32),
                ("lo", C.c_double * 3), ("spacing", C.c_double * 3), ("bias_dist", C.c_double),
                ("var_floor", C.c_double), ("d_max", C.c_double),
                ("irr", C.c_void_p), ("dep", C.c_void_p), ("mlp", C.c_void_p),
                ("mlp_prec", C.c_int32), ("texel", C.c_int32),
                ("mlp_lo", C.c_double * 3), ("mlp_hi", C.c_double * 3)]


class OParams(C.Structure):
    _fields_ = [("M", C.c_int32), ("k", C.c_int32), ("unbiased", C.c_int32), ("M_light", C.c_int32),
                ("radius", C.c_double), ("g_max", C.c_double), ("cos_n", C.c_double),
                ("depth_rel", C.c_double), ("m_cap", C.c_double), ("subsample", C.c_int32),
                ("pad", C.c_int32), ("eye", C.c_double * 3), ("eye_prev", C.c_double * 3),
                ("foot_c", C.c_double), ("glossy_depth", C.c_int32), ("pad2", C.c_int32)]


_P = C.c_void_p


def _setup(L):
    L.o_set_threads.argtypes = [C.c_int]
    L.o_openmp.restype = C.c_int
    L.o_philox.argtypes = [C.c_uint32, C.c_uint32, _P, _P]
    L.o_cosine_dir.argtypes = [_P, C.c_double, C.c_double, _P]
    L.o_sphere_dir.argtypes = [C.c_double, C.c_double, _P]
    L.o_closest_hit.argtypes = [_P, _P, _P, C.c_double, _P]
    L.o_closest_hit.restype = C.c_int
    L.o_visible.argtypes = [_P, _P, _P, _P, _P, C.c_int]
    L.o_visible.restype = C.c_int
    L.o_gbuffer.argtypes = [_P, _P, _P, C.c_int64, _P]
    L.o_oct_encode.argtypes = [_P, _P]
    L.o_oct_decode.argtypes = [_P, _P]
    L.o_tile_fetch.argtypes = [_P, C.c_int, C.c_int, _P, _P]
    L.o_fill_gutter.argtypes = [_P, C.c_int, C.c_int]
    L.o_round_half.argtypes = [C.c_double]
    L.o_round_half.restype = C.c_double
    L.o_probe_query.argtypes = [_P, C.c_int64, _P, _P, C.c_int, _P]
    L.o_probe_update.argtypes = [_P, _P, _P, _P, C.c_int, C.c_double, C.c_double, C.c_double, C.c_uint64,
                                 C.c_uint32, _P, C.c_int64]
    L.o_resample_initial.argtypes = [_P, C.c_int32, C.c_int32, _P, _P, _P, C.c_uint64, C.c_uint32,
                                     _P, C.c_int64, _P, _P]
    L.o_reproject.argtypes = [_P, _P]
    L.o_reproject.restype = C.c_int64
    L.o_resample_temporal.argtypes = [_P, C.c_int32, C.c_int32, _P, _P, _P, _P, _P, _P, C.c_uint64,
                                      C.c_uint32, _P, C.c_int64, _P]
    L.o_spatial_candidate.argtypes = [C.c_int32, C.c_int32, C.c_int64, C.c_int, C.c_double,
                                      C.c_uint64, C.c_uint32, C.c_int, _P]
    L.o_spatial_candidate.restype = C.c_int64
    L.o_resample_spatial.argtypes = [_P, C.c_int32, C.c_int32, _P, _P, _P, C.c_int, C.c_uint64,
                                     C.c_uint32, _P, C.c_int64, _P]
    L.o_shade.argtypes = [_P, C.c_int32, C.c_int32, _P, _P, _P, _P, _P, _P, C.c_int64, _P, C.c_uint64,
                          C.c_uint32]
    L.o_ggx.argtypes = [_P, _P, _P, C.c_double, _P]
    L.o_ggx_sample.argtypes = [_P, _P, C.c_double, C.c_double, C.c_double, _P]
    L.o_ggx_sample.restype = C.c_int
    L.o_glossy_term.argtypes = [_P, _P, _P, _P, C.c_double, C.c_double, C.c_double, C.c_double, _P]


def set_threads(n: int) -> int:
    """Threads of the oracle's pixel and probe loops (1 by default).  Every
    iteration writes only its own outputs, so results do not depend on it.
    Returns the count in effect (1 when the library was built without OpenMP)."""
    n = max(1, int(n)) if lib().o_openmp() else 1
    lib().o_set_threads(n)
    return n


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


# --------------------------------------------------------------------------
# input conversion
# --------------------------------------------------------------------------
class _Scene:
    def __init__(self, scene):
        rec = np.asarray(scene.prims, np.float32)
        p = rec.astype(np.float64)
        if len(rec):
            p[:, 3] = rec.view(np.uint32)[:, 3].astype(np.float64)
        self.prims = np.ascontiguousarray(p)
        s = OScene()
        s.n_prims = len(rec)
        s.has_room = 1 if scene.has_room else 0
        s.prims = self.prims.ctypes.data if len(rec) else None
        for name in ("room_lo", "room_hi", "wall_albedo", "wall_emit", "sky"):
            getattr(s, name)[:] = [float(v) for v in np.asarray(getattr(scene, name), np.float32)]
        s.eps = float(np.float32(scene.eps))
        # a specular layer on any primitive (slot 11 = k_s, slot 15 = GGX roughness)
        s.glossy = 1 if len(rec) and np.any(rec[:, 11] > 0) else 0
        self.s = s

    @property
    def ref(self):
        return C.byref(self.s)


def _scene(scene):
    if isinstance(scene, _Scene):
        return scene
    cached = getattr(scene, "_oracle_cache", None)
    if cached is None:
        cached = _Scene(scene)
        try:
            scene._oracle_cache = cached
        except AttributeError:
            pass
    return cached


def _camera(cam) -> OCamera:
    c = OCamera()
    for name in ("eye", "fwd", "right", "up"):
        getattr(c, name)[:] = [float(v) for v in np.asarray(getattr(cam, name), np.float32)]
    c.tan_half_fovy = float(np.float32(cam.tan_half_fovy))
    c.width, c.height = int(cam.width), int(cam.height)
    return c


class MlpTarget:
    """A learned cache used as the target: flat FP64 parameters, precision
    ('f64' or 'bf16') and the position normalisation box."""

    def __init__(self, params, lo, hi, prec="bf16"):
        self.params = _f64(params)
        self.lo, self.hi = [float(v) for v in np.asarray(lo, np.float32)], \
            [float(v) for v in np.asarray(hi, np.float32)]
        self.prec = 1 if prec == "bf16" else 0


def texel_code(grid) -> int:
    """The oracle's texel-precision switch for a probe grid: 0 keeps texels
    at full precision (the FP32 textures), 1 rounds them as the binary16
    textures store them."""
    t = getattr(grid, "texel", "f32")
    if t not in ("f32", "f16"):
        raise ValueError(f"unknown probe texel format {t!r}")
    return 1 if t == "f16" else 0


class _Probes:
    def __init__(self, grid, irr, dep, mlp: "MlpTarget" = None):
        self.irr = _f64(np.asarray(irr)[..., :3])
        self.dep = _f64(np.asarray(dep)[..., :2])
        p = OProbes()
        p.dims[:] = list(grid.dims)
        p.irr_res, p.dep_res = grid.irr_res, grid.dep_res
        p.lo[:] = [float(v) for v in np.asarray(grid.lo, np.float32)]
        p.spacing[:] = [float(v) for v in np.asarray(grid.spacing, np.float32)]
        p.bias_dist = float(np.float32(grid.bias_dist))
        p.var_floor = float(np.float32(grid.var_floor))
        p.d_max = float(np.float32(grid.d_max))
        p.irr = self.irr.ctypes.data
        p.dep = self.dep.ctypes.data
        p.texel = texel_code(grid)
        self.mlp = mlp
        if mlp is not None:
            p.mlp = mlp.params.ctypes.data
            p.mlp_prec = mlp.prec
            p.mlp_lo[:], p.mlp_hi[:] = mlp.lo, mlp.hi
        self.p = p

    @property
    def ref(self):
        return C.byref(self.p)


def _params(pr, eye=None, eye_prev=None) -> OParams:
    """Resampling parameters; eye / eye_prev are the camera positions of the
    current and previous frame (the view direction of glossy primary vertices)."""
    o = OParams()
    o.M, o.k, o.unbiased = int(pr.M), int(pr.k), int(pr.unbiased)
    o.M_light = int(getattr(pr, "M_light", 0))
    o.radius = float(np.float32(pr.radius))
    o.g_max = float(np.float32(pr.g_max))
    o.cos_n = float(np.float32(pr.cos_n))
    o.depth_rel = float(np.float32(pr.depth_rel))
    o.m_cap = float(np.float32(pr.m_cap))
    o.subsample = int(getattr(pr, "subsample", 1))
    o.foot_c = float(np.float32(getattr(pr, "foot_c", 0.2)))
    o.glossy_depth = int(getattr(pr, "glossy_depth", 8))
    for name, v in (("eye", eye), ("eye_prev", eye_prev if eye_prev is not None else eye)):
        if v is not None:
            getattr(o, name)[:] = [float(t) for t in np.asarray(v, np.float32).reshape(3)]
    return o


def _pix(pixels):
    if pixels is None:
        return None, 0, None
    arr = np.ascontiguousarray(np.asarray(pixels, dtype=np.int32))
    return arr, len(arr), _ptr(arr)


# --------------------------------------------------------------------------
# primitives
# --------------------------------------------------------------------------
def philox(seed: int, ctr) -> np.ndarray:
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32))
    out = np.zeros(4, np.uint32)
    lib().o_philox(seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF, _ptr(c), _ptr(out))
    return out


def cosine_dir(n, u0, u1) -> np.ndarray:
    nn, out = _f64(n), np.zeros(3)
    lib().o_cosine_dir(_ptr(nn), float(u0), float(u1), _ptr(out))
    return out


def sphere_dir(u0, u1) -> np.ndarray:
    out = np.zeros(3)
    lib().o_sphere_dir(float(u0), float(u1), _ptr(out))
    return out


def closest_hit(scene, o, d, tmax=math.inf):
    s = _scene(scene)
    oo, dd, out = _f64(o), _f64(d), np.zeros(5)
    hit = lib().o_closest_hit(s.ref, _ptr(oo), _ptr(dd), float(tmax), _ptr(out))
    return bool(hit), out[0], int(out[1]), out[2:5].copy()


def visible(scene, a, na, b, nb, b_is_dir=False) -> bool:
    s = _scene(scene)
    arrs = [_f64(v) for v in (a, na, b, nb)]
    return bool(lib().o_visible(s.ref, *[_ptr(v) for v in arrs], int(b_is_dir)))


def oct_encode(v) -> np.ndarray:
    vv, out = _f64(v), np.zeros(2)
    lib().o_oct_encode(_ptr(vv), _ptr(out))
    return out


def oct_decode(uv) -> np.ndarray:
    u, out = _f64(uv), np.zeros(3)
    lib().o_oct_decode(_ptr(u), _ptr(out))
    return out


def tile_fetch(tile, N, v) -> np.ndarray:
    t = _f64(tile)
    Cc = t.shape[-1]
    vv, out = _f64(v), np.zeros(Cc)
    lib().o_tile_fetch(_ptr(t), int(N), int(Cc), _ptr(vv), _ptr(out))
    return out


def round_half(x) -> float:
    """IEEE binary16 rounding of x (nearest, ties to even), as a float: the
    storage precision of a binary16 probe volume's texels."""
    return lib().o_round_half(float(x))


def fill_gutter(tile, N) -> np.ndarray:
    t = _f64(tile).copy()
    lib().o_fill_gutter(_ptr(t), int(N), int(t.shape[-1]))
    return t


# --------------------------------------------------------------------------
# passes
# --------------------------------------------------------------------------
def gbuffer(scene, cam, pixels=None, out=None) -> np.ndarray:
    s, c = _scene(scene), _camera(cam)
    n = cam.width * cam.height
    gb = np.zeros((n, GB_N)) if out is None else out
    arr, npix, pp = _pix(pixels)
    lib().o_gbuffer(s.ref, C.byref(c), pp, npix, _ptr(gb))
    return gb


def probe_query(grid, irr, dep, p, n, flags=0) -> np.ndarray:
    pr = _Probes(grid, irr, dep)
    pp, nn = _f64(p).reshape(-1, 3), _f64(n).reshape(-1, 3)
    out = np.zeros_like(pp)
    lib().o_probe_query(pr.ref, len(pp), _ptr(pp), _ptr(nn), int(flags), _ptr(out))
    return out


def probe_update(scene, grid, irr, dep, rays, hysteresis, sharpness, seed, frame, probes=None, slider=0.0):
    s = _scene(scene)
    pr = _Probes(grid, irr, dep)
    irr_out, dep_out = pr.irr.copy(), pr.dep.copy()
    arr, n, pp = _pix(probes)
    lib().o_probe_update(s.ref, pr.ref, _ptr(irr_out), _ptr(dep_out), int(rays), float(hysteresis),
                         float(sharpness), float(np.float32(slider)), int(seed), int(frame) & 0xFFFFFFFF, pp, n)
    return irr_out, dep_out


def fill_probes(scene, grid, upd, seed, irr=None, dep=None):
    """Fill passes before frame 0: hysteresis 0, frame = FILL_FRAME_BASE + pass."""
    if irr is None:
        P = grid.count
        irr = np.zeros((P, (grid.irr_res + 2) ** 2, 3))
        dep = np.zeros((P, (grid.dep_res + 2) ** 2, 2))
    for k in range(upd.fill_passes):
        irr, dep = probe_update(scene, grid, irr, dep, upd.fill_rays, 0.0, upd.sharpness, seed,
                                FILL_FRAME_BASE + k, slider=getattr(upd, "distance_slider", 0.0))
    return irr, dep


def resample_initial(scene, W, H, gb, grid, irr, dep, params, seed, frame, pixels=None,
                     res=None, resid=None, mlp=None, eye=None):
    s, pr, pp = _scene(scene), _Probes(grid, irr, dep, mlp), _params(params, eye)
    gb = _f64(gb)
    res = np.zeros((W * H, R_N)) if res is None else res
    resid = np.zeros((W * H, 3)) if resid is None else resid
    arr, n, px = _pix(pixels)
    lib().o_resample_initial(s.ref, W, H, _ptr(gb), pr.ref, C.byref(pp), int(seed),
                             int(frame) & 0xFFFFFFFF, px, n, _ptr(res), _ptr(resid))
    return res, resid


def view_bias(y, x, d) -> np.ndarray:
    yy, xx, out = _f64(y), _f64(x), np.zeros(3)
    L = lib()
    L.o_view_bias.argtypes = [_P, _P, C.c_double, _P]
    L.o_view_bias(_ptr(yy), _ptr(xx), float(d), _ptr(out))
    return out


def reproject(cam, x) -> int:
    c, xx = _camera(cam), _f64(x)
    return int(lib().o_reproject(C.byref(c), _ptr(xx)))


def resample_temporal(scene, W, H, gb, gb_prev, cam_prev, cur, hist, params, seed, frame,
                      pixels=None, out=None, eye=None, eye_prev=None):
    s, c, pp = _scene(scene), _camera(cam_prev), _params(params, eye, eye_prev)
    gb, gb_prev, cur, hist = _f64(gb), _f64(gb_prev), _f64(cur), _f64(hist)
    out = np.zeros((W * H, R_N)) if out is None else out
    arr, n, px = _pix(pixels)
    lib().o_resample_temporal(s.ref, W, H, _ptr(gb), _ptr(gb_prev), C.byref(c), _ptr(cur),
                              _ptr(hist), C.byref(pp), int(seed), int(frame) & 0xFFFFFFFF, px, n,
                              _ptr(out))
    return out


def spatial_candidate(W, H, p, j, radius, seed, frame, spass) -> int:
    u2 = C.c_double()
    return int(lib().o_spatial_candidate(W, H, int(p), int(j), float(np.float32(radius)), int(seed),
                                         int(frame) & 0xFFFFFFFF, int(spass), C.byref(u2)))


def resample_spatial(scene, W, H, gb, res_in, params, spass, seed, frame, pixels=None, out=None, eye=None):
    s, pp = _scene(scene), _params(params, eye)
    gb, res_in = _f64(gb), _f64(res_in)
    out = np.zeros((W * H, R_N)) if out is None else out
    arr, n, px = _pix(pixels)
    lib().o_resample_spatial(s.ref, W, H, _ptr(gb), _ptr(res_in), C.byref(pp), int(spass),
                             int(seed), int(frame) & 0xFFFFFFFF, px, n, _ptr(out))
    return out


def shade(scene, W, H, gb, grid, irr, dep, res, resid, params, pixels=None, out=None, mlp=None,
          seed=0, frame=0, eye=None):
    """Shading; seed / frame drive the specular recursion of a glossy scene."""
    s, pr, pp = _scene(scene), _Probes(grid, irr, dep, mlp), _params(params, eye)
    gb, res, resid = _f64(gb), _f64(res), _f64(resid)
    out = np.zeros((W * H, 3)) if out is None else out
    arr, n, px = _pix(pixels)
    lib().o_shade(s.ref, W, H, _ptr(gb), pr.ref, _ptr(res), _ptr(resid), C.byref(pp), px, n,
                  _ptr(out), int(seed), int(frame) & 0xFFFFFFFF)
    return out


# --------------------------------------------------------------------------
# whole frames
# --------------------------------------------------------------------------
class Sequence:
    """Runs the method frame after frame on full images, keeping the history
    (last spatial output) and the previous G-buffer/camera."""

    def __init__(self, scene, grid, irr, dep, params, seed, mlp=None):
        self.scene, self.grid, self.irr, self.dep = scene, grid, irr, dep
        self.params, self.seed, self.mlp = params, seed, mlp
        self.hist = self.gb_prev = self.cam_prev = None

    def frame(self, cam, frame):
        W, H, pr = cam.width, cam.height, self.params
        gb = gbuffer(self.scene, cam)
        eye = cam.eye
        eye_prev = self.cam_prev.eye if self.cam_prev is not None else eye
        res, resid = resample_initial(self.scene, W, H, gb, self.grid, self.irr, self.dep, pr,
                                      self.seed, frame, mlp=self.mlp, eye=eye)
        stages = {"gbuffer": gb, "initial": res, "resid": resid}
        if pr.temporal and self.hist is not None:
            res = resample_temporal(self.scene, W, H, gb, self.gb_prev, self.cam_prev, res,
                                    self.hist, pr, self.seed, frame, eye=eye, eye_prev=eye_prev)
            stages["temporal"] = res
        for sp in range(pr.n_spatial):
            res = resample_spatial(self.scene, W, H, gb, res, pr, sp, self.seed, frame, eye=eye)
            stages[f"spatial{sp}"] = res
        img = shade(self.scene, W, H, gb, self.grid, self.irr, self.dep, res, resid, pr, mlp=self.mlp,
                    seed=self.seed, frame=frame, eye=eye)
        stages["image"] = img
        self.hist, self.gb_prev, self.cam_prev = res, gb, cam
        return img, stages


def mape(v, ref, eps=0.01) -> float:
    """Mean absolute percentage error of Sec. 4: mean |v - ref| / (ref + eps)."""
    v, ref = np.asarray(v, np.float64), np.asarray(ref, np.float64)
    return float(np.mean(np.abs(v - ref) / (ref + eps)))


def tag_origin(tag):
    t = np.asarray(tag).astype(np.uint64)
    return (t >> 9) & 0x7FFFFF


def brute_force(scene, W, H, gb, grid, irr, dep, pixels, nsamples, seed=12345) -> np.ndarray:
    s, pr = _scene(scene), _Probes(grid, irr, dep)
    gb = _f64(gb)
    arr, n, px = _pix(pixels)
    out = np.zeros((n, 3))
    L = lib()
    L.o_brute_force.argtypes = [_P, _P, _P, C.c_int32, C.c_int32, _P, C.c_int64, C.c_int64,
                                C.c_uint64, _P]
    L.o_brute_force(s.ref, pr.ref, _ptr(gb), W, H, px, n, int(nsamples), int(seed), _ptr(out))
    return out


def mlp_batch(scene, W, H, gb, grid, irr, dep, M, B, seed, frame):
    """Training samples of the learned cache (see o_mlp_batch): returns
    (pos (B,3), nrm (B,3), target (B,3), valid (B,), qprobe (B,3))."""
    s, pr = _scene(scene), _Probes(grid, irr, dep)
    gb = _f64(gb)
    pos, nrm, tgt, qp = np.zeros((B, 3)), np.zeros((B, 3)), np.zeros((B, 3)), np.zeros((B, 3))
    valid = np.zeros(B, np.int32)
    L = lib()
    L.o_mlp_batch.argtypes = [_P, _P, C.c_int32, C.c_int32, _P, C.c_int32, C.c_int64, C.c_uint64, C.c_uint32,
                              _P, _P, _P, _P, _P]
    L.o_mlp_batch(s.ref, pr.ref, W, H, _ptr(gb), int(M), int(B), int(seed), int(frame) & 0xFFFFFFFF,
                  _ptr(pos), _ptr(nrm), _ptr(tgt), _ptr(valid), _ptr(qp))
    return pos, nrm, tgt, valid.astype(bool), qp


def mlp_forward(params, prec, lo, hi, pos, nrm) -> np.ndarray:
    """The C oracle's MLP forward (prec 'f64' or 'bf16') for n points."""
    p = _f64(params)
    pos, nrm = _f64(pos).reshape(-1, 3), _f64(nrm).reshape(-1, 3)
    lo_, hi_ = _f64(np.asarray(lo, np.float32)), _f64(np.asarray(hi, np.float32))
    out = np.zeros((len(pos), 3))
    L = lib()
    L.o_mlp_forward.argtypes = [_P, C.c_int, _P, _P, _P, _P, _P]
    for i in range(len(pos)):
        L.o_mlp_forward(_ptr(p), 1 if prec == "bf16" else 0, _ptr(lo_), _ptr(hi_), _ptr(pos[i]),
                        _ptr(nrm[i]), out[i].ctypes.data_as(C.c_void_p))
    return out


def path_trace(scene, gb, pixels, spp, seed, s0=0, eye=None) -> np.ndarray:
    """Reference path tracer (o_path_trace) for the listed pixels: (n, 3);
    eye (the camera position) is needed for a glossy scene."""
    s = _scene(scene)
    gb = _f64(gb)
    pix = np.ascontiguousarray(np.asarray(pixels, np.int32))
    out = np.zeros((len(pix), 3))
    e = _f64(np.zeros(3) if eye is None else np.asarray(eye, np.float32))
    L = lib()
    L.o_path_trace.argtypes = [_P, _P, _P, C.c_int64, C.c_int32, C.c_uint32, C.c_uint64, _P, _P]
    L.o_path_trace(s.ref, _ptr(gb), _ptr(pix), len(pix), int(spp), int(s0) & 0xFFFFFFFF, int(seed), _ptr(e),
                   _ptr(out))
    return out


# --------------------------------------------------------------------------
# glossy layer (test hooks)
# --------------------------------------------------------------------------
def ggx(n, wo, wi, a):
    """(f_g / k_s, solid-angle sampling density) of the GGX lobe."""
    out = np.zeros(2)
    lib().o_ggx(_ptr(_f64(n)), _ptr(_f64(wo)), _ptr(_f64(wi)), float(a), _ptr(out))
    return float(out[0]), float(out[1])


def ggx_many(n, wo, wis, a):
    """(f_g / k_s, density) of the GGX lobe for rows of directions wis."""
    wis = _f64(np.asarray(wis).reshape(-1, 3))
    f, pdf = np.zeros(len(wis)), np.zeros(len(wis))
    L = lib()
    L.o_ggx_many.argtypes = [_P, _P, _P, C.c_int64, C.c_double, _P, _P]
    L.o_ggx_many(_ptr(_f64(n)), _ptr(_f64(wo)), _ptr(wis), len(wis), float(a), _ptr(f), _ptr(pdf))
    return f, pdf


def ggx_sample(n, wo, a, u0, u1):
    """A direction from the GGX lobe about wo, or None below the surface."""
    wi = np.zeros(3)
    ok = lib().o_ggx_sample(_ptr(_f64(n)), _ptr(_f64(wo)), float(a), float(u0), float(u1), _ptr(wi))
    return wi if ok else None


def glossy_term(grid, irr, dep, pb, n, wo, ks, a, u0, u1):
    """One-sample glossy part of L_DDGI+ (Eq. 6) at the biased point pb."""
    pr = _Probes(grid, irr, dep)
    out = np.zeros(3)
    lib().o_glossy_term(pr.ref, _ptr(_f64(pb)), _ptr(_f64(n)), _ptr(_f64(wo)), float(ks), float(a), float(u0),
                        float(u1), _ptr(out))
    return out
