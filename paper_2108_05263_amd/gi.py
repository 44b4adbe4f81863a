"""Python binding of libgi.so (argument marshalling only).

Every step of the method runs in the library's HIP kernels; this module
allocates caller-owned device buffers with torch, fills the C structs of
include/gi.h and forwards the current torch stream.  There is no fallback:
if libgi.so cannot be loaded, or a call returns an error, it raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

from . import scenegen as sg

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgi.so")
MISS = 0xFFFFFFFF
EMPTY_TAG = 0xFFFFFFFF
OPT_NO_LDS = 1
OPT_GLOSSY = 2

_lib = None

# every symbol include/gi.h declares
EXPORTS = ["gi_status_string", "gi_device", "gi_build_hash", "gi_trace_gbuffer", "gi_probe_update", "gi_probe_query",
           "gi_resample_initial", "gi_resample_temporal", "gi_resample_spatial", "gi_shade",
           "gi_accel_build_host", "gi_philox", "gi_trace_rays",
           "gi_mlp_init", "gi_mlp_prepare", "gi_mlp_infer", "gi_mlp_make_batch", "gi_mlp_train_workspace_bytes",
           "gi_mlp_grad", "gi_mlp_adam", "gi_mlp_train_step", "gi_mlp_train_step_noalloc", "gi_initial_mlp_workspace_bytes",
           "gi_resample_initial_mlp", "gi_shade_mlp_workspace_bytes", "gi_shade_mlp", "gi_path_trace"]

MLP_N_PARAMS = 17731
MLP_WEIGHT_BYTES = 40064
MLP_MAX_BATCH = 1 << 20
MLP_PRECISION = {"bf16": 0, "fp8": 1}
MLP_MODE = {"auto": 0, "always": 1, "never": 2}
# words of the device state (GI_MLP_STATE_*)
MLP_STATE = {"usable": 0, "steps": 1, "nonfinite": 2, "ema_err": 3, "loss": 4, "valid": 5, "batch_err": 6}


class GiError(RuntimeError):
    pass


# --------------------------------------------------------------------------
# C structs (layouts of include/gi.h)
# --------------------------------------------------------------------------
F3 = C.c_float * 3
U3 = C.c_uint32 * 3


class GiScene(C.Structure):
    _fields_ = [("prims", C.c_void_p), ("n_prims", C.c_uint32), ("has_room", C.c_uint32),
                ("room_lo", F3), ("room_hi", F3), ("wall_albedo", F3), ("wall_emit", F3), ("sky", F3),
                ("eps", C.c_float), ("grid_res", U3), ("grid_lo", F3), ("grid_hi", F3),
                ("cell_start", C.c_void_p), ("cell_items", C.c_void_p), ("n_items", C.c_uint32),
                ("options", C.c_uint32), ("n_emitters", C.c_uint32), ("emitters", C.c_uint32 * 32)]


class GiCamera(C.Structure):
    _fields_ = [("eye", F3), ("fwd", F3), ("right", F3), ("up", F3), ("tan_half_fovy", C.c_float),
                ("width", C.c_uint32), ("height", C.c_uint32)]


class GiGBuffer(C.Structure):
    _fields_ = [("width", C.c_uint32), ("height", C.c_uint32), ("pos_depth", C.c_void_p),
                ("nrm_prim", C.c_void_p), ("albedo", C.c_void_p), ("emit", C.c_void_p),
                ("format", C.c_uint32), ("pad", C.c_uint32), ("eye", C.c_float * 3), ("pad2", C.c_float)]


GB_FORMAT = {"f32": 0, "f16": 1}


TEXEL_FORMAT = {"f32": 0, "f16": 1}


class GiProbes(C.Structure):
    _fields_ = [("dims", U3), ("irr_res", C.c_uint32), ("dep_res", C.c_uint32), ("lo", F3),
                ("spacing", F3), ("bias_dist", C.c_float), ("var_floor", C.c_float),
                ("d_max", C.c_float), ("texel", C.c_uint32), ("irr", C.c_void_p), ("dep", C.c_void_p)]


class GiReservoirs(C.Structure):
    _fields_ = [("width", C.c_uint32), ("height", C.c_uint32), ("y_W", C.c_void_p),
                ("n_wsum", C.c_void_p), ("L_M", C.c_void_p), ("tag_prim", C.c_void_p)]


class GiParams(C.Structure):
    _fields_ = [("M", C.c_uint32), ("k", C.c_uint32), ("radius", C.c_float), ("g_max", C.c_float),
                ("cos_n", C.c_float), ("depth_rel", C.c_float), ("m_cap", C.c_float),
                ("unbiased", C.c_uint32), ("M_light", C.c_uint32), ("subsample", C.c_uint32),
                ("foot_c", C.c_float), ("glossy_depth", C.c_uint32)]


class GiProbeParams(C.Structure):
    _fields_ = [("rays", C.c_uint32), ("hysteresis", C.c_float), ("sharpness", C.c_float),
                ("distance_slider", C.c_float)]


class GiMlp(C.Structure):
    _fields_ = [("params", C.c_void_p), ("adam_m", C.c_void_p), ("adam_v", C.c_void_p),
                ("ema", C.c_void_p), ("weights", C.c_void_p), ("scales", C.c_void_p), ("state", C.c_void_p),
                ("pos_lo", F3), ("pos_hi", F3), ("precision", C.c_uint32), ("mode", C.c_uint32),
                ("warmup_steps", C.c_uint32), ("max_rel_err", C.c_float), ("ema_decay", C.c_float),
                ("pad", C.c_uint32)]


_P = C.c_void_p


def load():
    """Load libgi.so (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise GiError(f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                      "python paper_2108_05263_amd/build.py")
    from . import build as _build
    have, want = _build.built_hash(), _build.source_hash()
    if have != want:
        raise GiError(f"{LIB_PATH} was built from other sources (hash {have}, tree {want}); "
                      "run __graft_entry__.build() or python paper_2108_05263_amd/build.py")
    L = C.CDLL(LIB_PATH)
    L.gi_build_hash.restype = C.c_char_p
    L.gi_status_string.restype = C.c_char_p
    L.gi_status_string.argtypes = [C.c_int]
    L.gi_device.restype = C.c_int
    for name, args in {
        "gi_trace_gbuffer": [_P, _P, _P, _P],
        "gi_probe_update": [_P, _P, _P, _P, C.c_uint64, C.c_uint32, _P],
        "gi_probe_query": [_P, C.c_uint32, _P, _P, _P, _P],
        "gi_resample_initial": [_P, _P, _P, _P, _P, _P, C.c_uint64, C.c_uint32, _P],
        "gi_resample_temporal": [_P, _P, _P, _P, _P, _P, _P, _P, C.c_uint64, C.c_uint32, _P],
        "gi_resample_spatial": [_P, _P, _P, _P, C.c_uint32, _P, C.c_uint64, C.c_uint32, _P],
        "gi_shade": [_P, _P, _P, _P, _P, _P, _P, C.c_uint64, C.c_uint32, _P],
        "gi_accel_build_host": [_P, C.c_uint32, _P, _P, _P, _P, _P, C.c_uint32, _P],
        "gi_philox": [C.c_uint64, C.c_uint32, _P, _P, _P],
        "gi_trace_rays": [_P, C.c_uint32, _P, _P, _P, _P, _P],
        "gi_mlp_init": [_P, C.c_uint64, _P],
        "gi_mlp_prepare": [_P, _P],
        "gi_mlp_infer": [_P, C.c_uint32, _P, _P, _P, _P],
        "gi_mlp_make_batch": [_P, _P, _P, C.c_uint32, C.c_uint32, C.c_uint64, C.c_uint32, _P, _P, _P, _P, _P],
        "gi_mlp_grad": [_P, C.c_uint32, _P, _P, _P, _P, _P, _P, C.c_uint64, _P],
        "gi_mlp_adam": [_P, _P, C.c_uint32, C.c_float, _P],
        "gi_mlp_train_step": [_P, C.c_uint32, _P, _P, _P, _P, C.c_uint32, C.c_float, _P, C.c_uint64, _P],
        "gi_mlp_train_step_noalloc": [_P, C.c_uint32, _P, _P, _P, _P, C.c_uint32, C.c_float, _P],
        "gi_resample_initial_mlp": [_P, _P, _P, _P, _P, _P, _P, _P, C.c_uint64, C.c_uint64, C.c_uint32, _P],
        "gi_shade_mlp": [_P, _P, _P, _P, _P, _P, _P, _P, _P, C.c_uint64, _P],
        "gi_path_trace": [_P, _P, C.c_uint32, C.c_uint32, C.c_uint64, _P, _P],
    }.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = C.c_int
    for name, args in {"gi_mlp_train_workspace_bytes": [C.c_uint32],
                       "gi_initial_mlp_workspace_bytes": [C.c_uint32, C.c_uint32, C.c_uint32],
                       "gi_shade_mlp_workspace_bytes": [C.c_uint32, C.c_uint32]}.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = C.c_uint64
    _lib = L
    return L


def check(status: int, what: str):
    if status != 0:
        msg = load().gi_status_string(status).decode()
        raise GiError(f"{what}: {msg} (status {status})")


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t: torch.Tensor, dtype=None):
    """Device pointer of a contiguous device tensor, of `dtype` when given (the
    library reads and writes raw records: a buffer of another element type
    would be misread, so it is refused)."""
    if not (t.is_cuda and t.is_contiguous()):
        raise GiError("buffers passed to the library must be contiguous device tensors")
    if dtype is not None and t.dtype != dtype:
        raise GiError(f"buffer of dtype {t.dtype} where {dtype} is required")
    return C.c_void_p(t.data_ptr())


F32 = torch.float32


def _f3(v):
    return F3(*[float(x) for x in np.asarray(v, np.float32).reshape(3)])


# --------------------------------------------------------------------------
# device-side objects
# --------------------------------------------------------------------------
class DeviceScene:
    """Primitive records (and the optional grid accelerator) on the device."""

    def __init__(self, scene: sg.Scene, grid_res=None, device="cuda", lds=True):
        self.scene = scene
        rec = np.ascontiguousarray(scene.prims.astype(np.float32))
        self.prims = torch.from_numpy(rec.copy()).to(device)
        s = GiScene()
        s.prims = self.prims.data_ptr() if len(rec) else None
        s.n_prims = len(rec)
        s.has_room = 1 if scene.has_room else 0
        s.room_lo, s.room_hi = _f3(scene.room_lo), _f3(scene.room_hi)
        s.wall_albedo, s.wall_emit = _f3(scene.wall_albedo), _f3(scene.wall_emit)
        s.sky = _f3(scene.sky)
        s.eps = float(scene.eps)
        s.options = 0 if lds else OPT_NO_LDS
        # a glossy layer on any primitive (record slot 11 = k_s > 0) selects the glossy kernels
        self.glossy = bool(len(rec) and np.any(rec[:, 11] > 0))
        if self.glossy:
            s.options |= OPT_GLOSSY
        # emitters light sampling draws from: the emissive spheres, in index order
        em = [i for i in range(len(rec)) if rec.view(np.uint32)[i, 3] == sg.PRIM_SPHERE and np.any(rec[i, 12:15] > 0)]
        if len(em) > 32:
            raise GiError("more than 32 emissive spheres")
        s.n_emitters = len(em)
        for j, e in enumerate(em):
            s.emitters[j] = e
        self.cell_start = self.cell_items = None
        if grid_res is not None:
            lo, hi = scene.bounds()
            res = (C.c_uint32 * 3)(*[int(v) for v in grid_res])
            lo_c, hi_c = _f3(lo), _f3(hi)
            ncell = int(grid_res[0]) * int(grid_res[1]) * int(grid_res[2])
            start = np.zeros(ncell + 1, np.uint32)
            n_items = C.c_uint32()
            L = load()
            st = L.gi_accel_build_host(rec.ctypes.data_as(_P), len(rec), lo_c, hi_c, res,
                                       start.ctypes.data_as(_P), None, 0, C.byref(n_items))
            items = np.zeros(max(int(n_items.value), 1), np.uint32)
            st = L.gi_accel_build_host(rec.ctypes.data_as(_P), len(rec), lo_c, hi_c, res,
                                       start.ctypes.data_as(_P), items.ctypes.data_as(_P),
                                       len(items), C.byref(n_items))
            check(st, "gi_accel_build_host")
            self.cell_start = torch.from_numpy(start.view(np.int32).copy()).to(device)
            self.cell_items = torch.from_numpy(items.view(np.int32).copy()).to(device)
            s.grid_res = res
            s.grid_lo, s.grid_hi = lo_c, hi_c
            s.cell_start = self.cell_start.data_ptr()
            s.cell_items = self.cell_items.data_ptr()
            s.n_items = int(n_items.value)
            self.n_items = int(n_items.value)
        self.c = s

    @property
    def ref(self):
        return C.byref(self.c)


def camera_struct(cam: sg.Camera) -> GiCamera:
    c = GiCamera()
    c.eye, c.fwd, c.right, c.up = _f3(cam.eye), _f3(cam.fwd), _f3(cam.right), _f3(cam.up)
    c.tan_half_fovy = float(cam.tan_half_fovy)
    c.width, c.height = int(cam.width), int(cam.height)
    return c


class GBuffer:
    """G-buffer planes; fmt 'f16' stores normals and albedo in half precision."""

    def __init__(self, W, H, device="cuda", fmt="f32"):
        self.W, self.H, self.fmt = W, H, fmt
        n = W * H
        half = torch.float16 if fmt == "f16" else torch.float32
        self.pos_depth = torch.zeros(n, 4, dtype=torch.float32, device=device)
        self.nrm_prim = torch.zeros(n, 4, dtype=half, device=device)
        self.albedo = torch.zeros(n, 4, dtype=half, device=device)
        self.emit = torch.zeros(n, 4, dtype=torch.float32, device=device)
        g = GiGBuffer()
        g.width, g.height = W, H
        g.pos_depth, g.nrm_prim = self.pos_depth.data_ptr(), self.nrm_prim.data_ptr()
        g.albedo, g.emit = self.albedo.data_ptr(), self.emit.data_ptr()
        g.format = GB_FORMAT[fmt]
        self.c = g

    @property
    def ref(self):
        return C.byref(self.c)

    def to_records(self) -> np.ndarray:
        """(W*H, 14) float64 records in the oracle's G-buffer layout."""
        pd, npm = self.pos_depth.cpu().numpy(), self.nrm_prim.cpu().numpy()
        al, em = self.albedo.cpu().numpy(), self.emit.cpu().numpy()
        rec = np.zeros((self.W * self.H, 14))
        rec[:, 0:3], rec[:, 3:6] = pd[:, 0:3], npm[:, 0:3]
        rec[:, 6:9], rec[:, 9:12] = al[:, 0:3], em[:, 0:3]
        rec[:, 12] = pd[:, 3]
        if self.fmt == "f16":
            p16 = npm[:, 3].view(np.uint16).astype(np.uint64)
            rec[:, 13] = np.where(p16 == 0xFFFF, MISS, p16)
        else:
            rec[:, 13] = npm[:, 3].view(np.uint32)
        return rec

    def load_records(self, rec, pixels=None, scene=None, eye=None):
        """Fill from (W*H, 14) oracle-layout records (rounded to float32); with
        `pixels`, rec holds one record per listed pixel and only those rows
        are written.  A glossy scene's layer (k_s, roughness) is looked up by
        primitive id from `scene`; eye sets the camera position of the buffer."""
        rec = np.asarray(rec, np.float64)
        n = len(rec) if pixels is not None else self.W * self.H
        half = np.float16 if self.fmt == "f16" else np.float32
        pd = np.zeros((n, 4), np.float32)
        npm = np.zeros((n, 4), half)
        al = np.zeros((n, 4), half)
        em = np.zeros((n, 4), np.float32)
        pd[:, 0:3], pd[:, 3] = rec[:, 0:3], rec[:, 12]
        npm[:, 0:3] = rec[:, 3:6]
        prim = rec[:, 13].astype(np.uint64)
        if self.fmt == "f16":
            npm.view(np.uint16)[:, 3] = np.where(prim == MISS, 0xFFFF, prim).astype(np.uint16)
        else:
            npm.view(np.uint32)[:, 3] = prim.astype(np.uint32)
        al[:, 0:3], em[:, 0:3] = rec[:, 6:9], rec[:, 9:12]
        em[:, 3] = 1.0
        if scene is not None and len(scene.prims):
            pr = np.asarray(scene.prims, np.float32)
            own = prim < len(pr)
            ids = np.where(own, prim, 0).astype(np.int64)
            al[:, 3] = np.where(own, pr[ids, 11], 0.0)
            em[:, 3] = np.where(own, pr[ids, 15], 1.0)
        if eye is not None:
            self.c.eye[:] = [float(v) for v in np.asarray(eye, np.float32).reshape(3)]
        idx = None if pixels is None else torch.as_tensor(np.asarray(pixels, np.int64), device=self.pos_depth.device)
        for t, a in ((self.pos_depth, pd), (self.nrm_prim, npm), (self.albedo, al), (self.emit, em)):
            if idx is None:
                t.copy_(torch.from_numpy(a))
            else:
                t[idx] = torch.from_numpy(a).to(t.device)


class Reservoirs:
    def __init__(self, W, H, device="cuda"):
        self.W, self.H = W, H
        n = W * H
        self.y_W = torch.zeros(n, 4, dtype=torch.float32, device=device)
        self.n_wsum = torch.zeros(n, 4, dtype=torch.float32, device=device)
        self.L_M = torch.zeros(n, 4, dtype=torch.float32, device=device)
        self.tag_prim = torch.zeros(n, 2, dtype=torch.int32, device=device)
        r = GiReservoirs()
        r.width, r.height = W, H
        r.y_W, r.n_wsum = self.y_W.data_ptr(), self.n_wsum.data_ptr()
        r.L_M, r.tag_prim = self.L_M.data_ptr(), self.tag_prim.data_ptr()
        self.c = r

    @property
    def ref(self):
        return C.byref(self.c)

    def to_records(self) -> np.ndarray:
        """(W*H, 14) float64 records in the oracle's reservoir layout."""
        a, b = self.y_W.cpu().numpy(), self.n_wsum.cpu().numpy()
        c, d = self.L_M.cpu().numpy(), self.tag_prim.cpu().numpy().view(np.uint32)
        rec = np.zeros((self.W * self.H, 14))
        rec[:, 0:3], rec[:, 10] = a[:, 0:3], a[:, 3]
        rec[:, 3:6], rec[:, 9] = b[:, 0:3], b[:, 3]
        rec[:, 6:9], rec[:, 11] = c[:, 0:3], c[:, 3].view(np.uint32)
        rec[:, 12], rec[:, 13] = d[:, 0], d[:, 1]
        return rec

    def load_records(self, rec, pixels=None):
        """Fill from oracle-layout records; with `pixels`, only those rows."""
        rec = np.asarray(rec, np.float64)
        n = len(rec) if pixels is not None else self.W * self.H
        a = np.zeros((n, 4), np.float32)
        b = np.zeros((n, 4), np.float32)
        c = np.zeros((n, 4), np.float32)
        d = np.zeros((n, 2), np.uint32)
        a[:, 0:3], a[:, 3] = rec[:, 0:3], rec[:, 10]
        b[:, 0:3], b[:, 3] = rec[:, 3:6], rec[:, 9]
        c[:, 0:3] = rec[:, 6:9]
        c.view(np.uint32)[:, 3] = rec[:, 11].astype(np.uint32)
        d[:, 0], d[:, 1] = rec[:, 12].astype(np.uint64), rec[:, 13].astype(np.uint64)
        idx = None if pixels is None else torch.as_tensor(np.asarray(pixels, np.int64), device=self.y_W.device)
        for t, arr in ((self.y_W, a), (self.n_wsum, b), (self.L_M, c), (self.tag_prim, d.view(np.int32))):
            if idx is None:
                t.copy_(torch.from_numpy(arr))
            else:
                t[idx] = torch.from_numpy(arr).to(t.device)


def tiles_to_quads(tiles, N):
    """Gutter-padded tiles (P, (N+2)^2, C) -> bilinear quad records
    (P, (N+1)^2, 4C): record (cx, cy) = texels (cx,cy), (cx+1,cy), (cx,cy+1),
    (cx+1,cy+1)."""
    t = np.asarray(tiles)
    P, C_ = t.shape[0], t.shape[-1]
    T = t.reshape(P, N + 2, N + 2, C_)
    q = np.stack([T[:, :N + 1, :N + 1], T[:, :N + 1, 1:], T[:, 1:, :N + 1], T[:, 1:, 1:]], axis=3)
    return q.reshape(P, (N + 1) ** 2, 4 * C_)


def quads_to_tiles(quads, N, C_):
    """Inverse of tiles_to_quads."""
    q = np.asarray(quads)
    P = q.shape[0]
    Q = q.reshape(P, N + 1, N + 1, 4, C_)
    T = np.zeros((P, N + 2, N + 2, C_), q.dtype)
    T[:, :N + 1, :N + 1] = Q[:, :, :, 0]
    T[:, :N + 1, N + 1] = Q[:, :, N, 1]
    T[:, N + 1, :N + 1] = Q[:, N, :, 2]
    T[:, N + 1, N + 1] = Q[:, N, N, 3]
    return T.reshape(P, (N + 2) ** 2, C_)


class Probes:
    """Probe textures in the library's quad-record layout (see gi.h):
    irradiance records quad-major (record, probe, 12), depth records
    probe-major (probe, record, 8), in the grid's texel format: FP32 with
    depth texels as (mean, mean square), or binary16 with depth texels as
    (mean, variance)."""

    def __init__(self, grid: sg.ProbeGrid, device="cuda"):
        self.grid = grid
        self.texel = getattr(grid, "texel", "f32")
        if self.texel not in TEXEL_FORMAT:
            raise GiError(f"unknown probe texel format {self.texel!r}")
        dt = torch.float16 if self.texel == "f16" else torch.float32
        P = grid.count
        self.irr = torch.zeros((grid.irr_res + 1) ** 2, P, 12, dtype=dt, device=device)
        self.dep = torch.zeros(P, (grid.dep_res + 1) ** 2, 8, dtype=dt, device=device)
        p = GiProbes()
        p.texel = TEXEL_FORMAT[self.texel]
        p.dims = (C.c_uint32 * 3)(*grid.dims)
        p.irr_res, p.dep_res = grid.irr_res, grid.dep_res
        p.lo, p.spacing = _f3(grid.lo), _f3(grid.spacing)
        p.bias_dist, p.var_floor, p.d_max = grid.bias_dist, grid.var_floor, grid.d_max
        p.irr, p.dep = self.irr.data_ptr(), self.dep.data_ptr()
        self.c = p

    @property
    def ref(self):
        return C.byref(self.c)

    def load(self, irr, dep):
        """Fill from gutter-padded tiles: irr (P, (N+2)^2, >=3), dep (P, (Nd+2)^2, 2)."""
        g = self.grid
        d = np.asarray(dep, np.float64)[..., :2]
        if self.texel == "f16":
            # binary16 straight from the caller's values (one rounding, nearest even)
            qi = tiles_to_quads(np.asarray(irr, np.float64)[..., :3], g.irr_res).astype(np.float16)
            # depth texels stored as binary16 (mean, variance) from (mean, mean square)
            mv = np.stack([d[..., 0], d[..., 1] - d[..., 0] * d[..., 0]], axis=-1)
            qd = tiles_to_quads(mv, g.dep_res).astype(np.float16)
        else:
            qi = tiles_to_quads(np.asarray(irr, np.float64)[..., :3], g.irr_res).astype(np.float32)
            qd = tiles_to_quads(d, g.dep_res).astype(np.float32)
        self.irr.copy_(torch.from_numpy(np.ascontiguousarray(qi.swapaxes(0, 1))))
        self.dep.copy_(torch.from_numpy(np.ascontiguousarray(qd)))

    def tiles(self):
        """(irr (P, (N+2)^2, 3), dep (P, (Nd+2)^2, 2)) as gutter-padded tiles."""
        g = self.grid
        return (quads_to_tiles(self.irr_quads(), g.irr_res, 3),
                quads_to_tiles(self.dep_quads(), g.dep_res, 2))

    def dep_quads(self):
        """Depth records (P, (Nd+1)^2, 8) as (mean, mean square) per texel (a
        binary16 volume's mean square rebuilt from its stored mean and variance)."""
        q = self.dep.cpu().numpy().astype(np.float64).reshape(self.grid.count, -1, 4, 2)
        if self.texel == "f16":
            q = np.stack([q[..., 0], q[..., 1] + q[..., 0] * q[..., 0]], axis=-1)
        return q.reshape(self.grid.count, -1, 8)

    def irr_quads(self):
        """Irradiance records probe-major, (P, (N+1)^2, 12), as tiles_to_quads makes them."""
        return np.ascontiguousarray(self.irr.cpu().numpy().astype(np.float32).swapaxes(0, 1))


def params_struct(p: sg.Params) -> GiParams:
    g = GiParams()
    g.M, g.k, g.radius, g.g_max = int(p.M), int(p.k), float(p.radius), float(p.g_max)
    g.cos_n, g.depth_rel, g.m_cap = float(p.cos_n), float(p.depth_rel), float(p.m_cap)
    g.unbiased = int(p.unbiased)
    g.M_light = int(getattr(p, "M_light", 0))
    g.subsample = int(getattr(p, "subsample", 1))
    g.foot_c = float(getattr(p, "foot_c", 0.2))
    g.glossy_depth = int(getattr(p, "glossy_depth", 8))
    return g


# --------------------------------------------------------------------------
# entry points (same names as the C ABI)
# --------------------------------------------------------------------------
def trace_gbuffer(scene: DeviceScene, cam, gb: GBuffer, stream=None):
    c = camera_struct(cam)
    gb.c.eye[:] = [float(v) for v in np.asarray(cam.eye, np.float32).reshape(3)]
    check(load().gi_trace_gbuffer(scene.ref, C.byref(c), gb.ref, _stream(stream)), "gi_trace_gbuffer")


def probe_update(scene: DeviceScene, pin: Probes, pout: Probes, rays, hysteresis, sharpness, seed,
                 frame, stream=None, slider=0.0):
    pp = GiProbeParams(int(rays), float(hysteresis), float(sharpness), float(slider))
    check(load().gi_probe_update(scene.ref, pin.ref, pout.ref, C.byref(pp), int(seed),
                                 int(frame) & 0xFFFFFFFF, _stream(stream)), "gi_probe_update")


def probe_query(probes: Probes, p: torch.Tensor, n: torch.Tensor, stream=None) -> torch.Tensor:
    p, n = p.contiguous().float(), n.contiguous().float()
    out = torch.empty_like(p)
    check(load().gi_probe_query(probes.ref, p.shape[0], _ptr(p, F32), _ptr(n, F32), _ptr(out), _stream(stream)),
          "gi_probe_query")
    return out


def resample_initial(scene, gb, probes, params, out: Reservoirs, resid: torch.Tensor, seed, frame,
                     stream=None):
    pp = params_struct(params)
    check(load().gi_resample_initial(scene.ref, gb.ref, probes.ref, C.byref(pp), out.ref, _ptr(resid, F32),
                                     int(seed), int(frame) & 0xFFFFFFFF, _stream(stream)),
          "gi_resample_initial")


def resample_temporal(scene, gb, gb_prev, cam_prev, cur, hist, params, out, seed, frame, stream=None):
    pp = params_struct(params)
    c = camera_struct(cam_prev)
    check(load().gi_resample_temporal(scene.ref, gb.ref, gb_prev.ref, C.byref(c), cur.ref, hist.ref,
                                      C.byref(pp), out.ref, int(seed), int(frame) & 0xFFFFFFFF,
                                      _stream(stream)), "gi_resample_temporal")


def resample_spatial(scene, gb, res_in, params, spass, out, seed, frame, stream=None):
    pp = params_struct(params)
    check(load().gi_resample_spatial(scene.ref, gb.ref, res_in.ref, C.byref(pp), int(spass), out.ref,
                                     int(seed), int(frame) & 0xFFFFFFFF, _stream(stream)),
          "gi_resample_spatial")


def shade(scene, gb, probes, res, resid, params, out_rgba: torch.Tensor, stream=None, seed=0, frame=0):
    """seed and frame drive the specular recursion of a glossy scene."""
    pp = params_struct(params)
    check(load().gi_shade(scene.ref, gb.ref, probes.ref, res.ref, _ptr(resid, F32), C.byref(pp),
                          _ptr(out_rgba, F32), int(seed), int(frame) & 0xFFFFFFFF, _stream(stream)), "gi_shade")


def path_trace(scene: DeviceScene, gb: GBuffer, spp, seed, sample0=0, out_rgba=None, stream=None):
    """Reference path tracer: mean of spp samples per pixel (float4 plane)."""
    if out_rgba is None:
        out_rgba = torch.zeros(gb.W * gb.H, 4, dtype=torch.float32, device=gb.pos_depth.device)
    check(load().gi_path_trace(scene.ref, gb.ref, int(spp), int(sample0) & 0xFFFFFFFF, int(seed),
                               _ptr(out_rgba, F32), _stream(stream)), "gi_path_trace")
    return out_rgba


def philox(seed: int, ctr: torch.Tensor, stream=None) -> torch.Tensor:
    ctr = ctr.contiguous()
    out = torch.empty_like(ctr)
    check(load().gi_philox(int(seed), ctr.shape[0], _ptr(ctr), _ptr(out), _stream(stream)), "gi_philox")
    return out


def trace_rays(scene: DeviceScene, org: torch.Tensor, d: torch.Tensor, stream=None):
    org, d = org.contiguous().float(), d.contiguous().float()
    n = org.shape[0]
    out = torch.empty(n, 4, dtype=torch.float32, device=org.device)
    prim = torch.empty(n, dtype=torch.int32, device=org.device)
    check(load().gi_trace_rays(scene.ref, n, _ptr(org, F32), _ptr(d, F32), _ptr(out, F32), _ptr(prim, torch.int32),
                               _stream(stream)), "gi_trace_rays")
    return out, prim


# --------------------------------------------------------------------------
# learned radiance cache
# --------------------------------------------------------------------------
class Mlp:
    """Device state of the learned cache: FP32 master parameters, Adam
    moments, inference operands, FP8 scales and the usability state words."""

    def __init__(self, lo, hi, precision="bf16", mode="auto", warmup_steps=16, max_rel_err=1.0,
                 ema_decay=None, device="cuda"):
        f32 = dict(dtype=torch.float32, device=device)
        self.params = torch.zeros(MLP_N_PARAMS, **f32)
        self.adam_m = torch.zeros(MLP_N_PARAMS, **f32)
        self.adam_v = torch.zeros(MLP_N_PARAMS, **f32)
        self.weights = torch.zeros(MLP_WEIGHT_BYTES, dtype=torch.uint8, device=device)
        self.scales = torch.ones(16, **f32)
        self.state = torch.zeros(16, dtype=torch.int32, device=device)
        self.ema = torch.zeros(MLP_N_PARAMS, **f32) if ema_decay is not None else None
        self.step = 0
        m = GiMlp()
        m.params, m.adam_m, m.adam_v = self.params.data_ptr(), self.adam_m.data_ptr(), self.adam_v.data_ptr()
        m.weights, m.scales, m.state = self.weights.data_ptr(), self.scales.data_ptr(), self.state.data_ptr()
        m.ema = self.ema.data_ptr() if self.ema is not None else None
        m.ema_decay = float(ema_decay or 0.0)
        m.pos_lo, m.pos_hi = _f3(lo), _f3(hi)
        m.precision = MLP_PRECISION[precision]
        m.mode = MLP_MODE[mode]
        m.warmup_steps = int(warmup_steps)
        m.max_rel_err = float(max_rel_err)
        self.c = m

    @property
    def ref(self):
        return C.byref(self.c)

    @property
    def precision(self):
        return {v: k for k, v in MLP_PRECISION.items()}[self.c.precision]

    def set_precision(self, precision, stream=None):
        self.c.precision = MLP_PRECISION[precision]
        self.prepare(stream)

    def set_mode(self, mode):
        self.c.mode = MLP_MODE[mode]

    def init(self, seed, stream=None):
        check(load().gi_mlp_init(self.ref, int(seed), _stream(stream)), "gi_mlp_init")
        self.step = 0

    def prepare(self, stream=None):
        check(load().gi_mlp_prepare(self.ref, _stream(stream)), "gi_mlp_prepare")

    def load_params(self, flat, stream=None):
        """Set the master parameters (rounded to FP32) and prepare."""
        self.params.copy_(torch.from_numpy(np.asarray(flat, np.float32)))
        self.prepare(stream)

    def state_words(self) -> dict:
        w = self.state.cpu().numpy().view(np.uint32)
        out = {}
        for k, i in MLP_STATE.items():
            out[k] = float(w[i:i + 1].view(np.float32)[0]) if k in ("ema_err", "loss", "batch_err") else int(w[i])
        return out


def mlp_infer(mlp: Mlp, pos4: torch.Tensor, nrm4: torch.Tensor, stream=None) -> torch.Tensor:
    pos4, nrm4 = pos4.contiguous().float(), nrm4.contiguous().float()
    out = torch.empty(pos4.shape[0], 4, dtype=torch.float32, device=pos4.device)
    check(load().gi_mlp_infer(mlp.ref, pos4.shape[0], _ptr(pos4, F32), _ptr(nrm4, F32), _ptr(out), _stream(stream)),
          "gi_mlp_infer")
    return out


class MlpBatch:
    """Training samples (float4 planes)."""

    def __init__(self, n, device="cuda"):
        self.n = n
        self.pos = torch.zeros(n, 4, dtype=torch.float32, device=device)
        self.nrm = torch.zeros(n, 4, dtype=torch.float32, device=device)
        self.target = torch.zeros(n, 4, dtype=torch.float32, device=device)
        self.qprobe = torch.zeros(n, 4, dtype=torch.float32, device=device)

    def slice(self, a, b):
        s = MlpBatch.__new__(MlpBatch)
        s.n = b - a
        s.pos, s.nrm, s.target, s.qprobe = self.pos[a:b], self.nrm[a:b], self.target[a:b], self.qprobe[a:b]
        return s


def mlp_make_batch(scene, gb, probes, M, batch: MlpBatch, seed, frame, stream=None):
    check(load().gi_mlp_make_batch(scene.ref, gb.ref, probes.ref, int(M), batch.n, int(seed),
                                   int(frame) & 0xFFFFFFFF, _ptr(batch.pos, F32), _ptr(batch.nrm, F32),
                                   _ptr(batch.target, F32), _ptr(batch.qprobe, F32), _stream(stream)), "gi_mlp_make_batch")


def train_workspace(n, device="cuda") -> torch.Tensor:
    return torch.empty(int(load().gi_mlp_train_workspace_bytes(n)), dtype=torch.uint8, device=device)


def mlp_grad(mlp: Mlp, batch: MlpBatch, grad: torch.Tensor, ws: torch.Tensor, stream=None, qprobe=True):
    check(load().gi_mlp_grad(mlp.ref, batch.n, _ptr(batch.pos, F32), _ptr(batch.nrm, F32), _ptr(batch.target, F32),
                             _ptr(batch.qprobe, F32) if qprobe else None, _ptr(grad, F32), _ptr(ws), ws.numel(),
                             _stream(stream)), "gi_mlp_grad")


def mlp_adam(mlp: Mlp, grad: torch.Tensor, t, lr=1e-2, stream=None):
    check(load().gi_mlp_adam(mlp.ref, _ptr(grad, F32), int(t), float(lr), _stream(stream)), "gi_mlp_adam")


def mlp_train_step(mlp: Mlp, batch: MlpBatch, t, lr, ws: torch.Tensor, stream=None):
    check(load().gi_mlp_train_step(mlp.ref, batch.n, _ptr(batch.pos, F32), _ptr(batch.nrm, F32), _ptr(batch.target, F32),
                                   _ptr(batch.qprobe, F32), int(t), float(lr), _ptr(ws), ws.numel(),
                                   _stream(stream)), "gi_mlp_train_step")


def mlp_train_step_noalloc(mlp: Mlp, batch: MlpBatch, t, lr, stream=None):
    """gi_mlp_train_step with the library's per-GPU scratch (no workspace)."""
    check(load().gi_mlp_train_step_noalloc(mlp.ref, batch.n, _ptr(batch.pos, F32), _ptr(batch.nrm, F32),
                                           _ptr(batch.target, F32), _ptr(batch.qprobe, F32), int(t), float(lr),
                                           _stream(stream)), "gi_mlp_train_step_noalloc")


def initial_mlp_workspace(W, H, M, device="cuda") -> torch.Tensor:
    return torch.empty(int(load().gi_initial_mlp_workspace_bytes(W, H, M)), dtype=torch.uint8, device=device)


def shade_mlp_workspace(W, H, device="cuda") -> torch.Tensor:
    return torch.empty(int(load().gi_shade_mlp_workspace_bytes(W, H)), dtype=torch.uint8, device=device)


def resample_initial_mlp(scene, gb, probes, mlp: Mlp, params, out: Reservoirs, resid, ws, seed, frame,
                         stream=None):
    pp = params_struct(params)
    check(load().gi_resample_initial_mlp(scene.ref, gb.ref, probes.ref, mlp.ref, C.byref(pp), out.ref,
                                         _ptr(resid, F32), _ptr(ws), ws.numel(), int(seed), int(frame) & 0xFFFFFFFF,
                                         _stream(stream)), "gi_resample_initial_mlp")


def shade_mlp(scene, gb, probes, mlp: Mlp, res, resid, params, out_rgba, ws, stream=None):
    pp = params_struct(params)
    check(load().gi_shade_mlp(scene.ref, gb.ref, probes.ref, mlp.ref, res.ref, _ptr(resid, F32), C.byref(pp),
                              _ptr(out_rgba, F32), _ptr(ws), ws.numel(), _stream(stream)), "gi_shade_mlp")


# --------------------------------------------------------------------------
# frame driver
# --------------------------------------------------------------------------
FILL_FRAME_BASE = 0xF0000000


class Renderer:
    """Runs the path frame after frame on the device: G-buffer, (probe
    update), initial RIS, temporal reuse against the last frame's final
    reservoirs, spatial passes (ping-pong) and shading."""

    def __init__(self, cfg: sg.Config, seed: int = 1, width=None, height=None, use_grid=True,
                 device="cuda", scene=None, params=None, lds=True, mlp=None, mlp_mode="auto",
                 mlp_batch=1 << 16, mlp_steps=4, mlp_lr=1e-2, mlp_warmup=16, mlp_seed=7, mlp_ema=0.99,
                 train=True, gb_format="f32"):
        self.cfg = cfg
        self.seed = seed
        self.W, self.H = int(width or cfg.width), int(height or cfg.height)
        self.scene = scene if scene is not None else sg.make_scene(cfg)
        self.dscene = DeviceScene(self.scene, cfg.grid_res if use_grid else None, device, lds=lds)
        self.grid = sg.make_probe_grid(cfg)
        self.params = params if params is not None else cfg.params
        self.probes = [Probes(self.grid, device), Probes(self.grid, device)]
        self.cur_probe = 0
        self.gb = [GBuffer(self.W, self.H, device, gb_format), GBuffer(self.W, self.H, device, gb_format)]
        self.res = [Reservoirs(self.W, self.H, device) for _ in range(4)]
        self.resid = torch.zeros(self.W * self.H, 4, dtype=torch.float32, device=device)
        self.img = torch.zeros(self.W * self.H, 4, dtype=torch.float32, device=device)
        self.hist = None
        self.cam_prev = None
        self.frame_index = 0
        # learned cache (mlp = 'bf16' or 'fp8'): the target of the initial pass
        # and of shading; trained after every frame on the frame's candidates,
        # mlp_steps Adam steps of mlp_batch/mlp_steps samples; inference uses
        # the average of the parameters (decay mlp_ema; None: the parameters)
        self.mlp = None
        if mlp is not None:
            lo, hi = self.scene.bounds()
            self.mlp = Mlp(lo, hi, precision=mlp, mode=mlp_mode, warmup_steps=mlp_warmup, ema_decay=mlp_ema,
                           device=device)
            self.mlp.init(mlp_seed)
            self.train = train
            self.mlp_steps, self.mlp_lr = int(mlp_steps), float(mlp_lr)
            self.batch = MlpBatch(int(mlp_batch), device)
            self.ws_init = initial_mlp_workspace(self.W, self.H, self.params.M, device)
            self.ws_shade = shade_mlp_workspace(self.W, self.H, device)
            self.ws_train = train_workspace(int(mlp_batch) // self.mlp_steps, device)

    @property
    def probe(self) -> Probes:
        return self.probes[self.cur_probe]

    def update_probes(self, rays, hysteresis, frame, stream=None):
        src, dst = self.probes[self.cur_probe], self.probes[1 - self.cur_probe]
        probe_update(self.dscene, src, dst, rays, hysteresis, self.cfg.probe_update.sharpness,
                     self.seed, frame, stream, slider=self.cfg.probe_update.distance_slider)
        self.cur_probe = 1 - self.cur_probe

    def fill_probes(self, stream=None):
        u = self.cfg.probe_update
        for k in range(u.fill_passes):
            self.update_probes(u.fill_rays, 0.0, FILL_FRAME_BASE + k, stream)

    def camera(self, f):
        return sg.make_camera(self.cfg, f, self.W, self.H)

    def frame(self, f=None, stream=None, cam=None):
        """Render frame f; returns the final reservoirs object (history)."""
        f = self.frame_index if f is None else f
        cam = cam if cam is not None else self.camera(f)
        pr = self.params
        gb, gb_prev = self.gb[f & 1], self.gb[(f & 1) ^ 1]
        if self.cfg.probe_update.per_frame:
            u = self.cfg.probe_update
            self.update_probes(u.rays, u.hysteresis, f, stream)
        trace_gbuffer(self.dscene, cam, gb, stream)
        bufs = [r for r in self.res if r is not self.hist]
        a = bufs[0]
        if self.mlp is not None:
            resample_initial_mlp(self.dscene, gb, self.probe, self.mlp, pr, a, self.resid, self.ws_init,
                                 self.seed, f, stream)
            if self.train:
                mlp_make_batch(self.dscene, gb, self.probe, pr.M, self.batch, self.seed, f, stream)
        else:
            resample_initial(self.dscene, gb, self.probe, pr, a, self.resid, self.seed, f, stream)
        cur = a
        spare = bufs[1:]
        if pr.temporal and self.hist is not None:
            t = spare[0]
            resample_temporal(self.dscene, gb, gb_prev, self.cam_prev, cur, self.hist, pr, t, self.seed,
                              f, stream)
            cur = t
        pool = [b for b in self.res if b is not cur and b is not self.hist] + \
            ([self.hist] if self.hist is not None else [])
        for sp in range(pr.n_spatial):
            dst = next(b for b in pool if b is not cur)
            resample_spatial(self.dscene, gb, cur, pr, sp, dst, self.seed, f, stream)
            cur = dst
        if self.mlp is not None:
            shade_mlp(self.dscene, gb, self.probe, self.mlp, cur, self.resid, pr, self.img, self.ws_shade, stream)
            if self.train:
                self.train_mlp(stream)
        else:
            shade(self.dscene, gb, self.probe, cur, self.resid, pr, self.img, stream, seed=self.seed, frame=f)
        self.hist = cur
        self.cam_prev = cam
        self.frame_index = f + 1
        return cur

    def train_mlp(self, stream=None):
        """mlp_steps Adam steps on consecutive slices of the current batch."""
        n = self.batch.n // self.mlp_steps
        for k in range(self.mlp_steps):
            self.mlp.step += 1
            mlp_train_step(self.mlp, self.batch.slice(k * n, (k + 1) * n), self.mlp.step, self.mlp_lr,
                           self.ws_train, stream)
