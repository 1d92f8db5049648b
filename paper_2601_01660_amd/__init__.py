"""Python binding of the MI355X DGSM library (``libdgsm.so``, C ABI in include/dgsm.h).

Argument marshalling only: every step of the build, query and transfer runs
in the library's HIP kernels.  Tensors must be contiguous float32 CUDA (ROCm)
tensors; calls are enqueued on ``torch.cuda.current_stream()``.  There is no
CPU fallback: if the library is missing, every entry point raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdgsm.so")

DGSM_SHELLS_UNIFORM, DGSM_SHELLS_GEOMETRIC = 0, 1
DGSM_F32, DGSM_F16 = 0, 1


class _Gaussians(ctypes.Structure):
    _fields_ = [("mean", ctypes.c_void_p), ("scale", ctypes.c_void_p), ("rot", ctypes.c_void_p),
                ("opacity", ctypes.c_void_p), ("n", ctypes.c_int64)]


class _Lights(ctypes.Structure):
    _fields_ = [("pos", ctypes.c_void_p), ("n", ctypes.c_int32), ("kappa", ctypes.c_float), ("beta_mode", ctypes.c_int32)]


BETA_MODES = {"trace": 0, "constant": 1, "density": 2}   # dgsm_beta_mode
PARAMS = {"octahedral": 0, "cubemap": 1}                  # dgsm_param


class _AtlasDesc(ctypes.Structure):
    _fields_ = [("H", ctypes.c_int32), ("W", ctypes.c_int32), ("K", ctypes.c_int32),
                ("spacing", ctypes.c_int32), ("r0", ctypes.c_float), ("r1", ctypes.c_float),
                ("dtype", ctypes.c_int32), ("cull_eps", ctypes.c_float), ("param", ctypes.c_int32)]


class _ShParams(ctypes.Structure):
    _fields_ = [("n_theta", ctypes.c_int32), ("n_phi", ctypes.c_int32), ("q", ctypes.c_float),
                ("clip_max", ctypes.c_float), ("eps", ctypes.c_float), ("gamma", ctypes.c_float),
                ("centroid", ctypes.c_void_p)]


class _MlpTrain(ctypes.Structure):
    _fields_ = [("batch", ctypes.c_int64), ("steps", ctypes.c_int32), ("step0", ctypes.c_int32),
                ("lr0", ctypes.c_float), ("lr1", ctypes.c_float), ("seed", ctypes.c_uint32),
                ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float)]


MLP_PARAMS = 66177


class _RoiBox(ctypes.Structure):
    _fields_ = [("cx", ctypes.c_float), ("cy", ctypes.c_float), ("half", ctypes.c_float), ("zmin", ctypes.c_float),
                ("zmax", ctypes.c_float)]


class _PlanOpts(ctypes.Structure):
    _fields_ = [("frames", ctypes.c_int32), ("static_cache", ctypes.c_int32), ("autotune", ctypes.c_int32),
                ("tile_waves", ctypes.c_int32), ("split_units", ctypes.c_int32), ("chains", ctypes.c_int32),
                ("motion", ctypes.c_int32), ("groups", ctypes.c_int32),
                ("group_start", ctypes.POINTER(ctypes.c_int64)), ("packed", ctypes.c_int32)]


class _AccumOpts(ctypes.Structure):
    _fields_ = [("tile_waves", ctypes.c_int32), ("split_units", ctypes.c_int32), ("packed", ctypes.c_int32)]


MOTIONS = {"rigid": 0, "free": 1}   # dgsm_motion


_LIB = None

# exported symbol -> (restype, argtypes)
SIGNATURES = {
    "dgsm_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "dgsm_build_workspace_size": (ctypes.c_size_t, [ctypes.POINTER(_AtlasDesc), ctypes.c_int64, ctypes.c_int32]),
    "dgsm_build": (ctypes.c_int, [ctypes.POINTER(_Lights), ctypes.POINTER(_Gaussians), ctypes.POINTER(_AtlasDesc),
                                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "dgsm_build_workspace_size_entries": (ctypes.c_size_t, [ctypes.POINTER(_AtlasDesc), ctypes.c_int64,
                                                            ctypes.c_int32, ctypes.c_int64]),
    "dgsm_count_entries": (ctypes.c_int, [ctypes.POINTER(_Lights), ctypes.POINTER(_Gaussians),
                                          ctypes.POINTER(_AtlasDesc), ctypes.c_void_p, ctypes.c_size_t,
                                          ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p]),
    "dgsm_list_entries": (ctypes.c_int, [ctypes.POINTER(_AtlasDesc), ctypes.c_int64, ctypes.c_int32,
                                         ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32,
                                         ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p]),
    "dgsm_build_noalloc": (ctypes.c_int, [ctypes.POINTER(_Lights), ctypes.POINTER(_Gaussians),
                                          ctypes.POINTER(_AtlasDesc), ctypes.c_void_p, ctypes.c_void_p]),
    "dgsm_build_noalloc_max_bytes": (ctypes.c_size_t, []),
    "dgsm_build_roi": (ctypes.c_int, [ctypes.POINTER(_Lights), ctypes.POINTER(_Gaussians), ctypes.POINTER(_AtlasDesc),
                                      ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(_RoiBox), ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "dgsm_bin": (ctypes.c_int, [ctypes.POINTER(_Lights), ctypes.POINTER(_Gaussians), ctypes.POINTER(_AtlasDesc),
                                ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "dgsm_accumulate": (ctypes.c_int, [ctypes.POINTER(_Lights), ctypes.POINTER(_AtlasDesc), ctypes.c_int64,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                       ctypes.c_void_p]),
    "dgsm_query": (ctypes.c_int, [ctypes.POINTER(_Lights), ctypes.POINTER(_AtlasDesc), ctypes.c_void_p,
                                  ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]),
    "sh_transfer_workspace_size": (ctypes.c_size_t, [ctypes.c_int32, ctypes.c_int32]),
    "sh_transfer": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(_Gaussians), ctypes.c_void_p,
                                   ctypes.POINTER(_ShParams), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "dgsm_alpha_centroid": (ctypes.c_int, [ctypes.POINTER(_Gaussians), ctypes.c_void_p, ctypes.c_void_p]),
    "dgsm_plan_create": (ctypes.c_int, [ctypes.POINTER(_Lights), ctypes.POINTER(_AtlasDesc),
                                        ctypes.POINTER(_Gaussians), ctypes.c_int64, ctypes.POINTER(_PlanOpts),
                                        ctypes.POINTER(ctypes.c_void_p)]),
    "dgsm_plan_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Gaussians), ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_int32, ctypes.c_void_p]),
    "dgsm_work_units": (ctypes.c_int, [ctypes.POINTER(_AtlasDesc), ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p,
                                       ctypes.c_size_t, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                       ctypes.c_void_p]),
    "dgsm_query_footprint": (ctypes.c_int, [ctypes.POINTER(_Lights), ctypes.POINTER(_AtlasDesc), ctypes.c_void_p,
                                            ctypes.POINTER(_Gaussians), ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    "dgsm_footprint_stencil7": (None, [ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)]),
    "dgsm_probe_fit_workspace_size": (ctypes.c_size_t, [ctypes.c_int32]),
    "dgsm_probe_fit": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                      ctypes.c_int32, ctypes.c_float, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_size_t, ctypes.c_void_p]),
    "dgsm_check_gaussians": (ctypes.c_int, [ctypes.POINTER(_Gaussians), ctypes.c_void_p,
                                            ctypes.POINTER(ctypes.c_longlong), ctypes.c_void_p]),
    "dgsm_plan_tile_waves": (ctypes.c_int32, [ctypes.c_void_p]),
    "dgsm_plan_split_units": (ctypes.c_int32, [ctypes.c_void_p]),
    "dgsm_plan_packed": (ctypes.c_int32, [ctypes.c_void_p]),
    "dgsm_plan_tuned_from_cache": (ctypes.c_int32, [ctypes.c_void_p]),
    "dgsm_plan_static_knobs": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)]),
    "dgsm_autotune_cache_clear": (None, []),
    "dgsm_plan_time_frame": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Gaussians), ctypes.c_void_p,
                                            ctypes.c_void_p, ctypes.POINTER(ctypes.c_float), ctypes.c_void_p]),
    "dgsm_accumulate_ex": (ctypes.c_int, [ctypes.POINTER(_Lights), ctypes.POINTER(_AtlasDesc), ctypes.c_int64,
                                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                          ctypes.POINTER(_AccumOpts), ctypes.c_void_p, ctypes.c_void_p]),
    "dgsm_plan_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "dgsm_mlp_workspace_size": (ctypes.c_size_t, [ctypes.c_int64]),
    "dgsm_mlp_infer_workspace_size": (ctypes.c_size_t, [ctypes.c_int32]),
    "dgsm_mlp_grad": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(_AtlasDesc),
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                     ctypes.c_void_p]),
    "dgsm_mlp_train": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(_AtlasDesc), ctypes.c_void_p,
                                      ctypes.POINTER(_MlpTrain), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                      ctypes.c_void_p]),
    "dgsm_mlp_check": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_AtlasDesc), ctypes.c_void_p, ctypes.c_int64,
                                      ctypes.c_uint32, ctypes.c_float, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "dgsm_mlp_check_grid_workspace_size": (ctypes.c_size_t, [ctypes.POINTER(_AtlasDesc), ctypes.c_int32]),
    "dgsm_mlp_check_grid": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_AtlasDesc), ctypes.c_void_p,
                                           ctypes.c_int32, ctypes.c_uint32, ctypes.c_float, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "dgsm_mlp_save": (ctypes.c_int, [ctypes.c_char_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                     ctypes.POINTER(_AtlasDesc)]),
    "dgsm_mlp_load": (ctypes.c_int, [ctypes.c_char_p, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(_AtlasDesc)]),
    "dgsm_mlp_infer": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Lights), ctypes.POINTER(_AtlasDesc),
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
}


def lib():
    """The loaded ``libdgsm.so``; raises if it has not been built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"DGSM HIP library not built: {LIB_PATH} is missing "
                               "(run `python -m paper_2601_01660_amd.build`)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB


class DGSMError(RuntimeError):
    pass


def _check(status: int):
    if status != 0:
        raise DGSMError(f"dgsm status {status}: {lib().dgsm_status_string(status).decode()}")


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _cuda(t, name):
    """Require an existing CUDA tensor (buffers the library writes in place)."""
    if t is not None and (not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous CUDA tensor")
    return t


def _buf(t, shape, dtype, name):
    """Require a contiguous CUDA tensor of exactly this shape and dtype: the library
    reads or writes it through a raw pointer sized from the other arguments."""
    _cuda(t, name)
    if t is not None and (tuple(t.shape) != tuple(shape) or t.dtype != dtype):
        raise ValueError(f"{name} must be a {dtype} tensor of shape {tuple(shape)}, "
                         f"got {t.dtype} of shape {tuple(t.shape)}")
    return t


def _rows(t, width, name):
    """Require an [n, width] tensor (after conversion to a float32 CUDA tensor)."""
    if t.dim() != 2 or t.shape[1] != width:
        raise ValueError(f"{name} must be [n, {width}], got shape {tuple(t.shape)}")
    return t


def _shape(t, shape, name, rows=None, width=None):
    """Check the shape of an input before it is moved to the device (None passes):
    an exact ``shape``, or ``rows`` in an allowed set with ``width`` columns."""
    if t is None:
        return None
    got = tuple(t.shape) if hasattr(t, "shape") else tuple(torch.as_tensor(t).shape)
    if shape is not None and got != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {got}")
    if rows is not None and (len(got) != 2 or got[0] not in rows or got[1] != width):
        raise ValueError(f"{name} must be [n, {width}] with n in {rows}, got {got}")
    return t


def _dev(t, dtype=torch.float32):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        t = torch.as_tensor(t)
    if not t.is_cuda:
        t = t.cuda()
    if t.dtype != dtype:
        t = t.to(dtype)
    return t.contiguous()


@dataclass
class GaussianSet:
    """Device-resident Gaussian set (structure of arrays, float32)."""

    mean: torch.Tensor     # [N, 3]
    scale: torch.Tensor    # [N, 3]
    rot: torch.Tensor      # [N, 4] (w, x, y, z)
    opacity: torch.Tensor  # [N]

    @property
    def n(self) -> int:
        return int(self.mean.shape[0])

    @staticmethod
    def from_host(g) -> "GaussianSet":
        """From any object with numpy .mean/.scale/.rot/.opacity (e.g. synth.Gaussians)."""
        return GaussianSet(_dev(g.mean), _dev(g.scale), _dev(g.rot), _dev(g.opacity))

    def struct(self) -> _Gaussians:
        """The C struct of the set, after checking every array against N = mean.shape[0]:
        the library reads 3, 3, 4 and 1 floats per Gaussian through raw pointers."""
        n = int(self.mean.shape[0]) if self.mean.dim() >= 1 else -1
        for f, shape in (("mean", (n, 3)), ("scale", (n, 3)), ("rot", (n, 4)), ("opacity", (n,))):
            t = getattr(self, f)
            if not isinstance(t, torch.Tensor) or tuple(t.shape) != shape:
                got = tuple(t.shape) if isinstance(t, torch.Tensor) else type(t).__name__
                raise ValueError(f"GaussianSet.{f} must have shape {shape}, got {got}")
            if t.dtype != torch.float32:
                raise ValueError(f"GaussianSet.{f} must be float32")
        for f in ("mean", "scale", "rot", "opacity"):
            _cuda(getattr(self, f), f"GaussianSet.{f}")
        return _Gaussians(self.mean.data_ptr(), self.scale.data_ptr(), self.rot.data_ptr(),
                          self.opacity.data_ptr(), self.n)


@dataclass
class Atlas:
    """Atlas description (mirrors dgsm_atlas_desc_t)."""

    H: int
    W: int
    K: int
    spacing: str = "geometric"
    r0: float = 0.05
    r1: float = 8.0
    dtype: str = "f32"
    cull_eps: float = 1e-8
    param: str = "octahedral"

    def struct(self) -> _AtlasDesc:
        sp = {"uniform": DGSM_SHELLS_UNIFORM, "geometric": DGSM_SHELLS_GEOMETRIC}[self.spacing]
        dt = {"f32": DGSM_F32, "f16": DGSM_F16}[self.dtype]
        return _AtlasDesc(self.H, self.W, self.K, sp, self.r0, self.r1, dt, self.cull_eps, PARAMS[self.param])

    @staticmethod
    def cube(F: int, K: int, **kw) -> "Atlas":
        """Cube-map atlas of six F x F faces stored as 2F x 3F texels."""
        return Atlas(2 * F, 3 * F, K, param="cubemap", **kw)

    @property
    def torch_dtype(self):
        return torch.float16 if self.dtype == "f16" else torch.float32

    @staticmethod
    def from_spec(spec, **kw) -> "Atlas":
        """From an object with H, W, K, spacing, r0, r1 (e.g. synth.AtlasSpec)."""
        return Atlas(spec.H, spec.W, spec.K, spec.spacing, spec.r0, spec.r1, **kw)


def dgsm_build_workspace_size(atlas: Atlas, n_gauss: int, n_lights: int) -> int:
    d = atlas.struct()
    return int(lib().dgsm_build_workspace_size(ctypes.byref(d), n_gauss, n_lights))


def dgsm_build_workspace_size_entries(atlas: Atlas, n_gauss: int, n_lights: int, entries: int) -> int:
    """Bytes of a build workspace whose lists hold ``entries`` entries per light."""
    d = atlas.struct()
    return int(lib().dgsm_build_workspace_size_entries(ctypes.byref(d), n_gauss, n_lights, entries))


def dgsm_count_entries(lights, gaussians: GaussianSet, atlas: Atlas, kappa: float = 1.0, workspace=None,
                       beta: str = "trace") -> int:
    """List entries per light (maximum over lights) that this set needs; synchronises."""
    lights = _rows(_dev(lights), 3, "lights")
    L = int(lights.shape[0])
    d = atlas.struct()
    if workspace is None:
        need = dgsm_build_workspace_size_entries(atlas, gaussians.n, L, 0)
        if need == 0:
            raise DGSMError("invalid atlas description")
        workspace = torch.empty(need, dtype=torch.uint8, device=lights.device)
    _cuda(workspace, "workspace")
    lt = _Lights(lights.data_ptr(), L, kappa, BETA_MODES[beta])
    gs = gaussians.struct()
    out = ctypes.c_int64(0)
    _check(lib().dgsm_count_entries(ctypes.byref(lt), ctypes.byref(gs), ctypes.byref(d), _ptr(workspace),
                                    workspace.numel(), ctypes.byref(out), _stream()))
    return int(out.value)


def dgsm_list_entries(atlas: Atlas, n_gauss: int, n_lights: int, workspace, light: int):
    """(entries the last binning of ``light`` needed, capacity of ``workspace``)."""
    _cuda(workspace, "workspace")
    d = atlas.struct()
    out = (ctypes.c_int64 * 2)()
    _check(lib().dgsm_list_entries(ctypes.byref(d), n_gauss, n_lights, _ptr(workspace), workspace.numel(), light,
                                   out, _stream()))
    return int(out[0]), int(out[1])


def dgsm_build(lights, gaussians: GaussianSet, atlas: Atlas, kappa: float = 1.0, out=None, workspace=None,
               beta: str = "trace"):
    """Build T[L, K, H, W] (see dgsm_build in include/dgsm.h)."""
    lights = _rows(_dev(lights), 3, "lights")
    L = int(lights.shape[0])
    d = atlas.struct()
    ws_bytes = dgsm_build_workspace_size(atlas, gaussians.n, L)
    if ws_bytes == 0:
        raise DGSMError("invalid atlas description")
    if workspace is None:   # worst case; a caller's workspace may be sized for its set (dgsm_count_entries)
        workspace = torch.empty(ws_bytes, dtype=torch.uint8, device=lights.device)
    if out is None:
        out = torch.empty((L, atlas.K, atlas.H, atlas.W), dtype=atlas.torch_dtype, device=lights.device)
    _buf(out, (L, atlas.K, atlas.H, atlas.W), atlas.torch_dtype, "out")
    _cuda(workspace, "workspace")
    lt = _Lights(lights.data_ptr(), L, kappa, BETA_MODES[beta])
    gs = gaussians.struct()
    _check(lib().dgsm_build(ctypes.byref(lt), ctypes.byref(gs), ctypes.byref(d), _ptr(out), _ptr(workspace),
                            workspace.numel(), _stream()))
    return out


def dgsm_build_noalloc(lights, gaussians: GaussianSet, atlas: Atlas, out, kappa: float = 1.0,
                       beta: str = "trace"):
    """dgsm_build into a caller-allocated ``out`` [L, K, H, W] with the library's
    fixed scratch array as workspace (no device allocation by the library;
    requests above ``dgsm_build_noalloc_max_bytes()`` raise)."""
    lights = _rows(_dev(lights), 3, "lights")
    L = int(lights.shape[0])
    _buf(out, (L, atlas.K, atlas.H, atlas.W), atlas.torch_dtype, "out")
    d = atlas.struct()
    lt = _Lights(lights.data_ptr(), L, kappa, BETA_MODES[beta])
    gs = gaussians.struct()
    _check(lib().dgsm_build_noalloc(ctypes.byref(lt), ctypes.byref(gs), ctypes.byref(d), _ptr(out), _stream()))
    return out


def dgsm_build_noalloc_max_bytes() -> int:
    return int(lib().dgsm_build_noalloc_max_bytes())


def dgsm_build_roi(lights, gaussians: GaussianSet, atlas: Atlas, receivers, box=None, kappa: float = 1.0, out=None,
                   workspace=None, beta: str = "trace"):
    """Build T[L, K, H, W] restricted to the receivers' region (see dgsm_build_roi in
    include/dgsm.h); box = (cx, cy, half, zmin, zmax) or None (every receiver)."""
    lights = _rows(_dev(lights), 3, "lights")
    receivers = _rows(_dev(receivers), 3, "receivers")
    L = int(lights.shape[0])
    d = atlas.struct()
    ws_bytes = dgsm_build_workspace_size(atlas, gaussians.n, L)
    if ws_bytes == 0:
        raise DGSMError("invalid atlas description")
    if workspace is None:
        workspace = torch.empty(ws_bytes, dtype=torch.uint8, device=lights.device)
    if out is None:
        out = torch.empty((L, atlas.K, atlas.H, atlas.W), dtype=atlas.torch_dtype, device=lights.device)
    _buf(out, (L, atlas.K, atlas.H, atlas.W), atlas.torch_dtype, "out")
    _cuda(workspace, "workspace")
    bx = _RoiBox(*(box if box is not None else (0.0, 0.0, 0.0, 0.0, 0.0)))
    lt = _Lights(lights.data_ptr(), L, kappa, BETA_MODES[beta])
    gs = gaussians.struct()
    _check(lib().dgsm_build_roi(ctypes.byref(lt), ctypes.byref(gs), ctypes.byref(d), _ptr(receivers),
                                int(receivers.shape[0]), ctypes.byref(bx), _ptr(out), _ptr(workspace),
                                workspace.numel(), _stream()))
    return out


def dgsm_bin(lights, gaussians: GaussianSet, atlas: Atlas, workspace, kappa: float = 1.0, beta: str = "trace"):
    """First build phase: culling cones and supertile lists into ``workspace``."""
    lights = _rows(_dev(lights), 3, "lights")
    _cuda(workspace, "workspace")
    d = atlas.struct()
    lt = _Lights(lights.data_ptr(), int(lights.shape[0]), kappa, BETA_MODES[beta])
    gs = gaussians.struct()
    _check(lib().dgsm_bin(ctypes.byref(lt), ctypes.byref(gs), ctypes.byref(d), _ptr(workspace),
                          workspace.numel(), _stream()))


def dgsm_accumulate(lights, atlas: Atlas, n_gauss: int, out, workspace, stats=None):
    """Second build phase: per-tile closed-form accumulation into ``out`` [L, K, H, W].

    ``stats`` (optional int64 CUDA tensor of >= 8 entries, zeroed by the caller)
    receives the work counters documented in dgsm.h."""
    lights = _rows(_dev(lights), 3, "lights")
    _buf(out, (int(lights.shape[0]), atlas.K, atlas.H, atlas.W), atlas.torch_dtype, "out")
    _cuda(workspace, "workspace")
    _cuda(stats, "stats")
    if stats is not None and (stats.dtype != torch.int64 or stats.numel() < 8):
        raise ValueError("stats must be an int64 tensor of at least 8 entries")
    d = atlas.struct()
    lt = _Lights(lights.data_ptr(), int(lights.shape[0]), 1.0)
    _check(lib().dgsm_accumulate(ctypes.byref(lt), ctypes.byref(d), n_gauss, _ptr(out), _ptr(workspace),
                                 workspace.numel(), _ptr(stats), _stream()))
    return out


def dgsm_accumulate_ex(lights, atlas: Atlas, n_gauss: int, out, workspace, tile_waves: int = 8,
                       split_units: int = 0, packed: bool = False, stats=None):
    """dgsm_accumulate with the knobs of the tile accumulation (bitwise the same atlas for every choice)."""
    lights = _rows(_dev(lights), 3, "lights")
    _buf(out, (int(lights.shape[0]), atlas.K, atlas.H, atlas.W), atlas.torch_dtype, "out")
    _cuda(workspace, "workspace")
    _cuda(stats, "stats")
    if stats is not None and (stats.dtype != torch.int64 or stats.numel() < 8):
        raise ValueError("stats must be an int64 tensor of at least 8 entries")
    d = atlas.struct()
    lt = _Lights(lights.data_ptr(), int(lights.shape[0]), 1.0)
    o = _AccumOpts(int(tile_waves), int(split_units), int(packed))
    _check(lib().dgsm_accumulate_ex(ctypes.byref(lt), ctypes.byref(d), n_gauss, _ptr(out), _ptr(workspace),
                                    workspace.numel(), ctypes.byref(o), _ptr(stats), _stream()))
    return out


def dgsm_query_footprint(lights, atlas: Atlas, table, gaussians: GaussianSet, z, w, out=None):
    """Footprint-averaged T[L, N] (offsets z [n, 3] in the principal-axes frame, weights w [n])."""
    lights = _rows(_dev(lights), 3, "lights")
    z = _dev(z)
    w = _dev(w)
    L = int(lights.shape[0])
    if z.numel() != 3 * w.numel():
        raise ValueError("z must be [n, 3] for n weights")
    if out is None:
        out = torch.empty((L, gaussians.n), dtype=torch.float32, device=gaussians.mean.device)
    _buf(out, (L, gaussians.n), torch.float32, "out")
    _buf(table, (L, atlas.K, atlas.H, atlas.W), atlas.torch_dtype, "table")
    d = atlas.struct()
    lt = _Lights(lights.data_ptr(), L, 1.0)
    gs = gaussians.struct()
    _check(lib().dgsm_query_footprint(ctypes.byref(lt), ctypes.byref(d), _ptr(table), ctypes.byref(gs), _ptr(z),
                                      _ptr(w), int(w.numel()), _ptr(out), _stream()))
    return out


def dgsm_footprint_stencil7():
    """(z [7, 3], w [7]) of the library's 7-point stencil, host float32 tensors."""
    z = (ctypes.c_float * 21)()
    w = (ctypes.c_float * 7)()
    lib().dgsm_footprint_stencil7(z, w)
    return torch.tensor(list(z), dtype=torch.float32).reshape(7, 3), torch.tensor(list(w), dtype=torch.float32)


def dgsm_work_units(atlas: Atlas, n_gauss: int, n_lights: int, workspace, light: int):
    """(extra slices, split tiles, hits per slice, total hits) of the last accumulation of ``light``."""
    _cuda(workspace, "workspace")
    d = atlas.struct()
    out = (ctypes.c_int32 * 4)()
    _check(lib().dgsm_work_units(ctypes.byref(d), n_gauss, n_lights, _ptr(workspace), workspace.numel(), light,
                                 out, _stream()))
    return tuple(int(x) for x in out)


def dgsm_query(lights, atlas: Atlas, table, points, out=None):
    """Trilinear lookup T[L, P] of the atlas at points [P, 3]."""
    lights = _rows(_dev(lights), 3, "lights")
    points = _rows(_dev(points), 3, "points")
    L = int(lights.shape[0])
    P = int(points.shape[0])
    if out is None:
        out = torch.empty((L, P), dtype=torch.float32, device=points.device)
    _buf(out, (L, P), torch.float32, "out")
    _buf(table, (L, atlas.K, atlas.H, atlas.W), atlas.torch_dtype, "table")
    d = atlas.struct()
    lt = _Lights(lights.data_ptr(), L, 1.0)
    _check(lib().dgsm_query(ctypes.byref(lt), ctypes.byref(d), _ptr(table), _ptr(points), P, _ptr(out), _stream()))
    return out


def dgsm_probe_fit(Y, D, w, Kp: int = 16, lam: float = 0.0, out=None, workspace=None):
    """SH probe A [Kp, 3] by weighted ridge least squares from samples Y [n, 3] at
    directions D [n, 3] with weights w [n] (Sec. 3.4)."""
    Y, D, w = _dev(Y), _dev(D), _dev(w)
    n = int(w.numel())
    if Y.numel() != 3 * n or D.numel() != 3 * n:
        raise ValueError("Y and D must be [n, 3] for n weights")
    need = int(lib().dgsm_probe_fit_workspace_size(Kp))
    if need == 0:
        raise ValueError("Kp must be 1, 4, 9 or 16")
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=w.device)
    if out is None:
        out = torch.empty((Kp, 3), dtype=torch.float32, device=w.device)
    _buf(out, (Kp, 3), torch.float32, "out")
    _check(lib().dgsm_probe_fit(_ptr(Y), _ptr(D), _ptr(w), n, Kp, lam, _ptr(out), _ptr(workspace),
                                workspace.numel(), _stream()))
    return out


def dgsm_check_gaussians(gaussians: GaussianSet) -> int:
    """Number of Gaussians outside the method's domain (see dgsm.h); synchronises."""
    counter = torch.empty(1, dtype=torch.int64, device=gaussians.mean.device)
    n_bad = ctypes.c_longlong(0)
    gs = gaussians.struct()
    _check(lib().dgsm_check_gaussians(ctypes.byref(gs), _ptr(counter), ctypes.byref(n_bad), _stream()))
    return int(n_bad.value)


def dgsm_alpha_centroid(gaussians: GaussianSet, out=None):
    if out is None:
        out = torch.empty(3, dtype=torch.float32, device=gaussians.mean.device)
    _buf(out, (3,), torch.float32, "out")
    gs = gaussians.struct()
    _check(lib().dgsm_alpha_centroid(ctypes.byref(gs), _ptr(out), _stream()))
    return out


def sh_transfer(probe_sh, gaussians: GaussianSet, colour_sh=None, centroid=None, n_theta=32, n_phi=64,
                q=1.0, clip_max=4.0, eps=1e-6, gamma=1.0, out=None, workspace=None):
    """Per-Gaussian lighting scale [N,3], relit SH [N,16,3] and RGB [N,3] (Sec. 3.5);
    ``out`` = (scale, colour, rgb) buffers to write instead of new ones."""
    N = gaussians.n
    _shape(probe_sh, None, "probe_sh", rows=(1, 4, 9, 16), width=3)
    _shape(colour_sh, (N, 16, 3), "colour_sh")
    _shape(centroid, (3,), "centroid")
    gaussians.struct()
    probe_sh = _dev(probe_sh)
    colour_sh = _dev(colour_sh)
    if centroid is None:
        centroid = dgsm_alpha_centroid(gaussians)
    centroid = _dev(centroid)
    dev = gaussians.mean.device
    if out is not None:
        s, f_out, rgb = out
        _buf(s, (N, 3), torch.float32, "out[0]")
        if colour_sh is not None:
            _buf(f_out, (N, 16, 3), torch.float32, "out[1]")
            _buf(rgb, (N, 3), torch.float32, "out[2]")
        else:
            f_out = rgb = None
    else:
        s = torch.empty((N, 3), dtype=torch.float32, device=dev)
        f_out = torch.empty((N, 16, 3), dtype=torch.float32, device=dev) if colour_sh is not None else None
        rgb = torch.empty((N, 3), dtype=torch.float32, device=dev) if colour_sh is not None else None
    prm = _ShParams(n_theta, n_phi, q, clip_max, eps, gamma, centroid.data_ptr())
    gs = gaussians.struct()
    need = int(lib().sh_transfer_workspace_size(n_theta, n_phi))
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    _cuda(workspace, "workspace")
    _check(lib().sh_transfer(_ptr(probe_sh), int(probe_sh.shape[0]), ctypes.byref(gs), _ptr(colour_sh),
                             ctypes.byref(prm), _ptr(s), _ptr(f_out), _ptr(rgb), _ptr(workspace),
                             workspace.numel(), _stream()))
    return s, f_out, rgb


class Plan:
    """Batched build + query over animation frames (dgsm_plan_* in include/dgsm.h).

    The static set is copied into the plan; each run evaluates ``frames`` frames of
    the static set plus the dynamic set: with ``motion="rigid"`` the groups of the
    dynamic set (``group_start``: G + 1 ascending offsets, default one group)
    translated by ``translations[f][g]``; with ``motion="free"`` frame f of
    per-frame dynamic arrays.
    """

    def __init__(self, lights, atlas: Atlas, static: GaussianSet, n_dynamic: int, frames: int,
                 static_cache: bool = True, autotune: bool = True, tile_waves: int = 8, split_units: int = 0,
                 kappa: float = 1.0, beta: str = "trace", chains: int = 0, motion: str = "rigid",
                 group_start=None, packed: bool = False):
        lights = _rows(_dev(lights), 3, "lights")
        self.L = int(lights.shape[0])
        self.atlas = atlas
        self.n_static = static.n
        self.n_dynamic = int(n_dynamic)
        self.frames = int(frames)
        self.motion = motion
        starts = [0, self.n_dynamic] if group_start is None else [int(x) for x in group_start]
        if motion not in MOTIONS:
            raise ValueError(f"motion must be one of {sorted(MOTIONS)}")
        if starts[0] != 0 or starts[-1] != self.n_dynamic or any(b < a for a, b in zip(starts, starts[1:])):
            raise ValueError("group_start must ascend from 0 to n_dynamic")
        self.groups = len(starts) - 1
        d = atlas.struct()
        lt = _Lights(lights.data_ptr(), self.L, kappa, BETA_MODES[beta])
        gs = static.struct()
        gst = (ctypes.c_int64 * len(starts))(*starts)
        opts = _PlanOpts(self.frames, int(static_cache), int(autotune), int(tile_waves), int(split_units),
                         int(chains), MOTIONS[motion], self.groups, gst, int(packed))
        h = ctypes.c_void_p()
        _check(lib().dgsm_plan_create(ctypes.byref(lt), ctypes.byref(d), ctypes.byref(gs), self.n_dynamic,
                                      ctypes.byref(opts), ctypes.byref(h)))
        self._h = h

    @property
    def n_points(self) -> int:
        return self.n_static + self.n_dynamic

    @property
    def tile_waves(self) -> int:
        return int(lib().dgsm_plan_tile_waves(self._h))

    @property
    def split_units(self) -> int:
        return int(lib().dgsm_plan_split_units(self._h))

    @property
    def packed(self) -> bool:
        return bool(lib().dgsm_plan_packed(self._h))

    @property
    def static_knobs(self):
        """(waves per tile, work units) of the once-per-run static build."""
        out = (ctypes.c_int32 * 2)()
        lib().dgsm_plan_static_knobs(self._h, out)
        return int(out[0]), int(out[1])

    @property
    def tuned_from_cache(self) -> bool:
        return bool(lib().dgsm_plan_tuned_from_cache(self._h))

    def run(self, dynamic: GaussianSet, translations, out=None, use_graph: bool = True):
        """T[frames, L, n_static + n_dynamic] for one run; enqueued on the current stream.
        Without ``out`` the result is the plan's own buffer, overwritten by the next run."""
        dev = dynamic.mean.device
        if self.motion == "rigid":
            translations = _dev(translations)
            shapes = [(self.frames, self.groups, 3)] + ([(self.frames, 3)] if self.groups == 1 else [])
            if tuple(translations.shape) not in shapes:
                raise ValueError(f"translations must be {shapes[0]}, got shape {tuple(translations.shape)}")
            if dynamic.n != self.n_dynamic:
                raise ValueError(f"the plan was made for {self.n_dynamic} dynamic Gaussians, got {dynamic.n}")
            gs = dynamic.struct()
            tptr = _ptr(translations)
        else:
            F, n = self.frames, self.n_dynamic
            for f, w in (("mean", 3), ("scale", 3), ("rot", 4), ("opacity", None)):
                t = getattr(dynamic, f)
                shape = (F, n, w) if w else (F, n)
                if not isinstance(t, torch.Tensor) or tuple(t.shape) != shape or t.dtype != torch.float32:
                    raise ValueError(f"free motion: dynamic.{f} must be float32 {shape}")
                _cuda(t, f"dynamic.{f}")
                if not t.is_contiguous():
                    raise ValueError(f"dynamic.{f} must be contiguous")
            gs = _Gaussians(dynamic.mean.data_ptr(), dynamic.scale.data_ptr(), dynamic.rot.data_ptr(),
                            dynamic.opacity.data_ptr(), n)
            tptr = None
        if out is None:
            # one plan-owned output, so that the captured graph's key stays the same
            # from run to run (a new pointer forces a recapture)
            if getattr(self, "_out", None) is None:
                self._out = torch.empty((self.frames, self.L, self.n_points), dtype=torch.float32, device=dev)
            out = self._out
        _buf(out, (self.frames, self.L, self.n_points), torch.float32, "out")
        _check(lib().dgsm_plan_run(self._h, ctypes.byref(gs), tptr, _ptr(out), int(use_graph), _stream()))
        return out

    def time_frame(self, dynamic: GaussianSet, translations, out):
        """(binning, accumulation, query, restore, static accumulation) ms of frame 0, eagerly
        on the current stream."""
        if self.motion != "rigid":
            raise ValueError("time_frame takes the rigid form of the dynamic set")
        translations = _dev(translations)
        _buf(out, (self.frames, self.L, self.n_points), torch.float32, "out")
        gs = dynamic.struct()
        ms = (ctypes.c_float * 5)()
        _check(lib().dgsm_plan_time_frame(self._h, ctypes.byref(gs), _ptr(translations), _ptr(out), ms, _stream()))
        return tuple(float(x) for x in ms)

    def close(self):
        if getattr(self, "_h", None):
            lib().dgsm_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# learned per-light transmittance field
# ---------------------------------------------------------------------------

def mlp_grad(params, uvrt, atlas: Atlas, grad=None, loss=None, workspace=None):
    """Loss gradient [MLP_PARAMS] at params on samples uvrt [B, 4] = (u, v, rho, target)."""
    params, uvrt = _dev(params), _rows(_dev(uvrt), 4, "uvrt")
    if params.numel() != MLP_PARAMS:
        raise ValueError(f"params must hold {MLP_PARAMS} values")
    B = int(uvrt.shape[0])
    need = int(lib().dgsm_mlp_workspace_size(B))
    if need == 0:
        raise DGSMError("batch must be a positive multiple of 32")
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=params.device)
    grad = torch.empty(MLP_PARAMS, dtype=torch.float32, device=params.device) if grad is None else grad
    loss = torch.empty(1, dtype=torch.float32, device=params.device) if loss is None else loss
    _buf(grad, (MLP_PARAMS,), torch.float32, "grad")
    _buf(loss, (1,), torch.float32, "loss")
    d = atlas.struct()
    _check(lib().dgsm_mlp_grad(_ptr(params), _ptr(uvrt), B, ctypes.byref(d), _ptr(grad), _ptr(loss),
                               _ptr(workspace), workspace.numel(), _stream()))
    return grad, loss


def mlp_train(params, adam_mv, atlas: Atlas, table_l, steps, batch=16384, step0=0, lr0=1e-3, lr1=1e-4,
              seed=1, beta1=0.9, beta2=0.999, eps=1e-8, workspace=None):
    """``steps`` Adam steps (in place on params / adam_mv); returns the per-step losses."""
    _buf(params, (MLP_PARAMS,), torch.float32, "params")
    _buf(adam_mv, (2 * MLP_PARAMS,), torch.float32, "adam_mv")
    _buf(table_l, (atlas.K, atlas.H, atlas.W), atlas.torch_dtype, "table_l")
    need = int(lib().dgsm_mlp_workspace_size(batch))
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=params.device)
    losses = torch.empty(max(steps, 1), dtype=torch.float32, device=params.device)
    opt = _MlpTrain(batch, steps, step0, lr0, lr1, seed, beta1, beta2, eps)
    d = atlas.struct()
    _check(lib().dgsm_mlp_train(_ptr(params), _ptr(adam_mv), ctypes.byref(d), _ptr(table_l), ctypes.byref(opt),
                                _ptr(losses), _ptr(workspace), workspace.numel(), _stream()))
    return losses[:steps]


def mlp_regions(atlas: Atlas) -> int:
    return ((atlas.K + 7) // 8) * ((atlas.H + 7) // 8) * ((atlas.W + 7) // 8)


def mlp_check(params, atlas: Atlas, table_l, n_check=262144, seed=12345, thresh=1e-2):
    """Fallback mask [regions] (uint8) and (flagged samples, max |dT|) on a held-out sample set."""
    params = _dev(params)
    if params.numel() != MLP_PARAMS:
        raise ValueError(f"params must hold {MLP_PARAMS} values")
    _buf(table_l, (atlas.K, atlas.H, atlas.W), atlas.torch_dtype, "table_l")
    dev = params.device
    mask = torch.zeros(mlp_regions(atlas), dtype=torch.uint8, device=dev)
    stats = torch.zeros(2, dtype=torch.int32, device=dev)
    need = int(lib().dgsm_mlp_infer_workspace_size(1)) + ((16 * n_check + 255) // 256) * 256
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    d = atlas.struct()
    _check(lib().dgsm_mlp_check(_ptr(params), ctypes.byref(d), _ptr(table_l), n_check, seed, thresh, _ptr(mask),
                                _ptr(stats), _ptr(ws), ws.numel(), _stream()))
    torch.cuda.current_stream().synchronize()
    st = stats.cpu()
    return mask, int(st[0]), float(st[1:2].view(torch.float32)[0])


def mlp_check_grid(params, atlas: Atlas, table_l, n_per_region=64, seed=12345, thresh=1e-2):
    """Fallback mask [regions] (uint8) and (flagged samples, max |dT|) from every texel centre x shell
    plus n_per_region uniform points in each region."""
    params = _dev(params)
    if params.numel() != MLP_PARAMS:
        raise ValueError(f"params must hold {MLP_PARAMS} values")
    _buf(table_l, (atlas.K, atlas.H, atlas.W), atlas.torch_dtype, "table_l")
    dev = params.device
    d = atlas.struct()
    need = int(lib().dgsm_mlp_check_grid_workspace_size(ctypes.byref(d), n_per_region))
    if need == 0:
        raise DGSMError("invalid atlas for the learned field, or n_per_region < 0")
    mask = torch.zeros(mlp_regions(atlas), dtype=torch.uint8, device=dev)
    stats = torch.zeros(2, dtype=torch.int32, device=dev)
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    _check(lib().dgsm_mlp_check_grid(_ptr(params), ctypes.byref(d), _ptr(table_l), n_per_region, seed, thresh,
                                     _ptr(mask), _ptr(stats), _ptr(ws), ws.numel(), _stream()))
    torch.cuda.current_stream().synchronize()
    st = stats.cpu()
    return mask, int(st[0]), float(st[1:2].view(torch.float32)[0])


def mlp_save(path, params, atlas: Atlas, adam_mv=None, step: int = 0):
    """Write a checkpoint (parameters, optional Adam moments and step, atlas geometry)."""
    p = params.detach().to("cpu", torch.float32).contiguous()
    if p.numel() != MLP_PARAMS:
        raise ValueError(f"params must hold {MLP_PARAMS} values")
    m = None
    if adam_mv is not None:
        m = adam_mv.detach().to("cpu", torch.float32).contiguous()
        if m.numel() != 2 * MLP_PARAMS:
            raise ValueError(f"adam_mv must hold {2 * MLP_PARAMS} values")
    d = atlas.struct()
    _check(lib().dgsm_mlp_save(os.fsencode(path), p.data_ptr(), m.data_ptr() if m is not None else None, int(step),
                               ctypes.byref(d)))


def mlp_load(path, adam: bool = True):
    """(params [MLP_PARAMS], adam_mv [2 MLP_PARAMS] or None, step, Atlas) from a checkpoint, on the host."""
    p = torch.empty(MLP_PARAMS, dtype=torch.float32)
    m = torch.empty(2 * MLP_PARAMS, dtype=torch.float32) if adam else None
    step = ctypes.c_int32(0)
    d = _AtlasDesc()
    _check(lib().dgsm_mlp_load(os.fsencode(path), p.data_ptr(), m.data_ptr() if m is not None else None,
                               ctypes.byref(step), ctypes.byref(d)))
    sp = {DGSM_SHELLS_UNIFORM: "uniform", DGSM_SHELLS_GEOMETRIC: "geometric"}[d.spacing]
    return p, m, int(step.value), Atlas(d.H, d.W, d.K, sp, d.r0, d.r1)


def mlp_infer(params, lights, atlas: Atlas, points, table=None, mask=None, out=None, workspace=None):
    """T[L, P] of each light's network at points; flagged regions fall back to the atlas."""
    params, lights, points = _dev(params), _rows(_dev(lights), 3, "lights"), _rows(_dev(points), 3, "points")
    L, P = int(lights.shape[0]), int(points.shape[0])
    if params.numel() != L * MLP_PARAMS:
        raise ValueError(f"params must hold {L} x {MLP_PARAMS} values")
    _buf(table, (L, atlas.K, atlas.H, atlas.W), atlas.torch_dtype, "table")
    if mask is not None:
        _cuda(mask, "mask")
        if mask.dtype != torch.uint8 or mask.numel() != L * mlp_regions(atlas):
            raise ValueError(f"mask must be uint8 with {L} x {mlp_regions(atlas)} entries")
    _buf(out, (L, P), torch.float32, "out")
    need = int(lib().dgsm_mlp_infer_workspace_size(L))
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=points.device)
    if out is None:
        out = torch.empty((L, P), dtype=torch.float32, device=points.device)
    lt = _Lights(lights.data_ptr(), L, 1.0)
    d = atlas.struct()
    _check(lib().dgsm_mlp_infer(_ptr(params), ctypes.byref(lt), ctypes.byref(d), _ptr(table), _ptr(mask),
                                _ptr(points), P, _ptr(out), _ptr(workspace), workspace.numel(), _stream()))
    return out
