"""Python binding of libnvgs.so, the NVGS per-frame renderer for MI355X.

Argument marshalling only: every step of the frame runs in the library's HIP
kernels.  PyTorch supplies device memory (the library's scratch comes from
torch's caching allocator through the allocator callback) and the stream.
The names follow the C ABI in include/nvgs.h.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Iterable, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnvgs.so")

OK, E_INVALID, E_STATE, E_NOMEM, E_CAPACITY, E_DEVICE = range(6)
PREC_FP32, PREC_BF16, PREC_FP8, PREC_FP32_SPLIT = 0, 1, 2, 3
RENDER_RECORD_CONTRIB, RENDER_KEEP_DEBUG, RENDER_GRAPH, RENDER_NO_TEST_COUNT = 1, 2, 4, 8
_PREC = {"fp32": PREC_FP32, "bf16": PREC_BF16, "fp8": PREC_FP8, "fp32s": PREC_FP32_SPLIT}


class NvgsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"nvgs status {status}: {msg}")
        self.status = status


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class Allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", C.c_void_p)]


class CreateInfo(C.Structure):
    _fields_ = [("device", C.c_int32), ("stream", C.c_void_p), ("allocator", Allocator)]


class MLP(C.Structure):
    _fields_ = [("width", C.c_int32), ("bands", C.c_int32), ("params", C.c_void_p),
                ("mean_scale", C.c_float), ("cam_scale", C.c_float), ("train_focal", C.c_float),
                ("d_min", C.c_float), ("d_max", C.c_float), ("kind", C.c_int32)]


class Asset(C.Structure):
    _fields_ = [("n", C.c_int64), ("sh_degree", C.c_int32), ("mean", C.c_void_p), ("scale", C.c_void_p),
                ("quat", C.c_void_p), ("opacity", C.c_void_p), ("sh", C.c_void_p), ("mlp", MLP)]


class Instance(C.Structure):
    _fields_ = [("asset", C.c_int32), ("R", C.c_float * 9), ("s", C.c_float), ("t", C.c_float * 3)]


class Camera(C.Structure):
    _fields_ = [("pos", C.c_float * 3), ("R", C.c_float * 9), ("fovy", C.c_float), ("width", C.c_int32),
                ("height", C.c_int32), ("near_plane", C.c_float)]


class RenderOpts(C.Structure):
    _fields_ = [("tile", C.c_int32), ("use_mlp", C.c_int32), ("precision", C.c_int32), ("bg", C.c_float * 3),
                ("flags", C.c_uint32), ("contrib", C.c_void_p), ("split_len", C.c_int32), ("det_clip", C.c_float)]


NUM_STAGES = 8
STAGES = ["setup", "cull_mlp", "compact", "project", "depth_sort", "bin", "tile_sort", "blend"]


class FrameStats(C.Structure):
    _fields_ = [("pairs", C.c_int64), ("in_frustum", C.c_int64), ("queried", C.c_int64), ("kept", C.c_int64),
                ("duplicates", C.c_int64), ("blend_tests", C.c_int64), ("workspace_bytes", C.c_int64),
                ("ms_total", C.c_float),
                ("ms_stage", C.c_float * NUM_STAGES), ("blend_items", C.c_int64), ("chunk_len", C.c_int32),
                ("reserved", C.c_int32)]


class DebugView(C.Structure):
    _fields_ = [("n_splats", C.c_int64), ("n_dup", C.c_int64), ("pair", C.c_void_p), ("rec_a", C.c_void_p),
                ("rec_b", C.c_void_p), ("rec_c", C.c_void_p), ("rect", C.c_void_p), ("sorted_key", C.c_void_p),
                ("sorted_id", C.c_void_p), ("ranges", C.c_void_p), ("tiles_x", C.c_int32), ("tiles_y", C.c_int32),
                ("rec_d", C.c_void_p)]


class MlpShape(C.Structure):
    _fields_ = [("gaussians_per_wave", C.c_int32), ("segments_per_group", C.c_int32)]


class TuneEntry(C.Structure):
    _fields_ = [("tile", C.c_int32), ("gaussians_per_wave", C.c_int32), ("segments_per_group", C.c_int32),
                ("ms", C.c_float)]


class Workspace(C.Structure):
    _fields_ = [(n, C.c_int64) for n in ("total", "assets", "pairs", "splats", "entries", "tiles", "debug", "other",
                                         "splat_capacity", "entry_capacity")]


class TrainOpts(C.Structure):
    _fields_ = [("batch", C.c_int64), ("steps", C.c_int32), ("precision", C.c_int32), ("lr", C.c_float),
                ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float), ("seed", C.c_uint64),
                ("threshold", C.c_float), ("tile", C.c_int32), ("weighting", C.c_int32), ("schedule", C.c_int32),
                ("lr_final", C.c_float)]


# exported symbols of the C ABI and their signatures
_SIGS = {
    "nvgs_create": ([C.POINTER(CreateInfo), C.POINTER(C.c_void_p)], C.c_int32),
    "nvgs_destroy": ([C.c_void_p], None),
    "nvgs_last_error": ([C.c_void_p], C.c_char_p),
    "nvgs_load_assets": ([C.c_void_p, C.POINTER(Asset), C.c_int32], C.c_int32),
    "nvgs_set_instances": ([C.c_void_p, C.POINTER(Instance), C.c_int32], C.c_int32),
    "nvgs_query_visibility": ([C.c_void_p, C.POINTER(Camera), C.c_int32, C.c_int32, C.c_void_p, C.c_void_p],
                              C.c_int32),
    "nvgs_render": ([C.c_void_p, C.POINTER(Camera), C.c_int32, C.POINTER(RenderOpts), C.c_void_p,
                     C.POINTER(FrameStats)], C.c_int32),
    "nvgs_debug_buffers": ([C.c_void_p, C.POINTER(DebugView)], C.c_int32),
    "nvgs_reserve": ([C.c_void_p, C.c_int64, C.c_int64], C.c_int32),
    "nvgs_frame_watermarks": ([C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                               C.c_int32], C.c_int32),
    "nvgs_set_mlp_shape": ([C.c_void_p, C.POINTER(MlpShape)], C.c_int32),
    "nvgs_get_mlp_shape": ([C.c_void_p, C.POINTER(MlpShape)], C.c_int32),
    "nvgs_autotune": ([C.c_void_p, C.POINTER(Camera), C.c_int32, C.POINTER(RenderOpts), C.c_void_p, C.c_int32,
                       C.POINTER(TuneEntry), C.c_int32, C.POINTER(C.c_int32)], C.c_int32),
    "nvgs_make_labels": ([C.c_void_p, C.c_int32, C.POINTER(Camera), C.c_int32, C.c_float, C.c_int32, C.c_int32,
                          C.c_float, C.c_void_p], C.c_int32),
    "nvgs_train_visibility": ([C.c_void_p, C.c_int32, C.POINTER(Camera), C.c_int32, C.c_void_p,
                               C.POINTER(TrainOpts), C.c_void_p, C.c_void_p], C.c_int32),
    "nvgs_mlp_forward": ([C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_int64, C.c_int32, C.c_void_p],
                         C.c_int32),
    "nvgs_mlp_backward": ([C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_int64, C.c_void_p, C.c_int32,
                           C.c_void_p, C.c_void_p], C.c_int32),
    "nvgs_mlp_backward_noalloc": ([C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_int64, C.c_void_p, C.c_int32,
                                   C.c_void_p, C.c_void_p], C.c_int32),
    "nvgs_workspace_info": ([C.c_void_p, C.c_void_p], C.c_int32),
    "nvgs_sort_pairs": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_int32], C.c_int32),
    "nvgs_cmlp_forward": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_void_p], C.c_int32),
    "nvgs_cmlp_backward": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int32, C.c_void_p],
                           C.c_int32),
}

NUM_PARAMS_W64 = 72 * 64 + 64 + 2 * (64 * 64 + 64) + 64 + 1
NUM_PARAMS_W128 = 72 * 128 + 128 + 2 * (128 * 128 + 128) + 128 + 1


def _mlp_width(params):
    """Hidden width of a packed frequency-form MLP from its parameter count."""
    n = int(params.numel())
    if n == NUM_PARAMS_W64:
        return 64
    if n == NUM_PARAMS_W128:
        return 128
    raise ValueError(f"{n} parameters: not a width-64 ({NUM_PARAMS_W64}) or width-128 ({NUM_PARAMS_W128}) MLP")
NUM_PARAMS_COMPACT = (32 * 16 + 32 + 32 * 32 + 32 + 32 + 1) + (32 * 8 + 32 + 32 * 32 + 32 + 6 * 32 + 6)

_lib = None


def lib():
    """Load libnvgs.so; raises if it has not been built (no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "(python -m paper_2511_19202_amd.build)")
        L = C.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


_hip = None


def _hiprt():
    global _hip
    if _hip is None:
        _hip = C.CDLL("libamdhip64.so")
        _hip.hipMemcpyAsync.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int, C.c_void_p]
        _hip.hipMemcpyAsync.restype = C.c_int
        _hip.hipStreamSynchronize.argtypes = [C.c_void_p]
        _hip.hipStreamSynchronize.restype = C.c_int
    return _hip


def _torch():
    import torch
    return torch


# ----------------------------------------------------------------------------
# marshalling helpers
# ----------------------------------------------------------------------------
def camera_struct(cam) -> Camera:
    c = Camera()
    c.pos[:] = [float(v) for v in np.asarray(cam.pos, np.float32).ravel()]
    c.R[:] = [float(v) for v in np.asarray(cam.R, np.float32).ravel()]
    c.fovy = float(cam.fovy)
    c.width = int(cam.width)
    c.height = int(cam.height)
    c.near_plane = float(cam.near)
    return c


def instance_struct(inst) -> Instance:
    h = Instance()
    h.asset = int(inst.asset)
    h.R[:] = [float(v) for v in np.asarray(inst.R, np.float32).ravel()]
    h.s = float(inst.s)
    h.t[:] = [float(v) for v in np.asarray(inst.t, np.float32).ravel()]
    return h


class DeviceAsset:
    """Device copies (torch tensors) of one asset's arrays; owned by the caller."""

    def __init__(self, asset, device):
        torch = _torch()
        f = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float32)).to(device)
        self.mean, self.scale, self.quat = f(asset.mean), f(asset.scale), f(asset.quat)
        self.opacity, self.sh = f(asset.opacity), f(asset.sh)
        self.params = f(asset.mlp.params)
        self.n = int(asset.mean.shape[1])
        self.sh_degree = int(asset.sh_degree)
        self.spec = asset.mlp

    def struct(self) -> Asset:
        a = Asset()
        a.n = self.n
        a.sh_degree = self.sh_degree
        a.mean, a.scale, a.quat = self.mean.data_ptr(), self.scale.data_ptr(), self.quat.data_ptr()
        a.opacity, a.sh = self.opacity.data_ptr(), self.sh.data_ptr()
        sp = self.spec
        a.mlp = MLP(int(sp.width), int(sp.bands), self.params.data_ptr(), float(sp.mean_scale), float(sp.cam_scale),
                    float(sp.train_focal), float(sp.d_min), float(sp.d_max), int(sp.kind))
        return a


def torch_allocator(device, blocks: dict):
    """Allocator callbacks backed by torch's caching allocator; `blocks` keeps
    the tensors alive by address.  They never raise: ctypes leaves a raising
    callback's return value undefined, which the library would take for
    memory.  A failed allocation returns NULL (the library reports E_NOMEM)."""
    torch = _torch()

    def _alloc(nbytes, user):
        for attempt in range(2):
            try:
                t = torch.empty(int(nbytes), dtype=torch.uint8, device=device)
                p = t.data_ptr()
                blocks[p] = t
                return p
            except Exception:
                if attempt == 0 and getattr(device, "type", str(device)) == "cuda":
                    try:
                        torch.cuda.empty_cache()
                    except Exception:
                        return None
        return None

    def _free(ptr, user):
        try:
            t = blocks.pop(int(ptr or 0), None)
            if t is not None and t.numel() >= (1 << 30) and t.is_cuda:
                del t
                torch.cuda.empty_cache()  # hand large blocks back so a larger buffer can take their place
        except Exception:
            pass

    return ALLOC_FN(_alloc), FREE_FN(_free)


class Context:
    """One renderer context on a device and torch stream."""

    def __init__(self, device: int = 0, stream=None):
        global _train_methods_installed
        if not _train_methods_installed:
            _train_methods()
            _train_methods_installed = True
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible to torch")
        self.L = lib()
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._blocks = {}
        self._alloc_cb, self._free_cb = torch_allocator(self.device, self._blocks)
        info = CreateInfo(device, C.c_void_p(self.stream.cuda_stream), Allocator(self._alloc_cb, self._free_cb, None))
        h = C.c_void_p()
        st = self.L.nvgs_create(C.byref(info), C.byref(h))
        if st != OK:
            raise NvgsError(st, "nvgs_create failed")
        self.h = h
        self.assets = []
        self.instances = []
        self.P = 0

    def close(self):
        if getattr(self, "h", None):
            self.L.nvgs_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int):
        if st != OK:
            raise NvgsError(st, self.L.nvgs_last_error(self.h).decode())

    # -- asset store and instances ------------------------------------------
    def load_assets(self, assets: Sequence):
        self.assets = [a if isinstance(a, DeviceAsset) else DeviceAsset(a, self.device) for a in assets]
        arr = (Asset * len(self.assets))(*[a.struct() for a in self.assets])
        self._check(self.L.nvgs_load_assets(self.h, arr, len(self.assets)))

    def set_instances(self, instances: Sequence):
        arr = (Instance * len(instances))(*[instance_struct(i) for i in instances])
        self._check(self.L.nvgs_set_instances(self.h, arr, len(instances)))
        self.instances = list(instances)
        self.P = sum(self.assets[i.asset].n for i in instances)

    # -- per frame -----------------------------------------------------------
    def _cams(self, cams):
        cams = list(cams)
        return (Camera * len(cams))(*[camera_struct(c) for c in cams]), len(cams)

    def query_visibility(self, cams: Iterable, precision="fp32", want_logits: bool = True):
        torch = _torch()
        arr, n = self._cams(cams)
        state = torch.empty((n, self.P), dtype=torch.uint8, device=self.device)
        logits = torch.empty((n, self.P), dtype=torch.float32, device=self.device) if want_logits else None
        self._check(self.L.nvgs_query_visibility(self.h, arr, n, _PREC.get(precision, precision), state.data_ptr(),
                                                 logits.data_ptr() if logits is not None else None))
        return state, logits

    def render(self, cams: Iterable, tile: int = 16, use_mlp: bool = True, precision="fp32", bg=(0.0, 0.0, 0.0),
               contrib=None, keep_debug: bool = False, stats: bool = False, out=None, graph: bool = False,
               split: int = 0, det_clip: float = 0.0, count_tests: bool = True):
        """One frame for all cameras.  graph=True: persistent frame (captured
        HIP graph, no synchronisation unless stats); without `out` the image
        goes to a context-owned tensor that the next graph frame overwrites.
        count_tests=False (with stats): blend_tests is -1 and the compositing
        kernels are those of a frame without stats."""
        torch = _torch()
        arr, n = self._cams(cams)
        W, H = arr[0].width, arr[0].height
        if out is not None:
            rgb = out
        elif graph:
            key = (n, H, W)
            if getattr(self, "_graph_out_key", None) != key:
                self._graph_out = torch.empty((n, H, W, 3), dtype=torch.float32, device=self.device)
                self._graph_out_key = key
            rgb = self._graph_out
        else:
            rgb = torch.empty((n, H, W, 3), dtype=torch.float32, device=self.device)
        flags = (RENDER_RECORD_CONTRIB if contrib is not None else 0) | (RENDER_KEEP_DEBUG if keep_debug else 0) | \
            (RENDER_GRAPH if graph else 0) | (0 if count_tests else RENDER_NO_TEST_COUNT)
        opts = RenderOpts(int(tile), int(bool(use_mlp)), _PREC.get(precision, precision), (C.c_float * 3)(*bg), flags,
                          contrib.data_ptr() if contrib is not None else None, int(split), float(det_clip))
        fs = FrameStats() if stats else None
        self._check(self.L.nvgs_render(self.h, arr, n, C.byref(opts), rgb.data_ptr(),
                                       C.byref(fs) if fs is not None else None))
        if stats:
            return rgb, {"pairs": fs.pairs, "in_frustum": fs.in_frustum, "queried": fs.queried, "kept": fs.kept,
                         "duplicates": fs.duplicates, "blend_tests": fs.blend_tests,
                         "workspace_bytes": fs.workspace_bytes, "ms": fs.ms_total,
                         "ms_stage": dict(zip(STAGES, list(fs.ms_stage))), "blend_items": fs.blend_items,
                         "chunk_len": fs.chunk_len}
        return rgb

    def reserve(self, max_splats: int, max_duplicates: int):
        self._check(self.L.nvgs_reserve(self.h, int(max_splats), int(max_duplicates)))

    def workspace_info(self) -> dict:
        """Device memory the context holds, by class (nvgs_workspace)."""
        w = Workspace()
        self._check(self.L.nvgs_workspace_info(self.h, C.byref(w)))
        return {name: int(getattr(w, name)) for name, _ in Workspace._fields_}

    def sort_pairs(self, keys, vals, begin_bit: int = 0, end_bit: int = 32):
        """Stable radix sort, in place, of two contiguous 32-bit device tensors
        (int32 or uint32) of equal length by key bits [begin_bit, end_bit)."""
        torch = _torch()
        ok = (torch.int32, getattr(torch, "uint32", torch.int32))
        if keys.dtype not in ok or vals.dtype not in ok or keys.numel() != vals.numel():
            raise ValueError("sort_pairs: keys and vals must be 32-bit tensors of equal length")
        if not (keys.is_contiguous() and vals.is_contiguous()):
            raise ValueError("sort_pairs: keys and vals must be contiguous")
        if keys.device != self.device or vals.device != self.device:
            raise ValueError("sort_pairs: keys and vals must be on the context's device")
        self._check(self.L.nvgs_sort_pairs(self.h, keys.data_ptr(), vals.data_ptr(), int(keys.numel()),
                                           int(begin_bit), int(end_bit)))

    def watermarks(self, reset: bool = False) -> dict:
        a, b, o = C.c_int64(), C.c_int64(), C.c_int32()
        self._check(self.L.nvgs_frame_watermarks(self.h, C.byref(a), C.byref(b), C.byref(o), int(bool(reset))))
        return {"max_splats": a.value, "max_duplicates": b.value, "overflowed": bool(o.value)}

    @property
    def mlp_shape(self):
        s = MlpShape()
        self._check(self.L.nvgs_get_mlp_shape(self.h, C.byref(s)))
        return (s.gaussians_per_wave, s.segments_per_group)

    @mlp_shape.setter
    def mlp_shape(self, shape):
        s = MlpShape(int(shape[0]), int(shape[1]))
        self._check(self.L.nvgs_set_mlp_shape(self.h, C.byref(s)))

    def autotune(self, cams: Iterable, tile: int = 16, use_mlp: bool = True, precision="fp32", bg=(0.0, 0.0, 0.0),
                 reps: int = 3):
        """Library autotuner: returns (best tile, best MLP shape, table)."""
        torch = _torch()
        arr, n = self._cams(cams)
        rgb = torch.empty((n, arr[0].height, arr[0].width, 3), dtype=torch.float32, device=self.device)
        opts = RenderOpts(int(tile), int(bool(use_mlp)), _PREC.get(precision, precision), (C.c_float * 3)(*bg), 0,
                          None, 0, 0.0)
        cap = 64
        table = (TuneEntry * cap)()
        cnt = C.c_int32()
        self._check(self.L.nvgs_autotune(self.h, arr, n, C.byref(opts), rgb.data_ptr(), int(reps), table, cap,
                                         C.byref(cnt)))
        rows = [{"tile": e.tile, "gaussians_per_wave": e.gaussians_per_wave,
                 "segments_per_group": e.segments_per_group, "ms": e.ms} for e in table[:min(cnt.value, cap)]]
        return opts.tile, self.mlp_shape, rows

    def debug_buffers(self) -> dict:
        """Copies of the last frame's intermediate buffers as torch tensors."""
        torch = _torch()
        v = DebugView()
        self._check(self.L.nvgs_debug_buffers(self.h, C.byref(v)))
        hip = _hiprt()
        ns, nd = int(v.n_splats), int(v.n_dup)

        def grab(ptr, shape, dtype):
            t = torch.empty(shape, dtype=dtype, device=self.device)
            nbytes = t.numel() * t.element_size()
            if ptr and nbytes:
                hip.hipMemcpyAsync(t.data_ptr(), ptr, nbytes, 3, self.stream.cuda_stream)  # device to device
            return t

        out = {
            "n_splats": ns, "n_dup": nd, "tiles_x": int(v.tiles_x), "tiles_y": int(v.tiles_y),
            "rec_a": grab(v.rec_a, (ns, 4), torch.float32),
            "rec_b": grab(v.rec_b, (ns, 4), torch.float32),
            "rec_c": grab(v.rec_c, (ns, 4), torch.float32),
            "rec_d": grab(v.rec_d, (ns, 2), torch.float32),
            "rect": grab(v.rect, (ns, 4), torch.int32),
            "sorted_key": grab(v.sorted_key, (nd,), torch.int32),
            "sorted_id": grab(v.sorted_id, (nd,), torch.int32),
        }
        if v.pair:
            out["pair"] = grab(v.pair, (ns,), torch.int32)
        hip.hipStreamSynchronize(self.stream.cuda_stream)
        return out


def _ptr(t):
    return None if t is None else t.data_ptr()


def _train_methods():
    torch = _torch()

    def make_labels(self, asset: int, views, threshold: float = 1.0 / 255.0, tile: int = 16, aux: int = 0,
                    aux_angle: float = 0.0):
        """Label bits [V][ceil(n/32)] (int32 view of uint32) rendered by the library."""
        arr, V = self._cams(views)
        words = (self.assets[asset].n + 31) // 32
        lab = torch.empty((V, words), dtype=torch.int32, device=self.device)
        self._check(self.L.nvgs_make_labels(self.h, asset, arr, V, float(threshold), int(tile), int(aux),
                                            float(aux_angle), lab.data_ptr()))
        return lab

    def train_visibility(self, asset: int, views, params, labels=None, batch: int = 65536, steps: int = 5000,
                         precision="bf16", lr: float = 1e-3, betas=(0.9, 0.999), eps: float = 1e-8, seed: int = 1,
                         threshold: float = 1.0 / 255.0, tile: int = 16, weighting: int = 0,
                         lr_final: float = 0.0):
        """Train in place; params is a device float32 tensor [13057] (width 64) or
        [42497] (width 128), the asset's own width; returns the loss curve.
        lr_final > 0 selects the warm-up + exponential-decay schedule from lr to lr_final."""
        arr, V = self._cams(views)
        opts = TrainOpts(int(batch), int(steps), _PREC.get(precision, precision), float(lr), float(betas[0]),
                         float(betas[1]), float(eps), int(seed), float(threshold), int(tile), int(weighting),
                         1 if lr_final > 0 else 0, float(lr_final))
        curve = (C.c_float * int(steps))()
        self._check(self.L.nvgs_train_visibility(self.h, asset, arr, V, _ptr(labels), C.byref(opts),
                                                 params.data_ptr(), curve))
        return np.frombuffer(curve, dtype=np.float32).copy()

    def mlp_forward(self, params, X, precision="fp32"):
        z = torch.empty(X.shape[0], dtype=torch.float32, device=self.device)
        self._check(self.L.nvgs_mlp_forward(self.h, params.data_ptr(), _mlp_width(params), X.data_ptr(), X.shape[0],
                                            _PREC.get(precision, precision), z.data_ptr()))
        return z

    def mlp_backward(self, params, X, dlogits, precision="fp32", want_dx=True):
        dp = torch.empty(params.numel(), dtype=torch.float32, device=self.device)
        dx = torch.empty_like(X) if want_dx else None
        self._check(self.L.nvgs_mlp_backward(self.h, params.data_ptr(), _mlp_width(params), X.data_ptr(), X.shape[0],
                                             dlogits.data_ptr(), _PREC.get(precision, precision), dp.data_ptr(),
                                             _ptr(dx)))
        return dp, dx

    def mlp_backward_noalloc(self, params, X, dlogits, dparams, dx=None, precision="fp32"):
        """nvgs_mlp_backward into caller-provided outputs, with no device allocation."""
        self._check(self.L.nvgs_mlp_backward_noalloc(self.h, params.data_ptr(), _mlp_width(params), X.data_ptr(),
                                                     X.shape[0],
                                                     dlogits.data_ptr(), _PREC.get(precision, precision),
                                                     dparams.data_ptr(), _ptr(dx)))
        return dparams, dx

    def cmlp_forward(self, params, X, precision="fp32"):
        """Logits of the compact model on raw inputs X [B, 18]."""
        z = torch.empty(X.shape[0], dtype=torch.float32, device=self.device)
        self._check(self.L.nvgs_cmlp_forward(self.h, params.data_ptr(), X.data_ptr(), X.shape[0],
                                             _PREC.get(precision, precision), z.data_ptr()))
        return z

    def cmlp_backward(self, params, X, dlogits, precision="fp32"):
        dp = torch.empty(NUM_PARAMS_COMPACT, dtype=torch.float32, device=self.device)
        self._check(self.L.nvgs_cmlp_backward(self.h, params.data_ptr(), X.data_ptr(), X.shape[0],
                                              dlogits.data_ptr(), _PREC.get(precision, precision), dp.data_ptr()))
        return dp

    Context.make_labels = make_labels
    Context.train_visibility = train_visibility
    Context.mlp_forward = mlp_forward
    Context.mlp_backward = mlp_backward
    Context.mlp_backward_noalloc = mlp_backward_noalloc
    Context.cmlp_forward = cmlp_forward
    Context.cmlp_backward = cmlp_backward


_train_methods_installed = False


def visibility_mlp_function():
    """torch.autograd.Function over the library's MLP forward and hand-written
    backward: apply(X [B, 72], params [13057 or 42497], ctx, precision) -> logits [B]."""
    torch = _torch()

    class VisibilityMLPFunction(torch.autograd.Function):
        @staticmethod
        def forward(fctx, X, params, nctx, precision="fp32"):
            X = X.contiguous()
            params = params.contiguous()
            fctx.save_for_backward(X, params)
            fctx.nctx = nctx
            fctx.precision = precision
            return nctx.mlp_forward(params, X, precision)

        @staticmethod
        def backward(fctx, grad):
            X, params = fctx.saved_tensors
            dp, dx = fctx.nctx.mlp_backward(params, X, grad.contiguous().float(), fctx.precision,
                                            want_dx=fctx.needs_input_grad[0])
            return dx, dp, None, None

    return VisibilityMLPFunction


def compact_mlp_function():
    """torch.autograd.Function over the compact model's forward and
    hand-written backward: apply(X [B, 18], params [3175], ctx, precision)
    -> logits [B]; gradients flow to the parameters only."""
    torch = _torch()

    class CompactMLPFunction(torch.autograd.Function):
        @staticmethod
        def forward(fctx, X, params, nctx, precision="fp32"):
            X = X.contiguous()
            params = params.contiguous()
            fctx.save_for_backward(X, params)
            fctx.nctx = nctx
            fctx.precision = precision
            return nctx.cmlp_forward(params, X, precision)

        @staticmethod
        def backward(fctx, grad):
            X, params = fctx.saved_tensors
            if fctx.needs_input_grad[0]:
                raise NotImplementedError("the compact model's backward gives parameter gradients only")
            return None, fctx.nctx.cmlp_backward(params, X, grad.contiguous().float(), fctx.precision), None, None

    return CompactMLPFunction


def exported_symbols() -> list:
    return list(_SIGS)
