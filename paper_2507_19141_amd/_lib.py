"""ctypes binding of libhash4d.so (declared in include/hash4d.h).

Argument marshalling only: every function here forwards to the C entry point of
the same name, passing raw device pointers (``tensor.data_ptr()``) and the
current HIP stream.  Nothing is computed in Python, and there is no fallback:
if the library is missing or fails to load, every call raises.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhash4d.so")

MAX_LEVELS = 32
F32, BF16, F64 = 0, 1, 2
QUERY_MAJOR, LEVEL_MAJOR = 0, 1
GRAD_OVERWRITE = 0x100  # or-ed into a backward's layout: the gradient output is written, not accumulated
SCHEDULE_GEOMETRIC, SCHEDULE_DOUBLING = 0, 1
STATUS = {0: "H4D_OK", -1: "H4D_EINVAL", -2: "H4D_EUNSUPPORTED", -3: "H4D_EHIP", -4: "H4D_ENOPLAN"}


class H4DError(RuntimeError):
    def __init__(self, fn: str, status: int, msg: str):
        super().__init__(f"{fn} -> {STATUS.get(status, status)}: {msg}")
        self.status = status


class Grid(ctypes.Structure):
    """Mirror of h4d_grid."""
    _fields_ = [("L", ctypes.c_int32), ("F", ctypes.c_int32), ("T", ctypes.c_int64),
                ("res_s", ctypes.c_int32 * MAX_LEVELS), ("res_t", ctypes.c_int32 * MAX_LEVELS),
                ("offset", ctypes.c_int64 * (MAX_LEVELS + 1)), ("dense", ctypes.c_uint8 * MAX_LEVELS),
                ("prime", ctypes.c_uint32 * 4)]

    @property
    def E(self) -> int:
        return int(self.offset[self.L])

    def dense_list(self) -> list:
        return [bool(self.dense[l]) for l in range(self.L)]

    def offsets(self) -> list:
        return [int(self.offset[l]) for l in range(self.L + 1)]


class Grid3(ctypes.Structure):
    """Mirror of h4d_grid3."""
    _fields_ = [("L", ctypes.c_int32), ("F", ctypes.c_int32), ("T", ctypes.c_int64),
                ("res", ctypes.c_int32 * MAX_LEVELS), ("offset", ctypes.c_int64 * (MAX_LEVELS + 1)),
                ("dense", ctypes.c_uint8 * MAX_LEVELS), ("prime", ctypes.c_uint32 * 3)]

    @property
    def E(self) -> int:
        return int(self.offset[self.L])

    def dense_list(self) -> list:
        return [bool(self.dense[l]) for l in range(self.L)]

    def offsets(self) -> list:
        return [int(self.offset[l]) for l in range(self.L + 1)]


class Mlp(ctypes.Structure):
    """Mirror of h4d_mlp."""
    _fields_ = [("in_", ctypes.c_int32), ("hidden", ctypes.c_int32), ("out", ctypes.c_int32)]


MAX_SCENES, MAX_TIMES, MAX_TUNED = 16, 8, 64
PLAN_AUTOTUNE, PLAN_ZERO_GRADS, PLAN_GRAPH = 1, 2, 4


class SceneDesc(ctypes.Structure):
    """Mirror of h4d_scene_desc."""
    _fields_ = [("grid", Grid), ("n", ctypes.c_int64), ("xyz", ctypes.c_void_p), ("n_times", ctypes.c_int32),
                ("times", ctypes.c_float * MAX_TIMES), ("table", ctypes.c_void_p),
                ("table_master", ctypes.c_void_p), ("params", ctypes.c_void_p),
                ("params_master", ctypes.c_void_p), ("feat", ctypes.c_void_p), ("delta", ctypes.c_void_p),
                ("d_delta", ctypes.c_void_p), ("d_table", ctypes.c_void_p), ("d_params", ctypes.c_void_p)]


class TuneResult(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int32), ("qpt", ctypes.c_int32), ("lpb", ctypes.c_int32),
                ("grid", ctypes.c_int32), ("ms", ctypes.c_float)]


class BatchedInfo(ctypes.Structure):
    _fields_ = [("queries", ctypes.c_int64), ("segments", ctypes.c_int32), ("encode_qpt", ctypes.c_int32),
                ("encode_lpb", ctypes.c_int32), ("encode_grid", ctypes.c_int32), ("scatter_tiles", ctypes.c_int32),
                ("scatter_rows_per_tile", ctypes.c_int32), ("graph", ctypes.c_int32),
                ("n_tuned", ctypes.c_int32), ("tuned", TuneResult * MAX_TUNED)]


class Adam(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float),
                ("step", ctypes.c_int32), ("grad_scale", ctypes.c_float)]


ADAM_LAZY, ADAM_ZERO_GRAD = 1, 2

_P = ctypes.c_void_p
_I32, _I64, _F32, _SZ = ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_size_t
_GP = ctypes.POINTER(Grid)
_MP = ctypes.POINTER(Mlp)
_G3P = ctypes.POINTER(Grid3)

# name -> (restype, argtypes); the order follows include/hash4d.h
SIGNATURES = {
    "h4d_last_error": (ctypes.c_char_p, []),
    "h4d_version": (ctypes.c_char_p, []),
    "h4d_grid_schedule": (_I32, [_I32, _I32, _I32, _I32, ctypes.POINTER(_I32)]),
    "h4d_grid_init": (_I32, [_GP, _I32, _I32, ctypes.POINTER(_I32), ctypes.POINTER(_I32), _I64]),
    "h4d_grid3_init": (_I32, [_G3P, _I32, _I32, ctypes.POINTER(_I32), _I64]),
    "hash3d_encode": (_I32, [_G3P, _I32, _P, _P, _I32, _I64, _I32, _P, _P]),
    "h4d_grid_rows": (_I64, [_GP]),
    "hash4d_encode": (_I32, [_GP, _I32, _P, _P, _I64, _I32, _P, _P]),
    "hash4d_encode_backward_workspace_bytes": (_SZ, [_GP, _I64]),
    "hash4d_encode_backward": (_I32, [_GP, _I32, _P, _I64, _I32, _P, _F32, _P, _P, _SZ, _P]),
    "hash4d_encode_backward_checked": (_I32, [_GP, _I32, _P, _I64, _I32, _P, _F32, _P, _P, _SZ, _P, _P]),
    "hash4d_encode_backward_noalloc": (_I32, [_GP, _I32, _P, _I64, _I32, _P, _F32, _P, _P]),
    "hash4d_encode_backward_input_workspace_bytes": (_SZ, [_GP, _I32, _I64]),
    "hash4d_encode_backward_input": (_I32, [_GP, _I32, _P, _P, _I64, _I32, _P, _F32, _P, _P, _SZ, _P]),
    "hash4d_corner_indices": (_I32, [_GP, _P, _I64, _P, _P, _P]),
    "hash4d_deform_apply": (_I32, [_P, _I64, _I32, _P, _P, _P, _P, _P, _P, _P]),
    "smoothness_workspace_bytes": (_SZ, [_GP, _I32, _I64]),
    "smoothness_reg": (_I32, [_GP, _I32, _P, _P, _P, _I64, _F32, _P, _P, _P, _SZ, _P]),
    "hash4d_encode_backward_smooth": (_I32, [_GP, _I32, _P, _P, _P, _I64, _I32, _P, _F32, _F32, _P, _P, _P, _SZ,
                                             _P]),
    "h4d_cast_bf16": (_I32, [_P, _P, _I64, _P]),
    "h4d_count_nonfinite": (_I32, [_P, _I64, _P, _P]),
    "deform_mlp_workspace_bytes": (_SZ, [_MP, _I32, _I64]),
    "deform_mlp_forward": (_I32, [_MP, _I32, _P, _P, _I64, _I32, _I32, _P, _P]),
    "deform_mlp_backward": (_I32, [_MP, _I32, _P, _P, _I64, _I32, _I32, _P, _F32, _F32, _P, _P, _P, _SZ, _P]),
    "deform_mlp_backward_checked": (_I32, [_MP, _I32, _P, _P, _I64, _I32, _I32, _P, _F32, _F32, _P, _P, _P, _SZ, _P,
                                           _P]),
    "hash4d_deform_workspace_bytes": (_SZ, [_GP, _MP, _I32, _I64]),
    "hash4d_deform_forward": (_I32, [_GP, _MP, _I32, _P, _P, _P, _I64, _P, _P, _P]),
    "hash4d_deform_backward": (_I32, [_GP, _MP, _I32, _P, _P, _I64, _P, _P, _F32, _F32, _P, _P, _P, _SZ, _P]),
    "hash4d_batched_plan_create": (_I32, [ctypes.POINTER(_P), ctypes.POINTER(SceneDesc), _I32, _MP, _I32, _F32,
                                          _I32, _P]),
    "hash4d_batched_forward": (_I32, [_P, _P]),
    "hash4d_batched_backward": (_I32, [_P, _P]),
    "hash4d_batched_run": (_I32, [_P, _P]),
    "hash4d_batched_plan_info": (_I32, [_P, ctypes.POINTER(BatchedInfo)]),
    "hash4d_batched_plan_destroy": (None, [_P]),
    "hash4d_collision_workspace_bytes": (_SZ, [_GP, _I32, _I64]),
    "hash4d_collision_census": (_I32, [_GP, _I32, _P, _I64, _P, _P, _SZ, _P]),
    "hash4d_decompose_workspace_bytes": (_SZ, [_I64]),
    "hash4d_decompose": (_I32, [_P, _I64, _F32, _F32, _P, _P, _P, _P, _P, _P, _SZ, _P]),
    "h4d_adam_step": (_I32, [_P, _P, _P, _P, _I64, _I32, ctypes.POINTER(Adam), _P, _I32, _P]),
    "h4d_probe_gather": (_I32, [_P, _I64, _I32, _I64, ctypes.c_uint32, _P, _P]),
    "h4d_probe_scatter": (_I32, [_P, _I64, _I64, ctypes.c_uint32, _I32, _P]),
    "h4d_probe_copy": (_I32, [_P, _P, _I64, _P]),
    "h4d_probe_lds_atomic": (_I32, [_I32, _I32, _I32, ctypes.c_uint32, _I32, _P, _P]),
}

_lib = None


def load() -> ctypes.CDLL:
    """Load the library once.  torch is imported first so that the library binds to
    the HIP runtime torch already loaded (one runtime per process)."""
    global _lib
    if _lib is not None:
        return _lib
    try:
        import torch  # noqa: F401  (binds libamdhip64.so.7 before the library does)
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2507_19141_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def last_error() -> str:
    return load().h4d_last_error().decode()


def _check(fn: str, st: int) -> None:
    if st != 0:
        raise H4DError(fn, st, last_error())


def ptr(x) -> int | None:
    """Device (or host) address of a tensor, an int address, or None."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def stream_handle(stream=None) -> int | None:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# ------------------------------------------------------------------ grid ----
def h4d_grid_schedule(L: int, n_min: int, n_max: int, rule: int = SCHEDULE_GEOMETRIC) -> list:
    out = (_I32 * L)()
    _check("h4d_grid_schedule", load().h4d_grid_schedule(L, n_min, n_max, rule, out))
    return list(out)


def h4d_grid_init(L: int, F: int, res_s, res_t, T: int) -> Grid:
    g = Grid()
    rs = (_I32 * L)(*[int(v) for v in res_s])
    rt = (_I32 * L)(*[int(v) for v in res_t])
    _check("h4d_grid_init", load().h4d_grid_init(ctypes.byref(g), L, F, rs, rt, T))
    return g


def h4d_grid3_init(L: int, F: int, res, T: int) -> Grid3:
    g = Grid3()
    r = (_I32 * L)(*[int(v) for v in res])
    _check("h4d_grid3_init", load().h4d_grid3_init(ctypes.byref(g), L, F, r, T))
    return g


def h4d_grid_rows(g: Grid) -> int:
    return int(load().h4d_grid_rows(ctypes.byref(g)))


# --------------------------------------------------------------- encoder ----
def hash4d_encode(g: Grid, table_dt: int, table, xyzt, n: int, feat, layout: int = QUERY_MAJOR,
                  stream=None) -> None:
    _check("hash4d_encode", load().hash4d_encode(ctypes.byref(g), table_dt, ptr(table), ptr(xyzt), n, layout,
                                                 ptr(feat), stream_handle(stream)))


def hash3d_encode(g: Grid3, table_dt: int, table, xyz, stride: int, n: int, feat, layout: int = QUERY_MAJOR,
                  stream=None) -> None:
    _check("hash3d_encode", load().hash3d_encode(ctypes.byref(g), table_dt, ptr(table), ptr(xyz), stride, n, layout,
                                                 ptr(feat), stream_handle(stream)))


def hash4d_encode_backward_workspace_bytes(g: Grid, n: int) -> int:
    return int(load().hash4d_encode_backward_workspace_bytes(ctypes.byref(g), n))


def hash4d_encode_backward(g: Grid, grad_dt: int, xyzt, n: int, d_feat, grad_scale: float, d_table, workspace,
                           ws_bytes: int, layout: int = QUERY_MAJOR, stream=None) -> None:
    _check("hash4d_encode_backward",
           load().hash4d_encode_backward(ctypes.byref(g), grad_dt, ptr(xyzt), n, layout, ptr(d_feat), grad_scale,
                                         ptr(d_table), ptr(workspace), ws_bytes, stream_handle(stream)))


def hash4d_encode_backward_checked(g: Grid, grad_dt: int, xyzt, n: int, d_feat, grad_scale: float, d_table,
                                   workspace, ws_bytes: int, nonfinite, layout: int = QUERY_MAJOR,
                                   stream=None) -> None:
    _check("hash4d_encode_backward_checked",
           load().hash4d_encode_backward_checked(ctypes.byref(g), grad_dt, ptr(xyzt), n, layout, ptr(d_feat),
                                                 grad_scale, ptr(d_table), ptr(workspace), ws_bytes, ptr(nonfinite),
                                                 stream_handle(stream)))


def hash4d_encode_backward_noalloc(g: Grid, grad_dt: int, xyzt, n: int, d_feat, grad_scale: float, d_table,
                                   layout: int = QUERY_MAJOR, stream=None) -> None:
    _check("hash4d_encode_backward_noalloc",
           load().hash4d_encode_backward_noalloc(ctypes.byref(g), grad_dt, ptr(xyzt), n, layout, ptr(d_feat),
                                                 grad_scale, ptr(d_table), stream_handle(stream)))


def hash4d_encode_backward_input_workspace_bytes(g: Grid, table_dt: int, n: int) -> int:
    return load().hash4d_encode_backward_input_workspace_bytes(ctypes.byref(g), table_dt, n)


def hash4d_encode_backward_input(g: Grid, table_dt: int, table, xyzt, n: int, d_feat, grad_scale: float, d_xyzt,
                                 layout: int = QUERY_MAJOR, workspace=None, ws_bytes: int = 0, stream=None) -> None:
    _check("hash4d_encode_backward_input",
           load().hash4d_encode_backward_input(ctypes.byref(g), table_dt, ptr(table), ptr(xyzt), n, layout,
                                               ptr(d_feat), grad_scale, ptr(d_xyzt), ptr(workspace), ws_bytes,
                                               stream_handle(stream)))


def hash4d_corner_indices(g: Grid, xyzt, n: int, rows, w, stream=None) -> None:
    _check("hash4d_corner_indices", load().hash4d_corner_indices(ctypes.byref(g), ptr(xyzt), n, ptr(rows), ptr(w),
                                                                 stream_handle(stream)))


def hash4d_deform_apply(delta, n: int, out: int, xyz, rot, scale, xyz_out, rot_out, scale_out, stream=None) -> None:
    _check("hash4d_deform_apply", load().hash4d_deform_apply(ptr(delta), n, out, ptr(xyz), ptr(rot), ptr(scale),
                                                             ptr(xyz_out), ptr(rot_out), ptr(scale_out),
                                                             stream_handle(stream)))


# ------------------------------------------------------------ smoothness ----
def smoothness_workspace_bytes(g: Grid, table_dt: int, n: int) -> int:
    return int(load().smoothness_workspace_bytes(ctypes.byref(g), table_dt, n))


def smoothness_reg(g: Grid, table_dt: int, table, xyzt, eps, n: int, lam: float, loss, d_table, workspace=None,
                   ws_bytes: int = 0, stream=None) -> None:
    _check("smoothness_reg", load().smoothness_reg(ctypes.byref(g), table_dt, ptr(table), ptr(xyzt), ptr(eps), n, lam,
                                                   ptr(loss), ptr(d_table), ptr(workspace), ws_bytes,
                                                   stream_handle(stream)))


def hash4d_encode_backward_smooth(g: Grid, table_dt: int, table, xyzt, eps, n: int, d_feat, grad_scale: float,
                                  lam: float, loss, d_table, workspace, ws_bytes: int, layout: int = QUERY_MAJOR,
                                  stream=None) -> None:
    _check("hash4d_encode_backward_smooth",
           load().hash4d_encode_backward_smooth(ctypes.byref(g), table_dt, ptr(table), ptr(xyzt), ptr(eps), n, layout,
                                                ptr(d_feat), grad_scale, lam, ptr(loss), ptr(d_table),
                                                ptr(workspace), ws_bytes, stream_handle(stream)))


# ------------------------------------------------------- precision form ----
def h4d_cast_bf16(src, dst, count: int, stream=None) -> None:
    _check("h4d_cast_bf16", load().h4d_cast_bf16(ptr(src), ptr(dst), count, stream_handle(stream)))


def h4d_count_nonfinite(p, count: int, counter, stream=None) -> None:
    _check("h4d_count_nonfinite", load().h4d_count_nonfinite(ptr(p), count, ptr(counter), stream_handle(stream)))


# --------------------------------------------------------------- decoder ----
def mlp_shape(n_in: int, hidden: int = 64, out: int = 10) -> Mlp:
    return Mlp(n_in, hidden, out)


def deform_mlp_workspace_bytes(m: Mlp, dt: int, n: int) -> int:
    return int(load().deform_mlp_workspace_bytes(ctypes.byref(m), dt, n))


def deform_mlp_forward(m: Mlp, dt: int, params, feat, n: int, out, layout: int = QUERY_MAJOR, F: int = 0,
                       stream=None) -> None:
    _check("deform_mlp_forward", load().deform_mlp_forward(ctypes.byref(m), dt, ptr(params), ptr(feat), n, layout, F,
                                                           ptr(out), stream_handle(stream)))


def deform_mlp_backward(m: Mlp, dt: int, params, feat, n: int, d_out, loss_scale: float, grad_scale: float,
                        d_feat, d_params, workspace, ws_bytes: int, layout: int = QUERY_MAJOR, F: int = 0,
                        stream=None) -> None:
    _check("deform_mlp_backward",
           load().deform_mlp_backward(ctypes.byref(m), dt, ptr(params), ptr(feat), n, layout, F, ptr(d_out),
                                      loss_scale, grad_scale, ptr(d_feat), ptr(d_params), ptr(workspace), ws_bytes,
                                      stream_handle(stream)))


def deform_mlp_backward_checked(m: Mlp, dt: int, params, feat, n: int, d_out, loss_scale: float, grad_scale: float,
                                d_feat, d_params, workspace, ws_bytes: int, nonfinite, layout: int = QUERY_MAJOR,
                                F: int = 0, stream=None) -> None:
    _check("deform_mlp_backward_checked",
           load().deform_mlp_backward_checked(ctypes.byref(m), dt, ptr(params), ptr(feat), n, layout, F, ptr(d_out),
                                              loss_scale, grad_scale, ptr(d_feat), ptr(d_params), ptr(workspace),
                                              ws_bytes, ptr(nonfinite), stream_handle(stream)))


# ------------------------------------------------------ deformation path ----
def hash4d_deform_workspace_bytes(g: Grid, m: Mlp, dt: int, n: int) -> int:
    return int(load().hash4d_deform_workspace_bytes(ctypes.byref(g), ctypes.byref(m), dt, n))


def hash4d_deform_forward(g: Grid, m: Mlp, dt: int, table, params, xyzt, n: int, feat, delta, stream=None) -> None:
    _check("hash4d_deform_forward",
           load().hash4d_deform_forward(ctypes.byref(g), ctypes.byref(m), dt, ptr(table), ptr(params), ptr(xyzt), n,
                                        ptr(feat), ptr(delta), stream_handle(stream)))


def hash4d_deform_backward(g: Grid, m: Mlp, dt: int, params, xyzt, n: int, feat, d_delta, loss_scale: float,
                           grad_scale: float, d_table, d_params, workspace, ws_bytes: int, stream=None) -> None:
    _check("hash4d_deform_backward",
           load().hash4d_deform_backward(ctypes.byref(g), ctypes.byref(m), dt, ptr(params), ptr(xyzt), n, ptr(feat),
                                         ptr(d_delta), loss_scale, grad_scale, ptr(d_table), ptr(d_params),
                                         ptr(workspace), ws_bytes, stream_handle(stream)))


# ----------------------------------------------------------- batched form ----
class BatchedPlan:
    """Owns an h4d_batched_plan handle (and keeps the scene array alive)."""

    def __init__(self, scenes: list, m: Mlp, dt: int, loss_scale: float = 1.0, flags: int = 0, stream=None):
        arr = (SceneDesc * len(scenes))(*scenes)
        h = ctypes.c_void_p()
        _check("hash4d_batched_plan_create",
               load().hash4d_batched_plan_create(ctypes.byref(h), arr, len(scenes), ctypes.byref(m), dt, loss_scale,
                                                 flags, stream_handle(stream)))
        self.handle, self._scenes = h, arr

    def forward(self, stream=None) -> None:
        _check("hash4d_batched_forward", load().hash4d_batched_forward(self.handle, stream_handle(stream)))

    def backward(self, stream=None) -> None:
        _check("hash4d_batched_backward", load().hash4d_batched_backward(self.handle, stream_handle(stream)))

    def run(self, stream=None) -> None:
        _check("hash4d_batched_run", load().hash4d_batched_run(self.handle, stream_handle(stream)))

    def info(self) -> BatchedInfo:
        info = BatchedInfo()
        _check("hash4d_batched_plan_info", load().hash4d_batched_plan_info(self.handle, ctypes.byref(info)))
        return info

    def destroy(self) -> None:
        if self.handle:
            load().hash4d_batched_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def scene_desc(grid: Grid, n: int, xyz, times, table, params, feat, delta, d_delta, d_table, d_params,
               table_master=None, params_master=None) -> SceneDesc:
    d = SceneDesc()
    d.grid = grid
    d.n = n
    d.xyz = ptr(xyz)
    d.n_times = len(times)
    for i, t in enumerate(times):
        d.times[i] = float(t)
    d.table, d.params = ptr(table), ptr(params)
    d.table_master, d.params_master = ptr(table_master), ptr(params_master)
    d.feat, d.delta, d.d_delta = ptr(feat), ptr(delta), ptr(d_delta)
    d.d_table, d.d_params = ptr(d_table), ptr(d_params)
    return d


# -------------------------------------------------------- roofline probes ----
def h4d_probe_gather(table, rows: int, row_bytes: int, n_loads: int, seed: int, sink, stream=None) -> None:
    _check("h4d_probe_gather", load().h4d_probe_gather(ptr(table), rows, row_bytes, n_loads, seed, ptr(sink),
                                                       stream_handle(stream)))


def h4d_probe_scatter(table, rows: int, n_updates: int, seed: int, mode: int = 0, stream=None) -> None:
    _check("h4d_probe_scatter", load().h4d_probe_scatter(ptr(table), rows, n_updates, seed, mode,
                                                         stream_handle(stream)))


def h4d_probe_copy(src, dst, nbytes: int, stream=None) -> None:
    _check("h4d_probe_copy", load().h4d_probe_copy(ptr(src), ptr(dst), nbytes, stream_handle(stream)))


def h4d_probe_lds_atomic(blocks: int, per_thread: int, active: int, seed: int, mode: int, sink, stream=None) -> None:
    _check("h4d_probe_lds_atomic", load().h4d_probe_lds_atomic(blocks, per_thread, active, seed, mode, ptr(sink),
                                                               stream_handle(stream)))


def hash4d_collision_workspace_bytes(g: Grid, level: int, n: int) -> int:
    return int(load().hash4d_collision_workspace_bytes(ctypes.byref(g), level, n))


def hash4d_collision_census(g: Grid, level: int, xyzt, n: int, counts, workspace, ws_bytes: int, stream=None) -> None:
    _check("hash4d_collision_census", load().hash4d_collision_census(ctypes.byref(g), level, ptr(xyzt), n, ptr(counts),
                                                                     ptr(workspace), ws_bytes, stream_handle(stream)))


def hash4d_decompose_workspace_bytes(n: int) -> int:
    return int(load().hash4d_decompose_workspace_bytes(n))


def hash4d_decompose(dp, n: int, k_percent: float, lambda_s: float, dynamic_idx, n_dynamic, is_dynamic, loss, d_dp,
                     workspace, ws_bytes: int, stream=None) -> None:
    _check("hash4d_decompose", load().hash4d_decompose(ptr(dp), n, k_percent, lambda_s, ptr(dynamic_idx),
                                                       ptr(n_dynamic), ptr(is_dynamic), ptr(loss), ptr(d_dp),
                                                       ptr(workspace), ws_bytes, stream_handle(stream)))


def h4d_adam_step(params, grad, m, v, count: int, lr: float, beta1: float, beta2: float, eps: float, step: int,
                  grad_scale: float = 1.0, bf16_out=None, row: int = 1, flags: int = 0, stream=None) -> None:
    hp = Adam(lr, beta1, beta2, eps, step, grad_scale)
    _check("h4d_adam_step", load().h4d_adam_step(ptr(params), ptr(grad), ptr(m), ptr(v), count, row, ctypes.byref(hp),
                                                 ptr(bf16_out), flags, stream_handle(stream)))


def hip_runtimes_loaded() -> list:
    """Distinct libamdhip64 files mapped into this process (should be exactly one)."""
    seen = set()
    with open("/proc/self/maps") as fh:
        for line in fh:
            parts = line.split()
            if len(parts) >= 6 and "libamdhip64" in parts[-1]:
                seen.add(os.path.realpath(parts[-1]))
    return sorted(seen)
