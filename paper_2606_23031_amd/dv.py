"""ctypes binding of the C ABI in include/dv.h (argument marshalling only).

Functions keep the C names (``dv_build_scene``, ``dv_render``,
``dv_render_backward``, ``dv_serve_submit``, ``dv_serve_poll`` ...); they
take torch tensors / numpy arrays / dicts, build the C structs and call the
library.  Every step of rendering runs in the HIP library: if ``libdvox.so``
is missing this module raises at import time.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdvox.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with "
        "`python -m paper_2606_23031_amd.build` (hipcc, gfx950)")
# torch first: the library then binds to the HIP runtime torch brought into
# the process, so tensors and streams of both are the same runtime's (a
# second runtime loaded ahead of torch's would see no device in one of them)
import torch  # noqa: E402,F401
_lib = C.CDLL(LIB_PATH)

DV_OK = 0
DV_PENDING = 1
STATUS_NAMES = {0: "DV_OK", 1: "DV_PENDING", -1: "DV_ERR_INVALID",
                -2: "DV_ERR_OOM", -3: "DV_ERR_DEVICE", -4: "DV_ERR_OVERLAP",
                -5: "DV_ERR_RANGE", -6: "DV_ERR_LIMIT", -7: "DV_ERR_TICKET",
                -8: "DV_ERR_SHUTDOWN"}
DV_OUT_RGB, DV_OUT_DEPTH, DV_OUT_NORMAL, DV_OUT_T = 1, 2, 4, 8


class DVError(RuntimeError):
    def __init__(self, status, where):
        msg = _lib.dv_last_error().decode()
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _check(st, where):
    if st != DV_OK:
        raise DVError(st, where)
    return st


# ------------------------------------------------------------------ structs
class dv_octree_desc(C.Structure):
    _fields_ = [("root_min", C.c_double * 3), ("root_size", C.c_double),
                ("n_voxels", C.c_int32), ("max_level", C.c_int32),
                ("n_corners", C.c_int32), ("sh_degree", C.c_int32),
                ("level", C.c_void_p), ("ijk", C.c_void_p),
                ("corner_idx", C.c_void_p), ("corner_density", C.c_void_p),
                ("sh", C.c_void_p), ("has_box", C.c_int32),
                ("box_min", C.c_double * 3), ("box_max", C.c_double * 3)]


class dv_track_desc(C.Structure):
    _fields_ = [("n_keys", C.c_int32), ("t", C.c_void_p), ("yaw", C.c_void_p),
                ("trans", C.c_void_p)]


class dv_view(C.Structure):
    _fields_ = [("fx", C.c_double), ("fy", C.c_double), ("cx", C.c_double),
                ("cy", C.c_double), ("W", C.c_int32), ("H", C.c_int32),
                ("x0", C.c_int32), ("y0", C.c_int32), ("w", C.c_int32),
                ("h", C.c_int32), ("c2w", C.c_double * 12), ("t", C.c_double)]


class dv_render_opts(C.Structure):
    _fields_ = [("K", C.c_int32), ("eps_stop", C.c_float),
                ("tau_near", C.c_float), ("bg", C.c_float * 3),
                ("explin_c", C.c_float), ("out_mask", C.c_uint32),
                ("sky", C.c_void_p), ("sky_w", C.c_int32), ("sky_h", C.c_int32),
                ("feat", C.POINTER(C.c_void_p)), ("feat_dim", C.c_int32),
                ("feat_group", C.c_int32)]


class dv_outputs(C.Structure):
    _fields_ = [("rgb", C.c_void_p), ("depth", C.c_void_p),
                ("normal", C.c_void_p), ("T", C.c_void_p)]


class dv_out_grads(C.Structure):
    _fields_ = [("rgb", C.c_void_p), ("depth", C.c_void_p),
                ("normal", C.c_void_p), ("T", C.c_void_p)]


class dv_octree_grads(C.Structure):
    _fields_ = [("corner", C.c_void_p), ("sh", C.c_void_p), ("feat", C.c_void_p)]


class dv_param_grads(C.Structure):
    _fields_ = [("octrees", C.POINTER(dv_octree_grads)),
                ("pose", C.c_void_p), ("sky", C.c_void_p)]


class dv_state_info(C.Structure):
    _fields_ = [("n_views", C.c_int32), ("n_visible", C.c_int64),
                ("n_pairs", C.c_int64), ("n_actor_pairs", C.c_int64),
                ("n_tiles", C.c_int64), ("key_bits", C.c_int32),
                ("tile_bits", C.c_int32), ("n_items", C.c_int64),
                ("n_chunk_slots", C.c_int64), ("n_actor_items", C.c_int64),
                ("n_actor_chunk_slots", C.c_int64)]


NUM_STAGES = 14


class dv_stage_times(C.Structure):
    _fields_ = [("ms", C.c_double * NUM_STAGES),
                ("calls", C.c_int64 * NUM_STAGES),
                ("entries_fwd", C.c_int64), ("pieces_fwd", C.c_int64),
                ("entries_bwd", C.c_int64), ("pieces_bwd", C.c_int64),
                ("entries_actor_fwd", C.c_int64), ("pieces_actor_fwd", C.c_int64),
                ("entries_actor_bwd", C.c_int64), ("pieces_actor_bwd", C.c_int64),
                ("wave_entries_fwd", C.c_int64), ("wave_hits_fwd", C.c_int64),
                ("wave_entries_bwd", C.c_int64), ("wave_hits_bwd", C.c_int64)]


class dv_serve_opts(C.Structure):
    _fields_ = [("max_inflight", C.c_int32), ("mem_budget", C.c_int64),
                ("batched", C.c_int32), ("max_batch", C.c_int32),
                ("opts", dv_render_opts)]


class dv_request(C.Structure):
    _fields_ = [("view", dv_view), ("out", dv_outputs)]


class dv_result(C.Structure):
    _fields_ = [("status", C.c_int32), ("t_submit", C.c_double),
                ("t_admit", C.c_double), ("t_done", C.c_double)]


_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t, C.c_int32,
                        C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_size_t, C.c_int32,
                       C.c_void_p)


class dv_allocator(C.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("user", C.c_void_p)]


class dv_loss_view(C.Structure):
    _fields_ = [("h", C.c_int32), ("w", C.c_int32)] + [
        (k, C.c_void_p) for k in ("rgb", "depth", "normal", "T", "rgb_gt",
                                  "depth_lidar", "normal_pseudo", "sky_mask",
                                  "g_rgb", "g_depth", "g_normal", "g_T")]


class dv_loss_weights(C.Structure):
    _fields_ = [(k, C.c_float) for k in ("color", "ssim", "depth", "normal", "sky")]


class dv_adam_param(C.Structure):
    _fields_ = [("p", C.c_void_p), ("g", C.c_void_p), ("m", C.c_void_p),
                ("v", C.c_void_p), ("n", C.c_int64)]


class dv_edit_out(C.Structure):
    _fields_ = [("level", C.c_void_p), ("ijk", C.c_void_p),
                ("corner_idx", C.c_void_p), ("corner_density", C.c_void_p),
                ("sh", C.c_void_p), ("leaf_src", C.c_void_p),
                ("corner_src", C.c_void_p)]


class dv_adam_opts(C.Structure):
    _fields_ = [("lr", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double),
                ("eps", C.c_double), ("step", C.c_int32)]


_P = C.c_void_p
_sig = {
    "dv_loss": (C.c_int32, [_P, C.POINTER(dv_loss_view), C.c_int32,
                            C.POINTER(dv_loss_weights), _P, _P]),
    "dv_adam": (C.c_int32, [_P, C.POINTER(dv_adam_param), C.c_int32,
                            C.POINTER(dv_adam_opts), _P]),
    "dv_ctx_create": (C.c_int32, [C.c_int32, C.POINTER(dv_allocator),
                                  C.POINTER(_P)]),
    "dv_ctx_trim": (C.c_int32, [_P]),
    "dv_ctx_memory": (C.c_int32, [_P, C.POINTER(C.c_int64),
                                  C.POINTER(C.c_int64)]),
    "dv_ctx_destroy": (None, [_P]),
    "dv_last_error": (C.c_char_p, []),
    "dv_version": (C.c_char_p, []),
    "dv_build_scene": (C.c_int32, [_P, C.POINTER(dv_octree_desc), C.c_int32,
                                   C.POINTER(dv_track_desc), C.POINTER(_P)]),
    "dv_scene_destroy": (None, [_P]),
    "dv_validate_octree_host": (C.c_int32, [_P, _P, _P, C.c_int32, C.c_int32,
                                            C.c_int32, C.c_int32, C.c_char_p,
                                            C.c_int32]),
    "dv_track_pose": (C.c_int32, [C.POINTER(dv_track_desc), C.c_double,
                                  C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "dv_render": (C.c_int32, [_P, _P, C.POINTER(dv_view), C.c_int32, _P,
                              C.POINTER(dv_render_opts),
                              C.POINTER(dv_outputs), C.POINTER(_P), _P]),
    "dv_render_backward": (C.c_int32, [_P, _P, _P, C.POINTER(dv_out_grads),
                                       C.POINTER(dv_param_grads), _P]),
    "dv_render_noalloc": (C.c_int32, [_P, _P, C.POINTER(dv_view), C.c_int32, _P,
                                      C.POINTER(dv_render_opts),
                                      C.POINTER(dv_outputs), _P]),
    "dv_noalloc_capacity": (C.c_int64, []),
    "dv_fwd_state_release": (None, [_P]),
    "dv_fwd_state_info": (C.c_int32, [_P, C.POINTER(dv_state_info)]),
    "dv_fwd_state_export_lists": (C.c_int32, [_P, C.c_int32, _P, _P, _P,
                                              C.c_int64, _P, _P, C.c_int64]),
    "dv_ctx_set_profiling": (C.c_int32, [_P, C.c_int32]),
    "dv_ctx_stage_times": (C.c_int32, [_P, C.POINTER(dv_stage_times), C.c_int32]),
    "dv_stage_name": (C.c_char_p, [C.c_int32]),
    "dv_nearest_distance": (C.c_int32, [_P, _P, C.c_int64, _P, C.c_int64,
                                        C.c_double, _P, _P]),
    "dv_corner_prior": (C.c_int32, [_P, C.POINTER(dv_octree_desc), _P, C.c_int64,
                                    C.c_double, C.c_double, C.c_double,
                                    C.c_double, _P, _P]),
    "dv_proximity_flags": (C.c_int32, [_P, C.POINTER(dv_octree_desc), _P,
                                       C.c_int64, C.c_double, _P, _P]),
    "dv_edit_plan": (C.c_int32, [_P, C.POINTER(dv_octree_desc), _P, C.c_int32,
                                 C.POINTER(_P), C.POINTER(C.c_int64),
                                 C.POINTER(C.c_int64), _P]),
    "dv_refine_plan": (C.c_int32, [_P, C.POINTER(dv_octree_desc), _P, C.c_int64,
                                   C.c_double, C.c_double, C.c_int32,
                                   C.POINTER(_P), C.POINTER(C.c_int64),
                                   C.POINTER(C.c_int64), C.POINTER(C.c_int32), _P]),
    "dv_edit_apply": (C.c_int32, [_P, C.POINTER(dv_edit_out), _P]),
    "dv_edit_release": (None, [_P]),
    "dv_serve_create": (C.c_int32, [_P, _P, C.POINTER(dv_serve_opts),
                                    C.POINTER(_P)]),
    "dv_serve_submit": (C.c_int32, [_P, C.POINTER(dv_request),
                                    C.POINTER(C.c_uint64)]),
    "dv_serve_poll": (C.c_int32, [_P, C.c_uint64, C.c_int32,
                                  C.POINTER(dv_result)]),
    "dv_serve_destroy": (C.c_int32, [_P]),
}

EXPORTED = []
for _name, (_res, _args) in _sig.items():
    if hasattr(_lib, _name):
        _f = getattr(_lib, _name)
        _f.restype = _res
        _f.argtypes = _args
        EXPORTED.append(_name)


def lib():
    return _lib


def version():
    return _lib.dv_version().decode()


# ------------------------------------------------------------------ helpers
def _ptr(t):
    if t is None:
        return None
    return C.c_void_p(t.data_ptr())


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def make_view(v):
    """dict (as produced by ``synth``) -> dv_view."""
    cv = dv_view()
    cv.fx, cv.fy, cv.cx, cv.cy = v["fx"], v["fy"], v["cx"], v["cy"]
    cv.W, cv.H = v["W"], v["H"]
    cv.x0, cv.y0, cv.w, cv.h = v["x0"], v["y0"], v["w"], v["h"]
    cv.c2w[:] = [float(x) for x in np.asarray(v["c2w"], np.float64).reshape(12)]
    cv.t = v["t"]
    return cv


def make_opts(o, mask=DV_OUT_RGB | DV_OUT_DEPTH | DV_OUT_T):
    co = dv_render_opts()
    co.K = int(o.get("K", 1))
    co.eps_stop = float(o.get("eps_stop", 1e-4))
    co.tau_near = float(o.get("tau_near", 0.0))
    co.bg[:] = [float(x) for x in o.get("bg", (0.0, 0.0, 0.0))]
    co.explin_c = float(o.get("explin_c", 1.1))
    co.out_mask = int(o.get("out_mask", mask))
    # sky map: a float32 CUDA tensor [3][H][W] kept alive by the caller
    sky = o.get("sky")
    if sky is not None:
        if not (hasattr(sky, "is_cuda") and sky.is_cuda and sky.dim() == 3
                and sky.shape[0] == 3 and sky.is_contiguous()
                and str(sky.dtype) == "torch.float32"):
            raise ValueError("opts['sky'] must be a contiguous float32 CUDA "
                             "tensor [3][H][W]")
        co.sky = sky.data_ptr()
        co.sky_h, co.sky_w = int(sky.shape[1]), int(sky.shape[2])
    # feature render: per octree a float32 CUDA tensor [F][N], and the
    # group of three channels this render composites
    feat = o.get("feat")
    if feat is not None:
        F = int(feat[0].shape[0])
        arr = (C.c_void_p * len(feat))()
        for k, t in enumerate(feat):
            if not (t.is_cuda and t.dim() == 2 and t.shape[0] == F
                    and t.is_contiguous() and str(t.dtype) == "torch.float32"):
                raise ValueError("opts['feat'] entries must be contiguous float32 "
                                 "CUDA tensors [F][N] with one F")
            arr[k] = t.data_ptr()
        co.feat = C.cast(arr, C.POINTER(C.c_void_p))
        co._feat_arr = arr           # kept alive with the struct
        co.feat_dim = F
        co.feat_group = int(o.get("feat_group", 0))
    return co


# ------------------------------------------------------------------ context
def _torch_alloc(user, nbytes, device, stream):
    try:
        return torch.cuda.caching_allocator_alloc(int(nbytes), int(device),
                                                  int(stream or 0))
    except Exception:          # out of memory: the pool trims and retries
        return None


def _torch_free(user, ptr, nbytes, device, stream):
    torch.cuda.caching_allocator_delete(int(ptr))


# the C callbacks must outlive every context created with them
_TORCH_ALLOCATOR = dv_allocator(_ALLOC_FN(_torch_alloc), _FREE_FN(_torch_free),
                                None)


def dv_ctx_create(device=0, torch_memory=True):
    """Context on HIP device ``device``.  With ``torch_memory`` the library's
    device pool takes its blocks from torch's caching allocator (the memory
    shows in torch.cuda.memory_allocated), else from hipMalloc."""
    h = C.c_void_p()
    alloc = C.byref(_TORCH_ALLOCATOR) if torch_memory else None
    _check(_lib.dv_ctx_create(device, alloc, C.byref(h)), "dv_ctx_create")
    return h


def dv_ctx_destroy(ctx):
    _lib.dv_ctx_destroy(ctx)


def dv_ctx_trim(ctx):
    """Hand the pool's idle blocks back to the provider (synchronises)."""
    _check(_lib.dv_ctx_trim(ctx), "dv_ctx_trim")


def dv_ctx_memory(ctx):
    """(bytes in use, bytes cached) of the context's device pool."""
    a, b = C.c_int64(), C.c_int64()
    _check(_lib.dv_ctx_memory(ctx, C.byref(a), C.byref(b)), "dv_ctx_memory")
    return a.value, b.value


PROFILE_EVENTS, PROFILE_COUNTERS = 1, 2


def dv_ctx_set_profiling(ctx, flags):
    _check(_lib.dv_ctx_set_profiling(ctx, flags), "dv_ctx_set_profiling")


def dv_ctx_stage_times(ctx, reset=True):
    """dict: per-stage {name: (ms, calls)} plus work counters."""
    t = dv_stage_times()
    _check(_lib.dv_ctx_stage_times(ctx, C.byref(t), 1 if reset else 0),
           "dv_ctx_stage_times")
    out = {_lib.dv_stage_name(i).decode(): (t.ms[i], t.calls[i])
           for i in range(NUM_STAGES)}
    out["_counters"] = dict(entries_fwd=t.entries_fwd, pieces_fwd=t.pieces_fwd,
                            entries_bwd=t.entries_bwd, pieces_bwd=t.pieces_bwd,
                            entries_actor_fwd=t.entries_actor_fwd,
                            pieces_actor_fwd=t.pieces_actor_fwd,
                            entries_actor_bwd=t.entries_actor_bwd,
                            pieces_actor_bwd=t.pieces_actor_bwd,
                            wave_entries_fwd=t.wave_entries_fwd,
                            wave_hits_fwd=t.wave_hits_fwd,
                            wave_entries_bwd=t.wave_entries_bwd,
                            wave_hits_bwd=t.wave_hits_bwd)
    return out


def dv_validate_octree_host(level, ijk, corner_idx, max_level, n_corners,
                            sh_degree):
    """Host-only structural validation; returns (status, message)."""
    level = np.ascontiguousarray(level, np.uint8)
    ijk = np.ascontiguousarray(ijk, np.int32)
    corner_idx = np.ascontiguousarray(corner_idx, np.int32)
    n = level.shape[0]
    buf = C.create_string_buffer(512)
    st = _lib.dv_validate_octree_host(
        level.ctypes.data_as(C.c_void_p), ijk.ctypes.data_as(C.c_void_p),
        corner_idx.ctypes.data_as(C.c_void_p), n, max_level, n_corners,
        sh_degree, buf, 512)
    return st, buf.value.decode()


def dv_track_pose(track, t):
    """(active, R [3,3], p [3]) from a track dict, FP64 on the host."""
    tt = np.ascontiguousarray(track["t"], np.float64)
    yy = np.ascontiguousarray(track["yaw"], np.float64)
    pp = np.ascontiguousarray(track["trans"], np.float64)
    d = dv_track_desc(len(tt), tt.ctypes.data, yy.ctypes.data, pp.ctypes.data)
    R = (C.c_double * 9)()
    p = (C.c_double * 3)()
    act = _lib.dv_track_pose(C.byref(d), t, R, p)
    return bool(act), np.array(R[:]).reshape(3, 3), np.array(p[:])


class Scene:
    """Device-resident scene: torch tensors for every octree array (caller
    owned, referenced by the library) plus the built dv_scene handle."""

    def __init__(self, ctx, scene, device="cuda"):
        import torch
        self.ctx = ctx
        self.tensors = []
        self.octs = []
        descs = (dv_octree_desc * len(scene["octrees"]))()
        for k, o in enumerate(scene["octrees"]):
            t = dict(
                level=torch.from_numpy(np.ascontiguousarray(o["level"], np.uint8)).to(device),
                ijk=torch.from_numpy(np.ascontiguousarray(o["ijk"], np.int32)).to(device),
                corner_idx=torch.from_numpy(np.ascontiguousarray(o["corner_idx"], np.int32)).to(device),
                corner_density=torch.from_numpy(np.ascontiguousarray(o["corner_density"], np.float32)).to(device),
                sh=torch.from_numpy(np.ascontiguousarray(o["sh"], np.float32)).to(device))
            self.octs.append(t)
            d = descs[k]
            d.root_min[:] = [float(x) for x in o["root_min"]]
            d.root_size = float(o["root_size"])
            d.n_voxels = int(o["level"].shape[0])
            d.max_level = int(o["max_level"])
            d.n_corners = int(o["corner_density"].shape[0])
            d.sh_degree = int(o["sh_degree"])
            d.level = t["level"].data_ptr()
            d.ijk = t["ijk"].data_ptr()
            d.corner_idx = t["corner_idx"].data_ptr()
            d.corner_density = t["corner_density"].data_ptr()
            d.sh = t["sh"].data_ptr()
            if "box_min" in o:
                d.has_box = 1
                d.box_min[:] = [float(x) for x in o["box_min"]]
                d.box_max[:] = [float(x) for x in o["box_max"]]
        n_act = len(scene["octrees"]) - 1
        self.n_octrees = len(scene["octrees"])
        self.n_actors = n_act
        self._track_arrays = []
        tracks = (dv_track_desc * max(1, n_act))()
        for i in range(n_act):
            tr = scene["tracks"][i + 1]
            tt = np.ascontiguousarray(tr["t"], np.float64)
            yy = np.ascontiguousarray(tr["yaw"], np.float64)
            pp = np.ascontiguousarray(tr["trans"], np.float64)
            self._track_arrays += [tt, yy, pp]
            tracks[i] = dv_track_desc(len(tt), tt.ctypes.data, yy.ctypes.data,
                                      pp.ctypes.data)
        torch.cuda.synchronize()
        self.handle = dv_build_scene(ctx, descs, tracks if n_act else None)

    def close(self):
        if self.handle is not None:
            dv_scene_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def dv_build_scene(ctx, descs, tracks):
    h = C.c_void_p()
    _check(_lib.dv_build_scene(ctx, descs, len(descs), tracks, C.byref(h)),
           "dv_build_scene")
    return h


def dv_scene_destroy(h):
    _lib.dv_scene_destroy(h)


def alloc_outputs(views, mask=DV_OUT_RGB | DV_OUT_DEPTH | DV_OUT_T,
                  device="cuda"):
    import torch
    outs = []
    for v in views:
        h, w = v["h"], v["w"]
        outs.append(dict(
            rgb=torch.zeros(3, h, w, device=device) if mask & DV_OUT_RGB else None,
            depth=torch.zeros(h, w, device=device) if mask & DV_OUT_DEPTH else None,
            normal=torch.zeros(3, h, w, device=device) if mask & DV_OUT_NORMAL else None,
            T=torch.zeros(h, w, device=device) if mask & DV_OUT_T else None))
    return outs


class FwdState(C.c_void_p):
    """Forward-state handle of dv_render; remembers the shape [3, H, W] of
    the sky map its render used (None without a map), which a sky gradient
    buffer of dv_render_backward must match."""
    sky_shape = None


def dv_render(ctx, scene, views, opts, outs, pose_override=None, keep=False,
              stream=None):
    """Render ``views`` (list of view dicts) into ``outs`` (list of dicts of
    torch tensors).  Returns a forward-state handle if keep, else None."""
    nv = len(views)
    cviews = (dv_view * nv)(*[make_view(v) for v in views])
    couts = (dv_outputs * nv)()
    for i, o in enumerate(outs):
        couts[i] = dv_outputs(_ptr(o.get("rgb")), _ptr(o.get("depth")),
                              _ptr(o.get("normal")), _ptr(o.get("T")))
    po = None
    if pose_override is not None:
        pov = np.ascontiguousarray(pose_override, np.float64)
        po = pov.ctypes.data_as(C.c_void_p)
    st = FwdState()
    if opts.sky:
        st.sky_shape = (3, int(opts.sky_h), int(opts.sky_w))
    rc = _lib.dv_render(ctx, scene.handle, cviews, nv, po, C.byref(opts),
                        couts, C.byref(st) if keep else None,
                        _stream_handle(stream))
    _check(rc, "dv_render")
    return st if keep else None


def dv_render_noalloc(ctx, scene, views, opts, outs, pose_override=None,
                      stream=None):
    """dv_render without allocations: scratch from the library's static
    workspace (dv_noalloc_capacity() bytes); no forward state."""
    nv = len(views)
    cviews = (dv_view * nv)(*[make_view(v) for v in views])
    couts = (dv_outputs * nv)()
    for i, o in enumerate(outs):
        couts[i] = dv_outputs(_ptr(o.get("rgb")), _ptr(o.get("depth")),
                              _ptr(o.get("normal")), _ptr(o.get("T")))
    po = None
    if pose_override is not None:
        pov = np.ascontiguousarray(pose_override, np.float64)
        po = pov.ctypes.data_as(C.c_void_p)
    _check(_lib.dv_render_noalloc(ctx, scene.handle, cviews, nv, po, C.byref(opts),
                                  couts, _stream_handle(stream)),
           "dv_render_noalloc")


def feature_groups(F):
    return (int(F) + 2) // 3


def render_features(ctx, scene, views, opts, feats, out_feat, mask=DV_OUT_T,
                    keep=False, stream=None):
    """F-channel feature render (colour step replaced by per-leaf features):
    one dv_render per group of three channels, each into a scratch [3][h][w]
    plane whose valid channels are copied into ``out_feat`` (list per view
    of [F][h][w] tensors).  Returns the forward states per group if keep."""
    import torch
    F = int(feats[0].shape[0])
    states = []
    for g in range(feature_groups(F)):
        tmp = alloc_outputs(views, DV_OUT_RGB | mask)
        copts = make_opts(dict(opts, feat=feats, feat_group=g), DV_OUT_RGB | mask)
        st = dv_render(ctx, scene, views, copts, tmp, keep=keep, stream=stream)
        nc = min(3, F - 3 * g)
        for o, t in zip(out_feat, tmp):
            o[3 * g:3 * g + nc].copy_(t["rgb"][:nc])
        states.append((st, tmp))
    return states if keep else None


LOSS_TERMS = ("total", "color", "l1", "ssim", "depth", "normal", "sky", "_")


def dv_loss(ctx, views, weights, stream=None):
    """Training losses of several views.  views: list of dicts with the
    rendered planes (rgb, depth, normal, T), the targets (rgb_gt,
    depth_lidar, normal_pseudo, sky_mask) and the gradient planes to write
    (g_rgb, g_depth, g_normal, g_T); weights: dict color, ssim, depth,
    normal, sky.  Returns a CUDA float64 tensor [n_views, 8] of the terms
    (total, color, l1, ssim, depth, normal, sky, 0)."""
    import torch
    nv = len(views)
    cv = (dv_loss_view * nv)()
    for i, v in enumerate(views):
        ref = next(v[k] for k in ("rgb", "depth", "T", "rgb_gt") if v.get(k) is not None)
        h, w = int(ref.shape[-2]), int(ref.shape[-1])
        cv[i] = dv_loss_view(h, w, *[_ptr(v.get(k)) for k, _ in dv_loss_view._fields_[2:]])
    lw = dv_loss_weights(*[float(weights[k]) for k in ("color", "ssim", "depth",
                                                       "normal", "sky")])
    terms = torch.zeros(nv, 8, dtype=torch.float64, device="cuda")
    _check(_lib.dv_loss(ctx, cv, nv, C.byref(lw), _ptr(terms), _stream_handle(stream)),
           "dv_loss")
    return terms


def dv_adam(ctx, params, lr, step, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    """One Adam step over params: list of dicts p, g, m, v (float32 CUDA
    tensors of one size each), updated in place."""
    n = len(params)
    cp = (dv_adam_param * n)()
    for i, q in enumerate(params):
        cp[i] = dv_adam_param(_ptr(q["p"]), _ptr(q["g"]), _ptr(q["m"]), _ptr(q["v"]),
                              int(q["p"].numel()))
    o = dv_adam_opts(float(lr), float(beta1), float(beta2), float(eps), int(step))
    _check(_lib.dv_adam(ctx, cp, n, C.byref(o), _stream_handle(stream)), "dv_adam")


def dv_noalloc_capacity():
    return int(_lib.dv_noalloc_capacity())


def dv_render_backward(ctx, scene, state, grads, acc_octrees, pose_grad=None,
                       stream=None, sky_grad=None):
    """grads: list per view of dicts (rgb/depth/normal/T upstream gradient
    tensors or None); acc_octrees: list per octree of dicts with 'corner'
    and 'sh' accumulator tensors (or None).  sky_grad: float32 CUDA tensor
    of the forward's sky map shape (checked here: the kernels scatter into
    it by texel index), or None."""
    if sky_grad is not None:
        shape = getattr(state, "sky_shape", None)
        if shape is None:
            raise ValueError("sky_grad given but the forward state has no sky "
                             "map (or was not made by dv_render)")
        if not (hasattr(sky_grad, "is_cuda") and sky_grad.is_cuda
                and tuple(sky_grad.shape) == shape and sky_grad.is_contiguous()
                and str(sky_grad.dtype) == "torch.float32"):
            raise ValueError(f"sky_grad must be a contiguous float32 CUDA tensor "
                             f"of shape {shape}")
    nv = len(grads)
    cg = (dv_out_grads * nv)()
    for i, g in enumerate(grads):
        cg[i] = dv_out_grads(_ptr(g.get("rgb")), _ptr(g.get("depth")),
                             _ptr(g.get("normal")), _ptr(g.get("T")))
    no = len(acc_octrees)
    co = (dv_octree_grads * no)()
    for k, a in enumerate(acc_octrees):
        a = a or {}
        co[k] = dv_octree_grads(_ptr(a.get("corner")), _ptr(a.get("sh")),
                                _ptr(a.get("feat")))
    pg = dv_param_grads(co, _ptr(pose_grad), _ptr(sky_grad))
    _check(_lib.dv_render_backward(ctx, scene.handle, state, cg, C.byref(pg),
                                   _stream_handle(stream)),
           "dv_render_backward")


def dv_fwd_state_release(state):
    _lib.dv_fwd_state_release(state)


def dv_fwd_state_info(state):
    info = dv_state_info()
    _check(_lib.dv_fwd_state_info(state, C.byref(info)), "dv_fwd_state_info")
    return {f: getattr(info, f) for f, _ in dv_state_info._fields_}


def dv_fwd_state_export_lists(state, view, n_tiles, capacity, actor_capacity=0):
    ts = np.zeros(n_tiles + 1, np.int64)
    eo = np.zeros(max(capacity, 1), np.int32)
    el = np.zeros(max(capacity, 1), np.int32)
    ast = np.zeros(n_tiles + 1, np.int64)
    ao = np.zeros(max(actor_capacity, 1), np.int32)
    _check(_lib.dv_fwd_state_export_lists(
        state, view, ts.ctypes.data, eo.ctypes.data, el.ctypes.data, capacity,
        ast.ctypes.data, ao.ctypes.data, actor_capacity),
        "dv_fwd_state_export_lists")
    return ts, eo[:ts[-1]], el[:ts[-1]], ast, ao[:ast[-1]]


# ------------------------------------------------------------------ serving
def dv_serve_create(ctx, scene, opts, max_inflight=8, mem_budget=8 << 30,
                    batched=True, max_batch=8):
    """batched: True / 1 continuous batching, False / 0 one launch per
    request, 2 the persistent drain (refused by this build)."""
    mode = (1 if batched else 0) if isinstance(batched, bool) else int(batched)
    so = dv_serve_opts(max_inflight, mem_budget, mode, max_batch, opts)
    h = C.c_void_p()
    _check(_lib.dv_serve_create(ctx, scene.handle, C.byref(so), C.byref(h)),
           "dv_serve_create")
    return h


def dv_serve_submit(srv, view, out):
    req = dv_request(make_view(view),
                     dv_outputs(_ptr(out.get("rgb")), _ptr(out.get("depth")),
                                _ptr(out.get("normal")), _ptr(out.get("T"))))
    t = C.c_uint64()
    _check(_lib.dv_serve_submit(srv, C.byref(req), C.byref(t)),
           "dv_serve_submit")
    return t.value


def dv_serve_poll(srv, ticket, wait_us=0):
    """Returns (status, t_submit, t_admit, t_done)."""
    r = dv_result()
    st = _lib.dv_serve_poll(srv, ticket, wait_us, C.byref(r))
    return st, r.t_submit, r.t_admit, r.t_done


def dv_serve_destroy(srv):
    _check(_lib.dv_serve_destroy(srv), "dv_serve_destroy")


# ------------------------------------------------------------------ structure
DV_EDIT_SUBDIVIDE, DV_EDIT_PRUNE = 0, 1


def octree_tensors(o, device="cuda"):
    """Device tensors of one octree dict (level, ijk, corner_idx,
    corner_density, sh) and its dv_octree_desc (the tensors must outlive
    the desc's use)."""
    t = dict(
        level=torch.from_numpy(np.ascontiguousarray(o["level"], np.uint8)).to(device),
        ijk=torch.from_numpy(np.ascontiguousarray(o["ijk"], np.int32)).to(device),
        corner_idx=torch.from_numpy(np.ascontiguousarray(o["corner_idx"], np.int32)).to(device),
        corner_density=torch.from_numpy(
            np.ascontiguousarray(o["corner_density"], np.float32)).to(device))
    if o.get("sh") is not None:
        t["sh"] = torch.from_numpy(np.ascontiguousarray(o["sh"], np.float32)).to(device)
    return t, octree_desc(o, t)


def octree_desc(o, t):
    """dv_octree_desc of the device tensors t (level, ijk, corner_idx,
    corner_density, optional sh) with o's root, max_level and sh_degree."""
    d = dv_octree_desc()
    d.root_min[:] = [float(x) for x in o["root_min"]]
    d.root_size = float(o["root_size"])
    d.n_voxels = int(t["level"].shape[0])
    d.max_level = int(o["max_level"])
    d.n_corners = int(t["corner_density"].shape[0])
    d.sh_degree = int(o.get("sh_degree", 0)) if t.get("sh") is not None else 0
    d.level = t["level"].data_ptr()
    d.ijk = t["ijk"].data_ptr()
    d.corner_idx = t["corner_idx"].data_ptr()
    d.corner_density = t["corner_density"].data_ptr()
    d.sh = t["sh"].data_ptr() if t.get("sh") is not None else None
    return d


def _points(points):
    if not (points.is_cuda and points.dim() == 2 and points.shape[0] == 3
            and points.is_contiguous() and points.dtype == torch.float64):
        raise ValueError("points must be a contiguous float64 CUDA tensor [3][n]")
    return _ptr(points), int(points.shape[1])


def dv_nearest_distance(ctx, points, queries, r_max, stream=None):
    """Exact nearest-point distance of each query (float64 CUDA [3][m]);
    +inf where none is within r_max."""
    pp, n = _points(points)
    qp, m = _points(queries)
    dist = torch.empty(m, dtype=torch.float64, device="cuda")
    _check(_lib.dv_nearest_distance(ctx, pp, n, qp, m, float(r_max), _ptr(dist),
                                    _stream_handle(stream)), "dv_nearest_distance")
    return dist


def dv_corner_prior(ctx, desc, points, s, v_close=-2.0, v_far=-10.0, r_cut=None,
                    stream=None):
    """Eq. 1 for every corner of the octree desc: float32 CUDA [n_corners]."""
    pp, n = _points(points)
    out = torch.empty(max(desc.n_corners, 0), dtype=torch.float32, device="cuda")
    r = 3.0 * s if r_cut is None else r_cut
    _check(_lib.dv_corner_prior(ctx, C.byref(desc), pp, n, float(s), float(v_close),
                                float(v_far), float(r), _ptr(out),
                                _stream_handle(stream)), "dv_corner_prior")
    return out


def dv_proximity_flags(ctx, desc, points, ratio, stream=None):
    pp, n = _points(points)
    flags = torch.empty(max(desc.n_voxels, 0), dtype=torch.uint8, device="cuda")
    _check(_lib.dv_proximity_flags(ctx, C.byref(desc), pp, n, float(ratio),
                                   _ptr(flags), _stream_handle(stream)),
           "dv_proximity_flags")
    return flags


def _apply(edit, n, nc, sh_rows, stream):
    out = dict(level=torch.empty(n, dtype=torch.uint8, device="cuda"),
               ijk=torch.empty(3, n, dtype=torch.int32, device="cuda"),
               corner_idx=torch.empty(8, n, dtype=torch.int32, device="cuda"),
               corner_density=torch.empty(nc, dtype=torch.float32, device="cuda"),
               leaf_src=torch.empty(n, dtype=torch.int32, device="cuda"),
               corner_src=torch.empty(nc, dtype=torch.int32, device="cuda"))
    if sh_rows:
        out["sh"] = torch.empty(sh_rows // 3, 3, n, dtype=torch.float32, device="cuda")
    eo = dv_edit_out(*[_ptr(out.get(k)) for k, _ in dv_edit_out._fields_])
    _check(_lib.dv_edit_apply(edit, C.byref(eo), _stream_handle(stream)),
           "dv_edit_apply")
    return out


def _sh_rows(desc):
    return 3 * (desc.sh_degree + 1) ** 2 if desc.sh else 0


def dv_edit(ctx, desc, flags, op, stream=None):
    """Subdivide (op 0) or prune (op 1) by flags (uint8 CUDA [N]): dict of
    the new tables (level, ijk, corner_idx, corner_density, leaf_src,
    corner_src, and sh when the desc has SH)."""
    h = C.c_void_p()
    n, nc = C.c_int64(), C.c_int64()
    _check(_lib.dv_edit_plan(ctx, C.byref(desc), _ptr(flags), int(op), C.byref(h),
                             C.byref(n), C.byref(nc), _stream_handle(stream)),
           "dv_edit_plan")
    try:
        return _apply(h, n.value, nc.value, _sh_rows(desc), stream)
    finally:
        torch.cuda.current_stream().synchronize()
        _lib.dv_edit_release(h)


def dv_refine(ctx, desc, points, ratio, min_size, max_rounds=32, stream=None):
    """Proximity subdivision rounds: (tables dict as dv_edit's, rounds)."""
    pp, np_ = _points(points)
    h = C.c_void_p()
    n, nc, r = C.c_int64(), C.c_int64(), C.c_int32()
    _check(_lib.dv_refine_plan(ctx, C.byref(desc), pp, np_, float(ratio),
                               float(min_size), int(max_rounds), C.byref(h),
                               C.byref(n), C.byref(nc), C.byref(r),
                               _stream_handle(stream)), "dv_refine_plan")
    try:
        return _apply(h, n.value, nc.value, _sh_rows(desc), stream), r.value
    finally:
        torch.cuda.current_stream().synchronize()
        _lib.dv_edit_release(h)
