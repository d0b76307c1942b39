"""Python binding of libdare, the MI355X directionality-aware reslicing library.

Thin ctypes marshalling over the C ABI in include/dare.h: every step of the
reconstruction and reslice runs in the library's HIP kernels.  torch supplies
device memory (arenas, frames, outputs) and streams.  There is no fallback:
importing this package without the built library raises.

The functions named like the C entry points (``dare_reconstruct_frames``,
``dare_reslice``, ``dare_reslice_batch``, ...) take the same arguments with
Python/torch types; ``Volume`` bundles a volume handle with its arena.
"""
from __future__ import annotations

import ctypes as ct
import os
import warnings

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdare.so")

F32, BF16, F16, FP8 = 0, 1, 2, 3
DTYPES = {"f32": F32, "fp32": F32, "bf16": BF16, "f16": F16, "fp16": F16, "fp8": FP8, "fp8_e4m3": FP8}
DTYPE_NAMES = {F32: "fp32", BF16: "bf16", F16: "fp16", FP8: "fp8"}

OK, ERR_INVALID_ARG, ERR_BAD_POSE, ERR_BUDGET, ERR_HIP, WARN_BINS_SATURATED, ERR_NOT_READY, ERR_QUEUE_FULL = range(8)


class Geometry(ct.Structure):
    _fields_ = [("origin_mm", ct.c_double * 3), ("spacing_mm", ct.c_double), ("dims", ct.c_int32 * 3),
                ("calib", ct.c_double * 16)]


class Params(ct.Structure):
    _fields_ = [("k_normal", ct.c_double), ("k_inplane", ct.c_double), ("thr_normal_deg", ct.c_double),
                ("thr_inplane_deg", ct.c_double), ("radius_vox", ct.c_double), ("bin_tol_deg", ct.c_double),
                ("max_bins", ct.c_int32), ("normal_axis", ct.c_int32)]


class SliceSpec(ct.Structure):
    _fields_ = [("probe_pose", ct.c_double * 16), ("width", ct.c_int32), ("height", ct.c_int32),
                ("pitch_mm", ct.c_double * 2)]


class VolumeInfo(ct.Structure):
    _fields_ = [("bins", ct.c_int32), ("saturated", ct.c_int32), ("bricks_used", ct.c_int64),
                ("bricks_capacity", ct.c_int64), ("bytes_per_brick", ct.c_int64), ("brick_grid", ct.c_int64 * 3)]


class Fan(ct.Structure):
    _fields_ = [("apex_mm", ct.c_double * 2), ("r0_mm", ct.c_double), ("dr_mm", ct.c_double),
                ("sectors", ct.c_int32)]


class ServerConfig(ct.Structure):
    _fields_ = [("max_tick_pixels", ct.c_int64), ("max_tick_requests", ct.c_int32), ("n_streams", ct.c_int32),
                ("max_queue", ct.c_int32), ("use_graphs", ct.c_int32), ("volume_budget_bytes", ct.c_uint64)]


class ServerStats(ct.Structure):
    _fields_ = [("submitted", ct.c_int64), ("completed", ct.c_int64), ("rejected", ct.c_int64),
                ("ticks", ct.c_int64), ("pixels", ct.c_int64), ("busy_seconds", ct.c_double),
                ("frames", ct.c_int64), ("compound_seconds", ct.c_double), ("kernel_seconds", ct.c_double),
                ("device_busy_seconds", ct.c_double), ("untimed_ticks", ct.c_int64)]


class RequestTimes(ct.Structure):
    _fields_ = [("t_submit", ct.c_double), ("t_admit", ct.c_double), ("t_launch", ct.c_double),
                ("t_device_done", ct.c_double), ("t_host_done", ct.c_double)]


# numpy views of the same layouts, for the grouped server calls
SPEC_DTYPE = np.dtype([("probe_pose", "<f8", (16,)), ("width", "<i4"), ("height", "<i4"), ("pitch_mm", "<f8", (2,))],
                      align=True)
TIMES_DTYPE = np.dtype([(n, "<f8") for n, _ in RequestTimes._fields_])
assert SPEC_DTYPE.itemsize == ct.sizeof(SliceSpec) and TIMES_DTYPE.itemsize == ct.sizeof(RequestTimes)


def spec_array(poses, widths, heights, pitches) -> np.ndarray:
    """SPEC_DTYPE array of n slice specs (poses (n, 4, 4), pitches (n, 2))."""
    poses = np.asarray(poses, np.float64).reshape(-1, 16)
    a = np.zeros(len(poses), SPEC_DTYPE)
    a["probe_pose"] = poses
    a["width"] = widths
    a["height"] = heights
    a["pitch_mm"] = np.asarray(pitches, np.float64).reshape(-1, 2)
    return a


class DareError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {status_str(status)} (status {status})")


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_2605_26325_amd/build.py`")
    lib = ct.CDLL(LIB_PATH)
    P, V, I32, I64, U64, D = ct.c_void_p, ct.c_void_p, ct.c_int32, ct.c_int64, ct.c_uint64, ct.c_double
    sig = {
        "dare_default_params": (None, [ct.POINTER(Params)]),
        "dare_status_str": (ct.c_char_p, [ct.c_int]),
        "dare_volume_arena_bytes": (U64, [ct.POINTER(Geometry), ct.POINTER(Params), ct.c_int, I64]),
        "dare_volume_create": (ct.c_int, [ct.POINTER(Geometry), ct.POINTER(Params), ct.c_int, P, U64,
                                          ct.POINTER(V)]),
        "dare_volume_destroy": (ct.c_int, [V]),
        "dare_reconstruct_frames": (ct.c_int, [V, P, I32, I32, I32, ct.POINTER(D), P, P]),
        "dare_reconstruct_fan": (ct.c_int, [V, P, I32, I32, I32, ct.POINTER(Fan), P, P, P]),
        "dare_reslice": (ct.c_int, [V, ct.POINTER(SliceSpec), P, P]),
        "dare_reslice_batch_workspace_bytes": (U64, [ct.POINTER(V), ct.POINTER(SliceSpec), I32]),
        "dare_reslice_batch": (ct.c_int, [ct.POINTER(V), ct.POINTER(SliceSpec), ct.POINTER(P), I32, P, U64, P]),
        "dare_reslice_batch_noalloc": (ct.c_int, [ct.POINTER(V), ct.POINTER(SliceSpec), ct.POINTER(P), I32, P]),
        "dare_bounds_from_frames": (ct.c_int, [P, I32, I32, I32, ct.POINTER(D), ct.POINTER(D), D,
                                               ct.POINTER(Geometry)]),
        "dare_volume_get_info": (ct.c_int, [V, ct.POINTER(VolumeInfo)]),
        "dare_volume_get_codebook": (ct.c_int, [V, ct.POINTER(D), ct.POINTER(D), ct.POINTER(I32)]),
        "dare_volume_download_sums": (ct.c_int, [V, P, P, I32, P]),
        "dare_volume_download_storage": (ct.c_int, [V, P, P, I32, P]),
        "dare_volume_upload_sums": (ct.c_int, [V, ct.POINTER(D), ct.POINTER(D), I32, P, P, P]),
        "dare_copy_probe": (ct.c_int, [P, P, U64, P]),
        "dare_slice_active_bins": (ct.c_int, [V, ct.POINTER(SliceSpec), ct.POINTER(I32), ct.POINTER(D),
                                              ct.POINTER(I32)]),
        "dare_now_seconds": (D, []),
        "dare_default_server_config": (None, [ct.POINTER(ServerConfig)]),
        "dare_server_create": (ct.c_int, [ct.POINTER(ServerConfig), P, U64, ct.POINTER(V)]),
        "dare_server_add_volume": (ct.c_int, [V, V, ct.POINTER(I32)]),
        "dare_server_remove_volume": (ct.c_int, [V, I32, D]),
        "dare_server_volume_bytes": (ct.c_int, [V, ct.POINTER(U64), ct.POINTER(I32)]),
        "dare_server_submit": (ct.c_int, [V, I32, ct.POINTER(SliceSpec), P, ct.POINTER(U64)]),
        "dare_server_poll": (ct.c_int, [V, U64, ct.POINTER(RequestTimes)]),
        "dare_server_submit_many": (ct.c_int, [V, I32, P, P, P, P, ct.POINTER(I32)]),
        "dare_server_submit_frames": (ct.c_int, [V, I32, P, I32, I32, I32, ct.POINTER(D), P, ct.POINTER(U64)]),
        "dare_server_poll_many": (ct.c_int, [V, I32, P, P, P, D, ct.POINTER(I32)]),
        "dare_server_drain": (ct.c_int, [V]),
        "dare_server_get_stats": (ct.c_int, [V, ct.POINTER(ServerStats)]),
        "dare_server_destroy": (ct.c_int, [V]),
        "dare_samples_arena_bytes": (U64, [ct.POINTER(Geometry), I64, I32]),
        "dare_samples_create": (ct.c_int, [ct.POINTER(Geometry), I64, I32, P, U64, ct.POINTER(V)]),
        "dare_samples_destroy": (ct.c_int, [V]),
        "dare_samples_build": (ct.c_int, [V, P, I32, I32, I32, ct.POINTER(D), P, I32, P]),
        "dare_samples_count": (ct.c_int, [V, ct.POINTER(I64), ct.POINTER(I32)]),
        "dare_samples_reslice": (ct.c_int, [V, ct.POINTER(Params), ct.POINTER(SliceSpec), I32, P, P]),
        "dare_compare_workspace_bytes": (U64, []),
        "dare_volume_save_bytes": (U64, [V]),
        "dare_volume_save": (ct.c_int, [V, P, U64]),
        "dare_volume_load": (ct.c_int, [P, U64, P, U64, ct.POINTER(V)]),
        "dare_volume_evict_outside": (ct.c_int, [V, ct.POINTER(I32), ct.POINTER(I32), P]),
        "dare_volume_restore_box": (ct.c_int, [V, ct.POINTER(I32), ct.POINTER(I32), P]),
        "dare_volume_set_spill": (ct.c_int, [V, I32]),
        "dare_volume_held": (ct.c_int, [V, ct.POINTER(I64), ct.POINTER(U64)]),
        "dare_compare_to_frame": (ct.c_int, [P, P, I32, I32, P, U64, ct.POINTER(D), P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def status_str(s: int) -> str:
    return lib.dare_status_str(int(s)).decode()


def _check(status: int, where: str, allow_warn: bool = True) -> int:
    if status == OK:
        return status
    if status == WARN_BINS_SATURATED and allow_warn:
        warnings.warn(f"{where}: {status_str(status)}", RuntimeWarning, stacklevel=3)
        return status
    raise DareError(status, where)


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ct.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _ptr(t) -> ct.c_void_p:
    return ct.c_void_p(t.data_ptr())


def _torch():
    import torch
    return torch


def default_params(**over) -> Params:
    p = Params()
    lib.dare_default_params(ct.byref(p))
    for k, v in over.items():
        setattr(p, k, v)
    return p


def make_geometry(origin, spacing, dims, calib) -> Geometry:
    g = Geometry()
    g.origin_mm[:] = [float(v) for v in origin]
    g.spacing_mm = float(spacing)
    g.dims[:] = [int(v) for v in dims]
    g.calib[:] = [float(v) for v in np.asarray(calib, np.float64).reshape(16)]
    return g


def make_spec(probe_pose, width, height, pitch) -> SliceSpec:
    s = SliceSpec()
    s.probe_pose[:] = [float(v) for v in np.asarray(probe_pose, np.float64).reshape(16)]
    s.width, s.height = int(width), int(height)
    s.pitch_mm[:] = [float(pitch[0]), float(pitch[1])]
    return s


def dare_volume_arena_bytes(geometry: Geometry, params: Params, dtype: int, bricks: int) -> int:
    return int(lib.dare_volume_arena_bytes(ct.byref(geometry), ct.byref(params), int(dtype), int(bricks)))


def dare_bounds_from_frames(probe_poses, width, height, pitch, calib, spacing) -> Geometry:
    P = np.ascontiguousarray(np.asarray(probe_poses, np.float32).reshape(-1, 16))
    g = Geometry()
    pitch_arr = (ct.c_double * 2)(float(pitch[0]), float(pitch[1]))
    cal = (ct.c_double * 16)(*[float(v) for v in np.asarray(calib, np.float64).reshape(16)])
    _check(lib.dare_bounds_from_frames(P.ctypes.data_as(ct.c_void_p), len(P), int(width), int(height), pitch_arr,
                                       cal, float(spacing), ct.byref(g)), "dare_bounds_from_frames")
    return g


def dare_reconstruct_frames(vol: "Volume", frames, width, height, pitch, probe_poses, stream=None) -> int:
    n = int(frames.shape[0]) if frames.dim() == 3 else int(frames.shape[0])
    pitch_arr = (ct.c_double * 2)(float(pitch[0]), float(pitch[1]))
    return _check(lib.dare_reconstruct_frames(vol.handle, _ptr(frames), n, int(width), int(height), pitch_arr,
                                              _ptr(probe_poses), _stream(stream)), "dare_reconstruct_frames")


def dare_reslice(vol: "Volume", spec: SliceSpec, out, stream=None) -> int:
    return _check(lib.dare_reslice(vol.handle, ct.byref(spec), _ptr(out), _stream(stream)), "dare_reslice")


def dare_reslice_batch_workspace_bytes(vols, specs) -> int:
    n = len(vols)
    hv = (ct.c_void_p * n)(*[v.handle for v in vols])
    hs = (SliceSpec * n)(*specs)
    return int(lib.dare_reslice_batch_workspace_bytes(hv, hs, n))


NOALLOC_WORKSPACE_BYTES = 32 << 20     # DARE_NOALLOC_WORKSPACE_BYTES


def dare_reslice_batch_noalloc(vols, specs, outs, stream=None) -> int:
    """dare_reslice_batch with the library's own per-device workspace (allocates nothing)."""
    n = len(vols)
    hv = (ct.c_void_p * n)(*[v.handle for v in vols])
    hs = (SliceSpec * n)(*specs)
    ho = (ct.c_void_p * n)(*[o.data_ptr() for o in outs])
    return _check(lib.dare_reslice_batch_noalloc(hv, hs, ho, n, _stream(stream)), "dare_reslice_batch_noalloc")


def dare_reslice_batch(vols, specs, outs, workspace, stream=None) -> int:
    n = len(vols)
    hv = (ct.c_void_p * n)(*[v.handle for v in vols])
    hs = (SliceSpec * n)(*specs)
    ho = (ct.c_void_p * n)(*[o.data_ptr() for o in outs])
    return _check(lib.dare_reslice_batch(hv, hs, ho, n, _ptr(workspace), int(workspace.numel()),
                                         _stream(stream)), "dare_reslice_batch")


def dare_copy_probe(src, dst, nbytes, stream=None) -> int:
    return _check(lib.dare_copy_probe(_ptr(src), _ptr(dst), int(nbytes), _stream(stream)), "dare_copy_probe")


class Volume:
    """A volume handle plus the torch-owned device arena it lives in."""

    def __init__(self, geometry: Geometry, params: Params | None = None, dtype="f32", bricks: int | None = None,
                 arena_bytes: int | None = None, device="cuda"):
        import torch
        self.geometry = geometry
        self.params = params if params is not None else default_params()
        self.dtype = DTYPES[dtype] if isinstance(dtype, str) else int(dtype)
        if arena_bytes is None:
            if bricks is None:
                # every (bin, brick) when that fits in 2 GiB, else room for 8 bins' worth
                nb = 1
                for d in geometry.dims:
                    nb *= (int(d) + 7) // 8
                bricks = nb * int(self.params.max_bins)
                if dare_volume_arena_bytes(geometry, self.params, self.dtype, bricks) > (2 << 30):
                    bricks = nb * 8
            arena_bytes = dare_volume_arena_bytes(geometry, self.params, self.dtype, bricks)
            if arena_bytes == 0:
                raise DareError(ERR_INVALID_ARG, "dare_volume_arena_bytes")
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=device)
        h = ct.c_void_p()
        _check(lib.dare_volume_create(ct.byref(geometry), ct.byref(self.params), self.dtype, _ptr(self.arena),
                                      int(arena_bytes), ct.byref(h)), "dare_volume_create")
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            lib.dare_volume_destroy(self.handle)
            self.handle = None

    def save(self) -> np.ndarray:
        """The volume's whole state as a host byte array (dare_volume_save)."""
        n = int(lib.dare_volume_save_bytes(self.handle))
        if n == 0:
            raise DareError(ERR_INVALID_ARG, "dare_volume_save_bytes")
        buf = np.empty(n, np.uint8)
        _check(lib.dare_volume_save(self.handle, buf.ctypes.data_as(ct.c_void_p), n), "dare_volume_save")
        return buf

    @classmethod
    def load(cls, buf, arena_bytes: int, device="cuda") -> "Volume":
        """A new volume holding a saved state, in a fresh arena of ``arena_bytes``."""
        import torch
        buf = np.ascontiguousarray(buf, np.uint8)
        self = cls.__new__(cls)
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=device)
        h = ct.c_void_p()
        _check(lib.dare_volume_load(buf.ctypes.data_as(ct.c_void_p), buf.nbytes, _ptr(self.arena), int(arena_bytes),
                                    ct.byref(h)), "dare_volume_load")
        self.handle = h
        hdr = Geometry()
        ct.memmove(ct.byref(hdr), buf.ctypes.data + 16, ct.sizeof(Geometry))
        self.geometry = hdr
        prm = Params()
        ct.memmove(ct.byref(prm), buf.ctypes.data + 16 + ct.sizeof(Geometry), ct.sizeof(Params))
        self.params = prm
        self.dtype = int(np.frombuffer(buf[16 + ct.sizeof(Geometry) + ct.sizeof(Params):][:4].tobytes(), np.int32)[0])
        return self

    def evict_outside(self, lo, hi, stream=None):
        """Move every resident brick that does not meet the voxel box lo..hi (inclusive) to host
        memory (dare_volume_evict_outside)."""
        a, b = (ct.c_int32 * 3)(*[int(x) for x in lo]), (ct.c_int32 * 3)(*[int(x) for x in hi])
        _check(lib.dare_volume_evict_outside(self.handle, a, b, _stream(stream)), "dare_volume_evict_outside")

    def restore_box(self, lo, hi, stream=None):
        """Bring back every held brick that meets the voxel box lo..hi (dare_volume_restore_box)."""
        a, b = (ct.c_int32 * 3)(*[int(x) for x in lo]), (ct.c_int32 * 3)(*[int(x) for x in hi])
        _check(lib.dare_volume_restore_box(self.handle, a, b, _stream(stream)), "dare_volume_restore_box")

    def set_spill(self, enabled: bool):
        """Hold least recently touched bricks in host memory instead of failing a batch for room."""
        _check(lib.dare_volume_set_spill(self.handle, 1 if enabled else 0), "dare_volume_set_spill")

    def held(self):
        """(bricks held in host memory, their host bytes)."""
        n, b = ct.c_int64(), ct.c_uint64()
        _check(lib.dare_volume_held(self.handle, ct.byref(n), ct.byref(b)), "dare_volume_held")
        return n.value, b.value

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def dims(self):
        return tuple(int(d) for d in self.geometry.dims)

    def reconstruct(self, frames, probe_poses, pitch, stream=None) -> int:
        F, H, W = frames.shape
        return dare_reconstruct_frames(self, frames, W, H, pitch, probe_poses, stream)

    def reconstruct_fan(self, frames, probe_poses, apex, r0, dr, sectors, beams, stream=None) -> int:
        """Fan frames (F, H, W) uint8; beams: (W, 2) float64 device tensor of unit beam
        directions (dare_reconstruct_fan)."""
        F, H, W = frames.shape
        fan = Fan((ct.c_double * 2)(float(apex[0]), float(apex[1])), float(r0), float(dr), int(sectors))
        return _check(lib.dare_reconstruct_fan(self.handle, _ptr(frames), int(F), int(W), int(H), ct.byref(fan),
                                               _ptr(beams), _ptr(probe_poses), _stream(stream)),
                      "dare_reconstruct_fan")

    def reslice(self, probe_pose, width, height, pitch, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty((height, width), dtype=torch.float32, device=self.arena.device)
        dare_reslice(self, make_spec(probe_pose, width, height, pitch), out, stream)
        return out

    def active_bins(self, probe_pose, width, height, pitch):
        """(bins, weights) that pass both angular thresholds for this slice."""
        b = (ct.c_int32 * 64)()
        w = (ct.c_double * 64)()
        n = ct.c_int32()
        _check(lib.dare_slice_active_bins(self.handle, ct.byref(make_spec(probe_pose, width, height, pitch)), b, w,
                                          ct.byref(n)), "dare_slice_active_bins")
        return list(b[:n.value]), list(w[:n.value])

    def info(self) -> VolumeInfo:
        inf = VolumeInfo()
        _check(lib.dare_volume_get_info(self.handle, ct.byref(inf)), "dare_volume_get_info")
        return inf

    def codebook(self):
        rn = (ct.c_double * (64 * 3))()
        rx = (ct.c_double * (64 * 3))()
        k = ct.c_int32()
        _check(lib.dare_volume_get_codebook(self.handle, rn, rx, ct.byref(k)), "dare_volume_get_codebook")
        K = k.value
        return (np.array(rn[:K * 3]).reshape(K, 3), np.array(rx[:K * 3]).reshape(K, 3))

    def _dense(self, dtype):
        import torch
        K = self.info().bins
        nx, ny, nz = self.dims
        shape = (K, nz, ny, nx)
        return K, torch.zeros(shape, dtype=dtype, device=self.arena.device), \
            torch.zeros(shape, dtype=dtype, device=self.arena.device)

    def download_sums(self, stream=None):
        import torch
        K, S, C = self._dense(torch.int32)
        if K:
            _check(lib.dare_volume_download_sums(self.handle, _ptr(S), _ptr(C), K, _stream(stream)),
                   "dare_volume_download_sums")
        return S, C

    def download_storage(self, stream=None):
        import torch
        K, A, C = self._dense(torch.float32)
        if K:
            _check(lib.dare_volume_download_storage(self.handle, _ptr(A), _ptr(C), K, _stream(stream)),
                   "dare_volume_download_storage")
        return A, C

    def upload_sums(self, rep_n, rep_x, S, C, stream=None):
        """S, C: int32/uint32 (K, nz, ny, nx) device tensors; rep_n, rep_x: (K, 3) arrays."""
        K = int(S.shape[0])
        rn = (ct.c_double * max(1, 3 * K))(*np.asarray(rep_n, np.float64).reshape(-1).tolist())
        rx = (ct.c_double * max(1, 3 * K))(*np.asarray(rep_x, np.float64).reshape(-1).tolist())
        return _check(lib.dare_volume_upload_sums(self.handle, rn, rx, K, _ptr(S.contiguous()),
                                                  _ptr(C.contiguous()), _stream(stream)), "dare_volume_upload_sums")


def compare_to_frame(image, frame, workspace=None, stream=None):
    """(NCC, mean SSIM, pixels used, windows used) of a float32 reslice against a uint8 frame of
    the same shape, both device tensors (Sec. 3's evaluation measures)."""
    import torch
    H, W = image.shape
    if workspace is None:
        workspace = torch.empty(int(lib.dare_compare_workspace_bytes()), dtype=torch.uint8, device=image.device)
    out = (ct.c_double * 4)()
    _check(lib.dare_compare_to_frame(_ptr(image.contiguous()), _ptr(frame.contiguous()), int(W), int(H),
                                     _ptr(workspace), int(workspace.numel()), out, _stream(stream)),
           "dare_compare_to_frame", allow_warn=False)
    return out[0], out[1], int(out[2]), int(out[3])


LITERAL_MODES = {"box": 0, "tent": 1}


class SampleStore:
    """Per-sample store (every in-grid frame pixel kept with its own frame's orientation) in a
    torch-owned device arena; reslices it in the box or tent reading."""

    def __init__(self, geometry: Geometry, max_samples: int, max_frames: int, device="cuda"):
        import torch
        self.geometry = geometry
        nbytes = lib.dare_samples_arena_bytes(ct.byref(geometry), int(max_samples), int(max_frames))
        if nbytes == 0:
            raise DareError(ERR_INVALID_ARG, "dare_samples_arena_bytes")
        self.arena = torch.empty(int(nbytes), dtype=torch.uint8, device=device)
        h = ct.c_void_p()
        _check(lib.dare_samples_create(ct.byref(geometry), int(max_samples), int(max_frames), _ptr(self.arena),
                                       int(nbytes), ct.byref(h)), "dare_samples_create")
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            lib.dare_samples_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def build(self, frames, probe_poses, pitch, normal_axis=2, stream=None) -> int:
        """frames: (F, H, W) uint8 device tensor; probe_poses: (F, 4, 4) float32 device tensor."""
        F, H, W = frames.shape
        p = (ct.c_double * 2)(float(pitch[0]), float(pitch[1]))
        _check(lib.dare_samples_build(self.handle, _ptr(frames.contiguous()), int(F), int(W), int(H), p,
                                      _ptr(probe_poses.contiguous()), int(normal_axis), _stream(stream)),
               "dare_samples_build", allow_warn=False)
        return self.count()[0]

    def count(self):
        n = ct.c_int64()
        f = ct.c_int32()
        _check(lib.dare_samples_count(self.handle, ct.byref(n), ct.byref(f)), "dare_samples_count")
        return n.value, f.value

    def reslice(self, probe_pose, width, height, pitch, params: Params | None = None, mode="box", out=None,
                stream=None):
        import torch
        if out is None:
            out = torch.empty((height, width), dtype=torch.float32, device=self.arena.device)
        prm = params if params is not None else default_params()
        _check(lib.dare_samples_reslice(self.handle, ct.byref(prm), ct.byref(make_spec(probe_pose, width, height,
                                                                                         pitch)),
                                        LITERAL_MODES[mode] if isinstance(mode, str) else int(mode), _ptr(out),
                                        _stream(stream)), "dare_samples_reslice", allow_warn=False)
        return out


def default_server_config(**over) -> ServerConfig:
    c = ServerConfig()
    lib.dare_default_server_config(ct.byref(c))
    for k, v in over.items():
        setattr(c, k, v)
    return c


class Server:
    """Continuous-batching reslice server (C++ scheduler thread inside the library).

    ``arena_bytes`` of device memory hold one workspace per stream and the
    result slots; requests wait in FIFO order until a slot of their size fits.
    Volumes are admitted against ``volume_budget_bytes`` (0: no limit)."""

    def __init__(self, arena_bytes: int, device="cuda", **cfg):
        import torch
        self.config = default_server_config(**cfg)
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=device)
        h = ct.c_void_p()
        _check(lib.dare_server_create(ct.byref(self.config), _ptr(self.arena), int(arena_bytes), ct.byref(h)),
               "dare_server_create")
        self.handle = h
        self._volumes = []

    def add_volume(self, vol: "Volume") -> int:
        vid = ct.c_int32()
        _check(lib.dare_server_add_volume(self.handle, vol.handle, ct.byref(vid)), "dare_server_add_volume")
        self._volumes.append(vol)
        return vid.value

    def remove_volume(self, volume_id: int, wait_seconds: float = 60.0):
        """Unregister a volume once its queued requests have completed (dare_server_remove_volume)."""
        _check(lib.dare_server_remove_volume(self.handle, int(volume_id), float(wait_seconds)),
               "dare_server_remove_volume")

    def volume_bytes(self):
        """(resident volume bytes, resident volumes)."""
        b, n = ct.c_uint64(), ct.c_int32()
        _check(lib.dare_server_volume_bytes(self.handle, ct.byref(b), ct.byref(n)), "dare_server_volume_bytes")
        return int(b.value), int(n.value)

    def submit(self, volume_id: int, probe_pose, width, height, pitch, host_out):
        """Queue a request; returns its ticket, or None when the queue is full."""
        t = ct.c_uint64()
        st = lib.dare_server_submit(self.handle, int(volume_id), ct.byref(make_spec(probe_pose, width, height, pitch)),
                                    _ptr(host_out), ct.byref(t))
        if st == ERR_QUEUE_FULL:
            return None
        _check(st, "dare_server_submit")
        return t.value

    def submit_frames(self, volume_id: int, frames, probe_poses, pitch):
        """Queue frames (uint8 (n, h, w), device) with their probe poses (float32 (n, 4, 4),
        device) for compounding in request order; returns the ticket, or None when the queue is
        full.  Both tensors must stay alive until the ticket completes (poll returns the
        compounding status)."""
        if frames.dtype != _torch().uint8 or not frames.is_cuda or not frames.is_contiguous():
            raise ValueError("frames: contiguous uint8 device tensor (n, h, w)")
        if probe_poses.dtype != _torch().float32 or not probe_poses.is_cuda or not probe_poses.is_contiguous():
            raise ValueError("probe_poses: contiguous float32 device tensor (n, 4, 4)")
        n, h, w = (int(x) for x in frames.shape)
        if tuple(probe_poses.shape) != (n, 4, 4):
            raise ValueError("probe_poses: one 4x4 pose per frame")
        t = ct.c_uint64()
        pit = (ct.c_double * 2)(float(pitch[0]), float(pitch[1]))
        st = lib.dare_server_submit_frames(self.handle, int(volume_id), _ptr(frames), n, w, h, pit,
                                           _ptr(probe_poses), ct.byref(t))
        if st == ERR_QUEUE_FULL:
            return None
        _check(st, "dare_server_submit_frames")
        return t.value

    def poll_frames(self, ticket: int):
        """(status, RequestTimes) once the frames are compounded, else None."""
        tm = RequestTimes()
        st = lib.dare_server_poll(self.handle, ct.c_uint64(ticket), ct.byref(tm))
        if st == ERR_NOT_READY:
            return None
        if st == ERR_INVALID_ARG:
            _check(st, "dare_server_poll")
        return st, tm

    def submit_many(self, volume_ids, specs: np.ndarray, host_out_ptrs):
        """Queue requests in order: volume_ids (n,), specs a SPEC_DTYPE array (n,), host_out_ptrs
        (n,) addresses.  Returns (tickets of the accepted prefix, status of the first refused one
        or OK); QUEUE_FULL is a status, other refusals raise."""
        n = len(specs)
        vid = np.ascontiguousarray(volume_ids, np.int32)
        sp = np.ascontiguousarray(specs, SPEC_DTYPE)
        outs = np.ascontiguousarray(host_out_ptrs, np.uint64)
        if len(vid) != n or len(outs) != n:
            raise ValueError("submit_many: arrays of different lengths")
        tickets = np.zeros(n, np.uint64)
        acc = ct.c_int32()
        st = lib.dare_server_submit_many(self.handle, n, vid.ctypes.data, sp.ctypes.data, outs.ctypes.data,
                                         tickets.ctypes.data, ct.byref(acc))
        if st not in (OK, ERR_QUEUE_FULL):
            _check(st, "dare_server_submit_many")
        return tickets[:acc.value], st

    def poll_many(self, tickets, wait_seconds: float = 0.0):
        """(states (n,) int32, times (n,) TIMES_DTYPE) for the tickets; finished ones are retired."""
        tk = np.ascontiguousarray(tickets, np.uint64)
        n = len(tk)
        states = np.zeros(n, np.int32)
        times = np.zeros(n, TIMES_DTYPE)
        nd = ct.c_int32()
        _check(lib.dare_server_poll_many(self.handle, n, tk.ctypes.data, times.ctypes.data, states.ctypes.data,
                                         float(wait_seconds), ct.byref(nd)), "dare_server_poll_many")
        return states, times

    def poll(self, ticket: int):
        """RequestTimes once the result is in host memory, else None."""
        tm = RequestTimes()
        st = lib.dare_server_poll(self.handle, ct.c_uint64(ticket), ct.byref(tm))
        if st == ERR_NOT_READY:
            return None
        _check(st, "dare_server_poll")
        return tm

    def drain(self):
        _check(lib.dare_server_drain(self.handle), "dare_server_drain")

    def stats(self) -> ServerStats:
        st = ServerStats()
        _check(lib.dare_server_get_stats(self.handle, ct.byref(st)), "dare_server_get_stats")
        return st

    def close(self):
        if getattr(self, "handle", None):
            lib.dare_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def now_seconds() -> float:
    return float(lib.dare_now_seconds())
