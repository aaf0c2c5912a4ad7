"""MI355X (gfx950) closest-hit ray tracing through a BVH built with the
SAH-plus-spatial-distance split of arXiv 2208.10008 (Sec. II-B, Eq. (2)).

Thin ctypes binding of ``librt_mi355x.so`` (C ABI in ``include/rt_mi355x.h``).
Every step of the path runs in the library's HIP kernels; this module only
marshals arguments.  PyTorch supplies device memory (CUDA tensors) and
streams.  Importing works without a GPU; any call that needs the library
raises :class:`RtError` if it has not been built (``python -m
paper_2208_10008_amd._build``) -- there is no CPU fallback.

Low-level functions keep the C names (:func:`rt_build`, :func:`rt_trace`,
:func:`rt_trace_bounces`, ...); :class:`BVH` wraps a handle.

Typical use (all tensors on the GPU)::

    bvh = BVH(tris, SplitParams(alpha=0.4, src=tx))          # Eq. (2) tree for this Tx
    out, path_len, n_hits = bvh.trace_bounces(rays, 6)       # reflection chains
    rx = Receivers(points, delta, cap=1 << 16)               # receiving spheres, Eq. (4)
    bvh.trace_receive(rays, 6, rx); rx.dedup(out, 6)         # ... and one record per path
    e = Energy(material, refl, Energy.k0_for(2.4e9), 1e-10)  # energy stop rule
    bvh.trace_energy(rays, 6, e, receivers=rx)
    nbr = rt_wedges(tris)                                    # diffracting edges
    rec, count = rt_diffract_segments(tris, nbr, seg, out, 6, delta, cone, cap)
    batch = Batch(64); batch.set(queries); batch.autotune(); batch.launch()
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librt_mi355x.so")

RT_OK, RT_EINVAL, RT_ENOMEM, RT_EHIP, RT_EDEPTH = 0, -1, -2, -3, -4
RT_TRACE_NO_PAD = 1  # rt_trace_opts.flags: rows after a chain's miss are not written
D_MODES = {"mean": 0, "sum": 1, "kweighted": 2, "parent": 3}
D_NORMS = {"unit": 0, "raw": 1}
NODE_FORMATS = {"bin2": 0, "f4": 1, "q4": 2}
MAX_BOUNCES = 64
LEAF_HIST = 16  # RT_LEAF_HIST


class RtError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class rt_split_params(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_float), ("t_isect", ctypes.c_float),
                ("t_trav", ctypes.c_float), ("src", ctypes.c_float * 3),
                ("max_leaf", ctypes.c_int32), ("nbins", ctypes.c_int32),
                ("d_mode", ctypes.c_int32), ("d_norm", ctypes.c_int32),
                ("max_depth", ctypes.c_int32), ("depth_limit", ctypes.c_int32),
                ("node_format", ctypes.c_int32)]


class rt_bvh_info(ctypes.Structure):
    _fields_ = [("n_tris", ctypes.c_int64), ("n_nodes", ctypes.c_int64),
                ("n_internal", ctypes.c_int64), ("n_leaves", ctypes.c_int64),
                ("depth", ctypes.c_int32), ("n_levels", ctypes.c_int32),
                ("device_bytes", ctypes.c_int64), ("trace_bytes", ctypes.c_int64),
                ("root_lo", ctypes.c_float * 3), ("root_hi", ctypes.c_float * 3),
                ("node_format", ctypes.c_int32), ("n_trace_nodes", ctypes.c_int32),
                ("has_stats", ctypes.c_int32), ("max_leaf_count", ctypes.c_int32),
                ("tree_cost", ctypes.c_double), ("root_area", ctypes.c_double),
                ("leaf_hist", ctypes.c_int64 * LEAF_HIST)]


class rt_trace_opts(ctypes.Structure):
    _fields_ = [("seg_rays", ctypes.c_void_p), ("ray_stats", ctypes.c_void_p),
                ("block", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("refill", ctypes.c_int32), ("lanes_per_ray", ctypes.c_int32),
                ("cut", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("chain_ws", ctypes.c_void_p), ("chain_ws_bytes", ctypes.c_int64),
                ("batch_order", ctypes.c_void_p)]


class rt_query(ctypes.Structure):
    _fields_ = [("bvh", ctypes.c_void_p), ("rays", ctypes.c_void_p), ("n", ctypes.c_int64),
                ("max_bounces", ctypes.c_int32), ("status", ctypes.c_int32),
                ("out", ctypes.c_void_p), ("path_len", ctypes.c_void_p),
                ("n_hits", ctypes.c_void_p), ("receivers", ctypes.c_void_p)]


class rt_batch_config(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("grid", ctypes.c_int32), ("order", ctypes.c_int32),
                ("graph", ctypes.c_int32)]


class rt_receivers(ctypes.Structure):
    _fields_ = [("pos", ctypes.c_void_p), ("n", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("delta", ctypes.c_double), ("rec", ctypes.c_void_p), ("cap", ctypes.c_int64),
                ("count", ctypes.c_void_p)]


class rt_energy(ctypes.Structure):
    _fields_ = [("material", ctypes.c_void_p), ("refl", ctypes.c_void_p),
                ("n_materials", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("k0", ctypes.c_double), ("min_power", ctypes.c_double),
                ("power", ctypes.c_void_p)]


# numpy view of rt_reception (32 bytes)
RECEPTION_DTYPE = np.dtype([("rx", "<i4"), ("ray", "<i4"), ("order", "<i4"), ("keep", "<i4"),
                            ("l", "<f8"), ("dist", "<f8")])
assert RECEPTION_DTYPE.itemsize == 32

# numpy view of rt_diffracted (64 bytes)
DIFFRACTED_DTYPE = np.dtype([("ray", "<i4"), ("order", "<i4"), ("facet", "<i4"), ("edge", "<i4"),
                             ("cone", "<i4"), ("pad", "<i4"), ("path", "<f8"), ("ray8", "<f4", 8)])
assert DIFFRACTED_DTYPE.itemsize == 64

BATCH_MODES = {"direct": 0, "queue": 1}
BATCH_ORDERS = {"given": 0, "cost": 1}

# numpy view of rt_node_rec (64 bytes)
NODE_DTYPE = np.dtype([("lo", "<f4", 3), ("hi", "<f4", 3), ("left", "<i4"), ("first", "<i4"),
                       ("count", "<i4"), ("depth", "<i4"), ("axis", "<i4"), ("plane", "<i4"),
                       ("flags", "<i4"), ("reserved", "<i4"), ("cost", "<f8")])
assert NODE_DTYPE.itemsize == 64

EXPORTS = ("rt_split_params_default", "rt_build", "rt_rebuild", "rt_rebuild_async", "rt_bvh_wait",
           "rt_trace",
           "rt_trace_bounces", "rt_trace_ex", "rt_bvh_info_get", "rt_bvh_stats", "rt_bvh_download",
           "rt_bvh_export_trace_nodes", "rt_bvh_destroy", "rt_last_error", "rt_batch_create",
           "rt_batch_set", "rt_batch_configure", "rt_batch_get_config", "rt_batch_launch",
           "rt_batch_autotune", "rt_batch_destroy", "rt_rays_from_directions",
           "rt_rays_from_directions_many", "rt_trace_receive", "rt_receive_segments", "rt_receive_dedup_workspace",
           "rt_receive_dedup", "rt_trace_energy", "rt_wedges", "rt_wedges_noalloc",
           "rt_diffract_segments", "rt_trace_chain_ws_bytes", "rt_rays_batch_order",
           "rt_rays_batch_order_ws_bytes", "rt_split_cus_mask",
           "rt_streams_split_cus", "rt_stream_destroy")
PROBE_EXPORTS = ("rt_probe_read", "rt_probe_copy")  # include/rt_probe.h

_lib = None


def load(path: str = LIB_PATH):
    """Loads the HIP library; raises RtError if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RtError(RT_EHIP, f"{path} is not built; run python -m paper_2208_10008_amd._build")
    lib = ctypes.CDLL(path)
    P, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    lib.rt_split_params_default.argtypes = [ctypes.POINTER(rt_split_params)]
    lib.rt_split_params_default.restype = None
    lib.rt_build.argtypes = [P, i64, ctypes.POINTER(rt_split_params), ctypes.POINTER(P), P]
    lib.rt_rebuild.argtypes = [P, P, i64, ctypes.POINTER(rt_split_params), P]
    lib.rt_rebuild_async.argtypes = [P, P, i64, ctypes.POINTER(rt_split_params), P]
    lib.rt_bvh_wait.argtypes = [P]
    lib.rt_trace.argtypes = [P, P, i64, P, P]
    lib.rt_trace_bounces.argtypes = [P, P, i64, i32, P, P, P, P]
    lib.rt_trace_ex.argtypes = [P, P, i64, i32, P, P, P, ctypes.POINTER(rt_trace_opts), P]
    lib.rt_trace_chain_ws_bytes.argtypes = [i64]
    lib.rt_trace_chain_ws_bytes.restype = i64
    lib.rt_bvh_info_get.argtypes = [P, ctypes.POINTER(rt_bvh_info)]
    lib.rt_bvh_stats.argtypes = [P, ctypes.POINTER(rt_bvh_info)]
    lib.rt_bvh_download.argtypes = [P, P, i64, P, i64]
    lib.rt_bvh_export_trace_nodes.argtypes = [P, P, ctypes.POINTER(i64)]
    lib.rt_bvh_destroy.argtypes = [P]
    lib.rt_bvh_destroy.restype = None
    lib.rt_last_error.argtypes = []
    lib.rt_last_error.restype = ctypes.c_char_p
    lib.rt_probe_read.argtypes = [P, i64, i64, i32, i32, P, P]
    lib.rt_batch_create.argtypes = [i32, ctypes.POINTER(P)]
    lib.rt_batch_set.argtypes = [P, ctypes.POINTER(rt_query), i32]
    lib.rt_batch_configure.argtypes = [P, ctypes.POINTER(rt_batch_config)]
    lib.rt_batch_get_config.argtypes = [P, ctypes.POINTER(rt_batch_config)]
    lib.rt_batch_launch.argtypes = [P, P]
    lib.rt_batch_autotune.argtypes = [P, i32, P, ctypes.POINTER(ctypes.c_float)]
    f32 = ctypes.c_float
    lib.rt_rays_from_directions.argtypes = [P, i64, f32, f32, f32, f32, f32, P, P]
    lib.rt_rays_from_directions_many.argtypes = [P, i64, P, i32, f32, f32, P, i64, P]
    lib.rt_rays_batch_order.argtypes = [P, i64, i32, P, P, P]
    lib.rt_rays_batch_order_ws_bytes.argtypes = [i64]
    lib.rt_rays_batch_order_ws_bytes.restype = i64
    lib.rt_streams_split_cus.argtypes = [i32, ctypes.POINTER(P), ctypes.POINTER(P)]
    lib.rt_stream_destroy.argtypes = [P]
    lib.rt_split_cus_mask.argtypes = [i32, P]
    lib.rt_batch_destroy.argtypes = [P]
    lib.rt_batch_destroy.restype = None
    lib.rt_probe_copy.argtypes = [P, P, i64, P]
    RX = ctypes.POINTER(rt_receivers)
    lib.rt_trace_receive.argtypes = [P, P, i64, i32, P, P, P, RX, P]
    lib.rt_receive_segments.argtypes = [P, P, i64, i32, RX, P]
    lib.rt_receive_dedup_workspace.argtypes = [i64, i32]
    lib.rt_receive_dedup_workspace.restype = i64
    lib.rt_receive_dedup.argtypes = [P, i64, i32, RX, P, i64, P]
    lib.rt_trace_energy.argtypes = [P, P, i64, i32, ctypes.POINTER(rt_energy), P, P, P, RX, P]
    lib.rt_wedges.argtypes = [P, i64, P, P]
    lib.rt_wedges_noalloc.argtypes = [P, i64, P, P]
    lib.rt_diffract_segments.argtypes = [P, i64, P, P, P, i64, i32, ctypes.c_double, P, i32, P,
                                         i64, P, P]
    for name in ("rt_build", "rt_rebuild", "rt_rebuild_async", "rt_bvh_wait", "rt_trace",
                 "rt_trace_bounces", "rt_trace_ex",
                 "rt_bvh_info_get", "rt_bvh_stats", "rt_bvh_download",
                 "rt_bvh_export_trace_nodes", "rt_probe_read", "rt_probe_copy", "rt_batch_create", "rt_batch_set",
                 "rt_batch_configure", "rt_batch_get_config", "rt_batch_launch",
                 "rt_batch_autotune", "rt_rays_from_directions", "rt_rays_from_directions_many",
                 "rt_rays_batch_order", "rt_streams_split_cus", "rt_stream_destroy",
                 "rt_split_cus_mask",
                 "rt_trace_receive",
                 "rt_receive_segments", "rt_receive_dedup", "rt_trace_energy", "rt_wedges",
                 "rt_wedges_noalloc", "rt_diffract_segments"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc):
    if rc != RT_OK:
        raise RtError(rc, load().rt_last_error().decode())


@dataclasses.dataclass
class SplitParams:
    """Eq. (2) split parameters (rt_split_params)."""
    alpha: float = 1.0
    t_isect: float = 1.0
    t_trav: float = 1.0
    src: tuple = (0.0, 0.0, 0.0)
    max_leaf: int = 4
    nbins: int = 16
    d_mode: str = "mean"
    d_norm: str = "unit"
    max_depth: int = 32
    depth_limit: int = 64
    node_format: str = "bin2"

    def c(self) -> rt_split_params:
        p = rt_split_params()
        p.alpha, p.t_isect, p.t_trav = self.alpha, self.t_isect, self.t_trav
        for k in range(3):
            p.src[k] = self.src[k]
        p.max_leaf, p.nbins = self.max_leaf, self.nbins
        p.d_mode, p.d_norm = D_MODES[self.d_mode], D_NORMS[self.d_norm]
        p.max_depth, p.depth_limit = self.max_depth, self.depth_limit
        p.node_format = NODE_FORMATS[self.node_format]
        return p


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _dev(t, dtype, cols, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise RtError(RT_EINVAL, f"{name} must be a CUDA tensor")
    if t.dtype != dtype or t.dim() != 2 or t.shape[1] != cols or not t.is_contiguous():
        raise RtError(RT_EINVAL, f"{name} must be a contiguous {dtype} tensor [n, {cols}]")
    return t


# ---- C-named entry points -------------------------------------------------
def rt_build(tris, params: SplitParams | rt_split_params, stream=None) -> ctypes.c_void_p:
    """rt_build(tris [n, 9] float32 CUDA tensor, params) -> handle."""
    lib = load()
    _dev(tris, __import__("torch").float32, 9, "tris")
    cp = params.c() if isinstance(params, SplitParams) else params
    h = ctypes.c_void_p()
    _check(lib.rt_build(_ptr(tris), tris.shape[0], ctypes.byref(cp), ctypes.byref(h), _stream(stream)))
    return h


def rt_rebuild(handle, tris, params, stream=None):
    lib = load()
    _dev(tris, __import__("torch").float32, 9, "tris")
    cp = params.c() if isinstance(params, SplitParams) else params
    _check(lib.rt_rebuild(handle, _ptr(tris), tris.shape[0], ctypes.byref(cp), _stream(stream)))


def rt_rebuild_async(handle, tris, params, stream=None):
    """Queues the build on `stream` and returns; the tree is usable after
    rt_bvh_wait(handle).  tris must stay alive until the build has run."""
    lib = load()
    _dev(tris, __import__("torch").float32, 9, "tris")
    cp = params.c() if isinstance(params, SplitParams) else params
    _check(lib.rt_rebuild_async(handle, _ptr(tris), tris.shape[0], ctypes.byref(cp),
                                _stream(stream)))


def rt_bvh_wait(handle):
    _check(load().rt_bvh_wait(handle))


def rt_trace(handle, rays, out, stream=None):
    """rays [n, 8] float32, out [n, 4] int32 view of rt_hit (CUDA tensors)."""
    lib = load()
    _check(lib.rt_trace(handle, _ptr(rays), rays.shape[0], _ptr(out), _stream(stream)))


def rt_trace_bounces(handle, rays, max_bounces, out, path_len=None, n_hits=None, stream=None):
    lib = load()
    _check(lib.rt_trace_bounces(handle, _ptr(rays), rays.shape[0], max_bounces, _ptr(out),
                                _ptr(path_len), _ptr(n_hits), _stream(stream)))


def rt_trace_chain_ws_bytes(n: int) -> int:
    return int(load().rt_trace_chain_ws_bytes(n))


def rt_trace_ex(handle, rays, max_bounces, out, path_len=None, n_hits=None, seg_rays=None,
                ray_stats=None, block=0, grid=0, refill=0, lanes_per_ray=0, cut=0, chain_ws=None,
                stream=None, flags=0, batch_order=None):
    lib = load()
    o = rt_trace_opts()
    o.batch_order = None if batch_order is None else batch_order.data_ptr()
    o.seg_rays = None if seg_rays is None else seg_rays.data_ptr()
    o.ray_stats = None if ray_stats is None else ray_stats.data_ptr()
    o.block, o.grid, o.refill, o.lanes_per_ray = block, grid, refill, lanes_per_ray
    o.cut, o.flags = cut, flags
    if chain_ws is not None:
        o.chain_ws = chain_ws.data_ptr()
        o.chain_ws_bytes = chain_ws.numel() * chain_ws.element_size()
    _check(lib.rt_trace_ex(handle, _ptr(rays), rays.shape[0], max_bounces, _ptr(out),
                           _ptr(path_len), _ptr(n_hits), ctypes.byref(o), _stream(stream)))


def rt_rays_batch_order_ws_bytes(n: int) -> int:
    return int(load().rt_rays_batch_order_ws_bytes(n))


def rt_rays_batch_order(rays, axis=2, order=None, keys=None, stream=None):
    """Dispatch order of the rays' batches of 64 (rt_trace_opts.batch_order):
    returns order, an int32 CUDA tensor of ceil(n / 64) batch indices.  keys:
    int32 workspace of rt_rays_batch_order_ws_bytes(n) / 4 entries (its first
    ceil(n / 64) are left holding the batch keys)."""
    import torch
    lib = load()
    _dev(rays, torch.float32, 8, "rays")
    n = rays.shape[0]
    nb = (n + 63) // 64
    nk = rt_rays_batch_order_ws_bytes(n) // 4
    if order is None:
        order = torch.empty(nb, dtype=torch.int32, device=rays.device)
    if keys is None:
        keys = torch.empty(nk, dtype=torch.int32, device=rays.device)
    if order.numel() < nb or keys.numel() < nk or order.dtype != torch.int32 or keys.dtype != torch.int32:
        raise RtError(RT_EINVAL, "order: int32 [ceil(n / 64)]; keys: int32 "
                                 "[rt_rays_batch_order_ws_bytes(n) / 4]")
    _check(lib.rt_rays_batch_order(_ptr(rays), rays.shape[0], axis, _ptr(order), _ptr(keys),
                                   _stream(stream)))
    return order


def rt_split_cus_mask(k: int) -> np.ndarray:
    """The CU mask rt_streams_split_cus gives its `small` stream (host only)."""
    m = (ctypes.c_uint32 * 8)()
    _check(load().rt_split_cus_mask(k, m))
    return np.array(list(m), dtype=np.uint32)


class SplitStreams:
    """rt_streams_split_cus: `small` runs on k compute units, `large` on the
    rest (torch external streams; close() or garbage collection frees them)."""

    def __init__(self, k: int):
        import torch
        lib = load()
        a, b = ctypes.c_void_p(), ctypes.c_void_p()
        _check(lib.rt_streams_split_cus(k, ctypes.byref(a), ctypes.byref(b)))
        self._raw = [a.value, b.value]
        self.small = torch.cuda.ExternalStream(a.value)
        self.large = torch.cuda.ExternalStream(b.value)

    def close(self):
        if self._raw:
            import torch
            torch.cuda.synchronize()
            for h in self._raw:
                _check(load().rt_stream_destroy(ctypes.c_void_p(h)))
            self._raw = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def rt_trace_receive(handle, rays, max_bounces, out, path_len, n_hits, receivers: "Receivers",
                     stream=None):
    lib = load()
    c = receivers.c()
    _check(lib.rt_trace_receive(handle, _ptr(rays), rays.shape[0], max_bounces, _ptr(out),
                                _ptr(path_len), _ptr(n_hits), ctypes.byref(c), _stream(stream)))


def rt_receive_segments(seg_rays, hits, max_bounces, receivers: "Receivers", stream=None):
    """seg_rays [max_bounces, n, 8] float32, hits [max_bounces, n, 4] int32 view of rt_hit."""
    lib = load()
    c = receivers.c()
    _check(lib.rt_receive_segments(_ptr(seg_rays), _ptr(hits), hits.shape[1], max_bounces,
                                   ctypes.byref(c), _stream(stream)))


def rt_receive_dedup_workspace(cap, n_rx) -> int:
    return int(load().rt_receive_dedup_workspace(cap, n_rx))


def rt_receive_dedup(hits, max_bounces, receivers: "Receivers", work, stream=None):
    lib = load()
    c = receivers.c()
    _check(lib.rt_receive_dedup(_ptr(hits), hits.shape[1], max_bounces, ctypes.byref(c),
                                _ptr(work), work.numel() * work.element_size(), _stream(stream)))


class Receivers:
    """Field points (float64 [n, 3] CUDA tensor), the launch's ray spacing
    delta (radians) and a device buffer of `cap` reception records
    (rt_reception) with its counter."""

    def __init__(self, pos, delta: float, cap: int):
        import torch
        _dev(pos, torch.float64, 3, "pos")
        self.pos = pos
        self.delta = float(delta)
        self.cap = int(cap)
        self.rec = torch.zeros((max(self.cap, 1), 8), dtype=torch.int32, device=pos.device)
        self.count_buf = torch.zeros(1, dtype=torch.int64, device=pos.device)
        self._work = None

    def c(self) -> rt_receivers:
        c = rt_receivers()
        c.pos = self.pos.data_ptr() if self.pos.shape[0] else None
        c.n = self.pos.shape[0]
        c.reserved = 0
        c.delta = self.delta
        c.rec = self.rec.data_ptr()
        c.cap = self.cap
        c.count = self.count_buf.data_ptr()
        return c

    def count(self) -> int:
        """Receptions found by the last call (may exceed cap); synchronises."""
        return int(self.count_buf.item())

    def records(self) -> np.ndarray:
        """The stored records as a numpy RECEPTION_DTYPE array (synchronises)."""
        k = min(self.count(), self.cap)
        return self.rec[:k].cpu().numpy().view(RECEPTION_DTYPE).reshape(-1)

    def dedup(self, hits, max_bounces, stream=None):
        """Marks one record per (field point, order, facet sequence) as kept."""
        import torch
        need = rt_receive_dedup_workspace(self.cap, self.pos.shape[0])
        if self._work is None or self._work.numel() < need:
            self._work = torch.empty(max(need, 256), dtype=torch.uint8, device=self.pos.device)
        rt_receive_dedup(hits, max_bounces, self, self._work, stream)


class Energy:
    """The energy stop rule (Sec. III-B): material index per facet (int32
    [n_tris] CUDA tensor, caller's facet order), power reflection coefficient
    per material (float64 [n_materials] CUDA tensor), the free-space constant
    k0 = (lambda / 4 pi)^2 and the threshold min_power; ``power`` (float64 [n])
    receives each chain's power ratio after its last hit when given."""

    def __init__(self, material, refl, k0: float, min_power: float, power=None):
        import torch
        if material.dtype != torch.int32 or material.dim() != 1 or not material.is_cuda:
            raise RtError(RT_EINVAL, "material must be an int32 CUDA tensor [n_tris]")
        if refl.dtype != torch.float64 or refl.dim() != 1 or not refl.is_cuda:
            raise RtError(RT_EINVAL, "refl must be a float64 CUDA tensor [n_materials]")
        self.material, self.refl = material.contiguous(), refl.contiguous()
        self.k0, self.min_power, self.power = float(k0), float(min_power), power

    @staticmethod
    def k0_for(frequency_hz: float) -> float:
        """(lambda / (4 pi))^2 for a frequency in Hz (isotropic antennas)."""
        lam = 299_792_458.0 / frequency_hz
        return (lam / (4.0 * np.pi)) ** 2

    def c(self) -> rt_energy:
        e = rt_energy()
        e.material = self.material.data_ptr()
        e.refl = self.refl.data_ptr() if self.refl.numel() else None
        e.n_materials = self.refl.numel()
        e.reserved = 0
        e.k0, e.min_power = self.k0, self.min_power
        e.power = None if self.power is None else self.power.data_ptr()
        return e


def rt_trace_energy(handle, rays, max_bounces, energy: Energy, out, path_len, n_hits,
                    receivers: "Receivers | None" = None, stream=None):
    lib = load()
    e = energy.c()
    rx = None if receivers is None else ctypes.byref(receivers.c())
    _check(lib.rt_trace_energy(handle, _ptr(rays), rays.shape[0], max_bounces, ctypes.byref(e),
                               _ptr(out), _ptr(path_len), _ptr(n_hits), rx, _stream(stream)))


def rt_wedges(tris, nbr=None, stream=None):
    """Neighbour of every half-edge (int32 [n, 3] CUDA tensor): the other
    facet of a wedge edge, -1 free, -2 not diffracting.  Synchronises."""
    import torch
    _dev(tris, torch.float32, 9, "tris")
    if nbr is None:
        nbr = torch.empty((tris.shape[0], 3), dtype=torch.int32, device=tris.device)
    _check(load().rt_wedges(_ptr(tris), tris.shape[0], _ptr(nbr), _stream(stream)))
    return nbr


def rt_wedges_noalloc(tris, nbr, stream=None):
    """rt_wedges without device allocation (up to 262,144 facets); nbr is the
    caller's int32 [n, 3] CUDA tensor.  Synchronises."""
    import torch
    _dev(tris, torch.float32, 9, "tris")
    _check(load().rt_wedges_noalloc(_ptr(tris), tris.shape[0], _ptr(nbr), _stream(stream)))
    return nbr


def rt_diffract_segments(tris, nbr, seg_rays, hits, max_bounces, delta, cone, cap, out=None,
                         count=None, stream=None):
    """Diffracted rays of stored chains; returns (records int32 [cap, 16]
    tensor viewing rt_diffracted, count int64 [1] tensor).  cone: float64
    [n_cone, 2] CUDA tensor of (cos, sin)."""
    import torch
    _dev(tris, torch.float32, 9, "tris")
    if out is None:
        out = torch.zeros((max(int(cap), 1), 16), dtype=torch.int32, device=tris.device)
    if count is None:
        count = torch.zeros(1, dtype=torch.int64, device=tris.device)
    n = hits.shape[1]
    _check(load().rt_diffract_segments(_ptr(tris), tris.shape[0], _ptr(nbr), _ptr(seg_rays),
                                       _ptr(hits), n, max_bounces, float(delta), _ptr(cone),
                                       cone.shape[0], _ptr(out), int(cap), _ptr(count),
                                       _stream(stream)))
    return out, count


def diffracted_records(out, count, cap) -> np.ndarray:
    """The stored rt_diffracted records as a numpy DIFFRACTED_DTYPE array."""
    k = min(int(count.item()), int(cap))
    return out[:k].cpu().numpy().view(DIFFRACTED_DTYPE).reshape(-1)


def diffracted_rays(out, k):
    """The first k diffracted rays as a contiguous float32 [k, 8] ray tensor."""
    import torch
    return out[:k, 8:16].contiguous().view(torch.float32)


def rt_bvh_info_get(handle) -> rt_bvh_info:
    info = rt_bvh_info()
    _check(load().rt_bvh_info_get(handle, ctypes.byref(info)))
    return info


def rt_bvh_stats(handle) -> rt_bvh_info:
    """Sizes, Eq. (1) tree cost and leaf-size histogram (synchronises)."""
    info = rt_bvh_info()
    _check(load().rt_bvh_stats(handle, ctypes.byref(info)))
    return info


def rt_bvh_download(handle):
    info = rt_bvh_info_get(handle)
    nodes = np.zeros(info.n_nodes, dtype=NODE_DTYPE)
    perm = np.zeros(info.n_tris, dtype=np.int32)
    _check(load().rt_bvh_download(handle, nodes.ctypes.data_as(ctypes.c_void_p), info.n_nodes,
                                  perm.ctypes.data_as(ctypes.c_void_p), info.n_tris))
    return nodes, perm


def rt_bvh_export_trace_nodes(handle) -> np.ndarray:
    """Raw traversal node records (uint8 bytes) as the GPU reads them."""
    lib = load()
    nbytes = ctypes.c_int64(0)
    _check(lib.rt_bvh_export_trace_nodes(handle, None, ctypes.byref(nbytes)))
    buf = np.zeros(nbytes.value, dtype=np.uint8)
    _check(lib.rt_bvh_export_trace_nodes(handle, buf.ctypes.data_as(ctypes.c_void_p),
                                         ctypes.byref(nbytes)))
    return buf


def rt_probe_read(buf, span_bytes, passes, groups, sink, stream=None):
    """Each of `groups` work-groups streams `span_bytes` of `buf` (a device
    tensor) `passes` times; `sink` is a device int32 tensor of >= groups
    entries.  Returns the bytes moved."""
    nbytes = buf.numel() * buf.element_size()
    _check(load().rt_probe_read(buf.data_ptr(), nbytes, span_bytes, passes, groups,
                                sink.data_ptr(), _stream(stream)))
    return span_bytes * passes * groups


def rt_probe_copy(src, dst, stream=None):
    """Plain device copy of src into dst (same byte size)."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() < nbytes:
        raise RtError(RT_EINVAL, "rt_probe_copy: dst too small")
    _check(load().rt_probe_copy(src.data_ptr(), dst.data_ptr(), nbytes, _stream(stream)))


def rt_bvh_destroy(handle):
    if handle:
        load().rt_bvh_destroy(handle)


# ---- handle wrapper ---------------------------------------------------------
def chain_workspace(n: int, device="cuda"):
    """Device workspace of a two-launch trace of n rays (torch uint8, 256-byte
    aligned by the caching allocator)."""
    import torch
    return torch.empty(rt_trace_chain_ws_bytes(n), dtype=torch.uint8, device=device)


class BVH:
    """Owns one rt_bvh handle; tensors passed in stay owned by the caller."""

    def __init__(self, tris, params: SplitParams | None = None, stream=None):
        self.params = params or SplitParams()
        self.handle = rt_build(tris, self.params, stream)

    def rebuild(self, tris, params: SplitParams | None = None, stream=None):
        if params is not None:
            self.params = params
        rt_rebuild(self.handle, tris, self.params, stream)

    def rebuild_async(self, tris, params: SplitParams | None = None, stream=None):
        """rt_rebuild_async: the tree is usable after wait()."""
        if params is not None:
            self.params = params
        rt_rebuild_async(self.handle, tris, self.params, stream)

    def wait(self):
        rt_bvh_wait(self.handle)

    def info(self) -> rt_bvh_info:
        return rt_bvh_info_get(self.handle)

    def stats(self) -> rt_bvh_info:
        return rt_bvh_stats(self.handle)

    def download(self):
        return rt_bvh_download(self.handle)

    def trace_nodes(self) -> np.ndarray:
        return rt_bvh_export_trace_nodes(self.handle)

    def hits_buffer(self, n, max_bounces=1):
        import torch
        return torch.empty((max_bounces, n, 4), dtype=torch.int32, device="cuda")

    def trace(self, rays, out=None, stream=None):
        _dev(rays, __import__("torch").float32, 8, "rays")
        if out is None:
            out = self.hits_buffer(rays.shape[0])[0]
        rt_trace(self.handle, rays, out, stream)
        return out

    def trace_bounces(self, rays, max_bounces, out=None, path_len=None, n_hits=None,
                      seg_rays=None, ray_stats=None, block=0, grid=0, refill=0, lanes_per_ray=0,
                      cut=0, chain_ws=None, stream=None, pad=True, batch_order=None):
        """cut >= 1: two launches (see rt_trace_opts.cut); chain_ws is made
        (rt_trace_chain_ws_bytes(n) bytes) when not given.  pad=False sets
        RT_TRACE_NO_PAD: rows of ``out`` after each chain's miss keep what they
        held, and ``n_hits`` tells where each chain ends."""
        import torch
        _dev(rays, torch.float32, 8, "rays")
        n = rays.shape[0]
        if cut > 0 and chain_ws is None:
            chain_ws = chain_workspace(n, rays.device)
        if out is None:
            out = self.hits_buffer(n, max_bounces)
        if path_len is None:
            path_len = torch.empty(n, dtype=torch.float64, device=rays.device)
        if n_hits is None:
            n_hits = torch.empty(n, dtype=torch.int32, device=rays.device)
        if (seg_rays is None and ray_stats is None and block == 0 and grid == 0 and refill == 0
                and lanes_per_ray == 0 and cut == 0 and pad and batch_order is None):
            rt_trace_bounces(self.handle, rays, max_bounces, out, path_len, n_hits, stream)
        else:
            rt_trace_ex(self.handle, rays, max_bounces, out, path_len, n_hits, seg_rays,
                        ray_stats, block, grid, refill, lanes_per_ray, cut, chain_ws, stream,
                        0 if pad else RT_TRACE_NO_PAD, batch_order)
        return out, path_len, n_hits

    def trace_receive(self, rays, max_bounces, receivers: Receivers, out=None, path_len=None,
                      n_hits=None, stream=None):
        """Reflection chains with every segment tested against the field
        points (Sec. III-C); the receptions land in ``receivers``."""
        import torch
        _dev(rays, torch.float32, 8, "rays")
        n = rays.shape[0]
        if out is None:
            out = self.hits_buffer(n, max_bounces)
        if path_len is None:
            path_len = torch.empty(n, dtype=torch.float64, device=rays.device)
        if n_hits is None:
            n_hits = torch.empty(n, dtype=torch.int32, device=rays.device)
        rt_trace_receive(self.handle, rays, max_bounces, out, path_len, n_hits, receivers, stream)
        return out, path_len, n_hits

    def trace_energy(self, rays, max_bounces, energy: Energy, receivers: Receivers | None = None,
                     out=None, path_len=None, n_hits=None, stream=None):
        """Reflection chains that also stop by energy (Sec. III-B); with
        ``receivers``, every traced segment is tested as in trace_receive."""
        import torch
        _dev(rays, torch.float32, 8, "rays")
        n = rays.shape[0]
        if out is None:
            out = self.hits_buffer(n, max_bounces)
        if path_len is None:
            path_len = torch.empty(n, dtype=torch.float64, device=rays.device)
        if n_hits is None:
            n_hits = torch.empty(n, dtype=torch.int32, device=rays.device)
        rt_trace_energy(self.handle, rays, max_bounces, energy, out, path_len, n_hits, receivers,
                        stream)
        return out, path_len, n_hits

    def close(self):
        if getattr(self, "handle", None):
            rt_bvh_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def rt_rays_from_directions(dirs, n, src, tmin, tmax, rays=None, stream=None):
    """Rays [n, 8] from src along the first n rows of dirs (float32 [m, 3]
    CUDA tensor, m >= n)."""
    import torch
    if not isinstance(dirs, torch.Tensor) or not dirs.is_cuda or dirs.dtype != torch.float32 \
            or dirs.dim() != 2 or dirs.shape[1] != 3 or not dirs.is_contiguous() or dirs.shape[0] < n:
        raise RtError(RT_EINVAL, "dirs must be a contiguous float32 CUDA tensor [>= n, 3]")
    if rays is None:
        rays = torch.empty((n, 8), dtype=torch.float32, device=dirs.device)
    _check(load().rt_rays_from_directions(dirs.data_ptr(), n, float(src[0]), float(src[1]),
                                          float(src[2]), float(tmin), float(tmax),
                                          rays.data_ptr(), _stream(stream)))
    return rays


# numpy view of rt_ray_launch (32 bytes): one launch of rt_rays_from_directions_many
RAY_LAUNCH_DTYPE = np.dtype([("src", "<f4", 3), ("reserved", "<i4"), ("first", "<i8"), ("n", "<i8")])
assert RAY_LAUNCH_DTYPE.itemsize == 32


def rt_rays_from_directions_many(dirs, table, tmin, tmax, rays, stream=None):
    """Rays of many launches with one kernel: table is a CUDA tensor holding
    RAY_LAUNCH_DTYPE records (e.g. uint8 [count * 32]) sorted by first; rays
    float32 [total, 8] CUDA tensor.  Rows no record covers are left as they are."""
    import torch
    if not isinstance(dirs, torch.Tensor) or not dirs.is_cuda or dirs.dtype != torch.float32 \
            or dirs.dim() != 2 or dirs.shape[1] != 3 or not dirs.is_contiguous():
        raise RtError(RT_EINVAL, "dirs must be a contiguous float32 CUDA tensor [m, 3]")
    if not table.is_cuda or not table.is_contiguous() or table.numel() * table.element_size() % 32:
        raise RtError(RT_EINVAL, "table must be a contiguous CUDA tensor of 32-byte records")
    _dev(rays, torch.float32, 8, "rays")
    count = table.numel() * table.element_size() // 32
    _check(load().rt_rays_from_directions_many(dirs.data_ptr(), dirs.shape[0], table.data_ptr(),
                                               count, float(tmin), float(tmax), rays.data_ptr(),
                                               rays.shape[0], _stream(stream)))
    return rays


class Batch:
    """Many trace queries in one launch (rt_batch).  A query is a dict with
    keys bvh (BVH), rays (float32 [n, 8] CUDA tensor), max_bounces, and
    optionally out, path_len, n_hits (allocated when missing)."""

    def __init__(self, max_queries: int):
        h = ctypes.c_void_p()
        _check(load().rt_batch_create(max_queries, ctypes.byref(h)))
        self.handle = h
        self.queries = []

    def set(self, queries):
        """Queries: dicts with bvh, rays, max_bounces and optionally out,
        path_len, n_hits (allocated when missing) and receivers (a Receivers:
        the query's chains are traced with the reception test)."""
        import torch
        arr = (rt_query * max(len(queries), 1))()
        held = []  # rt_receivers structs, alive until rt_batch_set has read them
        for k, q in enumerate(queries):
            rays = _dev(q["rays"], torch.float32, 8, "rays")
            n, nb = rays.shape[0], int(q["max_bounces"])
            if q.get("out") is None:
                q["out"] = torch.empty((nb, n, 4), dtype=torch.int32, device=rays.device)
            if q.get("path_len") is None:
                q["path_len"] = torch.empty(n, dtype=torch.float64, device=rays.device)
            if q.get("n_hits") is None:
                q["n_hits"] = torch.empty(n, dtype=torch.int32, device=rays.device)
            arr[k].bvh = q["bvh"].handle
            arr[k].rays = rays.data_ptr()
            arr[k].n = n
            arr[k].max_bounces = nb
            arr[k].out = q["out"].data_ptr()
            arr[k].path_len = q["path_len"].data_ptr()
            arr[k].n_hits = q["n_hits"].data_ptr()
            if q.get("receivers") is not None:
                held.append(q["receivers"].c())
                arr[k].receivers = ctypes.addressof(held[-1])
        _check(load().rt_batch_set(self.handle, arr, len(queries)))
        self.queries = queries
        return [arr[k].status for k in range(len(queries))]

    def set_table(self, arr, count: int):
        """Sets queries from a ctypes array of rt_query that the caller built
        (device pointers and sizes as the C ABI takes them, e.g. slices of
        pooled buffers); the caller keeps the buffers alive.  Returns the
        statuses."""
        _check(load().rt_batch_set(self.handle, arr, count))
        self.queries = []
        return [arr[k].status for k in range(count)]

    def configure(self, mode="direct", grid=0, order="cost", graph=False):
        c = rt_batch_config(BATCH_MODES[mode], grid, BATCH_ORDERS[order], int(bool(graph)))
        _check(load().rt_batch_configure(self.handle, ctypes.byref(c)))

    def config(self) -> dict:
        c = rt_batch_config()
        _check(load().rt_batch_get_config(self.handle, ctypes.byref(c)))
        inv_m = {v: k for k, v in BATCH_MODES.items()}
        inv_o = {v: k for k, v in BATCH_ORDERS.items()}
        return {"mode": inv_m[c.mode], "grid": c.grid, "order": inv_o[c.order], "graph": bool(c.graph)}

    def launch(self, stream=None):
        _check(load().rt_batch_launch(self.handle, _stream(stream)))

    def autotune(self, reps=2, stream=None) -> float:
        ms = ctypes.c_float()
        _check(load().rt_batch_autotune(self.handle, reps, _stream(stream), ctypes.byref(ms)))
        return ms.value

    def close(self):
        if getattr(self, "handle", None):
            load().rt_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def split_hits(out):
    """int32 [..., 4] view of rt_hit -> (tri_id int32, t, u, v float32) tensors."""
    ids = out[..., 0]
    tuv = out[..., 1:].view(__import__("torch").float32)
    return ids, tuv[..., 0], tuv[..., 1], tuv[..., 2]
