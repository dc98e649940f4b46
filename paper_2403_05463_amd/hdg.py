"""Python binding of the C ABI in ``include/hdg.h`` (argument marshalling only).

Every function keeps the C name and forwards plain pointers and sizes to
``libhdg.so``; device buffers are torch tensors on the GPU (used only for
memory and streams).  There is no fallback: if the library or a GPU is
missing the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhdg.so")

HDG_OK, HDG_EINVAL, HDG_ENOMEM, HDG_EHIP, HDG_EUNSUPPORTED, HDG_EMESH, HDG_ENONFINITE = 0, -1, -2, -3, -4, -5, -6
HDG_F64, HDG_F32 = 0, 1
HDG_WALL, HDG_FARFIELD = -1, -2
HDG_LES_NONE, HDG_LES_SMAGORINSKY, HDG_LES_VREMAN = 0, 1, 2
HDG_ROE, HDG_RUSANOV = 0, 1
HDG_KERNEL_VISCOUS, HDG_KERNEL_RESIDUAL, HDG_KERNEL_MORTAR, HDG_KERNEL_COUNT = 0, 1, 2, 3
KERNEL_NAMES = {0: "viscous", 1: "residual", 2: "mortar"}

EXPORTED = [
    "hdg_init", "hdg_finalize", "hdg_mesh_create", "hdg_mesh_destroy", "hdg_mesh_set_flags",
    "hdg_mesh_set_params", "hdg_mesh_info", "hdg_mesh_metric_blocks", "hdg_mesh_node_coords", "hdg_mesh_geometry", "hdg_residual",
    "hdg_rk3_steps",
    "hdg_reduce", "hdg_reduce_noalloc", "hdg_max_wave_speed", "hdg_timing_enable", "hdg_timing_read", "hdg_timing_samples", "hdg_stream_copy",
    "hdg_last_error",
    "hdg_mesh_autotune", "hdg_mesh_get_launch", "hdg_mesh_set_launch", "hdg_mesh_set_graphs",
    "hdg_batch_create", "hdg_batch_destroy", "hdg_batch_add", "hdg_batch_remove", "hdg_batch_info",
    "hdg_batch_rk3_steps", "hdg_batch_set_graphs", "hdg_batch_autotune", "hdg_batch_get_launch",
    "hdg_cluster_features", "hdg_cluster_fit",
]


class HdgError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"hdg status {status}: {msg}")
        self.status = status


class GmmOpts(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("pad", C.c_int32), ("reg_covar", C.c_double), ("tol", C.c_double)]


class GmmResult(C.Structure):
    _fields_ = [("feat_mean", C.c_double * 3), ("feat_std", C.c_double * 3), ("weight", C.c_double * 2),
                ("mean", (C.c_double * 3) * 2), ("cov", ((C.c_double * 3) * 3) * 2),
                ("log_likelihood", C.c_double), ("iterations", C.c_int32), ("degenerate", C.c_int32),
                ("converged", C.c_int32), ("pad", C.c_int32), ("n_viscous", C.c_int64)]


class MeshDesc(C.Structure):
    _fields_ = [("n_elem", C.c_int32), ("P", C.POINTER(C.c_int32)), ("geom_order", C.c_int32),
                ("xyz_geom", C.POINTER(C.c_double)), ("flag", C.POINTER(C.c_uint8)),
                ("nbr", C.POINTER(C.c_int32)), ("nbr_face", C.POINTER(C.c_int8)),
                ("orient", C.POINTER(C.c_int8))]


class Params(C.Structure):
    _fields_ = [("c0sq", C.c_double), ("nu", C.c_double), ("les_model", C.c_int32),
                ("C_les", C.c_double), ("mixed_face", C.c_int32), ("q_inf", C.c_double * 4),
                ("riemann", C.c_int32)]


class LaunchCfg(C.Structure):
    _fields_ = [("block", C.c_int32), ("persistent", C.c_int32), ("us_per_launch", C.c_double)]


_lib = None


def lib() -> C.CDLL:
    """Load ``libhdg.so``; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2403_05463_amd.build.build()")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, dp = C.c_void_p, C.c_int32, C.c_int64, C.POINTER(C.c_double)
        L.hdg_init.argtypes = [C.POINTER(vp), i32]
        L.hdg_finalize.argtypes = [vp]
        L.hdg_finalize.restype = None
        L.hdg_mesh_create.argtypes = [vp, C.POINTER(MeshDesc), C.POINTER(Params), C.POINTER(vp)]
        L.hdg_mesh_destroy.argtypes = [vp]
        L.hdg_mesh_destroy.restype = None
        L.hdg_mesh_set_flags.argtypes = [vp, C.POINTER(C.c_uint8)]
        L.hdg_mesh_set_params.argtypes = [vp, C.POINTER(Params)]
        L.hdg_mesh_info.argtypes = [vp, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64), C.POINTER(i32)]
        L.hdg_mesh_metric_blocks.argtypes = [vp, C.POINTER(i64)]
        L.hdg_mesh_node_coords.argtypes = [vp, dp]
        L.hdg_mesh_geometry.argtypes = [C.POINTER(MeshDesc), dp, dp, dp, dp, dp, dp]
        L.hdg_residual.argtypes = [vp, vp, vp, i32, vp]
        L.hdg_rk3_steps.argtypes = [vp, vp, vp, C.c_double, i32, i32, vp]
        L.hdg_reduce.argtypes = [vp, vp, dp, dp, dp, vp]
        L.hdg_reduce_noalloc.argtypes = [vp, vp, vp, vp]
        L.hdg_max_wave_speed.argtypes = [vp, vp, dp, vp]
        L.hdg_timing_enable.argtypes = [vp, i32]
        L.hdg_timing_read.argtypes = [vp, i32, dp, C.POINTER(i64)]
        L.hdg_timing_samples.argtypes = [vp, i32, C.POINTER(C.c_float), i64, C.POINTER(i64)]
        L.hdg_stream_copy.argtypes = [vp, vp, vp, i64, vp]
        L.hdg_cluster_features.argtypes = [vp, vp, vp, vp]
        L.hdg_cluster_fit.argtypes = [vp, vp, C.POINTER(GmmOpts), C.POINTER(GmmResult), vp, vp,
                                      C.POINTER(C.c_uint8), vp]
        L.hdg_mesh_autotune.argtypes = [vp, vp, i32, vp]
        L.hdg_mesh_get_launch.argtypes = [vp, i32, i32, i32, C.POINTER(LaunchCfg)]
        L.hdg_mesh_set_launch.argtypes = [vp, i32, i32, i32, C.POINTER(LaunchCfg)]
        L.hdg_mesh_set_graphs.argtypes = [vp, i32]
        L.hdg_batch_create.argtypes = [vp, i32, C.POINTER(vp)]
        L.hdg_batch_destroy.argtypes = [vp]
        L.hdg_batch_destroy.restype = None
        L.hdg_batch_add.argtypes = [vp, vp, vp, vp, C.c_double, C.POINTER(i32)]
        L.hdg_batch_remove.argtypes = [vp, i32]
        L.hdg_batch_info.argtypes = [vp, C.POINTER(i32), C.POINTER(i64), C.POINTER(i64)]
        L.hdg_batch_rk3_steps.argtypes = [vp, i32, i32, vp]
        L.hdg_batch_set_graphs.argtypes = [vp, i32]
        L.hdg_batch_autotune.argtypes = [vp, i32, vp]
        L.hdg_batch_get_launch.argtypes = [vp, i32, i32, i32, C.POINTER(LaunchCfg)]
        L.hdg_last_error.argtypes = []
        L.hdg_last_error.restype = C.c_char_p
        for name in EXPORTED:
            f = getattr(L, name)
            if name not in ("hdg_finalize", "hdg_mesh_destroy", "hdg_batch_destroy", "hdg_last_error"):
                f.restype = C.c_int
        _lib = L
    return _lib


def _check(status: int, what: str = ""):
    if status != HDG_OK:
        raise HdgError(status, (what + ": " if what else "") + lib().hdg_last_error().decode())


def hdg_last_error() -> str:
    return lib().hdg_last_error().decode()


def make_params(c0sq=25.0, nu=1e-3, les_model=HDG_LES_SMAGORINSKY, C_les=0.1, mixed_face=0,
                q_inf=(0.0, 0.0, 0.0, 0.0), riemann=0) -> Params:
    p = Params()
    p.c0sq, p.nu, p.les_model, p.C_les, p.mixed_face = c0sq, nu, les_model, C_les, mixed_face
    p.riemann = int(riemann)
    for k in range(4):
        p.q_inf[k] = float(q_inf[k])
    return p


def _ptr(t) -> int:
    """Device pointer of a torch tensor (or an int address)."""
    if isinstance(t, int):
        return t
    return int(t.data_ptr())


def _stream(stream) -> int | None:
    if stream is None:
        import torch
        return int(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


class Context:
    def __init__(self, handle: int, device: int):
        self.handle, self.device = handle, device

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.hdg_finalize(self.handle)
            self.handle = None


class Mesh:
    """Owner of an ``hdg_mesh`` handle plus its sizes.  With one order the
    state has shape (n_elem, 4, N^3); with several it is flat, element after
    element ([4][N_e^3] each), and ``offsets`` gives each element's first node."""

    def __init__(self, ctx: Context, handle: int, n_elem: int, P):
        Ps = np.broadcast_to(np.asarray(P, dtype=np.int32), (n_elem,)).copy()
        self.ctx, self.handle, self.n_elem = ctx, handle, n_elem
        self.Ps = Ps
        self.uniform = bool(np.all(Ps == Ps[0]))
        self.P = int(Ps[0]) if self.uniform else None
        self.N3 = (self.P + 1) ** 3 if self.uniform else None
        n3 = (Ps.astype(np.int64) + 1) ** 3
        self.nodes = int(n3.sum())
        self.offsets = np.concatenate([[0], np.cumsum(n3)[:-1]])

    @property
    def state_shape(self):
        return (self.n_elem, 4, self.N3) if self.uniform else (4 * self.nodes,)

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.hdg_mesh_destroy(self.handle)
            self.handle = None


def hdg_init(device: int = 0) -> Context:
    h = C.c_void_p()
    _check(lib().hdg_init(C.byref(h), int(device)), "hdg_init")
    return Context(h.value, device)


def hdg_mesh_create(ctx: Context, mesh, P, flag, params: Params) -> Mesh:
    """Create a device mesh from a ``workloads.HexMesh``-like object; P is one
    order or one per element."""
    ne = int(mesh.xyz_geom.shape[0])
    keep = dict(
        P=np.ascontiguousarray(np.broadcast_to(np.asarray(P, dtype=np.int32), (ne,))),
        xyz=np.ascontiguousarray(mesh.xyz_geom, dtype=np.float64),
        flag=np.ascontiguousarray(flag, dtype=np.uint8),
        nbr=np.ascontiguousarray(mesh.nbr, dtype=np.int32),
        nf=np.ascontiguousarray(mesh.nbr_face, dtype=np.int8),
        o=np.ascontiguousarray(mesh.orient, dtype=np.int8),
    )
    if keep["flag"].shape != (ne,):
        raise ValueError("flag must have one entry per element")
    d = MeshDesc()
    d.n_elem = ne
    d.P = keep["P"].ctypes.data_as(C.POINTER(C.c_int32))
    d.geom_order = int(mesh.Pg)
    d.xyz_geom = keep["xyz"].ctypes.data_as(C.POINTER(C.c_double))
    d.flag = keep["flag"].ctypes.data_as(C.POINTER(C.c_uint8))
    d.nbr = keep["nbr"].ctypes.data_as(C.POINTER(C.c_int32))
    d.nbr_face = keep["nf"].ctypes.data_as(C.POINTER(C.c_int8))
    d.orient = keep["o"].ctypes.data_as(C.POINTER(C.c_int8))
    h = C.c_void_p()
    _check(lib().hdg_mesh_create(ctx.handle, C.byref(d), C.byref(params), C.byref(h)), "hdg_mesh_create")
    return Mesh(ctx, h.value, ne, keep["P"])


def hdg_mesh_set_flags(mesh: Mesh, flag):
    f = np.ascontiguousarray(flag, dtype=np.uint8)
    if f.shape != (mesh.n_elem,):
        raise ValueError("flag must have one entry per element")
    _check(lib().hdg_mesh_set_flags(mesh.handle, f.ctypes.data_as(C.POINTER(C.c_uint8))), "hdg_mesh_set_flags")


def hdg_mesh_set_params(mesh: Mesh, params: Params):
    _check(lib().hdg_mesh_set_params(mesh.handle, C.byref(params)), "hdg_mesh_set_params")


def hdg_mesh_metric_blocks(mesh: Mesh) -> int:
    n = C.c_int64()
    _check(lib().hdg_mesh_metric_blocks(mesh.handle, C.byref(n)), "hdg_mesh_metric_blocks")
    return n.value


def hdg_mesh_info(mesh: Mesh) -> dict:
    a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
    v = C.c_int32()
    _check(lib().hdg_mesh_info(mesh.handle, C.byref(a), C.byref(b), C.byref(c), C.byref(v)), "hdg_mesh_info")
    return dict(n_nodes=a.value, state_len=b.value, device_bytes=c.value, n_viscous=v.value)


def hdg_mesh_node_coords(mesh: Mesh) -> np.ndarray:
    x = np.zeros((mesh.n_elem, 3, mesh.N3) if mesh.uniform else (3 * mesh.nodes,))
    _check(lib().hdg_mesh_node_coords(mesh.handle, x.ctypes.data_as(C.POINTER(C.c_double))), "node_coords")
    return x


def _geometry_desc(mesh, Pa):
    """A mesh description for the host-only geometry call; the arrays it
    points to are kept on the returned structure."""
    ne = int(mesh.xyz_geom.shape[0])
    keep = dict(P=Pa, xyz=np.ascontiguousarray(mesh.xyz_geom, dtype=np.float64),
                flag=np.zeros(ne, dtype=np.uint8), nbr=np.ascontiguousarray(mesh.nbr, dtype=np.int32),
                nf=np.ascontiguousarray(mesh.nbr_face, dtype=np.int8),
                o=np.ascontiguousarray(mesh.orient, dtype=np.int8))
    d = MeshDesc()
    d._keep = keep
    d.n_elem = ne
    d.P = keep["P"].ctypes.data_as(C.POINTER(C.c_int32))
    d.geom_order = int(mesh.Pg)
    d.xyz_geom = keep["xyz"].ctypes.data_as(C.POINTER(C.c_double))
    d.flag = keep["flag"].ctypes.data_as(C.POINTER(C.c_uint8))
    d.nbr = keep["nbr"].ctypes.data_as(C.POINTER(C.c_int32))
    d.nbr_face = keep["nf"].ctypes.data_as(C.POINTER(C.c_int8))
    d.orient = keep["o"].ctypes.data_as(C.POINTER(C.c_int8))
    return d


def hdg_mesh_geometry(mesh, P) -> dict:
    """Host-only geometry of a mesh description: node coordinates, J, Ja and the GLL rule.

    P is one order or one per element.  With several orders the arrays are
    flat, element after element (x: [3][N_e^3], J: [N_e^3], Ja: [3][3][N_e^3]
    each), and the GLL rule is not returned."""
    ne = int(mesh.xyz_geom.shape[0])
    Pa = np.ascontiguousarray(np.broadcast_to(np.asarray(P, dtype=np.int32), (ne,)))
    if ne and (Pa != Pa[0]).any():
        nodes = int(((Pa.astype(np.int64) + 1) ** 3).sum())
        out = dict(x=np.zeros(3 * nodes), J=np.zeros(nodes), Ja=np.zeros(9 * nodes))
        d = _geometry_desc(mesh, Pa)
        dp = C.POINTER(C.c_double)
        _check(lib().hdg_mesh_geometry(C.byref(d), *(out[k].ctypes.data_as(dp) for k in ("x", "J", "Ja")),
                                       None, None, None), "hdg_mesh_geometry")
        return out
    N = int(Pa[0]) + 1 if ne else int(np.max(P)) + 1
    N3 = N ** 3
    d = _geometry_desc(mesh, Pa)
    out = dict(x=np.zeros((ne, 3, N3)), J=np.zeros((ne, N3)), Ja=np.zeros((ne, 3, 3, N3)),
               xi=np.zeros(N), w=np.zeros(N), D=np.zeros((N, N)))
    dp = C.POINTER(C.c_double)
    _check(lib().hdg_mesh_geometry(C.byref(d), *(out[k].ctypes.data_as(dp) for k in ("x", "J", "Ja", "xi", "w", "D"))),
           "hdg_mesh_geometry")
    return out


def _check_state(mesh: Mesh, t, name: str, f32: bool = False):
    if isinstance(t, int):
        return
    import torch
    dt = torch.float32 if f32 else torch.float64
    if not t.is_cuda or t.dtype != dt or not t.is_contiguous() or t.numel() != 4 * mesh.nodes:
        raise ValueError(f"{name}: need a contiguous {dt} CUDA tensor of {4 * mesh.nodes} entries")


def hdg_residual(mesh: Mesh, q, r, prec: int = HDG_F64, stream=None):
    """R = dq/dt; q is always float64, r is float64 (HDG_F64) or float32 (HDG_F32)."""
    _check_state(mesh, q, "q")
    _check_state(mesh, r, "r", f32=(prec == HDG_F32))
    _check(lib().hdg_residual(mesh.handle, _ptr(q), _ptr(r), prec, _stream(stream)), "hdg_residual")


def hdg_rk3_steps(mesh: Mesh, q, dq, dt: float, nsteps: int, prec: int = HDG_F64, stream=None):
    _check_state(mesh, q, "q")
    _check_state(mesh, dq, "dq")
    _check(lib().hdg_rk3_steps(mesh.handle, _ptr(q), _ptr(dq), float(dt), int(nsteps), prec, _stream(stream)),
           "hdg_rk3_steps")


def hdg_reduce(mesh: Mesh, r, stream=None, allow_nonfinite: bool = False) -> dict:
    _check_state(mesh, r, "r")
    s, l2, mx = (C.c_double * 4)(), (C.c_double * 4)(), (C.c_double * 4)()
    st = lib().hdg_reduce(mesh.handle, _ptr(r), s, l2, mx, _stream(stream))
    out = dict(sum=np.array(s[:]), l2=np.array(l2[:]), max=np.array(mx[:]), finite=st != HDG_ENONFINITE)
    if not (allow_nonfinite and st == HDG_ENONFINITE):
        _check(st, "hdg_reduce")
    return out


def hdg_reduce_noalloc(mesh: Mesh, r, out, stream=None):
    """Allocation-free reductions into the device buffer ``out`` (13 doubles):
    sums [0:4], sums of squares [4:8], max [8:12], non-finite flag [12]."""
    import torch
    _check_state(mesh, r, "r")
    if out is None or out.dtype != torch.float64 or out.numel() < 13 or not out.is_cuda or not out.is_contiguous():
        raise HdgError(HDG_EINVAL, "hdg_reduce_noalloc: out must be a contiguous float64 device tensor of 13 values")
    _check(lib().hdg_reduce_noalloc(mesh.handle, _ptr(r), _ptr(out), _stream(stream)), "hdg_reduce_noalloc")


def hdg_max_wave_speed(mesh: Mesh, q, stream=None) -> float:
    """Largest |u| + sqrt(|u|^2 + c0^2) over the nodes of state q."""
    _check_state(mesh, q, "q")
    out = C.c_double()
    _check(lib().hdg_max_wave_speed(mesh.handle, _ptr(q), C.byref(out), _stream(stream)), "hdg_max_wave_speed")
    return out.value


def hdg_timing_enable(mesh: Mesh, enable: bool = True):
    _check(lib().hdg_timing_enable(mesh.handle, 1 if enable else 0), "hdg_timing_enable")


def hdg_timing_read(mesh: Mesh, kernel_class: int) -> tuple[float, int]:
    ms, n = C.c_double(), C.c_int64()
    _check(lib().hdg_timing_read(mesh.handle, kernel_class, C.byref(ms), C.byref(n)), "hdg_timing_read")
    return ms.value, n.value


def hdg_timing_samples(mesh: Mesh, kernel_class: int) -> list[float]:
    """Per-launch durations in microseconds, in launch order."""
    n = C.c_int64()
    _check(lib().hdg_timing_samples(mesh.handle, kernel_class, None, 0, C.byref(n)), "hdg_timing_samples")
    buf = (C.c_float * max(n.value, 1))()
    _check(lib().hdg_timing_samples(mesh.handle, kernel_class, buf, n.value, C.byref(n)), "hdg_timing_samples")
    return [float(buf[i]) for i in range(n.value)]


def hdg_mesh_autotune(mesh: Mesh, q, reps: int = 5, stream=None):
    _check_state(mesh, q, "q")
    _check(lib().hdg_mesh_autotune(mesh.handle, _ptr(q), int(reps), _stream(stream)), "hdg_mesh_autotune")


def hdg_mesh_get_launch(mesh: Mesh, kernel_class: int, prec: int, N: int) -> dict:
    c = LaunchCfg()
    _check(lib().hdg_mesh_get_launch(mesh.handle, kernel_class, prec, N, C.byref(c)), "hdg_mesh_get_launch")
    return dict(block=c.block, persistent=bool(c.persistent), us_per_launch=c.us_per_launch)


def hdg_mesh_set_launch(mesh: Mesh, kernel_class: int, prec: int, N: int, block: int, persistent: bool):
    c = LaunchCfg(int(block), 1 if persistent else 0, 0.0)
    _check(lib().hdg_mesh_set_launch(mesh.handle, kernel_class, prec, N, C.byref(c)), "hdg_mesh_set_launch")


def hdg_mesh_set_graphs(mesh: Mesh, enable: bool):
    _check(lib().hdg_mesh_set_graphs(mesh.handle, 1 if enable else 0), "hdg_mesh_set_graphs")


class Batch:
    """Owner of an ``hdg_batch`` handle; keeps its members (mesh and the torch
    tensors of their state and RK register) alive while they are in it."""

    def __init__(self, ctx: Context, max_members: int):
        h = C.c_void_p()
        _check(lib().hdg_batch_create(ctx.handle, int(max_members), C.byref(h)), "hdg_batch_create")
        self.handle = h
        self.ctx = ctx
        self.members = {}

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.hdg_batch_destroy(self.handle)
            self.handle = None


def hdg_batch_create(ctx: Context, max_members: int) -> Batch:
    return Batch(ctx, max_members)


def hdg_batch_add(batch: Batch, mesh: Mesh, q, dq, dt: float) -> int:
    _check_state(mesh, q, "q")
    _check_state(mesh, dq, "dq")
    slot = C.c_int32()
    _check(lib().hdg_batch_add(batch.handle, mesh.handle, _ptr(q), _ptr(dq), float(dt), C.byref(slot)),
           "hdg_batch_add")
    batch.members[slot.value] = (mesh, q, dq)
    return slot.value


def hdg_batch_remove(batch: Batch, slot: int):
    _check(lib().hdg_batch_remove(batch.handle, int(slot)), "hdg_batch_remove")
    batch.members.pop(slot, None)


def hdg_batch_info(batch: Batch) -> dict:
    nm, ne, nn = C.c_int32(), C.c_int64(), C.c_int64()
    _check(lib().hdg_batch_info(batch.handle, C.byref(nm), C.byref(ne), C.byref(nn)), "hdg_batch_info")
    return dict(n_members=nm.value, n_elements=ne.value, n_nodes=nn.value)


def hdg_batch_rk3_steps(batch: Batch, nsteps: int, prec: int = HDG_F64, stream=None):
    _check(lib().hdg_batch_rk3_steps(batch.handle, int(nsteps), prec, _stream(stream)), "hdg_batch_rk3_steps")


def hdg_batch_set_graphs(batch: Batch, enable: bool):
    _check(lib().hdg_batch_set_graphs(batch.handle, 1 if enable else 0), "hdg_batch_set_graphs")


def hdg_batch_autotune(batch: Batch, reps: int = 3, stream=None):
    _check(lib().hdg_batch_autotune(batch.handle, int(reps), _stream(stream)), "hdg_batch_autotune")


def hdg_batch_get_launch(batch: Batch, kernel_class: int, prec: int, N: int) -> dict:
    c = LaunchCfg()
    _check(lib().hdg_batch_get_launch(batch.handle, kernel_class, prec, N, C.byref(c)), "hdg_batch_get_launch")
    return dict(block=c.block, persistent=bool(c.persistent), us_per_launch=c.us_per_launch)


def _check_f64(t, n: int, name: str):
    import torch
    if not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous() or t.numel() != n:
        raise ValueError(f"{name}: need a contiguous float64 CUDA tensor of {n} entries")


def hdg_cluster_features(mesh: Mesh, q, features, stream=None):
    """Node features (Q_S, R_S, Q_Omega) of state q into the device array
    ``features`` of 3 * nodes doubles ([3][nodes])."""
    _check_state(mesh, q, "q")
    _check_f64(features, 3 * mesh.nodes, "features")
    _check(lib().hdg_cluster_features(mesh.handle, _ptr(q), _ptr(features), _stream(stream)), "hdg_cluster_features")


def hdg_cluster_fit(mesh: Mesh, features, iterations: int = 100, reg_covar: float = 1e-6, p_visc=None,
                    elem_pv=None, stream=None, tol: float = 0.0):
    """Gaussian mixture over the features and element regions; returns
    (result dict, flags as a uint8 array with one entry per element)."""
    _check_f64(features, 3 * mesh.nodes, "features")
    if p_visc is not None:
        _check_f64(p_visc, mesh.nodes, "p_visc")
    if elem_pv is not None:
        _check_f64(elem_pv, mesh.n_elem, "elem_pv")
    opts = GmmOpts(int(iterations), 0, float(reg_covar), float(tol))
    res = GmmResult()
    flags = np.zeros(mesh.n_elem, dtype=np.uint8)
    _check(lib().hdg_cluster_fit(mesh.handle, _ptr(features), C.byref(opts), C.byref(res),
                                 _ptr(p_visc) if p_visc is not None else None,
                                 _ptr(elem_pv) if elem_pv is not None else None,
                                 flags.ctypes.data_as(C.POINTER(C.c_uint8)), _stream(stream)), "hdg_cluster_fit")
    out = dict(feat_mean=np.array(res.feat_mean[:]), feat_std=np.array(res.feat_std[:]),
               weight=np.array(res.weight[:]), mean=np.array([list(r) for r in res.mean]),
               cov=np.array([[list(r) for r in c] for c in res.cov]), log_likelihood=res.log_likelihood,
               iterations=res.iterations, degenerate=bool(res.degenerate), converged=bool(res.converged),
               n_viscous=res.n_viscous)
    return out, flags


def hdg_stream_copy(ctx: Context, dst, src, nbytes: int, stream=None):
    _check(lib().hdg_stream_copy(ctx.handle, _ptr(dst), _ptr(src), int(nbytes), _stream(stream)), "hdg_stream_copy")
