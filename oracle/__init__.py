"""ctypes loader for the FP64 CPU oracle (``hdg_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
benchmark's CPU-baseline leg.  The product package never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hdg_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def needs_build() -> bool:
    return not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc (always recompiles)."""
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-fPIC", "-shared",
           "-Wall", "-Wno-unused-function", "-o", tmp, _SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


class Params(C.Structure):
    _fields_ = [("c0sq", C.c_double), ("nu", C.c_double), ("les_model", C.c_int),
                ("C_les", C.c_double), ("mixed_face", C.c_int), ("q_inf", C.c_double * 4),
                ("riemann", C.c_int)]


def make_params(c0sq=25.0, nu=1e-3, les_model=1, C_les=0.1, mixed_face=0, q_inf=(0, 0, 0, 0), riemann=0):
    p = Params()
    p.c0sq, p.nu, p.les_model, p.C_les, p.mixed_face = c0sq, nu, les_model, C_les, mixed_face
    p.riemann = riemann
    for k in range(4):
        p.q_inf[k] = float(q_inf[k])
    return p


def lib():
    global _lib
    if _lib is None:
        if needs_build():
            build()
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        L.orc_lgl.argtypes = [C.c_int, dp, dp, dp]
        L.orc_mesh_new.restype = C.c_void_p
        L.orc_mesh_new.argtypes = [C.c_int, C.c_int, C.c_int, dp, C.POINTER(C.c_int),
                                   C.POINTER(C.c_byte), C.POINTER(C.c_byte), C.POINTER(C.c_ubyte)]
        L.orc_mesh_new_mixed.restype = C.c_void_p
        L.orc_mesh_new_mixed.argtypes = [C.c_int, C.POINTER(C.c_int), C.c_int, dp, C.POINTER(C.c_int),
                                         C.POINTER(C.c_byte), C.POINTER(C.c_byte), C.POINTER(C.c_ubyte)]
        L.orc_mesh_nodes.restype = C.c_size_t
        L.orc_mesh_nodes.argtypes = [C.c_void_p]
        L.orc_mesh_free.argtypes = [C.c_void_p]
        L.orc_last_error.restype = C.c_char_p
        L.orc_set_flags.argtypes = [C.c_void_p, C.POINTER(C.c_ubyte)]
        L.orc_node_coords.argtypes = [C.c_void_p, dp]
        L.orc_metrics.argtypes = [C.c_void_p, dp, dp]
        L.orc_filter_width.restype = C.c_double
        L.orc_filter_width.argtypes = [C.c_void_p, C.c_int]
        L.orc_roe_flux.argtypes = [C.c_double, dp, dp, dp, dp]
        L.orc_rusanov_flux.argtypes = [C.c_double, dp, dp, dp, dp]
        L.orc_les_nut.restype = C.c_double
        L.orc_les_nut.argtypes = [C.c_int, C.c_double, C.c_double, dp]
        L.orc_gradient.argtypes = [C.c_void_p, C.POINTER(Params), dp, dp]
        L.orc_residual.argtypes = [C.c_void_p, C.POINTER(Params), dp, dp]
        L.orc_rk3_steps.argtypes = [C.c_void_p, C.POINTER(Params), dp, C.c_double, C.c_int]
        L.orc_rk3_linear.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int, dp, dp]
        L.orc_rk3_riccati.restype = C.c_double
        L.orc_rk3_riccati.argtypes = [C.c_double, C.c_double, C.c_int]
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_get_threads.restype = C.c_int
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def lgl(P: int):
    N = P + 1
    xi, w, D = np.zeros(N), np.zeros(N), np.zeros((N, N))
    lib().orc_lgl(P, _dp(xi), _dp(w), _dp(D))
    return xi, w, D


def roe_flux(c0sq, qL, qR, n):
    qL = np.ascontiguousarray(qL, dtype=np.float64)
    qR = np.ascontiguousarray(qR, dtype=np.float64)
    n = np.ascontiguousarray(n, dtype=np.float64)
    F = np.zeros(4)
    lib().orc_roe_flux(c0sq, _dp(qL), _dp(qR), _dp(n), _dp(F))
    return F


def rusanov_flux(c0sq, qL, qR, n):
    qL = np.ascontiguousarray(qL, dtype=np.float64)
    qR = np.ascontiguousarray(qR, dtype=np.float64)
    n = np.ascontiguousarray(n, dtype=np.float64)
    F = np.zeros(4)
    lib().orc_rusanov_flux(c0sq, _dp(qL), _dp(qR), _dp(n), _dp(F))
    return F


def les_nut(model, C_les, delta, G):
    G = np.ascontiguousarray(G, dtype=np.float64).reshape(9)
    return lib().orc_les_nut(model, C_les, delta, _dp(G))


def rk3_linear(lam: complex, dt: float, nsteps: int, y0: complex = 1.0) -> complex:
    yr, yi = C.c_double(complex(y0).real), C.c_double(complex(y0).imag)
    lib().orc_rk3_linear(lam.real, lam.imag, dt, nsteps, C.byref(yr), C.byref(yi))
    return complex(yr.value, yi.value)


def rk3_riccati(y0, dt, nsteps):
    return lib().orc_rk3_riccati(y0, dt, nsteps)


def max_wave_speed(q: np.ndarray, c0sq: float) -> float:
    """Largest wave speed over the nodes of a state q given as (nodes, 4)
    rows p, u, v, w.  The artificial-compressibility flux along a unit normal
    n, F_n(q) = [c0^2 u.n ; u (u.n) + p n], has the Jacobian eigenvalues u.n
    and u.n +- sqrt((u.n)^2 + c0^2) (Sec. 2.3 time step; the system of App. B
    in the artificial-compressibility reading), whose largest magnitude over
    all n is |u| + sqrt(|u|^2 + c0^2), reached at n parallel to u."""
    u = np.asarray(q, dtype=np.float64)[:, 1:4]
    a = np.sqrt((u * u).sum(axis=1))
    return float(np.max(a + np.sqrt(a * a + c0sq)))


def set_threads(n: int):
    lib().orc_set_threads(int(n))


def get_threads() -> int:
    return int(lib().orc_get_threads())


class OracleMesh:
    """An oracle-side mesh: geometry, metrics and connectivity in FP64 host memory.

    ``P`` is one order for every element, or one per element.  With one order,
    arrays have shape (n_elem, fields, N^3); with several, they are flat,
    element after element ([fields][N_e^3] each), and ``offsets`` gives each
    element's first node."""

    def __init__(self, mesh, P, flag):
        Ps = np.broadcast_to(np.asarray(P, dtype=np.int32), (mesh.n_elem,)).copy()
        self.Ps = Ps
        self.uniform = bool(np.all(Ps == Ps[0]))
        self.P = int(Ps[0]) if self.uniform else None
        self.N = self.P + 1 if self.uniform else None
        self.N3 = self.N ** 3 if self.uniform else None
        self.n_elem = mesh.n_elem
        n3 = (Ps.astype(np.int64) + 1) ** 3
        self.offsets = np.concatenate([[0], np.cumsum(n3)[:-1]])
        self.nodes = int(n3.sum())
        self._keep = (
            np.ascontiguousarray(mesh.xyz_geom, dtype=np.float64),
            np.ascontiguousarray(mesh.nbr, dtype=np.int32),
            np.ascontiguousarray(mesh.nbr_face, dtype=np.int8),
            np.ascontiguousarray(mesh.orient, dtype=np.int8),
            np.ascontiguousarray(flag, dtype=np.uint8),
            Ps,
        )
        x, nb, nf, o, fl, pp = self._keep
        h = lib().orc_mesh_new_mixed(mesh.n_elem, pp.ctypes.data_as(C.POINTER(C.c_int)), mesh.Pg, _dp(x),
                                     nb.ctypes.data_as(C.POINTER(C.c_int)), nf.ctypes.data_as(C.POINTER(C.c_byte)),
                                     o.ctypes.data_as(C.POINTER(C.c_byte)), fl.ctypes.data_as(C.POINTER(C.c_ubyte)))
        if not h:
            raise ValueError("oracle mesh rejected: " + lib().orc_last_error().decode())
        self._h = h
        self.flag = fl
        assert lib().orc_mesh_nodes(h) == self.nodes

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_mesh_free(h)
            self._h = None

    def set_flags(self, flag):
        fl = np.ascontiguousarray(flag, dtype=np.uint8).copy()
        lib().orc_set_flags(self._h, fl.ctypes.data_as(C.POINTER(C.c_ubyte)))
        self.flag = fl

    def _shape(self, fields):
        return (self.n_elem, fields, self.N3) if self.uniform else (fields * self.nodes,)

    def element(self, arr, e, fields):
        """Element e's block [fields][N_e^3] of a flat (or uniform) array."""
        if self.uniform:
            return arr[e]
        n3 = (int(self.Ps[e]) + 1) ** 3
        o = fields * int(self.offsets[e])
        return arr[o:o + fields * n3].reshape(fields, n3)

    def node_coords(self):
        x = np.zeros(self._shape(3))
        lib().orc_node_coords(self._h, _dp(x))
        return x

    def metrics(self):
        J = np.zeros(self._shape(1)) if not self.uniform else np.zeros((self.n_elem, self.N3))
        Ja = np.zeros((self.n_elem, 3, 3, self.N3)) if self.uniform else np.zeros(9 * self.nodes)
        lib().orc_metrics(self._h, _dp(J), _dp(Ja))
        return J, Ja

    def filter_width(self, e: int) -> float:
        return lib().orc_filter_width(self._h, e)

    def _chk(self, q):
        q = np.ascontiguousarray(q, dtype=np.float64)
        if q.shape != self._shape(4):
            raise ValueError(f"state shape {q.shape} != {self._shape(4)}")
        return q

    def gradient(self, params: Params, q):
        q = self._chk(q)
        G = np.zeros((self.n_elem, 3, 3, self.N3)) if self.uniform else np.zeros(9 * self.nodes)
        lib().orc_gradient(self._h, C.byref(params), _dp(q), _dp(G))
        return G

    def residual(self, params: Params, q):
        q = self._chk(q)
        R = np.zeros_like(q)
        lib().orc_residual(self._h, C.byref(params), _dp(q), _dp(R))
        return R

    def rk3(self, params: Params, q, dt: float, nsteps: int):
        q = self._chk(q).copy()
        lib().orc_rk3_steps(self._h, C.byref(params), _dp(q), dt, nsteps)
        return q
