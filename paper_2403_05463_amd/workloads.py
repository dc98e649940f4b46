"""Seeded synthetic inputs shared by the GPU path, the oracle and the benchmark.

This module only builds *data*: hexahedral meshes (geometry control points,
corner topology, face connectivity and orientation codes), equation masks and
initial states.  It holds none of the discretisation's arithmetic (no
quadrature rule, derivative matrix, metric term or flux).  Node coordinates,
where an initial state needs them, are passed in by the caller.

Geometry convention (same as ``include/hdg.h``): every element carries
``(Pg+1)^3`` control points at equispaced reference positions
``-1 + 2k/Pg`` per direction, x-index fastest, stored ``[e][3][(Pg+1)^3]``.
Local faces: 0 xi-, 1 xi+, 2 eta-, 3 eta+, 4 zeta-, 5 zeta+.  Face-local
coordinates ``(a, b)``: (eta, zeta) on faces 0/1, (xi, zeta) on 2/3 and
(xi, eta) on 4/5.  An orientation code ``o`` maps my face coordinates to the
neighbour's: ``(s, t) = (b, a) if o & 1 else (a, b)``; ``a' = M - s if o & 2``
and ``b' = M - t if o & 4`` (``M`` = nodes per edge minus one).

The workloads mirror the paper's cases: an airfoil section at high angle of
attack (Sec. 3.1, NACA0012 at 10-20 degrees) with viscous elements near the
wall and in the wake (Sec. 2.1), and periodic boxes for Taylor-Green decay.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

WALL = -1
FARFIELD = -2

# corner (ci, cj, ck) -> local corner index ci + 2 cj + 4 ck
_FACE_CORNERS = []
for _f in range(6):
    _d, _side = divmod(_f, 2)
    _cs = []
    for _b in range(2):
        for _a in range(2):
            if _d == 0:
                ijk = (_side, _a, _b)
            elif _d == 1:
                ijk = (_a, _side, _b)
            else:
                ijk = (_a, _b, _side)
            _cs.append(ijk[0] + 2 * ijk[1] + 4 * ijk[2])
    _FACE_CORNERS.append(_cs)  # order: (a,b) = (0,0),(1,0),(0,1),(1,1)


def orient_map(o: int, a: int, b: int, M: int) -> tuple[int, int]:
    """Apply orientation code ``o`` to face coordinates (a, b) on an edge of M+1 nodes."""
    s, t = (b, a) if (o & 1) else (a, b)
    if o & 2:
        s = M - s
    if o & 4:
        t = M - t
    return s, t


@dataclass
class HexMesh:
    """A conforming hexahedral mesh as plain arrays (the boundary's mesh description)."""

    Pg: int
    xyz_geom: np.ndarray            # (n_elem, 3, (Pg+1)^3) float64
    corners: np.ndarray             # (n_elem, 8) int64 global vertex ids
    nbr: np.ndarray                 # (n_elem, 6) int32, >=0 element, WALL, FARFIELD
    nbr_face: np.ndarray            # (n_elem, 6) int8
    orient: np.ndarray              # (n_elem, 6) int8
    centroid: np.ndarray            # (n_elem, 3) float64 (element-centre control point)
    name: str = "mesh"
    extra: dict = field(default_factory=dict)

    @property
    def n_elem(self) -> int:
        return int(self.xyz_geom.shape[0])


def connectivity(corners: np.ndarray, boundary_type) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Face-to-face connectivity of a conforming hex mesh from its corner vertex ids.

    ``boundary_type(e, f)`` returns WALL or FARFIELD for faces that have no
    partner.  Returns (nbr, nbr_face, orient) arrays of shape (n_elem, 6).
    """
    ne = corners.shape[0]
    nbr = np.full((ne, 6), 0, dtype=np.int32)
    nbr_face = np.zeros((ne, 6), dtype=np.int8)
    orient = np.zeros((ne, 6), dtype=np.int8)
    fc = np.asarray(_FACE_CORNERS)                      # (6, 4)
    face_ids = corners[:, fc]                           # (ne, 6, 4)
    keys = np.sort(face_ids, axis=2)
    flat = keys.reshape(-1, 4)
    order = np.lexsort(flat.T[::-1])
    sk = flat[order]
    same = np.all(sk[1:] == sk[:-1], axis=1)
    if np.any(same[:-1] & same[1:]):
        raise ValueError("non-manifold face shared by more than two elements")
    # faces with equal corner sets come in adjacent pairs of the sorted order
    start = np.nonzero(same)[0]
    g0, g1 = order[start], order[start + 1]
    paired = np.zeros(flat.shape[0], dtype=bool)
    paired[g0] = paired[g1] = True
    # corner k = a + 2 b of a face maps to corner s + 2 t of the other side's
    # face under orientation code o
    omap = np.array([[orient_map(o, k % 2, k // 2, 1)[0] + 2 * orient_map(o, k % 2, k // 2, 1)[1]
                      for k in range(4)] for o in range(8)])
    flat_ids = face_ids.reshape(-1, 4)
    for ga, gb in ((g0, g1), (g1, g0)):
        ca, cb = flat_ids[ga], flat_ids[gb]
        ok = np.stack([np.all(ca == cb[:, omap[o]], axis=1) for o in range(8)], axis=1)
        if not np.all(ok.any(axis=1)):
            raise ValueError("matching face corners admit no orientation code")
        code = np.argmax(ok, axis=1)                    # the first code that matches
        ea, fa = np.divmod(ga, 6)
        eb, fb = np.divmod(gb, 6)
        nbr[ea, fa] = eb
        nbr_face[ea, fa] = fb
        orient[ea, fa] = code
    for g in np.nonzero(~paired)[0]:
        e, f = divmod(int(g), 6)
        nbr[e, f] = boundary_type(e, f)
        nbr_face[e, f] = -1
        orient[e, f] = 0
    return nbr, nbr_face, orient


def _element_control_points(gx, gy, gz, ei, ej, ek, Pg):
    """Gather (Pg+1)^3 control points of element (ei, ej, ek) from global control grids."""
    r = np.arange(Pg + 1)
    I = (ei[:, None] * Pg + r[None, :])
    J = (ej[:, None] * Pg + r[None, :])
    K = (ek[:, None] * Pg + r[None, :])
    # index grid (e, k, j, i) -> x fastest
    II = I[:, None, None, :]
    JJ = J[:, None, :, None]
    KK = K[:, :, None, None]
    X = gx(II, JJ, KK)
    Y = gy(II, JJ, KK)
    Z = gz(II, JJ, KK)
    ne = ei.shape[0]
    P3 = (Pg + 1) ** 3
    out = np.empty((ne, 3, P3))
    out[:, 0] = np.broadcast_to(X, (ne, Pg + 1, Pg + 1, Pg + 1)).reshape(ne, P3)
    out[:, 1] = np.broadcast_to(Y, (ne, Pg + 1, Pg + 1, Pg + 1)).reshape(ne, P3)
    out[:, 2] = np.broadcast_to(Z, (ne, Pg + 1, Pg + 1, Pg + 1)).reshape(ne, P3)
    return out


def periodic_box(n: int, L: float = 2 * math.pi, Pg: int = 1, curve_amp: float = 0.0,
                 n_xyz: tuple[int, int, int] | None = None) -> HexMesh:
    """Triply periodic box [0, L]^3 of n^3 hexahedra (or nx*ny*nz).

    With ``curve_amp > 0`` the interior control points are displaced by a
    smooth L-periodic field, giving curved elements of geometry order Pg.
    Element order: x index fastest, then y, then z.
    """
    nx, ny, nz = n_xyz if n_xyz is not None else (n, n, n)
    if min(nx, ny, nz) < 3:
        # with two elements a face's corner ids no longer identify it uniquely
        raise ValueError("periodic directions need at least three elements")
    hx, hy, hz = L / (nx * Pg), L / (ny * Pg), L / (nz * Pg)
    k = 2 * math.pi / L

    def base(I, J, K):
        return I * hx, J * hy, K * hz

    def gx(I, J, K):
        X, Y, Z = base(I, J, K)
        return X + curve_amp * np.sin(k * Y) * np.sin(k * Z)

    def gy(I, J, K):
        X, Y, Z = base(I, J, K)
        return Y + curve_amp * np.sin(k * X) * np.sin(k * Z)

    def gz(I, J, K):
        X, Y, Z = base(I, J, K)
        return Z + curve_amp * np.sin(k * X) * np.sin(k * Y)

    e = np.arange(nx * ny * nz)
    ei, ej, ek = e % nx, (e // nx) % ny, e // (nx * ny)
    xyz = _element_control_points(gx, gy, gz, ei, ej, ek, Pg)
    corners = np.empty((e.size, 8), dtype=np.int64)
    for c in range(8):
        ci, cj, ck = c & 1, (c >> 1) & 1, (c >> 2) & 1
        corners[:, c] = ((ei + ci) % nx) + nx * (((ej + cj) % ny) + ny * ((ek + ck) % nz))
    nbr, nbr_face, orient = connectivity(corners, lambda e_, f_: (_ for _ in ()).throw(
        ValueError("periodic box has no boundary faces")))
    mid = (Pg + 1) ** 3 // 2 if Pg % 2 == 0 else None
    if mid is not None:
        cen = xyz[:, :, mid].copy()
    else:
        cen = xyz.mean(axis=2)
    return HexMesh(Pg=Pg, xyz_geom=xyz, corners=corners, nbr=nbr, nbr_face=nbr_face,
                   orient=orient, centroid=cen, name=f"box{nx}x{ny}x{nz}_Pg{Pg}",
                   extra={"L": L, "n_xyz": (nx, ny, nz)})


def box(n_xyz: tuple[int, int, int], lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0),
        Pg: int = 1, boundary: int = FARFIELD, skew: float = 0.0,
        periodic: tuple[bool, bool, bool] = (False, False, False)) -> HexMesh:
    """Box of affine hexahedra; outer faces of non-periodic directions get the
    given boundary type.

    ``skew`` shears x by ``skew * y`` so the elements are parallelepipeds.
    """
    nx, ny, nz = n_xyz
    h = [(hi[d] - lo[d]) / (n_xyz[d] * Pg) for d in range(3)]

    def gx(I, J, K):
        return lo[0] + I * h[0] + skew * (lo[1] + J * h[1])

    def gy(I, J, K):
        return lo[1] + J * h[1] + 0 * I + 0 * K

    def gz(I, J, K):
        return lo[2] + K * h[2] + 0 * I + 0 * J

    e = np.arange(nx * ny * nz)
    ei, ej, ek = e % nx, (e // nx) % ny, e // (nx * ny)
    xyz = _element_control_points(gx, gy, gz, ei, ej, ek, Pg)
    for d, per in enumerate(periodic):
        if per and n_xyz[d] < 3:
            raise ValueError("periodic directions need at least three elements")
    vx, vy, vz = [n_xyz[d] if periodic[d] else n_xyz[d] + 1 for d in range(3)]
    corners = np.empty((e.size, 8), dtype=np.int64)
    for c in range(8):
        ci, cj, ck = c & 1, (c >> 1) & 1, (c >> 2) & 1
        corners[:, c] = ((ei + ci) % vx) + vx * (((ej + cj) % vy) + vy * ((ek + ck) % vz))
    nbr, nbr_face, orient = connectivity(corners, lambda e_, f_: boundary)
    return HexMesh(Pg=Pg, xyz_geom=xyz, corners=corners, nbr=nbr, nbr_face=nbr_face,
                   orient=orient, centroid=xyz.mean(axis=2), name=f"box{nx}x{ny}x{nz}")


# ---------------------------------------------------------------------------
# Element re-orientation (test of orientation handling)
# ---------------------------------------------------------------------------

def _cube_rotations():
    """The 24 orientation-preserving symmetries of the cube as (perm, flips)."""
    import itertools
    out = []
    for perm in itertools.permutations(range(3)):
        sgn = 1
        p = list(perm)
        for i in range(3):
            for j in range(i + 1, 3):
                if p[i] > p[j]:
                    sgn = -sgn
        for flips in itertools.product((0, 1), repeat=3):
            det = sgn * (-1) ** sum(flips)
            if det == 1:
                out.append((perm, flips))
    return out


def index_map(perm, flips, M: int) -> np.ndarray:
    """new linear index of each old node for a lattice of (M+1)^3 nodes, x fastest."""
    n1 = M + 1
    old = np.arange(n1 ** 3)
    oi = np.stack([old % n1, (old // n1) % n1, old // (n1 * n1)])
    new = np.empty_like(oi)
    for d in range(3):
        v = oi[perm[d]]
        new[d] = M - v if flips[d] else v
    return new[0] + n1 * new[1] + n1 * n1 * new[2]


def reorient(mesh: HexMesh, seed: int) -> tuple[HexMesh, list]:
    """Give every element a random local frame (one of the 24 cube rotations).

    Returns the new mesh and the per-element (perm, flips) so callers can map
    nodal arrays: ``new[e][index_map(perm, flips, M)] = old[e][:]``.
    """
    rng = np.random.default_rng(seed)
    rots = _cube_rotations()
    choice = rng.integers(0, len(rots), size=mesh.n_elem)
    Pg = mesh.Pg
    xyz = np.empty_like(mesh.xyz_geom)
    corners = np.empty_like(mesh.corners)
    frames = []
    # recover boundary types from the old mesh by corner key
    old_keys = {}
    fc = np.asarray(_FACE_CORNERS)
    for e in range(mesh.n_elem):
        for f in range(6):
            if mesh.nbr[e, f] < 0:
                old_keys[tuple(sorted(mesh.corners[e, fc[f]]))] = int(mesh.nbr[e, f])
    for e in range(mesh.n_elem):
        perm, flips = rots[choice[e]]
        frames.append((perm, flips))
        mg = index_map(perm, flips, Pg)
        xyz[e][:, mg] = mesh.xyz_geom[e]
        mc = index_map(perm, flips, 1)
        corners[e][mc] = mesh.corners[e]

    def btype(e, f):
        return old_keys[tuple(sorted(corners[e, fc[f]]))]

    nbr, nbr_face, orient = connectivity(corners, btype)
    new = HexMesh(Pg=Pg, xyz_geom=xyz, corners=corners, nbr=nbr, nbr_face=nbr_face,
                  orient=orient, centroid=mesh.centroid.copy(), name=mesh.name + "_reoriented",
                  extra=dict(mesh.extra))
    return new, frames


# ---------------------------------------------------------------------------
# NACA0012 O-grid
# ---------------------------------------------------------------------------

def naca_thickness(x, t=0.12):
    """NACA 4-digit half thickness with the closed-trailing-edge last coefficient."""
    return 5.0 * t * (0.2969 * np.sqrt(np.maximum(x, 0.0)) - 0.1260 * x - 0.3516 * x ** 2
                      + 0.2843 * x ** 3 - 0.1036 * x ** 4)


def naca_ogrid(ni: int = 96, nj: int = 48, nk: int = 8, Pg: int = 2, radius: float = 20.0,
               growth: float = 1.128, span: float = 1.0, t: float = 0.12, growth_layers: int = 48) -> HexMesh:
    """Extruded O-grid around a NACA 00xx section (chord 1, leading edge at the origin).

    Around-index i runs trailing edge -> lower surface -> leading edge -> upper
    surface (periodic); j runs from the wall (faces eta-, WALL) to a circle of
    ``radius`` about mid-chord (faces eta+, FARFIELD) with geometric growth;
    k is the periodic span of length ``span``.  The radial map is fixed (growth
    per layer of a ``growth_layers``-layer grid), so more radial elements
    refine the same grid.  Each element is the degree-Pg Lagrange interpolant
    of the analytic map.
    """
    S = ni * Pg           # control points around (periodic)
    R = nj * Pg + 1       # radial
    Kz = nk * Pg + 1      # span (first and last identified by periodicity)

    s = np.arange(S) / S
    # sigma: 0 at the trailing edge, 1 at the leading edge on either surface;
    # x = (1 - sigma)^2 (1 + sigma) clusters points at the leading edge and
    # keeps a finite wall speed at the (sharp) trailing edge.
    sig = np.where(s <= 0.5, 2 * s, 2 * (1 - s))
    xw = (1 - sig) ** 2 * (1 + sig)
    yw = naca_thickness(xw, t) * np.where(s < 0.5, -1.0, 1.0)
    yw[0] = 0.0
    th = -2 * np.pi * s
    xo = 0.5 + radius * np.cos(th)
    yo = radius * np.sin(th)
    r = np.arange(R) / (nj * Pg)
    fr = (growth ** (growth_layers * r) - 1.0) / (growth ** growth_layers - 1.0)
    Xg = (1 - fr[None, :]) * xw[:, None] + fr[None, :] * xo[:, None]   # (S, R)
    Yg = (1 - fr[None, :]) * yw[:, None] + fr[None, :] * yo[:, None]
    zg = span * np.arange(Kz) / (nk * Pg)

    def gx(I, J, K):
        return Xg[I % S, J] + 0.0 * K

    def gy(I, J, K):
        return Yg[I % S, J] + 0.0 * K

    def gz(I, J, K):
        return zg[K] + 0.0 * I + 0.0 * J

    e = np.arange(ni * nj * nk)
    ei, ej, ek = e % ni, (e // ni) % nj, e // (ni * nj)
    xyz = _element_control_points(gx, gy, gz, ei, ej, ek, Pg)
    corners = np.empty((e.size, 8), dtype=np.int64)
    for c in range(8):
        ci, cj, ck = c & 1, (c >> 1) & 1, (c >> 2) & 1
        corners[:, c] = ((ei + ci) % ni) + ni * ((ej + cj) + (nj + 1) * ((ek + ck) % nk))

    def btype(e_, f_):
        if f_ == 2:
            return WALL
        if f_ == 3:
            return FARFIELD
        raise ValueError("unexpected boundary face in O-grid")

    nbr, nbr_face, orient = connectivity(corners, btype)
    mid = ((Pg + 1) ** 3) // 2 if Pg % 2 == 0 else None
    cen = xyz[:, :, mid].copy() if mid is not None else xyz.mean(axis=2)
    wall = np.stack([xw, yw], axis=1)
    return HexMesh(Pg=Pg, xyz_geom=xyz, corners=corners, nbr=nbr, nbr_face=nbr_face,
                   orient=orient, centroid=cen, name=f"naca0012_ogrid_{ni}x{nj}x{nk}_Pg{Pg}",
                   extra={"wall": wall, "ni": ni, "nj": nj, "nk": nk})


def naca_mask(mesh: HexMesh, alpha_deg: float = 20.0, wall_dist: float = 0.2,
              wedge_full_deg: float = 15.0) -> np.ndarray:
    """Viscous flag: element centre within ``wall_dist`` chords of the wall, or inside
    a wake wedge with apex at the trailing edge, axis along the free stream and the
    given full opening angle.  Stands in for the clustering's element region ID."""
    wall = mesh.extra["wall"]
    c = mesh.centroid[:, :2]
    dmin = np.full(c.shape[0], np.inf)
    # dense wall sampling between stored points
    wx = np.concatenate([wall[:, 0], wall[:1, 0]])
    wy = np.concatenate([wall[:, 1], wall[:1, 1]])
    fine = np.linspace(0, 1, 8, endpoint=False)
    sx = (wx[:-1, None] * (1 - fine) + wx[1:, None] * fine).ravel()
    sy = (wy[:-1, None] * (1 - fine) + wy[1:, None] * fine).ravel()
    for lo in range(0, c.shape[0], 4096):
        cc = c[lo:lo + 4096]
        d2 = (cc[:, 0:1] - sx[None, :]) ** 2 + (cc[:, 1:2] - sy[None, :]) ** 2
        dmin[lo:lo + 4096] = np.sqrt(d2.min(axis=1))
    a = math.radians(alpha_deg)
    ax = np.array([math.cos(a), math.sin(a)])
    rel = c - np.array([1.0, 0.0])
    rn = np.linalg.norm(rel, axis=1)
    cosang = (rel @ ax) / np.maximum(rn, 1e-300)
    in_wedge = (rn > 0) & (cosang >= math.cos(math.radians(wedge_full_deg / 2)))
    return ((dmin < wall_dist) | in_wedge).astype(np.uint8)


def bernoulli_mask(n_elem: int, p: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return (rng.random(n_elem) < p).astype(np.uint8)


def mixed_orders(flag: np.ndarray, seed: int, orders=(2, 3, 4, 5, 6),
                 w_viscous=(0.0, 0.1, 0.2, 0.3, 0.4), w_euler=(0.4, 0.3, 0.2, 0.1, 0.0)) -> np.ndarray:
    """Seeded per-element polynomial order: viscous elements draw from
    `w_viscous`, Euler elements from `w_euler` (higher orders where the
    viscous/turbulent region is, as the paper's P-adaptation cases do)."""
    rng = np.random.default_rng(seed)
    orders = np.asarray(orders)
    pv = np.asarray(w_viscous, dtype=float) / np.sum(w_viscous)
    pe = np.asarray(w_euler, dtype=float) / np.sum(w_euler)
    P = np.where(np.asarray(flag) != 0, rng.choice(orders, size=len(flag), p=pv),
                 rng.choice(orders, size=len(flag), p=pe))
    return P.astype(np.int32)


def flat_offsets(P: np.ndarray) -> np.ndarray:
    """First node of each element in element-after-element layouts."""
    n3 = (np.asarray(P, dtype=np.int64) + 1) ** 3
    return np.concatenate([[0], np.cumsum(n3)[:-1]])


# ---------------------------------------------------------------------------
# Initial states, layout [e][4][N^3] with fields (p, u, v, w)
# ---------------------------------------------------------------------------

def taylor_green_state(node_xyz: np.ndarray, amp: float, seed: int) -> np.ndarray:
    """Taylor-Green vortex at the given nodes plus i.i.d. U[-amp, amp] velocity noise.

    ``node_xyz`` has shape (n_elem, 3, N^3).
    """
    x, y, z = node_xyz[:, 0], node_xyz[:, 1], node_xyz[:, 2]
    q = np.empty((node_xyz.shape[0], 4, node_xyz.shape[2]))
    q[:, 0] = (np.cos(2 * x) + np.cos(2 * y)) * (np.cos(2 * z) + 2.0) / 16.0
    q[:, 1] = np.sin(x) * np.cos(y) * np.cos(z)
    q[:, 2] = -np.cos(x) * np.sin(y) * np.cos(z)
    q[:, 3] = 0.0
    if amp > 0:
        rng = np.random.default_rng(seed)
        q[:, 1:4] += rng.uniform(-amp, amp, size=q[:, 1:4].shape)
    return q


def uniform_inflow_state(n_elem: int, N3: int, alpha_deg: float, u_inf: float,
                         noise: float, seed: int) -> np.ndarray:
    """Uniform stream at angle ``alpha_deg`` in the x-y plane, p = 0, plus i.i.d.
    U[-noise*u_inf, noise*u_inf] velocity noise."""
    a = math.radians(alpha_deg)
    q = np.zeros((n_elem, 4, N3))
    q[:, 1] = u_inf * math.cos(a)
    q[:, 2] = u_inf * math.sin(a)
    if noise > 0:
        rng = np.random.default_rng(seed)
        q[:, 1:4] += rng.uniform(-noise * u_inf, noise * u_inf, size=q[:, 1:4].shape)
    return q


def uniform_inflow_state_flat(P: np.ndarray, alpha_deg: float, u_inf: float, noise: float,
                              seed: int) -> np.ndarray:
    """The same stream for per-element orders: element after element, [4][N_e^3]
    each, noise drawn for all velocity entries in that order."""
    a = math.radians(alpha_deg)
    n3 = (np.asarray(P, dtype=np.int64) + 1) ** 3
    q = np.zeros(4 * int(n3.sum()))
    off = 4 * np.concatenate([[0], np.cumsum(n3)[:-1]])
    rng = np.random.default_rng(seed)
    for e, (o, n) in enumerate(zip(off, n3)):
        q[o + n:o + 2 * n] = u_inf * math.cos(a)
        q[o + 2 * n:o + 3 * n] = u_inf * math.sin(a)
    if noise > 0:
        vel = np.concatenate([np.arange(o + n, o + 4 * n) for o, n in zip(off, n3)])
        q[vel] += rng.uniform(-noise * u_inf, noise * u_inf, size=vel.size)
    return q


def developed_airfoil_state(X: np.ndarray, alpha_deg: float = 20.0, u_inf: float = 1.0, t: float = 0.12,
                            delta: float = 0.02, wake: float = 0.5, w0: float = 0.05, spread: float = 0.1,
                            span: float = 1.0) -> np.ndarray:
    """Analytic stand-in for a developed flow around the NACA section (chord
    1, leading edge at the origin), to be clustered: free stream at angle
    alpha, damped to zero at the wall over a boundary-layer thickness
    ``delta`` (tanh of a wall-distance proxy: distance to the chord segment
    less the local half thickness), times a Gaussian wake deficit behind the
    trailing edge of depth ``wake`` and width w0 + spread sqrt(s) at a
    distance s downstream, modulated along the span (period ``span``) by 20 %
    with a spanwise velocity of 5 % of the deficit, so the wake is
    three-dimensional.  Zero pressure.  X: node coordinates, (ne, 3, N3)
    or flat [3 N_e^3] per element; returns the state in the same layout."""
    flat = X.ndim == 1
    if flat:
        raise ValueError("use developed_airfoil_state_flat for meshes of mixed order")
    x, y, z = X[:, 0], X[:, 1], X[:, 2]
    u = _developed_velocity(x, y, z, alpha_deg, u_inf, t, delta, wake, w0, spread, span)
    q = np.zeros((X.shape[0], 4, X.shape[2]))
    q[:, 1], q[:, 2], q[:, 3] = u
    return q


def _developed_velocity(x, y, z, alpha_deg, u_inf, t, delta, wake, w0, spread, span):
    xc = np.clip(x, 0.0, 1.0)
    dy = np.maximum(np.abs(y) - naca_thickness(xc, t), 0.0)
    d = np.sqrt((x - xc) ** 2 + dy ** 2)
    a = math.radians(alpha_deg)
    s = (x - 1.0) * math.cos(a) + y * math.sin(a)
    n = -(x - 1.0) * math.sin(a) + y * math.cos(a)
    sp = np.maximum(s, 0.0)
    sig = w0 + spread * np.sqrt(sp)
    deficit = np.where(s > 0.0, wake * (w0 / sig) * np.exp(-(n / sig) ** 2), 0.0)
    ph = 2.0 * math.pi * z / span
    deficit = deficit * (1.0 + 0.2 * np.sin(ph))
    bl = np.tanh(d / delta)
    mag = u_inf * bl * (1.0 - deficit)
    return mag * math.cos(a), mag * math.sin(a), 0.05 * u_inf * bl * deficit * np.cos(ph)


def developed_airfoil_state_flat(X: np.ndarray, Ps: np.ndarray, **kw) -> np.ndarray:
    """developed_airfoil_state for a flat coordinate array of a mesh of mixed order."""
    n3 = (np.asarray(Ps, dtype=np.int64) + 1) ** 3
    off = np.concatenate([[0], np.cumsum(n3)[:-1]])
    q = np.zeros(4 * int(n3.sum()))
    for e in range(len(Ps)):
        blk = X[3 * off[e]:3 * (off[e] + n3[e])].reshape(3, n3[e])
        v = developed_airfoil_state(blk[None], **kw)[0]
        q[4 * off[e]:4 * (off[e] + n3[e])] = v.ravel()
    return q


def free_stream(alpha_deg: float, u_inf: float = 1.0) -> np.ndarray:
    a = math.radians(alpha_deg)
    return np.array([0.0, u_inf * math.cos(a), u_inf * math.sin(a), 0.0])


def min_edge_length(mesh: HexMesh) -> float:
    """Smallest corner-to-corner element edge length (used to size a stable dt)."""
    Pg = mesh.Pg
    n1 = Pg + 1
    cidx = [ci * Pg + n1 * (cj * Pg) + n1 * n1 * (ck * Pg)
            for ck in (0, 1) for cj in (0, 1) for ci in (0, 1)]
    C = mesh.xyz_geom[:, :, cidx]            # (ne, 3, 8)
    edges = [(0, 1), (2, 3), (4, 5), (6, 7), (0, 2), (1, 3), (4, 6), (5, 7),
             (0, 4), (1, 5), (2, 6), (3, 7)]
    m = np.inf
    for a, b in edges:
        m = min(m, float(np.linalg.norm(C[:, :, a] - C[:, :, b], axis=1).min()))
    return m


def cfl_dt(mesh: HexMesh, P: int, q0: np.ndarray, c0sq: float, cfl: float = 0.5) -> float:
    """dt = cfl * h_min / ((P+1)^2 * lambda_max), lambda_max = max |u| + sqrt(|u|^2 + c0^2)."""
    u2 = (q0[:, 1:4] ** 2).sum(axis=1)
    lam = float(np.max(np.sqrt(u2) + np.sqrt(u2 + c0sq)))
    return cfl * min_edge_length(mesh) / ((P + 1) ** 2 * lam)


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    mesh: HexMesh
    P: int | np.ndarray        # one order, or one per element
    flag: np.ndarray
    params: dict
    dt: float | None
    nsteps: int
    state: str                 # "tgv" or "inflow"
    state_args: dict


def tgv_box_small() -> Workload:
    """Periodic [0, 2pi]^3, 4^3 elements, P = 3, Taylor-Green + 1e-2 noise,
    nu = 1e-3, Smagorinsky Cs = 0.1, Bernoulli(0.5) mask (seed 1), dt = 1e-3."""
    mesh = periodic_box(4, Pg=1)
    flag = bernoulli_mask(mesh.n_elem, 0.5, seed=1)
    params = dict(c0sq=25.0, nu=1e-3, les_model=1, C_les=0.1, mixed_face=0,
                  q_inf=[0.0, 0.0, 0.0, 0.0])
    return Workload("tgv_box4_P3", mesh, 3, flag, params, 1e-3, 10, "tgv",
                    dict(amp=1e-2, seed=0))


def naca_working(ni=96, nj=48, nk=8, P=4) -> Workload:
    """NACA0012 O-grid 96x48x8, quadratic geometry, P = 4, Re = 1e4 (nu = 1e-4, c = 1,
    U = 1), alpha = 20 deg, inflow + 1% noise, wall/wake viscous mask.

    dt = 2e-8: the impulsive no-slip start gives eddy viscosities of ~4e-3 on
    wall nodes ~1e-3 apart at the sharp trailing edge, so the explicit viscous
    limit (~4e-8) is far below the convective one (~3e-6); 2e-8 keeps a margin
    of two."""
    mesh = naca_ogrid(ni, nj, nk, Pg=2)
    flag = naca_mask(mesh, 20.0)
    params = dict(c0sq=25.0, nu=1e-4, les_model=1, C_les=0.1, mixed_face=0,
                  q_inf=list(free_stream(20.0)))
    return Workload(f"naca0012_ogrid_{ni}x{nj}x{nk}_P{P}", mesh, P, flag, params, 2e-8, 100,
                    "inflow", dict(alpha_deg=20.0, u_inf=1.0, noise=0.01, seed=0))


def tgv_box_precision(n=32, P=5) -> Workload:
    """Periodic [0, 2pi]^3 box of 32^3 elements, P = 5 (7,077,888 nodes),
    decaying Taylor-Green vortex at Re = 1600 (nu = 1/1600), Smagorinsky
    Cs = 0.1, seeded Bernoulli(0.5) mask.  dt = 2e-4: half the convective
    limit 0.5 h / ((P+1)^2 lambda) with h = 2 pi / 32 and lambda = |u| +
    sqrt(|u|^2 + c0^2) ~ 6.1."""
    mesh = periodic_box(n, Pg=1)
    flag = bernoulli_mask(mesh.n_elem, 0.5, seed=1)
    params = dict(c0sq=25.0, nu=1.0 / 1600.0, les_model=1, C_les=0.1, mixed_face=0,
                  q_inf=[0.0, 0.0, 0.0, 0.0])
    return Workload(f"tgv_box{n}_P{P}", mesh, P, flag, params, 2e-4, 1000, "tgv",
                    dict(amp=0.0, seed=0))


def naca_mixed(ni: int = 192, nj: int = 96, nk: int = 16, seed: int = 0) -> Workload:
    """The airfoil O-grid refined twice (192 x 96 x 16 elements), quadratic
    elements as on the one-order airfoil, with a per-element order drawn from
    P = 2..6, higher orders in the viscous region (wall band and wake wedge).
    Re = 1e4, alpha = 20 deg, inflow + 1 % noise."""
    mesh = naca_ogrid(ni, nj, nk, Pg=2)
    flag = naca_mask(mesh)
    P = mixed_orders(flag, seed)
    params = dict(c0sq=25.0, nu=1e-4, les_model=1, C_les=0.1, mixed_face=0, q_inf=free_stream(20.0))
    return Workload(f"naca0012_ogrid_{ni}x{nj}x{nk}_mixedP2-6", mesh, P, flag, params, 5e-9, 100, "inflow",
                    dict(alpha_deg=20.0, u_inf=1.0, noise=0.01, seed=0))


def initial_state(w: Workload, node_xyz: np.ndarray | None) -> np.ndarray:
    if np.ndim(w.P) > 0:
        if w.state != "inflow":
            raise ValueError("per-element orders: inflow states only")
        return uniform_inflow_state_flat(w.P, **w.state_args)
    N3 = (w.P + 1) ** 3
    if w.state == "tgv":
        if node_xyz is None:
            raise ValueError("Taylor-Green state needs node coordinates")
        return taylor_green_state(node_xyz, **w.state_args)
    return uniform_inflow_state(w.mesh.n_elem, N3, **w.state_args)
