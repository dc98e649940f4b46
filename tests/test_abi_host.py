"""CPU tests of the C-ABI library (no device calls) and of the host logic."""
import re
import subprocess
import os

import numpy as np
import pytest

from paper_2403_05463_amd import hdg, workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "hdg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_ \*]*?\b(hdg_[a-z0-9_]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_binding_declares_argument_types():
    """Every binding has explicit argument types, so 64-bit handles and
    pointers are never passed as C ints."""
    L = hdg.lib()
    for name in hdg.EXPORTED:
        assert getattr(L, name).argtypes is not None, name


def test_library_exports_every_declared_symbol():
    declared = _declared_functions()
    assert len(declared) >= 15
    L = hdg.lib()
    for name in declared:
        assert hasattr(L, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", hdg.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (hdg_[a-z0-9_]+)", out))
    assert set(declared) <= exported
    assert set(hdg.EXPORTED) == set(declared)


def test_library_is_gfx950_code_object():
    out = subprocess.run(["readelf", "-S", hdg.LIB_PATH], capture_output=True, text=True).stdout
    assert ".hip_fatbin" in out
    blob = open(hdg.LIB_PATH, "rb").read()
    assert b"gfx950" in blob


@pytest.mark.parametrize("mesh,P", [
    (W.periodic_box(3, Pg=2, curve_amp=0.35), 4),
    (W.naca_ogrid(24, 8, 3, Pg=2), 3),
    (W.reorient(W.periodic_box(3, Pg=3, curve_amp=0.3), 3)[0], 5),
])
def test_host_geometry_matches_oracle(orc, mesh, P):
    g = hdg.hdg_mesh_geometry(mesh, P)
    om = orc.OracleMesh(mesh, P, np.zeros(mesh.n_elem, np.uint8))
    J, Ja = om.metrics()
    xi, w, D = orc.lgl(P)
    np.testing.assert_allclose(g["xi"], xi, atol=1e-15)
    np.testing.assert_allclose(g["w"], w, rtol=1e-14)
    np.testing.assert_allclose(g["D"], D, atol=1e-13 * P * P)
    np.testing.assert_allclose(g["x"], om.node_coords(), atol=1e-13)
    np.testing.assert_allclose(g["J"], J, rtol=1e-12)
    assert np.abs(g["Ja"] - Ja).max() < 1e-12 * np.abs(Ja).max()


@pytest.mark.parametrize("Pg,seed", [(2, 1), (3, 2), (1, 3)])
def test_host_geometry_of_mixed_orders_matches_oracle(orc, Pg, seed):
    """Curved meshes of mixed order: the library's restriction of the
    curl-form product field where orders meet gives the oracle's metric terms."""
    m = W.periodic_box(3, Pg=Pg, curve_amp=0.2 if Pg > 1 else 0.25)
    if seed == 2:
        m = W.reorient(m, 5)[0]
    flag = W.bernoulli_mask(m.n_elem, 0.5, seed)
    P = np.maximum(W.mixed_orders(flag, seed), max(Pg, 2)).astype(np.int32)
    g = hdg.hdg_mesh_geometry(m, P)
    om = orc.OracleMesh(m, P, flag)
    J, Ja = om.metrics()
    np.testing.assert_allclose(g["x"], om.node_coords(), atol=1e-13)
    np.testing.assert_allclose(g["J"], J, rtol=1e-12)
    assert np.abs(g["Ja"] - Ja).max() < 1e-12 * np.abs(Ja).max()


def test_host_geometry_rejects_bad_meshes():
    m = W.periodic_box(3, Pg=1)
    bad = W.HexMesh(Pg=1, xyz_geom=m.xyz_geom, corners=m.corners, nbr=m.nbr.copy(), nbr_face=m.nbr_face,
                    orient=m.orient, centroid=m.centroid)
    bad.nbr[0, 1] = 5                                  # asymmetric
    with pytest.raises(hdg.HdgError) as ex:
        hdg.hdg_mesh_geometry(bad, 3)
    assert ex.value.status == hdg.HDG_EMESH
    o = m.orient.copy()
    o[0, 1] = 1                                        # codes no longer inverse
    bad2 = W.HexMesh(Pg=1, xyz_geom=m.xyz_geom, corners=m.corners, nbr=m.nbr, nbr_face=m.nbr_face,
                     orient=o, centroid=m.centroid)
    with pytest.raises(hdg.HdgError) as ex:
        hdg.hdg_mesh_geometry(bad2, 3)
    assert ex.value.status == hdg.HDG_EMESH
    flipped = m.xyz_geom.copy()
    flipped[0, 0] = flipped[0, 0][[1, 0, 3, 2, 5, 4, 7, 6]]  # mirror element 0 -> J < 0
    bad3 = W.HexMesh(Pg=1, xyz_geom=flipped, corners=m.corners, nbr=m.nbr, nbr_face=m.nbr_face,
                     orient=m.orient, centroid=m.centroid)
    with pytest.raises(hdg.HdgError) as ex:
        hdg.hdg_mesh_geometry(bad3, 3)
    assert ex.value.status == hdg.HDG_EMESH
    with pytest.raises(hdg.HdgError) as ex:
        hdg.hdg_mesh_geometry(m, 8)
    assert ex.value.status == hdg.HDG_EUNSUPPORTED
    empty = W.HexMesh(Pg=1, xyz_geom=m.xyz_geom[:0], corners=m.corners[:0], nbr=m.nbr[:0],
                      nbr_face=m.nbr_face[:0], orient=m.orient[:0], centroid=m.centroid[:0])
    with pytest.raises(hdg.HdgError) as ex:                      # no elements
        hdg.hdg_mesh_geometry(empty, 3)
    assert ex.value.status == hdg.HDG_EINVAL


@pytest.mark.parametrize("make", [
    lambda: W.periodic_box(4),
    lambda: W.naca_ogrid(24, 8, 3),
    lambda: W.reorient(W.periodic_box(3, Pg=2), 1)[0],
    lambda: W.box((3, 3, 4), periodic=(False, True, False)),
])
def test_generated_connectivity_is_consistent(make):
    m = make()
    ne = m.n_elem
    for e in range(ne):
        for f in range(6):
            e2 = int(m.nbr[e, f])
            if e2 < 0:
                assert e2 in (W.WALL, W.FARFIELD)
                continue
            f2 = int(m.nbr_face[e, f])
            assert m.nbr[e2, f2] == e and m.nbr_face[e2, f2] == f
            o, o2 = int(m.orient[e, f]), int(m.orient[e2, f2])
            for b in range(3):
                for a in range(3):
                    a2, b2 = W.orient_map(o, a, b, 2)
                    assert W.orient_map(o2, a2, b2, 2) == (a, b)


def test_workload_shapes():
    w = W.tgv_box_small()
    assert w.mesh.n_elem == 64 and w.P == 3 and w.nsteps == 10 and w.dt == 1e-3
    assert 20 < int(w.flag.sum()) < 44
    w2 = W.naca_working()
    assert w2.mesh.n_elem == 96 * 48 * 8 and w2.P == 4
    assert (w2.mesh.nbr == W.WALL).sum() == 96 * 8 and (w2.mesh.nbr == W.FARFIELD).sum() == 96 * 8
    q = W.initial_state(w2, None)
    assert q.shape == (w2.mesh.n_elem, 4, 125)
    assert abs(q[:, 1].mean() - np.cos(np.radians(20))) < 1e-3
    u_inf = W.free_stream(20.0)
    assert np.abs(q - u_inf[None, :, None]).max() <= 0.01 + 1e-12
