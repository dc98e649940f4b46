"""Shared helpers of the GPU parity tests: run the HIP path and the oracle on
the same seeded inputs and compare them field by field."""
from __future__ import annotations

import numpy as np

# FP64 target: per-field relative error of the residual <= 1e-12, in the
# mass-weighted L2 norm and in the max norm.  The denominator of field f is
# max(||R_f||, 1e-3 max_g ||R_g||): the pressure residual -c0^2 div u of a
# nearly divergence-free field is a small difference of large terms, so its
# own norm alone would measure cancellation, not the kernels.
TOL_F64 = 1e-12


def field_errors(R_gpu: np.ndarray, R_ref: np.ndarray, mass: np.ndarray) -> dict:
    d = R_gpu - R_ref
    m = mass[:, None, :]
    l2 = np.sqrt((m * d * d).sum(axis=(0, 2)))
    l2_ref = np.sqrt((m * R_ref * R_ref).sum(axis=(0, 2)))
    mx = np.abs(d).max(axis=(0, 2))
    mx_ref = np.abs(R_ref).max(axis=(0, 2))
    fl2 = np.maximum(l2_ref, 1e-3 * l2_ref.max())
    fmx = np.maximum(mx_ref, 1e-3 * mx_ref.max())
    return dict(l2=l2 / fl2, max=mx / fmx, l2_raw=l2 / np.maximum(l2_ref, 1e-300),
                max_raw=mx / np.maximum(mx_ref, 1e-300),
                l2_vec=l2 / l2_ref.max(), max_vec=mx / mx_ref.max())


# FP32 target (precision form): per-field relative L2 error of the residual
# <= 1e-5.  For the pressure row, whose residual -c0^2 div u cancels between
# terms of size c0^2 |grad u| (to discretisation error on a divergence-free
# field), the denominator is max(||R_p||, c0^2 ||grad u||_F): an FP32 sum of
# such terms cannot be more accurate than its terms.  Velocity rows keep the
# floored norm above.
TOL_F32 = 1e-5


def fp32_errors(R32, R_ref, mass, p_scale):
    """Per-field errors in both norms; ``p_scale`` = (L2, max) pressure term scale."""
    e = field_errors(R32, R_ref, mass)
    d = R32 - R_ref
    m = mass[:, None, :]
    l2 = np.sqrt((m * d * d).sum(axis=(0, 2)))
    l2_ref = np.sqrt((m * R_ref * R_ref).sum(axis=(0, 2)))
    den = np.maximum(l2_ref, 1e-3 * l2_ref.max())
    den[0] = max(l2_ref[0], p_scale[0])
    mx = np.abs(d).max(axis=(0, 2))
    mx_ref = np.abs(R_ref).max(axis=(0, 2))
    dmx = np.maximum(mx_ref, 1e-3 * mx_ref.max())
    dmx[0] = max(mx_ref[0], p_scale[1])
    e["l2_f32"] = l2 / den
    e["max_f32"] = mx / dmx
    return e


def pressure_term_scale(orc, om, params, q, flag, c0sq):
    """c0^2 |grad u|_F in the mass-weighted L2 norm and in the max norm, from the
    oracle's BR1 gradient on every element."""
    om.set_flags(np.ones_like(flag))
    G = om.gradient(params, q)
    om.set_flags(flag)
    J, _ = om.metrics()
    _, w, _ = orc.lgl(om.P)
    mass = J * np.einsum("k,j,i->kji", w, w, w).ravel()[None]
    g2 = (G * G).sum(axis=(1, 2))
    return c0sq * float(np.sqrt((mass * g2).sum())), c0sq * float(np.sqrt(g2.max()))


def increment_errors(q_gpu, q_ref, q0, mass):
    """Per-field errors of RK increments, q_gpu - q0 against q_ref - q0, in the
    floored norms of ``field_errors`` (denominators: the reference increment),
    and the rounding floor of such a comparison: each final state carries
    about one FP64 unit in the last place of q, so an increment cannot be
    compared more closely than 4 eps ||q_f|| / (denominator) whatever the
    arithmetic that produced it (returned as ``floor_l2`` / ``floor_max``)."""
    e = field_errors(q_gpu - q0, q_ref - q0, mass)
    m = mass[:, None, :]
    dref = q_ref - q0
    l2_ref = np.sqrt((m * dref * dref).sum(axis=(0, 2)))
    mx_ref = np.abs(dref).max(axis=(0, 2))
    eps = np.finfo(np.float64).eps
    e["floor_l2"] = 4 * eps * np.sqrt((m * q_ref * q_ref).sum(axis=(0, 2))) / np.maximum(l2_ref, 1e-3 * l2_ref.max())
    e["floor_max"] = 4 * eps * np.abs(q_ref).max(axis=(0, 2)) / np.maximum(mx_ref, 1e-3 * mx_ref.max())
    return e


def assert_increment_parity(q_gpu, q_ref, q0, mass, tol=TOL_F64, what=""):
    """RK parity on the increments q - q0 per field: relative error <= tol, or
    <= the state's own rounding floor where that is larger (reported)."""
    assert np.all(np.isfinite(q_gpu)), f"{what}: non-finite GPU values"
    e = increment_errors(q_gpu, q_ref, q0, mass)
    bl2 = np.maximum(tol, e["floor_l2"])
    bmx = np.maximum(tol, e["floor_max"])
    assert np.all(e["l2"] <= bl2) and np.all(e["max"] <= bmx), \
        f"{what}: increment errors l2={e['l2']} max={e['max']} (bounds l2={bl2} max={bmx})"
    return e


def assert_parity(R_gpu, R_ref, mass, tol=TOL_F64, what=""):
    assert np.all(np.isfinite(R_gpu)), f"{what}: non-finite GPU values"
    e = field_errors(R_gpu, R_ref, mass)
    worst = max(e["l2"].max(), e["max"].max())
    assert worst <= tol, f"{what}: per-field errors l2={e['l2']} max={e['max']} (tol {tol})"
    return e


def oracle_mass(orc, om, P):
    J, _ = om.metrics()
    _, w, _ = orc.lgl(P)
    return J * np.einsum("k,j,i->kji", w, w, w).ravel()[None]


# Meshes of mixed order: states are flat, element after element, [4][N_e^3] each.

def flat_fields(om, arr):
    """Per-field flat vectors of an element-after-element array: node n of
    element e, field f sits at 4 off_e + f n3_e + (n - off_e)."""
    n3e = (om.Ps.astype(np.int64) + 1) ** 3
    off, n3 = np.repeat(om.offsets.astype(np.int64), n3e), np.repeat(n3e, n3e)
    n = np.arange(om.nodes, dtype=np.int64)
    flat = np.asarray(arr).ravel()
    return [flat[n + 3 * off + f * n3] for f in range(4)]


def flat_mass(orc, om):
    """w_a w_b w_c J per node of a mesh of mixed order (flat, node order)."""
    J, _ = om.metrics()
    J = np.asarray(J).ravel()
    out = np.empty(om.nodes)
    off = om.offsets.astype(np.int64)
    for P in np.unique(om.Ps):
        _, w, _ = orc.lgl(int(P))
        cube = np.einsum("k,j,i->kji", w, w, w).ravel()
        sel = off[om.Ps == P]
        idx = (sel[:, None] + np.arange(cube.size)[None]).ravel()
        out[idx] = J[idx] * np.tile(cube, sel.size)
    return out


def flat_errors(om, mass, got, ref):
    """Per-field relative errors (L2, max) of flat arrays, floored as in
    ``field_errors``."""
    g, r = flat_fields(om, got), flat_fields(om, ref)
    l2 = np.array([np.sqrt((mass * (a - b) ** 2).sum()) for a, b in zip(g, r)])
    l2r = np.array([np.sqrt((mass * b ** 2).sum()) for b in r])
    mx = np.array([np.abs(a - b).max() for a, b in zip(g, r)])
    mxr = np.array([np.abs(b).max() for b in r])
    return l2 / np.maximum(l2r, 1e-3 * l2r.max()), mx / np.maximum(mxr, 1e-3 * mxr.max())
