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
