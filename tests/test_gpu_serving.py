"""The request loop on the device: a short Poisson stream of independent
solves under a memory budget that forces queueing; every result equals the
same solve run alone, bitwise."""
import sys

import numpy as np
import pytest

from paper_2403_05463_amd import hdg, serving as S, workloads as W
from parity import TOL_F32, TOL_F64, increment_errors, oracle_mass

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.parametrize("prec", [hdg.HDG_F32, hdg.HDG_F64])
def test_served_results_equal_alone(torch_cuda, prec):
    torch = torch_cuda
    ctx = hdg.hdg_init(0)
    reqs = S.make_requests(14, rate=60.0, seed=5, n_range=(3, 7), p_range=(2, 6), nsteps=12)
    budget = 2 * max(S.footprint_bytes(r.n, r.P) for r in reqs)
    _say(f"serving 14 requests, prec {prec}, budget {budget / 1e6:.1f} MB, 4 slots")
    be = S.HdgBackend(ctx, max_members=4, prec=prec, torch=torch, keep_results=True)
    st = S.serve(reqs, be, mem_budget=budget, max_members=4, max_steps_per_call=5, setup_workers=2)
    summ = st.summary()
    _say(f"summary: {summ}")
    assert summ["requests"] == 14
    assert st.peak_bytes <= budget
    assert summ["p99_latency_s"] >= summ["p50_latency_s"] > 0
    alone = S.HdgBackend(ctx, max_members=1, prec=prec, torch=torch)
    for r in st.requests:
        out, dt = r.result["q"], r.result["dt"]
        m, q, dq, dt2 = alone.make_alone(r)
        assert dt2 == dt
        assert np.array_equal(q.cpu().numpy(), r.result["q0"])
        hdg.hdg_rk3_steps(m, q, dq, dt, r.nsteps, prec=prec)
        torch.cuda.synchronize()
        assert np.all(np.isfinite(out))
        assert np.array_equal(q.cpu().numpy(), out), f"request {r.rid} (n={r.n}, P={r.P}) differs alone"


@pytest.mark.parametrize("prec", [hdg.HDG_F64, hdg.HDG_F32])
def test_served_results_match_oracle(orc, torch_cuda, prec):
    """A short served stream (continuous batching, queueing under a budget):
    every result against the FP64 oracle's RK3 from the same initial state and
    time step, per field on the increments: FP64 within 1e-12 (or the states'
    rounding floor), FP32 residual arithmetic within 1e-5 on the velocity rows."""
    torch = torch_cuda
    ctx = hdg.hdg_init(0)
    reqs = S.make_requests(6, rate=80.0, seed=9, n_range=(3, 4), p_range=(2, 5), nsteps=6)
    budget = 2 * max(S.footprint_bytes(r.n, r.P) for r in reqs)
    _say(f"serving 6 requests vs oracle, prec {prec}")
    be = S.HdgBackend(ctx, max_members=3, prec=prec, torch=torch, keep_results=True)
    st = S.serve(reqs, be, mem_budget=budget, max_members=3, max_steps_per_call=4, setup_workers=2)
    assert len(st.requests) == 6 and not st.refused
    for r in st.requests:
        mesh = W.periodic_box(r.n, Pg=1)
        flag = W.bernoulli_mask(mesh.n_elem, r.frac, r.seed)
        om = orc.OracleMesh(mesh, r.P, flag)
        po = orc.make_params(c0sq=be.C0SQ, nu=r.nu, les_model=1, C_les=0.1)
        q0 = r.result["q0"]
        ref = om.rk3(po, q0, r.result["dt"], r.nsteps)
        e = increment_errors(r.result["q"], ref, q0, oracle_mass(orc, om, r.P))
        _say(f"request {r.rid} (n={r.n}, P={r.P}): increment errors L2 {e['l2']}, max {e['max']}")
        if prec == hdg.HDG_F64:
            assert np.all(e["l2"] <= np.maximum(TOL_F64, e["floor_l2"]))
            assert np.all(e["max"] <= np.maximum(TOL_F64, e["floor_max"]))
        else:
            assert e["l2"][1:].max() <= TOL_F32 and e["max"][1:].max() <= 10 * TOL_F32
