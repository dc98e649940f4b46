"""The request loop on the device: a short Poisson stream of independent
solves under a memory budget that forces queueing; every result equals the
same solve run alone, bitwise."""
import sys

import numpy as np
import pytest

from paper_2403_05463_amd import hdg, serving as S

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
        out, dt = r.result
        m, q, dq, dt2 = alone.make_alone(r)
        assert dt2 == dt
        hdg.hdg_rk3_steps(m, q, dq, dt, r.nsteps, prec=prec)
        torch.cuda.synchronize()
        assert np.all(np.isfinite(out))
        assert np.array_equal(q.cpu().numpy(), out), f"request {r.rid} (n={r.n}, P={r.P}) differs alone"
