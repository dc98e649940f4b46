"""Host-side checks of the benchmark's roofline numerator: the algorithmic
bytes of a launch, counted here field by field for the airfoil workload."""
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import bench  # noqa: E402

NE, NV, N = 36864, 10856, 5          # airfoil O-grid 96x48x8, P = 4, flagged elements
N3, N2 = N ** 3, N ** 2


def test_fused_stage_bytes_fp64():
    # per node: q 32, 1/J and Ja 80, dq written 32 and read 32, next state 32;
    # three owned faces of N^2 nodes with n and s (4 doubles) per element;
    # flagged: viscous volume part 3 doubles per node, both sides' traces
    # 3 doubles per face node on six faces
    later = NE * (N3 * (32 + 80 + 32 + 32 + 32) + 3 * N2 * 4 * 8) + NV * (N3 * 3 * 8 + 6 * N2 * 3 * 8)
    first = later - NE * N3 * 32                      # A = 0: dq is not read
    assert bench.algorithmic_bytes(1, NE, NV, N, fused_rk=True) == later
    assert bench.algorithmic_bytes(1, NE, NV, N, fused_rk=True, first_stage=True) == first
    assert later == 1118587200


def test_fused_stage_bytes_fp32():
    # metric, face geometry and viscous parts in FP32; state and RK in FP64
    later = NE * (N3 * (32 + 40 + 96) + 3 * N2 * 4 * 4) + NV * (N3 * 3 * 4 + 6 * N2 * 3 * 4)
    assert bench.algorithmic_bytes(1, NE, NV, N, fused_rk=True, f32=True) == later
    assert bench.algorithmic_bytes(1, NE, NV, N, fused_rk=True, f32=True, first_stage=True) == \
        later - NE * N3 * 32


def test_residual_only_and_viscous_bytes():
    # residual form: R written instead of the RK traffic
    assert bench.algorithmic_bytes(1, NE, NV, N, fused_rk=False) == \
        NE * (N3 * (32 + 80 + 32) + 3 * N2 * 32) + NV * (N3 * 24 + 6 * N2 * 24)
    # viscous kernel, flagged elements: velocity 24 + metric 80 in, viscous part
    # 24 and six faces of traces out
    assert bench.algorithmic_bytes(0, NE, NV, N, fused_rk=True) == NV * ((24 + 80 + 24) * N3 + 6 * N2 * 24)


def test_more_than_one_gpu_is_refused(capsys, monkeypatch):
    # one GPU only: asking for more, or running under a launcher with
    # WORLD_SIZE > 1, exits with status 2 and a message, before any GPU work
    assert bench.main(["--gpus", "2"]) == 2
    assert "exactly one GPU" in capsys.readouterr().err
    monkeypatch.setenv("WORLD_SIZE", "4")
    assert bench.main([]) == 2
    assert "WORLD_SIZE 4" in capsys.readouterr().err
