"""Host-side checks of the benchmark's roofline numerator: the algorithmic
bytes of a launch, counted here field by field for the airfoil workload."""
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import bench  # noqa: E402

NE, NV, N = 36864, 10856, 5          # airfoil O-grid 96x48x8, P = 4, flagged elements
N3, N2 = N ** 3, N ** 2


def test_fused_stage_bytes_fp64():
    # the operator's bytes per node: q 32, 1/J and Ja 80, dq written 32 and
    # read 32, next state 32; three owned faces of N^2 nodes with n and s (4
    # doubles) per element.  The viscous intermediates are not counted.
    later = NE * (N3 * (32 + 80 + 32 + 32 + 32) + 3 * N2 * 4 * 8)
    first = later - NE * N3 * 32                      # A = 0: dq is not read
    assert bench.algorithmic_bytes(NE, N, fused_rk=True) == later
    assert bench.algorithmic_bytes(NE, N, fused_rk=True, first_stage=True) == first
    assert later == 1046937600
    # averaged over the three stages: (208 + 208 + 176 + 3 * 96 / N) / 3 B/node
    avg = sum(bench.algorithmic_bytes(NE, N, fused_rk=True, first_stage=(s == 0)) for s in range(3)) / 3
    assert abs(avg / (NE * N3) - (592 / 3 + 96 / N)) < 1e-9


def test_fused_stage_bytes_fp32():
    # metric and face geometry in FP32; state and RK in FP64
    later = NE * (N3 * (32 + 40 + 96) + 3 * N2 * 4 * 4)
    assert bench.algorithmic_bytes(NE, N, fused_rk=True, f32=True) == later
    assert bench.algorithmic_bytes(NE, N, fused_rk=True, f32=True, first_stage=True) == later - NE * N3 * 32


def test_residual_only_intermediate_and_viscous_bytes():
    # the residual-only operator: state 32 + metric terms 80 + R 32 B/node, three owned faces of geometry
    assert bench.algorithmic_bytes(NE, N, fused_rk=False) == NE * N3 * (144 + 96 / N)
    # viscous part (3 doubles per node) and both sides' traces (3 doubles per face node, six faces)
    assert bench.intermediate_bytes(NV, N) == NV * (N3 * 24 + 6 * N2 * 24)
    assert bench.intermediate_bytes(NV, N, f32=True) == NV * (N3 * 12 + 6 * N2 * 12)
    # viscous kernel, flagged elements: velocity 24 + metric 80 in, viscous part
    # 24 and six faces of traces out
    assert bench.viscous_kernel_bytes(NV, N) == NV * ((24 + 80 + 24) * N3 + 6 * N2 * 24)


def test_flops_summary_parsing(tmp_path, monkeypatch):
    from paper_2403_05463_amd import profiling as prof
    rows = ["Kernel_Name,Counter_Name,Counter_Value"]
    for c, v in zip(prof.FLOP_COUNTERS[64], (10, 20, 30, 5)):
        rows.append(f"\"k_residual<double, 1, 5, 128, false>(StageArgs)\",{c},{v}")
    rows32 = ["Kernel_Name,Counter_Name,Counter_Value"]
    for c, v in zip(prof.FLOP_COUNTERS[32], (1, 2, 3, 4)):
        rows32.append(f"\"k_residual<double, 1, 5, 128, false>(StageArgs)\",{c},{v}")
    a, b = tmp_path / "a.csv", tmp_path / "b.csv"
    a.write_text("\n".join(rows) + "\n")
    b.write_text("\n".join(rows32) + "\n")
    out = tmp_path / "flops.txt"
    out.write_text(prof.flops_summary(str(a), str(b), "cmd64", "cmd32"))
    r = prof.flops_for(str(out), "k_residual<double, 1, 5, 128, false>", 1e-6)
    assert r["flops_per_launch"] == 64.0 * (10 + 20 + 5 + 2 * 30)
    assert r["other_precision_flops"] == 64.0 * (1 + 2 + 4 + 2 * 3)
    assert abs(r["achieved_tflops"] - r["flops_per_launch"] / 1e-6 / 1e12) < 1e-9
    assert r["peak_tflops"] == 78.6
    # a summary taken from other kernel sources is not used
    monkeypatch.setattr(prof, "kernel_source_hash", lambda: "0" * 16)
    assert prof.flops_for(str(out), "k_residual<double, 1, 5, 128, false>", 1e-6) is None


def test_more_than_one_gpu_is_refused(capsys, monkeypatch):
    # one GPU only: asking for more, or running under a launcher with
    # WORLD_SIZE > 1, exits with status 2 and a message, before any GPU work
    assert bench.main(["--gpus", "2"]) == 2
    assert "exactly one GPU" in capsys.readouterr().err
    monkeypatch.setenv("WORLD_SIZE", "4")
    assert bench.main([]) == 2
    assert "WORLD_SIZE 4" in capsys.readouterr().err


def test_shared_metric_saving():
    """Translated elements share one metric block: the bytes not moved are
    the metric terms of every element but one per block, 80 B/node in FP64
    and 40 in FP32; the fraction against them uses the remaining bytes."""
    N, E, Bk = 5, 36864, 4608
    assert bench.shared_metric_saving(E, E, N) == 0.0
    assert bench.shared_metric_saving(E, Bk, N) == (E - Bk) * 80 * N ** 3
    assert bench.shared_metric_saving(E, Bk, N, f32=True) == (E - Bk) * 40 * N ** 3
    alg = bench.algorithmic_bytes(E, N, fused_rk=True)
    sv = bench.shared_metric_saving(E, Bk, N)
    r = bench.with_shared_metrics(alg, sv, 1e-4)
    assert r["bytes"] == alg - sv
    assert abs(r["achieved"] - (alg - sv) / 1e-4 / 1e9) < 1e-9
    assert abs(r["frac"] - r["achieved"] / bench.HBM_PEAK_GBS) < 1e-15


def test_mixed_traffic_sums_the_kernels_a_stage_launches(tmp_path, monkeypatch):
    """The mixed-order step's measured traffic: per stage, each order's
    viscous kernel (flagged elements present) and residual kernel in the
    mesh's launch shape, each pair's flux kernel and, where a side is
    flagged, its lift kernel; three stages per step."""
    import numpy as np

    from paper_2403_05463_amd import profiling

    class Mesh:   # two elements per order pair along x: orders 2 | 3, flags 0 | 1
        nbr = np.array([[1, 1, -1, -1, -1, -1], [0, 0, -1, -1, -1, -1]])

    P = np.array([2, 3])
    flag = np.array([0, 1], dtype=np.uint8)
    text = "\n".join([f"kernel source hash: {profiling.kernel_source_hash()}", "",
                      "k_residual<double,1,3,256,false> 0 0 1000 1",
                      "k_residual<double,1,4,128,true> 0 0 2000 1",
                      "k_viscous<double,4,256,false> 0 0 300 1",
                      "k_mortar_flux<3,4,double> 0 0 40 1",
                      "k_mortar_lift<3,4,double> 0 0 5 1"]) + "\n"
    path = tmp_path / "traffic.txt"
    path.write_text(text)
    monkeypatch.setattr(bench, "MIXED_TRAFFIC_SUMMARY", str(path))

    class Hdg:
        HDG_F64, HDG_F32, HDG_KERNEL_VISCOUS, HDG_KERNEL_RESIDUAL = 0, 1, 0, 1

        @staticmethod
        def hdg_mesh_get_launch(mesh, kind, prec, N):
            return {(1, 3): dict(block=256, persistent=False), (1, 4): dict(block=128, persistent=True),
                    (0, 4): dict(block=256, persistent=False)}[(kind, N)]

    assert bench.mixed_traffic_per_step(None, Hdg, Mesh, P, flag, False) == 3 * (1000 + 2000 + 300 + 40 + 5)
    # an order without flagged elements launches no viscous kernel; a pair
    # without a flagged side no lift kernel
    assert bench.mixed_traffic_per_step(None, Hdg, Mesh, P, np.zeros(2, np.uint8), False) == 3 * (1000 + 2000 + 40)
    # a kernel missing from the summary: no figure
    assert bench.mixed_traffic_per_step(None, Hdg, Mesh, P, flag, True) is None


def test_timeline_summary_gaps(tmp_path):
    """The dispatch timeline: times relative to the first listed dispatch, and
    the gap to the latest end among earlier dispatches (negative: overlap)."""
    from paper_2403_05463_amd import profiling

    path = tmp_path / "trace.csv"
    path.write_text('"Kernel_Name","Start_Timestamp","End_Timestamp","Queue_Id"\n'
                    '"k_residual<double, 1, 5, 256, false>(x)",1000000,1255000,1\n'
                    '"k_viscous<double, 5, 256, false>(x)",1010000,1150000,4\n'
                    '"k_other(x)",1100000,1200000,2\n'
                    '"k_residual<double, 1, 5, 256, false>(x)",1150000,1274000,4\n'
                    '"k_residual<double, 1, 5, 256, false>(x)",1284000,1500000,1\n')
    text = profiling.timeline_summary(str(path), ["k_residual<double, 1, 5, 256, false>",
                                                  "k_viscous<double, 5, 256, false>"], "cmd")
    rows = [ln.split() for ln in text.splitlines()[5:]]
    assert [r[0] for r in rows] == ["0.0", "10.0", "150.0", "284.0"]
    assert rows[1][3] == "-245.0" and rows[2][3] == "-105.0" and rows[3][3] == "10.0"
    assert all("k_other" not in ln for ln in text.splitlines())


def test_timer_windows_mean_of_serial_runs(tmp_path):
    """Timer windows: runs of dispatches that overlap nothing and follow one
    another closely; the named kernel's mean in each run with exactly the
    requested count.  Overlapped dispatches (graph replays) break a run."""
    from paper_2403_05463_amd import profiling

    R, V = "k_residual<double, 1, 5, 256, false>", "k_viscous<double, 5, 256, false>"
    rows = [(R, 0, 100), (V, 50, 120)]                            # overlapped: not a window
    t = 1_000_000
    for k, d in ((V, 60), (R, 120), (R, 70), (V, 62), (R, 118), (R, 72)):   # serial, 10 us gaps
        rows.append((k, t, t + d * 1000))
        t += d * 1000 + 10_000
    path = tmp_path / "trace.csv"
    path.write_text('"Kernel_Name","Start_Timestamp","End_Timestamp"\n' +
                    "".join(f'"{k}(x)",{a},{b}\n' for k, a, b in rows))
    means = profiling.timer_windows(str(path), R, 4)
    assert means == [(120 + 70 + 118 + 72) * 1000 / 4]
    assert profiling.timer_windows(str(path), R, 3) == []
