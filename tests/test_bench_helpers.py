"""CPU checks of bench.py's counter records: a record applies only to the launch
shape and the kernel sources it was taken for."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_traffic_records_match_their_kernels():
    import bench
    cell = bench.measured_traffic(22000)
    mf = bench.measured_traffic(64000, bench.MF_TRAFFIC_RECORD, bench.MF_SOURCES)
    assert cell is not None and mf is not None
    # measured bytes are close to the algorithmic ones (no large re-reads)
    assert 1.0 < cell / 7.98e9 < 1.2
    assert 1.0 <= mf / 4.2148e9 < 1.05


def test_traffic_record_rejects_other_shapes_and_sources():
    import bench
    assert bench.measured_traffic(22001) is None
    assert bench.measured_traffic(64000, bench.MF_TRAFFIC_RECORD, bench.CELL_SOURCES) is None
    assert bench.measured_traffic(22000, bench.MF_TRAFFIC_RECORD, bench.MF_SOURCES) is None
    assert bench.kernel_fingerprint(bench.CELL_SOURCES) != bench.kernel_fingerprint(bench.MF_SOURCES)


def test_fastest_pass_respects_the_eigenvalue_bar():
    import bench
    out = {"s_per_pass": 6.1,
           "mixed": {"s_per_pass": 4.2, "max_dtheta_vs_fp64_Ha": 2.6e-7},
           "mixed_resid": {"s_per_pass": 4.19, "max_dtheta_vs_fp64_Ha": 9.3e-8},
           "matrix_free": {"s_per_pass": 2.37, "max_dtheta_vs_cell_fp64_Ha": 2e-14,
                           "mixed": {"s_per_pass": 2.06, "max_dtheta_vs_cell_fp64_Ha": 3.6e-8},
                           "mixed_resid": {"s_per_pass": 2.15, "max_dtheta_vs_cell_fp64_Ha": 7e-9}}}
    best = bench.fastest_pass(out)
    assert best["form"] == "matrix-free, FP32 applies 1..m-1" and best["s_per_pass"] == 2.06
    out["matrix_free"]["mixed"]["max_dtheta_vs_cell_fp64_Ha"] = 2e-7     # misses the bar
    assert bench.fastest_pass(out)["form"] == "matrix-free, FP32 residual form"
    assert bench.fastest_pass({"s_per_pass": 6.1})["form"] == "cell matrices, FP64"
