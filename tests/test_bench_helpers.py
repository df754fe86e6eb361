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


def test_fastest_pass_respects_the_converged_eigenvalue_bar():
    import bench

    def eb(**errs):
        return {"forms": {k.replace("__", "/"): {"max_dtheta_wanted_vs_cell_fp64_Ha": v} for k, v in errs.items()}}

    out = {"s_per_pass": 6.1,
           "mixed": {"s_per_pass": 4.2}, "mixed_resid": {"s_per_pass": 4.19},
           "matrix_free": {"s_per_pass": 2.37, "mixed": {"s_per_pass": 2.06}, "mixed_resid": {"s_per_pass": 2.15}},
           "eig_bar": eb(cell__fp64=0.0, cell__mixed=2.6e-7, cell__mixed_resid=9.3e-8, matrix_free__fp64=2e-14,
                         matrix_free__mixed=3.6e-8, matrix_free__mixed_resid=7e-9)}
    best = bench.fastest_pass(out)
    assert best["form"] == "matrix-free, FP32 applies 1..m-1" and best["s_per_pass"] == 2.06
    out["eig_bar"]["forms"]["matrix_free/mixed"]["max_dtheta_wanted_vs_cell_fp64_Ha"] = 2e-7   # misses the bar
    assert bench.fastest_pass(out)["form"] == "matrix-free, FP32 residual form"
    # without a converged comparison only the FP64 forms qualify
    del out["eig_bar"]
    assert bench.fastest_pass(out)["form"] == "matrix-free, FP64"
    assert bench.fastest_pass({"s_per_pass": 6.1})["form"] == "cell matrices, FP64"


def test_cell_roofline_counts_the_pauli_form_work():
    import bench
    # the last measured FP64 launch: 4.819e11 flop (4M count) in 5.994 ms
    r = bench.cell_roofline(4.819e11, 0.75 * 4.819e11 * 352 / 343, 5.994, True, bench.PEAK_FP64)
    assert 0.0 < r["frac"] <= 1.0
    assert abs(r["achieved"] - 0.75 * 4.819e11 / 5.994e-3 / 1e12) < 1e-3
    assert r["dense_4M_equivalent_tflops"] > bench.PEAK_FP64 * r["frac"]
    # with the k-term the Pauli form does the full 4M count
    rk = bench.cell_roofline(4.819e11, 4.819e11, 8.0, False, bench.PEAK_FP64)
    assert abs(rk["achieved"] - rk["dense_4M_equivalent_tflops"]) < 1e-9
