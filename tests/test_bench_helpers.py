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
