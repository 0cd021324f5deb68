"""The measurement's recorded inputs stay tied to the code they describe:
the HBM bytes bench.py reports for the dense local-solve GEMM (two counter
runs, FETCH_SIZE and WRITE_SIZE, on the 2-D L = 256, h = 1/64 workload) are
valid only for the kernel source they were taken from.  If that source
changes, the counters must be taken again; this test then fails instead of the
bench line quietly reporting a null traffic figure."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def test_counted_gemm_traffic_matches_the_source():
    import bench
    c = bench.COUNTED_TRAFFIC
    t = bench.counted_traffic(c["workload"], c["local_prec"])
    assert t is not None, "k_dense_gemm or k_coarse.h changed since the counters were taken"
    # the figure itself: FETCH x 2.0 + WRITE x 1.0 (copy calibration), about 84 MB
    assert 70e6 < t < 100e6


def test_counted_traffic_only_for_its_workload():
    import bench
    assert bench.counted_traffic("2d-L256-ne64", "bf16x3") is None
    assert bench.counted_traffic("3d-p2-L16-ne16", "bf16") is None
