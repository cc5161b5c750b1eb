"""The benchmark's records on the host: the ladder traffic that bench.py
reports comes from the committed counter summary of the kernel in the
source tree (its digest matches), and the roofline's kernel name follows
the autotuner's variant numbers."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    sys.path.insert(0, ROOT)
    import bench
    return bench


def test_ladder_traffic_summary_matches_the_kernel_source():
    b = _bench()
    assert b.gemm_kernel_digest() is not None
    t = b.ladder_traffic(16)
    assert t is not None and 7.8e9 < t < 2e11  # above the algorithmic bytes, below the worst variant
    assert b.ladder_traffic(13) is None  # only the direct-load variants are reported


def test_kernel_names_of_the_variants():
    b = _bench()
    assert b.gemm_kernel_name(16) == "k_zgemm_dma"
    assert b.gemm_kernel_name(18) == "k_zgemm_dma"
    assert b.gemm_kernel_name(14) == "k_zgemm_w1"
    assert b.gemm_kernel_name(10) == "k_zgemm_p1"
    assert b.gemm_kernel_name(3) == "k_zgemm_p"
    assert b.gemm_kernel_name(19) == "k_zgemm_p1"
    assert b.gemm_kernel_name(120) == "k_zgemm_p"
