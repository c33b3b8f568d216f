"""The committed HBM counter summaries describe the kernels as built from the
current sources (each carries a hash of the sources of its kernel; the
benchmark reports no traffic when it differs), and the bytes they hold are
not below what the sweep must move: 192 (compact) or 304 (pair state) bytes
per node of the 256^3 lattice."""
import pytest

import bench

NODES = 256 ** 3
ALGORITHMIC = {"k_step_compact": 192 * NODES, "k_step_fused": 304 * NODES}


@pytest.mark.parametrize("kernel", sorted(bench.TRAFFIC_FILES))
def test_traffic_summary_is_current(kernel):
    moved = bench.read_traffic(kernel)
    assert moved is not None, f"{bench.TRAFFIC_FILES[kernel]} is missing or was taken from other sources"
    ratio = moved / ALGORITHMIC[kernel]
    assert 1.0 <= ratio < 1.3, ratio
