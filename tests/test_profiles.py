"""The committed HBM counter summaries describe the kernels as built from the
current sources (each carries a hash of the sources of its kernel; the
benchmark reports no traffic when it differs), and the bytes they hold are
not below what the step must move: 192 (compact) or 304 (pair state) bytes
per node of the 256^3 lattice, 308 per fluid node of the 512 x 128 x 64
junction (pairs and link word; the split step also moves psi and moments,
up to 104 bytes more, and re-reads neighbours), 196 on the compact state's
split step (totals, record and link word; it also re-reads its senders'
records)."""
import pytest

import bench

NODES = 256 ** 3
JUNCTION_FLUID = 1198336
ALGORITHMIC = {"k_step_compact": 192 * NODES, "k_step_fused": 304 * NODES, "geo_split": 308 * JUNCTION_FLUID,
               "geo_split_compact": 196 * JUNCTION_FLUID}
LIMIT = {"k_step_compact": 1.3, "k_step_fused": 1.3, "geo_split": 1.8, "geo_split_compact": 2.5}


@pytest.mark.parametrize("kernel", sorted(bench.TRAFFIC_FILES))
def test_traffic_summary_is_current(kernel):
    moved = bench.read_traffic(kernel)
    assert moved is not None, f"{bench.TRAFFIC_FILES[kernel]} is missing or was taken from other sources"
    ratio = moved / ALGORITHMIC[kernel]
    assert 1.0 <= ratio < LIMIT[kernel], ratio


def test_bench_refuses_more_than_one_gpu():
    # one GPU only: any other count ends with a JSON line that says so
    import json
    import subprocess
    import sys
    r = subprocess.run([sys.executable, bench.__file__, "--gpus", "2"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]
