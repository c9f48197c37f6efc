"""The counter traffic the benchmark line reports comes from the committed
rocprofv3 summaries under profiles/, keyed by a hash of the kernels' source:
a figure is reported only while the summary's hash equals the hash of the
source as it stands, and an unknown kernel or workload gives none."""
import os

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _recorded(workload, key):
    with open(bench.traffic_file(workload)) as fh:
        for line in fh:
            if line.startswith(key + " ="):
                return line.split("=")[1].strip()
    return None


@pytest.mark.parametrize("workload,kernel,key,now", [
    ("cant3pt-192x96x96", "k_apply_K_plane<double>", "operator_source_sha256_16",
     bench.operator_source_hash),
    ("cant3pt-192x96x96", "k_gs_mf<float>", "kernel_source_sha256_16", bench.kernel_source_hash),
    ("cant3case-192x96x96", "k_ml_gs<9, true>", "multiload_source_sha256_16",
     bench.multiload_source_hash),
])
def test_traffic_is_reported_only_for_the_source_it_was_measured_on(workload, kernel, key, now):
    v = bench.measured_traffic(workload, kernel)
    if _recorded(workload, key) == now():
        assert v is not None and v > 0
    else:
        assert v is None


def test_unknown_kernel_or_workload_gives_none():
    assert bench.measured_traffic("cant3case-192x96x96", "k_no_such_kernel") is None
    assert bench.measured_traffic("no-such-workload", "k_apply_K_plane<double>") is None


def test_recorded_K_traffic_is_near_its_algorithmic_bytes():
    # K(rho)x at 192x96x96: 16 n_dof + 8 m bytes per launch
    n_dof, m = 5447811, 1769472
    with open(bench.traffic_file("cant3pt-192x96x96")) as fh:
        line = [x for x in fh if x.startswith("traffic_bytes_per_launch k_apply_K_plane<double> =")]
    k = float(line[0].split("=")[1])
    assert 1.0 <= k / (16 * n_dof + 8 * m) < 1.5
