"""Host-side logic of bench.py (no GPU): the one-GPU guard, the workload table, the trap,
the traffic table and the oracle baseline record."""
import math
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_before_touching_a_device():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


@pytest.mark.parametrize("name", sorted(bench.WORKLOADS))
def test_workload_shapes(name):
    ndim, _ = bench.WORKLOADS[name]
    expect = {"1d_two_soliton_scattering": [16384], "2d_vortex_pair": [2048, 2048],
              "3d_vortex_lines": [256, 256, 256], "3d_vortex_lines_512": [512, 512, 512]}[name]
    if ndim == 3 and expect[0] > 256:
        pytest.skip("the 512^3 state takes 10.7 GB of host memory to build")
    w = bench.workload_input(name, 10)
    assert bench.workload_shape(w, ndim) == expect
    assert w.psi[0].shape == (5, *expect)


def test_trap_reaches_one_half_at_the_edge_midpoints():
    class W:
        eps = 0.1
        nx, ny, nz = [64], [48], [1]
    V, mu = bench.trap_potential(W, 2)
    assert V.shape == (48, 64) and mu == 0.5
    # V = omega^2 r^2 / 4 vanishes at the centre and reaches 1/2 at the midpoints of the longer edges
    assert V[24, 32] == 0.0
    assert math.isclose(V[24, 0], 0.5, rel_tol=1e-12)
    assert V.max() > 0.5 and np.all(V >= 0)


def test_traffic_table_is_consistent():
    t = bench.TRAFFIC
    assert math.isclose(t["fetch_scale"], 2.0, rel_tol=1e-3) and t["write_scale"] == 1.0
    sites = {"1d_two_soliton_scattering": 16384, "2d_vortex_pair": 2048 ** 2, "3d_vortex_lines": 256 ** 3,
             "3d_vortex_lines_512": 512 ** 3}
    if t["kib"]:
        assert t["sources_sha256_16"] == bench.kernel_sources_sha()   # measured on these sources
    for entry, plans in t["kib"].items():
        workload, storage, split = entry.split("/")
        assert storage in ("c64", "c128") and split in ("interleaved", "plain")
        ndim = bench.WORKLOADS[workload][0]
        half = bench.BYTES_PER_SITE_PASS[storage] // 2
        for key, (fetch, write) in plans.items():
            assert fetch > 0 and write > 0
            # the y half over two launches (key suffix /ysplit) writes and reads the state twice
            passes = bench.PASSES_PER_STEP[ndim] * (2 if key.endswith("/ysplit") else 1)
            # a launch writes at least the state it produces: 10 amplitudes per site per pass (KiB here)
            assert write >= 0.99 * half * sites[workload] * passes / 1024, (entry, key)
            # and reads at least the state it consumes
            assert fetch * t["fetch_scale"] >= 0.99 * half * sites[workload] * passes / 1024


def test_oracle_baseline_record():
    import qlg_inputs as qi
    w = qi.two_solitons_1d_L16384(L=512, nsteps=10)
    r = bench.cpu_baseline(w, 10, 1)
    assert r["kind"] == "oracle" and r["unit"] == "site-updates/s" and r["value"] > 0
    assert r["cores"] >= 1 and r["per_core"]["cores"] == 1 and r["per_core"]["value"] > 0
    assert "512" in r["sample"] and "10 steps" in r["sample"]
