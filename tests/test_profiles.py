"""The committed rocprofv3 summaries match the sources they describe (CPU only).

bench.py reports the measured HBM traffic of the collide-stream kernel from
profiles/hydro_traffic_spreading_256x256x128.json only while the sha256 of the
sources that define k_hydro equals the one recorded with the counters; a
change to those sources without new counters would turn the reported traffic
into null.  These tests catch that, and check that the summaries the design
notes cite exist and give their commands.
"""
import json
import os

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROF = os.path.join(ROOT, "profiles")


def test_hydro_traffic_is_reported_only_for_the_kernel_it_was_taken_on():
    d = json.load(open(os.path.join(PROF, "hydro_traffic_spreading_256x256x128.json")))
    t = bench.measured_traffic("spreading_256x256x128")
    if d["kernel_source_sha256_16"] != bench.kernel_source_hash():
        # the kernel changed since the counters were taken: no traffic is reported
        assert t is None
    else:
        # between the algorithmic 220 B and 300 B per node of the 256 x 256 x 128 lattice
        assert t is not None and 220 * 256 * 256 * 128 < t < 300 * 256 * 256 * 128
    assert bench.measured_traffic("sessile_32x32x32") is None


def test_summaries_exist_and_name_their_commands():
    for name in ("kernel_stats_spreading_256x256x128.md", "hbm_traffic_spreading_256x256x128.md",
                 "kernel_stats_orifice_192x192x768.md", "hbm_traffic_orifice_192x192x768.md",
                 "kernel_stats_batch64_and_adjoint_128x128x64.md", "hbm_traffic_adjoint_128x128x64.md",
                 "kernel_stats_r1_spreading_256x256x128.md", "valu_lds_counters_spreading_256x256x128.md"):
        text = open(os.path.join(PROF, name)).read()
        assert "rocprofv3" in text and "bench.py" in text, name
        assert "| kernel |" in text, name


def test_orifice_traffic_is_the_benchmark_workloads():
    """The benchmark line's workload (orifice 192 x 192 x 768) has its own
    counter summary, reported while the kernel sources are unchanged."""
    d = json.load(open(os.path.join(PROF, "hydro_traffic_orifice_192x192x768.json")))
    t = bench.measured_traffic("orifice_192x192x768")
    if d["kernel_source_sha256_16"] == bench.kernel_source_hash():
        assert t is not None and 220 * d["fluid_nodes"] < t < 300 * d["fluid_nodes"]
    else:
        assert t is None
