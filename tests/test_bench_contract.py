"""Host-side checks of the benchmark's roofline inputs: the algorithmic byte count per
element restated from its parts, and the committed traffic measurement taken on the stage
kernel as it stands (the benchmark reports traffic only then)."""
import json
import os

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def dimp(n):
    return (n + 1) * (n + 2) * (n + 3) // 6


def test_algorithmic_bytes_from_their_parts():
    # q and res read and written (4 fields each), c^2_M, the 25-word geometry record, and
    # four int32 neighbour ids
    for n, m in ((3, 1), (5, 2), (9, 4)):
        for word in (4, 8):
            parts = 4 * 4 * dimp(n) * word + dimp(m) * word + 25 * word + 4 * 4
            assert bench.algorithmic_bytes_per_element(n, m, word) == parts
    assert bench.algorithmic_bytes_per_element(5, 2, 8) == 7464  # the benchmark configuration


def test_committed_traffic_matches_the_kernel_source():
    with open(os.path.join(ROOT, "profiles", "stage_kernel_cube196k_N5_M2_traffic.json")) as fh:
        t = json.load(fh)
    assert t["kernel_code_sha256_16"] == bench.kernel_source_hash(), \
        "profiles were taken on another stage-kernel source: re-take them"
    for dt, word in (("f64", 8), ("f32", 4)):
        alg = bench.algorithmic_bytes_per_element(5, 2, word) * 196608
        ratio = t["bytes_per_launch_" + dt] / alg
        assert 1.0 <= ratio < 1.5, (dt, ratio)  # measured at or above the algorithmic bytes
        assert bench.measured_traffic(dt) == t["bytes_per_launch_" + dt]


def test_stage_kernel_profiles_name_the_current_source():
    """Every stage-kernel profile summary states the hash of the source it was taken on; a
    summary left from another source would quote times and counters of a different kernel.
    (The first design's summary, `*_baseline.md`, is a record of that design on purpose.)"""
    import re
    names = sorted(n for n in os.listdir(os.path.join(ROOT, "profiles")) if n.startswith("stage_kernel_"))
    summaries = [n for n in names if n.endswith(".md") and not n.endswith("_baseline.md")]
    assert summaries
    for n in summaries:
        with open(os.path.join(ROOT, "profiles", n)) as fh:
            m = re.search(r"Kernel code sha256\[:16\] = ([0-9a-f]{16})", fh.read())
        assert m, n
        assert m.group(1) == bench.kernel_source_hash(), n
