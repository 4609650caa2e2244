"""Host-side logic of the benchmark script (no GPU): reading the committed
HBM-traffic summary that the roofline's traffic field comes from."""

import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_traffic_summary_values_with_trailing_notes():
    txt = ("Some text: with a colon\n"
           "- source_sha256: `00ff` (csrc/k_local.hip at the time of the counters)\n"
           "- traffic_bytes_per_launch: 7.199072e+10\n")
    vals = bench.parse_traffic_summary(txt)
    assert vals == {"source_sha256": "00ff", "traffic_bytes_per_launch": "7.199072e+10"}


def test_committed_traffic_summary_parses():
    path = os.path.join(ROOT, "profiles", "k_local_setup_channel8192_fp64_traffic.md")
    vals = bench.parse_traffic_summary(open(path).read())
    assert len(vals["source_sha256"]) == 64
    int(vals["source_sha256"], 16)
    assert float(vals["traffic_bytes_per_launch"]) > 1e10
