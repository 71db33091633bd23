"""The committed rocprofv3 summaries match the pass kernels' current source
(CPU only): every summary that records a source hash records the current
one, and the benchmark can read the dominant pass's measured traffic from
the traffic summary (its roofline `traffic` would otherwise be null)."""
import os
import re
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

PROFILES = os.path.join(ROOT, "profiles")


def test_summaries_record_the_current_kernel_source():
    cur = bench.kernel_source_hash()
    seen = 0
    for name in sorted(os.listdir(PROFILES)):
        text = open(os.path.join(PROFILES, name)).read()
        for h in re.findall(r"sha256\[:16\]: ([0-9a-f]{16})", text):
            assert h == cur, (name, h, cur)
            seen += 1
    assert seen >= 4


def test_dominant_pass_traffic_is_readable():
    plan = {"kind": 1, "n": 256, "cols": 8, "wide": 1, "variant": 1, "blocks": 1}
    t = bench.committed_traffic("inv_axis2_update_fwd_axis2", plan)
    assert t is not None
    # calibrated bytes per launch of the fused pass at 256^3: 180 B/cell
    assert abs(t / 256 ** 3 - 180.0) < 2.0


def test_every_summary_names_its_command():
    for name in sorted(os.listdir(PROFILES)):
        if name == "README.md":
            continue
        text = open(os.path.join(PROFILES, name)).read()
        assert "bench.py" in text and ("command" in text.lower()), name
