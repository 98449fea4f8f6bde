"""The committed profile summaries were taken with the kernel sources in the
tree: the counters file that bench.py scales its traffic figure from, and
the summaries' recorded source hashes, match the current sources."""
import hashlib
import json
import os
import re
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2609_16575_amd", "csrc")
PROFILES = os.path.join(ROOT, "profiles")


def _sha(files):
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(CSRC, f), "rb").read())
    return h.hexdigest()[:16]


def test_counters_match_the_kernel_sources():
    sys.path.insert(0, ROOT)
    import bench
    c = json.load(open(os.path.join(PROFILES, "push_fused_thermal_ep_128_counters.json")))
    assert c["kernel_source_sha"] == bench.kernel_sha()


def test_summaries_name_the_current_sources():
    push = _sha(["push_f32.hip", "pic_math.hpp", "internal.hpp"])
    adj = _sha(["adjoint.hip"])
    seen = 0
    for name in sorted(os.listdir(PROFILES)):
        if not name.endswith(".md"):
            continue
        text = open(os.path.join(PROFILES, name)).read()
        m = re.search(r"sha256\[:16\] of the kernel's sources \(push_f32.hip, pic_math.hpp, "
                      r"internal.hpp\): `([0-9a-f]{16})`", text)
        if m:
            assert m.group(1) == push, name
            seen += 1
        m = re.search(r"sha256\[:16\] of adjoint.hip: `([0-9a-f]{16})`", text)
        if m:
            assert m.group(1) == adj, name
            seen += 1
    assert seen >= 6
