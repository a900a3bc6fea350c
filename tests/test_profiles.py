"""The counter summaries under profiles/ that bench.py reads: the traffic
fingerprint ignores comments but not code, and every summary it reads carries
a fingerprint and a per-launch byte count."""
import os
import re

import bench


def test_fingerprint_ignores_comments_not_code(tmp_path):
    base = "int f(int x) {\n    return x + 1;   // next\n}\n"
    p = tmp_path / "a.hip"
    p.write_text(base)
    h0 = bench.kernel_code_sha256(str(p))
    p.write_text("// header\n\n" + base.replace("// next", "// the successor") + "\n\n")
    assert bench.kernel_code_sha256(str(p)) == h0
    p.write_text(base.replace("x + 1", "x + 2"))
    assert bench.kernel_code_sha256(str(p)) != h0


def test_traffic_summaries_parse():
    for prefix in bench.TRAFFIC_PROFILES.values():
        names = [f for f in os.listdir(os.path.join(bench.ROOT, "profiles"))
                 if f.startswith(prefix) and f.endswith("_hbm_traffic.md")]
        assert names, prefix
        for name in names:
            text = open(os.path.join(bench.ROOT, "profiles", name)).read()
            sha = re.search(r"- `kernel_code_sha256`: `([0-9a-f]+)`", text)
            tb = re.search(r"- `traffic_bytes_per_launch`: `(\d+)`", text)
            assert sha and len(sha.group(1)) == 64, name
            assert tb and int(tb.group(1)) > 0, name
            assert "rocprofv3 --pmc FETCH_SIZE" in text and "rocprofv3 --pmc WRITE_SIZE" in text, name
