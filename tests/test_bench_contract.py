"""bench.py's contract on the CPU: a run on more than one GPU is refused with
a message before any device work, and the committed counter records under
profiles/ were taken on the kernel sources as they stand (bench.py reports
their traffic only while the hash of those sources matches)."""
import glob
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and "not implemented" in r.stderr


def test_traffic_records_match_the_kernel_sources():
    recs = sorted(glob.glob(os.path.join(ROOT, "profiles", "traffic_*.json")))
    assert recs, "no counter records under profiles/"
    sha = bench.kernel_sha()
    for path in recs:
        with open(path) as fh:
            rec = json.load(fh)
        assert rec["kernel_sha"] == sha, f"{os.path.basename(path)} was taken on other kernel sources"
        assert rec["hbm_bytes_per_launch"] > 0
        assert os.path.exists(os.path.join(ROOT, rec["summary"])), rec["summary"]
        kernel, workload = rec["kernel"], rec["workload"]
        assert bench.stored_traffic(workload, kernel) == rec["hbm_bytes_per_launch"]


def test_kernel_hash_ignores_comments_and_layout(tmp_path):
    """The hash covers code, not comments or blank space: rewording a comment
    keeps the counter records valid, changing a line of code does not."""
    import shutil
    src = os.path.join(ROOT, "paper_1609_07008_amd", "csrc")
    for f in bench.KERNEL_SOURCES:
        shutil.copy(os.path.join(src, f), tmp_path / f)
    base = bench.kernel_sha(str(tmp_path))
    assert base == bench.kernel_sha()
    k = tmp_path / "products.h"
    text = k.read_text()
    k.write_text("// a reworded note\n/* and a block\n   comment */\n" + text.replace("\n", "\n\n", 3))
    assert bench.kernel_sha(str(tmp_path)) == base
    k.write_text(text.replace("kTau16Big = 0xfffeu", "kTau16Big = 0xfffdu", 1))
    assert bench.kernel_sha(str(tmp_path)) != base
