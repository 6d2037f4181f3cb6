"""The benchmark's command-line contract that can be checked without a GPU:
more than one GPU is refused with a message, the help text lists every
configuration, and the sweep's traffic record is tied to the kernel source."""

import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_help_lists_every_configuration():
    r = run("--help")
    assert r.returncode == 0
    for name in ("headline", "masks", "precision", "loops", "blocks"):
        assert name in r.stdout


def test_traffic_record_names_its_kernel_source():
    rec = json.load(open(os.path.join(ROOT, "profiles", "sweep_f32_257x257x513_traffic.json")))
    assert len(rec["kernel_source_sha256_16"]) == 16
    assert set(rec["tile"]) == {"vec", "rows", "kchunk", "flags", "occupancy"}
    assert rec["hbm_bytes_per_launch"] == rec["hbm_read_bytes_per_launch"] + rec["hbm_write_bytes_per_launch"]
    assert rec["algorithmic_bytes_per_launch"] == 56 * 255 * 255 * 511


def test_traffic_record_is_for_the_current_kernel_source():
    """The benchmark reports counter traffic only for the kernel source it was
    taken on; the committed record must match the committed kernels."""
    import hashlib

    rec = json.load(open(os.path.join(ROOT, "profiles", "sweep_f32_257x257x513_traffic.json")))
    src = os.path.join(ROOT, "paper_2011_03602_amd", "csrc", "kernels.hip")
    assert rec["kernel_source_sha256_16"] == hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
