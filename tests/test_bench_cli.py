"""bench.py command line on the host: more than one GPU is refused with a
message and a non-zero exit status, before any GPU work."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert res.returncode != 0
    assert "one GPU" in (res.stdout + res.stderr)


def test_kernel_source_hash_ignores_comments_only(tmp_path, monkeypatch):
    """The hash that ties committed counter runs to the kernel sources covers
    their code: a comment or blank-line edit keeps it, a code edit changes it."""
    import shutil

    sys.path.insert(0, ROOT)
    import bench

    src = os.path.join(ROOT, "paper_2606_12650_amd", "csrc")
    dst = tmp_path / "paper_2606_12650_amd" / "csrc"
    shutil.copytree(src, dst)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    base_k, base_c = bench._kernel_source_hash(), bench._cg_source_hash()
    f = dst / "sem_cg_dev.h"
    text = f.read_text()
    f.write_text("// a new comment line\n\n" + text.replace("\n", "  /* note */\n", 1))
    assert bench._cg_source_hash() == base_c and bench._kernel_source_hash() == base_k
    f.write_text(text + "\nnamespace semk { constexpr int kProbe = 1; }\n")
    assert bench._cg_source_hash() != base_c
    assert bench._kernel_source_hash() == base_k  # not one of the operator's sources
