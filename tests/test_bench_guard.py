"""The guard that keeps a profiled traffic figure in the bench line only
while the forward kernels are the ones profiled: the hash of the kernel
code ignores comments and layout but not code, nor the build flags of
its sources."""
import os
import shutil

import bench


def _hash_with(tmp_path, name, edit):
    csrc = os.path.join(bench.ROOT, "paper_2102_01747_amd", "csrc")
    dst = tmp_path / "paper_2102_01747_amd" / "csrc"
    dst.mkdir(parents=True, exist_ok=True)
    for f in bench.KERNEL_SOURCES:
        shutil.copy(os.path.join(csrc, f), dst / f)
    if edit is not None:
        p = dst / name
        p.write_text(edit(p.read_text()))
    root = bench.ROOT
    try:
        bench.ROOT = str(tmp_path)
        return bench.kernel_sources_sha256()
    finally:
        bench.ROOT = root


def test_hash_matches_the_tree(tmp_path):
    assert _hash_with(tmp_path, None, None) == bench.kernel_sources_sha256()


def test_comments_and_layout_do_not_change_the_hash(tmp_path):
    base = _hash_with(tmp_path, None, None)
    assert _hash_with(tmp_path, "frt_trace.hip", lambda s: "// a new comment\n/* and\n another */\n" + s) == base
    assert _hash_with(tmp_path, "frt_job.hpp", lambda s: s.replace("\n", "\n\n", 5)) == base


def test_code_changes_the_hash(tmp_path):
    base = _hash_with(tmp_path, None, None)
    assert _hash_with(tmp_path, "frt_trace.hip", lambda s: s.replace("kMaxBodiesPerTrip = 64", "kMaxBodiesPerTrip = 32")) != base


def test_build_flags_change_the_hash(monkeypatch):
    from paper_2102_01747_amd import _build

    base = bench.kernel_sources_sha256()
    flags = dict(_build.SOURCE_FLAGS)
    flags["frt_trace.hip"] = [f for f in flags.get("frt_trace.hip", []) if f != "-fno-signed-zeros"]
    monkeypatch.setattr(_build, "SOURCE_FLAGS", flags)
    assert bench.kernel_sources_sha256() != base
