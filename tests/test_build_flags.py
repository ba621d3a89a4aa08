"""The build's per-file code-generation flags name files it compiles, and the
kernel hash that validates the committed counter profiles covers them."""
import os

from paper_2401_07965_amd import build as B


def test_per_file_flags_name_compiled_sources():
    names = {os.path.basename(s) for s in B.SOURCES}
    for f in B.FILE_FLAGS:
        assert f in names, f
    for s in B.SOURCES:
        assert os.path.exists(s), s


def test_kernel_hash_covers_the_flags(monkeypatch):
    import bench
    h0 = bench.kernel_source_hash()
    monkeypatch.setattr(B, "FILE_FLAGS", {})
    assert bench.kernel_source_hash() != h0
