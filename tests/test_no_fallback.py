"""The product path has no CPU fallback: without the built library every entry point of the
binding raises instead of computing anything.  CPU only."""
import pytest

from paper_1801_09803_amd import binding


@pytest.fixture
def no_library(monkeypatch, tmp_path):
    monkeypatch.setattr(binding, "_lib", None)
    monkeypatch.setattr(binding, "lib_path", lambda: str(tmp_path / "libxsec.so"))


def test_plan_creation_raises_without_the_library(no_library):
    with pytest.raises(ImportError, match="is missing"):
        binding.Plan(0.0, 100.0, 1001, 18.0)


def test_loading_raises_without_the_library(no_library):
    with pytest.raises(ImportError, match="is missing"):
        binding.load_library()


def test_nothing_outside_tests_imports_the_oracle():
    import os
    import re
    from tests.conftest import ROOT
    pat = re.compile(r"^\s*(import oracle|from oracle)", re.M)
    offenders = []
    for sub in ("paper_1801_09803_amd", "synth", "include"):
        for dirpath, _, files in os.walk(os.path.join(ROOT, sub)):
            for f in files:
                if f.endswith((".py", ".cpp", ".hip", ".hpp", ".h")):
                    with open(os.path.join(dirpath, f), encoding="utf-8", errors="replace") as fh:
                        if pat.search(fh.read()):
                            offenders.append(os.path.join(dirpath, f))
    assert not offenders, offenders
