"""The Python binding (CPU): no fallback when the native library is absent."""
import pytest


def test_product_fails_loudly_without_the_library(tmp_path, monkeypatch):
    """With the native library absent, loading raises instead of computing anything elsewhere."""
    from paper_1606_06790_amd import lib
    monkeypatch.setattr(lib, "LIB_PATH", str(tmp_path / "libidmrg.so"))
    monkeypatch.setattr(lib, "_lib", None)
    with pytest.raises(RuntimeError, match="missing"):
        lib.load()
