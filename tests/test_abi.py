"""The C-ABI library loads and exports every symbol include/kc.h declares; argument
checks that run before any device call reject bad input (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kc.h")
LIB = os.path.join(ROOT, "paper_2407_07718_amd", "libkc.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(kc_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_entry_points():
    names = declared_functions()
    for n in ["kc_count", "kc_count_device", "kc_count_device_async", "kc_workspace_size", "kc_result_free",
              "kc_last_error", "kc_version"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "libkc.so not built"
    lib = ctypes.CDLL(LIB)
    for n in declared_functions():
        assert hasattr(lib, n), f"{n} not exported"


def test_binding_imports_and_versions():
    from paper_2407_07718_amd import kc
    assert "gfx950" in kc.kc_version()


@pytest.mark.parametrize("k,m,lo,hi,H", [(0, 1, 2, 3, 16), (64, 20, 2, 3, 16), (31, 31, 2, 3, 16),
                                        (31, 0, 2, 3, 16), (40, 33, 2, 3, 16), (31, 15, 0, 3, 16),
                                        (31, 15, 5, 3, 16), (31, 15, 2, 3, 1)])
def test_host_api_rejects_bad_arguments(k, m, lo, hi, H):
    from paper_2407_07718_amd import kc
    reads = np.frombuffer(b"ACGT" * 20, dtype=np.uint8)
    offsets = np.array([0, 80], dtype=np.uint64)
    with pytest.raises(kc.KCError) as e:
        kc.kc_count(reads, offsets, k, m, lo, hi, H)
    assert e.value.code == kc.KC_EINVAL


def test_host_api_rejects_decreasing_offsets():
    from paper_2407_07718_amd import kc
    reads = np.frombuffer(b"ACGT" * 20, dtype=np.uint8)
    offsets = np.array([0, 50, 40, 80], dtype=np.uint64)
    with pytest.raises(kc.KCError) as e:
        kc.kc_count(reads, offsets, 11, 5, 1, 10, 16)
    assert e.value.code == kc.KC_EINVAL and "decrease" in str(e.value)


def test_workspace_size_scales():
    from paper_2407_07718_amd import kc
    a = kc.kc_workspace_size(1_000_000, 10_000, 31)
    b = kc.kc_workspace_size(2_000_000, 20_000, 31)
    c = kc.kc_workspace_size(1_000_000, 10_000, 51)
    assert 0 < a < b and c > a
    assert kc.kc_workspace_size(1000, 10, 0) == 0
    assert kc.kc_workspace_size(1000, 10, 64) == 0
