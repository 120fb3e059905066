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


def test_partition_inspection_rejects_bad_arguments():
    from paper_2407_07718_amd import kc
    reads = np.frombuffer(b"ACGT" * 20, dtype=np.uint8)
    for k, m, offsets in [(0, 1, [0, 80]), (31, 31, [0, 80]), (64, 21, [0, 80]), (11, 5, [0, 50, 40, 80])]:
        with pytest.raises(kc.KCError) as e:
            kc.kc_partition_inspect(reads, np.array(offsets, dtype=np.uint64), k, m)
        assert e.value.code == kc.KC_EINVAL
    with pytest.raises(kc.KCError) as e:
        kc.kc_partition_inspect(reads, np.array([0, 80], dtype=np.uint64), 31, 15, kc.make_config(log2_buckets=21))
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


def test_largest_input_accepted_and_one_base_more_refused():
    """A count takes at most 2^32 - 1 bases (windows, read indices and positions are
    32-bit); the workspace queries and the host APIs agree on that limit, and the host
    APIs refuse from the offsets alone, before touching the reads."""
    from paper_2407_07718_amd import kc
    top = (1 << 32) - 1
    for k in (31, 51):
        assert kc.kc_workspace_size(top, 300_000, k) > 0
        assert kc.kc_workspace_size(top + 1, 300_000, k) == 0
        assert kc.kc_ext_workspace_size(top, 300_000, k) > 0
        assert kc.kc_ext_workspace_size(top + 1, 300_000, k) == 0
    assert kc.kc_ext_workspace_size(top, 1 << 32, 31) == 0
    reads = np.frombuffer(b"ACGT" * 8, dtype=np.uint8)
    offsets = np.array([0, 1 << 32], dtype=np.uint64)
    with pytest.raises(kc.KCError) as e:
        kc.kc_count(reads, offsets, 31, 17, 2, 50, 16)
    assert e.value.code == kc.KC_EINVAL and "2^32" in str(e.value)
    with pytest.raises(kc.KCError) as e:
        kc.kc_count_ext(reads, offsets, 31, 2, 50, 16)
    assert e.value.code == kc.KC_EINVAL and "2^32" in str(e.value)


def test_header_declares_batch_and_server_entry_points():
    names = declared_functions()
    for n in ["kc_count_batch", "kc_batch_create", "kc_batch_run", "kc_batch_result", "kc_batch_destroy",
              "kc_autotune", "kc_server_create", "kc_server_submit", "kc_server_poll", "kc_server_cancel",
              "kc_server_clock", "kc_server_destroy", "kc_profile", "kc_profile_read"]:
        assert n in names


def test_struct_sizes_match_header_layout():
    from paper_2407_07718_amd import kc
    assert ctypes.sizeof(kc.kc_totals) == 17 * 8
    assert ctypes.sizeof(kc.kc_config) == 4 * 4 + 8 + 4 * 4
    assert ctypes.sizeof(kc.kc_job) == 8 * 3 + 4 * 4 + 8
    assert ctypes.sizeof(kc.kc_server_cfg) == 8 + 2 * 4 + 8 + ctypes.sizeof(kc.kc_config)
    assert ctypes.sizeof(kc.kc_timing) == 3 * 8 + 2 * 8 + 2 * 4


def test_binding_structs_match_the_c_compiler(tmp_path):
    """Every field offset and struct size of the Python binding equals what a C compiler
    makes of include/kc.h."""
    import shutil
    import subprocess
    from paper_2407_07718_amd import kc
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    structs = [kc.kc_config, kc.kc_totals, kc.kc_result, kc.kc_ext_result, kc.kc_job, kc.kc_server_cfg,
               kc.kc_timing, kc.kc_stage_times, kc.kc_partition]
    lines = ["#include <stdio.h>", "#include <stddef.h>", f'#include "{HEADER}"', "int main(void) {"]
    for st in structs:
        name = st.__name__
        lines.append(f'  printf("{name} %zu\\n", sizeof({name}));')
        for f, _ in st._fields_:
            lines.append(f'  printf("{name}.{f} %zu\\n", offsetof({name}, {f}));')
    lines.append("  return 0;\n}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-o", str(exe), str(src)])
    got = dict(line.rsplit(" ", 1) for line in subprocess.check_output([str(exe)], text=True).splitlines())
    for st in structs:
        name = st.__name__
        assert int(got[name]) == ctypes.sizeof(st), name
        for f, _ in st._fields_:
            assert int(got[f"{name}.{f}"]) == getattr(st, f).offset, f"{name}.{f}"


def test_batch_rejects_bad_job_before_device_work():
    from paper_2407_07718_amd import kc
    reads = np.frombuffer(b"ACGT" * 20, dtype=np.uint8)
    good = kc.Job(reads, np.array([0, 80], dtype=np.uint64), 31, 15, 2, 10, 16)
    bad_m = kc.Job(reads, np.array([0, 80], dtype=np.uint64), 31, 31, 2, 10, 16)
    bad_off = kc.Job(reads, np.array([0, 50, 40, 80], dtype=np.uint64), 11, 5, 1, 10, 16)
    for jobs in ([good, bad_m], [bad_off, good]):
        with pytest.raises(kc.KCError) as e:
            kc.kc_count_batch(jobs)
        assert e.value.code == kc.KC_EINVAL


def test_server_rejects_bad_arguments_on_host():
    from paper_2407_07718_amd import kc
    with pytest.raises(kc.KCError) as e:
        kc.Server(hbm_budget=1000)
    assert e.value.code == kc.KC_EINVAL
    lib = kc._lib
    t = ctypes.c_uint64()
    assert lib.kc_server_submit(None, None, ctypes.byref(t)) == kc.KC_EINVAL
    assert lib.kc_server_poll(None, 1, None, None) == kc.KC_EINVAL
    assert lib.kc_server_cancel(None, 1) == kc.KC_EINVAL
    assert lib.kc_server_destroy(None) == kc.KC_OK


def test_header_declares_extension_entry_points():
    names = declared_functions()
    for n in ["kc_count_ext", "kc_ext_result_free", "kc_ext_workspace_size", "kc_count_ext_device",
              "kc_count_ext_device_async"]:
        assert n in names


def test_extension_struct_layout():
    from paper_2407_07718_amd import kc
    assert ctypes.sizeof(kc.kc_ext_result) == ctypes.sizeof(kc.kc_result) + 8 + 3 * 8


@pytest.mark.parametrize("k,lo,hi,H", [(0, 2, 3, 16), (64, 2, 3, 16), (31, 0, 3, 16), (31, 5, 3, 16),
                                      (31, 2, 3, 1)])
def test_extension_host_api_rejects_bad_arguments(k, lo, hi, H):
    from paper_2407_07718_amd import kc
    reads = np.frombuffer(b"ACGT" * 20, dtype=np.uint8)
    with pytest.raises(kc.KCError) as e:
        kc.kc_count_ext(reads, np.array([0, 80], dtype=np.uint64), k, lo, hi, H)
    assert e.value.code == kc.KC_EINVAL
    with pytest.raises(kc.KCError) as e:
        kc.kc_count_ext(reads, np.array([0, 50, 40, 80], dtype=np.uint64), 11, 1, 10, 16)
    assert e.value.code == kc.KC_EINVAL and "decrease" in str(e.value)


def test_extension_workspace_size_scales():
    from paper_2407_07718_amd import kc
    a = kc.kc_ext_workspace_size(1_000_000, 10_000, 31)
    b = kc.kc_ext_workspace_size(2_000_000, 20_000, 31)
    c = kc.kc_ext_workspace_size(1_000_000, 10_000, 51)
    assert 0 < a < b and c > a
    assert kc.kc_ext_workspace_size(1000, 10, 0) == 0 and kc.kc_ext_workspace_size(1000, 10, 64) == 0
