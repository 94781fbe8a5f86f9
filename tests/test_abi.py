"""CPU checks of the boundary: libkc.so loads (no GPU needed) and exports every
entry point include/kc.h declares; the binding fails loudly without the library."""
import os
import re

import pytest

from paper_1403_0734_amd import kc as K

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "kc.h")).read()
    return sorted(set(re.findall(r"^\s*(?:kc_status|void|const char \*)\s*(kc_\w+)\s*\(", text, re.M)))


def test_header_lists_the_abi():
    names = declared_symbols()
    assert "kc_orient" in names and "kc_count" in names and "kc_count_colored" in names
    assert sorted(K.EXPORTS) == names


def test_library_exports_every_declared_symbol():
    lib = K.load()
    for name in declared_symbols():
        assert hasattr(lib, name), name


def test_status_strings():
    lib = K.load()
    assert lib.kc_status_str(K.KC_OK) == b"ok"
    assert b"invalid" in lib.kc_status_str(K.KC_EINVAL)


def test_missing_library_raises(tmp_path):
    saved = K._lib
    try:
        K._lib = None
        with pytest.raises(ImportError):
            K.load(str(tmp_path / "nope.so"))
    finally:
        K._lib = saved


def test_null_arguments_rejected_without_device():
    # argument checks run before any HIP call
    with pytest.raises(K.KcError) as e:
        K.kc_graph_create(None, None, 5, 10, False, None)
    assert e.value.status == K.KC_EINVAL
    with pytest.raises(K.KcError) as e:
        K.kc_count(None, 3)
    assert e.value.status == K.KC_EINVAL


def test_peaks_library_exports_its_header():
    """The peak microbenchmark library exports every kcp_ entry point its header
    declares (no GPU needed to load it)."""
    from paper_1403_0734_amd import peaks
    text = open(os.path.join(ROOT, "include", "kc_peaks.h")).read()
    names = sorted(set(re.findall(r"^\s*int\s+(kcp_\w+)\s*\(", text, re.M)))
    assert names == sorted(peaks.EXPORTS)
    lib = peaks.load()
    for name in names:
        assert hasattr(lib, name), name

