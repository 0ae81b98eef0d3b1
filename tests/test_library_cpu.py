"""Host-side checks of the HIP library that need no GPU: it loads, it exports
every call that include/bcur.h declares, and its status strings are sane."""
import ctypes
import os
import re

import pytest

from paper_1703_06065_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bcur.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bcur_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(binding.LIB_PATH):
        from paper_1703_06065_amd import build
        build.build(verbose=False)
    return binding.load_library()


def test_header_and_binding_agree():
    assert declared_functions() == sorted(binding.SYMBOLS)


def test_library_exports_every_declared_call(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_status_strings(lib):
    assert lib.bcur_status_str(0) == b"ok"
    assert b"argument" in lib.bcur_status_str(1)
    assert lib.bcur_status_str(99) == b"unknown status"


def test_create_rejects_null_out(lib):
    assert lib.bcur_create(None, 0, None, 0) == binding.E_ARG


def test_calls_reject_null_context(lib):
    assert lib.bcur_destroy(None) == binding.E_ARG
    assert lib.bcur_synchronize(None) == binding.E_ARG
    assert lib.bcur_wait(None) == binding.E_ARG
    assert lib.bcur_test_matrix(None, 4, 4, 0, None, 4) == binding.E_ARG
    assert lib.bcur_last_error(None) == b""
