"""CPU checks of the C-ABI: the built library loads without a GPU and
exports every entry point declared in include/sch.h; the binding declares the
same set.  No compute calls are made here."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sch.h")
LIB = os.path.join(ROOT, "paper_2402_06927_amd", "libsch.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(sch_[a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def libsch():
    if not os.path.exists(LIB):
        import __graft_entry__

        __graft_entry__.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_filter_calls():
    names = declared_functions()
    for required in ("sch_ensemble_step", "sch_loglik", "sch_temper_ess", "sch_resample",
                     "sch_jitter_pcn"):
        assert required in names


def test_library_exports_every_declared_symbol(libsch):
    missing = [n for n in declared_functions() if not hasattr(libsch, n)]
    assert not missing, missing


def test_binding_matches_header():
    from paper_2402_06927_amd import sch

    assert sorted(sch.exported_names()) == declared_functions()


def test_error_paths_without_gpu(libsch):
    """Argument validation runs on the host before anything touches the GPU."""
    libsch.sch_last_error.restype = ctypes.c_char_p
    libsch.sch_ensemble_step.restype = ctypes.c_int
    rc = libsch.sch_ensemble_step(None, 1, 1, None, None, None, None, None, None, None)
    assert rc == -1
    assert b"model" in libsch.sch_last_error()
    libsch.sch_temper_ess.restype = ctypes.c_int
    rc = libsch.sch_temper_ess(0, None, None, None, ctypes.c_double(1.0), 0, None, None, None,
                               None, None)
    assert rc == -1
