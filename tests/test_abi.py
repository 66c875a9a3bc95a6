"""The C ABI library loads and exports every function include/*.h declares
(no GPU needed: nothing is called except the version string)."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1712_04495_amd", "libsched.so")


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w \*]*?\b(sched_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    import torch  # noqa: F401  (same HIP runtime as the binding)
    return ctypes.CDLL(LIB)


def test_header_declares_lifecycle():
    names = declared_functions()
    for n in ("sched_register", "sched_admit", "sched_alloc", "sched_release", "sched_wait"):
        assert n in names, n


def test_every_declared_symbol_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_exports(lib):
    from paper_1712_04495_amd import cosched
    cosched.lib()
    for n in cosched._SIGS:
        assert hasattr(lib, n)
    assert cosched.sched_version().startswith("sched-mi355x")


def test_struct_layouts_match_binding(lib):
    """Every structure the ABI passes has the size the binding assumes
    (a host-only call: no device is touched)."""
    from paper_1712_04495_amd import cosched
    for k, (theirs, mine) in enumerate(cosched.abi_layouts()):
        assert theirs == mine, (k, theirs, mine)
    assert cosched.lib().sched_abi_sizeof(99) == -1
