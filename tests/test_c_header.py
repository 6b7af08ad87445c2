"""The C header compiles as plain C11 with warnings as errors, and a C caller
can pass every argument with its declared type (no GPU needed)."""

import os
import re
import shutil
import subprocess

import pytest

from paper_2211_09938_amd import cgh

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CALLS = os.path.join(HERE, "c_abi_calls.c")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
@pytest.mark.parametrize("std", ["c11", "c17"])
def test_header_compiles_as_c_with_typed_calls(tmp_path, std):
    obj = tmp_path / "calls.o"
    r = subprocess.run(["gcc", f"-std={std}", "-Wall", "-Wextra", "-Werror", "-pedantic",
                        "-I", os.path.join(ROOT, "include"), "-c", CALLS, "-o", str(obj)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_every_declared_function_is_called_from_c():
    with open(CALLS) as f:
        text = f.read()
    called = set(re.findall(r"\b(cgh_[a-z_0-9]+)\s*\(", text)) - {"cgh_header_calls"}
    assert called == set(cgh.header_functions())
