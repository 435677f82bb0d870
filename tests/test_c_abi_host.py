"""The C ABI from plain C (no GPU needed): tests/c/abi_demo.c compiles with
-Wall -Werror against include/pf.h and links against libpfiso.so."""
import os

import pytest

from c_abi_build import build_demo, PKG


def test_c_program_builds_against_header(tmp_path):
    if not os.path.exists(os.path.join(PKG, "libpfiso.so")):
        pytest.skip("libpfiso.so not built")
    rc, err = build_demo(str(tmp_path / "abi_demo"))
    assert rc == 0, err
