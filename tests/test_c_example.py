"""The C example in README.md compiles as C99 against include/hh.h and links
against libhh.so and the HIP runtime (no GPU needed; nothing is run)."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB_DIR = os.path.join(ROOT, "paper_1612_06257_amd")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def test_readme_c_example_compiles_and_links(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    if not os.path.exists(os.path.join(LIB_DIR, "libhh.so")):
        pytest.skip("libhh.so is not built")
    readme = open(os.path.join(ROOT, "README.md")).read()
    blocks = re.findall(r"```c\n(.*?)```", readme, re.S)
    assert blocks, "README.md has no C example"
    src = tmp_path / "example.c"
    src.write_text(blocks[0])
    cmd = ["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROCM, "include"), str(src),
           "-L", LIB_DIR, "-lhh", "-L", os.path.join(ROCM, "lib"), "-lamdhip64",
           "-o", str(tmp_path / "example")]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
