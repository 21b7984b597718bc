"""The C example of the README compiles and links against the library."""
import os
import re
import subprocess

from paper_2307_03466_amd import pdhg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _build(tmp_path):
    text = open(os.path.join(ROOT, "README.md")).read()
    src = re.search(r"```c\n(.*?)```", text, re.S).group(1)
    c = tmp_path / "example.c"
    c.write_text(src)
    if not os.path.exists(pdhg.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    exe = tmp_path / "example"
    libdir = os.path.dirname(pdhg.LIB_PATH)
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(c), "-L", libdir,
                    "-lscylla_pdhg", "-Wl,-rpath," + libdir], check=True, timeout=120)
    return exe


def test_readme_c_example_builds(tmp_path):
    assert _build(tmp_path).exists()
