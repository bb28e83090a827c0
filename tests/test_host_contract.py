"""Host-side contract checks on the CPU: the benchmark refuses more than one
GPU with a message, and the product package refuses to import without its
HIP library (there is no CPU fallback)."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_several_gpus():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert p.returncode != 0
    assert "one GPU" in p.stderr
    assert p.stdout.strip() == ""


def test_package_import_fails_without_library(tmp_path):
    """A copy of the Python package without libclamp.so must raise on import."""
    import shutil
    pkg = tmp_path / "paper_2406_13651_amd"
    shutil.copytree(os.path.join(ROOT, "paper_2406_13651_amd"), pkg,
                    ignore=shutil.ignore_patterns("*.so", "_build", "__pycache__", "csrc"))
    code = "import paper_2406_13651_amd"
    p = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300, cwd=tmp_path,
                       env={**os.environ, "PYTHONPATH": str(tmp_path)})
    assert p.returncode != 0
    assert "libclamp.so is not built" in p.stderr


def test_build_script_loads_without_the_library(tmp_path):
    """build() must work in a fresh checkout, where libclamp.so does not exist
    yet: the build script is loaded without importing the package."""
    import shutil
    shutil.copytree(os.path.join(ROOT, "paper_2406_13651_amd"), tmp_path / "paper_2406_13651_amd",
                    ignore=shutil.ignore_patterns("*.so", "_build", "__pycache__"))
    shutil.copy(os.path.join(ROOT, "__graft_entry__.py"), tmp_path)
    code = ("import sys, __graft_entry__ as g; m = g._build_module(); "
            "assert callable(m.build) and 'paper_2406_13651_amd' not in sys.modules")
    p = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300, cwd=tmp_path,
                       env={**os.environ, "PYTHONPATH": str(tmp_path)})
    assert p.returncode == 0, p.stderr
