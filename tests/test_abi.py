"""The C ABI library loads on the host and exports every function include/cabinrom.h declares
(no compute call: there is no GPU here); the benchmark refuses more than one GPU."""
import ctypes
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2310_04734_amd", "libcabinrom.so")


def declared():
    src = open(os.path.join(ROOT, "include", "cabinrom.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cr_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ["cr_assemble", "cr_analyse", "cr_factor", "cr_solve", "cr_basis_build", "cr_basis_build_greedy",
                 "cr_project", "cr_sweep", "cr_sweep_batched", "cr_mlp_train_step"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "build the library first (paper_2310_04734_amd/build.py)"
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True)
    assert r.returncode == 2 and "one GPU" in r.stdout
