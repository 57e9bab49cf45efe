import os
import shutil
import subprocess
import sys

import pytest

REPO = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if REPO not in sys.path:
    sys.path.insert(0, REPO)

PINS = os.path.join(REPO, "tests", "pins")
TORCH_INCLUDE = None


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP C-ABI)")


@pytest.fixture(scope="session")
def pin_bin(tmp_path_factory):
    """Compile the pin helpers (enumerator, Philox harnesses) once per session."""
    d = tmp_path_factory.mktemp("pins")
    built = {}

    def get(name):
        if name in built:
            return built[name]
        out = str(d / name)
        if name == "saw_enum":
            subprocess.check_call(["gcc", "-O2", "-o", out, os.path.join(PINS, "saw_enum.c")])
        elif name == "philox_torch":
            import torch
            inc = os.path.join(os.path.dirname(torch.__file__), "include")
            subprocess.check_call(["g++", "-O1", "-std=c++17", "-I", inc, "-o", out,
                                   os.path.join(PINS, "philox_torch.cpp")])
        elif name == "philox_rocrand":
            hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
            subprocess.check_call([hipcc, "-O1", "-std=c++17", "-o", out,
                                   os.path.join(PINS, "philox_rocrand.cpp")])
        else:
            raise KeyError(name)
        built[name] = out
        return out

    return get


_ENUM_CACHE = {}


@pytest.fixture(scope="session")
def saw_enum(pin_bin):
    """Exact enumeration of n-step SAWs: dict(c, sum_r2, sum_n2rg2, w_hist, traps)."""
    def run(n):
        if n in _ENUM_CACHE:
            return _ENUM_CACHE[n]
        txt = subprocess.check_output([pin_bin("saw_enum"), str(n)], text=True)
        res = dict(w_hist={}, traps={})
        for line in txt.splitlines():
            f = line.split()
            if f[0] == "w":
                res["w_hist"][int(f[1])] = int(f[2])
            elif f[0] == "trap":
                res["traps"][(int(f[1]), int(f[2]))] = int(f[3])
            else:
                res[f[0]] = int(f[1])
        _ENUM_CACHE[n] = res
        return res
    return run
