import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: longer CPU test")


@pytest.fixture(scope="session")
def orc():
    from oracle import oracle as O
    if not os.path.exists(O.LIB):
        O.build(force=True)
    return O.default()


@pytest.fixture(scope="session")
def rocrand_ref(tmp_path_factory):
    """Host build of the rocRAND Philox reference helper; yields a query function."""
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND reference")
    exe = str(tmp_path_factory.mktemp("rocrand") / "rocrand_stream")
    src = os.path.join(ROOT, "tests", "rocrand_stream.cpp")
    subprocess.run([hipcc, "-O1", "--offload-arch=gfx950", src, "-o", exe], check=True,
                   stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)

    def query(lines):
        out = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True, check=True)
        return [[int(w, 16) for w in ln.split()] for ln in out.stdout.strip().splitlines()]

    return query
