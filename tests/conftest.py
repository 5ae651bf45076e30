import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: longer statistical checks")


# Independent Philox4x32-10: PyTorch's header-only engine compiled for the host.
_PROG = r"""
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdio>
int main() {
  unsigned k0, k1, c0, c1, c2, c3;
  while (std::scanf("%u %u %u %u %u %u", &k0, &k1, &c0, &c1, &c2, &c3) == 6) {
    uint64_t seed = (uint64_t)k0 | ((uint64_t)k1 << 32);
    uint64_t sub = (uint64_t)c2 | ((uint64_t)c3 << 32);
    uint64_t off = (uint64_t)c0 | ((uint64_t)c1 << 32);
    at::philox_engine e(seed, sub, off);
    unsigned o0 = e(), o1 = e(), o2 = e(), o3 = e();
    std::printf("%u %u %u %u\n", o0, o1, o2, o3);
  }
  return 0;
}
"""


@pytest.fixture(scope="session")
def torch_philox(tmp_path_factory):
    torch = pytest.importorskip("torch")
    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    d = tmp_path_factory.mktemp("philox_ref")
    src = d / "ref.cpp"
    exe = d / "ref"
    src.write_text(_PROG)
    subprocess.check_call(["g++", "-O1", "-std=c++17", f"-I{inc}", "-o", str(exe), str(src)])

    def run(rows):
        text = "\n".join(" ".join(str(int(v)) for v in row) for row in rows) + "\n"
        out = subprocess.run([str(exe)], input=text, capture_output=True, text=True, check=True)
        return np.array([[int(v) for v in line.split()] for line in out.stdout.strip().splitlines()],
                        dtype=np.uint64)

    return run


