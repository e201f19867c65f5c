"""The register DFTs of the HIP kernels (csrc/fft_reg.hpp, host-callable)
against the O(N^2) DFT definition in double, for every factor P and Q of a
compiled transform length.  Built with hipcc, run on the CPU."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _factors():
    out = set()
    with open(os.path.join(ROOT, "paper_2003_07504_amd", "csrc", "lengths.def")) as fh:
        for line in fh:
            m = re.match(r"\s*ILS_LEN\((\d+),\s*(\d+),\s*(\d+)\)", line)
            if m:
                out.update({int(m.group(2)), int(m.group(3))})
    return out


@pytest.fixture(scope="module")
def results(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("dft") / "dft_check")
    subprocess.run([HIPCC, "-x", "hip", "-O2", "-std=c++17", "--offload-arch=gfx950",
                    os.path.join(ROOT, "tests", "native", "dft_check.cpp"), "-o", exe],
                   check=True, capture_output=True)
    out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    return {int(n): (float(a), float(b)) for n, a, b in (ln.split() for ln in out.strip().splitlines())}


def test_every_compiled_factor_is_checked(results):
    assert _factors() <= set(results)


def test_register_dfts_match_definition(results):
    for n, (fwd, inv) in results.items():
        assert fwd < 1e-6 and inv < 1e-6, (n, fwd, inv)
