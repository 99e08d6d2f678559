"""The launch cost model of the sweeps, compiled host-only from the library's
header and run on the CPU: the z chunks and the FP32 tile height it picks are
the choices the measurements rest on."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def probe(tmp_path_factory):
    if not shutil.which(HIPCC) and not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("probe") / "probe")
    subprocess.run([HIPCC, "-x", "hip", "--offload-arch=gfx950", "--offload-host-only",
                    "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2207_08716_amd", "csrc"),
                    os.path.join(ROOT, "tests", "cost_model_probe.hip"), "-o", exe],
                   check=True, capture_output=True)

    def run(shapes):
        args = [str(v) for s in shapes for v in s]
        out = subprocess.run([exe, *args], check=True, capture_output=True, text=True).stdout.split("\n")
        return {tuple(map(int, l.split()[:3])): tuple(map(int, l.split()[3:])) for l in out if l.strip()}
    return run


SHAPES = [(2, 2, 2), (16, 16, 16), (63, 63, 63), (127, 127, 127), (191, 191, 191), (255, 255, 255),
          (383, 383, 383), (511, 511, 511), (767, 767, 767), (192, 84, 32), (70, 13, 130), (3, 64, 5)]


def test_choices_the_measurements_rest_on(probe):
    got = probe(SHAPES)
    # FP32 correction sweep: 10-row tiles up to 255^3, 14-row ones from 383^3
    for n in (63, 127, 191, 255):
        assert got[(n, n, n)][2] == 1, n
    for n in (383, 511, 767):
        assert got[(n, n, n)][2] == 0, n
    assert got[(192, 84, 32)][2] == 0          # the grid of the tall-tile GPU test
    # 511^3 thesis sweep: 256-plane chunks, 8 x 64 tiles -> 1024 blocks, 4 full rounds
    assert got[(511, 511, 511)][0] == 256
    # 63^3: short chunks, so that the blocks fill the compute units
    assert got[(63, 63, 63)][0] == 4
