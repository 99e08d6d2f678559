"""The launch cost model of the sweeps, compiled host-only from the library's
header and run on the CPU: z chunks and the FP32 tile height it picks match
a restatement of the model and the choices the measurements rest on."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _model(nx, ny, nz, by, bx=66, kz_max=256, kz_min=4, cus=256):
    """Cheapest chunk of {kz_max, ..., kz_min} by ceil(blocks/cus) rounds of
    (chunk + 2) plane steps (longer chunk on ties); returns (chunk, cost x rows)."""
    tiles = ((nx + bx - 3) // (bx - 2)) * ((ny + by - 3) // (by - 2))
    best, best_cost, kz = kz_max, None, kz_max
    while kz >= kz_min:
        blocks = tiles * ((nz + kz - 1) // kz)
        cost = ((blocks + cus - 1) // cus) * (min(kz, nz) + 2)
        if best_cost is None or cost < best_cost:
            best, best_cost = kz, cost
        kz //= 2
    return best, best_cost * by


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


def test_probe_matches_the_model(probe):
    got = probe(SHAPES)
    for s in SHAPES:
        kz_thesis, kz_fp32_tall, short = got[s]
        assert kz_thesis == _model(*s, by=10)[0], s
        assert kz_fp32_tall == _model(*s, by=14)[0], s
        assert bool(short) == (_model(*s, by=10)[1] < _model(*s, by=14)[1]), s


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
