"""Reactive porosity waves (thesis article 3): the HIP sweep through the C ABI
against the FP64 oracle, element by element.

* fixed iteration counts that cross pseudo-step refreshes and checks, on
  the two-anomaly workload and on ragged random grids (several x tiles, a
  ragged y tile, several z chunks), for both Damkoehler numbers;
* whole physical steps with the stopping rule: the same iteration counts;
* the stopping quantity itself;
* at the benchmark's size (506 x 506 x 2042, the paper's global grid) in the
  launch configuration it times: sampled cells against the oracle run on
  windows (after m iterations a cell depends only on cells within m of it;
  the pseudo step, a maximum over the whole grid, is passed in);
* a non-finite state is reported as divergence.
"""
import numpy as np
import pytest

from oracle.reactive import ReactiveOracle
from paper_2207_08716_amd import inputs

pytestmark = pytest.mark.gpu

FIELDS = ("xs", "pf", "phi", "dpfdt")
TOL = 1e-12


def _random_phi(shape, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return 1e-2 * (1.0 + 1.5 * rng.random(shape))


def _compare(w, o, tol=TOL):
    worst = {}
    for name in FIELDS:
        got, ref = w.get(name), o.f[name]
        scale = np.abs(ref).max()
        worst[name] = float(np.abs(got - ref).max() / scale) if scale > 0 else float(np.abs(got).max())
    print(worst, flush=True)
    assert all(v <= tol for v in worst.values()), worst


def _err_tol(o, tol=TOL):
    """The stopping quantity is a one-iteration change, max |x^(k+1) - x^k|
    over phi, Pf/10 and Xs: with each field within tol of its scale, the two
    sides' values differ by at most 2 tol times the largest scale (the
    change itself is far smaller than the fields, so a relative bound on it
    would ask for more digits than the fields carry)."""
    scale = max(np.abs(o.f["phi"]).max(), np.abs(o.f["pf"]).max() / 10.0, np.abs(o.f["xs"]).max())
    return 2.0 * tol * scale


def _pair(ph, nx, ny, nz, phi):
    from paper_2207_08716_amd.waves import Waves
    return Waves(ph, nx, ny, nz, phi), ReactiveOracle(ph, nx, ny, nz, phi)


@pytest.mark.parametrize("case", ["anomalies_da100", "anomalies_da0.01", "ragged_70x13x41", "ragged_33x66x9"])
def test_fixed_iterations_match_the_oracle(case):
    if case.startswith("anomalies"):
        cfg = inputs.config_reactive(16, da=float(case.split("da")[1]), nz=64)
        ph, (nx, ny, nz), phi = cfg.phys, (cfg.nx, cfg.ny, cfg.nz), inputs.porosity_field(cfg)
    else:
        nx, ny, nz = (int(v) for v in case.split("_")[1].split("x"))
        ph = inputs.WavePhysics(lx=nx * 0.3, ly=ny * 0.3, lz=nz * 0.3)
        phi = _random_phi((nz, ny, nx), nx * 1000 + nz)
    w, o = _pair(ph, nx, ny, nz, phi)
    w.begin_step()
    o.begin_step()
    w.iterate(25)        # pseudo steps before 1, 11, 21; checks after 10, 20
    o.iterate(25)
    _compare(w, o)
    assert abs(w.last_error() - o.last_err) <= _err_tol(o)
    # a second physical step continues from the first
    w.begin_step()
    o.begin_step()
    w.iterate(12)
    o.iterate(12)
    _compare(w, o)
    assert np.abs(o.f["pf"]).max() > 0 and np.abs(o.f["xs"] - o.f["xs_old"]).max() > 0


@pytest.mark.parametrize("da", [100.0, 0.01])
def test_physical_steps_with_the_stopping_rule(da):
    cfg = inputs.config_reactive(12, da=da, nz=48)
    ph = cfg.phys
    w, o = _pair(ph, cfg.nx, cfg.ny, cfg.nz, inputs.porosity_field(cfg))
    for _ in range(3):
        w.begin_step()
        o.begin_step()
        it_w, err_w, ok = w.solve_step(ph.eps, 5000)
        it_o, err_o = o.solve_step(ph.eps, 5000)
        assert ok and it_w == it_o, (it_w, it_o)
        assert abs(err_w - err_o) <= _err_tol(o, 1e-11)
        _compare(w, o, 1e-11)


def test_iteration_cap_is_reported_and_leaves_a_valid_state():
    from paper_2207_08716_amd import abi
    cfg = inputs.config_reactive(12, nz=48)
    w, o = _pair(cfg.phys, cfg.nx, cfg.ny, cfg.nz, inputs.porosity_field(cfg))
    w.begin_step()
    o.begin_step()
    it, err, ok = w.solve_step(1e-30, 15)      # 15: not a multiple of nup
    o.iterate(15)
    assert not ok and it == 15 and abs(err - o.last_err) <= _err_tol(o)
    _compare(w, o)
    w.set("pf", np.where(np.arange(12)[None, None, :] == 5, np.nan, w.get("pf")))
    with pytest.raises(abi.PTError) as e:
        w.solve_step(1e-8, 40)
    assert e.value.status == -3


def _sample_points(nx, ny, nz, rng, count):
    """Corners, x/y tile seams (64 x 8 tiles), every possible z-chunk seam
    (chunks are powers of two up to 256) and random cells."""
    pts = set()
    for k in (0, nz - 1):
        for j in (0, ny - 1):
            for i in (0, nx - 1):
                pts.add((k, j, i))
    for k in (255, 256, 1023, 1024, nz - 2):
        for i in (63, 64, 447, 448, nx - 2):
            pts.add((k, int(rng.integers(0, ny)), i))
        for j in (7, 8, 255, 256):
            pts.add((k, j, int(rng.integers(0, nx))))
    # the anomalies' cores
    pts.add((int(5.0 / 50 * nz), ny // 2, nx // 2))
    pts.add((int(11.5 / 50 * nz), ny // 2, nx // 2))
    while len(pts) < count:
        pts.add((int(rng.integers(0, nz)), int(rng.integers(0, ny)), int(rng.integers(0, nx))))
    return sorted(pts)


def _window(cfg, phi, p, r, dtau, m):
    ph = cfg.phys
    dx, dy, dz = ph.lx / cfg.nx, ph.ly / cfg.ny, ph.lz / cfg.nz
    lo = [max(0, c - r) for c in p]
    hi = [min(n, c + r + 1) for c, n in zip(p, (cfg.nz, cfg.ny, cfg.nx))]
    wz, wy, wx = (b - a for a, b in zip(lo, hi))
    sl = tuple(slice(a, b) for a, b in zip(lo, hi))
    o = ReactiveOracle(ph.replace(lx=wx * dx, ly=wy * dy, lz=wz * dz), wx, wy, wz, np.ascontiguousarray(phi[sl]))
    o.begin_step()
    o.iterate(m, dtau=dtau)
    return o, tuple(c - a for c, a in zip(p, lo))


def test_benchmark_size_sampled_against_windowed_oracle():
    """506 x 506 x 2042 (the paper's global grid of its 80-GPU run), 10
    iterations: the pseudo step before the first, the check variant of the
    sweep on the tenth, as the benchmark runs them."""
    import torch
    from paper_2207_08716_amd.waves import Waves
    cfg = inputs.config_reactive(506, da=100.0, nz=2042)
    phi = inputs.porosity_field(cfg)
    m = 10
    w = Waves(cfg.phys, cfg.nx, cfg.ny, cfg.nz, phi)
    w.begin_step()
    w.iterate(m)
    err_gpu = w.last_error()
    pts = _sample_points(cfg.nx, cfg.ny, cfg.nz, np.random.default_rng(3), 64)
    kk, jj, ii = (torch.tensor([p[a] for p in pts], device="cuda") for a in range(3))
    got = {}
    with torch.cuda.stream(w.stream):
        for name in FIELDS:
            got[name] = w.view(name)[kk, jj, ii].cpu().numpy()
    del w
    torch.cuda.empty_cache()
    # k/beta_P increases with phi (k ~ phi^3, beta_P affine with positive
    # coefficients), so the window around the porosity maximum holds the
    # grid's pseudo step
    pmax = np.unravel_index(int(np.argmax(phi)), phi.shape)
    o, _ = _window(cfg, phi, pmax, 3, None, 1)
    dtau = o.dtau
    ref = {name: np.zeros(len(pts)) for name in FIELDS}
    local_err = 0.0
    for q, p in enumerate(pts):
        o, lp = _window(cfg, phi, p, m + 3, dtau, m - 1)
        before = {name: o.f[name][lp] for name in ("xs", "pf", "phi")}
        o.iterate(1, dtau=dtau)
        for name in FIELDS:
            ref[name][q] = o.f[name][lp]
        local_err = max(local_err, abs(o.f["phi"][lp] - before["phi"]), abs(o.f["pf"][lp] - before["pf"]) / 10,
                        abs(o.f["xs"][lp] - before["xs"]))
    worst = {}
    for name in FIELDS:
        scale = np.abs(ref[name]).max()
        worst[name] = float(np.abs(got[name] - ref[name]).max() / scale)
    print(worst, err_gpu, local_err, flush=True)
    assert all(v <= TOL for v in worst.values()), worst
    # the grid's stopping quantity bounds every sampled cell's change
    slack = 2 * TOL * max(np.abs(ref["phi"]).max(), np.abs(ref["pf"]).max() / 10, np.abs(ref["xs"]).max())
    assert err_gpu >= local_err - slack and np.isfinite(err_gpu)
    assert np.abs(ref["pf"]).max() > 0
