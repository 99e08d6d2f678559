"""Seeded synthetic inputs for the two-phase PT solver.

This module only builds *inputs*: grid sizes, physical parameters and the
initial porosity / permeability fields of the synthetic porosity-anomaly
set-ups (thesis article 1, section 3.1 and Table 2; appendix two-phase script,
initial conditions).  It holds none of the solver's arithmetic: no residual,
no coefficient law, no update.  Both the GPU path and the CPU reference take
their starting state from here, as plain numpy arrays.

Conventions
-----------
* Arrays are numpy float64 in (z, y, x) order, x fastest (C order).
* Cell (i, j, k) has its centre at ((i+1/2)dx, (j+1/2)dy, (k+1/2)dz), dx = lx/nx.
* z points up; gravity acts along -z.
* Random numbers come from numpy's PCG64 with the stated seed, drawn in C
  order over the (nz, ny, nx) cell array.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Physics:
    """Non-dimensional physical and numerical parameters.

    Defaults: Table 2 of article 1 and the constants of the appendix two-phase
    script, with the readings listed in the design doc (decompaction factor 100,
    bulk compressibility from Table 2, drained compressibility 1.3x it,
    shear modulus 0.5/beta_phi).
    """
    lx: float = 1.0
    ly: float = 1.0
    lz: float = 1.0
    phi0: float = 1e-2        # background porosity
    kmuf0: float = 1.0        # k0 / mu_f, reference value (scalar k0)
    eta0: float = 1.0         # reference bulk viscosity factor
    mu0: float = 1.0          # reference shear viscosity factor (known DOF value)
    cmu: float = 0.1          # geometry coefficient: mu_s = Mn * phi0 * cmu
    rhofg: float = 1.0        # fluid density x gravity
    rhosg: float = 2.0        # solid density x gravity
    beta_phi: float = 3e-3    # 1/K_phi (effective bulk compressibility)
    beta_d: float = 3.9e-3    # 1/K_d (drained compressibility) = 1.3 beta_phi
    alpha: float = 0.9        # Biot-Willis coefficient
    B: float = 0.89           # Skempton coefficient
    G: float = 0.5 / 3e-3     # elastic shear modulus
    R0: float = 100.0         # decompaction weakening factor
    n_pow: float = 3.0        # power-law exponent
    tau0: float = 0.04        # characteristic stress of the power law
    coh: float = 1.0          # Drucker-Prager cohesion C
    fric_deg: float = 30.0    # Drucker-Prager friction angle
    tau_y_min: float = 1e-3   # floor of the yield stress
    dt: float = 1e-3          # physical time step
    dtS: float = 1e-3         # stress-history time step (= dt by default)
    beta_n: float = 10.0      # numerical compressibility
    rho_i: float = 1.0        # inertial density of the PT velocity update
    c_v: float = 6.1          # safety factor, velocity pseudo-step
    c_pf: float = 6.1         # safety factor, fluid-pressure pseudo-step
    damp_c: float = 1.0       # damping: d = 1 - damp_c / n
    nup: int = 15             # iterations between refreshes / error checks
    r_eta: float = 0.5        # log relaxation of the bulk viscosity
    r_mu: float = 0.1         # log relaxation of the shear viscosity
    powerlaw: bool = False    # eq (24) power-law shear viscosity
    dpcap: bool = False       # Drucker-Prager cap on the lagged viscosity
    mech_off: bool = False    # freeze V and Pt (linear Pf-diffusion limit)
    fp32_tall: bool = False   # launch shape only: FP32 correction sweep on its 14-row tiles
    shear_bg: float = 0.0     # background simple shear rate d(Vx_bg)/dy (eq (32)); 0: none
    dts_rule: bool = False    # stress-history step dtS = max(mu_s)/(G xi_w), renewed when due
    xsi_w: float = 1.0        # wanted xi of the dtS rule

    def replace(self, **kw) -> "Physics":
        return dataclasses.replace(self, **kw)


@dataclass
class WavePhysics:
    """Non-dimensional parameters of the reactive porosity-wave model (thesis
    article 3, eqs (8)-(10); the appendix reactive script's constants): the
    scales of eqs (5)-(7) are 1 (k0/mu_f = eta = drho = g = 1)."""
    lx: float = 12.5
    ly: float = 12.5
    lz: float = 50.0
    phi0: float = 1e-2        # background porosity
    k_muf0: float = 1.0       # k0 / mu_f
    eta: float = 1.0          # bulk viscosity
    rho_f: float = 0.5        # fluid density
    rho_s: float = 1.5        # solid density (rho_s - rho_f = 1)
    g: float = 1.0            # gravity
    beta_d: float = 1e-3      # drained compressibility (Deborah number 1e-3)
    beta_s: float = 1e-3 * 11.0 / 12.0   # solid compressibility without reaction
    beta_f: float = 6e-3      # fluid compressibility
    tau: float = 1e-2         # reaction time, 1/Da (Da = 100)
    beta_x: float = -0.2      # d Xs_eq / d Pf (negative Clapeyron slope)
    delta_x: float = 3.0      # solid density change with Xs
    xs_max: float = 0.05      # largest volatile mass fraction of the solid
    dt: float = 1e-6          # physical time step
    c_pf: float = 16.1        # safety factor of the fluid-pressure pseudo step
    phi_min: float = 1e-4     # porosity clamp
    phi_max: float = 1.0
    nup: int = 10             # iterations between pseudo-step refreshes / checks
    eps: float = 2e-8         # stopping value of the one-iteration change

    def replace(self, **kw) -> "WavePhysics":
        return dataclasses.replace(self, **kw)


@dataclass
class Anomaly:
    centre: tuple          # (x, y, z) in physical units
    amp: float             # amplitude in units of phi0
    width: float | tuple   # Gaussian width w: exp(-|x-c|^2 / w^2), or (wx, wy, wz) for an ellipsoid


@dataclass
class Config:
    """A complete synthetic workload: grid, physics and initial fields."""
    name: str
    nx: int
    ny: int
    nz: int
    phys: Physics
    anomalies: list = field(default_factory=list)
    noise_seed: int | None = None     # +-1e-3 multiplicative noise on phi
    noise_amp: float = 1e-3
    k0_kind: str = "scalar"           # "scalar" | "lognormal" | "grf"
    k0_seed: int | None = None
    k0_sigma: float = 0.5
    k0_corr: float = 0.1
    mode: str = "thesis"              # "thesis" (fixed iterations) | "picard"
    n_picard: int = 5
    rtol: float = 1e-8
    n_iter: int = 1000
    n_steps: int = 1

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def ncell(self):
        return self.nx * self.ny * self.nz

    def resized(self, n: int, name: str | None = None) -> "Config":
        """Same recipe on an n^3 grid (same domain, same seeds)."""
        return dataclasses.replace(self, nx=n, ny=n, nz=n,
                                   name=name or f"{self.name}@{n}")


def cell_centres(n: int, length: float) -> np.ndarray:
    d = length / n
    return (np.arange(n, dtype=np.float64) + 0.5) * d


def porosity_field(cfg: Config) -> np.ndarray:
    """phi = phi0 + sum_a amp_a*phi0*exp(-|x-c_a|^2/w_a^2), then noise."""
    p = cfg.phys
    x = cell_centres(cfg.nx, p.lx)[None, None, :]
    y = cell_centres(cfg.ny, p.ly)[None, :, None]
    z = cell_centres(cfg.nz, p.lz)[:, None, None]
    phi = np.full(cfg.shape, p.phi0, dtype=np.float64)
    for a in cfg.anomalies:
        cx, cy, cz = a.centre
        if isinstance(a.width, tuple):
            wx, wy, wz = a.width
            q = ((x - cx) / wx) ** 2 + ((y - cy) / wy) ** 2 + ((z - cz) / wz) ** 2
            phi += a.amp * p.phi0 * np.exp(-q)
        else:
            r2 = (x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2
            phi += a.amp * p.phi0 * np.exp(-r2 / (a.width * a.width))
    if cfg.noise_seed is not None:
        rng = np.random.Generator(np.random.PCG64(cfg.noise_seed))
        u = rng.random(cfg.shape)
        phi *= 1.0 + cfg.noise_amp * (2.0 * u - 1.0)
    return phi


def gaussian_random_field(shape, lengths, corr: float, seed: int) -> np.ndarray:
    """Zero-mean, unit-variance Gaussian random field with covariance
    proportional to exp(-r^2/corr^2), made by filtering white noise on a
    periodic box twice the domain size and cropping."""
    nz, ny, nx = shape
    lz, ly, lx = lengths
    big = (2 * nz, 2 * ny, 2 * nx)
    rng = np.random.Generator(np.random.PCG64(seed))
    w = rng.standard_normal(big)
    # spectral filter: sqrt of the power spectrum of exp(-r^2/l^2)
    kz = np.fft.fftfreq(big[0], d=lz / nz) * 2 * np.pi
    ky = np.fft.fftfreq(big[1], d=ly / ny) * 2 * np.pi
    kx = np.fft.rfftfreq(big[2], d=lx / nx) * 2 * np.pi
    k2 = kz[:, None, None] ** 2 + ky[None, :, None] ** 2 + kx[None, None, :] ** 2
    filt = np.exp(-k2 * corr * corr / 8.0)
    f = np.fft.irfftn(np.fft.rfftn(w) * filt, s=big, axes=(0, 1, 2))[:nz, :ny, :nx]
    f = f - f.mean()
    f = f / f.std()
    return np.ascontiguousarray(f)


def k0_field(cfg: Config) -> np.ndarray | None:
    """Per-cell k0/mu_f, or None for a scalar k0."""
    p = cfg.phys
    if cfg.k0_kind == "scalar":
        return None
    if cfg.k0_kind == "lognormal":
        rng = np.random.Generator(np.random.PCG64(cfg.k0_seed))
        xi = rng.standard_normal(cfg.shape)
        return p.kmuf0 * np.exp(cfg.k0_sigma * xi)
    if cfg.k0_kind == "grf":
        g = gaussian_random_field(cfg.shape, (p.lz, p.ly, p.lx), cfg.k0_corr, cfg.k0_seed)
        return p.kmuf0 * np.exp(cfg.k0_sigma * g)
    raise ValueError(cfg.k0_kind)


def random_centres(seed: int, count: int, lo, hi):
    rng = np.random.Generator(np.random.PCG64(seed))
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    return [tuple(lo + (hi - lo) * rng.random(3)) for _ in range(count)]


def sensor_cells(seed: int, count: int, shape, margin: int = 1) -> np.ndarray:
    """Distinct interior cell linear indices (C order over (nz, ny, nx))."""
    nz, ny, nx = shape
    rng = np.random.Generator(np.random.PCG64(seed))
    out = set()
    while len(out) < count:
        k = int(rng.integers(margin, nz - margin))
        j = int(rng.integers(margin, ny - margin))
        i = int(rng.integers(margin, nx - margin))
        out.add((k * ny + j) * nx + i)
    return np.array(sorted(out), dtype=np.int64)


# ---------------------------------------------------------------------------
# The five workloads
# ---------------------------------------------------------------------------

# Physical step of the Picard-schedule workloads on the unit cube.  The paper
# does not state one for these set-ups; with dt = 1e-3 the storage terms are
# so weak against Darcy diffusion that the thesis's PT iteration needs more
# than 6e4 iterations per linear solve already at 16^3, while 1e-5 keeps it in
# the storage-dominated regime the thesis runs in.
PICARD_DT = 1e-5

def config_parity(n: int = 32, seed: int = 1) -> Config:
    """FP64 parity workload: unit cube, one Gaussian anomaly of amplitude
    2*phi0 and width 0.1 at (0.5, 0.5, 0.25), +-1e-3 noise, scalar k0,
    1000 fixed iterations of the thesis schedule."""
    return Config(name=f"parity{n}", nx=n, ny=n, nz=n, phys=Physics(),
                  anomalies=[Anomaly((0.5, 0.5, 0.25), 2.0, 0.1)],
                  noise_seed=seed, mode="thesis", n_iter=1000)


def config_fp64_picard(n: int = 255, seed: int = 2) -> Config:
    """FP64 Picard workload: parity recipe plus lognormal (sigma 0.5) k0."""
    c = config_parity(n, seed)
    return dataclasses.replace(c, name=f"picard{n}", k0_kind="lognormal",
                               k0_seed=seed, mode="picard", n_picard=5, rtol=1e-8,
                               phys=c.phys.replace(dt=PICARD_DT, dtS=PICARD_DT))


def config_mixed(n: int = 511, seed: int = 3) -> Config:
    """Mixed-precision workload: two anomalies (2 and 1.5 phi0, width 0.1)
    at seeded centres in [0.3,0.7]^2 x [0.15,0.45], lognormal k0, and the
    Drucker-Prager cap (C = 1, 30 degrees)."""
    cen = random_centres(seed, 2, (0.3, 0.3, 0.15), (0.7, 0.7, 0.45))
    return Config(name=f"mixed{n}", nx=n, ny=n, nz=n,
                  phys=Physics(dpcap=True, coh=1.0, fric_deg=30.0, tau_y_min=1e-3,
                               dt=PICARD_DT, dtS=PICARD_DT),
                  anomalies=[Anomaly(cen[0], 2.0, 0.1), Anomaly(cen[1], 1.5, 0.1)],
                  noise_seed=seed, k0_kind="lognormal", k0_seed=seed,
                  mode="picard", n_picard=5, rtol=1e-8)


def config_adjoint(n: int = 127, seed: int = 4) -> Config:
    """Adjoint workload: parity porosity recipe, log k0 a Gaussian random
    field (correlation 0.1, sigma 0.5), 10 steps of 5 Picard stages."""
    c = config_parity(n, seed)
    return dataclasses.replace(c, name=f"adjoint{n}", k0_kind="grf", k0_seed=seed,
                               mode="picard", n_picard=5, rtol=1e-10, n_steps=10,
                               phys=c.phys.replace(dt=PICARD_DT, dtS=PICARD_DT))


def config_waves(n: int = 767, seed: int = 8) -> Config:
    """Porosity-wave workload: 30^3 domain, three sources (2 phi0, width 1)
    at seeded centres in [7.5,22.5]^2 x [3,10], DP cap, dt = 5e-4, 20 steps."""
    cen = random_centres(seed, 3, (7.5, 7.5, 3.0), (22.5, 22.5, 10.0))
    L = 30.0
    return Config(name=f"waves{n}", nx=n, ny=n, nz=n,
                  phys=Physics(lx=L, ly=L, lz=L, dt=5e-4, dtS=5e-4, dpcap=True),
                  anomalies=[Anomaly(c, 2.0, 1.0) for c in cen],
                  noise_seed=None, mode="picard", n_picard=5, rtol=1e-8, n_steps=20)


def config_production(nx: int = 511, ny: int = 511, nz: int = 1022) -> Config:
    """Production set-up of article 1, section 3.1 and Table 2: a 30 x 30 x 60
    box under background simple shear (tau_bg / mu0 = 1, eq (32)) with an
    ellipsoidal porosity anomaly of axes 14 x 14 x 3.5 (a Gaussian with
    semi-axis widths 7, 7, 1.75, peak 2 phi0) at one fifth of the depth,
    power-law shear viscosity (n = 3, tau0 = 0.04), decompaction factor
    2000, K_phi = 333.33 (beta_phi = 1/K_phi, beta_d = 1.3 beta_phi),
    G = 166.66, the stress-history step rule (xi_w = 1) and dt = 5e-6 (the
    production run's 4800 steps to t = 2.4e-2)."""
    beta_phi = 1.0 / 333.33
    ph = Physics(lx=30.0, ly=30.0, lz=60.0, R0=2000.0, powerlaw=True, n_pow=3.0, tau0=0.04,
                 beta_phi=beta_phi, beta_d=1.3 * beta_phi, G=166.66, shear_bg=1.0, dts_rule=True,
                 xsi_w=1.0, dt=5e-6, dtS=5e-6)
    return Config(name=f"production{nx}x{ny}x{nz}", nx=nx, ny=ny, nz=nz, phys=ph,
                  anomalies=[Anomaly((15.0, 15.0, 12.0), 1.0, (7.0, 7.0, 1.75))],
                  noise_seed=None, mode="thesis", n_iter=1000)


def config_reactive(n: int = 127, da: float = 100.0, nz: int | None = None) -> Config:
    """Reactive porosity waves (article 3; the appendix reactive script): a
    12.5 x 12.5 x 50 box on n x n x 4n cells, two vertically superposed
    spherical Gaussian anomalies (radius 1.5; amplitudes 1.5 phi0 at z = 5
    and 0.75 phi0 at z = 11.5, so the deeper one peaks at 2.5 %), Xs = Xs_max/2,
    Pf = 0; Damkoehler number da (tau = 1/da), dt = 1e-6 for da >= 1, else
    1e-5 (the paper's steps for its two Damkoehler numbers)."""
    ph = WavePhysics(tau=1.0 / da, dt=1e-6 if da >= 1.0 else 1e-5)
    nz = 4 * n if nz is None else nz
    return Config(name=f"reactive{n}x{n}x{nz}", nx=n, ny=n, nz=nz, phys=ph,
                  anomalies=[Anomaly((6.25, 6.25, 5.0), 1.5, 1.5), Anomaly((6.25, 6.25, 11.5), 0.75, 1.5)],
                  noise_seed=None, mode="thesis")


CONFIGS = {
    "parity": config_parity,
    "picard": config_fp64_picard,
    "mixed": config_mixed,
    "adjoint": config_adjoint,
    "waves": config_waves,
    "production": config_production,
    "reactive": config_reactive,
}


def initial_fields(cfg: Config) -> dict:
    """Initial state of every workload: V = R = 0, Pt = Pf = 0, stress
    history 0, porosity from the anomalies, Mn = mu0, and k0 if a field.

    Returns a dict of cell arrays {"phi": ..., "k0": ... or None}; the face
    and edge fields start at zero and are created by each solver."""
    return {"phi": porosity_field(cfg), "k0": k0_field(cfg)}


__all__ = ["Physics", "Anomaly", "Config", "CONFIGS", "config_parity",
           "config_fp64_picard", "config_mixed", "config_adjoint", "config_waves", "config_production",
           "config_reactive", "WavePhysics",
           "initial_fields", "porosity_field", "k0_field", "gaussian_random_field",
           "sensor_cells", "random_centres", "cell_centres", "PICARD_DT"]
