"""Seeded synthetic inputs for the FDTD hot path.

This module builds *inputs only*: grid sizes, per-cell material ids and
material tables, thin-wire runs, lumped current sources with their sampled
waveforms, and probe lists.  It holds none of the method's arithmetic (no
coefficients, no averaging, no field updates), so both the HIP library and
the FP64 reference can be fed from it without sharing any computation.

Geometry conventions (shared by every backend):
  * node (i, j, k) is the point (i, j, k) * dx; cell (i, j, k) spans
    [i, i+1] x [j, j+1] x [k, k+1] in units of dx;
  * an edge is (axis u, start node) and spans node -> node + e_u;
  * ``cell_mat`` is a uint8 array of shape (nz, ny, nx) (x fastest);
  * waveform sample n is the source current at time (n + 1/2) * dt, which
    is the time level of the electric-field update it enters (the lumped
    current density term of the Ampere-Maxwell law, eq. 1).

The three workloads follow the paper's model-file templates (Section 4.1,
Fig. 3 for the feed topology of a buried electrode) scaled to the sizes of
the three FDTD benchmark configurations.  Where the paper does not fix a
point (waveform definitions, electrode placement), the choice made is stated
at the function that makes it.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Tuple, Optional

import numpy as np

# Speed of light, used only to pick the default time step for sampling the
# source waveforms (inputs).  Each backend evaluates its own field equations.
C0 = 299792458.0

AX_X, AX_Y, AX_Z = 0, 1, 2
PR_E, PR_VLINE, PR_ILOOP = 0, 1, 2
LOSS_SEMI, LOSS_EXPLICIT = 0, 1


def courant_dt(dx: float, factor: float = 0.99) -> float:
    """Time step at ``factor`` times the 3D Courant limit for a cubic cell."""
    return factor * dx / (C0 * math.sqrt(3.0))


# ---------------------------------------------------------------------------
# Source waveforms (harness inputs)
# ---------------------------------------------------------------------------

def sample_times(n_steps: int, dt: float) -> np.ndarray:
    """Times (n + 1/2) dt at which current sample n is taken."""
    return (np.arange(n_steps, dtype=np.float64) + 0.5) * dt


def gaussian(n_steps: int, dt: float, t0: float, width: float, amp: float = 1.0) -> np.ndarray:
    """amp * exp(-((t - t0) / width)^2) sampled at (n + 1/2) dt."""
    t = sample_times(n_steps, dt)
    return amp * np.exp(-(((t - t0) / width) ** 2))


def _dexp_shape(alpha: float, beta: float):
    tp = math.log(beta / alpha) / (beta - alpha)
    k = 1.0 / (math.exp(-alpha * tp) - math.exp(-beta * tp))

    def f(t):
        return k * (math.exp(-alpha * t) - math.exp(-beta * t))

    return tp, k, f


def _bisect(g, lo, hi, it=200):
    glo = g(lo)
    for _ in range(it):
        mid = 0.5 * (lo + hi)
        gm = g(mid)
        if (gm > 0) == (glo > 0):
            lo, glo = mid, gm
        else:
            hi = mid
    return 0.5 * (lo + hi)


def dexp_times(alpha: float, beta: float) -> Tuple[float, float]:
    """(T1, T2) of a normalised double exponential.

    T1 = 1.25 (t90 - t10) on the front; the virtual origin is where the line
    through the 10 % and 90 % points meets zero, t_O = t10 - 0.1 T1; T2 is the
    time from t_O to the 50 % point on the tail (IEC impulse convention).
    """
    tp, _k, f = _dexp_shape(alpha, beta)
    t10 = _bisect(lambda t: f(t) - 0.1, 0.0, tp)
    t90 = _bisect(lambda t: f(t) - 0.9, 0.0, tp)
    hi = tp
    while f(hi) > 0.5:
        hi *= 2.0
    t50 = _bisect(lambda t: f(t) - 0.5, tp, hi)
    T1 = 1.25 * (t90 - t10)
    t0 = t10 - 0.1 * T1
    return T1, t50 - t0


def dexp_params(T1: float, T2: float) -> Tuple[float, float, float]:
    """Solve (alpha, beta, k) so that k (e^{-alpha t} - e^{-beta t}) has peak 1,
    front time T1 and time to half value T2 (see :func:`dexp_times`)."""
    from scipy.optimize import fsolve

    def resid(x):
        a, b = math.exp(x[0]), math.exp(x[1])
        if b <= a * 1.0001:
            return [1e3, 1e3]
        t1, t2 = dexp_times(a, b)
        return [math.log(t1 / T1), math.log(t2 / T2)]

    x0 = [math.log(0.7 / T2), math.log(2.5 / T1)]
    x = fsolve(resid, x0, xtol=1e-13, maxfev=2000)
    a, b = math.exp(x[0]), math.exp(x[1])
    _tp, k, _f = _dexp_shape(a, b)
    return a, b, k


def double_exponential(n_steps: int, dt: float, I0: float, T1: float, T2: float) -> np.ndarray:
    """I0 k (e^{-alpha t} - e^{-beta t}) sampled at (n + 1/2) dt."""
    a, b, k = dexp_params(T1, T2)
    t = sample_times(n_steps, dt)
    return I0 * k * (np.exp(-a * t) - np.exp(-b * t))


def heidler(n_steps: int, dt: float, I0: float, tau1: float, tau2: float, n: float, eta: float = 1.0,
            t_delay: float = 0.0) -> np.ndarray:
    """Heidler current (I0 / eta) x^n / (1 + x^n) exp(-t' / tau2), x = t' / tau1,
    t' = t - t_delay (0 before the delay), sampled at (n + 1/2) dt."""
    t = sample_times(n_steps, dt) - t_delay
    tp = np.maximum(t, 0.0)
    x = (tp / tau1) ** n
    return np.where(t > 0, (I0 / eta) * x / (1.0 + x) * np.exp(-tp / tau2), 0.0)


# ---------------------------------------------------------------------------
# Scenario container
# ---------------------------------------------------------------------------

@dataclass
class Scenario:
    name: str
    nx: int
    ny: int
    nz: int
    dx: float
    dt: float
    n_steps: int
    cell_mat: np.ndarray                      # uint8 (nz, ny, nx)
    materials: List[Tuple[float, float, float]]  # (eps_r, sigma [S/m], mu_r)
    npml: int = 0
    pml: Tuple[float, float, float, float, float] = (3.0, 1.0, 1.0, 0.0, 1.0)  # m, sigma_factor, kappa_max, alpha_max, m_a
    loss_mode: int = LOSS_SEMI
    wire_r0_factor: float = math.exp(-math.pi / 2)  # equivalent radius of a bare wire edge / dx
    wires: List[Tuple[int, int, int, int, int, float]] = field(default_factory=list)   # axis, i, j, k, n_cells, radius
    sources: List[Tuple[int, int, int, int, np.ndarray]] = field(default_factory=list)  # axis, i, j, k, amps
    probes: List[Tuple[str, int, int, int, int, int, int]] = field(default_factory=list)  # name, kind, axis, i, j, k, n_cells
    # Debye poles: (tau [s] per pole, increments [material][pole]); the
    # materials' eps_r is then eps_inf
    debye: Optional[Tuple[List[float], np.ndarray]] = None
    # lumped elements (kind 0 R [ohm], 1 C [F], axis, i, j, k, value) and
    # non-ideal sources (kind 0 current / 1 voltage, axis, i, j, k, amps, r)
    lumped: List[Tuple[int, int, int, int, int, float]] = field(default_factory=list)
    sources_r: List[Tuple[int, int, int, int, int, np.ndarray, float]] = field(default_factory=list)
    # oblique thin wires: (end a, end b in cells, radius, driven segment, amps, recorded segment)
    owires: List[tuple] = field(default_factory=list)
    # junctions of oblique wires: (wire ids, ends: 0 the wire's start, 1 its end)
    ojunctions: List[tuple] = field(default_factory=list)
    meta: dict = field(default_factory=dict)

    @property
    def cells(self) -> int:
        return self.nx * self.ny * self.nz

    def params(self) -> dict:
        m, sf, km, am, ma = self.pml
        return dict(nx=self.nx, ny=self.ny, nz=self.nz, dx=self.dx, dt=self.dt,
                    npml=self.npml, pml_m=m, pml_sigma_factor=sf, pml_kappa_max=km,
                    pml_alpha_max=am, pml_ma=ma, loss_mode=self.loss_mode,
                    wire_r0_factor=self.wire_r0_factor, max_steps=self.n_steps)


def apply(sc: Scenario, sim) -> List[int]:
    """Feed a scenario into any backend exposing set_materials / add_wire /
    add_source / add_probe (duck-typed).  Returns the probe ids in order."""
    sim.set_materials(sc.cell_mat, sc.materials)
    if sc.debye is not None:
        sim.set_debye(*sc.debye)
    for w in sc.wires:
        sim.add_wire(*w)
    for (ax, i, j, k, amps) in sc.sources:
        sim.add_source(ax, i, j, k, amps)
    for (kind, ax, i, j, k, amps, r) in sc.sources_r:
        sim.add_source_r(kind, ax, i, j, k, amps, r)
    for (kind, ax, i, j, k, v) in sc.lumped:
        sim.add_lumped(kind, ax, i, j, k, v)
    for (a, b, r, src, amps, rec) in sc.owires:
        sim.add_oblique_wire(a, b, r, src, amps, rec)
    for (ids, ends) in sc.ojunctions:
        sim.join_oblique_wires(ids, ends)
    ids = []
    for (_name, kind, ax, i, j, k, n) in sc.probes:
        ids.append(sim.add_probe(kind, ax, i, j, k, n))
    return ids


def random_case(nx, ny, nz, npml, seed, nsteps=60, n_mats=6):
    """Test input: a ragged grid with random materials (lossy, mu != 1),
    thin wires along all three axes, two current sources and one probe of
    each kind, for element-wise field comparison between backends."""
    rng = np.random.default_rng(seed)
    dx = 0.25
    dt = courant_dt(dx)
    mats = [(float(rng.uniform(1, 20)), float(rng.uniform(0, 0.05)), float(rng.uniform(1, 3)))
            for _ in range(n_mats)]
    cm = rng.integers(0, n_mats, size=(nz, ny, nx)).astype(np.uint8)
    amps = gaussian(nsteps, dt, 15 * dt, 5 * dt, 3.0)
    sc = Scenario(f"rand{seed}", nx, ny, nz, dx, dt, nsteps, cm, mats, npml=npml,
                    pml=(3.0, 1.0, 2.0, 0.02, 1.0))
    sc.wires = [(0, 1, ny // 2, nz // 2, nx - 2, 0.004), (2, nx // 3, ny // 3, 1, nz - 3, 0.01),
                (1, nx // 2, 1, nz // 3, ny - 2, 0.002)]
    sc.sources = [(2, nx // 2, ny // 2 + 1, nz // 2, amps), (0, nx // 4, ny // 3, nz // 3 + 1, -amps)]
    sc.probes = [("e", 0, 1, nx // 3, ny // 2, nz // 2 + 2, 1),
                 ("v", 1, 0, 1, ny // 2 + 2, nz // 2, nx - 3),
                 ("i", 2, 2, nx // 2, ny // 2 + 1, nz // 2, 1)]
    return sc


# ---------------------------------------------------------------------------
# Workloads
# ---------------------------------------------------------------------------

AIR = (1.0, 0.0, 1.0)


def config1(n_steps: int = 300) -> Scenario:
    """48^3 cells, dx 0.5 m, PEC box; lower 16 layers soil (eps_r 10,
    sigma 0.01 S/m); Gaussian soft current on Ez at the centre; 8 Ez probes
    at cells chosen by numpy.random.default_rng(1)."""
    n = 48
    dx = 0.5
    dt = courant_dt(dx)
    cm = np.zeros((n, n, n), np.uint8)
    cm[:16] = 1
    mats = [AIR, (10.0, 0.01, 1.0)]
    amps = gaussian(n_steps, dt, 40 * dt, 12 * dt, 1.0)
    rng = np.random.default_rng(1)
    probes = []
    seen = {(24, 24, 24)}
    while len(probes) < 8:
        i, j = (int(v) for v in rng.integers(1, 48, size=2))
        k = int(rng.integers(0, 48))
        if (i, j, k) in seen:
            continue
        seen.add((i, j, k))
        probes.append((f"Ez[{i},{j},{k}]", PR_E, AX_Z, i, j, k, 1))
    return Scenario("config1_48cube_pec", n, n, n, dx, dt, n_steps, cm, mats,
                    sources=[(AX_Z, 24, 24, 24, amps)], probes=probes)


def config2(nx: int = 512, ny: int = 512, nz: int = 384, dx: float = 0.5, npml: int = 10,
            wire_cells: int = 60, n_steps: int = 4000, e_probe_offsets=(10, 20, 40, 80, 160),
            I0: float = 1.0e4) -> Scenario:
    """Vertical thin wire over two-layer soil in an open (CPML) domain.

    Full size: 512 x 512 x 384 cells, dx 0.5 m, 10-cell CPML; soil below the
    mid plane k_s = nz/2: top 4 m sigma 0.005 S/m eps_r 15, below sigma
    0.02 S/m eps_r 8.  A 5 mm wire rises ``wire_cells`` cells from the
    ground surface, a current-source gap sits at its top, and a channel lead
    continues to the top of the domain.  10 kA double exponential 1/50 us.
    """
    dt = courant_dt(dx)
    ks = nz // 2
    l1 = int(round(4.0 / dx))
    cm = np.zeros((nz, ny, nx), np.uint8)
    cm[ks - l1:ks] = 1
    cm[:ks - l1] = 2
    mats = [AIR, (15.0, 0.005, 1.0), (8.0, 0.02, 1.0)]
    ic, jc = nx // 2, ny // 2
    kg = ks + wire_cells
    a = 0.005
    wires = [(AX_Z, ic, jc, ks, wire_cells, a),
             (AX_Z, ic, jc, kg + 1, nz - kg - 1, a)]
    amps = double_exponential(n_steps, dt, I0, 1.0e-6, 50.0e-6)
    probes = []
    iend = nx - npml
    for k in np.linspace(ks, kg, 4).round().astype(int):
        probes.append((f"V_Ex(k={k})", PR_VLINE, AX_X, ic, jc, int(k), iend - ic))
    for d in e_probe_offsets:
        if ic + d < iend:
            probes.append((f"Ex[{ic + d},{jc},{ks}]", PR_E, AX_X, ic + d, jc, ks, 1))
            probes.append((f"Ez[{ic + d},{jc},{ks}]", PR_E, AX_Z, ic + d, jc, ks, 1))
    probes.append(("I_base", PR_ILOOP, AX_Z, ic, jc, ks, 1))
    probes.append(("I_source", PR_ILOOP, AX_Z, ic, jc, kg, 1))
    return Scenario(f"config2_{nx}x{ny}x{nz}_cpml{npml}", nx, ny, nz, dx, dt, n_steps, cm, mats,
                    npml=npml, wires=wires, sources=[(AX_Z, ic, jc, kg, amps)], probes=probes,
                    meta=dict(ks=ks, kg=kg))


# Measured soil of the paper's buried-wire example (Section 4.1, four-term
# Debye expansion): eps_inf, static conductivity [S/m], and per pole
# (delta eps, tau [s]).
DEBYE_SOIL_EPS_INF = 16.381
DEBYE_SOIL_SIGMA0 = 2.684e-3
DEBYE_SOIL_POLES = ((92.103, 7.404e-6), (20.825, 1.062e-6), (374.768, 2.162e-5), (10.387, 1.008e-8))


def config2_debye(**kw) -> Scenario:
    """The config-2 scene (any of config2's size arguments) with both soil
    layers replaced by the paper's measured four-pole Debye soil."""
    sc = config2(**kw)
    sc.name = sc.name.replace("config2", "config2_debye")
    soil = (DEBYE_SOIL_EPS_INF, DEBYE_SOIL_SIGMA0, 1.0)
    sc.materials = [AIR, soil, soil]
    de = np.array([[0.0] * 4] + [[p[0] for p in DEBYE_SOIL_POLES]] * 2)
    sc.debye = ([p[1] for p in DEBYE_SOIL_POLES], de)
    return sc


def config2_lumped(**kw) -> Scenario:
    """The config-2 scene (any of config2's size arguments) with its ideal
    source gap replaced by a 10 kV-class resistive voltage source (series
    400 ohm) and a 1 kohm, 100 pF load across the wire's base edge."""
    sc = config2(**kw)
    sc.name = sc.name.replace("config2", "config2_lumped")
    ax, i, j, k, amps = sc.sources[0]
    sc.sources = []
    sc.sources_r = [(1, ax, i, j, k, amps * 400.0, 400.0)]
    ks = sc.meta["ks"]
    sc.lumped = [(0, AX_X, i, j, ks, 1000.0), (1, AX_X, i, j, ks, 1e-10)]
    return sc


# The apparent-resistivity array of the paper's third example (Section 4.3):
# three soil layers, each a four-pole Debye expansion of its Messier-model
# properties (eps_inf, sigma0 [S/m], (delta eps, tau [s]) per pole).
ARRAY_LAYERS = (
    (15.767, 5.0e-3, ((839.441, 3.096e-5), (143.901, 4.068e-6), (66.971, 7.217e-7), (31.515, 9.141e-8))),
    (13.488, 2.5e-3, ((593.525, 3.096e-5), (101.748, 4.066e-6), (47.348, 7.212e-7), (22.273, 9.132e-8))),
    (11.884, 1.25e-3, ((419.744, 3.097e-5), (71.960, 4.069e-6), (33.494, 7.218e-7), (15.757, 9.140e-8))),
)


def config_array(dx: float = 0.05, n_steps: int = 4000) -> Scenario:
    """The four-electrode array of the paper's apparent-soil example on its
    5 x 5 x 4 m volume (100 x 100 x 80 cells at dx 0.05 m): soil layers of
    1 m (z 2-3 m, 1-2 m, 0-1 m) under 1 m of air, a 0.5 m CPML; current
    electrodes at (1, 1) and (2, 1) m and potential electrodes at (4, 3) and
    (4, 4) m, 8 mm rods from z 2.95 to 3.15 m joined by 3 mm leads at
    3.15 m; a Heidler current (tau1 0.37 us, tau2 14 us, n 10, delayed
    0.185 us) in the gap of the current leads; probes: the source current and
    the voltage across the gap of the potential leads.  The full run is
    400 us.  Readings: the three layers' pole time constants agree to 0.1%
    and the grid shares one set, their per-pole mean; the CPML tuple reads as
    (thickness 0.5 m, sigma factor 1, kappa_max 1, alpha_max 1e-3, m 3, m_a 1);
    the Heidler arguments as (tau1, tau2, I0, n, eta, delay)."""
    m = lambda v: int(round(v / dx))
    nx, ny, nz = m(5.0), m(5.0), m(4.0)
    dt = courant_dt(dx)
    cm = np.zeros((nz, ny, nx), np.uint8)
    cm[m(2.0):m(3.0)] = 1
    cm[m(1.0):m(2.0)] = 2
    cm[:m(1.0)] = 3
    mats = [AIR] + [(L[0], L[1], 1.0) for L in ARRAY_LAYERS]
    tau = [float(np.mean([L[2][p][1] for L in ARRAY_LAYERS])) for p in range(4)]
    de = np.array([[0.0] * 4] + [[pole[0] for pole in L[2]] for L in ARRAY_LAYERS])
    k0, k1 = m(2.95), m(3.15)
    rod, lead = 0.008, 0.003
    wires = [(AX_Z, m(1.0), m(1.0), k0, k1 - k0, rod), (AX_Z, m(2.0), m(1.0), k0, k1 - k0, rod),
             (AX_X, m(1.0), m(1.0), k1, m(1.45) - m(1.0), lead), (AX_X, m(1.5), m(1.0), k1, m(2.0) - m(1.5), lead),
             (AX_Z, m(4.0), m(3.0), k0, k1 - k0, rod), (AX_Z, m(4.0), m(4.0), k0, k1 - k0, rod),
             (AX_Y, m(4.0), m(3.0), k1, m(3.45) - m(3.0), lead), (AX_Y, m(4.0), m(3.5), k1, m(4.0) - m(3.5), lead)]
    amps = heidler(n_steps, dt, 1.0, 3.7e-7, 1.4e-5, 10.0, 1.0, 1.85e-7)
    probes = [("I_source", PR_ILOOP, AX_X, m(1.45), m(1.0), k1, 1),
              ("V_potential", PR_VLINE, AX_Y, m(4.0), m(3.45), k1, 1)]
    return Scenario(f"array_{nx}x{ny}x{nz}", nx, ny, nz, dx, dt, n_steps, cm, mats, npml=m(0.5),
                    pml=(3.0, 1.0, 1.0, 1e-3, 1.0), wires=wires, sources=[(AX_X, m(1.45), m(1.0), k1, amps)],
                    probes=probes, debye=(tau, de), meta=dict(full_steps=int(math.ceil(400e-6 / dt))))


def config2_small(n_steps: int = 1200) -> Scenario:
    """The config-2 structure on a 96 x 96 x 80 grid (oracle-sized)."""
    return config2(nx=96, ny=96, nz=80, dx=0.5, npml=10, wire_cells=12, n_steps=n_steps,
                   e_probe_offsets=(5, 10, 20, 30))


@dataclass
class ElectrodeCase:
    """Physical inputs of one buried-electrode case (the surrogate's inputs)."""
    log10_sigma: float
    eps_r: float
    length: float    # m
    depth: float     # m
    T1: float        # s (front time of the injected current)


CONFIG3_RANGES = dict(log10_sigma=(-4.0, -1.0), eps_r=(4.0, 40.0), length=(5.0, 18.5),
                      depth=(0.5, 1.0), T1=(0.5e-6, 1.5e-6))


def electrode_grid(case: ElectrodeCase, dims: Tuple[int, int, int], dx: float = 0.25,
                   npml: int = 8, n_steps: int = 2000, T2: float = 10e-6,
                   name: str = "electrode", amps: np.ndarray = None) -> Scenario:
    """Buried horizontal electrode fed like the ground-potential-rise model
    file of Section 4.1 (Fig. 3): a riser from the electrode to one cell above
    the surface, a current-source gap on a horizontal stub with a lead into
    the absorbing layer, and a voltage gap on a perpendicular stub with its own
    lead (the remote reference).  ``amps`` (n_steps samples) replaces the
    double-exponential current when given."""
    nx, ny, nz = dims
    dt = courant_dt(dx)
    n_w = int(round(case.length / dx))
    n_air = max(4, int(round(0.25 * (nz - 16))))
    ks = nz - npml - n_air
    ke = ks - int(round(case.depth / dx))
    i_f, jc = 12, ny // 2
    kw = ks + 1
    if i_f + n_w + npml + 2 > nx:
        raise ValueError("electrode does not fit the grid")
    cm = np.zeros((nz, ny, nx), np.uint8)
    cm[:ks] = 1
    mats = [AIR, (case.eps_r, 10.0 ** case.log10_sigma, 1.0)]
    a = 0.005
    wires = [
        (AX_X, i_f, jc, ke, n_w, a),            # electrode
        (AX_Z, i_f, jc, ke, kw - ke, a),        # riser
        (AX_X, i_f - 2, jc, kw, 2, a),          # current stub
        (AX_X, 0, jc, kw, i_f - 3, a),          # current lead into the CPML
        (AX_Y, i_f, jc - 2, kw, 2, a),          # voltage stub
        (AX_Y, i_f, 0, kw, jc - 3, a),          # voltage lead into the CPML
    ]
    if amps is None:
        amps = double_exponential(n_steps, dt, 1.0, case.T1, T2)
    probes = [("V_gap", PR_VLINE, AX_Y, i_f, jc - 3, kw, 1),
              ("I_source", PR_ILOOP, AX_X, i_f - 3, jc, kw, 1)]
    return Scenario(name, nx, ny, nz, dx, dt, n_steps, cm, mats, npml=npml, wires=wires,
                    sources=[(AX_X, i_f - 3, jc, kw, amps)], probes=probes,
                    meta=dict(case=case, ks=ks, ke=ke))


def draw_cases(n: int, seed: int, widen: float = 0.0) -> List[ElectrodeCase]:
    """Electrode cases drawn uniformly from the configuration ranges
    (log-uniform in sigma), each range widened by ``widen`` of its width on
    each side (eps_r clamped at 1)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        vals = {}
        for key, (lo, hi) in CONFIG3_RANGES.items():
            w = hi - lo
            lo2, hi2 = lo - widen * w, hi + widen * w
            if key == "eps_r":
                lo2 = max(lo2, 1.0)
            vals[key] = float(rng.uniform(lo2, hi2))
        out.append(ElectrodeCase(**vals))
    return out


def grid_dims_for(case: ElectrodeCase, rng: np.random.Generator, dx: float = 0.25,
                  lo: int = 32, hi: int = 96) -> Tuple[int, int, int]:
    n_w = int(round(case.length / dx))
    nx_min = max(lo, n_w + 22)
    nx = int(rng.integers(nx_min, max(hi, nx_min) + 1))
    ny = int(rng.integers(lo, hi + 1))
    nz = int(rng.integers(lo, hi + 1))
    return nx, ny, nz


def config3(n_grids: int = 256, seed: int = 3, n_steps: int = 2000) -> List[Scenario]:
    """256 uneven electrode grids, sizes uniform in [32, 96]^3 (x grown to fit
    the electrode), dx 0.25 m, 8-cell CPML, 2000 steps each."""
    cases = draw_cases(n_grids, seed)
    rng = np.random.default_rng(seed + 1000)
    out = []
    for g, c in enumerate(cases):
        dims = grid_dims_for(c, rng)
        out.append(electrode_grid(c, dims, n_steps=n_steps, name=f"config3_g{g}"))
    return out


def config2_tower(**kw) -> Scenario:
    """A lightning strike to a lattice tower of oblique wires, like the
    tower example of Section 4.2 (whose dimensions the paper takes from an
    earlier publication; these are this scene's own): the config-2 grid and
    soil (any of config2's size arguments), without its mast and source.

    A 30 m tower: four legs (5 cm) from footings 1 m deep at the corners of
    an 8 m square to an apex, each cut at 15 m, where a ring of four wires
    (2 cm) joins them; two inclined cross-arms (3 cm) from the apex to tips
    7 m out and 3 m lower; above the apex a vertical channel wire (5 mm) to
    the top of the domain, driven at its lowest segment by the scene's
    10 kA 1/50 us current.  Five junctions: the apex (seven wire ends) and
    the four ring corners (four each).  Every point sits off the lattice by
    a fraction of a cell.  Probes: the voltage from each arm tip 2 m down
    (across an insulator string to a phase conductor that the scene leaves
    out), the ground-surface fields of config 2; records: the channel
    current and the current into one footing."""
    sc = config2(**kw)
    sc.name = sc.name.replace("config2", "config2_tower")
    _ax, ic, jc, ks, _n, _a = sc.wires[0]
    amps = sc.sources[0][4]
    sc.wires, sc.sources = [], []
    sc.probes = [p for p in sc.probes if p[1] == PR_E]
    dx, top = sc.dx, sc.nz - sc.npml - 2.6
    c = lambda x, y, z: (ic + x / dx + 0.3, jc + y / dx - 0.2, ks + z / dx + 0.4)
    T = np.array(c(0.0, 0.0, 30.0))
    feet = [np.array(c(sx * 4.0, sy * 4.0, -1.0)) for sx, sy in ((1, 1), (-1, 1), (-1, -1), (1, -1))]
    zr = ks + 15.0 / dx + 0.4
    rings = [F + (zr - F[2]) / (T[2] - F[2]) * (T - F) for F in feet]
    tips = [np.array(c(sx * 7.0, 0.0, 27.0)) for sx in (1, -1)]
    tup = lambda v: tuple(float(x) for x in v)
    ow = [(tup(T), (T[0], T[1], top), 0.005, 0, amps, 0)]                      # 0: channel
    ow += [(tup(F), tup(M), 0.05, -1, None, 0 if q == 0 else -1) for q, (F, M) in enumerate(zip(feet, rings))]
    ow += [(tup(M), tup(T), 0.05, -1, None, -1) for M in rings]                # 5..8: upper legs
    ow += [(tup(rings[q]), tup(rings[(q + 1) % 4]), 0.02, -1, None, -1) for q in range(4)]  # 9..12: ring
    ow += [(tup(T), tup(A), 0.03, -1, None, -1) for A in tips]                 # 13, 14: cross-arms
    sc.owires = ow
    sc.ojunctions = [([0, 5, 6, 7, 8, 13, 14], [0, 1, 1, 1, 1, 0, 0])]
    for q in range(4):
        sc.ojunctions.append(([1 + q, 5 + q, 9 + q, 9 + (q - 1) % 4], [1, 0, 0, 1]))
    drop = max(1, int(round(2.0 / dx)))
    for name, A in zip(("V_arm+x", "V_arm-x"), tips):
        i, j, k = (int(np.floor(v)) for v in A)
        sc.probes.append((name, PR_VLINE, AX_Z, i, j, k - drop, drop))
    sc.meta.update(tower_top=tup(T), arm_tips=[tup(A) for A in tips])
    return sc


def config2_oblique(**kw) -> Scenario:
    """The config-2 scene (any of config2's size arguments) plus a slanted
    5 cm conductor in the air beside the vertical wire, like a tower leg:
    it rises 30 cells over a 20 x 12-cell run, is driven at its lowest
    segment by a tenth of the scene's source current, and its top segment's
    current is recorded."""
    sc = config2(**kw)
    sc.name = sc.name.replace("config2", "config2_oblique")
    _ax, ic, jc, ks, _n, _a = sc.wires[0]
    a = (ic + 12.25, jc - 6.5, ks + 4.4)
    b = (ic + 32.25, jc + 5.5, ks + 34.4)
    n_seg = int(np.floor(np.sqrt(20.0 ** 2 + 12.0 ** 2 + 30.0 ** 2)))
    sc.owires = [(a, b, 0.05, 0, sc.sources[0][4] * 0.1, n_seg - 1)]
    return sc
