"""Seeded synthetic inputs for the electronic-temperature sub-step path.

This module is shared by the CPU oracle side of the tests and by the GPU
path.  It holds input recipes only: FCC geometry, initial electronic
temperature fields, lattice velocities and parameter sets.  It holds none of
the method's arithmetic (no exchange term, no lattice-temperature estimate,
no source evaluation, no integration).

Units everywhere: Angstrom, femtosecond, eV, Kelvin, amu.

Workloads (sizes follow the configurations the method is exercised on):

* ``c1`` plain FP64 case: 10^3 FCC cells (4,000 atoms), Gaussian hotspot.
* ``c2`` Fourier-limit case: 200x8x8 cells (51,200 atoms), sinusoidal T_e, G=0.
* ``c3`` large single system: 100^3 cells (4,000,000 atoms), jittered,
  Maxwell velocities with a hot core, Gaussian electronic deposition.
* ``c4`` batch: 256 FCC slabs of log-uniform size in [500, 200,000] atoms,
  each heated by a laser pulse on its free x surface.
* ``c5`` differentiation: 64 systems of 20^3 cells (32,000 atoms).

Every generator takes ``scale`` style arguments so tests can build the same
recipe at sizes the oracle finishes in seconds.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# --- physical constants (CODATA 2018) and material numbers -----------------
K_B = 8.617333262e-5                 # Boltzmann constant, eV/K
AMU_A2_PER_FS2_IN_EV = 103.64269652680505   # 1 amu*A^2/fs^2 in eV
J_PER_CM2_IN_EV_PER_A2 = 624.150907446076   # 1 J/cm^2 in eV/A^2
MASS_NI = 58.6934                    # amu
A_LAT = 3.61                         # FCC lattice constant used by the configs, A
T_MAX = 20000.0                      # normalisation ceiling, K
DT_E = 0.05                          # electronic sub-step, fs

# Ni electronic constants converted to per-atom quantities at a = 3.61 A.
# G = 3.6e17 W m^-3 K^-1  ->  g = G * V_atom (eV fs^-1 K^-1 per atom)
# C_e = 3.6886e5 J m^-3 K^-1 -> c = C_e * V_atom (eV/K per atom)
# K from the exchange-rate relation with kappa = 91 W/m/K, d = 3 and a
# lattice sum of 12 a^2 over the 1.1a neighbour shell.
V_ATOM = A_LAT ** 3 / 4.0            # A^3
G_NI = 2.6427e-8
C_NI = 2.7078e-5
K_NI = 0.9465

CE_CONST, CE_LINEAR, CE_CAPPED = 0, 1, 2

FCC_BASIS = np.array([[0.0, 0.0, 0.0],
                      [0.5, 0.5, 0.0],
                      [0.5, 0.0, 0.5],
                      [0.0, 0.5, 0.5]])


def default_params(**kw) -> dict:
    """Parameter set with every field of the library's parameter struct."""
    p = dict(T_min=0.0, T_max=T_MAX, K=K_NI, dt=DT_E, g=G_NI,
             ce_model=CE_CONST, ce_const=C_NI, gamma=1e-4, ce_cap=0.0,
             ke_eps=1e-5,
             laser_on=0, laser_fluence=0.0, laser_lp=100.0, laser_t0=150.0,
             laser_sigma=100.0 / (2.0 * math.sqrt(2.0 * math.log(2.0))),
             laser_x0=0.0, v_atom=V_ATOM)
    for k, v in kw.items():
        if k not in p:
            raise KeyError(f"unknown parameter {k}")
        p[k] = v
    return p


@dataclass
class System:
    """One independent atomic system: geometry, initial fields, parameters."""
    pos: np.ndarray                 # (3, N) float64, SoA
    box_lo: np.ndarray              # (3,)
    box_len: np.ndarray             # (3,)
    periodic: np.ndarray            # (3,) int32 (1 = periodic)
    T_e0: np.ndarray                # (N,) float64, K
    params: dict
    T_l: np.ndarray | None = None   # (N,) float64, K (given directly) ...
    vel: np.ndarray | None = None   # ... or (3, N) velocities A/fs
    mass: np.ndarray | None = None  # (N,) amu

    @property
    def n(self) -> int:
        return int(self.pos.shape[1])


@dataclass
class Workload:
    name: str
    systems: list
    r_cut: float
    n_substeps: int
    precision: str                  # "fp64" or "fp32c"
    checkpoint_every: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def n_atoms(self) -> int:
        return sum(s.n for s in self.systems)


# --- geometry ----------------------------------------------------------------
def fcc(nx: int, ny: int, nz: int, a: float = A_LAT):
    """FCC lattice, atom index 4*((ix*ny + iy)*nz + iz) + b, SoA (3, N)."""
    ix, iy, iz = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz),
                             indexing="ij")
    cells = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1).astype(np.float64)
    pos = (cells[:, None, :] + FCC_BASIS[None, :, :]).reshape(-1, 3) * a
    box_len = np.array([nx * a, ny * a, nz * a], dtype=np.float64)
    return np.ascontiguousarray(pos.T), box_len


def jitter(pos: np.ndarray, sigma: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return pos + rng.normal(0.0, sigma, size=pos.shape)


def wrap_periodic(pos: np.ndarray, box_lo, box_len, periodic) -> np.ndarray:
    out = pos.copy()
    for d in range(3):
        if periodic[d]:
            out[d] = box_lo[d] + np.mod(out[d] - box_lo[d], box_len[d])
    return out


def gaussian_hotspot(pos, center, base, peak, sigma):
    """base + peak * exp(-|x - center|^2 / (2 sigma^2)) (plain distance)."""
    r2 = sum((pos[d] - center[d]) ** 2 for d in range(3))
    return base + peak * np.exp(-r2 / (2.0 * sigma * sigma))


def maxwell_velocities(n: int, T, mass, seed: int) -> np.ndarray:
    """Gaussian velocity components with variance k_B T / m (A/fs)."""
    rng = np.random.default_rng(seed)
    T = np.broadcast_to(np.asarray(T, dtype=np.float64), (n,))
    m = np.broadcast_to(np.asarray(mass, dtype=np.float64), (n,))
    sd = np.sqrt(K_B * T / (m * AMU_A2_PER_FS2_IN_EV))
    return rng.normal(0.0, 1.0, size=(3, n)) * sd[None, :]


def remove_com(vel: np.ndarray, mass: np.ndarray) -> np.ndarray:
    m = np.asarray(mass, dtype=np.float64)
    vcom = (vel * m[None, :]).sum(axis=1) / m.sum()
    return vel - vcom[:, None]


# --- configurations -----------------------------------------------------------
def c1(n_cells: int = 10, n_substeps: int = 1000) -> Workload:
    """FP64 plain case: FCC n^3 cells, periodic, r_c = 1.1a, Gaussian
    hotspot 300 K + 9,700 K (sigma 8 A) at the centre, c = gamma*T with
    gamma = 1e-4 eV/K^2 per atom, T_l = 300 K."""
    pos, L = fcc(n_cells, n_cells, n_cells)
    center = L / 2.0
    Te = gaussian_hotspot(pos, center, 300.0, 9700.0, 8.0)
    p = default_params(ce_model=CE_LINEAR, gamma=1e-4)
    s = System(pos=pos, box_lo=np.zeros(3), box_len=L,
               periodic=np.ones(3, np.int32), T_e0=Te, params=p,
               T_l=np.full(pos.shape[1], 300.0))
    return Workload("c1_fcc%d_fp64" % n_cells, [s], r_cut=1.1 * A_LAT,
                    n_substeps=n_substeps, precision="fp64", checkpoint_every=50)


def c2(nx: int = 200, ny: int = 8, nz: int = 8, amplitude: float = 500.0,
       n_substeps: int = 5000, precision: str = "fp32c") -> Workload:
    """Fourier-limit case: T_e = 1000 K + A sin(2 pi x / L_x), G = 0,
    constant c, r_c = 1.1a, periodic."""
    pos, L = fcc(nx, ny, nz)
    Te = 1000.0 + amplitude * np.sin(2.0 * np.pi * pos[0] / L[0])
    p = default_params(g=0.0, ce_model=CE_CONST, ce_const=C_NI)
    s = System(pos=pos, box_lo=np.zeros(3), box_len=L,
               periodic=np.ones(3, np.int32), T_e0=Te, params=p,
               T_l=np.full(pos.shape[1], 300.0))
    return Workload("c2_fcc%dx%dx%d_%s" % (nx, ny, nz, precision), [s],
                    r_cut=1.1 * A_LAT, n_substeps=n_substeps, precision=precision,
                    checkpoint_every=500, extra=dict(amplitude=amplitude))


def c3(n_cells: int = 100, n_substeps: int = 10000, seed_pos: int = 3001,
       seed_vel: int = 3002) -> Workload:
    """Large single system: FCC n^3 cells, positions jittered N(0, 0.05 A),
    Maxwell velocities at 300 K with a 15 A core at 3,000 K (global COM
    removed), r_c = 1.2a, Gaussian electronic deposition of 2 eV/atom peak
    with radius (sigma) 20 A, c = min(gamma T, 3 k_B)."""
    pos, L = fcc(n_cells, n_cells, n_cells)
    lo = np.zeros(3)
    per = np.ones(3, np.int32)
    pos = wrap_periodic(jitter(pos, 0.05, seed_pos), lo, L, per)
    n = pos.shape[1]
    center = L / 2.0
    r2 = sum((pos[d] - center[d]) ** 2 for d in range(3))
    T_lat0 = np.where(r2 <= 15.0 ** 2, 3000.0, 300.0)
    mass = np.full(n, MASS_NI)
    vel = remove_com(maxwell_velocities(n, T_lat0, mass, seed_vel), mass)
    # deposited energy E_i (eV/atom) raises T_e above 300 K through the
    # capped heat capacity, which is 3 k_B above 2.6 K: T = 300 + E/(3 k_B)
    cap = 3.0 * K_B
    E = 2.0 * np.exp(-r2 / (2.0 * 20.0 ** 2))
    Te = 300.0 + E / cap
    p = default_params(ce_model=CE_CAPPED, gamma=1e-4, ce_cap=cap)
    s = System(pos=pos, box_lo=lo, box_len=L, periodic=per, T_e0=Te, params=p,
               vel=vel, mass=mass)
    return Workload("c3_fcc%d_jitter_fp32c" % n_cells, [s], r_cut=1.2 * A_LAT,
                    n_substeps=n_substeps, precision="fp32c", checkpoint_every=1000)


def c3_shard(w: Workload, n_parts: int, part: int | None = None):
    """One GPU's share of the 4M-atom system cut into n_parts slabs along x:
    the atoms of slab `part` (default n_parts // 2, whose lower face passes
    through the hotspot centre) and, as ghosts, the atoms of the neighbouring
    slabs within r_c of its two faces (x wraps around the periodic box).  The
    share is one system, free in x (its box spans the ghosts) and periodic in
    y and z.  Returns the system and the ghost mask (1.0 on ghosts), whose
    T_e a multi-GPU run would take from the neighbours' exchange."""
    s = w.systems[0]
    if part is None:
        part = n_parts // 2
    Lx = float(s.box_len[0])
    rc = float(w.r_cut)
    width = Lx / n_parts
    dx = np.mod(s.pos[0] - part * width, Lx)
    own = dx < width
    hi = (dx >= width) & (dx < width + rc)
    lo = dx >= Lx - rc
    keep = own | hi | lo
    xs = np.where(lo, dx - Lx, dx)[keep]
    pos = np.vstack([xs, s.pos[1][keep], s.pos[2][keep]])
    pad = 1e-3
    box_lo = np.array([-rc - pad, 0.0, 0.0])
    box_len = np.array([width + 2.0 * rc + 2.0 * pad, s.box_len[1], s.box_len[2]])
    sh = System(pos=pos, box_lo=box_lo, box_len=box_len,
                periodic=np.array([0, 1, 1], np.int32), T_e0=s.T_e0[keep].copy(),
                params=dict(s.params), vel=s.vel[:, keep].copy(), mass=s.mass[keep].copy())
    return sh, (~own[keep]).astype(np.float64)


def c4_sizes(n_systems: int = 256, lo: float = 500.0, hi: float = 2e5,
             seed: int = 4001) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.exp(rng.uniform(math.log(lo), math.log(hi), size=n_systems))


def c4_slab(n_target: float, fluence_j_cm2: float, n_substeps_hint: int = 6000) -> System:
    """FCC slab free in x, periodic in y, z; laser on the x = 0 face."""
    nyz = int(min(32, max(3, round((n_target / 4.0) ** (1.0 / 3.0)))))
    nx = int(max(3, round(n_target / (4.0 * nyz * nyz))))
    pos, L = fcc(nx, nyz, nyz)
    n = pos.shape[1]
    box_lo = np.array([-0.25 * A_LAT, 0.0, 0.0])
    box_len = np.array([nx * A_LAT, L[1], L[2]])
    per = np.array([0, 1, 1], np.int32)
    p = default_params(ce_model=CE_LINEAR, gamma=1e-4,
                       laser_on=1,
                       laser_fluence=fluence_j_cm2 * J_PER_CM2_IN_EV_PER_A2,
                       laser_lp=100.0, laser_t0=150.0, laser_x0=0.0)
    return System(pos=pos, box_lo=box_lo, box_len=box_len, periodic=per,
                  T_e0=np.full(n, 300.0), params=p, T_l=np.full(n, 300.0))


def c4(n_systems: int = 256, n_substeps: int = 6000, size_lo: float = 500.0,
       size_hi: float = 2e5, seed_sizes: int = 4001, seed_fluence: int = 4002) -> Workload:
    """Batch of independent laser-heated slabs, log-uniform atom counts,
    absorbed fluence U[0.05, 0.5] J/cm^2, penetration depth 100 A, pulse
    FWHM 100 fs centred at 150 fs, c = gamma*T, r_c = 1.1a."""
    sizes = c4_sizes(n_systems, size_lo, size_hi, seed_sizes)
    rng = np.random.default_rng(seed_fluence)
    flu = rng.uniform(0.05, 0.5, size=n_systems)
    systems = [c4_slab(float(sz), float(f)) for sz, f in zip(sizes, flu)]
    return Workload("c4_batch%d_laser_fp32c" % n_systems, systems, r_cut=1.1 * A_LAT,
                    n_substeps=n_substeps, precision="fp32c", checkpoint_every=1000)


C5_C = 2.345e-5          # eV/K, lambda * 300 K per atom
C5_K0 = 0.05             # fs^-1
C5_G0 = 1.1727e-7        # eV fs^-1 K^-1 per atom (g0/c = 5e-3 fs^-1)


# --- two-temperature 1D Ni bar (Section 3.1), per-node units ---------------------
A0_BAR = 3.562                       # A, fcc Ni lattice constant quoted for the bar
B_BAR = A0_BAR / math.sqrt(2.0)      # A, node spacing b = a0/sqrt(2)
EV_J = 1.602176634e-19               # J per eV
V_BAR = (A0_BAR * 1e-10) ** 3 / 4.0  # m^3 per node (cancels from every rate)
G_BAR = 3.6e17 * V_BAR / EV_J * 1e-15            # g = G V, eV/(fs K)
C_E_BAR = 3.6886e5 * V_BAR / EV_J                # c_e = C_e V, eV/K
C_L_BAR = 8890.0 * 400.0 * V_BAR / EV_J          # c_lat = rho C_l V, eV/K
# Eq. 3 with d = 1, Z = 2 over the chain: K = 2 kappa_e / (C_e 2 b^2)
K_E_BAR = 91.0 / (3.6886e5 * (B_BAR * 1e-10) ** 2) * 1e-15          # 1/fs
# three-point Fourier stencil of the lattice, kappa_lat = 0.05 kappa_e
K_L_BAR = 0.05 * 91.0 / (8890.0 * 400.0 * (B_BAR * 1e-10) ** 2) * 1e-15   # 1/fs


def c6_bar(n_nodes: int = 141, hot_T: float = 6000.0, hot_span_a0: float = 2.0,
           centre: int | None = None) -> System:
    """One periodic chain of n_nodes nodes spaced b (x), electrons and lattice
    at 300 K, electrons at hot_T over a span of hot_span_a0 * a0 around the
    centre node.  T_l holds the initial lattice temperature."""
    x = np.arange(n_nodes) * B_BAR
    pos = np.zeros((3, n_nodes))
    pos[0] = x
    c = n_nodes // 2 if centre is None else centre
    d = np.abs(x - x[c])
    d = np.minimum(d, n_nodes * B_BAR - d)
    Te = np.where(d <= 0.5 * hot_span_a0 * A0_BAR + 1e-9, hot_T, 300.0)
    p = default_params(T_max=T_MAX, K=K_E_BAR, dt=0.1, g=G_BAR, ce_model=CE_CONST,
                       ce_const=C_E_BAR, v_atom=V_BAR * 1e30)
    return System(pos=pos, box_lo=np.array([0.0, -1.0, -1.0]),
                  box_len=np.array([n_nodes * B_BAR, 2.0, 2.0]),
                  periodic=np.array([1, 0, 0], np.int32), T_e0=Te, params=p,
                  T_l=np.full(n_nodes, 300.0))


def c6(n_bars: int = 2048, n_nodes: int = 141, n_substeps: int = 30000,
       seed: int = 6001) -> Workload:
    """Batch of two-temperature 1D Ni bars (Section 3.1): bar 0 is the paper's
    (6,000 K over 2 a0 at the centre, 3 ps at dt = 0.1 fs); the others draw the
    hot temperature from U[3,000, 9,000] K, the span from U[1, 6] a0 and the
    centre node uniformly (seeded).  Electrons by Eq. 2 with K from Eq. 3
    (d = 1, Z = 2), lattice by the three-point Fourier stencil; the lattice
    rate and heat capacity are in extra."""
    rng = np.random.default_rng(seed)
    systems = [c6_bar(n_nodes)]
    for _ in range(n_bars - 1):
        systems.append(c6_bar(n_nodes, hot_T=float(rng.uniform(3000.0, 9000.0)),
                              hot_span_a0=float(rng.uniform(1.0, 6.0)),
                              centre=int(rng.integers(0, n_nodes))))
    return Workload("c6_ni_bar_2t_fp64", systems, r_cut=1.05 * B_BAR, n_substeps=n_substeps,
                    precision="fp64", checkpoint_every=1000,
                    extra={"K_lat": K_L_BAR, "c_lat": C_L_BAR})


def c5(n_systems: int = 64, n_cells: int = 20, n_substeps: int = 2000,
       seed: int = 5001) -> Workload:
    """Differentiation case: identical periodic FCC systems with the C1
    hotspot at the centre, constant c; per-system target parameters
    K0(1+u), g0(1+u'), u, u' ~ U[-0.2, 0.2]."""
    pos, L = fcc(n_cells, n_cells, n_cells)
    Te = gaussian_hotspot(pos, L / 2.0, 300.0, 9700.0, 8.0)
    rng = np.random.default_rng(seed)
    u = rng.uniform(-0.2, 0.2, size=(n_systems, 2))
    systems = []
    for s in range(n_systems):
        p = default_params(K=C5_K0, g=C5_G0, ce_model=CE_CONST, ce_const=C5_C)
        systems.append(System(pos=pos, box_lo=np.zeros(3), box_len=L,
                              periodic=np.ones(3, np.int32), T_e0=Te.copy(), params=p,
                              T_l=np.full(pos.shape[1], 300.0)))
    target_params = [(C5_K0 * (1.0 + u[s, 0]), C5_G0 * (1.0 + u[s, 1]))
                     for s in range(n_systems)]
    return Workload("c5_batch%d_fcc%d_adjoint" % (n_systems, n_cells), systems,
                    r_cut=1.1 * A_LAT, n_substeps=n_substeps, precision="fp32c",
                    checkpoint_every=100, extra=dict(target_params=target_params))
