"""Seeded synthetic inputs for the FIRE 2.0 hot path.

This module only builds geometry and parameter records: FCC lattice sites,
vacancy choice, random displacements, boxes, and the potential / FIRE parameter
values of each workload.  It computes no energy, force or FIRE step.  Both the
CPU oracle (through the tests) and the HIP library receive its arrays as plain
inputs, so neither side can leak arithmetic into the other through it.

Workloads (FCC crystals; the paper's own structures are not available, these
stand in for the bulk, slab and many-image cases of its test set, Sec. 5.3):

* ``lj_small``   255 atoms: LJ, 4x4x4 FCC cells, a = 1.5874 sigma, site 0
                 removed, uniform noise +-0.05 sigma.
* ``lj_bulk``    131,072 sites, 655 random vacancies, Gaussian noise
                 N(0, 0.05^2) sigma.
* ``gupta_bulk`` 256,000 sites (a = 3.61 A), 2,560 vacancies, uniform noise
                 +-0.05 A.
* ``batched``    512 systems of 500-4000 atoms, half free clusters, half
                 periodic boxes, vacancy fraction U[0, 0.02], noise +-0.1 A.
* ``gupta_slab`` 2,048,000 sites, periodic in x and y, free z, 10,240
                 vacancies, uniform noise +-0.05 A.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# Conventional FCC basis in units of the lattice constant.
FCC_BASIS = np.array(
    [[0.0, 0.0, 0.0], [0.5, 0.5, 0.0], [0.5, 0.0, 0.5], [0.0, 0.5, 0.5]],
    dtype=np.float64,
)

# 1 eV / (A * amu) expressed in A / ps^2 (force-to-acceleration unit factor).
EV_PER_A_AMU_IN_A_PER_PS2 = 9648.533212331
CU_MASS_AMU = 63.546


@dataclasses.dataclass
class Box:
    lo: tuple
    length: tuple
    periodic: tuple


@dataclasses.dataclass
class System:
    """One relaxation problem: positions (n, 3) float64, box, and parameters."""

    name: str
    pos: np.ndarray
    box: Box
    potential: dict
    fire: dict
    tol: float
    seed: int


def fcc_sites(nx: int, ny: int, nz: int, a: float) -> np.ndarray:
    """FCC sites of an nx x ny x nz block of cubic cells, ordered cell by cell
    (x fastest) and basis atom within the cell."""
    ix, iy, iz = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    cells = np.stack([ix.ravel(order="F"), iy.ravel(order="F"), iz.ravel(order="F")], axis=1)
    sites = (cells[:, None, :].astype(np.float64) + FCC_BASIS[None, :, :]) * a
    return sites.reshape(-1, 3)


def lj_potential(rc: float = 2.5) -> dict:
    """Energy-shifted 12-6 Lennard-Jones, eps = sigma = 1."""
    return {"kind": "lj", "eps": 1.0, "sigma": 1.0, "rc": rc}


def gupta_potential(convention: str = "rgl") -> dict:
    """Second-moment (Gupta / RGL) form with a cubic taper between r_in and r_out."""
    return {
        "kind": "gupta",
        "A": 0.1,
        "p": 10.0,
        "q": 2.0,
        "xi": 1.2,
        "r0": 2.55,
        "r_in": 4.5,
        "r_out": 5.0,
        "convention": convention,
    }


def harmonic_potential(k=(1.0, 0.0, 0.0)) -> dict:
    """Anisotropic quadratic well E = 1/2 sum_i sum_d k_d x_id^2 (test potential)."""
    return {"kind": "harmonic", "k": tuple(float(v) for v in k)}


def fire_params(dt_start: float, f2a: float = 1.0, **over) -> dict:
    """FIRE 2.0 parameters.  Defaults are the paper's recommended set (Table 1);
    the workloads override tmax, alpha0, delay, grow and shrink factors."""
    p = {
        "dt_start": dt_start,
        "tmax": 10.0,
        "tmin": 0.02,
        "delaystep": 20,
        "dtgrow": 1.1,
        "dtshrink": 0.5,
        "alpha0": 0.25,
        "alphashrink": 0.99,
        "vdfmax": 2000,
        "halfstepback": 1,
        "initialdelay": 1,
        "integrator": "eulerimplicit",
        "f2a": f2a,
        "criterion": "fmax",
        "variant": "fire2",
    }
    p.update(over)
    return p


def workload_fire(dt_start: float, f2a: float) -> dict:
    return fire_params(dt_start, f2a, tmax=10.0, alpha0=0.1, delaystep=5, dtgrow=1.1, dtshrink=0.5)


METAL_F2A = EV_PER_A_AMU_IN_A_PER_PS2 / CU_MASS_AMU


def _remove_and_perturb(sites, nvac, noise, kind, rng, vac_sites=None):
    n = sites.shape[0]
    if vac_sites is None:
        vac_sites = np.sort(rng.choice(n, size=nvac, replace=False)) if nvac > 0 else np.zeros(0, np.int64)
    keep = np.ones(n, dtype=bool)
    keep[vac_sites] = False
    pos = sites[keep].copy()
    if kind == "uniform":
        pos += rng.uniform(-noise, noise, size=pos.shape)
    elif kind == "gauss":
        pos += rng.normal(0.0, noise, size=pos.shape)
    else:
        raise ValueError(kind)
    return pos


def _wrap(pos, box: Box):
    out = pos.copy()
    for d in range(3):
        if box.periodic[d]:
            out[:, d] = box.lo[d] + np.mod(out[:, d] - box.lo[d], box.length[d])
    return out


def fcc_box_system(name, ncell, a, nvac, noise, noise_kind, seed, potential, fire, tol,
                   periodic=(1, 1, 1), vac_sites=None) -> System:
    """Periodic (or partly periodic) FCC block with vacancies and displacements."""
    nx, ny, nz = ncell
    rng = np.random.default_rng(seed)
    sites = fcc_sites(nx, ny, nz, a)
    pos = _remove_and_perturb(sites, nvac, noise, noise_kind, rng, vac_sites)
    box = Box(lo=(0.0, 0.0, 0.0), length=(nx * a, ny * a, nz * a), periodic=tuple(int(p) for p in periodic))
    pos = _wrap(pos, box)
    return System(name, np.ascontiguousarray(pos), box, potential, fire, tol, seed)


def lj_small(seed: int = 0) -> System:
    return fcc_box_system("lj_small", (4, 4, 4), 1.5874, 1, 0.05, "uniform", seed,
                          lj_potential(), workload_fire(0.005, 1.0), 1e-8, vac_sites=np.array([0]))


def lj_bulk(seed: int = 1, ncell: int = 32) -> System:
    nsite = 4 * ncell ** 3
    # neighbour-list skin 0.15 rc (0.375 sigma) instead of the library's
    # default 0.12 rc: three list builds per relaxation instead of four, and
    # a 16-cell grid per axis for this box
    fire = dict(workload_fire(0.005, 1.0), skin=0.15 * 2.5)
    return fcc_box_system("lj_bulk", (ncell,) * 3, 1.5874, int(round(0.005 * nsite)), 0.05, "gauss",
                          seed, lj_potential(), fire, 1e-6)


def gupta_bulk(seed: int = 2, ncell: int = 40, convention: str = "rgl") -> System:
    nsite = 4 * ncell ** 3
    return fcc_box_system("gupta_bulk", (ncell,) * 3, 3.61, int(round(0.01 * nsite)), 0.05, "uniform",
                          seed, gupta_potential(convention), workload_fire(0.001, METAL_F2A), 1e-6)


def gupta_slab(seed: int = 4, ncell: int = 80) -> System:
    nsite = 4 * ncell ** 3
    return fcc_box_system("gupta_slab", (ncell,) * 3, 3.61, int(round(0.005 * nsite)), 0.05, "uniform",
                          seed, gupta_potential(), workload_fire(0.001, METAL_F2A), 1e-6,
                          periodic=(1, 1, 0))


def lj_box(ncell, nvac=0, noise=0.05, seed=0, kind="uniform", periodic=(1, 1, 1), rc=2.5, a=1.5874) -> System:
    """Generic small LJ test crystal."""
    if isinstance(ncell, int):
        ncell = (ncell,) * 3
    return fcc_box_system(f"lj_{ncell[0]}x{ncell[1]}x{ncell[2]}", ncell, a, nvac, noise, kind, seed,
                          lj_potential(rc), workload_fire(0.005, 1.0), 1e-6, periodic=periodic)


def gupta_box(ncell, nvac=0, noise=0.05, seed=0, periodic=(1, 1, 1), convention="rgl", a=3.61) -> System:
    """Generic small Gupta test crystal."""
    if isinstance(ncell, int):
        ncell = (ncell,) * 3
    return fcc_box_system(f"gupta_{ncell[0]}x{ncell[1]}x{ncell[2]}", ncell, a, nvac, noise, "uniform", seed,
                          gupta_potential(convention), workload_fire(0.001, METAL_F2A), 1e-6, periodic=periodic)


def fcc_cluster(n_target: int, a: float, nvac: int, noise: float, rng) -> np.ndarray:
    """The n_target FCC sites nearest to a lattice site (free boundaries), then
    vacancies and uniform noise."""
    m = int(math.ceil((n_target / 4.0) ** (1.0 / 3.0))) + 2
    sites = fcc_sites(2 * m, 2 * m, 2 * m, a) - m * a
    d2 = np.einsum("ij,ij->i", sites, sites)
    order = np.argsort(d2, kind="stable")[:n_target]
    sel = sites[np.sort(order)]
    return _remove_and_perturb(sel, nvac, noise, "uniform", rng)


def batched(nsys: int = 512, seed: int = 3, nmin: int = 500, nmax: int = 4000):
    """Independent systems of uneven size: even s -> free cluster, odd s ->
    periodic box.  Returns a list of System."""
    a = 3.61
    out = []
    for s in range(nsys):
        rng = np.random.default_rng([seed, s])
        n_target = int(rng.integers(nmin, nmax + 1))
        fvac = float(rng.uniform(0.0, 0.02))
        if s % 2 == 0:
            nvac = int(round(fvac * n_target))
            pos = fcc_cluster(n_target, a, nvac, 0.1, rng)
            span = pos.max(axis=0) - pos.min(axis=0)
            box = Box(lo=tuple(pos.min(axis=0) - 1.0), length=tuple(span + 2.0), periodic=(0, 0, 0))
        else:
            nxy = max(3, int(math.floor((n_target / 4.0) ** (1.0 / 3.0))))
            nz = max(3, int(round(n_target / (4.0 * nxy * nxy))))
            nsite = 4 * nxy * nxy * nz
            nvac = int(round(fvac * nsite))
            sites = fcc_sites(nxy, nxy, nz, a)
            pos = _remove_and_perturb(sites, nvac, 0.1, "uniform", rng)
            box = Box(lo=(0.0, 0.0, 0.0), length=(nxy * a, nxy * a, nz * a), periodic=(1, 1, 1))
            pos = _wrap(pos, box)
        out.append(System(f"batched_{s}", np.ascontiguousarray(pos), box, gupta_potential(),
                          workload_fire(0.001, METAL_F2A), 1e-6, seed))
    return out


WORKLOADS = {
    "lj_small": lj_small,
    "lj_bulk": lj_bulk,
    "gupta_bulk": gupta_bulk,
    "gupta_slab": gupta_slab,
    "si_slab": lambda: si_slab(),
}


def random_directions(n: int, seed: int) -> np.ndarray:
    """Unit-norm random (n, 3) direction field for Hessian-vector and
    finite-difference probes."""
    rng = np.random.default_rng(seed)
    u = rng.normal(size=(n, 3))
    return u / np.linalg.norm(u)


def frozen_border(pos: np.ndarray, box: Box, width: float, top_bits: int = 3) -> np.ndarray:
    """Per-atom freeze bits (bit d: component d fixed) for a boundary-clamped
    test case: on every free axis the atoms within `width` of the lowest
    coordinate are fixed completely (bits 7) and those within `width` of the
    highest get `top_bits` (default 3: x and y fixed, free to move along the
    surface normal of a z slab).  Periodic axes get no border."""
    fz = np.zeros(len(pos), np.uint8)
    for k in range(3):
        if box.periodic[k]:
            continue
        lo, hi = pos[:, k].min(), pos[:, k].max()
        fz[pos[:, k] < lo + width] = 7
        fz[(pos[:, k] > hi - width) & (fz == 0)] |= np.uint8(top_bits)
    return fz


def random_masses(n: int, seed: int, lo: float = 0.5, hi: float = 4.0) -> np.ndarray:
    """Seeded per-atom masses, log-uniform in [lo, hi] (a multi-species mix
    relative to the reference mass)."""
    rng = np.random.default_rng(seed)
    return np.exp(rng.uniform(np.log(lo), np.log(hi), size=n))


# Stillinger-Weber silicon, the original parameterisation (Stillinger and
# Weber 1985): eps in eV, sigma in Angstrom, the rest dimensionless.
SW_SI = {"eps": 2.1683, "sigma": 2.0951, "A": 7.049556277, "B": 0.6022245584, "p": 4.0, "q": 0.0,
         "a": 1.80, "lambda": 21.0, "gamma": 1.20}
SI_MASS = 28.0855  # g/mol
DIAMOND_BASIS = np.array([[0.0, 0.0, 0.0], [0.0, 0.5, 0.5], [0.5, 0.0, 0.5], [0.5, 0.5, 0.0],
                          [0.25, 0.25, 0.25], [0.25, 0.75, 0.75], [0.75, 0.25, 0.75], [0.75, 0.75, 0.25]])


def sw_potential() -> dict:
    return dict(SW_SI, kind="sw")


def sw_lattice_constant(pot: dict | None = None) -> float:
    """Diamond lattice constant whose nearest-neighbour distance is
    2^(1/6) sigma (where the SW pair term has its minimum)."""
    s = (pot or SW_SI)["sigma"]
    return 4.0 * 2.0 ** (1.0 / 6.0) * s / np.sqrt(3.0)


def diamond_sites(nx: int, ny: int, nz: int, a: float) -> np.ndarray:
    ix, iy, iz = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    cells = np.stack([ix.ravel(order="F"), iy.ravel(order="F"), iz.ravel(order="F")], axis=1)
    return ((cells[:, None, :].astype(np.float64) + DIAMOND_BASIS[None, :, :]) * a).reshape(-1, 3)


def si_box(ncell, nvac=0, noise=0.05, seed=0, periodic=(1, 1, 1)) -> System:
    """Diamond Si (SW equilibrium lattice constant), nvac vacancies drawn
    without replacement, uniform +-noise Angstrom per component; on a free
    axis the box spans the atoms with a margin."""
    nc = (ncell,) * 3 if np.isscalar(ncell) else tuple(ncell)
    pot = sw_potential()
    a = sw_lattice_constant(pot)
    rng = np.random.default_rng(seed)
    sites = diamond_sites(*nc, a)
    keep = np.ones(len(sites), bool)
    if nvac:
        keep[rng.choice(len(sites), nvac, replace=False)] = False
    pos = sites[keep] + rng.uniform(-noise, noise, size=(int(keep.sum()), 3))
    lo, length = [0.0] * 3, [0.0] * 3
    for d in range(3):
        if periodic[d]:
            length[d] = nc[d] * a
        else:
            lo[d] = float(pos[:, d].min() - 4.0)
            length[d] = float(np.ptp(pos[:, d]) + 8.0)
    box = Box(tuple(lo), tuple(length), tuple(int(v) for v in periodic))
    pos = _wrap(pos, box)
    fire = workload_fire(0.001, EV_PER_A_AMU_IN_A_PER_PS2 / SI_MASS)
    return System(f"si_{nc[0]}x{nc[1]}x{nc[2]}", pos, box, pot, fire, 1e-6, seed)


def si_slab(seed: int = 5, ncell: int = 16, nvac: int = 5) -> System:
    """Vacancies in a Si slab: 16^3 diamond cells (32,768 sites, 8.69 nm),
    5 vacancies -> 32,763 atoms, periodic in x and y, free z."""
    s = si_box(ncell, nvac=nvac, noise=0.05, seed=seed, periodic=(1, 1, 0))
    return System("si_slab", s.pos, s.box, s.potential, s.fire, s.tol, seed)
