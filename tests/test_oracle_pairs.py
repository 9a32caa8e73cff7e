"""Pins of the oracle's pair set (the sums of Sec. 2.1 run over every pair
closer than the cutoff under the minimum image).

- An independent enumeration: every pair and every periodic image
  x_j + n L (n in {-1, 0, 1} on periodic axes) tested explicitly in numpy,
  with no minimum-image rounding.  With rc < L/2 at most one image of j lies
  within rc of i, and that set must be exactly the oracle's.
- The cell-grid search finds the same pairs in the same order as testing every
  pair, so energies, forces, Hessian products and FIRE trajectories are
  bit-identical with and without it (the cells only make the full-size
  workloads affordable).
"""
import itertools

import numpy as np
import pytest

import oracle
from paper_1908_02038_amd import inputs


def explicit_image_pairs(pos, box, rc):
    """Sorted partner lists from every pair and every image, O(n^2 * 27)."""
    n = len(pos)
    shifts = [np.array(s, dtype=float) * np.asarray(box.length)
              for s in itertools.product(*[(-1, 0, 1) if box.periodic[a] else (0,) for a in range(3)])]
    lists = [[] for _ in range(n)]
    seps = [[] for _ in range(n)]
    for i in range(n):
        for sh in shifts:
            d = pos[i][None, :] - (pos + sh[None, :])
            r2 = (d * d).sum(1)
            for j in np.nonzero(r2 < rc * rc)[0]:
                if j != i:
                    lists[i].append(int(j))
                    seps[i].append(d[j])
    order = [np.argsort(l, kind="stable") for l in lists]
    return [[lists[i][k] for k in order[i]] for i in range(n)], [[seps[i][k] for k in order[i]] for i in range(n)]


def tiny_systems():
    rng = np.random.default_rng(71)
    lj_box = inputs.lj_box(4, nvac=2, noise=0.12, seed=72)                              # 254 atoms, periodic
    lj_slab = inputs.lj_box((4, 4, 2), nvac=1, noise=0.12, seed=73, periodic=(1, 1, 0))
    gu_box = inputs.gupta_box(3, nvac=1, noise=0.1, seed=74)
    pos = inputs.fcc_cluster(80, 3.61, 2, 0.1, rng)
    cluster = inputs.System("cluster", pos, inputs.Box(tuple(pos.min(0) - 1), tuple(np.ptp(pos, 0) + 2), (0, 0, 0)),
                            inputs.gupta_potential(), inputs.workload_fire(0.001, inputs.METAL_F2A), 1e-6, 75)
    return {"lj_box": lj_box, "lj_slab": lj_slab, "gupta_box": gu_box, "gupta_cluster": cluster}


def cutoff(pot):
    return pot["rc"] if pot["kind"] == "lj" else pot["r_out"]


@pytest.mark.parametrize("name", list(tiny_systems()))
def test_pair_set_is_the_explicit_image_enumeration(name):
    s = tiny_systems()[name]
    rc = cutoff(s.potential)
    ref, _ = explicit_image_pairs(s.pos, s.box, rc)
    for cells in (False, True):
        with oracle.cells(cells):
            start, idx = oracle.pair_list(s.pos, s.box, rc)
        got = [list(idx[start[i]:start[i + 1]]) for i in range(len(s.pos))]
        assert got == ref
    assert sum(len(l) for l in ref) > 20 * len(s.pos)  # the systems are dense enough to matter


@pytest.mark.parametrize("name", ["lj_box", "lj_slab"])
def test_lj_energy_and_forces_over_explicit_images(name):
    """E and F from the explicitly enumerated images (pair terms written from
    the definition of the energy-shifted potential) against the oracle."""
    s = tiny_systems()[name]
    p = s.potential
    rc = cutoff(p)
    _, seps = explicit_image_pairs(s.pos, s.box, rc)
    sig, eps = p["sigma"], p["eps"]
    shift = 4 * eps * ((sig / rc) ** 12 - (sig / rc) ** 6)
    e = 0.0
    f = np.zeros_like(s.pos)
    for i, lst in enumerate(seps):
        for d in lst:
            r = np.linalg.norm(d)
            e += 0.5 * (4 * eps * ((sig / r) ** 12 - (sig / r) ** 6) - shift)
            f[i] += 24 * eps * (2 * (sig / r) ** 12 - (sig / r) ** 6) / r ** 2 * d
    e_o, f_o = oracle.energy_forces(s.pos, s.box, p)
    assert e_o == pytest.approx(e, rel=1e-13)
    assert np.abs(f_o - f).max() <= 1e-12 * np.abs(f).max()


@pytest.mark.parametrize("name", ["gupta_box", "gupta_cluster"])
def test_gupta_densities_over_explicit_images(name):
    s = tiny_systems()[name]
    p = s.potential
    _, seps = explicit_image_pairs(s.pos, s.box, p["r_out"])

    def taper(r):
        t = np.clip((r - p["r_in"]) / (p["r_out"] - p["r_in"]), 0.0, 1.0)
        return (1 - t) ** 2 * (1 + 2 * t)

    rho = np.array([sum(np.exp(-2 * p["q"] * (np.linalg.norm(d) / p["r0"] - 1)) * taper(np.linalg.norm(d))
                        for d in lst) for lst in seps])
    _, _, rho_o = oracle.energy_forces(s.pos, s.box, p, want_rho=True)
    np.testing.assert_allclose(rho_o, rho, rtol=1e-13)


def cell_edge_systems():
    out = dict(tiny_systems())
    # two cells per periodic axis (neighbour offsets -1 and +1 are the same cell)
    out["lj_two_cells"] = inputs.lj_box(4, nvac=3, noise=0.1, seed=76, rc=2.5)
    # one cell on the free axis of a thin slab
    out["lj_thin_slab"] = inputs.lj_box((4, 4, 1), nvac=0, noise=0.1, seed=77, periodic=(1, 1, 0), rc=2.0)
    # a sparse cloud in a wide free box
    rng = np.random.default_rng(78)
    pos = rng.uniform(0, 40, size=(60, 3))
    out["sparse"] = inputs.System("sparse", pos, inputs.Box((0, 0, 0), (40, 40, 40), (0, 0, 0)),
                                  inputs.lj_potential(rc=2.5), inputs.workload_fire(0.005, 1.0), 1e-6, 78)
    # the workload crystal itself (255 atoms, 2 cells per axis)
    out["lj_small"] = inputs.lj_small()
    out["gupta_half"] = inputs.gupta_box(4, nvac=2, noise=0.08, seed=79, convention="half")
    out["si_box"] = inputs.si_box(2, nvac=1, noise=0.05, seed=80)
    return out


@pytest.mark.parametrize("name", list(cell_edge_systems()))
def test_cell_search_gives_bit_identical_results(name):
    s = cell_edge_systems()[name]
    pot = s.potential
    rc = pot.get("rc", pot.get("r_out")) if pot["kind"] != "sw" else pot["a"] * pot["sigma"]
    u = np.random.default_rng(81).normal(size=s.pos.shape)
    fire = dict(s.fire, dt_start=s.fire["dt_start"])
    res = {}
    for cells in (False, True):
        with oracle.cells(cells):
            start, idx = oracle.pair_list(s.pos, s.box, rc)
            e, f, ea = oracle.energy_forces(s.pos, s.box, pot, want_atom_energy=True)
            h = oracle.hvp(s.pos, u, s.box, pot) if pot["kind"] != "sw" else np.zeros(1)
            r = oracle.fire_minimize(s.pos, s.box, pot, fire, 0.0, 25, trace=True)
        res[cells] = (start, idx, e, f, ea, h, r["pos"], r["trace"])
    for a, b in zip(res[False], res[True]):
        assert np.array_equal(np.asarray(a), np.asarray(b))


def test_cell_search_finds_overlaps():
    s = inputs.lj_box(4, nvac=0, noise=0.0)
    pos = s.pos.copy()
    pos[5] = pos[17]
    for cells in (False, True):
        with oracle.cells(cells), pytest.raises(oracle.OracleError) as e:
            oracle.energy_forces(pos, s.box, s.potential)
        assert e.value.name == "E_OVERLAP"


def test_sampled_forces_are_the_full_evaluation():
    for s in (inputs.lj_box(4, nvac=3, noise=0.1, seed=82), inputs.gupta_box(4, nvac=3, noise=0.1, seed=83),
              inputs.si_box(2, nvac=1, noise=0.05, seed=84)):
        idx = np.array([0, 3, len(s.pos) // 2, len(s.pos) - 1])
        _, f, ea = oracle.energy_forces(s.pos, s.box, s.potential, want_atom_energy=True)
        fs, es = oracle.sample_forces(s.pos, s.box, s.potential, idx)
        assert np.array_equal(fs, f[idx]) and np.array_equal(es, ea[idx])
