"""Edge cases of the GPU path against the oracle: one atom, a free dimer, an
isolated atom in the EAM form (rho = 0, R-P4), max_steps = 0, a relaxed
start, sizes at the wave and block boundaries, and one context reused across
systems that grow and shrink."""
import numpy as np
import pytest

import oracle
from paper_1908_02038_amd import inputs

pytestmark = pytest.mark.gpu

OPEN = inputs.Box((-50.0, -50.0, -50.0), (100.0, 100.0, 100.0), (0, 0, 0))


@pytest.fixture(scope="module")
def api():
    from paper_1908_02038_amd import api as a
    return a


@pytest.mark.parametrize("pot", [inputs.lj_potential(), inputs.gupta_potential(), inputs.sw_potential()],
                         ids=["lj", "gupta", "sw"])
def test_single_atom(api, pot):
    c = api.Context(0, inputs.workload_fire(0.001, 1.0))
    e, f = c.fire_energy_forces(np.array([[0.3, -0.2, 0.1]]), OPEN, pot)
    r = c.fire_minimize(np.array([[0.3, -0.2, 0.1]]), OPEN, pot, 1e-8, 100)
    c.close()
    assert e == 0.0 and np.array_equal(f, np.zeros((1, 3)))
    assert r["stop"] == "converged" and r["iterations"] == 0
    np.testing.assert_array_equal(r["pos"], [[0.3, -0.2, 0.1]])


def test_free_dimer_relaxes_to_the_pair_minimum(api):
    pos = np.array([[0.0, 0.0, 0.0], [1.3, 0.2, -0.1]])
    fire = inputs.workload_fire(0.005, 1.0)
    c = api.Context(0, fire)
    r = c.fire_minimize(pos, OPEN, inputs.lj_potential(), 1e-10, 100000)
    c.close()
    ref = oracle.fire_minimize(pos, OPEN, inputs.lj_potential(), fire, 1e-10, 100000)
    assert r["stop"] == ref["stop"] == "converged"
    assert np.linalg.norm(r["pos"][1] - r["pos"][0]) == pytest.approx(2.0 ** (1.0 / 6.0), rel=1e-9)
    assert abs(r["energy"] - ref["energy"]) <= 1e-12 * abs(ref["energy"])


def test_isolated_atom_in_the_eam_form(api):
    """A far atom has rho = 0: no embedding energy, F'(0) = 0, no force."""
    rng = np.random.default_rng(81)
    cl = inputs.fcc_cluster(60, 3.61, 0, 0.05, rng)
    pos = np.vstack([cl, cl.mean(axis=0) + [30.0, 0.0, 0.0]])
    pot = inputs.gupta_potential()
    c = api.Context(0, inputs.workload_fire(0.001, inputs.METAL_F2A))
    e, f = c.fire_energy_forces(pos, OPEN, pot)
    c.close()
    e_ref, f_ref, ea = oracle.energy_forces(pos, OPEN, pot, want_atom_energy=True)
    assert ea[-1] == 0.0 and np.array_equal(f[-1], np.zeros(3))
    assert abs(e - e_ref) <= 1e-13 * abs(e_ref)
    assert np.abs(f - f_ref).max() <= 1e-12 * np.abs(f_ref).max()


def test_zero_steps_and_relaxed_start(api):
    s = inputs.lj_small()
    c = api.Context(0, s.fire)
    r = c.fire_minimize(s.pos, s.box, s.potential, 1e-12, 0)
    assert r["stop"] == "max_steps" and r["iterations"] == 0 and r["force_evals"] == 1
    np.testing.assert_array_equal(r["pos"], s.pos)
    e_ref, f_ref = oracle.energy_forces(s.pos, s.box, s.potential)
    assert abs(r["energy"] - e_ref) <= 1e-13 * abs(e_ref)
    assert abs(r["fmax"] - np.linalg.norm(f_ref, axis=1).max()) <= 1e-12 * r["fmax"]
    a = inputs.sw_lattice_constant()
    crystal = inputs.diamond_sites(3, 3, 3, a)
    r = c.fire_minimize(crystal, inputs.Box((0.0,) * 3, (3 * a,) * 3, (1, 1, 1)), inputs.sw_potential(), 1e-8, 50)
    c.close()
    assert r["stop"] == "converged" and r["iterations"] == 0


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 255, 256, 257, 511, 512, 513])
def test_sizes_at_wave_and_block_boundaries(api, n):
    """n atoms of a random packing in a periodic box (min distance above
    0.8 sigma): the evaluation and the first FIRE steps against the oracle."""
    rng = np.random.default_rng(82 + n)
    L = max(5.1, (n / 0.7) ** (1.0 / 3.0))
    pos = []
    while len(pos) < n:
        p = rng.uniform(0.0, L, 3)
        d = np.array(pos) - p if pos else np.zeros((0, 3))
        d -= L * np.rint(d / L)
        if not pos or np.sqrt((d ** 2).sum(axis=1)).min() > 0.8:
            pos.append(p)
    pos = np.array(pos)
    box = inputs.Box((0.0,) * 3, (L,) * 3, (1, 1, 1))
    pot = inputs.lj_potential(rc=2.5)
    fire = inputs.workload_fire(0.002, 1.0)
    c = api.Context(0, fire)
    e, f = c.fire_energy_forces(pos, box, pot)
    r = c.fire_minimize(pos, box, pot, 0.0, 10)
    c.close()
    e_ref, f_ref = oracle.energy_forces(pos, box, pot)
    assert abs(e - e_ref) <= 1e-13 * max(1.0, abs(e_ref))
    assert np.abs(f - f_ref).max() <= 1e-12 * max(1.0, np.abs(f_ref).max())
    ref = oracle.fire_minimize(pos, box, pot, fire, 0.0, 10)
    d = r["pos"] - ref["pos"]
    d -= L * np.rint(d / L)
    assert np.abs(d).max() <= 1e-12


def test_context_reused_across_growing_and_shrinking_systems(api):
    """One context: large, small, large again, another potential, then the
    first system once more; every result as from a fresh context."""
    systems = [inputs.lj_box(6, nvac=7, noise=0.07, seed=21), inputs.lj_small(),
               inputs.gupta_box(5, nvac=6, noise=0.08, seed=23), inputs.si_box(3, nvac=2, noise=0.1, seed=83),
               inputs.lj_box(6, nvac=7, noise=0.07, seed=21)]
    c = api.Context(0)
    got = []
    for s in systems:
        c.fire_set_params(s.fire)
        got.append(c.fire_minimize(s.pos, s.box, s.potential, 0.0, 30))
    c.close()
    for s, r in zip(systems, got):
        f = api.Context(0, s.fire)
        fresh = f.fire_minimize(s.pos, s.box, s.potential, 0.0, 30)
        f.close()
        np.testing.assert_array_equal(r["pos"], fresh["pos"])
        assert r["energy"] == fresh["energy"]


def test_rebuild_launched_ahead_with_too_few_ghost_slots(api, capfd, monkeypatch):
    """After a first build the host launches a rebuild without waiting for the
    number of periodic images, which the kernels read on the device.  A free
    cluster (no images) followed, in the same context, by a periodic box of
    the same size (about 5,800 images) sends the box's first build past the
    slots it was launched with: it must be detected, built again, and give
    the bits of a fresh context."""
    monkeypatch.setenv("FIRE_DEBUG", "1")
    cluster = inputs.lj_box(10, nvac=0, noise=0.03, seed=31, periodic=(0, 0, 0))
    box = inputs.lj_box(10, nvac=0, noise=0.03, seed=32)
    assert len(cluster.pos) == len(box.pos) == 4000
    c = api.Context(0, box.fire)
    c.fire_minimize(cluster.pos, cluster.box, cluster.potential, 0.0, 5)
    capfd.readouterr()
    got = c.fire_minimize(box.pos, box.box, box.potential, 1e-6, 20000)
    err = capfd.readouterr().err
    c.close()
    assert "ghost slots of a build launched ahead; again" in err, err[-2000:]
    f = api.Context(0, box.fire)
    fresh = f.fire_minimize(box.pos, box.box, box.potential, 1e-6, 20000)
    f.close()
    np.testing.assert_array_equal(got["pos"], fresh["pos"])
    assert got["iterations"] == fresh["iterations"] and got["energy"] == fresh["energy"]
    assert got["stop"] == "converged"


@pytest.mark.parametrize("case", ["wide_box", "far_cluster", "cutoff_shell"])
def test_fp32_neighbour_search_misses_no_pair(api, case):
    """The neighbour search tests distances in FP32 (coordinates relative to
    the cell grid's origin) against a cutoff widened by their rounding bound.
    Cases where that matters: a sparse gas in a 240-sigma periodic box (large
    coordinates), a crystal centred 1e4 sigma from the origin with free
    boundaries, and pairs placed within 1e-9 of the list cutoff rc + skin and
    of rc itself.  Forces must equal the brute-force oracle's."""
    rng = np.random.default_rng(91)
    pot = inputs.lj_potential(rc=2.5)
    if case == "wide_box":
        L = 240.0
        pos = rng.uniform(0.0, L, (3000, 3))
        box = inputs.Box((0.0,) * 3, (L,) * 3, (1, 1, 1))
    elif case == "far_cluster":
        s = inputs.lj_box(4, nvac=3, noise=0.05, seed=92, periodic=(0, 0, 0))
        pos = s.pos + 1.0e4
        box = inputs.Box((0.0,) * 3, (1.0,) * 3, (0, 0, 0))
    else:
        # pairs along x at separations just inside and outside rc and the
        # default list cutoff 1.12 rc, far apart from each other
        seps = [2.5 - 1e-9, 2.5 + 1e-9, 2.8 - 1e-9, 2.8 + 1e-9, 2.0, 1.2]
        pos = []
        for k, d in enumerate(seps):
            base = np.array([10.0 * k, 3.0 * k, -2.0 * k])
            pos += [base, base + [d, 0.0, 0.0]]
        pos = np.array(pos)
        box = inputs.Box((0.0,) * 3, (1.0,) * 3, (0, 0, 0))
    pos = np.array(pos, dtype=np.float64)
    c = api.Context(0, inputs.workload_fire(0.001, 1.0))
    e, f = c.fire_energy_forces(pos, box, pot)
    c.close()
    e_ref, f_ref = oracle.energy_forces(pos, box, pot)
    scale = max(1.0, np.abs(f_ref).max())
    assert abs(e - e_ref) <= 1e-12 * max(1.0, abs(e_ref))
    assert np.abs(f - f_ref).max() <= 1e-12 * scale
