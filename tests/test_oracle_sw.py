"""Pins of the oracle's Stillinger-Weber energy and forces (the Si test case
of Sec. 5.3, original parameterisation), against facts the potential fixes
independently of any implementation: the fitted diamond crystal, the
vanishing three-body term at the tetrahedral angle, closed forms of small
clusters, a plain loop over every pair and triplet, finite differences and
symmetries."""
import numpy as np
import pytest

import oracle
from paper_1908_02038_amd import inputs

POT = inputs.sw_potential()
EPS, SIG = POT["eps"], POT["sigma"]
R0 = 2.0 ** (1.0 / 6.0) * SIG        # the pair term's minimum
OPEN = inputs.Box((-50.0, -50.0, -50.0), (100.0, 100.0, 100.0), (0, 0, 0))
TETRA = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]]) / np.sqrt(3.0)


def energy(pos, box=OPEN):
    return oracle.energy_forces(pos, box, POT)[0]


def test_diamond_crystal_is_the_fitted_minimum():
    """The parameters put the pair minimum at 2^(1/6) sigma with depth eps, and
    every bond angle of diamond is tetrahedral (no three-body energy), so the
    perfect crystal at that bond length has E/N = -2 eps and no forces."""
    a = inputs.sw_lattice_constant()
    pos = inputs.diamond_sites(3, 3, 3, a)
    box = inputs.Box((0.0, 0.0, 0.0), (3 * a,) * 3, (1, 1, 1))
    e, f = oracle.energy_forces(pos, box, POT)
    assert abs(e / len(pos) + 2 * EPS) <= 1e-9 * 2 * EPS
    assert np.abs(f).max() < 1e-12
    # and the lattice constant is the minimum of E(a): a parabola through
    # a(1 - d), a, a(1 + d) puts it within 1e-7 of a (relative)
    d = 1e-4
    ep = energy(pos * (1 + d), inputs.Box((0.0,) * 3, (3 * a * (1 + d),) * 3, (1, 1, 1)))
    em = energy(pos * (1 - d), inputs.Box((0.0,) * 3, (3 * a * (1 - d),) * 3, (1, 1, 1)))
    assert ep > e and em > e
    assert abs((ep - em) / (2 * d)) / ((ep + em - 2 * e) / d ** 2) < 1e-7


@pytest.mark.parametrize("r", [2.32, R0, 2.6])
def test_tetrahedral_cluster_has_no_three_body_energy(r):
    """A centre with four neighbours at tetrahedral angles (the ends are
    r sqrt(8/3) apart, beyond the 1.8 sigma cutoff for r > 2.31 A): E is four
    dimers exactly.  A sign slip in cos + 1/3 would leave six nonzero
    triplets."""
    assert r * np.sqrt(8.0 / 3.0) > POT["a"] * SIG
    centre = np.zeros((1, 3))
    pos = np.vstack([centre, r * TETRA])
    dimer = energy(np.array([[0.0, 0.0, 0.0], [r, 0.0, 0.0]]))
    assert dimer < 0
    assert abs(energy(pos) - 4 * dimer) <= 1e-13 * abs(dimer)


def test_linear_and_equilateral_trimers():
    """Three atoms with two bonds of length r at 180 degrees carry one triplet
    (cos + 1/3)^2 = 4/9; an equilateral triangle carries three with 25/36.
    The excess over the pair terms has the closed form lambda eps t g(r)^2."""
    r = 2.4
    g2 = np.exp(2 * POT["gamma"] * SIG / (r - POT["a"] * SIG))
    le = POT["lambda"] * EPS
    dimer = energy(np.array([[0.0, 0.0, 0.0], [r, 0.0, 0.0]]))
    lin = energy(np.array([[-r, 0.0, 0.0], [0.0, 0.0, 0.0], [r, 0.0, 0.0]]))  # ends 2r apart: no pair
    assert abs((lin - 2 * dimer) - le * 4.0 / 9.0 * g2) <= 1e-13 * abs(lin)
    tri = energy(np.array([[0.0, 0.0, 0.0], [r, 0.0, 0.0], [r / 2, r * np.sqrt(3) / 2, 0.0]]))
    assert abs((tri - 3 * dimer) - 3 * le * 25.0 / 36.0 * g2) <= 1e-13 * abs(tri)


def test_pair_term_vanishes_at_the_cutoff():
    rc = POT["a"] * SIG
    for r in (rc, rc + 1e-9, 5.0):
        assert energy(np.array([[0.0, 0.0, 0.0], [r, 0.0, 0.0]])) == 0.0
    assert abs(energy(np.array([[0.0, 0.0, 0.0], [rc - 1e-3, 0.0, 0.0]]))) < 1e-100


def _disordered(seed, periodic):
    return inputs.si_box(2, nvac=1, noise=0.25, seed=seed, periodic=periodic)


@pytest.mark.parametrize("periodic", [(1, 1, 1), (1, 1, 0), (0, 0, 0)])
def test_neighbour_sums_equal_the_plain_triplet_loop(periodic):
    s = _disordered(7, periodic)
    e, f = oracle.energy_forces(s.pos, s.box, POT)
    assert abs(e - oracle.sw_energy_direct(s.pos, s.box, POT)) <= 1e-13 * abs(e)
    assert np.abs(f.sum(axis=0)).max() <= 1e-12 * np.abs(f).max()


@pytest.mark.parametrize("periodic", [(1, 1, 1), (0, 0, 0)])
def test_forces_are_minus_the_gradient_of_the_plain_energy(periodic):
    s = _disordered(8, periodic)
    _, f = oracle.energy_forces(s.pos, s.box, POT)
    rng = np.random.default_rng(9)
    h = 1e-5
    for _ in range(12):
        i, d = rng.integers(len(s.pos)), rng.integers(3)
        xp, xm = s.pos.copy(), s.pos.copy()
        xp[i, d] += h
        xm[i, d] -= h
        fd = -(oracle.sw_energy_direct(xp, s.box, POT) - oracle.sw_energy_direct(xm, s.box, POT)) / (2 * h)
        assert abs(fd - f[i, d]) <= 1e-7 * max(1.0, abs(f[i, d]))
    # a random direction through every atom at once
    u = inputs.random_directions(len(s.pos), 10)
    fd = -(oracle.sw_energy_direct(s.pos + h * u, s.box, POT) -
           oracle.sw_energy_direct(s.pos - h * u, s.box, POT)) / (2 * h)
    assert abs(fd - (f * u).sum()) <= 1e-7 * np.abs(f).max()


def test_rotation_permutation_and_sample_forces():
    s = _disordered(11, (0, 0, 0))
    e, f = oracle.energy_forces(s.pos, s.box, POT)
    q, _ = np.linalg.qr(np.random.default_rng(12).normal(size=(3, 3)))
    c = s.pos.mean(axis=0)
    er, fr = oracle.energy_forces((s.pos - c) @ q.T, OPEN, POT)
    assert abs(er - e) <= 1e-13 * abs(e)
    assert np.abs(fr - f @ q.T).max() <= 1e-12 * np.abs(f).max()
    perm = np.random.default_rng(13).permutation(len(s.pos))
    ep, fp = oracle.energy_forces(s.pos[perm], s.box, POT)
    assert abs(ep - e) <= 1e-13 * abs(e)
    assert np.abs(fp - f[perm]).max() <= 1e-13 * np.abs(f).max()
    idx = np.array([0, 5, len(s.pos) - 1])
    fs, _ = oracle.sample_forces(s.pos, s.box, POT, idx)
    assert np.array_equal(fs, f[idx])


def test_periodic_image_invariance():
    s = _disordered(14, (1, 1, 1))
    e, f = oracle.energy_forces(s.pos, s.box, POT)
    shifted = s.pos + np.array([1.3, -2.1, 0.7])
    L = np.array(s.box.length)
    shifted = shifted - L * np.floor(shifted / L)
    e2, f2 = oracle.energy_forces(shifted, s.box, POT)
    assert abs(e2 - e) <= 1e-12 * abs(e)
    assert np.abs(f2 - f).max() <= 1e-11 * np.abs(f).max()


def test_vacancy_relaxes_below_the_crystal_energy_per_bond():
    """FIRE on a 63-atom periodic crystal with one vacancy: converges, lowers
    E, and the relaxed energy lies above the perfect crystal's (the vacancy
    costs energy) by less than the four broken bonds' 4 eps."""
    s = inputs.si_box(2, nvac=1, noise=0.05, seed=15)
    e0 = energy(s.pos, s.box)
    r = oracle.fire_minimize(s.pos, s.box, POT, s.fire, 1e-8, 20000)
    assert r["stop"] == "converged" and r["energy"] < e0
    crystal = -2 * EPS * len(s.pos)
    assert crystal < r["energy"] < crystal + 4 * EPS
