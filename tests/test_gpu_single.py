"""GPU parity of the single-system path (C ABI through the ctypes binding)
against the CPU oracle on the same seeded inputs.

Tolerances: FP64 forces within 1e-12 of max|F|, energies within 1e-13
relative (summation order is the only difference); FIRE trajectories within
1e-12 over the first 20 steps; relaxed E/N within 1e-10 relative and the same minimum.
"""
import numpy as np
import pytest

import oracle
from paper_1908_02038_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    from paper_1908_02038_amd import api as a
    return a


@pytest.fixture(scope="module")
def ctx(api):
    c = api.Context(0)
    yield c
    c.close()


from systems import SMALL, min_image_diff, relaxed_parity  # noqa: E402


@pytest.mark.parametrize("name", list(SMALL))
def test_single_evaluation_fp64(ctx, name):
    s = SMALL[name]()
    e, f = ctx.fire_energy_forces(s.pos, s.box, s.potential)
    e_ref, f_ref = oracle.energy_forces(s.pos, s.box, s.potential)
    assert abs(e - e_ref) <= 1e-13 * abs(e_ref) + 1e-14
    assert np.abs(f - f_ref).max() <= 1e-12 * np.abs(f_ref).max()


@pytest.mark.parametrize("name", ["lj_6", "gupta_5", "gupta_slab"])
def test_single_evaluation_mixed(api, name):
    s = SMALL[name]()
    c = api.Context(0, precision="mixed")
    e, f = c.fire_energy_forces(s.pos, s.box, s.potential)
    c.close()
    e_ref, f_ref = oracle.energy_forces(s.pos, s.box, s.potential)
    # FP32 pair terms: per-pair relative rounding ~6e-8 on pair forces of up
    # to ~100x the net force, accumulated over ~50 neighbours
    err = np.abs(f - f_ref).max()
    fs = np.abs(f_ref).max()
    print(f"{name}: mixed max|dF| = {err:.3e} (max|F| {fs:.3e}), |dE|/|E| = {abs(e - e_ref) / abs(e_ref):.3e}")
    assert err <= 2e-5 * fs + 1e-6
    assert abs(e - e_ref) <= 1e-6 * abs(e_ref)


def test_perfect_crystal_has_zero_force(ctx):
    s = inputs.lj_box(6, nvac=0, noise=0.0)
    e, f = ctx.fire_energy_forces(s.pos, s.box, s.potential)
    assert np.abs(f).max() < 1e-12
    g = inputs.gupta_box(5, nvac=0, noise=0.0)
    e, f = ctx.fire_energy_forces(g.pos, g.box, g.potential)
    assert np.abs(f).max() < 1e-12


@pytest.mark.parametrize("name", ["lj_small", "gupta_5", "gupta_slab", "gupta_cluster"])
@pytest.mark.parametrize("k", [1, 2, 5, 20])
def test_fire_first_steps_match_oracle(api, name, k):
    s = SMALL[name]()
    c = api.Context(0, s.fire)
    r = c.fire_minimize(s.pos, s.box, s.potential, 0.0, k, trace=True)
    c.close()
    ref = oracle.fire_minimize(s.pos, s.box, s.potential, s.fire, 0.0, k, trace=True)
    assert r["stop"] == ref["stop"] == "max_steps"
    assert r["iterations"] == ref["iterations"] == k
    d = min_image_diff(r["pos"], ref["pos"], s.box)
    assert np.abs(d).max() <= 1e-12
    tr, tref = r["trace"], ref["trace"]
    assert tr.shape == tref.shape
    np.testing.assert_array_equal(tr[:, [0, 7, 8]], tref[:, [0, 7, 8]])  # i, branch, N_P>0
    np.testing.assert_allclose(tr[:, [5, 6]], tref[:, [5, 6]], rtol=1e-15)  # dt, alpha
    np.testing.assert_allclose(tr[:, 1], tref[:, 1], rtol=1e-12)  # E
    np.testing.assert_allclose(tr[:, 2:4], tref[:, 2:4], rtol=1e-9, atol=1e-13)  # fmax, f2norm
    assert np.all(np.abs(tr[:, 4] - tref[:, 4]) <= 1e-9 * np.abs(tref[:, 4]) + 1e-14)  # P


@pytest.mark.parametrize("name", ["lj_small", "gupta_5", "gupta_cluster"])
def test_full_relaxation_matches_oracle(api, name):
    """Relax to the tolerance on both sides: the same stop, E/N within 1e-10,
    the same minimum; the oracle at the GPU's final positions confirms the
    reported energy and the stop test."""
    s = SMALL[name]()
    tol = s.tol
    c = api.Context(0, s.fire)
    r = c.fire_minimize(s.pos, s.box, s.potential, tol, 20000, trace=True)
    c.close()
    ref = oracle.fire_minimize(s.pos, s.box, s.potential, s.fire, tol, 20000, trace=True)
    relaxed_parity(r, ref, s, f"{name} (rebuilds {r['rebuilds']})")
    assert r["stop"] == "converged" and r["fmax"] < tol
    # cross-evaluation: the oracle at the GPU's final positions
    e_x, f_x = oracle.energy_forces(r["pos"], s.box, s.potential)
    assert abs(e_x - r["energy"]) <= 1e-12 * abs(e_x)
    assert np.linalg.norm(f_x, axis=1).max() < tol * (1 + 1e-6)


def test_quadratic_well_closed_form(api):
    k, dt, x0 = 2.0, 0.1, 1.5
    fire = inputs.fire_params(dt, 1.0, alpha0=0.1, delaystep=5)
    c = api.Context(0, fire)
    box = inputs.Box((-1e3,) * 3, (2e3,) * 3, (0, 0, 0))
    r = c.fire_minimize(np.array([[x0, 0, 0]]), box, inputs.harmonic_potential((k, 0, 0)), 0.0, 2)
    assert r["pos"][0, 0] == pytest.approx(x0 * (1 - 3 * k * dt ** 2 + k * k * dt ** 4), rel=1e-14)
    pos = np.array([[1.0, -0.5, 0.7], [-0.2, 0.3, 0.9]])
    r = c.fire_minimize(pos, box, inputs.harmonic_potential((1.0, 10.0, 3.0)), 1e-10, 100000)
    ref = oracle.fire_minimize(pos, box, inputs.harmonic_potential((1.0, 10.0, 3.0)), fire, 1e-10, 100000)
    c.close()
    assert r["stop"] == "converged" and np.abs(r["pos"]).max() < 1e-10
    assert r["iterations"] == ref["iterations"]


def test_stop_reasons_and_errors(api):
    from paper_1908_02038_amd._lib import FireError
    s = inputs.lj_small()
    c = api.Context(0, s.fire)
    r = c.fire_minimize(s.pos, s.box, s.potential, 1e-8, 1)
    assert r["stop"] == "max_steps" and r["iterations"] == 1 and r["force_evals"] == 2
    c.fire_set_params(s.fire, vdfmax=0)
    r = c.fire_minimize(s.pos, s.box, s.potential, 1e-8, 10)
    assert r["stop"] == "maxvdotf" and r["iterations"] == 0
    c.fire_set_params(s.fire)
    bad = s.pos.copy()
    bad[5, 1] = np.nan
    with pytest.raises(FireError) as ei:
        c.fire_minimize(bad, s.box, s.potential, 1e-8, 10)
    assert ei.value.name == "FIRE_E_NONFINITE"
    bad = s.pos.copy()
    bad[7] = bad[9]
    with pytest.raises(FireError) as ei:
        c.fire_energy_forces(bad, s.box, s.potential)
    assert ei.value.name == "FIRE_E_OVERLAP"
    small = inputs.Box((0, 0, 0), (4.9, 10, 10), (1, 1, 1))
    with pytest.raises(FireError) as ei:
        c.fire_energy_forces(s.pos, small, s.potential)
    assert ei.value.name == "FIRE_E_BOX"
    # the context still works after errors
    e, _ = c.fire_energy_forces(s.pos, s.box, s.potential)
    assert np.isfinite(e)
    c.close()


def test_runs_are_bitwise_reproducible(api):
    s = SMALL["gupta_5"]()
    c = api.Context(0, s.fire)
    a = c.fire_minimize(s.pos, s.box, s.potential, 1e-6, 400)
    b = c.fire_minimize(s.pos, s.box, s.potential, 1e-6, 400)
    c.close()
    assert np.array_equal(a["pos"], b["pos"]) and a["energy"] == b["energy"]
    assert a["iterations"] == b["iterations"]


def test_trace_does_not_change_the_run(api):
    """Recording the per-iteration trace (which also accumulates energies)
    leaves the trajectory bit for bit unchanged."""
    s = SMALL["gupta_cluster"]()
    c = api.Context(0, s.fire)
    a = c.fire_minimize(s.pos, s.box, s.potential, 1e-6, 300)
    b = c.fire_minimize(s.pos, s.box, s.potential, 1e-6, 300, trace=True)
    c.close()
    assert np.array_equal(a["pos"], b["pos"]) and a["iterations"] == b["iterations"]


@pytest.mark.parametrize("name", ["lj_6", "gupta_5", "gupta_half", "gupta_slab"])
def test_hvp_matches_oracle(ctx, name):
    s = SMALL[name]()
    u = inputs.random_directions(len(s.pos), 5)
    hu = ctx.fire_hvp(s.pos, u, s.box, s.potential)
    ref = oracle.hvp(s.pos, u, s.box, s.potential)
    assert np.abs(hu - ref).max() <= 1e-11 * np.abs(ref).max()


@pytest.mark.parametrize("name", ["lj_6", "gupta_5"])
def test_halo_budget_too_small_falls_back_to_gathers(api, name, monkeypatch):
    """An LDS budget below the tiles' halos (16 KB) makes the list build
    report the overflow and the passes gather from global memory: the same
    bits as the LDS-staged default."""
    s = SMALL[name]()
    c = api.Context(0, s.fire)
    a = c.fire_minimize(s.pos, s.box, s.potential, 0.0, 30)
    c.close()
    monkeypatch.setenv("FIRE_LDS", "16384")
    c = api.Context(0, s.fire)
    b = c.fire_minimize(s.pos, s.box, s.potential, 0.0, 30)
    c.close()
    np.testing.assert_array_equal(a["pos"], b["pos"])
    assert a["energy"] == b["energy"]


def test_outgrown_halo_reservation_grows_instead_of_gathering(api, monkeypatch, capfd):
    """With a wider skin (0.25 rc) the 253,440-atom EAM-form bulk has tile
    halos beyond the default 52 KB reservation (1,664 atoms).  The list build
    then reserves room for them and keeps the LDS-staged passes; they give
    the same bits as the global-gather passes."""
    s = inputs.gupta_bulk()
    skin = 0.25 * s.potential["r_out"]
    monkeypatch.setenv("FIRE_DEBUG", "1")
    c = api.Context(0, s.fire, skin=skin)
    e_l, f_l = c.fire_energy_forces(s.pos, s.box, s.potential)
    r_l = c.fire_minimize(s.pos, s.box, s.potential, 0.0, 10)
    c.close()
    import re
    err = capfd.readouterr().err
    caps = [int(m) for m in re.findall(r"LDS for (\d+) atoms per tile block", err)]
    assert len(caps) >= 2 and min(caps) > 1664, err[-2000:]
    monkeypatch.delenv("FIRE_DEBUG")
    monkeypatch.setenv("FIRE_LDS", "0")
    c = api.Context(0, s.fire, skin=skin)
    e, f = c.fire_energy_forces(s.pos, s.box, s.potential)
    r = c.fire_minimize(s.pos, s.box, s.potential, 0.0, 10)
    c.close()
    assert e == e_l and np.array_equal(f, f_l)
    np.testing.assert_array_equal(r["pos"], r_l["pos"])
    assert r["energy"] == r_l["energy"]


@pytest.mark.parametrize("name", ["lj_6", "gupta_5", "gupta_slab", "gupta_cluster"])
def test_global_gather_path_matches_oracle(api, name, monkeypatch):
    """The passes that gather neighbour positions from global memory (used
    when a tile's halo does not fit the LDS budget; forced here) agree with
    the oracle as well, and with the default LDS-staged passes bit for bit
    (same pairs in the same order)."""
    s = SMALL[name]()
    c = api.Context(0, s.fire)
    e_l, f_l = c.fire_energy_forces(s.pos, s.box, s.potential)
    r_l = c.fire_minimize(s.pos, s.box, s.potential, 0.0, 20)
    c.close()
    monkeypatch.setenv("FIRE_LDS", "0")
    c = api.Context(0, s.fire)
    e, f = c.fire_energy_forces(s.pos, s.box, s.potential)
    r = c.fire_minimize(s.pos, s.box, s.potential, 0.0, 20)
    c.close()
    e_ref, f_ref = oracle.energy_forces(s.pos, s.box, s.potential)
    assert abs(e - e_ref) <= 1e-13 * abs(e_ref) + 1e-14
    assert np.abs(f - f_ref).max() <= 1e-12 * np.abs(f_ref).max()
    ref = oracle.fire_minimize(s.pos, s.box, s.potential, s.fire, 0.0, 20)
    assert np.abs(min_image_diff(r["pos"], ref["pos"], s.box)).max() <= 1e-12
    assert e == e_l and np.array_equal(f, f_l) and np.array_equal(r["pos"], r_l["pos"])
