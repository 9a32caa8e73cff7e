"""Pins of the oracle's FIRE 2.0 loop (Algorithm 2, semi-implicit Euler with
mixing after the kick as in Algorithm 4; Table 1 parameter semantics; the stop
criteria of Sec. 3.4) against closed forms on quadratic wells, where the
dynamics reduce to the textbook symplectic-Euler map of a harmonic oscillator.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1908_02038_amd import inputs

OPEN = inputs.Box((-1e3, -1e3, -1e3), (2e3, 2e3, 2e3), (0, 0, 0))


def well(k):
    return inputs.harmonic_potential(k)


def params(**over):
    p = inputs.fire_params(0.1, 1.0, tmax=10.0, alpha0=0.1, delaystep=5, dtgrow=1.1, dtshrink=0.5)
    p.update(over)
    return p


def run(x0, k, max_steps, **over):
    pos = np.array([x0], dtype=float)
    return oracle.fire_minimize(pos, OPEN, well(k), params(**over), 0.0, max_steps, trace=True)


def test_first_two_steps_of_1d_well_are_symplectic_euler():
    k, dt, x0 = 2.0, 0.1, 1.5
    r1 = run([x0, 0, 0], (k, 0, 0), 1, dt_start=dt)
    assert r1["pos"][0, 0] == pytest.approx(x0 * (1 - k * dt * dt), rel=1e-15)
    r2 = run([x0, 0, 0], (k, 0, 0), 2, dt_start=dt)
    x2 = x0 * (1 - 3 * k * dt ** 2 + k * k * dt ** 4)
    assert r2["pos"][0, 0] == pytest.approx(x2, rel=1e-14)
    tr = r2["trace"]
    assert tr[1, 7] == -1 and tr[1, 4] == 0.0  # i = 1: P = 0 goes to the P <= 0 branch
    assert tr[2, 7] == 1 and tr[2, 8] == 1  # i = 2: P > 0, N_P>0 = 1
    assert tr[2, 5] == dt and tr[2, 6] == 0.1  # still inside the delay


def test_half_step_back_after_overshoot():
    """k dt^2 = 1.44 overshoots at i = 1; at i = 2 P < 0, so x goes back by
    dt v / 2 before v is zeroed, and the kick uses the force at the
    uncorrected position."""
    x0 = 1.0
    r = run([x0, 0, 0], (1.0, 0, 0), 2, dt_start=1.2)
    assert r["trace"][2, 7] == -1
    # x1 = -0.44; back: -0.44 + 0.6 * 1.2 = 0.28; v = 1.2 * 0.44; x2 = 0.28 + 1.2 v
    assert r["pos"][0, 0] == pytest.approx(0.28 + 1.2 * 1.2 * 0.44, rel=1e-14)
    r = run([x0, 0, 0], (1.0, 0, 0), 2, dt_start=1.2, halfstepback=0)
    assert r["pos"][0, 0] == pytest.approx(-0.44 + 1.2 * 1.2 * 0.44, rel=1e-14)


def test_2d_anisotropic_well_mixing_by_hand():
    k = np.array([1.0, 10.0])
    x0 = np.array([1.0, 0.4])
    dt, a0 = 0.05, 0.1
    r = run([x0[0], x0[1], 0], (k[0], k[1], 0), 2, dt_start=dt, alpha0=a0)
    # i = 1: v = 0, kick v = dt F0, mixing of a vector parallel to F is a no-op
    f0 = -k * x0
    v1 = dt * f0
    x1 = x0 + dt * v1
    # i = 2: P = F1.v1 > 0, N_P>0 = 1 <= delay: dt, alpha unchanged
    f1 = -k * x1
    assert float(f1 @ v1) > 0
    v = v1 + dt * f1
    v = (1 - a0) * v + a0 * np.linalg.norm(v) * f1 / np.linalg.norm(f1)
    x2 = x1 + dt * v
    assert np.allclose(r["pos"][0, :2], x2, rtol=1e-14, atol=0)
    # the mixing is not a no-op here
    assert abs(x2[1] - (x1 + dt * (v1 + dt * f1))[1]) > 1e-6


def test_dt_and_alpha_schedules_after_the_delay():
    """On a soft well P stays > 0: from step N_delay + 1 on, dt grows by
    dtgrow up to tmax * dt_start and alpha shrinks by alphashrink."""
    dt0 = 0.01
    r = run([1.0, 0, 0], (1e-3, 0, 0), 60, dt_start=dt0, tmax=3.0)
    tr = r["trace"]
    assert np.all(tr[2:, 7] == 1)
    for i in range(2, 61):
        npos = i - 1  # P > 0 from i = 2
        m = max(0, npos - 5)
        dt_ref, a_ref = dt0, 0.1
        for _ in range(m):
            dt_ref = min(dt_ref * 1.1, 3.0 * dt0)
            a_ref *= 0.99
        assert tr[i, 5] == pytest.approx(dt_ref, rel=1e-14)
        assert tr[i, 6] == pytest.approx(a_ref, rel=1e-14)
    assert tr[60, 5] == 3.0 * dt0  # capped


def test_vdfmax_zero_stops_at_first_iteration():
    r = run([1.0, 0, 0], (1.0, 0, 0), 10, vdfmax=0)
    assert r["stop"] == "maxvdotf" and r["iterations"] == 0 and r["force_evals"] == 1


def test_initialdelay_off_shrinks_dt_at_first_iteration():
    r = run([1.0, 0, 0], (1.0, 0, 0), 1, initialdelay=0)
    assert r["trace"][1, 5] == 0.05 and r["trace"][1, 6] == 0.1
    r = run([1.0, 0, 0], (1.0, 0, 0), 1, initialdelay=1)
    assert r["trace"][1, 5] == 0.1


def test_dt_floor_blocks_shrink_but_alpha_resets():
    r = run([1.0, 0, 0], (1.0, 0, 0), 1, initialdelay=0, tmin=0.6, alpha0=0.2)
    assert r["trace"][1, 5] == 0.1 and r["trace"][1, 6] == 0.2


def test_consecutive_uphill_counter_and_stop():
    """A stiff well with dt far beyond stability makes every step uphill:
    the run ends with MAXVDOTF after vdfmax + 1 consecutive P <= 0 steps."""
    r = run([1.0, 0, 0], (1.0, 0, 0), 1000, dt_start=5.0, vdfmax=7, tmin=1.0, initialdelay=0)
    assert r["stop"] == "maxvdotf"
    assert r["n_neg"] == 8
    assert np.all(r["trace"][1:, 7] == -1)


def test_converges_exactly_on_anisotropic_well():
    k = (1.0, 10.0, 3.0)
    pos = np.array([[1.0, -0.5, 0.7], [-0.2, 0.3, 0.9]])
    tol = 1e-10
    r = oracle.fire_minimize(pos, OPEN, well(k), params(dt_start=0.05), tol, 100000)
    assert r["stop"] == "converged"
    assert r["fmax"] < tol
    assert np.abs(r["pos"]).max() < tol / min(k)
    assert r["force_evals"] == r["iterations"] + 1


def test_perfect_crystal_converges_without_iterating():
    s = inputs.lj_box(4, nvac=0, noise=0.0)
    r = oracle.fire_minimize(s.pos, s.box, s.potential, s.fire, 1e-8, 10)
    assert r["stop"] == "converged" and r["iterations"] == 0 and r["force_evals"] == 1


def test_max_steps_stop():
    r = run([1.0, 0, 0], (1.0, 0, 0), 1)
    assert r["stop"] == "max_steps" and r["iterations"] == 1 and r["force_evals"] == 2


def test_f2norm_criterion_is_stricter():
    s = inputs.lj_small()
    fm = oracle.fire_minimize(s.pos, s.box, s.potential, s.fire, 1e-6, 5000)
    f2 = oracle.fire_minimize(s.pos, s.box, s.potential, dict(s.fire, criterion="f2norm"), 1e-6, 5000)
    assert fm["stop"] == f2["stop"] == "converged"
    assert f2["f2norm"] < 1e-6 and fm["fmax"] < 1e-6
    assert f2["iterations"] >= fm["iterations"]
    assert fm["f2norm"] >= fm["fmax"]


def test_original_fire_shrinks_at_first_step():
    """Algorithm 1 has no initial delay: P = 0 at i = 1 halves dt at once."""
    k, dt, x0 = 2.0, 0.1, 1.5
    r = run([x0, 0, 0], (k, 0, 0), 1, dt_start=dt, variant="fire1")
    assert r["pos"][0, 0] == pytest.approx(x0 * (1 - k * (dt / 2) ** 2), rel=1e-15)


def test_explicit_euler_moves_one_evaluation_late():
    """Algorithm 3 drifts with the old velocity: x1 = x0, x2 = x0 (1 - k dt^2)."""
    k, dt, x0 = 2.0, 0.1, 1.5
    r1 = run([x0, 0, 0], (k, 0, 0), 1, dt_start=dt, integrator="eulerexplicit")
    assert r1["pos"][0, 0] == x0
    r2 = run([x0, 0, 0], (k, 0, 0), 2, dt_start=dt, integrator="eulerexplicit")
    assert r2["pos"][0, 0] == pytest.approx(x0 * (1 - k * dt * dt), rel=1e-15)


def test_velocity_verlet_first_step():
    """Algorithm 6 from rest: x1 = x0 (1 - k dt^2 / 2) and
    v1 = -dt k (x0 + x1) / 2."""
    k, dt, x0 = 2.0, 0.1, 1.5
    r = oracle.fire_minimize(np.array([[x0, 0, 0]]), OPEN, well((k, 0, 0)),
                             params(dt_start=dt, integrator="verlet"), 0.0, 1, want_velocity=True)
    x1 = x0 * (1 - 0.5 * k * dt * dt)
    assert r["pos"][0, 0] == pytest.approx(x1, rel=1e-15)
    assert r["velocity"][0, 0] == pytest.approx(-0.5 * dt * k * (x0 + x1), rel=1e-14)


def test_lj_small_relaxes_below_tolerance():
    s = inputs.lj_small()
    e0, _ = oracle.energy_forces(s.pos, s.box, s.potential)
    r = oracle.fire_minimize(s.pos, s.box, s.potential, s.fire, s.tol, 20000)
    assert r["stop"] == "converged" and r["fmax"] < s.tol
    assert r["energy"] < e0
    e1, f1 = oracle.energy_forces(r["pos"], s.box, s.potential)
    assert e1 == r["energy"]
    assert np.abs(f1.sum(0)).max() < 1e-12


# ---- frozen degrees of freedom and per-atom masses (the frozen borders and
# the multi-species systems of the test cases, Sec. 5.3)

def test_unit_masses_and_no_frozen_bits_reproduce_the_plain_run():
    s = inputs.lj_box(3, nvac=1, noise=0.08, seed=61, rc=2.0)
    a = oracle.fire_minimize(s.pos, s.box, s.potential, s.fire, 0.0, 40)
    b = oracle.fire_minimize(s.pos, s.box, s.potential, s.fire, 0.0, 40,
                             frozen=np.zeros(len(s.pos), np.uint8), mass=np.ones(len(s.pos)))
    assert np.array_equal(a["pos"], b["pos"]) and a["energy"] == b["energy"]


def test_mass_scales_the_first_kick():
    # 1-D well, one atom of mass m: the first iteration is a plain kick and
    # drift (P = 0, v = 0; mixing is the identity in 1-D), x1 = x0 (1 - k dt^2 / m)
    k, dt, m, x0 = 2.0, 0.1, 3.5, 0.7
    pos = np.array([[x0, 0.0, 0.0]])
    r = oracle.fire_minimize(pos, OPEN, well((k, 0.0, 0.0)), params(), 0.0, 1, mass=np.array([m]))
    assert r["pos"][0, 0] == pytest.approx(x0 * (1.0 - k * dt * dt / m), rel=1e-15)


def test_rescaling_masses_and_time_step_together_leaves_the_trajectory():
    # Positions evolve through dt^2 / m (kick times drift) and the FIRE state
    # through dt ratios only: masses x c with dt0 x sqrt(c) is the same run
    s = inputs.lj_box(3, nvac=1, noise=0.08, seed=62, rc=2.0)
    m = np.random.default_rng(5).uniform(0.5, 3.0, len(s.pos))
    c = 4.0
    a = oracle.fire_minimize(s.pos, s.box, s.potential, s.fire, 0.0, 60, mass=m)
    b = oracle.fire_minimize(s.pos, s.box, s.potential, dict(s.fire, dt_start=s.fire["dt_start"] * math.sqrt(c)),
                             0.0, 60, mass=c * m)
    assert np.abs(a["pos"] - b["pos"]).max() <= 1e-11


def test_frozen_atom_stays_and_its_partner_relaxes_to_the_lj_minimum():
    box = inputs.Box((-50, -50, -50), (100, 100, 100), (0, 0, 0))
    pos = np.array([[0.0, 0.0, 0.0], [1.3, 0.2, -0.1]])
    pot = inputs.lj_potential(rc=2.5)
    r = oracle.fire_minimize(pos, box, pot, inputs.workload_fire(0.005, 1.0), 1e-10, 100000,
                             frozen=np.array([7, 0], np.uint8))
    assert r["stop"] == "converged"
    assert np.array_equal(r["pos"][0], pos[0])
    assert np.linalg.norm(r["pos"][1] - r["pos"][0]) == pytest.approx(2.0 ** (1.0 / 6.0), rel=1e-9)


def test_frozen_components_never_move_and_the_rest_relaxes():
    s = inputs.lj_box(3, nvac=1, noise=0.08, seed=63, rc=2.0)
    n = len(s.pos)
    frozen = np.zeros(n, np.uint8)
    frozen[::5] = 1      # x of every 5th atom
    frozen[1::7] = 6     # y and z of every 7th
    r = oracle.fire_minimize(s.pos, s.box, s.potential, s.fire, 1e-7, 100000, frozen=frozen)
    assert r["stop"] == "converged"
    moved = r["pos"] != s.pos
    for d in range(3):
        assert not moved[(frozen & (1 << d)) > 0, d].any()
    assert moved[frozen == 0].any()
    _, f = oracle.energy_forces(r["pos"], s.box, s.potential)
    f[(frozen[:, None] & (1 << np.arange(3))[None, :]) > 0] = 0.0
    assert np.linalg.norm(f, axis=1).max() < 1e-7


# ---- dmax: the largest displacement of any atom in one step (the melt case
# of Sec. 5.3); the drift, and the half step back, use the step
# min(dt, dmax / max_i |v_i|) of the velocity they move the atoms with

def test_dmax_above_every_step_changes_nothing():
    s = inputs.lj_box(3, nvac=1, noise=0.08, seed=64, rc=2.0)
    a = oracle.fire_minimize(s.pos, s.box, s.potential, s.fire, 0.0, 60, trace=True)
    b = oracle.fire_minimize(s.pos, s.box, s.potential, dict(s.fire, dmax=1e6), 0.0, 60, trace=True)
    assert np.array_equal(a["pos"], b["pos"]) and np.array_equal(a["trace"], b["trace"])


def test_dmax_caps_the_first_step_in_a_well():
    # 1-D well: the first step's drift would move x0 -> x0 (1 - k dt^2); with
    # dmax below k dt^2 x0 the atom moves by exactly dmax toward the minimum
    k, dt, x0 = 2.0, 0.1, 1.5
    assert k * dt * dt * x0 > 0.01
    r = run([x0, 0, 0], (k, 0, 0), 1, dt_start=dt, dmax=0.01)
    assert r["pos"][0, 0] == pytest.approx(x0 - 0.01, rel=1e-15)
    r = run([x0, 0, 0], (k, 0, 0), 1, dt_start=dt, dmax=0.5)  # not binding
    assert r["pos"][0, 0] == pytest.approx(x0 * (1 - k * dt * dt), rel=1e-15)
    # dt itself is unchanged by the cap: the second step's kick still uses dt
    r = run([x0, 0, 0], (k, 0, 0), 1, dt_start=dt, dmax=0.01)
    assert r["trace"][1, 5] == dt


@pytest.mark.parametrize("integrator", ["eulerimplicit", "eulerexplicit", "verlet"])
def test_dmax_bounds_every_drift_and_binds(integrator):
    """A strongly disordered LJ start (large forces): without the half step
    back only the drift moves atoms, so between consecutive iterations no
    atom moves more than dmax, and the cap is reached."""
    s = inputs.lj_box(3, nvac=2, noise=0.2, seed=65, rc=2.0)
    dmax = 0.01
    fire = dict(s.fire, dmax=dmax, halfstepback=0, integrator=integrator, dt_start=0.01)
    prev = s.pos
    hit = 0
    for k in range(1, 16):
        r = oracle.fire_minimize(s.pos, s.box, s.potential, fire, 0.0, k)
        d = r["pos"] - prev
        for a in range(3):
            d[:, a] -= s.box.length[a] * np.rint(d[:, a] / s.box.length[a])
        step = np.linalg.norm(d, axis=1).max()
        assert step <= dmax * (1 + 1e-12)
        hit += step > dmax * (1 - 1e-12)
        prev = r["pos"]
    assert hit >= 3
    # and the capped run still relaxes
    r = oracle.fire_minimize(s.pos, s.box, s.potential, fire, 1e-6, 50000)
    assert r["stop"] == "converged"


def test_dmax_caps_the_half_step_back():
    """1-D well k = 1, x0 = 1, dt = 1.2, dmax = 1.3 (f2a = 1, no dt change
    inside the delay).  i = 1: v = -1.2 and the drift is capped to dmax:
    x1 = -0.3.  i = 2: P = F v < 0, so the half step back undoes half of a
    capped step, dt_h = dmax / |v| = 1.3 / 1.2, moving the atom by +0.65
    (uncapped: +0.72); then v = 0, the kick with F(x1) = 0.3 gives v = 0.36,
    and the drift (not binding) adds 0.432: x2 = 0.782."""
    r1 = run([1.0, 0, 0], (1.0, 0, 0), 1, dt_start=1.2, dmax=1.3)
    assert r1["pos"][0, 0] == pytest.approx(-0.3, rel=1e-14)
    r2 = run([1.0, 0, 0], (1.0, 0, 0), 2, dt_start=1.2, dmax=1.3)
    assert r2["trace"][2, 7] == -1
    assert r2["pos"][0, 0] == pytest.approx(-0.3 + 0.65 + 1.2 * 1.2 * 0.3, rel=1e-14)


def test_dmax_keeps_a_hot_start_finite():
    """A strongly disordered LJ start with restarts (P <= 0 steps, each with
    its half step back) stays finite and lowers E under the cap."""
    s = inputs.lj_box(3, nvac=2, noise=0.2, seed=66, rc=2.0)
    fire = dict(s.fire, dmax=0.01, dt_start=0.01)
    r = oracle.fire_minimize(s.pos, s.box, s.potential, fire, 0.0, 400, trace=True)
    assert (r["trace"][1:, 7] == -1).sum() > 1
    assert np.isfinite(r["pos"]).all() and r["energy"] < oracle.energy_forces(s.pos, s.box, s.potential)[0]


# ---- the placement of the mixing, hand-evaluated on a 2-D anisotropic well
# (k = (1, 10)), where a velocity built from two different forces is not
# parallel to the force and the mixing v <- (1 - a) v + a |v| F/|F| changes
# it.  delaystep = 0 makes the downhill step i = 2 grow dt and decay alpha,
# so the tests also fix whether the mixing uses alpha before or after that
# decay, and which dt each MD step uses.  Each test also shows that the
# other placement lands more than 1e-10 away (the comparison is to 1e-14).

K2 = np.array([1.0, 10.0, 0.0])
X2 = np.array([1.0, 0.4, 0.0])


def f2d(x):
    return -K2 * x


def mixv(v, f, a):
    return (1 - a) * v + a * np.linalg.norm(v) * f / np.linalg.norm(f)


FA = 0.5  # alpha decay factor (a strong decay, so that alpha before and after it differ clearly)


def run2d(steps, **over):
    fire = params(dt_start=0.05, alpha0=0.1, delaystep=0, alphashrink=FA, **over)
    return oracle.fire_minimize(np.array([X2]), OPEN, well(tuple(K2)), fire, 0.0, steps, trace=True,
                                want_velocity=True)


def first_step_dt_alpha():
    # i = 1: P = 0 is uphill; outside the (empty) initial delay dt halves and
    # alpha resets; v restarts from 0
    return 0.05 * 0.5, 0.1


def test_fire2_semi_implicit_mixing_on_2d_well():
    """Algorithm 2 with Algorithm 4: kick, mix with the decayed alpha, drift."""
    dt1, a1 = first_step_dt_alpha()
    v1 = dt1 * f2d(X2)          # the mixing of a velocity parallel to F is the identity
    x1 = X2 + dt1 * v1
    dt2, a2 = dt1 * 1.1, a1 * FA     # i = 2: downhill, N_P>0 = 1 > delaystep
    assert f2d(x1) @ v1 > 0
    v = mixv(v1 + dt2 * f2d(x1), f2d(x1), a2)
    x2 = x1 + dt2 * v
    r = run2d(2)
    np.testing.assert_allclose(r["pos"][0], x2, rtol=1e-14, atol=1e-16)
    np.testing.assert_allclose(r["velocity"][0], v, rtol=1e-14, atol=1e-16)
    assert r["trace"][2, 5] == pytest.approx(dt2, rel=1e-15) and r["trace"][2, 6] == pytest.approx(a2, rel=1e-15)
    # the alpha before the decay would give another point: the test tells them apart
    x2_wrong = x1 + dt2 * mixv(v1 + dt2 * f2d(x1), f2d(x1), a1)
    assert np.abs(x2_wrong - x2).max() > 1e-10


def test_fire1_mixes_before_the_md_step_with_alpha_before_decay():
    """Algorithm 1: on a downhill step v is mixed with F(x) first, with the
    alpha in force before this step's decay; then dt grows and the MD step
    (kick, drift) runs with the grown dt and no further mixing."""
    dt1, a1 = first_step_dt_alpha()
    v1 = dt1 * f2d(X2)
    x1 = X2 + dt1 * v1
    f1 = f2d(x1)
    assert f1 @ v1 > 0
    v = mixv(v1, f1, a1)          # mixed first, alpha not yet decayed
    dt2 = dt1 * 1.1
    v = v + dt2 * f1
    x2 = x1 + dt2 * v
    r = run2d(2, variant="fire1")
    np.testing.assert_allclose(r["pos"][0], x2, rtol=1e-14, atol=1e-16)
    np.testing.assert_allclose(r["velocity"][0], v, rtol=1e-14, atol=1e-16)
    assert r["trace"][2, 6] == pytest.approx(a1 * FA, rel=1e-15)
    # mixing after the kick (the FIRE 2.0 placement) lands elsewhere
    x2_after = x1 + dt2 * mixv(v1 + dt2 * f1, f1, a1)
    assert np.abs(x2_after - x2).max() > 1e-10


def test_fire2_explicit_euler_mixing_on_2d_well():
    """Algorithm 3: mix, drift with the mixed v, kick with the force of the
    old positions.  Step 1 does not move the atom; the velocity of step 2 is
    still parallel to the first force; step 3 is the first that mixes."""
    dt1, a1 = first_step_dt_alpha()
    f0 = f2d(X2)
    x1, v1 = X2.copy(), dt1 * f0                 # i = 1: drift with v = 0, kick with F0
    dt2, a2 = dt1 * 1.1, a1 * FA               # i = 2: P = F0.v1 > 0
    x2 = x1 + dt2 * v1                           # mixing v1 with F(x1) = F0 is the identity
    v2 = v1 + dt2 * f0
    f2 = f2d(x2)
    assert f2 @ v2 > 0
    dt3, a3 = dt2 * 1.1, a2 * FA               # i = 3
    vm = mixv(v2, f2, a3)
    x3 = x2 + dt3 * vm
    v3 = vm + dt3 * f2
    r = run2d(3, integrator="eulerexplicit")
    np.testing.assert_allclose(r["pos"][0], x3, rtol=1e-14, atol=1e-16)
    np.testing.assert_allclose(r["velocity"][0], v3, rtol=1e-14, atol=1e-16)
    # kicking before the drift (semi-implicit order) lands elsewhere
    assert np.abs((x2 + dt3 * mixv(v2 + dt3 * f2, f2, a3)) - x3).max() > 1e-10


def test_fire2_velocity_verlet_mixing_on_2d_well():
    """Algorithm 6: half kick, mix, drift, new force, half kick with it."""
    dt1, a1 = first_step_dt_alpha()
    f0 = f2d(X2)
    vh = 0.5 * dt1 * f0
    x1 = X2 + dt1 * vh
    f1 = f2d(x1)
    v1 = vh + 0.5 * dt1 * f1
    assert f1 @ v1 > 0
    dt2, a2 = dt1 * 1.1, a1 * FA
    vh = mixv(v1 + 0.5 * dt2 * f1, f1, a2)
    x2 = x1 + dt2 * vh
    f2 = f2d(x2)
    v2 = vh + 0.5 * dt2 * f2
    r = run2d(2, integrator="verlet")
    np.testing.assert_allclose(r["pos"][0], x2, rtol=1e-14, atol=1e-16)
    np.testing.assert_allclose(r["velocity"][0], v2, rtol=1e-14, atol=1e-16)
    # mixing after the second half kick instead lands elsewhere
    vw = v1 + 0.5 * dt2 * f1
    assert np.abs((x1 + dt2 * vw) - x2).max() > 1e-10
