"""GPU parity of the batched path (fire_minimize_batched): many independent
FIRE 2.0 relaxations in one persistent launch, each with its own state."""
import numpy as np
import pytest

import oracle
from paper_1908_02038_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    from paper_1908_02038_amd import api as a
    return a


def small_batch(nsys=6, seed=7, nmin=150, nmax=600):
    return inputs.batched(nsys=nsys, seed=seed, nmin=nmin, nmax=nmax)


def min_image_diff(a, b, box):
    d = a - b
    for k in range(3):
        if box.periodic[k]:
            d[:, k] -= box.length[k] * np.rint(d[:, k] / box.length[k])
    return d


def test_small_batch_matches_oracle_relaxations(api):
    systems = small_batch()
    fire = systems[0].fire
    c = api.Context(0, fire)
    pos, res = c.fire_minimize_batched([(s.pos, s.box) for s in systems], systems[0].potential, 1e-6, 20000)
    c.close()
    for s, p, r in zip(systems, pos, res):
        ref = oracle.fire_minimize(s.pos, s.box, s.potential, s.fire, 1e-6, 20000)
        n = len(s.pos)
        print(f"{s.name}: n={n} gpu {r['stop']} {r['iterations']} it E/N {r['energy_per_atom']:.14f} | "
              f"oracle {ref['stop']} {ref['iterations']} it E/N {ref['energy'] / n:.14f}")
        assert r["stop"] == ref["stop"] == "converged"
        assert r["fmax"] < 1e-6
        assert abs(r["energy_per_atom"] - ref["energy"] / n) <= 1e-10 * abs(ref["energy"] / n)
        e_x, f_x = oracle.energy_forces(p, s.box, s.potential)
        assert abs(e_x - r["energy"]) <= 1e-12 * abs(e_x)
        assert np.linalg.norm(f_x, axis=1).max() < 1e-6 * (1 + 1e-6)


def test_first_steps_match_single_system_path(api):
    systems = small_batch(nsys=4, seed=8)
    fire = systems[0].fire
    c = api.Context(0, fire)
    pos, res = c.fire_minimize_batched([(s.pos, s.box) for s in systems], systems[0].potential, 0.0, 15)
    for s, p, r in zip(systems, pos, res):
        ref = oracle.fire_minimize(s.pos, s.box, s.potential, s.fire, 0.0, 15)
        assert r["stop"] == "max_steps" and r["iterations"] == 15
        assert np.abs(min_image_diff(p, ref["pos"], s.box)).max() <= 1e-12
    c.close()


def test_lj_batch_and_per_system_parameters(api):
    systems = [inputs.lj_box(4, nvac=k, noise=0.05, seed=30 + k) for k in range(1, 5)]
    params = [dict(s.fire, alpha0=a) for s, a in zip(systems, (0.1, 0.15, 0.2, 0.25))]
    c = api.Context(0, systems[0].fire)
    pos, res = c.fire_minimize_batched([(s.pos, s.box) for s in systems], systems[0].potential, 1e-6, 20000,
                                       per_sys=params)
    c.close()
    for s, prm, p, r in zip(systems, params, pos, res):
        ref = oracle.fire_minimize(s.pos, s.box, s.potential, prm, 1e-6, 20000)
        n = len(s.pos)
        assert r["stop"] == ref["stop"] == "converged"
        assert abs(r["energy_per_atom"] - ref["energy"] / n) <= 1e-10 * abs(ref["energy"] / n)


def test_a_stopped_system_does_not_disturb_the_others(api):
    systems = small_batch(nsys=5, seed=9)
    fire = systems[0].fire
    poisoned = [dict(fire) for _ in systems]
    poisoned[2]["vdfmax"] = 0  # stops with MAXVDOTF at its first iteration
    c = api.Context(0, fire)
    pos_a, res_a = c.fire_minimize_batched([(s.pos, s.box) for s in systems], systems[0].potential, 1e-6, 20000,
                                           per_sys=poisoned)
    keep = [0, 1, 3, 4]
    pos_b, res_b = c.fire_minimize_batched([(systems[k].pos, systems[k].box) for k in keep],
                                           systems[0].potential, 1e-6, 20000)
    c.close()
    assert res_a[2]["stop"] == "maxvdotf" and res_a[2]["iterations"] == 0
    assert np.array_equal(pos_a[2], systems[2].pos) or np.abs(
        min_image_diff(pos_a[2], systems[2].pos, systems[2].box)).max() < 1e-12
    for j, k in enumerate(keep):
        assert res_a[k]["iterations"] == res_b[j]["iterations"]
        assert np.array_equal(pos_a[k], pos_b[j])


def test_mixed_precision_batch(api):
    """FP32 pair terms, then FP64 below the switch: each system converges,
    the oracle agrees with its final state, and its E/N lies within 1e-6 of
    the oracle's own FP64 relaxation from the same start."""
    systems = small_batch(nsys=4, seed=10)
    c = api.Context(0, systems[0].fire, precision="mixed")
    pos, res = c.fire_minimize_batched([(s.pos, s.box) for s in systems], systems[0].potential, 1e-6, 20000)
    c.close()
    for s, p, r in zip(systems, pos, res):
        assert r["stop"] == "converged" and r["fmax"] < 1e-6
        assert r["iterations_low"] > 0 and r["precision_switched"]
        e_x, f_x = oracle.energy_forces(p, s.box, s.potential)
        assert np.linalg.norm(f_x, axis=1).max() < 1e-6 * (1 + 1e-6)
        assert abs(e_x - r["energy"]) <= 1e-12 * abs(e_x)
        ref = oracle.fire_minimize(s.pos, s.box, s.potential, s.fire, 1e-6, 20000)
        gap = abs(r["energy"] - ref["energy"]) / abs(ref["energy"])
        print(f"n {len(s.pos)}: mixed {r['iterations']} it ({r['iterations_low']} FP32), oracle {ref['iterations']} it, "
              f"|dE/N|/|E/N| {gap:.3e}")
        assert ref["stop"] == "converged" and gap <= 1e-6


def test_full_batched_workload_converges(api):
    """512 systems of 500-4000 atoms (clusters and periodic boxes): every
    system converges; a sample is cross-checked with the oracle."""
    systems = inputs.batched()
    c = api.Context(0, systems[0].fire)
    pos, res = c.fire_minimize_batched([(s.pos, s.box) for s in systems], systems[0].potential, 1e-6, 100000)
    c.close()
    stops = [r["stop"] for r in res]
    print("stops:", {k: stops.count(k) for k in set(stops)}, "iterations max", max(r["iterations"] for r in res))
    assert all(r["stop"] == "converged" for r in res)
    rng = np.random.default_rng(0)
    for k in rng.choice(len(systems), 6, replace=False):
        s = systems[k]
        e_x, f_x = oracle.energy_forces(pos[k], s.box, s.potential)
        assert abs(e_x - res[k]["energy"]) <= 1e-12 * abs(e_x)
        assert np.linalg.norm(f_x, axis=1).max() < 1e-6 * (1 + 1e-6)


def test_device_entry_point_matches_host_entry_point(api):
    """fire_minimize_batched_dev relaxes device positions in place to the same
    bits as the host-pointer call."""
    import torch
    systems = small_batch(nsys=5, seed=11)
    c = api.Context(0, systems[0].fire)
    pos_h, res_h = c.fire_minimize_batched([(s.pos, s.box) for s in systems], systems[0].potential, 1e-6, 20000)
    offs = np.cumsum([0] + [len(s.pos) for s in systems])
    d = torch.tensor(np.concatenate([s.pos for s in systems]), dtype=torch.float64, device="cuda")
    res_d = c.fire_minimize_batched_dev(d, offs, [s.box for s in systems], systems[0].potential, 1e-6, 20000)
    torch.cuda.synchronize()
    c.close()
    got = d.cpu().numpy()
    for k in range(len(systems)):
        assert res_d[k]["iterations"] == res_h[k]["iterations"]
        assert res_d[k]["energy"] == res_h[k]["energy"]
        assert np.array_equal(got[offs[k]:offs[k + 1]], pos_h[k])


def test_chunk_length_does_not_change_results(api, monkeypatch):
    """Systems advance by at most a chunk of iterations per launch, and the
    launch is replayed until none is running: short chunks (many replays,
    every system suspended and resumed often) give the bits of one long
    chunk."""
    systems = small_batch(nsys=5, seed=11)
    pot = systems[0].potential
    out = []
    for chunk in ("7", "100000"):
        monkeypatch.setenv("FIRE_BATCH_CHUNK", chunk)
        c = api.Context(0, systems[0].fire)
        out.append(c.fire_minimize_batched([(s.pos, s.box) for s in systems], pot, 1e-6, 20000))
        c.close()
    (pa, ra), (pb, rb) = out
    for a, b, x, y in zip(pa, pb, ra, rb):
        np.testing.assert_array_equal(a, b)
        assert x["iterations"] == y["iterations"] and x["energy"] == y["energy"] and x["stop"] == y["stop"]


def test_a_failing_system_does_not_disturb_the_others(api):
    """One system with a NaN coordinate (device entry point) and one with two
    atoms at the same place (host entry point): each ends with its own error
    as stop reason, and every other system gives the bits of a batch
    without them."""
    import torch
    systems = small_batch(nsys=6, seed=12)
    pot = systems[0].potential
    pos_in = [s.pos.copy() for s in systems]
    pos_in[2][7, 1] = np.nan
    pos_in[4][3] = pos_in[4][9]
    keep = [0, 1, 3, 5]
    c = api.Context(0, systems[0].fire)
    ref_pos, ref_res = c.fire_minimize_batched([(systems[k].pos, systems[k].box) for k in keep], pot, 1e-6, 20000)
    # device entry point, NaN in system 2 (and the overlap in system 4)
    offs = np.cumsum([0] + [len(p) for p in pos_in])
    d = torch.tensor(np.concatenate(pos_in), dtype=torch.float64, device="cuda")
    res_d = c.fire_minimize_batched_dev(d, offs, [s.box for s in systems], pot, 1e-6, 20000)
    torch.cuda.synchronize()
    got = d.cpu().numpy()
    # host entry point, the same poisoned batch
    pos_h, res_h = c.fire_minimize_batched([(p, s.box) for p, s in zip(pos_in, systems)], pot, 1e-6, 20000)
    c.close()
    for res, out in ((res_d, [got[offs[k]:offs[k + 1]] for k in range(len(systems))]), (res_h, pos_h)):
        assert res[2]["stop"] == "nonfinite" and res[2]["iterations"] == 0
        assert res[4]["stop"] == "overlap"
        assert np.isnan(out[2][7, 1])
        for j, k in enumerate(keep):
            assert res[k]["stop"] == ref_res[j]["stop"] == "converged"
            assert res[k]["iterations"] == ref_res[j]["iterations"] and res[k]["energy"] == ref_res[j]["energy"]
            assert np.array_equal(out[k], ref_pos[j])


def test_tuning_info_names_the_batched_team_shape(api):
    """After a batched call the context reports the persistent kernel's team
    size and chunk length (speed-only choices) and where they came from."""
    systems = small_batch(nsys=3, seed=14)
    c = api.Context(0, systems[0].fire)
    c.fire_minimize_batched([(s.pos, s.box) for s in systems], systems[0].potential, 1e-6, 20000)
    info = c.fire_tuning_info()
    c.close()
    assert info.startswith("batched: ") and "-thread teams" in info and "chunks of" in info


def _run_batched(api, monkeypatch, systems, pairs, team=None, precision="fp64", chunk=None, per_sys=None,
                 pos_in=None):
    if pairs is None:
        monkeypatch.delenv("FIRE_BATCH_PAIRS", raising=False)
    else:
        monkeypatch.setenv("FIRE_BATCH_PAIRS", pairs)
    if team:
        monkeypatch.setenv("FIRE_BATCH_TEAM", str(team))
    else:
        monkeypatch.delenv("FIRE_BATCH_TEAM", raising=False)
    if chunk:
        monkeypatch.setenv("FIRE_BATCH_CHUNK", str(chunk))
    else:
        monkeypatch.delenv("FIRE_BATCH_CHUNK", raising=False)
    c = api.Context(0, systems[0].fire, precision=precision)
    pos = pos_in if pos_in is not None else [s.pos for s in systems]
    out = c.fire_minimize_batched([(p, s.box) for p, s in zip(pos, systems)], systems[0].potential, 1e-6, 20000,
                                  per_sys=per_sys)
    info = c.fire_tuning_info()
    c.close()
    return out, info


def _assert_same_bits(a, b):
    (pa, ra), (pb, rb) = a, b
    for x, y, u, v in zip(pa, pb, ra, rb):
        np.testing.assert_array_equal(x, y)
        for k in ("stop", "iterations", "force_evals", "energy", "fmax", "dt", "alpha", "iterations_low"):
            assert u[k] == v[k], (k, u[k], v[k])


@pytest.mark.parametrize("team", [1024, 512])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_pairs_of_blocks_give_the_bits_of_teams_alone(api, monkeypatch, team, precision):
    """Every system split over a pair of blocks (two CUs exchanging
    positions, F'(rho) and records at barriers) ends with the bits of the same
    system relaxed by one block: the records of the two halves are reduced and
    added the same way in both cases."""
    systems = small_batch(nsys=6, seed=15, nmin=150, nmax=2600)
    (alone, info0) = _run_batched(api, monkeypatch, systems, "0", team, precision)
    (paired, info1) = _run_batched(api, monkeypatch, systems, "force", team, precision)
    assert "0 pairs" in info0 and "6 pairs of them for 6 systems of most work" in info1, (info0, info1)
    _assert_same_bits(alone, paired)
    for r in paired[1]:
        assert r["stop"] == "converged"


def test_pairs_on_lj_systems(api, monkeypatch):
    systems = [inputs.lj_box(k, nvac=k, noise=0.05, seed=40 + k) for k in (4, 5, 6)]
    (alone, _), (paired, info) = (_run_batched(api, monkeypatch, systems, "0"),
                                  _run_batched(api, monkeypatch, systems, "force"))
    assert "3 pairs" in info
    _assert_same_bits(alone, paired)
    for s, p, r in zip(systems, paired[0], paired[1]):
        ref = oracle.fire_minimize(s.pos, s.box, s.potential, s.fire, 1e-6, 20000)
        n = len(s.pos)
        assert r["stop"] == ref["stop"] == "converged"
        assert abs(r["energy_per_atom"] - ref["energy"] / n) <= 1e-10 * abs(ref["energy"] / n)


def test_large_systems_are_paired_by_default_and_match_the_oracle(api, monkeypatch):
    """Systems of more than 1.5 team widths get a partner block when CUs are
    spare: the default plan pairs them, with the bits of blocks alone, and the
    relaxations agree with the oracle's."""
    systems = inputs.batched(nsys=2, seed=16, nmin=2000, nmax=2600)
    (paired, info) = _run_batched(api, monkeypatch, systems, None, team=1024)
    assert "2 pairs of them for 2 systems of most work" in info, info
    (alone, _) = _run_batched(api, monkeypatch, systems, "0", team=1024)
    _assert_same_bits(alone, paired)
    for s, p, r in zip(systems, paired[0], paired[1]):
        ref = oracle.fire_minimize(s.pos, s.box, s.potential, s.fire, 1e-6, 20000)
        n = len(s.pos)
        assert r["stop"] == ref["stop"] == "converged"
        assert abs(r["energy_per_atom"] - ref["energy"] / n) <= 1e-10 * abs(ref["energy"] / n)
        e_x, f_x = oracle.energy_forces(p, s.box, s.potential)
        assert abs(e_x - r["energy"]) <= 1e-12 * abs(e_x)


def test_pairs_resume_across_chunks_and_keep_failures_apart(api, monkeypatch):
    """Forced pairs with 7-iteration chunks (every system suspended and
    resumed many times), one system with a NaN coordinate and one with two
    coinciding atoms: the failing systems end with their errors, the others
    with the bits of one long chunk of blocks alone."""
    systems = small_batch(nsys=6, seed=17, nmin=300, nmax=1800)
    pos_in = [s.pos.copy() for s in systems]
    pos_in[1][5, 0] = np.nan
    pos_in[3][2] = pos_in[3][11]
    (alone, _) = _run_batched(api, monkeypatch, systems, "0", pos_in=pos_in)
    (paired, _) = _run_batched(api, monkeypatch, systems, "force", chunk=7, pos_in=pos_in)
    assert paired[1][1]["stop"] == "nonfinite" and paired[1][3]["stop"] == "overlap"
    for k in (0, 2, 4, 5):
        np.testing.assert_array_equal(alone[0][k], paired[0][k])
        assert alone[1][k]["iterations"] == paired[1][k]["iterations"]
        assert alone[1][k]["energy"] == paired[1][k]["energy"]
        assert paired[1][k]["stop"] == "converged"
