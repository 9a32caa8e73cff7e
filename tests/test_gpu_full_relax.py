"""Full-size relaxations against the FP64 oracle's own relaxations
(Algorithm 2 with Algorithm 4, the Sec. 3.4 stop test), stored in
tests/golden/oracle_relaxations.json by tests/golden/make_oracle_relaxations.py
(the oracle takes minutes per relaxation at these sizes).

- FP64 (130,417-atom LJ crystal, 253,440-atom EAM-form crystal): relaxed to
  fmax < 1e-6 in the benchmark's configuration, final E/N within 1e-10 of the
  oracle's, and the same minimum (stored sample coordinates within 1e-5).
- The first 20 FP64 iterations of the LJ crystal and of the 2,037,760-atom
  slab: sampled positions within 1e-12, the FIRE branch sequence identical,
  dt and alpha to round-off.
- Mixed precision (FP32 pair terms, then FP64 below the switch): final E/N
  within 1e-6 of the FP64 oracle's (the measured gap is printed), and the
  pure FP32 path at a tolerance above its force floor.
- Batched (512 EAM-form systems in one launch): 16 systems against their own
  oracle relaxations, E/N within 1e-10.

Tolerance of the same-minimum check: both runs stop with every |F_i| < 1e-6;
near a minimum x - x* ~ F / k, and the softest long-wave modes of these
crystals have k of order 1e-2 (eV/A^2 or eps/sigma^2), so stopped states of
one minimum differ by up to ~1e-4; another minimum (a vacancy hop) is 0.1 away.
We assert 1e-5, which every recorded run meets by orders of magnitude.
"""
import hashlib
import json
import os

import numpy as np
import pytest

from paper_1908_02038_amd import inputs

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_relaxations.json")


@pytest.fixture(scope="module")
def golden():
    with open(GOLDEN) as f:
        return json.load(f)


@pytest.fixture(scope="module")
def api():
    from paper_1908_02038_amd import api as a
    return a


_CACHE = {}


def workload(name):
    if name not in _CACHE:
        _CACHE[name] = inputs.WORKLOADS[name]()
    return _CACHE[name]


def input_hash(s) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(s.pos, dtype=np.float64).tobytes())
    h.update(np.asarray(s.box.lo, np.float64).tobytes())
    h.update(np.asarray(s.box.length, np.float64).tobytes())
    h.update(np.asarray(s.box.periodic, np.int64).tobytes())
    return h.hexdigest()


def min_image_diff(a, b, box):
    d = np.asarray(a) - np.asarray(b)
    for k in range(3):
        if box.periodic[k]:
            d[:, k] -= box.length[k] * np.rint(d[:, k] / box.length[k])
    return d


def relax_dev(ctx, s, tol, max_steps):
    import torch
    x = torch.tensor(s.pos, dtype=torch.float64, device="cuda")
    r = ctx.fire_minimize_dev(x, s.box, s.potential, tol, max_steps)
    torch.cuda.synchronize()
    r["pos"] = x.cpu().numpy()
    return r


@pytest.mark.parametrize("name", ["lj_bulk", "gupta_bulk"])
def test_fp64_relaxation_matches_oracle(api, golden, name):
    g = golden[name]
    s = workload(name)
    assert input_hash(s) == g["input_sha256"], "the seeded input differs from the one the oracle relaxed"
    c = api.Context(0, s.fire, precision="fp64")
    r = relax_dev(c, s, s.tol, 100000)
    c.close()
    en = g["energy_per_atom"]
    dx = np.abs(min_image_diff(r["pos"][g["sample_idx"]], g["sample_pos"], s.box)).max()
    print(f"{name}: gpu {r['stop']} {r['iterations']} it E/N {r['energy_per_atom']:.15f} fmax {r['fmax']:.3e}; "
          f"oracle {g['stop']} {g['iterations']} it E/N {en:.15f} fmax {g['fmax']:.3e}; "
          f"|dE/N|/|E/N| {abs(r['energy_per_atom'] - en) / abs(en):.3e}; sample max|dx| {dx:.3e}")
    assert g["stop"] == r["stop"] == "converged"
    assert r["fmax"] < s.tol and g["fmax"] < s.tol
    assert abs(r["energy_per_atom"] - en) <= 1e-10 * abs(en)
    assert dx <= 1e-5


@pytest.mark.parametrize("name", ["lj_bulk", "gupta_slab"])
def test_first_20_fp64_iterations_match_oracle(api, golden, name):
    g = golden[name + "_first20"]
    s = workload(name)
    assert input_hash(s) == g["input_sha256"]
    c = api.Context(0, s.fire, precision="fp64")
    if name == "lj_bulk":
        r = c.fire_minimize(s.pos, s.box, s.potential, 0.0, 20, trace=True)
    else:
        r = relax_dev(c, s, 0.0, 20)
    c.close()
    assert r["stop"] == g["stop"] == "max_steps" and r["iterations"] == g["iterations"] == 20
    dx = np.abs(min_image_diff(r["pos"][g["sample_idx"]], g["sample_pos"], s.box)).max()
    print(f"{name}: 20 iterations, sample max|dx| {dx:.3e}, E {r['energy']:.15e} vs {g['energy']:.15e}")
    assert dx <= 1e-12
    assert abs(r["energy"] - g["energy"]) <= 1e-12 * abs(g["energy"])
    assert abs(r["fmax"] - g["fmax"]) <= 1e-9 * g["fmax"]
    assert r["dt"] == pytest.approx(g["dt"], rel=1e-15) and r["alpha"] == pytest.approx(g["alpha"], rel=1e-15)
    if "trace" in r:
        tr, tg = np.asarray(r["trace"]), np.asarray(g["trace"])
        np.testing.assert_array_equal(tr[:, [0, 7, 8]], tg[:, [0, 7, 8]])  # i, branch, N_P>0
        np.testing.assert_allclose(tr[:, [5, 6]], tg[:, [5, 6]], rtol=1e-15)
        np.testing.assert_allclose(tr[:, 1], tg[:, 1], rtol=1e-12)


@pytest.mark.parametrize("name", ["lj_bulk", "gupta_bulk"])
def test_mixed_relaxation_matches_fp64_oracle(api, golden, name):
    """FP32 pair terms until the criterion falls below the switch (100 tol),
    then FP64 to the tolerance: the relaxed E/N against the FP64 oracle's."""
    g = golden[name]
    s = workload(name)
    c = api.Context(0, s.fire, precision="mixed")
    r = relax_dev(c, s, s.tol, 100000)
    c.close()
    en = g["energy_per_atom"]
    gap = abs(r["energy_per_atom"] - en) / abs(en)
    print(f"{name} mixed: {r['stop']} {r['iterations']} it ({r['iterations_low']} with FP32 pair terms), "
          f"E/N {r['energy_per_atom']:.15f}, |dE/N|/|E/N| vs FP64 oracle {gap:.3e}")
    assert r["stop"] == "converged" and r["fmax"] < s.tol and r["precision_switched"]
    assert 0 < r["iterations_low"] < r["iterations"]
    assert gap <= 1e-6


@pytest.mark.parametrize("name", ["lj_bulk", "gupta_bulk"])
def test_pure_fp32_path(api, golden, name):
    """FIRE_FP32 keeps FP32 pair terms to the end.  Its forces carry a
    rounding floor (~1e-5 max|F_i| for these crystals), so it is run to a
    tolerance above that floor: converged, with E/N within 1e-6 of the FP64
    oracle's minimum.  At 1e-6 it cannot converge; the run must then stop on
    its own (MAXVDOTF or the step limit) with a finite state."""
    g = golden[name]
    s = workload(name)
    en = g["energy_per_atom"]
    c = api.Context(0, s.fire, precision="fp32")
    r = relax_dev(c, s, 1e-4, 100000)
    gap = abs(r["energy_per_atom"] - en) / abs(en)
    print(f"{name} fp32 to 1e-4: {r['stop']} {r['iterations']} it fmax {r['fmax']:.3e} "
          f"|dE/N|/|E/N| vs FP64 oracle {gap:.3e}")
    assert r["stop"] == "converged" and r["fmax"] < 1e-4 and not r["precision_switched"]
    assert r["iterations_low"] == r["iterations"]
    assert gap <= 1e-6
    r = relax_dev(c, s, s.tol, 3000)
    c.close()
    gap = abs(r["energy_per_atom"] - en) / abs(en)
    print(f"{name} fp32 to 1e-6: {r['stop']} after {r['iterations']} it, fmax {r['fmax']:.3e}, "
          f"|dE/N|/|E/N| {gap:.3e}")
    assert r["stop"] in ("converged", "maxvdotf", "max_steps")
    assert np.isfinite(r["energy_per_atom"]) and gap <= 1e-6


def test_batched_sample_matches_oracle(api, golden):
    """The 512-system batched workload in one persistent launch; the 16
    systems the oracle relaxed one by one agree to 1e-10 in E/N."""
    g = golden["batched_sample"]
    systems = inputs.batched()
    assert len(systems) == g["n_systems_in_batch"]
    c = api.Context(0, systems[0].fire)
    pos, res = c.fire_minimize_batched([(s.pos, s.box) for s in systems], systems[0].potential, 1e-6, 20000)
    c.close()
    assert all(r["stop"] == "converged" and r["fmax"] < 1e-6 for r in res)
    worst = 0.0
    for rec in g["systems"]:
        q = rec["system"]
        s, r = systems[q], res[q]
        assert input_hash(s) == rec["input_sha256"]
        en = rec["energy_per_atom"]
        gap = abs(r["energy_per_atom"] - en) / abs(en)
        worst = max(worst, gap)
        dx = np.abs(min_image_diff(pos[q][rec["sample_idx"]], rec["sample_pos"], s.box)).max()
        print(f"system {q} (n {rec['n']}): gpu {r['iterations']} it, oracle {rec['iterations']} it, "
              f"|dE/N|/|E/N| {gap:.3e}, sample max|dx| {dx:.3e}")
        assert rec["stop"] == "converged"
        assert gap <= 1e-10
        assert dx <= 1e-5
    print(f"worst E/N gap over the sample {worst:.3e}")


def test_batched_sample_mixed_matches_fp64_oracle(api, golden):
    """The 512-system batch with FP32 pair terms until each system's
    criterion falls below its switch (100 tol), then FP64: every system
    converges, and the 16 systems the oracle relaxed in FP64 agree with it
    to 1e-6 in E/N (the mixed path's bound)."""
    g = golden["batched_sample"]
    systems = inputs.batched()
    c = api.Context(0, systems[0].fire, precision="mixed")
    pos, res = c.fire_minimize_batched([(s.pos, s.box) for s in systems], systems[0].potential, 1e-6, 20000)
    c.close()
    assert all(r["stop"] == "converged" and r["fmax"] < 1e-6 for r in res)
    worst = 0.0
    for rec in g["systems"]:
        q = rec["system"]
        r = res[q]
        assert r["precision_switched"] and 0 < r["iterations_low"] < r["iterations"]
        en = rec["energy_per_atom"]
        gap = abs(r["energy_per_atom"] - en) / abs(en)
        worst = max(worst, gap)
        assert gap <= 1e-6
    print(f"mixed batch: worst E/N gap to the FP64 oracle over the sample {worst:.3e}")
