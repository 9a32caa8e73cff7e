"""GPU parity at the workloads' full sizes (130,417 / 253,440 / 2,037,760
atoms), in the launch configuration the benchmark times (global-gather passes,
graph-replayed FIRE loop).  The oracle is brute force, so it evaluates a
sample of atoms one by one: random atoms plus atoms next to the periodic faces
and the free surfaces, where the periodic images and the ghost slots matter.
Properties that hold at any size (sum of forces, relaxed minimum) cover the
rest."""
import numpy as np
import pytest

import oracle
from paper_1908_02038_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    from paper_1908_02038_amd import api as a
    return a


_CACHE = {}


def workload(name):
    if name not in _CACHE:
        _CACHE[name] = inputs.WORKLOADS[name]()
    return _CACHE[name]


def sample(s, m, seed):
    """m random atoms plus the atoms nearest each face of the box (lo and hi
    side of every axis) and, on free axes, the outermost atoms."""
    rng = np.random.default_rng(seed)
    idx = set(rng.choice(len(s.pos), m, replace=False).tolist())
    for k in range(3):
        o = np.argsort(s.pos[:, k])
        idx.update(o[:4].tolist())
        idx.update(o[-4:].tolist())
    return np.array(sorted(idx), dtype=np.int64)


def check_sampled_forces(f_gpu, s, idx, rel, abs_=0.0):
    f_ref, _ = oracle.sample_forces(s.pos, s.box, s.potential, idx)
    scale = np.abs(f_ref).max()
    err = np.abs(f_gpu[idx] - f_ref).max()
    print(f"{s.name}: {len(idx)} sampled atoms, max|F| {scale:.4g}, max err {err:.3e}")
    assert err <= rel * scale + abs_


@pytest.mark.parametrize("name", ["lj_bulk", "gupta_bulk", "gupta_slab"])
def test_full_size_forces_fp64(api, name):
    s = workload(name)
    c = api.Context(0, s.fire, precision="fp64")
    e, f = c.fire_energy_forces(s.pos, s.box, s.potential)
    c.close()
    check_sampled_forces(f, s, sample(s, 48 if name == "gupta_slab" else 160, 1), 1e-12)
    # Newton's third law over the whole system: the pair terms cancel exactly
    # up to the rounding of each atom's own sum
    fs = np.abs(f.sum(axis=0)).max()
    assert fs <= 1e-13 * len(s.pos) * np.abs(f).max()
    if name == "lj_bulk":  # the oracle's full O(N^2) energy still takes seconds here
        e_ref, _ = oracle.energy_forces(s.pos, s.box, s.potential)
        assert abs(e - e_ref) <= 1e-13 * abs(e_ref)


@pytest.mark.parametrize("name", ["lj_bulk", "gupta_bulk", "gupta_slab"])
def test_full_size_forces_mixed(api, name):
    s = workload(name)
    c = api.Context(0, s.fire, precision="mixed")
    _, f = c.fire_energy_forces(s.pos, s.box, s.potential)
    c.close()
    check_sampled_forces(f, s, sample(s, 48 if name == "gupta_slab" else 160, 2), 2e-5, 1e-6)


def test_lj_bulk_relaxation_cross_evaluated(api):
    """The benchmark's step: relax the 130,417-atom LJ crystal to fmax < 1e-6
    with the FP64 path; the oracle at the GPU's final positions (sampled,
    including the atom the GPU finds with the largest force) confirms it."""
    import torch
    s = workload("lj_bulk")
    c = api.Context(0, s.fire, precision="fp64")
    x = torch.tensor(s.pos, dtype=torch.float64, device="cuda")
    r = c.fire_minimize_dev(x, s.box, s.potential, s.tol, 100000)
    torch.cuda.synchronize()
    pos = x.cpu().numpy()
    _, f = c.fire_energy_forces(pos, s.box, s.potential)
    c.close()
    assert r["stop"] == "converged" and r["fmax"] < s.tol
    fn = np.linalg.norm(f, axis=1)
    assert abs(fn.max() - r["fmax"]) <= 1e-3 * r["fmax"]
    relaxed = inputs.System(s.name, pos, s.box, s.potential, s.fire, s.tol, s.seed)
    idx = np.union1d(sample(relaxed, 160, 3), np.argsort(fn)[-8:])
    f_ref, _ = oracle.sample_forces(pos, s.box, s.potential, idx)
    assert np.linalg.norm(f_ref, axis=1).max() < s.tol
    assert np.abs(f[idx] - f_ref).max() <= 1e-11


def test_slab_relaxation_is_a_minimum(api):
    """The 2,037,760-atom EAM-form slab (periodic x, y; free z), mixed
    precision: relaxed to fmax < 1e-6, confirmed by the oracle on a sample of
    the final positions, and its lowest curvature off the rigid translations
    (Lanczos on the HVP kernel) is positive."""
    import torch
    s = workload("gupta_slab")
    c = api.Context(0, s.fire, precision="mixed")
    x = torch.tensor(s.pos, dtype=torch.float64, device="cuda")
    r = c.fire_minimize_dev(x, s.box, s.potential, s.tol, 100000)
    torch.cuda.synchronize()
    pos = x.cpu().numpy()
    print(f"slab: {r['stop']} after {r['iterations']} iterations ({r['iterations_low']} with FP32 pair terms), "
          f"E/N {r['energy_per_atom']:.12f}, fmax {r['fmax']:.3e}")
    assert r["stop"] == "converged" and r["fmax"] < s.tol and r["precision_switched"]
    relaxed = inputs.System(s.name, pos, s.box, s.potential, s.fire, s.tol, s.seed)
    idx = sample(relaxed, 40, 4)
    f_ref, _ = oracle.sample_forces(pos, s.box, s.potential, idx)
    assert np.linalg.norm(f_ref, axis=1).max() < s.tol
    lam = c.fire_lowest_curvature(pos, s.box, s.potential, k=30)
    c.close()
    print(f"slab: lowest Ritz value {lam:.6e} eV/A^2")
    assert lam > 0
