"""Small seeded systems shared by the GPU parity tests: several 256-atom
blocks plus a ragged tail, periodic, slab and free-cluster boundaries, both
potentials and both Gupta pair conventions."""
import numpy as np

from paper_1908_02038_amd import inputs


def min_image_diff(a, b, box):
    d = a - b
    for k in range(3):
        if box.periodic[k]:
            d[:, k] -= box.length[k] * np.rint(d[:, k] / box.length[k])
    return d


SMALL = {
    "lj_small": inputs.lj_small,
    "lj_6": lambda: inputs.lj_box(6, nvac=7, noise=0.07, seed=21),  # 857 atoms: 4 blocks + ragged tail
    "lj_slab": lambda: inputs.lj_box((5, 5, 4), nvac=3, noise=0.07, seed=22, periodic=(1, 1, 0)),
    "gupta_5": lambda: inputs.gupta_box(5, nvac=6, noise=0.08, seed=23),
    "gupta_half": lambda: inputs.gupta_box(4, nvac=2, noise=0.08, seed=24, convention="half"),
    "gupta_slab": lambda: inputs.gupta_box((5, 5, 4), nvac=5, noise=0.08, seed=25, periodic=(1, 1, 0)),
    "gupta_cluster": lambda: _cluster(),
}


def _cluster():
    rng = np.random.default_rng(26)
    pos = inputs.fcc_cluster(700, 3.61, 7, 0.1, rng)
    box = inputs.Box(tuple(pos.min(0) - 1), tuple(np.ptp(pos, 0) + 2), (0, 0, 0))
    return inputs.System("gupta_cluster", pos, box, inputs.gupta_potential(),
                         inputs.workload_fire(0.001, inputs.METAL_F2A), 1e-6, 26)


def relaxed_parity(r, ref, s, label=""):
    """Parity of a GPU relaxation r with the oracle's ref from the same start.

    Both must stop for the same reason, with E/N within 1e-10 of each other
    and every coordinate within 1e-5 (one minimum: states that both stop
    with |F_i| < tol near it differ by ~F/k, far below that, while another
    minimum lies ~0.1 away).  Round-off in a different summation order can
    flip a P ~ 0 branch late in a run; the runs then reach the same minimum
    by different paths, and these bounds still hold (the first differing
    iteration is printed).  Returns that iteration or None."""
    n = len(s.pos)
    m = min(len(r["trace"]), len(ref["trace"])) if "trace" in r and "trace" in ref else 0
    diff = np.nonzero(r["trace"][:m, 7] != ref["trace"][:m, 7])[0] if m else []
    first = int(diff[0]) if len(diff) else None
    en = ref["energy"] / n
    gap = abs(r["energy_per_atom"] - en) / abs(en)
    dx = np.abs(min_image_diff(r["pos"], ref["pos"], s.box)).max()
    print(f"{label or s.name}: gpu {r['stop']} {r['iterations']} it, oracle {ref['stop']} {ref['iterations']} it, "
          f"first branch difference {first}, |dE/N|/|E/N| {gap:.3e}, max|dx| {dx:.3e}")
    assert r["stop"] == ref["stop"]
    assert gap <= 1e-10
    assert dx <= 1e-5
    return first
