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
