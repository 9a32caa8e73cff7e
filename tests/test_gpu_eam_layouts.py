"""The EAM form's three tile layouts (256-atom tiles at three or two blocks
per CU, 512-atom tiles; FIRE_EAM_LAYOUT fixes the tuner's choice) against
the FP64 oracle: the layout changes only which atoms share a block, so only
the order of the block reductions, never the pairs.

- the first 20 FIRE iterations within 1e-12 of the oracle's in position, for
  periodic, slab and cluster systems and the half-sum convention, in each
  layout;
- a 2,039-atom crystal (three full 512-atom tiles and a ragged one) relaxed
  to fmax < 1e-6 in each layout: the oracle's stop, E/N within 1e-10, the
  same minimum;
- with 512-atom tiles the global-gather passes give the LDS-staged passes'
  bits (they reduce over the same blocks).
"""
import numpy as np
import pytest

import oracle
from paper_1908_02038_amd import inputs

pytestmark = pytest.mark.gpu

from systems import SMALL, min_image_diff, relaxed_parity  # noqa: E402

LAYOUT_TEXT = {0: "256-atom tiles, three blocks per CU", 1: "256-atom tiles, two blocks per CU", 2: "512-atom tiles"}


@pytest.fixture(scope="module")
def api():
    from paper_1908_02038_amd import api as a
    return a


def crystal_2039():
    return inputs.gupta_box(8, nvac=9, noise=0.08, seed=31)


@pytest.mark.parametrize("layout", [0, 1, 2])
@pytest.mark.parametrize("name", ["gupta_5", "gupta_slab", "gupta_cluster", "gupta_half"])
def test_first_steps_in_each_layout(api, name, layout, monkeypatch):
    monkeypatch.setenv("FIRE_EAM_LAYOUT", str(layout))
    s = SMALL[name]()
    c = api.Context(0, s.fire)
    r = c.fire_minimize(s.pos, s.box, s.potential, 0.0, 20)
    info = c.fire_tuning_info()
    c.close()
    assert LAYOUT_TEXT[layout] in info, info
    ref = oracle.fire_minimize(s.pos, s.box, s.potential, s.fire, 0.0, 20)
    assert r["iterations"] == ref["iterations"] == 20
    assert np.abs(min_image_diff(r["pos"], ref["pos"], s.box)).max() <= 1e-12
    assert abs(r["energy"] - ref["energy"]) <= 1e-12 * abs(ref["energy"])


@pytest.fixture(scope="module")
def crystal_ref():
    s = crystal_2039()
    with oracle.cells():
        ref = oracle.fire_minimize(s.pos, s.box, s.potential, s.fire, s.tol, 20000, trace=True)
    return s, ref


@pytest.mark.parametrize("layout", [0, 1, 2])
def test_relaxation_in_each_layout(api, crystal_ref, layout, monkeypatch):
    s, ref = crystal_ref
    assert len(s.pos) == 2039
    monkeypatch.setenv("FIRE_EAM_LAYOUT", str(layout))
    c = api.Context(0, s.fire)
    r = c.fire_minimize(s.pos, s.box, s.potential, s.tol, 20000, trace=True)
    c.close()
    relaxed_parity(r, ref, s, f"layout {layout}")


def test_512_atom_tiles_gather_path_gives_the_same_bits(api, monkeypatch):
    s = crystal_2039()
    monkeypatch.setenv("FIRE_EAM_LAYOUT", "2")
    c = api.Context(0, s.fire)
    r_l = c.fire_minimize(s.pos, s.box, s.potential, 0.0, 20)
    e_l, f_l = c.fire_energy_forces(s.pos, s.box, s.potential)
    c.close()
    monkeypatch.setenv("FIRE_LDS", "0")
    c = api.Context(0, s.fire)
    r = c.fire_minimize(s.pos, s.box, s.potential, 0.0, 20)
    e, f = c.fire_energy_forces(s.pos, s.box, s.potential)
    c.close()
    np.testing.assert_array_equal(r["pos"], r_l["pos"])
    assert r["energy"] == r_l["energy"]
    assert e == e_l and np.array_equal(f, f_l)
