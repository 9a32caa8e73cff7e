"""The no-allocation batched entry point (fire_minimize_batched_noalloc)
against fire_minimize_batched_dev through the C ABI: the same kernels on
work buffers in the library's scratch array, so the same bits when both use
one team shape.  Two calls in a row, the second with a smaller batch (the
array keeps the first call's contents, which must not leak into the second),
then the limits."""
import numpy as np
import pytest

from paper_1908_02038_amd import inputs

pytestmark = pytest.mark.gpu


def batch(nsys, seed, nmin, nmax):
    return inputs.batched(nsys=nsys, seed=seed, nmin=nmin, nmax=nmax)


def run(ctx, systems, noalloc, per_sys=None, max_steps=20000):
    import torch
    offs = np.cumsum([0] + [len(s.pos) for s in systems])
    d = torch.tensor(np.concatenate([s.pos for s in systems]), dtype=torch.float64, device="cuda")
    res = ctx.fire_minimize_batched_dev(d, offs, [s.box for s in systems], systems[0].potential, 1e-6, max_steps,
                                        per_sys=per_sys, noalloc=noalloc)
    torch.cuda.synchronize()
    return d.cpu().numpy(), res


def test_noalloc_matches_the_allocating_entry_point(monkeypatch):
    from paper_1908_02038_amd import api
    monkeypatch.setenv("FIRE_BATCH_TEAM", "1024")
    first = batch(12, 14, 400, 1500)
    second = batch(5, 15, 150, 600)  # smaller: fewer systems and atoms
    c = api.Context(0, first[0].fire)
    for systems in (first, second):
        ref_pos, ref_res = run(c, systems, noalloc=False)
        got_pos, got_res = run(c, systems, noalloc=True)
        assert np.array_equal(got_pos, ref_pos)
        for a, b in zip(got_res, ref_res):
            assert a == b
        assert all(r["stop"] == "converged" for r in got_res)
    c.close()


def test_noalloc_per_system_parameters_and_failures(monkeypatch):
    from paper_1908_02038_amd import api
    monkeypatch.setenv("FIRE_BATCH_TEAM", "1024")
    systems = batch(6, 16, 200, 700)
    systems[3].pos[5, 0] = np.nan
    params = [dict(s.fire, alpha0=a) for s, a in zip(systems, (0.1, 0.12, 0.15, 0.2, 0.25, 0.3))]
    c = api.Context(0, systems[0].fire)
    ref_pos, ref_res = run(c, systems, noalloc=False, per_sys=params)
    got_pos, got_res = run(c, systems, noalloc=True, per_sys=params)
    c.close()
    assert got_res[3]["stop"] == "nonfinite"
    np.testing.assert_array_equal(got_pos, ref_pos)
    assert got_res == ref_res


def test_noalloc_rejects_a_batch_beyond_its_scratch():
    from paper_1908_02038_amd import api
    from paper_1908_02038_amd._lib import FireError
    import torch
    s = inputs.gupta_box(10, nvac=0, noise=0.05, seed=17)  # 4,000 atoms per system
    systems = [s] * 60                                       # 240,000 atoms in all
    c = api.Context(0, s.fire)
    offs = np.cumsum([0] + [len(x.pos) for x in systems])
    d = torch.tensor(np.concatenate([x.pos for x in systems]), dtype=torch.float64, device="cuda")
    before = d.clone()
    with pytest.raises(FireError) as e:
        c.fire_minimize_batched_dev(d, offs, [x.box for x in systems], s.potential, 1e-6, 100, noalloc=True)
    torch.cuda.synchronize()
    assert e.value.name == "FIRE_E_ARG"
    assert torch.equal(d, before)
    c.close()
