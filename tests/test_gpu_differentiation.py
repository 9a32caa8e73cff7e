"""GPU checks of the differentiation form: autograd energy whose backward is
the force kernel and whose double backward is the HVP kernel, against the
oracle and finite differences; Lanczos lowest curvature against a dense
eigensolve of the oracle's Hessian."""
import numpy as np
import pytest

import oracle
from paper_1908_02038_amd import inputs
from systems import SMALL

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    from paper_1908_02038_amd import api as a
    return a


@pytest.fixture(scope="module")
def ctx(api):
    c = api.Context(0, precision="fp64")
    yield c
    c.close()


@pytest.mark.parametrize("name", ["lj_6", "gupta_5", "gupta_slab", "gupta_cluster"])
def test_autograd_gradient_is_minus_oracle_force(ctx, name):
    import torch
    from paper_1908_02038_amd import autograd
    s = SMALL[name]()
    x = torch.tensor(s.pos, dtype=torch.float64, device="cuda", requires_grad=True)
    e = autograd.energy(ctx, x, s.box, s.potential)
    (g,) = torch.autograd.grad(e, x)
    e_ref, f_ref = oracle.energy_forces(s.pos, s.box, s.potential)
    assert abs(e.item() - e_ref) <= 1e-13 * abs(e_ref)
    assert np.abs(g.cpu().numpy() + f_ref).max() <= 1e-12 * np.abs(f_ref).max()


@pytest.mark.parametrize("name", ["lj_6", "gupta_5", "gupta_half"])
def test_double_backward_is_oracle_hvp(ctx, name):
    import torch
    from paper_1908_02038_amd import autograd
    s = SMALL[name]()
    u = inputs.random_directions(len(s.pos), 9)
    x = torch.tensor(s.pos, dtype=torch.float64, device="cuda", requires_grad=True)
    ut = torch.tensor(u, dtype=torch.float64, device="cuda")
    e = autograd.energy(ctx, x, s.box, s.potential)
    (g,) = torch.autograd.grad(e, x, create_graph=True)
    (hu,) = torch.autograd.grad((g * ut).sum(), x)
    ref = oracle.hvp(s.pos, u, s.box, s.potential)
    assert np.abs(hu.cpu().numpy() - ref).max() <= 1e-11 * np.abs(ref).max()


@pytest.mark.parametrize("name", ["lj_small", "gupta_5"])
def test_gradcheck_against_finite_differences(ctx, name):
    """torch.autograd.gradcheck: analytic (force kernel) against central
    differences of the GPU energy, and gradgradcheck: the HVP kernel against
    central differences of the GPU forces.  No pair sits within the step of
    the LJ cutoff or of the taper's ends (checked on the oracle side)."""
    import torch
    from paper_1908_02038_amd import autograd
    s = SMALL[name]()
    pot = s.potential
    edges = [pot["rc"]] if pot["kind"] == "lj" else [pot["r_in"], pot["r_out"]]
    d = s.pos[:, None, :] - s.pos[None, :, :]
    for k in range(3):
        if s.box.periodic[k]:
            d[..., k] -= s.box.length[k] * np.rint(d[..., k] / s.box.length[k])
    r = np.sqrt((d ** 2).sum(-1))
    assert min(np.abs(r - e).min() for e in edges) > 4e-6  # the step moves no coordinate by more than 1e-6
    x = torch.tensor(s.pos, dtype=torch.float64, device="cuda", requires_grad=True)
    f = lambda y: autograd.energy(ctx, y, s.box, pot)  # noqa: E731
    assert torch.autograd.gradcheck(f, (x,), eps=1e-6, atol=1e-5, rtol=1e-5, fast_mode=True)
    assert torch.autograd.gradgradcheck(f, (x,), eps=1e-6, atol=1e-5, rtol=1e-4, fast_mode=True)


def dense_lowest_off_translation(s):
    """Smallest eigenvalue of the oracle's Hessian on the complement of rigid
    translations (columns H e_k from the oracle's HVP)."""
    n = len(s.pos)
    m = 3 * n
    H = np.zeros((m, m))
    for k in range(m):
        e = np.zeros((n, 3))
        e[k // 3, k % 3] = 1.0
        H[:, k] = oracle.hvp(s.pos, e, s.box, s.potential).ravel()
    H = 0.5 * (H + H.T)
    T = np.zeros((m, 3))
    for d in range(3):
        T[d::3, d] = 1.0 / np.sqrt(n)
    q, _ = np.linalg.qr(np.hstack([T, np.eye(m)]))
    Q = q[:, 3:m]
    return np.linalg.eigvalsh(Q.T @ H @ Q)


@pytest.mark.parametrize("which", ["lj", "gupta"])
def test_lanczos_equals_dense_spectrum(ctx, which):
    """With as many Lanczos steps as dimensions (and full re-orthogonalisation)
    the smallest Ritz value is the smallest eigenvalue off the translations."""
    if which == "lj":
        s = inputs.lj_box(3, nvac=1, noise=0.08, seed=41, rc=2.0)
    else:
        rng = np.random.default_rng(42)
        pos = inputs.fcc_cluster(60, 3.61, 0, 0.1, rng)
        s = inputs.System("gupta_60", pos, inputs.Box(tuple(pos.min(0) - 1), tuple(np.ptp(pos, 0) + 2), (0, 0, 0)),
                          inputs.gupta_potential(), inputs.workload_fire(0.001, inputs.METAL_F2A), 1e-6, 42)
    lam = dense_lowest_off_translation(s)
    got, res = ctx.fire_lowest_curvature(s.pos, s.box, s.potential, k=min(500, 3 * len(s.pos)),
                                         want_residual=True)
    print(f"{which}: n={len(s.pos)} lanczos {got:.12e} dense {lam[0]:.12e} (next {lam[1]:.6e}), "
          f"residual {res:.3e}")
    assert abs(got - lam[0]) <= 1e-8 * np.abs(lam).max()
    assert res <= 1e-6 * np.abs(lam).max()


def test_relaxed_crystal_has_positive_curvature(api):
    s = SMALL["lj_6"]()
    c = api.Context(0, s.fire)
    r = c.fire_minimize(s.pos, s.box, s.potential, 1e-8, 20000)
    lam, res = c.fire_lowest_curvature(r["pos"], s.box, s.potential, k=60, want_residual=True)
    c.close()
    print(f"lj_6 relaxed: lowest Ritz value {lam:.6e}, residual {res:.3e}")
    assert r["stop"] == "converged"
    assert lam - res > 0


def linear_trimer():
    """Three LJ atoms on a line, relaxed along it: the end atoms attract
    (2r < rc) while each bond is compressed, so the line is a stationary
    point whose bending modes have negative curvature (a saddle)."""
    def f_pair(r):  # -dphi/dr of 4 (r^-12 - r^-6)
        return 24.0 * (2.0 * r ** -13 - r ** -7)
    lo, hi = 1.0, 2.0 ** (1.0 / 6.0)
    for _ in range(200):  # f(r) + f(2r) = 0 on the end atom: bisection
        mid = 0.5 * (lo + hi)
        if f_pair(mid) + f_pair(2.0 * mid) > 0:
            lo = mid
        else:
            hi = mid
    r = 0.5 * (lo + hi)
    pos = np.array([[-r, 0.0, 0.0], [0.0, 0.0, 0.0], [r, 0.0, 0.0]]) + 10.0
    box = inputs.Box((0.0, 0.0, 0.0), (20.0, 20.0, 20.0), (0, 0, 0))
    return inputs.System("lj_trimer", pos, box, inputs.lj_potential(rc=2.5), inputs.workload_fire(0.005, 1.0),
                         1e-8, 0)


def test_lanczos_flags_a_saddle(ctx):
    """Negative control: at the linear trimer the dense eigensolve finds a
    negative curvature, and the Lanczos of the tests above (k as large as
    the space allows) returns it, with a small residual."""
    s = linear_trimer()
    _, f = oracle.energy_forces(s.pos, s.box, s.potential)
    assert np.abs(f).max() < 1e-12  # a stationary point
    lam = dense_lowest_off_translation(s)
    got, res = ctx.fire_lowest_curvature(s.pos, s.box, s.potential, k=9, want_residual=True)
    print(f"trimer: dense {lam[:3]}, lanczos {got:.12e} residual {res:.3e}")
    assert lam[0] < -0.1
    assert got + res < 0
    assert abs(got - lam[0]) <= 1e-8 * np.abs(lam).max()
