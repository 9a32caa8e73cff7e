"""CPU FP64 oracle for the FIRE 2.0 hot path -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  It wraps ``oracle.c`` (plain C, brute-force pair sums, FP64)
through ctypes and shares nothing with the HIP library.

Functions (paper: Guenole et al., FIRE 2.0):
  energy_forces   E and F = -grad E (Sec. 2.1) for LJ, Gupta (Sec. 5.2 EAM form),
                  Stillinger-Weber (the Si case of Sec. 5.3) and a quadratic
                  test well, brute force over all pairs (and triplets).
  sw_energy_direct  Stillinger-Weber E by a plain pair and triplet loop.
  sample_forces   the same for selected atoms, each computed on its own.
  hvp             analytic Hessian-vector product of the same energy.
  pair_counts, pair_list
                  the pair set every sum above runs over (atoms closer than
                  the cutoff under the minimum image), per atom in index order.
  cells           context manager: find the pair set through a cell grid
                  instead of testing every pair.  The pairs and their order
                  are the same, so every result is bit-identical (pinned by
                  tests); only large systems get faster.
  fire_minimize   FIRE 2.0 (Algorithm 2) with semi-implicit Euler and mixing
                  after the kick (Algorithm 4), Table 1 parameters, Sec. 3.4
                  stop tests; original FIRE (Algorithm 1) and the explicit
                  Euler / velocity Verlet integrators (Algorithms 3, 6) as options.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

STOP_NAMES = {1: "converged", 2: "max_steps", 3: "maxvdotf"}
ERRORS = {-1: "E_ARG", -2: "E_BOX", -3: "E_NONFINITE", -4: "E_OVERLAP"}
TRACE_COLS = ["i", "energy", "fmax", "f2norm", "P", "dt", "alpha", "branch", "n_pos"]


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle error {code} ({ERRORS.get(code, '?')})")
        self.code = code
        self.name = ERRORS.get(code, "?")


class _Box(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_double * 3), ("len", ctypes.c_double * 3), ("periodic", ctypes.c_int * 3)]


class _Pot(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int), ("convention", ctypes.c_int),
        ("eps", ctypes.c_double), ("sigma", ctypes.c_double), ("rc", ctypes.c_double),
        ("A", ctypes.c_double), ("p", ctypes.c_double), ("q", ctypes.c_double), ("xi", ctypes.c_double),
        ("r0", ctypes.c_double), ("r_in", ctypes.c_double), ("r_out", ctypes.c_double),
        ("k", ctypes.c_double * 3),
        ("sw_B", ctypes.c_double), ("sw_a", ctypes.c_double), ("sw_lambda", ctypes.c_double),
        ("sw_gamma", ctypes.c_double),
    ]


class _Fire(ctypes.Structure):
    _fields_ = [
        ("dt_start", ctypes.c_double), ("tmax", ctypes.c_double), ("tmin", ctypes.c_double),
        ("dtgrow", ctypes.c_double), ("dtshrink", ctypes.c_double), ("alpha0", ctypes.c_double),
        ("alphashrink", ctypes.c_double), ("f2a", ctypes.c_double),
        ("delaystep", ctypes.c_int), ("vdfmax", ctypes.c_int), ("halfstepback", ctypes.c_int),
        ("initialdelay", ctypes.c_int), ("integrator", ctypes.c_int), ("criterion", ctypes.c_int),
        ("variant", ctypes.c_int), ("pad", ctypes.c_int), ("dmax", ctypes.c_double),
    ]


class _Result(ctypes.Structure):
    _fields_ = [
        ("stop", ctypes.c_int), ("iterations", ctypes.c_long), ("force_evals", ctypes.c_long),
        ("energy", ctypes.c_double), ("fmax", ctypes.c_double), ("f2norm", ctypes.c_double),
        ("dt", ctypes.c_double), ("alpha", ctypes.c_double), ("n_pos", ctypes.c_long), ("n_neg", ctypes.c_long),
    ]


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (-O2, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-msse4.1", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        dp = P(ctypes.c_double)
        lib.oracle_energy_forces.argtypes = [ctypes.c_long, dp, P(_Box), P(_Pot), dp, dp, dp, dp]
        lib.oracle_sample_forces.argtypes = [ctypes.c_long, dp, P(_Box), P(_Pot), ctypes.c_long,
                                             P(ctypes.c_long), dp, dp]
        lib.oracle_hvp.argtypes = [ctypes.c_long, dp, dp, P(_Box), P(_Pot), dp]
        lib.oracle_fire_minimize.argtypes = [ctypes.c_long, dp, P(_Box), P(_Pot), P(_Fire), ctypes.c_double,
                                             ctypes.c_long, P(_Result), dp, dp]
        lib.oracle_fire_minimize_ex.argtypes = [ctypes.c_long, dp, P(_Box), P(_Pot), P(_Fire), ctypes.c_void_p, dp,
                                                ctypes.c_double, ctypes.c_long, P(_Result), dp, dp]
        lib.oracle_sw_energy_direct.argtypes = [ctypes.c_long, dp, P(_Box), P(_Pot), dp]
        lib.oracle_pair_counts.argtypes = [ctypes.c_long, dp, P(_Box), ctypes.c_double, P(ctypes.c_long),
                                           P(ctypes.c_long)]
        lib.oracle_pair_list.argtypes = [ctypes.c_long, dp, P(_Box), ctypes.c_double, ctypes.c_long,
                                         P(ctypes.c_long), P(ctypes.c_long), P(ctypes.c_long)]
        lib.oracle_set_cells.argtypes = [ctypes.c_int]
        lib.oracle_get_cells.restype = ctypes.c_int
        lib.oracle_threads.restype = ctypes.c_int
        lib.oracle_set_threads.argtypes = [ctypes.c_int]
        _lib = lib
    return _lib


def threads() -> int:
    return _load().oracle_threads()


def set_threads(n: int) -> None:
    _load().oracle_set_threads(int(n))


class cells:
    """Within the block, the oracle finds pairs through a cell grid (same
    pairs, same order, same bits as testing every pair)."""

    def __init__(self, on: bool = True):
        self.on = bool(on)

    def __enter__(self):
        lib = _load()
        self.prev = lib.oracle_get_cells()
        lib.oracle_set_cells(int(self.on))
        return self

    def __exit__(self, *exc):
        _load().oracle_set_cells(self.prev)
        return False


def _lptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_long))


def pair_counts(pos, box, rc):
    """Number of partners of each atom closer than rc (minimum image)."""
    lib = _load()
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    n = pos.shape[0]
    cnt = np.zeros(n, dtype=np.int64)
    tot = ctypes.c_long()
    b = _box(box)
    _check(lib.oracle_pair_counts(n, _ptr(pos), ctypes.byref(b), float(rc), _lptr(cnt), ctypes.byref(tot)))
    return cnt


def pair_list(pos, box, rc):
    """(start[n+1], idx): atom i's partners closer than rc are
    idx[start[i]:start[i+1]], in increasing order."""
    lib = _load()
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    n = pos.shape[0]
    start = np.zeros(n + 1, dtype=np.int64)
    tot = ctypes.c_long()
    b = _box(box)
    _check(lib.oracle_pair_list(n, _ptr(pos), ctypes.byref(b), float(rc), 0, _lptr(start), None, ctypes.byref(tot)))
    idx = np.zeros(max(tot.value, 1), dtype=np.int64)
    _check(lib.oracle_pair_list(n, _ptr(pos), ctypes.byref(b), float(rc), idx.shape[0], _lptr(start), _lptr(idx),
                                ctypes.byref(tot)))
    return start, idx[: tot.value]


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if a is not None else None


def _box(box) -> _Box:
    b = _Box()
    for d in range(3):
        b.lo[d] = float(box.lo[d])
        b.len[d] = float(box.length[d])
        b.periodic[d] = int(box.periodic[d])
    return b


def _pot(pot: dict) -> _Pot:
    p = _Pot()
    kind = pot["kind"]
    if kind == "lj":
        p.kind = 1
        p.eps, p.sigma, p.rc = pot["eps"], pot["sigma"], pot["rc"]
    elif kind == "gupta":
        p.kind = 2
        p.convention = {"rgl": 0, "half": 1}[pot.get("convention", "rgl")]
        for f in ("A", "p", "q", "xi", "r0", "r_in", "r_out"):
            setattr(p, f, float(pot[f]))
    elif kind == "harmonic":
        p.kind = 3
        for d in range(3):
            p.k[d] = float(pot["k"][d])
    elif kind == "sw":
        p.kind = 4
        for f in ("eps", "sigma", "A", "p", "q"):
            setattr(p, f, float(pot[f]))
        p.sw_B, p.sw_a, p.sw_lambda, p.sw_gamma = (float(pot[f]) for f in ("B", "a", "lambda", "gamma"))
    else:
        raise ValueError(kind)
    return p


def _fire(fp: dict) -> _Fire:
    f = _Fire()
    for k in ("dt_start", "tmax", "tmin", "dtgrow", "dtshrink", "alpha0", "alphashrink", "f2a"):
        setattr(f, k, float(fp[k]))
    for k in ("delaystep", "vdfmax", "halfstepback", "initialdelay"):
        setattr(f, k, int(fp[k]))
    f.integrator = {"eulerimplicit": 0, "eulerexplicit": 1, "verlet": 2}[fp.get("integrator", "eulerimplicit")]
    f.criterion = {"fmax": 0, "f2norm": 1}[fp.get("criterion", "fmax")]
    f.variant = {"fire2": 0, "fire1": 1}[fp.get("variant", "fire2")]
    f.dmax = float(fp.get("dmax", 0.0))
    return f


def _check(rc):
    if rc != 0:
        raise OracleError(rc)


def energy_forces(pos, box, pot, want_atom_energy=False, want_rho=False):
    """Returns (E, F[n,3]) (+ per-atom energy shares, + Gupta densities)."""
    lib = _load()
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    n = pos.shape[0]
    f = np.zeros((n, 3))
    e = ctypes.c_double()
    ea = np.zeros(n) if want_atom_energy else None
    rho = np.zeros(n) if want_rho else None
    b, p = _box(box), _pot(pot)
    _check(lib.oracle_energy_forces(n, _ptr(pos), ctypes.byref(b), ctypes.byref(p), ctypes.byref(e),
                                    _ptr(f), _ptr(ea), _ptr(rho)))
    out = [e.value, f]
    if want_atom_energy:
        out.append(ea)
    if want_rho:
        out.append(rho)
    return tuple(out)


def sample_forces(pos, box, pot, idx):
    """Forces (m,3) and per-atom energy shares (m) of atoms idx, one by one."""
    lib = _load()
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    m = idx.shape[0]
    f = np.zeros((m, 3))
    ea = np.zeros(m)
    b, p = _box(box), _pot(pot)
    _check(lib.oracle_sample_forces(pos.shape[0], _ptr(pos), ctypes.byref(b), ctypes.byref(p), m,
                                    idx.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), _ptr(f), _ptr(ea)))
    return f, ea


def sw_energy_direct(pos, box, pot):
    """Stillinger-Weber E by a plain loop over every pair and triplet (small n)."""
    lib = _load()
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    e = ctypes.c_double()
    b, p = _box(box), _pot(pot)
    _check(lib.oracle_sw_energy_direct(pos.shape[0], _ptr(pos), ctypes.byref(b), ctypes.byref(p), ctypes.byref(e)))
    return e.value


def hvp(pos, u, box, pot):
    """Analytic H u, (n,3)."""
    lib = _load()
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.zeros_like(pos)
    b, p = _box(box), _pot(pot)
    _check(lib.oracle_hvp(pos.shape[0], _ptr(pos), _ptr(u), ctypes.byref(b), ctypes.byref(p), _ptr(out)))
    return out


def fire_minimize(pos, box, pot, fire: dict, tol: float, max_steps: int, trace: bool = False,
                  want_velocity: bool = False, frozen=None, mass=None):
    """Run FIRE; returns dict(pos, stop, iterations, force_evals, energy, fmax,
    f2norm, dt, alpha, n_pos, n_neg[, trace][, velocity]).  frozen: optional
    uint8 per atom (bit d freezes component d); mass: optional per-atom mass
    relative to the mass f2a implies."""
    lib = _load()
    pos = np.array(pos, dtype=np.float64, copy=True, order="C")
    n = pos.shape[0]
    res = _Result()
    tr = np.zeros((max_steps + 1, len(TRACE_COLS))) if trace else None
    vel = np.zeros_like(pos) if want_velocity else None
    b, p, f = _box(box), _pot(pot), _fire(fire)
    fz = None if frozen is None else np.ascontiguousarray(frozen, dtype=np.uint8)
    ms = None if mass is None else np.ascontiguousarray(mass, dtype=np.float64)
    if fz is not None:
        assert fz.shape == (n,)
    if ms is not None:
        assert ms.shape == (n,)
    _check(lib.oracle_fire_minimize_ex(n, _ptr(pos), ctypes.byref(b), ctypes.byref(p), ctypes.byref(f),
                                       None if fz is None else fz.ctypes.data_as(ctypes.c_void_p), _ptr(ms),
                                       float(tol), int(max_steps), ctypes.byref(res), _ptr(tr), _ptr(vel)))
    out = {
        "pos": pos,
        "stop": STOP_NAMES.get(res.stop, str(res.stop)),
        "iterations": res.iterations,
        "force_evals": res.force_evals,
        "energy": res.energy,
        "fmax": res.fmax,
        "f2norm": res.f2norm,
        "dt": res.dt,
        "alpha": res.alpha,
        "n_pos": res.n_pos,
        "n_neg": res.n_neg,
    }
    if trace:
        out["trace"] = tr[: res.iterations + 1]
    if want_velocity:
        out["velocity"] = vel
    return out
