"""Thin Python binding of libfire2 (names follow include/fire2.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Host-array calls take numpy arrays; *_dev calls take torch device
tensors and enqueue on torch's current stream.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib as L
from ._lib import FireError


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def make_box(box) -> L.fire_box:
    """fire_box from an object with lo, length, periodic (or a fire_box)."""
    if isinstance(box, L.fire_box):
        return box
    b = L.fire_box()
    for d in range(3):
        b.lo[d] = float(box.lo[d])
        b.len[d] = float(box.length[d])
        b.periodic[d] = int(box.periodic[d])
    return b


def make_potential(pot) -> L.fire_potential:
    """fire_potential from a dict (kind lj / gupta / harmonic / sw)."""
    if isinstance(pot, L.fire_potential):
        return pot
    p = L.fire_potential()
    p.kind = L.POT[pot["kind"]]
    if pot["kind"] == "lj":
        p.eps, p.sigma, p.rc = float(pot["eps"]), float(pot["sigma"]), float(pot["rc"])
    elif pot["kind"] == "gupta":
        p.convention = L.CONVENTION[pot.get("convention", "rgl")]
        for f in ("A", "p", "q", "xi", "r0", "r_in", "r_out"):
            setattr(p, f, float(pot[f]))
    elif pot["kind"] == "sw":
        for f in ("eps", "sigma", "A", "p", "q"):
            setattr(p, f, float(pot[f]))
        p.sw_B, p.sw_a, p.sw_lambda, p.sw_gamma = (float(pot[f]) for f in ("B", "a", "lambda", "gamma"))
    else:
        for d in range(3):
            p.k[d] = float(pot["k"][d])
    return p


def fire_params_default() -> L.fire_params:
    p = L.fire_params()
    L.load().fire_params_default(ctypes.byref(p))
    return p


def make_params(fire: dict | None = None, **over) -> L.fire_params:
    """fire_params from Table-1 style keys (dict as built by inputs.fire_params)."""
    p = fire_params_default()
    d = dict(fire or {})
    d.update(over)
    for k in ("dt_start", "tmax", "tmin", "dtgrow", "dtshrink", "alpha0", "alphashrink", "f2a",
              "mixed_switch", "skin", "dmax"):
        if k in d:
            setattr(p, k, float(d[k]))
    for k in ("delaystep", "vdfmax", "halfstepback", "initialdelay"):
        if k in d:
            setattr(p, k, int(d[k]))
    if "integrator" in d:
        p.integrator = L.INTEGRATOR[d["integrator"]]
    if "criterion" in d:
        p.criterion = L.CRITERION[d["criterion"]]
    if "variant" in d:
        p.variant = L.VARIANT[d["variant"]]
    if "precision" in d:
        p.precision = L.PRECISION[d["precision"]]
    return p


def _result(r: L.fire_result) -> dict:
    return {
        "stop": L.STOP.get(r.stop_reason, str(r.stop_reason)),
        "precision_switched": bool(r.precision_switched),
        "iterations": r.iterations,
        "force_evals": r.force_evals,
        "iterations_low": r.iterations_low,
        "rebuilds": r.rebuilds,
        "energy": r.energy,
        "energy_per_atom": r.energy_per_atom,
        "fmax": r.fmax,
        "f2norm": r.f2norm,
        "dt": r.dt,
        "alpha": r.alpha,
    }


class Context:
    """Owns one fire_ctx (fire_init / fire_finalize)."""

    def __init__(self, device: int = 0, fire: dict | None = None, **over):
        self.lib = L.load()
        self.handle = ctypes.c_void_p()
        p = make_params(fire, **over)
        rc = self.lib.fire_init(ctypes.byref(self.handle), int(device), ctypes.byref(p))
        if rc != 0:
            raise FireError(rc, "fire_init failed (is a gfx950 device visible?)")

    # ---------------------------------------------------------------- misc
    def close(self):
        if self.handle:
            self.lib.fire_finalize(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, rc):
        if rc != 0:
            msg = self.lib.fire_last_error(self.handle)
            raise FireError(rc, msg.decode() if msg else "")

    def fire_set_params(self, fire: dict | None = None, **over):
        p = make_params(fire, **over)
        self._check(self.lib.fire_set_params(self.handle, ctypes.byref(p)))

    def fire_tuning_info(self) -> str:
        """The speed-only choices of the last minimisation (list order)."""
        return self.lib.fire_tuning_info(self.handle).decode()

    def fire_get_params(self) -> L.fire_params:
        p = L.fire_params()
        self._check(self.lib.fire_get_params(self.handle, ctypes.byref(p)))
        return p

    # --------------------------------------------------------- host arrays
    def fire_energy_forces(self, pos, box, pot, want_forces: bool = True):
        pos = np.ascontiguousarray(pos, dtype=np.float64)
        n = pos.shape[0]
        e = ctypes.c_double()
        f = np.zeros((n, 3)) if want_forces else None
        b, p = make_box(box), make_potential(pot)
        self._check(self.lib.fire_energy_forces(self.handle, n, _dp(pos), ctypes.byref(b), ctypes.byref(p),
                                                ctypes.byref(e), _dp(f) if f is not None else None))
        return (e.value, f) if want_forces else e.value

    def fire_minimize(self, pos, box, pot, tol: float, max_steps: int, trace: bool = False,
                      frozen=None, mass=None):
        """frozen: optional uint8 per atom (bit d holds component d fixed);
        mass: optional per-atom mass relative to the one f2a implies."""
        x = np.array(pos, dtype=np.float64, copy=True, order="C")
        n = x.shape[0]
        r = L.fire_result()
        b, p = make_box(box), make_potential(pot)
        if frozen is not None or mass is not None:
            fz = None if frozen is None else np.ascontiguousarray(frozen, dtype=np.uint8)
            ms = None if mass is None else np.ascontiguousarray(mass, dtype=np.float64)
            for a in (fz, ms):
                if a is not None and a.shape != (n,):
                    raise ValueError("frozen and mass need one entry per atom")
            at = L.fire_atoms(None if fz is None else fz.ctypes.data, None if ms is None else ms.ctypes.data)
            tr = np.zeros((max_steps + 1, L.TRACE_COLS)) if trace else None
            self._check(self.lib.fire_minimize_ex(self.handle, n, _dp(x), ctypes.byref(b), ctypes.byref(p),
                                                  ctypes.byref(at), float(tol), int(max_steps), ctypes.byref(r),
                                                  _dp(tr) if trace else None))
        elif trace:
            tr = np.zeros((max_steps + 1, L.TRACE_COLS))
            self._check(self.lib.fire_minimize_traced(self.handle, n, _dp(x), ctypes.byref(b), ctypes.byref(p),
                                                      float(tol), int(max_steps), ctypes.byref(r), _dp(tr)))
        else:
            self._check(self.lib.fire_minimize(self.handle, n, _dp(x), ctypes.byref(b), ctypes.byref(p),
                                               float(tol), int(max_steps), ctypes.byref(r)))
        out = _result(r)
        out["pos"] = x
        if trace:
            out["trace"] = tr[: r.iterations + 1]
        return out

    def fire_hvp(self, pos, u, box, pot):
        pos = np.ascontiguousarray(pos, dtype=np.float64)
        u = np.ascontiguousarray(u, dtype=np.float64)
        hu = np.zeros_like(pos)
        b, p = make_box(box), make_potential(pot)
        self._check(self.lib.fire_hvp(self.handle, pos.shape[0], _dp(pos), _dp(u), ctypes.byref(b),
                                      ctypes.byref(p), _dp(hu)))
        return hu

    def fire_lowest_curvature(self, pos, box, pot, k: int = 40, u0=None, want_residual: bool = False):
        """Smallest Ritz value of k Lanczos steps (and its residual |Hz - theta z|)."""
        pos = np.ascontiguousarray(pos, dtype=np.float64)
        lam = ctypes.c_double()
        res = ctypes.c_double()
        b, p = make_box(box), make_potential(pot)
        u0p = None
        if u0 is not None:
            u0 = np.ascontiguousarray(u0, dtype=np.float64)
            u0p = _dp(u0)
        self._check(self.lib.fire_lowest_curvature(self.handle, pos.shape[0], _dp(pos), ctypes.byref(b),
                                                   ctypes.byref(p), u0p, int(k), ctypes.byref(lam),
                                                   ctypes.byref(res)))
        return (lam.value, res.value) if want_residual else lam.value

    def fire_minimize_batched(self, systems, pot, tol: float, max_steps: int, per_sys: list | None = None):
        """systems: list of (pos (n,3), box).  Returns (list of positions, list of result dicts)."""
        offs = np.zeros(len(systems) + 1, dtype=np.int64)
        for s, (x, _) in enumerate(systems):
            offs[s + 1] = offs[s] + len(x)
        allpos = np.ascontiguousarray(np.concatenate([np.asarray(x, np.float64) for x, _ in systems]))
        boxes = (L.fire_box * len(systems))(*[make_box(b) for _, b in systems])
        prm = None
        if per_sys is not None:
            prm = (L.fire_params * len(systems))(*[make_params(f) for f in per_sys])
        res = (L.fire_result * len(systems))()
        p = make_potential(pot)
        self._check(self.lib.fire_minimize_batched(
            self.handle, len(systems), offs.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong)), _dp(allpos),
            boxes, ctypes.byref(p), prm, float(tol), int(max_steps), res))
        out_pos = [allpos[offs[s]:offs[s + 1]].copy() for s in range(len(systems))]
        return out_pos, [_result(r) for r in res]

    def fire_minimize_batched_dev(self, pos, offsets, boxes, pot, tol: float, max_steps: int,
                                  per_sys: list | None = None, noalloc: bool = False):
        """pos: (ntot,3) float64 cuda tensor, relaxed in place; offsets: nsys+1
        atom offsets; boxes: nsys boxes.  Returns the list of result dicts.
        noalloc: call fire_minimize_batched_noalloc (no device allocation;
        work buffers in the library's per-device scratch array)."""
        import torch
        assert pos.is_cuda and pos.dtype == torch.float64 and pos.is_contiguous()
        nsys = len(boxes)
        offs = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
        assert offs.shape == (nsys + 1,) and offs[-1] == pos.shape[0]
        bx = (L.fire_box * nsys)(*[make_box(b) for b in boxes])
        prm = None
        if per_sys is not None:
            prm = (L.fire_params * nsys)(*[make_params(f) for f in per_sys])
        res = (L.fire_result * nsys)()
        p = make_potential(pot)
        fn = self.lib.fire_minimize_batched_noalloc if noalloc else self.lib.fire_minimize_batched_dev
        self._check(fn(
            self.handle, nsys, offs.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong)),
            ctypes.c_void_p(pos.data_ptr()), bx, ctypes.byref(p), prm, float(tol), int(max_steps), res,
            self._stream()))
        return [_result(r) for r in res]

    # -------------------------------------------------------- device tensors
    @staticmethod
    def _stream():
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

    def fire_energy_forces_dev(self, pos, box, pot, energy=None, forces=None):
        """pos: (n,3) float64 cuda tensor.  Writes into (or allocates) a 1-element
        energy tensor and an (n,3) force tensor; returns (energy, forces)."""
        import torch
        assert pos.is_cuda and pos.dtype == torch.float64 and pos.is_contiguous()
        n = pos.shape[0]
        if energy is None:
            energy = torch.empty(1, dtype=torch.float64, device=pos.device)
        if forces is None:
            forces = torch.empty_like(pos)
        b, p = make_box(box), make_potential(pot)
        self._check(self.lib.fire_energy_forces_dev(self.handle, n, ctypes.c_void_p(pos.data_ptr()),
                                                    ctypes.byref(b), ctypes.byref(p),
                                                    ctypes.c_void_p(energy.data_ptr()),
                                                    ctypes.c_void_p(forces.data_ptr()), self._stream()))
        return energy, forces

    def fire_hvp_dev(self, pos, u, box, pot, hu=None):
        import torch
        assert pos.is_cuda and u.is_cuda and pos.dtype == torch.float64 and u.dtype == torch.float64
        pos = pos.contiguous()
        u = u.contiguous()
        if hu is None:
            hu = torch.empty_like(pos)
        b, p = make_box(box), make_potential(pot)
        self._check(self.lib.fire_hvp_dev(self.handle, pos.shape[0], ctypes.c_void_p(pos.data_ptr()),
                                          ctypes.c_void_p(u.data_ptr()), ctypes.byref(b), ctypes.byref(p),
                                          ctypes.c_void_p(hu.data_ptr()), self._stream()))
        return hu

    def fire_minimize_dev(self, pos, box, pot, tol: float, max_steps: int, frozen=None, mass=None):
        """Minimise in place on the device tensor pos (n,3) float64; frozen
        (uint8) and mass (float64), if given, are device tensors of n entries."""
        import torch
        assert pos.is_cuda and pos.dtype == torch.float64 and pos.is_contiguous()
        r = L.fire_result()
        b, p = make_box(box), make_potential(pot)
        if frozen is not None or mass is not None:
            n = pos.shape[0]
            for a, dt in ((frozen, torch.uint8), (mass, torch.float64)):
                if a is not None:
                    assert a.is_cuda and a.dtype == dt and a.is_contiguous() and a.shape == (n,)
            at = L.fire_atoms(None if frozen is None else frozen.data_ptr(),
                              None if mass is None else mass.data_ptr())
            self._check(self.lib.fire_minimize_ex_dev(self.handle, n, ctypes.c_void_p(pos.data_ptr()),
                                                      ctypes.byref(b), ctypes.byref(p), ctypes.byref(at),
                                                      float(tol), int(max_steps), ctypes.byref(r), self._stream()))
            return _result(r)
        self._check(self.lib.fire_minimize_dev(self.handle, pos.shape[0], ctypes.c_void_p(pos.data_ptr()),
                                               ctypes.byref(b), ctypes.byref(p), float(tol), int(max_steps),
                                               ctypes.byref(r), self._stream()))
        return _result(r)


    def fire_repeat_forces_dev(self, reps: int, stream=None):
        """Re-run the force pass of the last system reps times on torch's
        current stream (measurement hook)."""
        st = self._stream() if stream is None else stream
        self._check(self.lib.fire_repeat_forces_dev(self.handle, int(reps), st))


def fire_init(device: int = 0, fire: dict | None = None, **over) -> Context:
    return Context(device, fire, **over)


def fire_finalize(ctx: Context) -> None:
    ctx.close()
