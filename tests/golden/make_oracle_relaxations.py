"""Write oracle_relaxations.json: FP64 oracle results of the full-size
workloads, for the GPU parity tests that cannot afford to run the oracle
themselves (minutes of CPU per relaxation).

Every value comes from the CPU oracle (oracle/, Algorithm 2 with the
semi-implicit Euler integrator of Algorithm 4, the Table 1 semantics and the
stop test of Sec. 3.4; pairs found through the cell grid, which is pinned to
give the same bits as testing every pair) on the seeded inputs of
paper_1908_02038_amd.inputs.  Nothing here runs or reads the HIP library.
Each record keeps a SHA-256 of its input arrays so that a test fails loudly
if the generator ever produced other atoms.

    python tests/golden/make_oracle_relaxations.py [case ...]

Cases:
  lj_bulk, gupta_bulk           relaxations to fmax < 1e-6 (130,417 and
                                253,440 atoms)
  lj_bulk_first20, gupta_slab_first20
                                the first 20 iterations (130,417 and
                                2,037,760 atoms): the trace and the positions
                                of a sample of atoms
  batched_sample                16 of the 512 systems of the batched workload,
                                each relaxed on its own
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1908_02038_amd import inputs  # noqa: E402

OUT = os.path.join(HERE, "oracle_relaxations.json")
SAMPLE = 96             # atoms whose final coordinates are stored (24 per batched system)
BATCH_PICK = [33 * k for k in range(16)]  # systems 0, 33, ..., 495: both kinds, the whole size range


def input_hash(s) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(s.pos, dtype=np.float64).tobytes())
    h.update(np.asarray(s.box.lo, np.float64).tobytes())
    h.update(np.asarray(s.box.length, np.float64).tobytes())
    h.update(np.asarray(s.box.periodic, np.int64).tobytes())
    return h.hexdigest()


def sample_idx(n: int, seed: int, m: int = SAMPLE) -> np.ndarray:
    return np.sort(np.random.default_rng(seed).choice(n, size=min(m, n), replace=False))


def relax(s, max_steps: int, tol: float, trace: bool = False):
    t0 = time.time()
    with oracle.cells():
        r = oracle.fire_minimize(s.pos, s.box, s.potential, s.fire, tol, max_steps, trace=trace)
    r["seconds"] = time.time() - t0
    return r


def record(s, r, with_trace: bool, seed: int, m: int = SAMPLE):
    n = len(s.pos)
    idx = sample_idx(n, seed, m)
    out = {
        "workload": s.name,
        "n": n,
        "input_sha256": input_hash(s),
        "tol": s.tol,
        "stop": r["stop"],
        "iterations": int(r["iterations"]),
        "energy": r["energy"],
        "energy_per_atom": r["energy"] / n,
        "fmax": r["fmax"],
        "f2norm": r["f2norm"],
        "dt": r["dt"],
        "alpha": r["alpha"],
        "sample_idx": idx.tolist(),
        "sample_pos": r["pos"][idx].tolist(),
        "oracle_seconds": round(r["seconds"], 1),
        "oracle_threads": oracle.threads(),
    }
    if with_trace:
        out["trace_cols"] = oracle.TRACE_COLS
        out["trace"] = r["trace"].tolist()
    return out


def case_relax(make):
    s = make()
    r = relax(s, 20000, s.tol)
    return record(s, r, False, 11)


def case_first20(make):
    s = make()
    r = relax(s, 20, 0.0, trace=True)
    return record(s, r, True, 12)


def case_batched():
    systems = inputs.batched()
    recs = []
    for q in BATCH_PICK:
        s = systems[q]
        r = relax(s, 20000, s.tol)
        rec = record(s, r, False, 13, SAMPLE // 4)
        rec["system"] = q
        recs.append(rec)
        print(f"  system {q}: n {rec['n']} {rec['stop']} {rec['iterations']} it, {r['seconds']:.1f} s", flush=True)
    return {"systems": recs, "n_systems_in_batch": len(systems)}


CASES = {
    "lj_bulk": lambda: case_relax(inputs.lj_bulk),
    "gupta_bulk": lambda: case_relax(inputs.gupta_bulk),
    "lj_bulk_first20": lambda: case_first20(inputs.lj_bulk),
    "gupta_slab_first20": lambda: case_first20(inputs.gupta_slab),
    "batched_sample": case_batched,
}


def main(names):
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    data["_about"] = ("FP64 CPU oracle results (oracle/, Algorithm 2 + Algorithm 4, Table 1, Sec. 3.4 stop test) "
                      "of the seeded workloads; written by tests/golden/make_oracle_relaxations.py")
    for name in names or list(CASES):
        t0 = time.time()
        print(f"{name} ...", flush=True)
        data[name] = CASES[name]()
        print(f"{name}: done in {time.time() - t0:.0f} s", flush=True)
        with open(OUT + ".tmp", "w") as f:
            json.dump(data, f, separators=(",", ":"))
            f.write("\n")
        os.replace(OUT + ".tmp", OUT)


if __name__ == "__main__":
    main(sys.argv[1:])
