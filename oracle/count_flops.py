"""Algorithmic floating-point operations per cell update of the MHM step,
derived from the oracle alone; writes ``flops_per_cell.json`` beside this file.

TEST / MEASUREMENT INFRASTRUCTURE: run by hand (``python oracle/count_flops.py``)
and checked by ``tests/test_oracle_opcount.py``; the benchmark reads the JSON
it writes, as the denominator of its flop roofline.

Per 16^3 group the step evaluates (Sec. 2.2 MHM with PLM and HLLC):
  * the primitive variables of every cell the stencil reaches,
  * the Hancock face states of every "state cell" (interior plus the first
    ghost layer across each face, no edges or corners),
  * one HLLC flux per interior-adjacent face,
  * the update (with its unphysical check) of every interior cell.
The multiplicities are enumerated here from those definitions, and each
stage's add / mul / div / sqrt count (each counted once) comes from the
oracle's operation-counting scalar on inputs that force the path counted:
every limiter active (both one-sided differences of one sign: the most work
a slope can take, and what a branch-free kernel executes anyway) and the HLLC
star branch (the branch of every subsonic face, the costliest of the four).
"""

import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

import oracle  # noqa: E402

N = 16


def state_cells():
    """Cells of [-1, 16]^3 with at most one coordinate outside [0, 15]."""
    r = range(-1, N + 1)
    return [(x, y, z) for z in r for y in r for x in r
            if sum(c < 0 or c >= N for c in (x, y, z)) <= 1]


def reachable_cells():
    """The state cells and their six axis neighbours (their limiter stencil)."""
    out = set()
    for (x, y, z) in state_cells():
        out.add((x, y, z))
        for d in range(3):
            for s in (-1, 1):
                c = [x, y, z]
                c[d] += s
                out.add(tuple(c))
    return out


def faces():
    """Faces between two cells of which at least one is interior, normal to x, y or z."""
    return 3 * (N + 1) * N * N


def stage_inputs(gamma=5.0 / 3.0):
    """Sample inputs that force every limiter active and the HLLC star branch."""
    U = np.array([1.2, 0.3, -0.2, 0.1, 2.5])
    Wc = oracle.cons_to_prim(U, gamma)
    Wm = np.tile(Wc * 0.95, 3)          # strictly monotone through the cell on every axis
    Wp = np.tile(Wc * 1.07, 3)
    UL = oracle.prim_to_cons(np.array([1.0, 0.2, 0.1, 0.0, 1.0]), gamma)   # subsonic, S* > 0
    UR = oracle.prim_to_cons(np.array([0.8, 0.1, 0.0, 0.1, 0.9]), gamma)
    return U, Wc, Wm, Wp, UL, UR, gamma


def count():
    U, Wc, Wm, Wp, UL, UR, gamma = stage_inputs()
    ops = oracle.count_ops(U, Wc, Wm, Wp, UL, UR, gamma, 1.5, 0.01)
    mult = {"cons_to_prim": len(reachable_cells()), "hancock_cell": len(state_cells()), "hllc_flux": faces(),
            "update": N ** 3}
    per_stage = {k: sum(v.values()) for k, v in ops.items()}
    total = sum(per_stage[k] * mult[k] for k in mult)
    return {"flops_per_cell_update": total / N ** 3, "per_group": total, "multiplicity": mult,
            "ops_per_item": ops, "path": "every limiter active, HLLC star branch (Einfeldt/Roe speeds)",
            "written_by": "oracle/count_flops.py"}


if __name__ == "__main__":
    rec = count()
    with open(os.path.join(HERE, "flops_per_cell.json"), "w") as fh:
        json.dump(rec, fh, indent=1, sort_keys=True)
        fh.write("\n")
    print(json.dumps(rec, sort_keys=True))
