"""Write the bulk-solvent quantities of Eq 19-21 that the library takes as
inputs (test infrastructure; calls only the oracle):

    python -m oracle.make_bulk           # writes tests/golden/solvent/*_bulk.json

For each stored solvent the 1D DRISM/KH solve of ``make_chi`` is repeated with
the same settings; its susceptibility must equal the stored table, and the
isothermal compressibility chi_T (A^3 mol/kcal) and the pressure of Eq 20
(kcal/(mol A^3)) are written beside the table.
"""
from __future__ import annotations

import json
import os
import sys

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(_HERE))

from oracle import rism1d  # noqa: E402
from oracle.make_chi import OUT_DIR, SOLVENTS  # noqa: E402


def make(name: str, out_dir: str = OUT_DIR) -> str:
    solvent = SOLVENTS[name]()
    res = rism1d.solve_solvent(solvent, drism=True, closure_kind="kh")
    with np.load(os.path.join(out_dir, f"{name}.npz"), allow_pickle=False) as z:
        diff = float(np.abs(res.chi_table() - z["chi"]).max())
    if diff > 1e-10:
        raise RuntimeError(f"{name}: the 1D solve no longer reproduces the stored table ({diff})")
    out = dict(solvent=name, compressibility=rism1d.compressibility(solvent, res),
               pressure=rism1d.bulk_pressure(solvent, res),
               units=dict(compressibility="A^3 mol/kcal", pressure="kcal/(mol A^3)"),
               closure="kh", drism=True, table_max_diff=diff)
    path = os.path.join(out_dir, f"{name}_bulk.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    return path


if __name__ == "__main__":
    for nm in (sys.argv[1:] or list(SOLVENTS)):
        print(make(nm), flush=True)
