"""Measured parity of the GPU path against the oracle, gathered across the GPU tests into one record.

Each call names the workload configuration, the precision, what was compared, the measured relative L1
(mean absolute difference over mean absolute value) and relative Linf (maximum over maximum), and the
tolerances the calling test holds them to. At the end of the session the record is written as one JSON
object to the file $HGKS_PARITY_TABLE names (when set). Bookkeeping only: the tests' own checks decide
pass or fail."""
import json
import os

import numpy as np

TABLE = {}


def record(cfg, precision, what, l1, linf, tol_l1, tol_linf=None, **extra):
    row = {"what": what, "l1_rel": float(l1), "linf_rel": float(linf), "tol_l1_rel": tol_l1, "tol_linf_rel": tol_linf,
           "within": bool(float(l1) <= tol_l1 and (tol_linf is None or float(linf) <= tol_linf))}
    for k, v in extra.items():
        if isinstance(v, (bool, np.bool_)):
            v = bool(v)
        elif not isinstance(v, (str, int, type(None))):
            v = float(v)
        row[k] = v
    TABLE.setdefault(cfg, {}).setdefault(precision, []).append(row)


def prec_name(precision):
    return "fp64" if int(precision) == 0 else "fp32_bulk"


def dump():
    path = os.environ.get("HGKS_PARITY_TABLE")
    if path and TABLE:
        with open(path, "w") as fh:
            json.dump({"parity": TABLE}, fh, indent=1, sort_keys=True)
            fh.write("\n")
