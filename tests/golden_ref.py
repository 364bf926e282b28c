"""Stored oracle solutions (tests/golden/*.npz, written by tests/golden/make_references.py
from oracle/ and synth/ only) and the comparison of a result with them.

A result A of the GPU path is compared with the reference A* by
  * the relative objective error |F - F*| / max(1, |F*|);
  * the support of the lower triangle: entries whose zero/nonzero status differs,
    except the stored exemptions (entries within 1e-8 of the threshold: a nonzero
    with |A*_ij| <= 1e-8, or a zero with ||g*_ij| - lambda| <= 1e-8);
  * where the values are stored, max |A_ij - A*_ij| over the lower triangle.
No solver arithmetic here."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name):
    """List of per-problem dicts of the file golden/<name>.npz."""
    z = np.load(os.path.join(GOLDEN, name + ".npz"), allow_pickle=False)
    out = []
    for k in range(int(z["count"])):
        d = {key[len(f"{k}_"):]: z[key] for key in z.files if key.startswith(f"{k}_")}
        out.append(d)
    return out


def lower_support(ref, n):
    """Boolean n x n lower-triangle support of the reference."""
    m = np.zeros((n, n), dtype=bool)
    if "bits" in ref:
        r, c = np.tril_indices(n)
        m[r, c] = np.unpackbits(ref["bits"], count=r.size).astype(bool)
    else:
        m[ref["rows"], ref["cols"]] = True
    return m


def compare(A, F, ref):
    """(relative F error, support mismatches outside the exemptions, max abs
    difference of A on the lower triangle or None when values are not stored)."""
    n = A.shape[0]
    relF = abs(F - float(ref["F"])) / max(1.0, abs(float(ref["F"])))
    sup_ref = lower_support(ref, n)
    sup = np.tril(A != 0)
    diff = sup != sup_ref
    diff[ref["ex_rows"], ref["ex_cols"]] = False
    dA = None
    if "vals" in ref:
        Aref = np.zeros((n, n))
        Aref[ref["rows"], ref["cols"]] = ref["vals"]
        dA = float(np.max(np.abs(np.tril(A) - Aref)))
    return relF, int(diff.sum()), dA
