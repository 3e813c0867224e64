"""Write tests/golden/structure.json from the oracle alone.

The paper prints no matrix elements, amplitudes or counts for any worked
example (its figures carry no data and its only table holds run times), so
no stored value here is the paper's.  This file records the oracle's own
pre-selected structure (nonzero cell-pair counts and a SHA-256 of the CSR
arrays) for the 40 x 40, 150 x 150 and 300 x 300 grids, as a regression fixture.  It is
produced by this script, which calls only oracle/.
"""
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle.wpcd as W  # noqa: E402


def digest(ptr, col):
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(ptr, dtype="<i8").tobytes())
    h.update(np.ascontiguousarray(col, dtype="<i4").tobytes())
    return h.hexdigest()


def main():
    out = {}
    for n in (40, 150, 300):
        p = W.cheb_edges(n, 10.0)
        ptr, col = W.preselect(p, p.copy())
        out[f"{n}x{n}"] = {"n_p": n, "n_q": n, "p_max": 10.0, "q_max": 10.0,
                           "nnz_cells": int(ptr[-1]), "max_row": int(np.diff(ptr).max()),
                           "sha256_rowptr_i64_col_i32": digest(ptr, col)}
    with open(os.path.join(HERE, "structure.json"), "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
        f.write("\n")
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
