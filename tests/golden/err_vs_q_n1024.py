"""Error of the butterfly against the direct sum as q grows, at the
benchmark's size: N = 1024, eq:ex1 (Sec. 5), s = 3, lm = 5, in the shape of
Table 1 (eq:err on 256 points).

Computed with the FP64 step model of ``oracle/butterfly.py`` restricted to
the ancestors of four target boxes at level L - s of T_X (8 x 8 points each,
256 points) and the C direct sum of ``oracle/direct.py`` on those points;
the sources are the first right-hand side of the benchmark's batch (complex
white noise, seed 3).  Writes ``err_vs_q_n1024.json`` beside this file.

Usage: python tests/golden/err_vs_q_n1024.py [q ...]   (default 5 7 ... 21)
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import direct as D  # noqa: E402
from oracle.butterfly import ButterflyModel  # noqa: E402
from workloads import white_noise  # noqa: E402

N = 1024
TARGETS = [(3, 17), (40, 101), (77, 5), (126, 64)]
SIDE = 8


def main(qs):
    f = white_noise(N, 3, nrhs=2)[0]
    rows = np.array([(a1 * SIDE + i) * N + a2 * SIDE + j for a1, a2 in TARGETS
                     for i in range(SIDE) for j in range(SIDE)], dtype=np.int64)
    out = {"N": N, "phase": "eq:ex1", "s": 3, "lm": 5, "targets_level": 7, "targets": TARGETS,
           "points": int(rows.size), "f": "white_noise(1024, seed 3), first right-hand side", "rows": {}}
    path = os.path.join(HERE, "err_vs_q_n1024.json")
    if os.path.exists(path):
        with open(path) as fh:
            out["rows"] = json.load(fh).get("rows", {})
    ref = {}
    for ph_name, ph in (("eq:ex1", D.Phase()), ("fourier", D.Phase(kind=D.FOURIER))):
        ref[ph_name] = D.forward(N, ph, f, rows)
    for q in qs:
        for ph_name, ph in (("eq:ex1", D.Phase()), ("fourier", D.Phase(kind=D.FOURIER))):
            t0 = time.time()
            m = ButterflyModel(N, q, ph)
            u = m.apply(f, targets=TARGETS).reshape(-1)[rows]
            e = D.rel_err(ref[ph_name], u)
            out["rows"][f"{ph_name} q={q}"] = e
            print(f"{ph_name} N={N} q={q}: eq:err {e:.3e} ({time.time() - t0:.0f} s)", flush=True)
            with open(path, "w") as fh:
                json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main([int(a) for a in sys.argv[1:]] or list(range(5, 22, 2)))
