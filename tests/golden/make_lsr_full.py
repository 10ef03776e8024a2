"""Writes lsr_1048576x256_s4096.json: the oracle's sketch-and-solve solution
x~ (eq. 4.2, Sec. 4.2) of the full-size least-squares workload for each
sketch family, for the GPU test that compares the library's x~ with it.

Workload: synth.lsr_fp32 with its default data seed (2^20 x 256 FP32 rows
g_i |t_i|, t_i Student-t with 2 degrees of freedom, b = A x* + noise of
variance 1e-3), sketch seed synth.sketch_seed(2), s = 4096.  The oracle's
sketch S^T [A | b] is accumulated over blocks of 8192 rows, each block of S
built explicitly from its definition (oracle.sketch.sketch_matrix with
global row indices), the block products summed in block order; then x~ by
Householder QR of the sketched system (oracle.lsr).  The FP32 data is
promoted exactly to FP64; the Gaussian entries are drawn in the FP32 mode
(24-bit uniforms), as the library's FP32 path draws them.

Only oracle/ and the input generators are used.  Run from the repository
root: python tests/golden/make_lsr_full.py  (about 10-20 minutes on 8 cores).
"""

import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import lsr as olsr, sketch as osk  # noqa: E402

M, D, S = 1 << 20, 256, 4096
BLOCK = 8192
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "lsr_1048576x256_s4096.json")
FAMILIES = [("countsketch", osk.COUNTSKETCH), ("srht", osk.SRHT), ("gaussian", osk.GAUSSIAN)]

_A = None
_b = None


def _block(args):
    kind, r0 = args
    rows = np.arange(r0, min(r0 + BLOCK, M))
    Sb = osk.sketch_matrix(kind, M, S, synth.sketch_seed(2), fp64=False, rows=rows)
    Db = np.concatenate([_A[rows].astype(np.float64), _b[rows, None].astype(np.float64)], axis=1)
    return Sb.T @ Db


def main():
    global _A, _b
    t0 = time.time()
    _A, _b, _ = synth.lsr_fp32()
    assert _A.shape == (M, D) and _A.dtype == np.float32
    out = {"m": M, "d": D, "s": S, "data_seed": synth.data_seed(2),
           "sketch_seed": synth.sketch_seed(2),
           "source": "oracle sketch-and-solve (eq. 4.2) on synth.lsr_fp32(); "
                     "written by tests/golden/make_lsr_full.py",
           "x": {}, "kappa": {}, "resid": {}}
    procs = int(os.environ.get("GOLDEN_PROCS", "6"))
    with mp.get_context("fork").Pool(procs) as pool:
        for name, kind in FAMILIES:
            Cs = np.zeros((S, D + 1))
            for part in pool.imap(_block, [(kind, r0) for r0 in range(0, M, BLOCK)]):
                Cs += part
            x, R = olsr._qr_solve(Cs[:, :D], Cs[:, D])
            sv = np.linalg.svd(Cs[:, :D], compute_uv=False)
            out["x"][name] = [float(v) for v in x]
            out["kappa"][name] = float(sv[0] / sv[-1])
            out["resid"][name] = float(np.linalg.norm(_A.astype(np.float64) @ x - _b))
            print(name, "done", round(time.time() - t0, 1), "s", flush=True)
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
