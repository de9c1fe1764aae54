"""Write channel_isovalues.json: Q isovalues of the turbulent-channel workload.

The workload (65,536 order-7 elements, 33,554,432 GLL points, tanh-stretched
channel, random-mode k^-5/3 velocity, seed 2312) extracts isosurfaces of Q
at its 90th, 95th and 99th percentiles.  They are computed here once from
the CPU FP64 oracle's Q over all stored node values (duplicated face nodes
included), with numpy's linear-interpolation percentile, and stored so that
the benchmark and the tests pass explicit isovalues to the library.

Calls only the oracle and the input generator.  Run from the repository
root:  python tests/golden/make_channel_isovalues.py   (a few minutes).
"""

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle import gll, sem  # noqa: E402

PCTS = (90.0, 95.0, 99.0)


def main():
    n = 7
    shape = W.CHANNEL_SHAPE
    e_tot = shape[0] * shape[1] * shape[2]
    d = gll.diff_matrix(n)
    q_all = np.empty((e_tot, n + 1, n + 1, n + 1))
    chunk = 2048
    t0 = time.time()
    for s in range(0, e_tot, chunk):
        els = np.arange(s, min(s + chunk, e_tot))
        x, y, z, u, v, w = W.channel_config(n, elements=els)
        q, _, bad = sem.qcrit(x, y, z, u, v, w, d)
        assert not bad.any()
        q_all[els] = q
        print(f"{s + len(els)}/{e_tot} elements, {time.time() - t0:.0f} s", flush=True)
    iso = [float(np.percentile(q_all, p, method="linear")) for p in PCTS]
    out = {
        "workload": "channel 64x32x32 elements, N=7, beta=2, seed 2312",
        "source": "oracle FP64 Q over all stored node values; numpy percentile (linear)",
        "percentiles": list(PCTS),
        "isovalues": iso,
        "q_min": float(q_all.min()),
        "q_max": float(q_all.max()),
    }
    with open(os.path.join(HERE, "channel_isovalues.json"), "w") as fh:
        json.dump(out, fh, indent=2)
        fh.write("\n")
    print(out)


if __name__ == "__main__":
    main()
