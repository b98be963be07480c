"""Writes uniform_fallback.json: a stream position whose first uniform draw the rejection rule
refuses, found with the oracle's sampler alone, so that a test can drive the fallback stream of
the GPU sampler with the parameter rule's own primes (where a rejection has probability below
2^-29 per draw).

Search: N = 8192 with four primes, the last prime q_3 (the farthest from 2^50), stream tag 4
(the encryption's uniform part), op 0, objects 0, 1, 2, ...; the low 50 bits of every draw are
read through the oracle's uniform sampler with modulus 2^50 (which keeps every draw), and the
first draw at or above q_3 is recorded.  Run from the repository root:
    python tests/golden/make_uniform_fallback.py
"""
import ctypes
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as orc  # noqa: E402
from paper_2305_18396_amd import workloads  # noqa: E402

N, L, PRIME, TAG, OP, REQUEST = 8192, 4, 3, 4, 0, 91


def main():
    p = orc.Params(N, L, 41, 14)
    q = int(p.q[PRIME])
    key = np.frombuffer(workloads.seed("client", REQUEST), np.uint8).copy()
    cdt = p.cdt_arr
    raw = np.zeros(N, np.uint64)
    for obj in range(1 << 22):
        orc.lib().orc_sample_poly(0, key.ctypes.data_as(ctypes.c_void_p), TAG, PRIME, OP, obj, N,
                                  1 << 50, 41, cdt.ctypes.data_as(ctypes.c_void_p),
                                  raw.ctypes.data_as(ctypes.c_void_p))
        hits = np.nonzero(raw >= np.uint64(q))[0]
        if len(hits):
            j = int(hits[0])
            out = {"source": "search with the oracle's uniform sampler (this script)",
                   "N": N, "L": L, "prime": PRIME, "q": q, "request": REQUEST, "tag": TAG,
                   "op": OP, "obj": obj, "j": j, "first_draw_low50": int(raw[j])}
            path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "uniform_fallback.json")
            with open(path, "w") as fh:
                json.dump(out, fh, indent=1)
            print(out)
            return
    raise SystemExit("no rejected draw found")


if __name__ == "__main__":
    main()
