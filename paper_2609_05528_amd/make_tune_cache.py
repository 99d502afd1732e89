"""Write the autotuner cache that bench.py replays: the kernel variants and launch modes of the
benchmark's workloads, timed with many repetitions on this GPU, under a header line naming the
digest of the operator source they were timed with (bench.py ignores a cache whose digest does not
match the source it runs, and then tunes afresh).

Usage: python -m paper_2609_05528_amd.make_tune_cache [output path] [repetitions]
"""
from __future__ import annotations

import hashlib
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
DEFAULT = os.path.join(HERE, "tune_cache.txt")


def operator_digest() -> str:
    with open(os.path.join(HERE, "csrc", "operator.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def main():
    out = sys.argv[1] if len(sys.argv) > 1 else DEFAULT
    reps = int(sys.argv[2]) if len(sys.argv) > 2 else 9
    sys.path.insert(0, ROOT)
    import paper_2609_05528_amd as rtt
    import synth
    body = out + ".body"
    if os.path.exists(body):
        os.remove(body)
    jobs = [(synth.batch_geometries(), synth.BATCH_HISTORIES), ([synth.geometry_for("cfg2")], 264),
            ([synth.geometry_for("cfg5")], 1), ([synth.geometry_for("cfg5")], 32)]
    jobs += [([geo], 1) for geo in synth.batch_geometries()]       # the plain per-instance loop
    for geos, nvec in jobs:
        G = rtt.Geometry(geos if len(geos) > 1 else geos[0])
        choice = G.tune(nvec=nvec, reps=reps, cache_path=body)
        print("tuned %d geometries, %d vectors: %s, modes %s" % (len(geos), nvec, [
            (rtt.variant_names(False)[a], rtt.variant_names(True)[b]) for a, b in choice], G.batch_mode), flush=True)
        del G
    with open(body) as f:
        lines = f.read()
    with open(out, "w") as f:
        f.write("# operator %s\n" % operator_digest())
        f.write(lines)
    os.remove(body)
    print("wrote", out)


if __name__ == "__main__":
    main()
