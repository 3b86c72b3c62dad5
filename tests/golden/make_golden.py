"""Write the oracle's results for the full-size workloads to tests/golden/*.json.

Expected values only ever come from here: this script calls the CPU oracle (oracle/) on the seeded
generators (graphgen/) and records digests of its output.  The GPU tests compare the library against these
files (the oracle needs minutes on these sizes, the GPU seconds).

  rmat22_plouvain_mod : R-MAT scale 22, edge factor 16, (0.57, 0.19, 0.19, 0.05), seed 2; pLouvain (Louvain+,
                        Alg. 1) with modularity, lambda = 1 / sum of weighted degrees (Sec. II-A)
  lattice4096_pleiden_cpm20 : 4096 x 4096 four-neighbour lattice, 10 % of edges deleted, weights uniform in
                        [1, 100], seed 3; pLeiden (Alg. 5) with CPM, lambda = 1/20, unit vertex weights
  rmat26_pleiden_cpm20_2levels : R-MAT scale 26, edge factor 16, same quadrant probabilities, seed 4; pLeiden
                        with CPM, lambda = 1/20, stopped after two levels (max_levels = 2): the local moves of
                        levels 0 and 1 with the alternate local move, the refinement and the contraction between
                        them, at full size (about 40 GB of host memory and tens of minutes for the oracle)

Usage: python tests/golden/make_golden.py [name ...]
"""
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import graphgen as gg  # noqa: E402
import oracle as O  # noqa: E402

WORKLOADS = {  # name: (generator, variant, lambda, vertex-weight mode, options other than the defaults)
    "rmat22_plouvain_mod": (gg.config2_rmat, O.PLOUVAIN, (1, 1, True), O.VW_WEIGHTED_DEGREE, {}),
    "lattice4096_pleiden_cpm20": (gg.config3a_lattice, O.PLEIDEN, (1, 20, False), O.VW_UNIT, {}),
    "rmat26_pleiden_cpm20_2levels": (gg.config3b_rmat, O.PLEIDEN, (1, 20, False), O.VW_UNIT, {"max_levels": 2}),
}


def sha(a) -> str:
    return hashlib.sha256(a.tobytes()).hexdigest()


def make(name):
    gen, variant, lam, mode, opts = WORKLOADS[name]
    g = gen()
    digest = g.digest()
    print(name, "graph", g.n, g.nnz, digest, flush=True)
    t = time.time()
    r = O.cluster(g, variant, lam=lam, vw_mode=mode, opts=O.make_opts(**opts) if opts else None, trace_cap=1 << 20)
    dt = time.time() - t
    assert r.status == 0
    out = dict(workload=name, graph_sha256=digest, n=g.n, nnz=g.nnz, variant=variant, lam=list(lam),
               vw_mode=mode, opts=opts, labels_sha256=sha(r.labels), N=str(r.N), q=r.q, p=r.p,
               num_clusters=r.num_clusters, levels=r.levels, flags=r.flags, trace=r.trace.tolist(),
               oracle_seconds=round(dt, 1))
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), name + ".json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(name, "written", round(dt, 1), "s", flush=True)


if __name__ == "__main__":
    for nm in (sys.argv[1:] or list(WORKLOADS)):
        make(nm)
