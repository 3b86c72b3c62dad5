"""Full-size parity: the library on the benchmark workloads against the oracle's stored results
(tests/golden/*.json, written by tests/golden/make_golden.py, which calls only the oracle).

Compared exactly: the SHA-256 of the labels, the objective numerator and denominator, cluster and level
counts, flags, and every per-pass / per-level trace record."""
import hashlib
import json
import os

import numpy as np
import pytest

import graphgen as gg
from tests import gpu_util as U

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
GENERATORS = {"rmat22_plouvain_mod": gg.config2_rmat, "lattice4096_pleiden_cpm20": gg.config3a_lattice}


@pytest.mark.parametrize("name", sorted(GENERATORS))
def test_full_size_against_golden(name):
    ref = json.load(open(os.path.join(GOLDEN, name + ".json")))
    g = GENERATORS[name]()
    assert g.digest() == ref["graph_sha256"]
    lab, res = U.run_gpu(g, ref["variant"], tuple(ref["lam"]), ref["vw_mode"])
    assert hashlib.sha256(np.ascontiguousarray(lab).tobytes()).hexdigest() == ref["labels_sha256"]
    assert res.N == int(ref["N"]) and res.obj_den == ref["q"]
    assert (res.num_clusters, res.levels, res.flags) == (ref["num_clusters"], ref["levels"], ref["flags"])
    assert res.trace.tolist() == ref["trace"]
