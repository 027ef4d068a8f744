"""The stored oracle path sums (tests/golden/oracle_sums_*.json) are the
oracle's: each file's chunks have the workload's shape and add up to
consistent totals, and one chunk per scheme recomputed here by the oracle
(same seed, path range and thread count) matches the stored one."""
import json
import os

import numpy as np
import pytest

import workloads

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
IDS = {"full": 0, "picard": 1, "first_order": 3, "second_order": 4}
CASES = [("oracle_sums_gpu_n20_2p20.json", workloads.gpu_scale, 5, ("full", "picard")),
         ("oracle_sums_mlp_n40_2p16.json", workloads.learned_drift, 3,
          ("full", "picard", "first_order", "second_order"))]


@pytest.mark.parametrize("fname,make,chunk,schemes", CASES)
def test_stored_oracle_sums_recompute(oracle_mod, fname, make, chunk, schemes):
    with open(os.path.join(GOLDEN, fname)) as f:
        g = json.load(f)
    ts = make()
    assert g["workload"] == ts.name and g["seed"] == 1
    assert (g["n_rates"], g["n_strikes"]) == (ts.n_rates, ts.n_strikes)
    n_chunks = g["n_paths"] // g["chunk_paths"]
    assert n_chunks * g["chunk_paths"] == g["n_paths"]
    o = oracle_mod.Oracle(ts, seed=1)
    for name in schemes:
        chunks = g["schemes"][name]
        assert len(chunks) == n_chunks
        itm = sum(np.asarray(c["n_itm"]) for c in chunks)
        assert np.all(itm <= g["n_paths"]) and np.all(np.diff(itm, axis=1) <= 0)
        p0 = chunk * g["chunk_paths"]
        r = o.price_sums(IDS[name], g["chunk_paths"], path0=p0, threads=g["threads"])
        for k in g["stat_keys"]:
            ref = np.asarray(chunks[chunk][k])
            assert np.allclose(r[k], ref, rtol=1e-12, atol=0), (name, k)
