"""Host logic of bench.py, without a GPU: the algorithmic flop counts, the
per-caplet error rule, the one-GPU guard, and that the stored counter figures
belong to the kernel sources in the tree."""
import io
import json
import contextlib

import numpy as np

import bench
import workloads


def _count_recursion_flops(n: int, q: int) -> int:
    """Operations of the suffix recursion for n live rates, counted by walking
    it: per node the top rate's R = ell E (1 flop), then for every lower rate
    C += W E R (an FMA) and, above the lowest live rate, R += ell E (1 + R)
    (two FMAs)."""
    if n < 2:
        return 0
    per_node = 1
    for j in range(n - 2, -1, -1):
        per_node += 2
        if j > 0:
            per_node += 4
    return q * per_node


def test_flop_counts_follow_the_recursion():
    for n in range(1, 41):
        rec = _count_recursion_flops(n, bench.Q)
        assert bench.flops_per_path_step("full", n) == rec + 8 * n + 40
        assert bench.flops_per_path_step("picard", n) == rec + 16 * n + 40
    ts = workloads.gpu_scale()
    # s N (N + 1) / 2 path-steps of decreasing live counts per path
    total = sum(ts.steps_per_period * bench.flops_per_path_step("full", ts.n_rates - m)
                for m in range(ts.n_rates))
    assert bench.flops_per_path(ts, "full") == total
    # the count the bench divides by: 1.506e12 flops per 2^20-path FULL launch
    assert abs(bench.flops_per_path(ts, "full") * (1 << 20) / 1.506e12 - 1) < 1e-3


def test_per_caplet_error_rule():
    ts = workloads.gpu_scale()
    N, S = ts.n_rates, ts.n_strikes
    ref_price = np.full((N, S), 1e-3)
    ref = {"price": ref_price, "n_itm": np.full((N, S), 500.0)}
    got = ref_price * (1 + 2e-5)
    got[3, 1] = ref_price[3, 1] * (1 + 5e-5)
    err = bench.per_caplet_error(got, ref, ts)
    assert abs(err["max"] - 5e-5) < 1e-12 and err["n_floored"] == 0
    # few in-the-money oracle paths: the error is taken against the ATM price
    ref["n_itm"][5, 2] = 10
    ref["price"][5, 2] = 1e-9
    got2 = ref["price"].copy()
    got2[5, 2] = 1e-9 + 1e-8
    atm = int(np.argmin(np.abs(ts.strikes[0] / ts.L0[0] - 1.0)))
    err = bench.per_caplet_error(got2, ref, ts)
    assert err["n_floored"] == 1
    assert abs(err["max"] - 1e-8 / ref["price"][5, atm]) < 1e-15


def test_more_than_one_gpu_is_refused():
    out = io.StringIO()
    with contextlib.redirect_stdout(out):
        rc = bench.main(["--gpus", "2"])
    assert rc == 2
    assert "one GPU" in json.loads(out.getvalue())["error"]


def test_stored_counters_match_the_kernel_sources():
    """The traffic and surrogate counter figures were taken on these sources."""
    assert bench.kernel_hash() in bench.TRAFFIC_BYTES
    assert bench.source_hash(bench.MLP_SOURCES) in bench.MLP_COUNTERS
    assert bench.fp32_bucket(20) == 20 and bench.fp32_bucket(21) == 24
    assert bench.fp32_bucket(40) == 40 and bench.fp32_bucket(1) == 8
