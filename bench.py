#!/usr/bin/env python3
"""Throughput of the Lévy LIBOR Monte Carlo path on one MI355X.

One step = one pass of the whole path over the N=20 semiannual workload
(L0_i = 0.03 + 0.002 i, lambda = 0.12 + 0.1 e^{-0.5 (T_i - t)}, NIG(18, -4, 1),
20 Euler steps per period, 2^20 paths, strikes {0.8, 1, 1.2} x forward) for
the full Euler drift and for the Picard drift: FP64 precompute, path kernel
(FP32 state, FP64 increments and sums) and the fixed-order reduction, each
scheme on the same stream.  `value` is path-steps per second over both
schemes (paths x Euler steps x schemes / wall time of the timed steps).

Prints one JSON line.  Only one GPU is used; --gpus above 1 exits.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402

PEAK_FP32 = 157.3e12   # MI355X vector FP32, FLOP/s

# HBM bytes per path-kernel launch from rocprofv3 --pmc FETCH_SIZE and
# WRITE_SIZE runs of this benchmark, each scaled by the same counter's reading
# for a 1 GiB device copy (FETCH_SIZE x 2.0, WRITE_SIZE x 1.0;
# profiles/path_kernel_gpu_n20_counters.md), keyed by the hash of the kernel
# sources they were taken on; any other hash reports null.
TRAFFIC_BYTES = {"92e05cbf6a5b5222": {"full": 146993080, "picard": 166064311}}
KERNEL_SOURCES = ["paper_1006_3340_amd/csrc/path_kernel.hpp",
                  "paper_1006_3340_amd/csrc/lll_device.hpp"]
MLP_SOURCES = ["paper_1006_3340_amd/csrc/mlp_path.hip", "paper_1006_3340_amd/csrc/mlp.hpp",
               "paper_1006_3340_amd/csrc/mlp_train.hip",
               "paper_1006_3340_amd/csrc/path_kernel.hpp",
               "paper_1006_3340_amd/csrc/lll_device.hpp"]
# rocprofv3 --pmc figures of the surrogate pricing kernel at 2^20 paths
# (profiles/mlp_kernels_mlp_n40_mfma_counters.md), by source hash: a changed
# kernel reports none
MLP_COUNTERS = {"653b1a0fa29f8bbc": {
    "source": "profiles/mlp_kernels_mlp_n40_mfma_counters.md",
    "mlp_path_kernel_ms": 524.01, "clock_ghz": 2.37,
    "counted_mfma_flop": 2.178e+14, "counted_mfma_tflops": 415.6,
    "mfma_busy": 0.167, "valu_busy": 0.853, "trans_share_of_valu": 0.222}}


def source_hash(sources) -> str:
    """Hash of kernel sources and the compile flags they are built with."""
    import hashlib
    from paper_1006_3340_amd import _build
    h = hashlib.sha256()
    for rel in sources:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    # the flags name include directories by absolute path: hash them relative
    flags = [f.replace(_build.ROOT, "<repo>") for f in _build.FLAGS + _build.PATH_FLAGS]
    h.update(repr(flags).encode())
    return h.hexdigest()[:16]


def fp32_bucket(n_rates: int) -> int:
    """Register slots of the FP32 single-structure path kernel that runs N rates."""
    return next(b for b in (8, 16, 20, 24, 32, 40) if n_rates <= b)


def kernel_hash() -> str:
    return source_hash(KERNEL_SOURCES)


Q = 64
METRIC = "path-steps/s: full Euler vs Picard vs MLP drift, at <=1e-4 rel caplet error"


def flops_per_path_step(scheme: str, n: int) -> int:
    """Algorithmic FP32 flops of one Euler step with n live rates (FMA = 2).
    FULL / PICARD, per quadrature node: the top rate's R = ell E (1), the n - 1
    coupled rates' C += W E R (2 each) and the n - 2 rates between them and
    the lowest live rate advancing R = R + ell E (1 + R) (4 each), i.e.
    6n - 9 per node; plus 8 per rate for ell and the update (16 for PICARD,
    which also advances its predictor) and 40 for the increment.
    SECOND_ORDER: 6n - 8 per node (the truncated product carries two sums).
    FIRST_ORDER: n (n - 1) / 2 FMAs of the closed-form sums.  FROZEN: the update."""
    node = Q * (6 * n - 9) if n >= 2 else 0
    if scheme == "full":
        return node + 8 * n + 40
    if scheme == "picard":
        return node + 16 * n + 40
    if scheme == "frozen":
        return 4 * n + 40
    if scheme == "first_order":
        return n * (n - 1) + 8 * n + 40
    if scheme == "second_order":
        return (Q * (6 * n - 8) if n >= 2 else 0) + 8 * n + 40
    raise ValueError(scheme)


def flops_per_path(ts, scheme: str) -> int:
    s, N = ts.steps_per_period, ts.n_rates
    return sum(s * flops_per_path_step(scheme, N - m) for m in range(N))


GOLDEN = os.path.join(ROOT, "tests", "golden")


def stored_oracle_prices(fname: str, scheme: str, ts) -> dict:
    """Prices of eq. (caplet) from the FP64 oracle's stored path sums (written
    by tests/golden/make_oracle_sums.py from the oracle alone): chunk sums
    added in order, delta_i B(0, T_*) sum p / n."""
    import json
    with open(os.path.join(GOLDEN, fname)) as f:
        g = json.load(f)
    sp = sum(np.asarray(c["sum_p"], dtype=np.float64) for c in g["schemes"][scheme])
    itm = sum(np.asarray(c["n_itm"], dtype=np.float64) for c in g["schemes"][scheme])
    B0T = ts.B0_T1 / np.prod(1.0 + ts.delta * ts.L0)
    return {"price": ts.delta[:, None] * B0T * sp / g["n_paths"], "n_itm": itm,
            "n_paths": g["n_paths"]}


def per_caplet_error(price, ref: dict, ts, itm_floor: int = 100) -> dict:
    """Error of each caplet-strike price against the oracle's: relative where
    the oracle has >= itm_floor in-the-money paths, else absolute over the
    at-the-money price of the same caplet (near-zero prices)."""
    atm = int(np.argmin(np.abs(ts.strikes[0] / ts.L0[0] - 1.0)))
    floored = ref["n_itm"] < itm_floor
    den = np.where(floored, np.abs(ref["price"][:, atm:atm + 1]), np.abs(ref["price"]))
    err = np.abs(price - ref["price"]) / den
    return {"max": float(err.max()), "per_caplet_max": [float(v) for v in err.max(axis=1)],
            "n_floored": int(floored.sum())}


def cpu_baseline(ts, n_sample: int, schemes) -> dict:
    """The FP64 oracle, as it stands, on a bounded sample of the same workload."""
    import oracle
    oracle.build(force=False)
    o = oracle.Oracle(ts, seed=1)
    total_steps = 0
    t0 = time.perf_counter()
    threads = 0
    for name in schemes:
        r = o.price_sums({"full": 0, "picard": 1}[name], n_sample)
        threads = r["threads"]
        total_steps += n_sample * ts.n_steps
    dt = time.perf_counter() - t0
    # one host thread on a smaller sample (the per-core rate)
    n1 = max(64, n_sample // 48)
    t1 = time.perf_counter()
    for name in schemes:
        o.price_sums({"full": 0, "picard": 1}[name], n1, threads=1)
    dt1 = time.perf_counter() - t1
    cpu = ""
    try:
        with open("/proc/cpuinfo") as f:
            cpu = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    return {"value": total_steps / dt, "unit": "path-steps/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu, "host_cpus": os.cpu_count(),
            "sample": f"{n_sample} paths x {ts.n_steps} steps x {len(schemes)} schemes "
                      f"({'+'.join(schemes)}) of the same workload, {dt:.1f} s",
            "one_thread": {"value": n1 * ts.n_steps * len(schemes) / dt1,
                           "sample": f"{n1} paths, {dt1:.1f} s"}}


def adjoint_flops_per_path(ts) -> int:
    """Algorithmic FP32 flops of the Greeks pass per path: the FULL forward pass,
    then for every caplet c (n = N - c rates carried) and every step up to its
    fixing, one recomputed FULL step plus the reverse step (18 flops per
    (rate, node): suffix product 3, F recursion 5, the adjoints of ell and E 10)."""
    N, s = ts.n_rates, ts.steps_per_period
    total = flops_per_path(ts, "full")
    for c in range(N):
        n = N - c
        per_step = flops_per_path_step("full", n) + 18 * Q * n + 10 * n
        total += (c + 1) * s * per_step
    return total


def vjp_flops_per_path(ts) -> int:
    """Algorithmic FP32 flops of the vector-Jacobian product per path: the FULL
    forward pass, then for every period m (n = N - m rates carried) and each of
    its steps one recomputed FULL step plus the reverse step."""
    N, s = ts.n_rates, ts.steps_per_period
    total = flops_per_path(ts, "full")
    for m in range(N):
        n = N - m
        total += s * (flops_per_path_step("full", n) + 18 * Q * n + 10 * n)
    return total


def bench_adjoint(lll, stream, n: int = 1 << 20) -> dict:
    """Pathwise Greeks of 40 ATM caplets (N=40 quarterly, 2^20 paths, FP32): the
    full Jacobian (one reverse sweep per caplet) and the vector-Jacobian product
    with unit weights (one sweep; what the autograd backward runs)."""
    ts = workloads.adjoint_greeks()
    with lll.Plan(ts, precision=lll.FP32, max_paths=n) as plan:
        plan.set_timing(True)
        plan.greeks(n, seed=1, stream=stream)   # warmup (allocates checkpoints)
        plan.greeks(n, seed=1, stream=stream)
        ms = plan.timing()["paths"]
        g = plan.greeks_results(stream)
        w = np.ones(ts.n_rates)
        plan.greeks_vjp(n, w, seed=1, stream=stream)   # warmup
        plan.greeks_vjp(n, w, seed=1, stream=stream)
        ms_vjp = plan.timing()["paths"]
        r = plan.greeks_vjp_results(stream)
    if not np.all(np.isfinite(g["dP_dL0"])):
        raise RuntimeError("non-finite Greeks")
    fl = adjoint_flops_per_path(ts) * n
    t = ms / 1e3
    fv = vjp_flops_per_path(ts) * n
    tv = ms_vjp / 1e3
    ref = w @ g["dP_dL0"]
    return {"workload": ts.name, "n_paths": n, "ms": ms,
            "forward_path_steps_per_s": n * ts.n_steps / t,
            "fp32_tflops": fl / t / 1e12, "frac_fp32_peak": fl / t / PEAK_FP32,
            "vjp": {"ms": ms_vjp, "fp32_tflops": fv / tv / 1e12, "frac_fp32_peak": fv / tv / PEAK_FP32,
                    "speedup_vs_jacobian": ms / ms_vjp,
                    "max_rel_diff_vs_jacobian": float(np.max(np.abs(r["vjp_L0"] - ref)) /
                                                      np.max(np.abs(ref)))}}


PEAK_BF16 = 2.5e15     # MI355X dense BF16 matrix cores, FLOP/s


def mlp_flops_per_rate_step(n_later: int) -> dict:
    """Algorithmic flops of the surrogate coupling of one rate with n_later later
    rates (FMA = 2): on the matrix cores the first layer over the later rates'
    states (2 x 64 x n_later; the time and one-hot inputs are a bias table), the
    two 64x64 hidden layers and the output dot (128); on the vector ALU the
    first-order expansion (2 per later rate) and three 64-wide GELU layers (8
    per unit)."""
    return {"mfma": 2 * 64 * n_later + 2 * 2 * 64 * 64 + 128,
            "valu": 2 * n_later + 3 * 8 * 64}


def bench_mlp(lll, stream, n: int = 1 << 20, train_steps: int = 3000) -> dict:
    """Learned drift (N=40 quarterly, 2^20 paths): datagen (~2^22 quadrature
    pairs), training on the device, then FULL, Picard, the first-order
    expansion alone and the surrogate on common random numbers, each judged
    against FULL (max relative caplet error over all caplets and strikes)."""
    ts = workloads.learned_drift()
    out = {"workload": ts.name, "n_paths": n}
    with lll.Plan(ts, precision=lll.FP32, max_paths=n) as plan, lll.Mlp(seed=1) as net:
        plan.set_timing(True)
        t0 = time.perf_counter()
        pairs = net.generate(plan, 12800, 16, seed=1, stream=stream)
        t1 = time.perf_counter()
        loss = net.train(train_steps, batch=16384, lr=2e-3, seed=1, stream=stream)
        t2 = time.perf_counter()
        out["train"] = {"pairs": pairs, "datagen_s": t1 - t0, "train_s": t2 - t1,
                        "steps": train_steps, "batch": 16384,
                        "loss_first": float(loss[:10].mean()), "loss_last": float(loss[-50:].mean())}
        legs = [("full", lambda: plan.execute(lll.FULL, n, seed=1, stream=stream)),
                ("picard", lambda: plan.execute(lll.PICARD, n, seed=1, stream=stream)),
                ("frozen", lambda: plan.execute(lll.FROZEN, n, seed=1, stream=stream)),
                ("first_order", lambda: plan.execute(lll.FIRST_ORDER, n, seed=1, stream=stream)),
                ("second_order", lambda: plan.execute(lll.SECOND_ORDER, n, seed=1, stream=stream)),
                ("mlp", lambda: plan.execute_mlp(net, True, n, seed=1, stream=stream))]
        prices = {}
        for name, run in legs:
            run()                       # warmup
            run()
            ms = plan.timing()["paths"]
            prices[name] = plan.results(stream)["price"]
            out[name] = {"kernel_ms": ms, "path_steps_per_s": n * ts.n_steps / (ms / 1e3)}
        live = prices["full"] > 0.0    # out-of-the-money caplets fixed at t = 0 price 0
        for name in prices:
            rel = np.abs(prices[name][live] / prices["full"][live] - 1)
            out[name]["max_rel_err_vs_full"] = float(np.max(rel))
        # the accuracy gate judged by the FP64 oracle's FULL prices (stored
        # sums, 2^16 paths, same streams)
        n16 = 1 << 16
        ref = stored_oracle_prices("oracle_sums_mlp_n40_2p16.json", "full", ts)
        gate = {}
        for name, run in legs:
            if name == "mlp":
                plan.execute_mlp(net, True, n16, seed=1, stream=stream)
            else:
                plan.execute(lll.SCHEMES[name], n16, seed=1, stream=stream)
            gate[name] = per_caplet_error(plan.results(stream)["price"], ref, ts)["max"]
        out["vs_oracle_full_2p16"] = gate
        plan.execute_mlp(net, True, n, seed=1, judge_stride=8, stream=stream)
        st = plan.mlp_stats(stream)
        out["mlp"]["judge"] = {"stride": 8, "rate_steps": st["rate_steps"],
                               "fallback_frac": st["fallbacks"] / st["rate_steps"],
                               "mean_abs_err_over_mean_abs_quad": st["judge_abs_err"] / st["judge_abs_quad"],
                               "max_rel": st["judge_max_rel"]}
    s, N = ts.steps_per_period, ts.n_rates
    mf = va = 0
    for m in range(N):
        for i in range(m, N - 1):      # the last rate has no coupling
            f = mlp_flops_per_rate_step(N - 1 - i)
            mf += s * f["mfma"]
            va += s * f["valu"]
    t = out["mlp"]["kernel_ms"] / 1e3
    out["mlp"].update({"mfma_tflops": mf * n / t / 1e12, "frac_bf16_peak": mf * n / t / PEAK_BF16,
                       "valu_tflops": va * n / t / 1e12, "frac_fp32_peak": va * n / t / PEAK_FP32,
                       "counters": MLP_COUNTERS.get(source_hash(MLP_SOURCES))})
    for name in ("full", "picard", "first_order", "second_order"):
        fl = flops_per_path(ts, name) * n
        out[name]["frac_fp32_peak"] = fl / (out[name]["kernel_ms"] / 1e3) / PEAK_FP32
    return out


def bench_parity(lll, plan, ts, n, stream, schemes) -> dict:
    """Prices of the timed launch configuration against the FP64 oracle on the
    same Philox streams, per caplet (the oracle's sums at 2^20 paths are
    stored: ~7 CPU-minutes), and each scheme against the oracle's FULL (the
    metric's accuracy condition)."""
    fname = "oracle_sums_gpu_n20_2p20.json"
    out = {"reference": f"FP64 oracle, {fname}", "bar": 1e-4}
    ref_full = stored_oracle_prices(fname, "full", ts)
    for name in schemes:
        plan.execute(lll.SCHEMES[name], n, seed=1, stream=stream)
        price = plan.results(stream)["price"]
        out[name] = per_caplet_error(price, stored_oracle_prices(fname, name, ts), ts)
        if name != "full":
            out[name]["vs_oracle_full"] = per_caplet_error(price, ref_full, ts)["max"]
    return out


def bench_reference_schemes(lll, plan, ts, n, stream) -> dict:
    """The frozen drift and the first- and second-order expansions on the benchmark workload:
    path-kernel time (HIP events) and max relative caplet error against FULL on
    the same streams (not part of `value`)."""
    plan.execute(lll.FULL, n, seed=1, stream=stream)
    full = plan.results(stream)["price"]
    live = full > 0.0
    out = {}
    for name in ("frozen", "first_order", "second_order"):
        plan.execute(lll.SCHEMES[name], n, seed=1, stream=stream)   # warmup
        ms = []
        for _ in range(3):
            plan.execute(lll.SCHEMES[name], n, seed=1, stream=stream)
            ms.append(plan.timing()["paths"])
        t = float(np.median(ms)) / 1e3
        price = plan.results(stream)["price"]
        out[name] = {"path_kernel_ms": t * 1e3, "path_steps_per_s": n * ts.n_steps / t,
                     "frac_fp32_peak": flops_per_path(ts, name) * n / t / PEAK_FP32,
                     "max_rel_err_vs_full": float(np.max(np.abs(price[live] / full[live] - 1)))}
    return out


# Section 4 of the paper (Kluge's example, 10^4 paths, 5 steps per period):
# implied-volatility errors against the full solution, basis points.
PAPER_KLUGE_BP = {"picard": {"max": 0.023}, "frozen": {"max": 17.0},
                  "first_order": {"max": 9.5, "mean": 0.41},
                  "second_order": {"max": 0.38, "mean": 0.013}}


def bench_kluge(lll, stream) -> dict:
    """The paper's numerical example on the GPU (FP64 kernels): caplet
    implied-volatility differences of each scheme against FULL (strikes
    0.8..1.2 x forward), at the paper's 10^4 paths and at 2^20 paths, next to
    the numbers the paper reports (its strike grid and random numbers differ).
    EXACT, the drift of the exact subset expansion, shows how far FULL's
    64-node rule is from the paper's own full solution."""
    from paper_1006_3340_amd import quotes
    ts = workloads.kluge_example()
    out = {"workload": ts.name, "strikes": "0.8..1.2 x forward", "paper_bp": PAPER_KLUGE_BP}
    names = {1: "picard", 2: "frozen", 3: "first_order", 4: "second_order", 6: "exact"}
    for n in (10000, 1 << 20):
        with lll.Plan(ts, precision=lll.FP64, max_paths=n) as plan:
            iv = {}
            for s in (0, 1, 2, 3, 4, 6):
                plan.execute(s, n, seed=1, stream=stream)
                iv[s] = quotes.caplet_implied_vols(ts, plan.results(stream)["price"])
        out[f"paths_{n}"] = {names[s]: {"max_bp": float(np.nanmax(np.abs(iv[s] - iv[0]) * 1e4)),
                                        "mean_bp": float(np.nanmean(np.abs(iv[s] - iv[0]) * 1e4))}
                             for s in names}
    return out


def exact_flops_per_path(ts) -> int:
    """Algorithmic flops of LLL_EXACT per path: per step of period m the
    2^{N-m} - 1 subset terms of the live rates (one FMA each) plus the update
    and the increment, as for FULL."""
    N, s = ts.n_rates, ts.steps_per_period
    return sum(s * (2 * ((1 << (N - m)) - 1) + 8 * (N - m) + 40) for m in range(N))


def exact_subset_flops_per_path(ts) -> int:
    """The subset-sum part of exact_flops_per_path, the work the matrix cores
    do: one multiply-add per subset term of every live rate and step."""
    N, s = ts.n_rates, ts.steps_per_period
    return sum(s * 2 * ((1 << (N - m)) - 1) for m in range(N))


# The paper's own timing of its full solution (exact drift) on the example of
# its Section 4: N = 9, 10^4 paths, 5 steps per period, Matlab on an 8-process
# Intel i7 (another machine: context, not a target).
PAPER_FULL_SOLUTION_S = 141.0


def bench_exact(lll, stream) -> dict:
    """LLL_EXACT (drift of the exact subset expansion, no quadrature): the
    paper's example at its own size in FP64 (beside the paper's 141 s), and
    the benchmark workload (N = 20, 2^16 paths, FP32) against FULL on the same
    paths."""
    out = {}
    ts = workloads.kluge_example()
    n = 10000
    with lll.Plan(ts, precision=lll.FP64, max_paths=n) as plan:
        plan.set_timing(True)
        plan.execute(lll.EXACT, n, seed=1, stream=stream)   # warmup (allocates the table)
        plan.execute(lll.EXACT, n, seed=1, stream=stream)
        t = plan.timing()
        pe = plan.results(stream)["price"]
        plan.execute(lll.FULL, n, seed=1, stream=stream)
        pf = plan.results(stream)["price"]
    ms = t["precompute"] + t["paths"] + t["reduce"]
    out["kluge_n9_fp64_10000"] = {
        "ms": ms, "path_kernel_ms": t["paths"], "path_steps_per_s": n * ts.n_steps / (ms / 1e3),
        "paper_full_solution_s": PAPER_FULL_SOLUTION_S,
        "max_rel_diff_vs_full": float(np.max(np.abs(pe[pf > 0] / pf[pf > 0] - 1)))}
    ts = workloads.gpu_scale()
    n = 1 << 16
    with lll.Plan(ts, precision=lll.FP32, max_paths=n) as plan:
        plan.set_timing(True)
        plan.execute(lll.EXACT, n, seed=1, stream=stream)   # warmup
        ms = []
        for _ in range(3):
            plan.execute(lll.EXACT, n, seed=1, stream=stream)
            ms.append(plan.timing()["paths"])
        ms = float(np.median(ms))
        pe = plan.results(stream)["price"]
        plan.execute(lll.FULL, n, seed=1, stream=stream)
        pf = plan.results(stream)["price"]
    fl = exact_flops_per_path(ts) * n
    mfma_probe = lll.fp32_mfma_peak()   # measured FP32 16x16x4 matrix-core rate, TFLOP/s
    achieved = exact_subset_flops_per_path(ts) * n / (ms / 1e3) / 1e12
    out["gpu_n20_fp32_65536"] = {
        "path_kernel_ms": ms, "path_steps_per_s": n * ts.n_steps / (ms / 1e3),
        "fp32_tflops": fl / (ms / 1e3) / 1e12, "frac_fp32_peak": fl / (ms / 1e3) / PEAK_FP32,
        # the subset sums run on v_mfma_f32_16x16x4f32: their rate against the
        # quoted dense FP32 matrix peak and the measured matrix-core ceiling
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP32 / 1e12,
                     "unit": "TFLOP/s", "frac": achieved * 1e12 / PEAK_FP32,
                     "mfma_ceiling_tflops": mfma_probe,
                     "frac_of_mfma_ceiling": achieved / mfma_probe},
        "max_rel_diff_vs_full": float(np.max(np.abs(pe[pf > 0] / pf[pf > 0] - 1)))}
    return out


def bench_swaptions(lll, stream, n: int = 1 << 20) -> dict:
    """Co-terminal payer swaptions on the benchmark workload (strikes 0.8, 1, 1.2
    x forward swap rate): path-kernel time per scheme (the multi-rate payoff is
    evaluated at each fixing date) and max relative error against FULL."""
    ts = workloads.coterminal_swaptions(workloads.gpu_scale(), [0.8, 1.0, 1.2])
    out = {"workload": ts.name}
    with lll.Plan(ts, precision=lll.FP32, max_paths=n) as plan:
        plan.set_timing(True)
        prices = {}
        for name in ("full", "picard", "first_order"):
            plan.execute(lll.SCHEMES[name], n, seed=1, stream=stream)   # warmup
            plan.execute(lll.SCHEMES[name], n, seed=1, stream=stream)
            ms = plan.timing()["paths"]
            prices[name] = plan.results(stream)["price"]
            out[name] = {"path_kernel_ms": ms, "path_steps_per_s": n * ts.n_steps / (ms / 1e3)}
    live = prices["full"] > 0.0
    for name in prices:
        out[name]["max_rel_err_vs_full"] = float(np.max(np.abs(prices[name][live] / prices["full"][live] - 1)))
    return out


def bench_maturity_parallel(lll, stream) -> dict:
    """Few paths, many rates: PICARD in the maturity-parallel layout (PICARD_MP)
    against the one-path-per-lane FULL and PICARD kernels at 10^4 paths (N = 20,
    40; N = 60 runs only as PICARD_MP), and at 2^17 paths where the path kernel
    fills the GPU.  Times are the library's HIP events around all of the
    scheme's kernels (PICARD_MP: increments, predictor, period items, payoffs);
    TFLOP/s counts PICARD's algorithmic flops.  Differences are max relative
    caplet differences over the non-zero prices, on the same random streams."""
    out = {}
    for wl, n in (("mp_n60", 10000), ("mlp_n40", 10000), ("gpu_n20", 10000), ("mlp_n40", 1 << 17)):
        ts = workloads.WORKLOADS[wl]()
        names = ["picard_mp"] + ([] if ts.n_rates > lll.N_MAX else ["full", "picard"])
        res, prices = {}, {}
        with lll.Plan(ts, precision=lll.FP32, max_paths=n) as plan:
            plan.set_timing(True)
            for name in names:
                plan.execute(lll.SCHEMES[name], n, seed=1, stream=stream)   # warmup
                ms = []
                for _ in range(3):
                    plan.execute(lll.SCHEMES[name], n, seed=1, stream=stream)
                    ms.append(plan.timing()["paths"])
                t = float(np.median(ms)) / 1e3
                prices[name] = plan.results(stream)["price"]
                fl = flops_per_path(ts, "picard" if name == "picard_mp" else name) * n
                res[name] = {"ms": t * 1e3, "path_steps_per_s": n * ts.n_steps / t,
                             "fp32_tflops": fl / t / 1e12, "frac_fp32_peak": fl / t / PEAK_FP32}
        for ref in ("picard", "full"):
            if ref in prices:
                live = prices[ref] > 0.0
                res["picard_mp"][f"max_rel_diff_vs_{ref}"] = float(
                    np.max(np.abs(prices["picard_mp"][live] / prices[ref][live] - 1)))
                res["picard_mp"][f"speedup_vs_{ref}"] = res[ref]["ms"] / res["picard_mp"]["ms"]
        out[f"{wl}_{n}"] = res
    return out


def bench_batched(lll, stream, schemes, n_each: int = 1 << 18, reps: int = 2) -> dict:
    """64 independent structures in one persistent launch: kernel time (HIP events
    recorded by the library), path-steps/s and FP32 fraction of peak."""
    structs = workloads.batched()
    out = {"workload": "batched_64", "n_structures": len(structs), "paths_each": n_each}
    with lll.Batch(structs, max_paths_each=n_each) as b:
        b.set_timing(True)
        for name in schemes:
            b.execute(lll.SCHEMES[name], n_each, seed=1, stream=stream)  # warmup
            ms = []
            for _ in range(reps):
                b.execute(lll.SCHEMES[name], n_each, seed=1, stream=stream)
                ms.append(b.timing())
            t = float(np.mean(ms)) / 1e3
            steps = sum(ts.n_steps for ts in structs) * n_each
            fl = sum(flops_per_path(ts, name) for ts in structs) * n_each
            out[name] = {"kernel_ms": t * 1e3, "path_steps_per_s": steps / t,
                         "fp32_tflops": fl / t / 1e12, "frac_fp32_peak": fl / t / PEAK_FP32}
    return out


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--paths", type=int, default=1 << 20)
    ap.add_argument("--schemes", default="full,picard")
    ap.add_argument("--cpu-sample", type=int, default=196608,
                    help="paths of the oracle timing sample (0 skips it)")
    ap.add_argument("--batched", type=int, default=1,
                    help="also time the 64-structure persistent launch (2^18 paths each)")
    ap.add_argument("--adjoint", type=int, default=1,
                    help="also time the pathwise Greeks pass (N=40, 2^20 paths)")
    ap.add_argument("--mlp", type=int, default=1,
                    help="also train the drift surrogate and time it (N=40, 2^20 paths)")
    ap.add_argument("--mlp-train-steps", type=int, default=3000,
                    help="Adam steps of the surrogate's training in the mlp leg")
    ap.add_argument("--mp", type=int, default=1,
                    help="also time the maturity-parallel PICARD layout (1) or not (0)")
    ap.add_argument("--kluge", type=int, default=1,
                    help="also reproduce the paper's example (implied-volatility errors, FP64)")
    ap.add_argument("--exact", type=int, default=1,
                    help="also time LLL_EXACT (the paper's example and N=20 at 2^16 paths)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run one device-to-device copy of this many MiB (a kernel of "
                         "known traffic for calibrating HBM counters)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        return 2

    import torch
    import paper_1006_3340_amd as lll

    ts = workloads.gpu_scale()
    schemes = [s for s in args.schemes.split(",") if s]
    n = args.paths
    stream = torch.cuda.current_stream()
    plan = lll.Plan(ts, precision=lll.FP32, max_paths=n)
    plan.set_timing(True)

    def one_step(record=None):
        for name in schemes:
            plan.execute(lll.SCHEMES[name], n, seed=1, stream=stream)
            if record is not None:
                t = plan.timing()
                record.setdefault(name, []).append(t)

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(args.steps):
        for name in schemes:
            plan.execute(lll.SCHEMES[name], n, seed=1, stream=stream)
    end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    elapsed = start.elapsed_time(end) / 1e3
    # per-stage kernel durations (HIP events recorded by the library on `stream`)
    rec = {}
    for _ in range(3):
        one_step(rec)
    # the FULL prices the one-shot call below must reproduce (launched back to
    # back with the timed work, so the GPU is still at its working clock)
    plan.execute(lll.FULL, n, seed=1, stream=stream)
    full_price = plan.results(stream)["price"]
    torch.cuda.synchronize()
    if args.copy_mib > 0:
        src = torch.ones(args.copy_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
    if not np.all(np.isfinite(full_price)):
        print(json.dumps({"error": "non-finite prices"}))
        return 1
    # host-to-host: the one-shot call (plan creation and HBM allocation, term
    # structure upload, precompute, the FULL pass, results back to the host)
    lll.price_caplets(ts, n, lll.FULL, seed=1, stream=stream)   # warmup
    t1 = time.perf_counter()
    one = lll.price_caplets(ts, n, lll.FULL, seed=1, stream=stream)
    host_ms = (time.perf_counter() - t1) * 1e3
    if not np.allclose(one["price"], full_price, rtol=1e-12, atol=0):
        print(json.dumps({"error": "one-shot prices differ from the plan's"}))
        return 1
    fma_probe = lll.fp32_fma_peak()   # measured non-packed FP32 FMA ceiling, TFLOP/s
    mix_probe = lll.fp32_mix_peak()   # the quadrature recursion's instruction mix, TFLOP/s

    path_steps = n * ts.n_steps * len(schemes) * args.steps
    value = path_steps / elapsed
    per_scheme = {}
    for name in schemes:
        ms = float(np.mean([r["paths"] for r in rec[name]]))
        fl = flops_per_path(ts, name) * n
        per_scheme[name] = {
            "path_kernel_ms": ms,
            "precompute_ms": float(np.mean([r["precompute"] for r in rec[name]])),
            "reduce_ms": float(np.mean([r["reduce"] for r in rec[name]])),
            "path_steps_per_s": n * ts.n_steps / (ms / 1e3),
            "fp32_tflops": fl / (ms / 1e3) / 1e12,
            "frac_fp32_peak": fl / (ms / 1e3) / PEAK_FP32,
        }
    dom = schemes[0]
    fl_dom = flops_per_path(ts, dom) * n
    ms_dom = per_scheme[dom]["path_kernel_ms"]
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "path-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": ts.name, "n_rates": ts.n_rates, "delta": 0.5,
                   "steps_per_period": ts.steps_per_period, "n_paths": n,
                   "n_strikes": ts.n_strikes, "driver": "NIG(18,-4,1)", "schemes": schemes},
        "roofline": {"bound": "alu", "kernel": f"path_kernel<float,{fp32_bucket(ts.n_rates)},{dom}>",
                     "achieved": fl_dom / (ms_dom / 1e3) / 1e12, "peak": PEAK_FP32 / 1e12,
                     "unit": "TFLOP/s", "frac": fl_dom / (ms_dom / 1e3) / PEAK_FP32,
                     "traffic": TRAFFIC_BYTES.get(kernel_hash(), {}).get(dom),
                     # the quoted FP32 peak counts packed FMAs, which this library
                     # keeps out of its code.  Measured on this GPU: FMAs with
                     # scalar-register operands (the FMA probe) run near one per
                     # lane and cycle (quoted / 2); the recursion's own mix (two
                     # FMAs with a scalar table operand, one on vector registers,
                     # per node and rate) is the attainable ceiling of the kernel
                     "single_issue_peak": PEAK_FP32 / 2 / 1e12,
                     "frac_of_single_issue": fl_dom / (ms_dom / 1e3) / (PEAK_FP32 / 2),
                     "fma_probe_tflops": fma_probe,
                     "mix_ceiling_tflops": mix_probe,
                     "frac_of_mix_ceiling": fl_dom / (ms_dom / 1e3) / 1e12 / mix_probe,
                     "kernel_hash": kernel_hash()},
        "schemes": per_scheme,
        "wall_s": wall,
        "host_io": {"call": "lll_price_caplets (one FULL pass, host buffers in and out)",
                    "ms": host_ms, "path_steps_per_s": n * ts.n_steps / (host_ms / 1e3)},
    }
    if n == 1 << 20:
        out["parity"] = bench_parity(lll, plan, ts, n, stream, schemes)
    out["reference_schemes"] = bench_reference_schemes(lll, plan, ts, n, stream)
    out["swaptions"] = bench_swaptions(lll, stream)
    if args.batched:
        out["batched"] = bench_batched(lll, stream, schemes)
    if args.adjoint:
        out["adjoint"] = bench_adjoint(lll, stream)
    if args.mlp:
        out["mlp"] = bench_mlp(lll, stream, train_steps=args.mlp_train_steps)
    if args.mp:
        out["maturity_parallel"] = bench_maturity_parallel(lll, stream)
    if args.kluge:
        out["kluge"] = bench_kluge(lll, stream)
    if args.exact:
        out["exact"] = bench_exact(lll, stream)
    if args.cpu_sample > 0:
        out["cpu_baseline"] = cpu_baseline(ts, args.cpu_sample, schemes)
    plan.close()
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
