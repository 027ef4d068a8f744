"""Device-memory inputs and outputs of the C ABI: initial forwards and vol
shifts read from device memory, prices, Greeks and vector-Jacobian products
written to device buffers, all on the caller's stream.  The same kernels run
as with host inputs, so the numbers must be the same bit for bit; inputs the
host cannot check are checked by the next pass (NaN prices, and the host
result calls report the status)."""
import numpy as np
import pytest

import workloads
from paper_1006_3340_amd.autograd import shifted

pytestmark = pytest.mark.gpu

FULL, PICARD = 0, 1


def _cuda(a):
    import torch
    return torch.tensor(np.asarray(a, dtype=np.float64), device="cuda")


def test_device_inputs_and_results_equal_host_path(gpu_lib):
    import torch
    ts = workloads.gpu_scale()
    N, S, n = ts.n_rates, ts.n_strikes, 20000
    rng = np.random.default_rng(4)
    L0 = ts.L0 * (1.0 + 0.05 * rng.uniform(-1, 1, N))
    shift = 0.01 * rng.uniform(-1, 1, N)
    host_ts = shifted(ts, L0, shift, np.zeros(N))
    stream = torch.cuda.current_stream()
    with gpu_lib.Plan(ts, precision=0, max_paths=n) as a, \
            gpu_lib.Plan(host_ts, precision=0, max_paths=n) as b:
        for scheme in (FULL, PICARD):
            print(f"device inputs: scheme {scheme}", flush=True)
            a.set_inputs_dev(L0=_cuda(L0), vol_shift=_cuda(shift), stream=stream)
            a.execute(scheme, n, seed=3, stream=stream)
            price = torch.full((N, S), -1.0, dtype=torch.float64, device="cuda")
            se = torch.full((N, S), -1.0, dtype=torch.float64, device="cuda")
            mart = torch.full((N,), -1.0, dtype=torch.float64, device="cuda")
            a.results_dev(price=price, stderr=se, mart_resid=mart, stream=stream)
            b.execute(scheme, n, seed=3, stream=stream)
            ref = b.results(stream)
            torch.cuda.synchronize()
            assert np.array_equal(price.cpu().numpy(), ref["price"])
            assert np.array_equal(se.cpu().numpy(), ref["stderr"])
            assert np.array_equal(mart.cpu().numpy(), ref["mart_resid"])
            assert np.array_equal(a.results(stream)["price"], ref["price"])
        # only the forwards: the shift set before stays in force
        a.set_inputs_dev(L0=_cuda(ts.L0), stream=stream)
        a.execute(FULL, n, seed=3, stream=stream)
        with gpu_lib.Plan(shifted(ts, ts.L0, shift, np.zeros(N)), precision=0, max_paths=n) as c:
            c.execute(FULL, n, seed=3, stream=stream)
            assert np.array_equal(a.results(stream)["price"], c.results(stream)["price"])
        # a zero shift restores the creation table exactly
        a.set_inputs_dev(vol_shift=_cuda(np.zeros(N)), stream=stream)
        a.execute(FULL, n, seed=3, stream=stream)
        with gpu_lib.Plan(ts, precision=0, max_paths=n) as c:
            c.execute(FULL, n, seed=3, stream=stream)
            assert np.array_equal(a.results(stream)["price"], c.results(stream)["price"])


def test_device_inputs_checked_by_the_pass(gpu_lib):
    import torch
    ts = workloads.plain_fp64()
    N, n = ts.n_rates, 4096
    with gpu_lib.Plan(ts, precision=0, max_paths=n) as p:
        bad = ts.L0.copy()
        bad[3] = -0.01
        p.set_inputs_dev(L0=_cuda(bad))
        p.execute(FULL, n, seed=1)
        price = torch.zeros((N, 1), dtype=torch.float64, device="cuda")
        p.results_dev(price=price)
        torch.cuda.synchronize()
        assert np.all(np.isnan(price.cpu().numpy()))
        with pytest.raises(gpu_lib.LLLError) as ei:
            p.results()
        assert ei.value.code == -1 and "device inputs" in str(ei.value)
        # vols beyond the moment condition (the live vols sum past alpha - beta)
        p.set_inputs_dev(L0=_cuda(ts.L0), vol_shift=_cuda(np.full(N, 3.0)))
        p.execute(FULL, n, seed=1)
        with pytest.raises(gpu_lib.LLLError) as ei:
            p.results()
        assert ei.value.code == -2 and "Lambda" in str(ei.value)
        # valid inputs again: the plan recovers
        p.set_inputs_dev(vol_shift=_cuda(np.zeros(N)))
        p.execute(FULL, n, seed=1)
        got = p.results()["price"]
        with gpu_lib.Plan(ts, precision=0, max_paths=n) as q:
            q.execute(FULL, n, seed=1)
            assert np.array_equal(got, q.results()["price"])
        with pytest.raises(ValueError):
            p.set_inputs_dev(L0=_cuda(ts.L0).float())     # float32 is refused by the binding


def test_device_vjp_and_greeks_equal_host_path(gpu_lib):
    import torch
    ts = workloads.adjoint_greeks()
    N, n = ts.n_rates, 8192
    w = np.linspace(-1.0, 2.0, N)
    stream = torch.cuda.current_stream()
    with gpu_lib.Plan(ts, precision=0, max_paths=n) as p:
        p.greeks_vjp(n, w, seed=2, stream=stream)
        ref = p.greeks_vjp_results(stream)
        p.greeks_vjp_dev(n, _cuda(w), seed=2, stream=stream)
        out = [torch.full((N,), -1.0, dtype=torch.float64, device="cuda") for _ in range(3)]
        p.greeks_vjp_results_dev(price=out[0], vjp_L0=out[1], vjp_vol=out[2], stream=stream)
        torch.cuda.synchronize()
        for t, key in zip(out, ("price", "vjp_L0", "vjp_vol")):
            assert np.array_equal(t.cpu().numpy(), ref[key]), key
        p.greeks(n, seed=2, stream=stream)
        g = p.greeks_results(stream)
        dev = [torch.zeros(N, dtype=torch.float64, device="cuda"),
               torch.zeros((N, N), dtype=torch.float64, device="cuda"),
               torch.zeros((N, N), dtype=torch.float64, device="cuda")]
        p.greeks_results_dev(price=dev[0], dP_dL0=dev[1], dP_dvol=dev[2], stream=stream)
        torch.cuda.synchronize()
        for t, key in zip(dev, ("price", "dP_dL0", "dP_dvol")):
            assert np.array_equal(t.cpu().numpy(), g[key]), key


def test_autograd_forward_does_not_wait_for_the_device(gpu_lib):
    """The device-resident op queues its work and returns: right after the
    forward call (N = 40, 2^20 paths, ~40 ms of kernels) the stream is still
    busy, and the prices then equal the host path's."""
    import torch
    from paper_1006_3340_amd.autograd import CapletPricer
    ts = workloads.adjoint_greeks()
    N, n = ts.n_rates, 1 << 20
    L0 = torch.tensor(ts.L0, dtype=torch.float64, device="cuda", requires_grad=True)
    lv = torch.full((N,), 0.12, dtype=torch.float64, device="cuda", requires_grad=True)
    with CapletPricer(ts, n, seed=1, base_levels=np.full(N, 0.12)) as price_fn:
        torch.cuda.synchronize()
        P = price_fn(L0, lv)
        done = torch.cuda.Event()
        done.record()
        assert not done.query(), "the forward pass waited for the device"
        P.sum().backward()
        torch.cuda.synchronize()
        with gpu_lib.Plan(ts, precision=0, max_paths=n) as plan:
            plan.execute(FULL, n, seed=1)
            ref = plan.results()["price"][:, 0]
    assert np.array_equal(P.detach().cpu().numpy(), ref)
    assert np.all(np.isfinite(L0.grad.cpu().numpy())) and np.all(np.isfinite(lv.grad.cpu().numpy()))


def test_surrogate_as_plan_scheme(gpu_lib):
    """LLL_MLP_DRIFT on a plan with an attached network equals the surrogate
    pass of lll_plan_execute_mlp; without a network, or from the one-shot
    calls, the scheme is refused."""
    ts = workloads.learned_drift()
    n = 4096
    with gpu_lib.Plan(ts, precision=0, max_paths=n) as plan, gpu_lib.Mlp(seed=1) as net:
        net.generate(plan, 256, 8, seed=5)
        net.train(20, batch=1024, lr=2e-3, seed=3)
        with pytest.raises(gpu_lib.LLLError) as ei:
            plan.execute(gpu_lib.MLP_DRIFT, n, seed=1)
        assert ei.value.code == -1
        plan.attach_mlp(net)
        plan.execute(gpu_lib.MLP_DRIFT, n, seed=1)
        a = plan.results()
        plan.execute_mlp(net, True, n, seed=1)
        b = plan.results()
        assert np.array_equal(a["price"], b["price"])
        with pytest.raises(gpu_lib.LLLError) as ei:
            plan.execute(gpu_lib.MLP_DRIFT, n, seed=1, path_offset=64)
        assert ei.value.code == -5
        plan.attach_mlp(None)
    with pytest.raises(gpu_lib.LLLError):
        gpu_lib.price_caplets(ts, n, gpu_lib.MLP_DRIFT)
